// Device-side building blocks shared by the gfx950 kernels: complex arithmetic
// on HIP vector types, the closed-form local substep, the spin-1 eigenbasis
// changes and the affine-map scans used by the partitioned line solves.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gp {

template <typename T> struct cx_of;
template <> struct cx_of<double> { using type = double2; };
template <> struct cx_of<float> { using type = float2; };
template <typename T> using cx = typename cx_of<T>::type;

template <typename T> __host__ __device__ inline cx<T> mk(T re, T im) { cx<T> z; z.x = re; z.y = im; return z; }
template <typename C> __device__ inline C cadd(C a, C b) { C z; z.x = a.x + b.x; z.y = a.y + b.y; return z; }
template <typename C> __device__ inline C csub(C a, C b) { C z; z.x = a.x - b.x; z.y = a.y - b.y; return z; }
template <typename C> __device__ inline C cmul(C a, C b) {
    C z; z.x = a.x * b.x - a.y * b.y; z.y = a.x * b.y + a.y * b.x; return z;
}
// a * conj(b)
template <typename C> __device__ inline C cmulc(C a, C b) {
    C z; z.x = a.x * b.x + a.y * b.y; z.y = a.y * b.x - a.x * b.y; return z;
}
template <typename C, typename T> __device__ inline C cscale(C a, T s) { C z; z.x = a.x * s; z.y = a.y * s; return z; }
template <typename C> __device__ inline C ctimes_i(C a) { C z; z.x = -a.y; z.y = a.x; return z; }     // i a
template <typename C> __device__ inline C ctimes_mi(C a) { C z; z.x = a.y; z.y = -a.x; return z; }    // -i a
template <typename C> __device__ inline C cconj(C a) { C z; z.x = a.x; z.y = -a.y; return z; }
template <typename C> __device__ inline auto cnorm2(C a) { return a.x * a.x + a.y * a.y; }
// a * s + b (s complex)
template <typename C> __device__ inline C cfma(C a, C s, C b) {
    C z; z.x = b.x + a.x * s.x - a.y * s.y; z.y = b.y + a.x * s.y + a.y * s.x; return z;
}

__device__ inline void dsincos(double x, double* s, double* c) { sincos(x, s, c); }
__device__ inline void dsincos(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ inline double dexp(double x) { return exp(x); }
__device__ inline float dexp(float x) { return expf(x); }
__device__ inline double dexpm1(double x) { return expm1(x); }
__device__ inline float dexpm1(float x) { return expm1f(x); }
__device__ inline double dsqrt(double x) { return sqrt(x); }
__device__ inline float dsqrt(float x) { return sqrtf(x); }

template <typename C> __device__ inline C zero_c() { C z; z.x = 0; z.y = 0; return z; }
template <typename C> __device__ inline C one_c() { C z; z.x = 1; z.y = 0; return z; }

__device__ inline double shfl_up_r(double v, int d) { return __shfl_up(v, d, 64); }
__device__ inline float shfl_up_r(float v, int d) { return __shfl_up(v, d, 64); }
__device__ inline double shfl_down_r(double v, int d) { return __shfl_down(v, d, 64); }
__device__ inline float shfl_down_r(float v, int d) { return __shfl_down(v, d, 64); }
template <typename C> __device__ inline C shfl_up_c(C v, int d) { C z; z.x = shfl_up_r(v.x, d); z.y = shfl_up_r(v.y, d); return z; }
template <typename C> __device__ inline C shfl_down_c(C v, int d) { C z; z.x = shfl_down_r(v.x, d); z.y = shfl_down_r(v.y, d); return z; }

// ---------------------------------------------------------------------------
// Thomas pivots of one line, tabulated on the host.  For the tridiagonal
// system  a u_{k-1} + b u_k + e u_{k+1} = r_k  with w_0 = b,
// w_k = b - a e / w_{k-1}:  m = 1/w_k, am = a m, cp = e m.  Entries past the
// table length repeat the converged limit.  The coefficients are rounded to
// the kernels' precision first and the pivots derived from the rounded
// values, so that the elimination inverts the very matrix whose rounded
// coefficients form the right-hand side.
// ---------------------------------------------------------------------------
template <typename T> struct Piv { cx<T> m, am, cp; };

template <typename T> struct LineSet {
    const Piv<T>* piv;   // [lines][K + 1]
    const cx<T>* ae;     // [lines][2] : a, e of each line
    cx<T> bm1;           // diagonal minus one, b - 1 (same for every line of the set)
    int K;               // pivots tabulated before the limit
    // Line-start correction of the solves that use the converged pivots from
    // the first point on.  Those factor the matrix A_inf whose first diagonal
    // entry is the limit pivot w instead of b: A = A_inf + (b - w) e0 e0^T, so
    // (Sherman-Morrison) A^{-1} r = z - gc (z_0) g with z = A_inf^{-1} r,
    // g = A_inf^{-1} e0 and gc = (b - w) / (1 + (b - w) g_0).  g decays like
    // the pivots' transient; it is tabulated up to Kg points.
    const cx<T>* g;      // [lines][Kg]
    const cx<T>* gc;     // [lines]
    int Kg;
};

template <typename T> __device__ inline Piv<T> piv_at(const LineSet<T>& ls, int line, int k) {
    return ls.piv[(size_t)line * (ls.K + 1) + (k < ls.K ? k : ls.K)];
}

// ---------------------------------------------------------------------------
// Per-condensate scalars.
// ---------------------------------------------------------------------------
struct Phys {
    int nx, ny;
    double dx, dy, x0, y0, dt;
    double c0, c2, rabi;
    double dtl;       // time step of each local substep: dt (Lie) or dt/2 (Strang, two per step)
    double gx2, gy2;  // trap V = (gx^2 x^2 + gy^2 y^2)/2
};

template <typename T> __device__ inline T trap_v(const Phys& ph, T x, T y) {
    return (T)0.5 * ((T)ph.gx2 * x * x + (T)ph.gy2 * y * y);
}

// ---------------------------------------------------------------------------
// Local substep, closed form.  With B = c2 F + R e_x, b = |B| and M = B.Sigma
// (spin 1: M^3 = b^2 M):
//   real time       exp(-i dt H_loc) = e^{-i t0} [I - i S1 M - S2 M^2]
//   imaginary time  exp(-dt H_loc)   = e^{-t0}   [I - S1 M + S2 M^2]
// t0 = dt (V + c0 rho), S1 = sin(th)/b or sinh(th)/b, S2 = (1 - cos th)/b^2
// or (cosh th - 1)/b^2, th = dt b, evaluated through half angles so that no
// cancellation occurs.  F_z = rho_{+1} - rho_{-1},
// F_x + i F_y = sqrt2 (conj(psi_{+1}) psi_0 + conj(psi_0) psi_{-1}).
// ---------------------------------------------------------------------------
// Small-argument series (Taylor polynomials), used where the argument is
// below 1/4 in magnitude; the truncation error there is below 1e-18 relative.
//   sinc(x) = sin x / x, cos x, sinhc(x) = sinh x / x, cosh x, expm1(x).
template <typename T> __device__ inline T poly_sinc(T x2) {
    return (T)1 - x2 * ((T)(1.0 / 6) - x2 * ((T)(1.0 / 120) - x2 * ((T)(1.0 / 5040) - x2 * ((T)(1.0 / 362880) - x2 * (T)(1.0 / 39916800)))));
}
template <typename T> __device__ inline T poly_cos(T x2) {
    return (T)1 - x2 * ((T)0.5 - x2 * ((T)(1.0 / 24) - x2 * ((T)(1.0 / 720) - x2 * ((T)(1.0 / 40320) - x2 * ((T)(1.0 / 3628800) - x2 * (T)(1.0 / 479001600))))));
}
template <typename T> __device__ inline T poly_sinhc(T x2) {
    return (T)1 + x2 * ((T)(1.0 / 6) + x2 * ((T)(1.0 / 120) + x2 * ((T)(1.0 / 5040) + x2 * ((T)(1.0 / 362880) + x2 * (T)(1.0 / 39916800)))));
}
template <typename T> __device__ inline T poly_cosh(T x2) {
    return (T)1 + x2 * ((T)0.5 + x2 * ((T)(1.0 / 24) + x2 * ((T)(1.0 / 720) + x2 * ((T)(1.0 / 40320) + x2 * ((T)(1.0 / 3628800) + x2 * (T)(1.0 / 479001600))))));
}
template <typename T> __device__ inline T poly_expm1(T x) {
    T s = (T)(1.0 / 6227020800.0);  // 1/13!
    const T c[12] = {(T)(1.0 / 479001600), (T)(1.0 / 39916800), (T)(1.0 / 3628800), (T)(1.0 / 362880),
                     (T)(1.0 / 40320), (T)(1.0 / 5040), (T)(1.0 / 720), (T)(1.0 / 120), (T)(1.0 / 24),
                     (T)(1.0 / 6), (T)0.5, (T)1};
#pragma unroll
    for (int k = 0; k < 12; ++k) s = s * x + c[k];
    return s * x;
}

// ---------------------------------------------------------------------------
// Local substep, closed form.  With B = c2 F + R e_x, b = |B| and M = B.Sigma
// (spin 1: M^3 = b^2 M):
//   real time       exp(-i dt H_loc) = e^{-i t0} [I - i S1 M - S2 M^2]
//   imaginary time  exp(-dt H_loc)   = e^{-t0}   [I - S1 M + S2 M^2]
// t0 = dt (V + c0 rho), S1 = sin(th)/b or sinh(th)/b, S2 = (1 - cos th)/b^2
// or (cosh th - 1)/b^2, th = dt b, evaluated through the half angle h = th/2
// (S1 = dt sinc(h) cos(h), S2 = dt^2 sinc(h)^2 / 2) so that no cancellation
// occurs.  F_z = rho_{+1} - rho_{-1},
// F_x + i F_y = sqrt2 (conj(psi_{+1}) psi_0 + conj(psi_0) psi_{-1}).
//
// The result is formed as psi + inc, inc = D psi + d (psi + D psi), with the
// scalar factor written as 1 + d and the spin factor as I + D: the increment
// is small, so its rounding errors are small relative to psi, and psi + inc is
// rounded once.  (A rounded unit-modulus FP32 factor (cos t0, -sin t0) is off
// in modulus by up to an ulp; where t0 barely changes from step to step that
// error would repeat with one sign.)
// ---------------------------------------------------------------------------
template <typename T, bool IMAG>
__device__ inline void local_substep(cx<T>& p, cx<T>& z, cx<T>& m, T V, T dt, T c0, T c2, T rabi) {
    using C = cx<T>;
    const T rp = cnorm2(p), r0 = cnorm2(z), rm = cnorm2(m);
    const T rho = rp + r0 + rm;
    const T s2 = (T)1.4142135623730950488;
    const T is2 = (T)0.70710678118654752440;
    const T Bz = c2 * (rp - rm);
    // F+ = sqrt2 (conj(p) z + conj(z) m)
    C Fp = cadd(cmulc(z, p), cmulc(m, z));
    C Bp = mk<T>(c2 * s2 * Fp.x + rabi, c2 * s2 * Fp.y);  // B_x + i B_y
    C Bm = cconj(Bp);
    const T b2 = Bz * Bz + cnorm2(Bp);
    const T h2 = (T)0.25 * dt * dt * b2;  // (half angle)^2
    T sc, ch;                             // sinc(h), cos(h)  (sinhc, cosh in imaginary time)
    if (h2 < (T)0.0625) {
        sc = IMAG ? poly_sinhc(h2) : poly_sinc(h2);
        ch = IMAG ? poly_cosh(h2) : poly_cos(h2);
    } else {
        const T h = dsqrt(h2);
        if (!IMAG) {
            T sh; dsincos(h, &sh, &ch); sc = sh / h;
        } else {
            const T e = dexp(h), ei = (T)1 / e;
            sc = (T)0.5 * (e - ei) / h; ch = (T)0.5 * (e + ei);
        }
    }
    const T S1 = sc * ch * dt;                // sin(th)/b   or sinh(th)/b
    const T S2 = (T)0.5 * sc * sc * dt * dt;  // (1-cos th)/b^2 or (cosh th - 1)/b^2
    // M v = (Bz p + Bm/sqrt2 z,  Bp/sqrt2 p + Bm/sqrt2 m,  Bp/sqrt2 z - Bz m)
    const C bpp = cscale(Bp, is2), bmm = cscale(Bm, is2);
    const C M1p = cadd(cscale(p, Bz), cmul(bmm, z));
    const C M1z = cadd(cmul(bpp, p), cmul(bmm, m));
    const C M1m = csub(cmul(bpp, z), cscale(m, Bz));
    const C M2p = cadd(cscale(M1p, Bz), cmul(bmm, M1z));
    const C M2z = cadd(cmul(bpp, M1p), cmul(bmm, M1m));
    const C M2m = csub(cmul(bpp, M1z), cscale(M1m, Bz));
    const T t0 = dt * (V + c0 * rho);
    C Dp, Dz, Dm, d;
    if (!IMAG) {
        // D v = -i S1 M v - S2 M^2 v ;  d = (cos t0 - 1) - i sin t0 = -2 sin^2(t0/2) - 2 i sin(t0/2) cos(t0/2)
        Dp = csub(cscale(ctimes_mi(M1p), S1), cscale(M2p, S2));
        Dz = csub(cscale(ctimes_mi(M1z), S1), cscale(M2z, S2));
        Dm = csub(cscale(ctimes_mi(M1m), S1), cscale(M2m, S2));
        const T x = (T)0.5 * t0;
        T sh, chh;
        if (x > (T)-0.25 && x < (T)0.25) {
            const T x2 = x * x;
            sh = x * poly_sinc(x2);
            chh = poly_cos(x2);
        } else {
            dsincos(x, &sh, &chh);
        }
        d = mk<T>((T)-2 * sh * sh, (T)-2 * sh * chh);
    } else {
        // D v = -S1 M v + S2 M^2 v ;  d = exp(-t0) - 1
        Dp = csub(cscale(M2p, S2), cscale(M1p, S1));
        Dz = csub(cscale(M2z, S2), cscale(M1z, S1));
        Dm = csub(cscale(M2m, S2), cscale(M1m, S1));
        d = mk<T>((t0 > (T)-0.25 && t0 < (T)0.25) ? poly_expm1(-t0) : dexpm1(-t0), (T)0);
    }
    const C ip = cfma(cadd(p, Dp), d, Dp), iz = cfma(cadd(z, Dz), d, Dz), im = cfma(cadd(m, Dm), d, Dm);
    p = cadd(p, ip); z = cadd(z, iz); m = cadd(m, im);
}

// ---------------------------------------------------------------------------
// Spin-1 eigenbases (unnormalised columns; the inverse carries the factors).
// Sigma_y (x sweep):  nu = +1: u - i sqrt2 psi_0,  nu = 0: v,  nu = -1: u + i sqrt2 psi_0
// Sigma_x (y sweep):  mu = +1: v + sqrt2 psi_0,    mu = 0: u,  mu = -1: v - sqrt2 psi_0
// with u = psi_{+1} - psi_{-1}, v = psi_{+1} + psi_{-1}.
// sqrt2 and 1/sqrt2 enter as unevaluated sums hi + lo applied with one fused
// multiply-add, so each product is rounded once from the exact constant.  A
// single rounded constant would make the three eigenvectors non-orthogonal by
// |2 - sqrt2_rounded^2| (7e-8 in FP32): the sweeps would then be non-unitary
// by the same amount at every step, a norm drift that accumulates linearly.
// ---------------------------------------------------------------------------
template <typename T> struct Sqrt2;
template <> struct Sqrt2<float> {
    static constexpr float hi = 1.4142135381698608f, lo = 2.4203234971764687e-08f;
    static constexpr float rhi = 0.7071067690849304f, rlo = 1.2101617485882343e-08f;
};
template <> struct Sqrt2<double> {
    static constexpr double hi = 1.4142135623730951, lo = -9.667293313452913e-17;
    static constexpr double rhi = 0.7071067811865476, rlo = -4.833646656726457e-17;
};
__device__ inline float dfma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double dfma(double a, double b, double c) { return fma(a, b, c); }
template <typename C, typename T> __device__ inline C mul_sqrt2(C z) {
    C o; o.x = dfma(z.x, Sqrt2<T>::hi, z.x * Sqrt2<T>::lo); o.y = dfma(z.y, Sqrt2<T>::hi, z.y * Sqrt2<T>::lo); return o;
}
template <typename C, typename T> __device__ inline C mul_rsqrt2(C z) {
    C o; o.x = dfma(z.x, Sqrt2<T>::rhi, z.x * Sqrt2<T>::rlo); o.y = dfma(z.y, Sqrt2<T>::rhi, z.y * Sqrt2<T>::rlo); return o;
}

template <typename C, typename T> __device__ inline void to_sy(C& p, C& z, C& m) {
    C u = csub(p, m), v = cadd(p, m), w = mul_sqrt2<C, T>(ctimes_mi(z));
    p = cadd(u, w); z = v; m = csub(u, w);
}
template <typename C, typename T> __device__ inline void from_sy(C& a, C& b, C& c) {
    // psi_{+1} = (a + c)/4 + b/2, psi_{-1} = -(a + c)/4 + b/2, psi_0 = i (a - c) / (2 sqrt2)
    const T q = (T)0.25, hb = (T)0.5;
    C s = cscale(cadd(a, c), q), d = cscale(csub(a, c), hb), hv = cscale(b, hb);
    C p = cadd(s, hv), m = csub(hv, s), z = mul_rsqrt2<C, T>(ctimes_i(d));
    a = p; b = z; c = m;
}
template <typename C, typename T> __device__ inline void to_sx(C& p, C& z, C& m) {
    C u = csub(p, m), v = cadd(p, m), w = mul_sqrt2<C, T>(z);
    p = cadd(v, w); z = u; m = csub(v, w);
}
template <typename C, typename T> __device__ inline void from_sx(C& a, C& b, C& c) {
    // psi_{+1} = (a + c)/4 + b/2, psi_{-1} = (a + c)/4 - b/2, psi_0 = (a - c) / (2 sqrt2)
    const T q = (T)0.25, hb = (T)0.5;
    C s = cscale(cadd(a, c), q), hv = cscale(b, hb), d = cscale(csub(a, c), hb);
    C p = cadd(s, hv), m = csub(s, hv), z = mul_rsqrt2<C, T>(d);
    a = p; b = z; c = m;
}

}  // namespace gp
