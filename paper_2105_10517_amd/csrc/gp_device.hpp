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
// table length repeat the converged limit.  In FP32 the coefficients are
// rounded first and the pivots derived from the rounded values, and m carries
// a second term mlo (m = m + mlo to ~2^-48), so that the elimination inverts
// the very matrix whose rounded coefficients form the right-hand side; in
// FP64 mlo is zero and unused.
// ---------------------------------------------------------------------------
template <typename T> struct Piv { cx<T> m, mlo, am, cp; };

// m r with the compensated multiplier in FP32.
template <typename T> __device__ inline cx<T> mul_m(const Piv<T>& pv, cx<T> r) {
    if (sizeof(T) == 4) return cfma(r, pv.mlo, cmul(pv.m, r));
    return cmul(pv.m, r);
}

template <typename T> struct LineSet {
    const Piv<T>* piv;   // [lines][K + 1]
    const cx<T>* ae;     // [lines][2] : a, e of each line
    cx<T> b;             // diagonal (same for every line of the set)
    int K;               // pivots tabulated before the limit
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
};

// ---------------------------------------------------------------------------
// Local substep, closed form.  With B = c2 F + R e_x, b = |B| and M = B.Sigma
// (spin 1: M^3 = b^2 M):
//   real time       exp(-i dt H_loc) = e^{-i t0} [I - i dt S1 M - dt^2 S2 M^2]
//   imaginary time  exp(-dt H_loc)   = e^{-t0}   [I - dt S1 M + dt^2 S2 M^2]
// t0 = dt (V + c0 rho), S1 = sin(th)/th or sinh(th)/th, S2 = (1 - cos th)/th^2
// or (cosh th - 1)/th^2, th = dt b, evaluated through half angles so that no
// cancellation occurs.  F_z = rho_{+1} - rho_{-1},
// F_x + i F_y = sqrt2 (conj(psi_{+1}) psi_0 + conj(psi_0) psi_{-1}).
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
    C Bp = mk<T>(c2 * s2 * Fp.x + rabi, c2 * s2 * Fp.y);   // B_x + i B_y
    C Bm = cconj(Bp);
    const T b2 = Bz * Bz + cnorm2(Bp);
    const T h = (T)0.5 * dt * dsqrt(b2);                     // half angle
    const T h2 = h * h;
    T sc, ch;                                               // sinc(h) (or sinhc), cos(h) (or cosh)
    const T small = sizeof(T) == 8 ? (T)1e-2 : (T)1e-1;
    if (!IMAG) {
        if (h < small) {
            sc = (T)1 - h2 * ((T)1 / 6 - h2 * ((T)1 / 120 - h2 * ((T)1 / 5040)));
            ch = (T)1 - h2 * ((T)0.5 - h2 * ((T)1 / 24 - h2 * ((T)1 / 720)));
        } else {
            T sh; dsincos(h, &sh, &ch); sc = sh / h;
        }
    } else {
        if (h < small) {
            sc = (T)1 + h2 * ((T)1 / 6 + h2 * ((T)1 / 120 + h2 * ((T)1 / 5040)));
            ch = (T)1 + h2 * ((T)0.5 + h2 * ((T)1 / 24 + h2 * ((T)1 / 720)));
        } else {
            const T e = dexp(h), ei = (T)1 / e;
            sc = (T)0.5 * (e - ei) / h; ch = (T)0.5 * (e + ei);
        }
    }
    const T S1 = sc * ch * dt;                  // sin(th)/b   or sinh(th)/b
    const T S2 = (T)0.5 * sc * sc * dt * dt;    // (1-cos th)/b^2 or (cosh th - 1)/b^2
    // M v = (Bz p + Bm/sqrt2 z,  Bp/sqrt2 p + Bm/sqrt2 m,  Bp/sqrt2 z - Bz m)
    const C bpp = cscale(Bp, is2), bmm = cscale(Bm, is2);
    C M1p = cadd(cscale(p, Bz), cmul(bmm, z));
    C M1z = cadd(cmul(bpp, p), cmul(bmm, m));
    C M1m = csub(cmul(bpp, z), cscale(m, Bz));
    C M2p = cadd(cscale(M1p, Bz), cmul(bmm, M1z));
    C M2z = cadd(cmul(bpp, M1p), cmul(bmm, M1m));
    C M2m = csub(cmul(bpp, M1z), cscale(M1m, Bz));
    const T t0 = dt * (V + c0 * rho);
    C np, nz, nm;
    if (!IMAG) {
        // v - i S1 M v - S2 M^2 v
        np = csub(csub(p, cscale(ctimes_i(M1p), S1)), cscale(M2p, S2));
        nz = csub(csub(z, cscale(ctimes_i(M1z), S1)), cscale(M2z, S2));
        nm = csub(csub(m, cscale(ctimes_i(M1m), S1)), cscale(M2m, S2));
        T sn, cs; dsincos(t0, &sn, &cs);
        const C ph = mk<T>(cs, -sn);
        p = cmul(np, ph); z = cmul(nz, ph); m = cmul(nm, ph);
        if (sizeof(T) == 4) {
            // exp(-i dt H_loc) is unitary, so rho is unchanged.  The FP32 phase
            // factor and spin rotation are not unitary to rounding, and where t0
            // barely changes from step to step that error would repeat with the
            // same sign.  Rescale to the input rho with factors computed from the
            // phase-rotated values, whose rounding varies from step to step.
            const T rho1 = cnorm2(p) + cnorm2(z) + cnorm2(m);
            if (rho1 > (T)0) {
                const T f = dsqrt(rho / rho1);
                p = cscale(p, f); z = cscale(z, f); m = cscale(m, f);
            }
        }
    } else {
        np = cadd(csub(p, cscale(M1p, S1)), cscale(M2p, S2));
        nz = cadd(csub(z, cscale(M1z, S1)), cscale(M2z, S2));
        nm = cadd(csub(m, cscale(M1m, S1)), cscale(M2m, S2));
        const T f = dexp(-t0);
        p = cscale(np, f); z = cscale(nz, f); m = cscale(nm, f);
    }
}

// ---------------------------------------------------------------------------
// Spin-1 eigenbases (unnormalised columns; the inverse carries the factors).
// Sigma_y (x sweep):  nu = +1: u - i sqrt2 psi_0,  nu = 0: v,  nu = -1: u + i sqrt2 psi_0
// Sigma_x (y sweep):  mu = +1: v + sqrt2 psi_0,    mu = 0: u,  mu = -1: v - sqrt2 psi_0
// with u = psi_{+1} - psi_{-1}, v = psi_{+1} + psi_{-1}.  The inverse divides by
// the same rounded sqrt2 that the forward change multiplied with, so that a
// round trip is the identity up to unbiased rounding (a multiplication by a
// rounded sqrt2/4 would shrink psi_0 by a fixed factor at every sweep).
// ---------------------------------------------------------------------------
template <typename T> __device__ inline T kSqrt2() { return (T)1.4142135623730950488; }

template <typename C, typename T> __device__ inline void to_sy(C& p, C& z, C& m) {
    C u = csub(p, m), v = cadd(p, m), w = cscale(ctimes_mi(z), kSqrt2<T>());
    p = cadd(u, w); z = v; m = csub(u, w);
}
template <typename C, typename T> __device__ inline void from_sy(C& a, C& b, C& c) {
    // psi_{+1} = (a + c)/4 + b/2, psi_{-1} = -(a + c)/4 + b/2, psi_0 = i (a - c) / (2 sqrt2)
    const T q = (T)0.25, hb = (T)0.5, s2 = kSqrt2<T>();
    C s = cscale(cadd(a, c), q), d = cscale(csub(a, c), hb), hv = cscale(b, hb);
    C p = cadd(s, hv), m = csub(hv, s), z = ctimes_i(d);
    z.x = z.x / s2; z.y = z.y / s2;
    a = p; b = z; c = m;
}
template <typename C, typename T> __device__ inline void to_sx(C& p, C& z, C& m) {
    C u = csub(p, m), v = cadd(p, m), w = cscale(z, kSqrt2<T>());
    p = cadd(v, w); z = u; m = csub(v, w);
}
template <typename C, typename T> __device__ inline void from_sx(C& a, C& b, C& c) {
    // psi_{+1} = (a + c)/4 + b/2, psi_{-1} = (a + c)/4 - b/2, psi_0 = (a - c) / (2 sqrt2)
    const T q = (T)0.25, hb = (T)0.5, s2 = kSqrt2<T>();
    C s = cscale(cadd(a, c), q), hv = cscale(b, hb), d = cscale(csub(a, c), hb);
    C p = cadd(s, hv), m = csub(s, hv), z = d;
    z.x = z.x / s2; z.y = z.y / s2;
    a = p; b = z; c = m;
}

}  // namespace gp
