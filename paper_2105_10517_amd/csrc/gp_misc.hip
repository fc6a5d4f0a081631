// Small kernels of the SSCN library on gfx950: the stand-alone local substep,
// scaling, norm reductions and the observables, plus their batched forms.
#include <hip/hip_ext.h>

#include "gp_solve.hpp"

namespace gp {

// ---------------------------------------------------------------------------
// Small kernels.
// ---------------------------------------------------------------------------
template <typename T, bool IMAG>
__global__ __launch_bounds__(256) void k_local(cx<T>* __restrict__ psi, size_t sp, Phys ph) {
    const size_t n = (size_t)ph.nx * ph.ny;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % ph.nx), j = (int)(idx / ph.nx);
        const T x = (T)(ph.x0 + i * ph.dx), y = (T)(ph.y0 + j * ph.dy);
        cx<T> p = psi[idx], z = psi[sp + idx], m = psi[2 * sp + idx];
        local_substep<T, IMAG>(p, z, m, trap_v<T>(ph, x, y), (T)ph.dt, (T)ph.c0, (T)ph.c2, (T)ph.rabi);
        psi[idx] = p; psi[sp + idx] = z; psi[2 * sp + idx] = m;
    }
}

// psi[m][0 .. n) *= scale[m] (the gaps between padded planes are not touched)
template <typename T>
__global__ __launch_bounds__(256) void k_scale(cx<T>* __restrict__ psi, size_t n, size_t sp,
                                              const double* __restrict__ scale) {
    const T s[3] = {(T)scale[0], (T)scale[1], (T)scale[2]};
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x)
#pragma unroll
        for (int m = 0; m < 3; ++m) psi[m * sp + idx] = cscale(psi[m * sp + idx], s[m]);
}

// Per-block partial component norms (partials[3 b + m]).
template <typename T>
__global__ __launch_bounds__(256) void k_norm_partials(const cx<T>* __restrict__ psi, size_t n, size_t sp,
                                                      double* __restrict__ partials) {
    __shared__ double shr[48];
    double acc[3] = {0, 0, 0};
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x)
#pragma unroll
        for (int m = 0; m < 3; ++m) acc[m] += (double)cnorm2(psi[m * sp + idx]);
    store_norm_partials(acc, shr, NormOut{partials}, (int)blockIdx.x);
}

__global__ void k_set_scale(double* scale, double v) {
    if (blockIdx.x == 0 && threadIdx.x < 3) scale[threadIdx.x] = v;
}

__global__ void k_set_flag(int* flag, int v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *flag = v;
}

// Sum the per-block partial component norms in a fixed order and turn them
// into the three scale factors (flag on a non-finite or non-positive result).
__device__ inline void finalize_norms(const double* __restrict__ partials, int n, double dxdy, NormRule rule,
                                      double* __restrict__ scale, int* __restrict__ flag, double* shr) {
    double acc[3] = {0, 0, 0};
    for (int k = threadIdx.x; k < n; k += blockDim.x)
#pragma unroll
        for (int m = 0; m < 3; ++m) acc[m] += partials[3 * k + m];
    block_sum3(acc, shr);
    if (threadIdx.x == 0) {
        const double N[3] = {acc[0] * dxdy, acc[1] * dxdy, acc[2] * dxdy};
        if (!norm_scales(N, rule, scale)) *flag = 1;
    }
}

// One block of 1024 threads; each thread keeps four independent sums per
// component, so that sixteen loads are in flight per thread (the partials of
// a 4096^2 grid are about 60 thousand triples).  The order of the additions
// depends only on n.
__global__ __launch_bounds__(1024) void k_norm_finalize(const double* __restrict__ partials, int n, double dxdy,
                                                       NormRule rule, double* __restrict__ scale, int* __restrict__ flag) {
    __shared__ double shr[48];
    // U independent loads per component in flight per thread (guarded, not a
    // tail loop: a 4096^2 grid's ten thousand partials take two rounds)
    constexpr int U = 8;
    const int nt = blockDim.x;
    double a[U][3];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u][0] = a[u][1] = a[u][2] = 0.0;
    for (int k0 = threadIdx.x; k0 < n; k0 += U * nt)
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * nt;
            if (k < n)
#pragma unroll
                for (int m = 0; m < 3; ++m) a[u][m] += partials[3 * k + m];
        }
    double acc[3];
#pragma unroll
    for (int m = 0; m < 3; ++m)
        acc[m] = ((a[0][m] + a[1][m]) + (a[2][m] + a[3][m])) + ((a[4][m] + a[5][m]) + (a[6][m] + a[7][m]));
    block_sum3(acc, shr);
    if (threadIdx.x == 0) {
        const double N[3] = {acc[0] * dxdy, acc[1] * dxdy, acc[2] * dxdy};
        if (!norm_scales(N, rule, scale)) *flag = 1;
    }
}

// ---------------------------------------------------------------------------
// Observables: per-point contributions accumulated in FP64.
// q: 0-2 rho_m, 3 kinetic, 4 trap, 5 interaction, 6 rotation (-Omega <Lz>),
//    7 SO, 8 Rabi, 9 <Lz>, 10-12 Re conj(psi_m) (H psi)_m.
// ---------------------------------------------------------------------------
struct ObsArgs {
    double c0, c2, rabi, gamma, omega;
    int eta;
};

template <typename T>
__global__ __launch_bounds__(256) void k_obs(const cx<T>* __restrict__ psi, size_t sp, Phys ph, ObsArgs oa,
                                            T* __restrict__ dens, double* __restrict__ partials) {
    __shared__ double shr[16];
    const int nx = ph.nx, ny = ph.ny;
    const size_t plane = (size_t)nx * ny;
    const double idx2 = 1.0 / (ph.dx * ph.dx), idy2 = 1.0 / (ph.dy * ph.dy);
    const double i2dx = 0.5 / ph.dx, i2dy = 0.5 / ph.dy;
    const double s2 = 1.4142135623730950488, is2 = 0.70710678118654752440;
    double acc[kObsCount];
#pragma unroll
    for (int q = 0; q < kObsCount; ++q) acc[q] = 0;
    auto ld = [&](int m, int j, int i) -> double2 {
        if (i < 0 || i >= nx || j < 0 || j >= ny) return make_double2(0.0, 0.0);
        const cx<T> z = psi[m * sp + (size_t)j * nx + i];
        return make_double2((double)z.x, (double)z.y);
    };
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < plane; idx += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % nx), j = (int)(idx / nx);
        const double x = ph.x0 + i * ph.dx, y = ph.y0 + j * ph.dy;
        double2 v[3], dxv[3], dyv[3], lap[3];
        for (int m = 0; m < 3; ++m) {
            v[m] = ld(m, j, i);
            const double2 xe = ld(m, j, i + 1), xw = ld(m, j, i - 1), yn = ld(m, j + 1, i), ys = ld(m, j - 1, i);
            dxv[m] = cscale(csub(xe, xw), i2dx);
            dyv[m] = cscale(csub(yn, ys), i2dy);
            lap[m] = cadd(cscale(csub(cadd(xe, xw), cscale(v[m], 2.0)), idx2),
                          cscale(csub(cadd(yn, ys), cscale(v[m], 2.0)), idy2));
            // kinetic: forward differences (plus the ghost-side difference at i = 0, j = 0)
            const double2 gx = csub(xe, v[m]), gy = csub(yn, v[m]);
            double k = cnorm2(gx) * idx2 + cnorm2(gy) * idy2;
            if (i == 0) k += cnorm2(v[m]) * idx2;
            if (j == 0) k += cnorm2(v[m]) * idy2;
            acc[3] += 0.5 * k;
        }
        const double rp = cnorm2(v[0]), r0 = cnorm2(v[1]), rm = cnorm2(v[2]);
        const double rho = rp + r0 + rm;
        const double V = 0.5 * (ph.gx2 * x * x + ph.gy2 * y * y);
        acc[0] += rp; acc[1] += r0; acc[2] += rm;
        acc[4] += V * rho;
        // spin density
        const double Fz = rp - rm;
        const double2 Fp = cscale(cadd(cmulc(v[1], v[0]), cmulc(v[2], v[1])), s2);  // Fx + i Fy
        const double F2 = Fz * Fz + cnorm2(Fp);
        acc[5] += 0.5 * (oa.c0 * rho * rho + oa.c2 * F2);
        acc[8] += oa.rabi * Fp.x;
        // H_loc psi with B = c2 F + R e_x, plus the scalar part
        const double2 Bp = make_double2(oa.c2 * Fp.x + oa.rabi, oa.c2 * Fp.y), Bm = cconj(Bp);
        const double Bz = oa.c2 * Fz;
        double2 Hv[3];
        Hv[0] = cadd(cscale(v[0], Bz), cscale(cmul(Bm, v[1]), is2));
        Hv[1] = cscale(cadd(cmul(Bp, v[0]), cmul(Bm, v[2])), is2);
        Hv[2] = csub(cscale(cmul(Bp, v[1]), is2), cscale(v[2], Bz));
        // SO: i gamma Sigma_y D_x psi - i eta gamma Sigma_x D_y psi
        //   Sigma_y w = i (-w0, w+ - w-, w0)/sqrt2 ; Sigma_x w = (w0, w+ + w-, w0)/sqrt2
        const double g = oa.gamma * is2, ge = oa.gamma * oa.eta * is2;
        double2 so[3];
        // i * i (-dx0) g = g dx0 ; i * i (dx+ - dx-) g = -g (dx+ - dx-) ; i*i dx0 g = -g dx0
        so[0] = csub(cscale(dxv[1], g), cscale(ctimes_i(dyv[1]), ge));
        so[1] = csub(cscale(csub(dxv[0], dxv[2]), -g), cscale(ctimes_i(cadd(dyv[0], dyv[2])), ge));
        so[2] = csub(cscale(dxv[1], -g), cscale(ctimes_i(dyv[1]), ge));
        for (int m = 0; m < 3; ++m) {
            // L_z psi = -i (x D_y - y D_x) psi
            const double2 lz = ctimes_mi(csub(cscale(dyv[m], x), cscale(dxv[m], y)));
            const double lzr = cmulc(lz, v[m]).x;  // Re conj(v) Lz v
            acc[9] += lzr;
            acc[6] += -oa.omega * lzr;
            acc[7] += cmulc(so[m], v[m]).x;
            double2 hm = cadd(cscale(lap[m], -0.5), cscale(v[m], V + oa.c0 * rho));
            hm = cadd(hm, Hv[m]);
            hm = csub(hm, cscale(lz, oa.omega));
            hm = cadd(hm, so[m]);
            acc[10 + m] += cmulc(hm, v[m]).x;
        }
        if (dens) {
            dens[idx] = (T)rp; dens[plane + idx] = (T)r0; dens[2 * plane + idx] = (T)rm;
        }
    }
    for (int q = 0; q < kObsCount; ++q) {
        const double tot = block_sum(acc[q], shr);
        if (threadIdx.x == 0) partials[(size_t)blockIdx.x * kObsCount + q] = tot;
    }
}

__global__ __launch_bounds__(256) void k_obs_finalize(const double* __restrict__ partials, int nblk,
                                                     double* __restrict__ out) {
    __shared__ double shr[16];
    for (int q = 0; q < kObsCount; ++q) {
        double acc = 0;
        for (int k = threadIdx.x; k < nblk; k += blockDim.x) acc += partials[(size_t)k * kObsCount + q];
        const double tot = block_sum(acc, shr);
        if (threadIdx.x == 0) out[q] = tot;
    }
}

// ---------------------------------------------------------------------------
// Batched forms (one launch over many condensates).
// ---------------------------------------------------------------------------
__global__ void k_set_scale_batch(const NSlot* __restrict__ slots, int n, double v) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < 3 * n) slots[s / 3].scale[s % 3] = v;
}

// One block per condensate: its norm totals and scale factors, as k_norm_finalize.
__global__ __launch_bounds__(256) void k_norm_finalize_batch(const NSlot* __restrict__ slots) {
    __shared__ double shr[48];
    const NSlot& s = slots[blockIdx.x];
    finalize_norms(s.partials, s.n, s.dxdy, s.rule, s.scale, s.flag, shr);
}

// Block b scales chunk (map & mask) of kScaleChunk values of condensate (map >> shift).
template <typename T>
__global__ __launch_bounds__(256) void k_scale_batch(const SSlot<T>* __restrict__ slots, const unsigned* __restrict__ map) {
    const unsigned e = map[blockIdx.x];
    const SSlot<T>& s = slots[e >> kMapShift];
    const size_t base = (size_t)(e & kMapMask) * kScaleChunk;
    const T f[3] = {(T)s.scale[0], (T)s.scale[1], (T)s.scale[2]};
    for (int k = threadIdx.x; k < kScaleChunk; k += blockDim.x) {
        const size_t i = base + k;
        if (i < 3 * s.n) {
            const size_t m = i / s.n, o = m * s.stride + (i - m * s.n);
            s.psi[o] = cscale(s.psi[o], f[m]);
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_local(cx<T>* psi, size_t sp, const Phys& ph, bool imag, hipStream_t st) {
    const size_t n = (size_t)ph.nx * ph.ny;
    const int nblk = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    if (imag) k_local<T, true><<<nblk, 256, 0, st>>>(psi, sp, ph);
    else k_local<T, false><<<nblk, 256, 0, st>>>(psi, sp, ph);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale(cx<T>* psi, size_t n, size_t sp, const double* scale, hipStream_t st, hipEvent_t e0,
                        hipEvent_t e1) {
    const int nblk = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    hipExtLaunchKernelGGL(k_scale<T>, dim3(nblk), dim3(256), 0, st, e0, e1, 0, psi, n, sp, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_norm_partials(const cx<T>* psi, size_t n, size_t sp, double* partials, int nblk, hipStream_t st) {
    k_norm_partials<T><<<nblk, 256, 0, st>>>(psi, n, sp, partials);
    return hipGetLastError();
}

hipError_t launch_set_scale(double* scale, double v, hipStream_t st) {
    k_set_scale<<<1, 64, 0, st>>>(scale, v);
    return hipGetLastError();
}

hipError_t launch_set_flag(int* flag, int v, hipStream_t st) {
    k_set_flag<<<1, 64, 0, st>>>(flag, v);
    return hipGetLastError();
}

hipError_t launch_norm_finalize(const double* partials, int n, double dxdy, NormRule rule, double* scale, int* flag,
                                hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    hipExtLaunchKernelGGL(k_norm_finalize, dim3(1), dim3(1024), 0, st, e0, e1, 0, partials, n, dxdy, rule, scale, flag);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_obs(const cx<T>* psi, size_t sp, const Phys& ph, const ObsLaunch& o, T* dens, double* partials,
                      int nblk, hipStream_t st) {
    ObsArgs oa{o.c0, o.c2, o.rabi, o.gamma, o.omega, o.eta};
    k_obs<T><<<nblk, 256, 0, st>>>(psi, sp, ph, oa, dens, partials);
    return hipGetLastError();
}

hipError_t launch_obs_finalize(const double* partials, int nblk, double* out, hipStream_t st) {
    k_obs_finalize<<<1, 256, 0, st>>>(partials, nblk, out);
    return hipGetLastError();
}

hipError_t launch_set_scale_batch(const NSlot* slots, int n, double v, hipStream_t st) {
    if (n <= 0) return hipErrorInvalidValue;
    k_set_scale_batch<<<(3 * n + 255) / 256, 256, 0, st>>>(slots, n, v);
    return hipGetLastError();
}

hipError_t launch_norm_finalize_batch(const NSlot* slots, int n, hipStream_t st) {
    if (n <= 0) return hipErrorInvalidValue;
    k_norm_finalize_batch<<<n, 256, 0, st>>>(slots);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_batch(const SSlot<T>* slots, const unsigned* map, int nblk, hipStream_t st) {
    if (nblk <= 0) return hipErrorInvalidValue;
    k_scale_batch<T><<<nblk, 256, 0, st>>>(slots, map);
    return hipGetLastError();
}

#define GP_INST(T)                                                                                             \
    template hipError_t launch_local<T>(cx<T>*, size_t, const Phys&, bool, hipStream_t);                       \
    template hipError_t launch_scale<T>(cx<T>*, size_t, size_t, const double*, hipStream_t, hipEvent_t,        \
                                        hipEvent_t);                                                           \
    template hipError_t launch_norm_partials<T>(const cx<T>*, size_t, size_t, double*, int, hipStream_t);      \
    template hipError_t launch_obs<T>(const cx<T>*, size_t, const Phys&, const ObsLaunch&, T*, double*, int,     \
                                      hipStream_t);                                                               \
    template hipError_t launch_scale_batch<T>(const SSlot<T>*, const unsigned*, int, hipStream_t);
GP_INST(double)
GP_INST(float)

}  // namespace gp
