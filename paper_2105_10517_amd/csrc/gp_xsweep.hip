// x sweep of the SSCN step on gfx950: the local substep (and a pending
// imaginary-time renormalisation) fused into the x Crank-Nicolson sweep.  One
// row per thread group, K consecutive points per thread in registers, exact
// partitioned Thomas (local recurrences + wave/LDS scans of the block
// carries).  k_x_scan serves one condensate; k_x_batch one launch over the
// rows of many condensates (a block map names each block's condensate).
#include <hip/hip_ext.h>

#include <algorithm>
#include <climits>

#include "gp_chain.hpp"

namespace gp {

// One block of the x sweep: rows row0 .. row0 + R - 1 below rlim of one
// condensate, G threads per row (threads past G R idle through the barriers).
// PF: load the line-start correction's factors before the solve (more
// registers, no load at the end of the row's chain).
template <typename T, bool IMAG, int K, bool LOCAL, bool SCALE, bool PF>
__device__ inline void x_rows(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, size_t sp, size_t dp, const Phys& ph,
                              const LineSet<T>& ls, const double* __restrict__ scale, NormIn nin, int G, int R,
                              int row0, int rlim) {
    using C = cx<T>;
    // scan totals: [direction][line][P (16 waves) | E (16 waves)]
    __shared__ C shS[2 * 3 * 32];
    __shared__ C shN[2 * 3 * 16];
    const int tid = threadIdx.x;
    const int r = tid / G, t = tid - r * G;
    const int lane = t & 63, w = t >> 6, nw = G >> 6;
    const int j = row0 + r;
    const bool row_ok = r < R && j < rlim;
    const int nx = ph.nx;
    const int i0 = t * K;
    const int jl = row_ok ? j : 0;
    const size_t rowoff = (size_t)(row_ok ? j : 0) * nx;
    const C* rowp = src + rowoff;
    C* rowq = dst + rowoff;
    C v[3][K];
    if (row_ok && i0 + K <= nx) {
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k) v[m][k] = rowp[m * sp + i0 + k];
    } else {
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k)
                v[m][k] = (row_ok && i0 + k < nx) ? rowp[m * sp + i0 + k] : zero_c<C>();
    }
    // the lines' coefficients, loaded with the row (before the barriers below)
    LineCoef<T> cf[3];
    line_coefs<T, 3>(ls, jl * 3, cf);
    if (SCALE) {
        double sc[3];
        if (nin.partials != nullptr) {
            // the scale factors from the previous y sweep's partials (same order in every block)
            __shared__ double shr3[48];
            __shared__ double shs[3];
            double acc[3] = {0, 0, 0};
            for (int k = tid; k < nin.n; k += blockDim.x)
#pragma unroll
                for (int m = 0; m < 3; ++m) acc[m] += nin.partials[3 * k + m];
            block_sum3(acc, shr3);
            if (tid == 0) {
                const double N[3] = {acc[0] * nin.dxdy, acc[1] * nin.dxdy, acc[2] * nin.dxdy};
                double f[3];
                if (!norm_scales(N, nin.rule, f)) *nin.flag = 1;
                shs[0] = f[0]; shs[1] = f[1]; shs[2] = f[2];
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 3; ++m) sc[m] = shs[m];
        } else {
#pragma unroll
            for (int m = 0; m < 3; ++m) sc[m] = scale[m];
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const T s = (T)sc[m];
#pragma unroll
            for (int k = 0; k < K; ++k) v[m][k] = cscale(v[m][k], s);
        }
    }
    if (LOCAL) {
        const T y = (T)(ph.y0 + (row_ok ? j : 0) * ph.dy);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T x = (T)(ph.x0 + (i0 + k) * ph.dx);
            local_substep<T, IMAG>(v[0][k], v[1][k], v[2][k], trap_v<T>(ph, x, y), (T)ph.dtl, (T)ph.c0,
                                   (T)ph.c2, (T)ph.rabi);
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) to_sy<C, T>(v[0][k], v[1][k], v[2][k]);
    // the line-start correction's factors, loaded before the solve (wave 0
    // holds every corrected point), so that the fix after it waits on no load
    C gcf[3], gk[3][K];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        gcf[q] = zero_c<C>();
#pragma unroll
        for (int k = 0; k < K; ++k) gk[q][k] = zero_c<C>();
    }
    if (PF && sizeof(T) * K <= 32 && w == 0 && i0 < ls.Kg) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            gcf[q] = ls.gc[jl * 3 + q];
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (i0 + k < ls.Kg) gk[q][k] = ls.g[(size_t)(jl * 3 + q) * ls.Kg + i0 + k];
        }
    }
    // neighbours of the block ends for all three components (ghost zeros beyond the row)
    C left[3], right[3];
    const int nrow = r * nw;  // first wave of this row in the block
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        left[q] = shfl_up_c(v[q][K - 1], 1);
        right[q] = shfl_down_c(v[q][0], 1);
        if (lane == 63) shN[(nrow + w) * 3 + q] = v[q][K - 1];
        if (lane == 0) shN[48 + (nrow + w) * 3 + q] = v[q][0];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        if (lane == 0) left[q] = (w > 0) ? shN[(nrow + w - 1) * 3 + q] : zero_c<C>();
        if (lane == 63) right[q] = (w + 1 < nw) ? shN[48 + (nrow + w + 1) * 3 + q] : zero_c<C>();
    }
    if constexpr (sizeof(T) * K <= 32) {
        // the three lines' chains interleaved (fits the register file for small blocks)
        auto fs = [&](const C (&P)[3], const C (&E)[3], C (&o)[3]) {
            row_scan<true, 3>(P, E, o, lane, w, nw, ScanShm<C>{shS + nrow});
        };
        auto bs = [&](const C (&P)[3], const C (&E)[3], C (&o)[3]) {
            row_scan<false, 3>(P, E, o, lane, w, nw, ScanShm<C>{shS + 3 * 32 + nrow});
        };
        C d[3];
        block_solve<T, K, IMAG, 3>(v, left, right, ls, cf, i0, nx, fs, bs, 0, d);
        // line-start correction with the increment at point 0 (thread 0 of the row);
        // the host keeps every corrected point in the row's first wave (Kg <= 64 K)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const C d0 = bperm_c(d[q], 0);  // lane 0 of this wave
            if (PF) {
                if (w == 0 && i0 < ls.Kg) {
                    const C f = cmul(gcf[q], d0);
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (i0 + k < ls.Kg) v[q][k] = csub(v[q][k], cmul(f, gk[q][k]));
                }
            } else if (w == 0) {
                line_start_fix<T, K>(v[q], ls, jl * 3 + q, d0, i0);
            }
        }
    } else {
        // one line after the other
        C* sa = shS + nrow;
        C* sb = shS + 16 + nrow;
        auto fs = [&](C P, C E) { return row_scan1<true>(P, E, lane, w, nw, sa, sb); };
        auto bs = [&](C P, C E) { return row_scan1<false>(P, E, lane, w, nw, sa, sb); };
#pragma unroll
        for (int q = 0; q < 3; ++q) block_solve1<T, K, IMAG>(v[q], left[q], right[q], ls, jl * 3 + q, i0, nx, fs, bs);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) from_sy<C, T>(v[0][k], v[1][k], v[2][k]);
    if (row_ok && i0 + K <= nx) {
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k) rowq[m * dp + i0 + k] = v[m][k];
    } else if (row_ok) {
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (i0 + k < nx) rowq[m * dp + i0 + k] = v[m][k];
    }
}

// ---------------------------------------------------------------------------
// x sweep over truncated windows (the y sweep's scheme turned along the rows):
// a wave holds 4 rows, each DPP row of 16 lanes the 16 segments of one row
// window, each lane KX consecutive points; windows of 16 KX points overlap by
// h points on each side and write their middle L = 16 KX - 2 h points, h such
// that the carries dropped at the window ends have decayed below the rounding
// level.  No shared memory and no barriers; the windows at the row start
// apply the line-start correction.  The local substep and the pending scale
// are applied to every point loaded, halo included.
// ---------------------------------------------------------------------------
template <typename T, bool IMAG, int KX, int NW, bool SEQ, bool LOCAL, bool SCALE>
__device__ inline void x_window(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, size_t sp, size_t dp, const Phys& ph,
                                const LineSet<T>& ls, const double* __restrict__ scale, int L, int h, int cs, int rt,
                                int rlo, int rhi) {
    using C = cx<T>;
    constexpr int RPB = 4 * NW;  // rows per block
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int seg = lane & 15, rw = lane >> 4;
    const int j = rt * RPB + wv * 4 + rw;
    const bool row_ok = j >= rlo && j < rhi;  // rows of this block's group that it owns
    const int nx = ph.nx;
    const int i0 = cs * L;           // first point written by this window
    const int g0 = i0 - h + seg * KX;  // first point of this lane
    const int jl = row_ok ? j : 0;
    const C* rowp = src + (size_t)jl * nx;
    C v[3][KX];
#pragma unroll
    for (int k = 0; k < KX; ++k) {
        const int g = g0 + k;
        const bool ok = row_ok && g >= 0 && g < nx;
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m][k] = ok ? rowp[m * sp + (ok ? g : 0)] : zero_c<C>();
    }
    if (SCALE) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const T s = (T)scale[m];
#pragma unroll
            for (int k = 0; k < KX; ++k) v[m][k] = cscale(v[m][k], s);
        }
    }
    if (LOCAL) {
        const T y = (T)(ph.y0 + jl * ph.dy);
#pragma unroll
        for (int k = 0; k < KX; ++k) {
            const T x = (T)(ph.x0 + (g0 + k) * ph.dx);
            local_substep<T, IMAG>(v[0][k], v[1][k], v[2][k], trap_v<T>(ph, x, y), (T)ph.dtl, (T)ph.c0, (T)ph.c2,
                                   (T)ph.rabi);
        }
    }
#pragma unroll
    for (int k = 0; k < KX; ++k) to_sy<C, T>(v[0][k], v[1][k], v[2][k]);
    // the windows holding point 0 of their rows apply the line-start correction
    // (block-uniform); point 0 sits h - i0 points into the window
    const int off0 = h - i0;
    window_solve<T, KX, IMAG, SEQ>(v, ls, jl * 3, g0, nx, off0 >= 0, off0 / KX, off0 % KX, lane);
#pragma unroll
    for (int k = 0; k < KX; ++k) from_sy<C, T>(v[0][k], v[1][k], v[2][k]);
    C* rowq = dst + (size_t)jl * nx;
#pragma unroll
    for (int k = 0; k < KX; ++k) {
        const int g = g0 + k;
        if (row_ok && g >= i0 && g < i0 + L && g < nx)
#pragma unroll
            for (int m = 0; m < 3; ++m) rowq[m * dp + g] = v[m][k];
    }
}

template <typename T, bool IMAG, int KX, int NW, bool SEQ, bool LOCAL, bool SCALE>
__global__ __launch_bounds__(64 * NW) void k_x_window(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst,
                                                      size_t sp, size_t dp, Phys ph, LineSet<T> ls, const double* __restrict__ scale, int L,
                                                      int h, int ncs, int nblk, int order, int bL, int bnrt) {
    constexpr int RPB = 4 * NW;
    int cs, rt, rlo = 0, rhi = ph.ny;
    if (order == 3 && bL > 0) {
        // row bands: XCD (b mod 8) takes the row groups overlapping its rows, all windows of each,
        // and computes only its own rows of a group shared with the next band
        const int jb = (int)blockIdx.x / kNumXcd;
        band_rows((int)blockIdx.x % kNumXcd, bnrt, bL, ph.ny, rlo, rhi);
        const int g0 = rlo / RPB, g1 = (rhi + RPB - 1) / RPB;
        if (jb >= (g1 - g0) * ncs) return;
        rt = g0 + jb / ncs;
        cs = jb % ncs;
    } else {
        const int lb = order_logical(order ? 1 : 0, (int)blockIdx.x, ncs, nblk / ncs);
        if (lb < 0) return;
        cs = lb % ncs;
        rt = lb / ncs;
    }
    x_window<T, IMAG, KX, NW, SEQ, LOCAL, SCALE>(src, dst, sp, dp, ph, ls, scale, L, h, cs, rt, rlo, rhi);
}

// A double that is the same in every lane, moved to scalar registers.
__device__ inline double wave_uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)b), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ---------------------------------------------------------------------------
// x sweep over chain windows (gp_chain.hpp): one row segment of W = 64 K
// points per wave, K consecutive points per lane, carries over nc lanes; the
// window starting at point cs L - h writes the points [cs L, cs L + L),
// L = W - 2 h.  Windows at the row ends take the EDGE path; the first window
// of a row also applies the line-start correction (point 0 is the window's
// point h).  Waves are independent (no shared memory, no barrier): wave w of
// logical block lb takes window lb NW + w of the row-major window list.
// ---------------------------------------------------------------------------
// One wave's window: wave gw of the sweep takes window gw mod nwin of row
// gw / nwin.
template <typename T, bool IMAG, int K, bool SEQ, bool LOCAL, bool SCALE>
__device__ __attribute__((always_inline)) inline void x_chain_wave(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, size_t sp, size_t dp,
                                    const Phys& ph, const LineSet<T>& ls, const double* __restrict__ scale,
                                    const NormIn& nin, int h, int nc, int L, int nwin, int gw) {
    using C = cx<T>;
    const int lane = threadIdx.x & 63;
    const int nx = ph.nx;
    // The window index is the same in every lane of the wave.  Said so (FP64),
    // the window's row, line coefficients and row base live in scalar
    // registers: 130 instead of 152 vector registers at 4 points per lane, 78
    // instead of 126 at 2 points (6 waves per SIMD instead of 3), and the
    // 2-point windows then run ~15% faster at 4096^2.  FP32 measured ~2%
    // slower with it (66 instead of 78 registers) and keeps the lane values.
    if constexpr (sizeof(T) == 8) gw = __builtin_amdgcn_readfirstlane(gw);
    if (gw >= nwin * ph.ny) return;  // whole waves
    const int j = gw / nwin, cs = gw - j * nwin;
    const int i0 = cs * L;           // first point written
    const int s0 = i0 - h;           // first point of the window
    const int g0 = s0 + lane * K;    // first point of this lane
    const C* rowp = src + (size_t)j * nx;
    const bool edge = s0 < 0 || s0 + 64 * K > nx;  // wave-uniform
    // the pending scale factors, formed before the loads and held in scalar
    // registers (the same in every lane)
    double sc[3] = {1.0, 1.0, 1.0};
    int bad = 0;  // a non-finite norm total (flagged at the end: a store here would
                  // keep the later loads of the line tables off the scalar path)
    if (SCALE) {
        if (nin.partials != nullptr) {
            // from the previous y sweep's few partials (total norm one; the host
            // folds no other rule here), summed by every wave in the same order:
            // lane sums, then an xor butterfly (commutative at each stage, so
            // every lane holds the same total)
            double acc[3] = {0, 0, 0};
            for (int k = lane; k < nin.n; k += 64)
#pragma unroll
                for (int m = 0; m < 3; ++m) acc[m] += nin.partials[3 * k + m];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
                for (int m = 0; m < 3; ++m) acc[m] += __shfl_xor(acc[m], o, 64);
            const double N[3] = {acc[0] * nin.dxdy, acc[1] * nin.dxdy, acc[2] * nin.dxdy};
            bad = __builtin_amdgcn_readfirstlane(norm_scale_total(N, sc) ? 0 : 1);
#pragma unroll
            for (int m = 0; m < 3; ++m) sc[m] = wave_uniform(sc[m]);
        } else {
#pragma unroll
            for (int m = 0; m < 3; ++m) sc[m] = scale[m];
        }
    }
    C v[3][K];
    if (!edge) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int m = 0; m < 3; ++m) v[m][k] = rowp[m * sp + g0 + k];
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int g = g0 + k;
            const bool ok = g >= 0 && g < nx;
#pragma unroll
            for (int m = 0; m < 3; ++m) v[m][k] = ok ? rowp[m * sp + (ok ? g : 0)] : zero_c<C>();
        }
    }
    if (SCALE) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const T f = (T)sc[m];
#pragma unroll
            for (int k = 0; k < K; ++k) v[m][k] = cscale(v[m][k], f);
        }
    }
    if (LOCAL) {
        const T y = (T)(ph.y0 + j * ph.dy);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T x = (T)(ph.x0 + (g0 + k) * ph.dx);
            local_substep<T, IMAG>(v[0][k], v[1][k], v[2][k], trap_v<T>(ph, x, y), (T)ph.dtl, (T)ph.c0, (T)ph.c2,
                                   (T)ph.rabi);
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) to_sy<C, T>(v[0][k], v[1][k], v[2][k]);
    if (!edge) chain_lines<T, K, IMAG, true, false, SEQ>(v, ls, j * 3, nc, g0, nx, false, 0, 0);
    else chain_lines<T, K, IMAG, true, true, SEQ>(v, ls, j * 3, nc, g0, nx, cs == 0, h / K, h % K);
#pragma unroll
    for (int k = 0; k < K; ++k) from_sy<C, T>(v[0][k], v[1][k], v[2][k]);
    C* rowq = dst + (size_t)j * nx;
    const int i1 = min(i0 + L, nx);
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (g0 + k >= i0 && g0 + k < i1)
#pragma unroll
            for (int m = 0; m < 3; ++m) rowq[m * dp + g0 + k] = v[m][k];
    if (bad) *nin.flag = 1;  // (the same value from every lane)
}

template <typename T, bool IMAG, int K, int NW, bool SEQ, bool LOCAL, bool SCALE>
__global__ __launch_bounds__(64 * NW) void k_x_chain(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst,
                                                     size_t sp, size_t dp, Phys ph, LineSet<T> ls,
                                                     const double* __restrict__ scale, NormIn nin, int h, int nc, int L,
                                                     int nwin, int nblk, int order) {
    const int lb = order_logical(order ? 1 : 0, (int)blockIdx.x, nblk, 1);
    if (lb < 0) return;
    x_chain_wave<T, IMAG, K, SEQ, LOCAL, SCALE>(src, dst, sp, dp, ph, ls, scale, nin, h, nc, L, nwin,
                                                lb * NW + (int)(threadIdx.x >> 6));
}

// Many condensates in one launch: map entry b names the condensate and its
// block, NW waves of that condensate's windows (local substep and pending
// scale fused as in the single sweep).
template <typename T, bool IMAG, int K, int NW, bool SEQ>
__global__ __launch_bounds__(64 * NW) void k_x_chain_batch(const XCSlot<T>* __restrict__ slots,
                                                           const unsigned* __restrict__ map) {
    const unsigned e = map[blockIdx.x];
    const XCSlot<T>& s = slots[e >> kMapShift];
    x_chain_wave<T, IMAG, K, SEQ, true, IMAG>(s.src, s.dst, s.sp, s.dp, s.ph, s.ls, s.scale,
                                              NormIn{nullptr, 0, 0.0, NormRule{0, 0.0}, nullptr}, s.h, s.nc, s.L, s.nwin,
                                              (int)(e & kMapMask) * NW + (int)(threadIdx.x >> 6));
}

template <typename T, bool IMAG, int K, bool LOCAL, bool SCALE, int LB>
__global__ __launch_bounds__(LB) void k_x_scan(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, size_t sp,
                                               size_t dp, Phys ph,
                                               LineSet<T> ls, const double* __restrict__ scale, NormIn nin, int G,
                                               int R, int bL, int bnrt) {
    int row0 = (int)blockIdx.x * R, rlim = ph.ny;
    if (bL > 0) {
        // row bands: XCD (b mod 8) takes the rows of its y row tiles, R at a time
        int r0, r1;
        band_rows((int)blockIdx.x % kNumXcd, bnrt, bL, ph.ny, r0, r1);
        row0 = r0 + (int)blockIdx.x / kNumXcd * R;
        rlim = r1;
        if (row0 >= rlim) return;
    }
    x_rows<T, IMAG, K, LOCAL, SCALE, true>(src, dst, sp, dp, ph, ls, scale, nin, G, R, row0, rlim);
}

template <typename T, bool IMAG, int K, int LB>
__global__ __launch_bounds__(LB) void k_x_batch(const XSlot<T>* __restrict__ slots, const unsigned* __restrict__ map) {
    const unsigned e = map[blockIdx.x];
    const XSlot<T>& s = slots[e >> kMapShift];
    // (many condensates fill the chip: the batch keeps the smaller register footprint)
    x_rows<T, IMAG, K, true, IMAG, false>(s.src, s.dst, s.sp, s.dp, s.ph, s.ls, s.scale, NormIn{nullptr, 0, 0.0, NormRule{0, 0.0}, nullptr},
                                   s.G, s.R, (int)(e & kMapMask) * s.R, s.ph.ny);
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <typename T, bool IMAG, bool LOCAL, bool SCALE>
static hipError_t launch_x_k(int K, const cx<T>* src, cx<T>* dst, size_t sp, size_t dp, const Phys& ph, const LineSet<T>& ls,
                             const double* scale, NormIn nin, int G, int R, int bL, int bnrt, hipStream_t st,
                             hipEvent_t e0, hipEvent_t e1) {
    // the line-start correction of the three-line path must lie in each row's first wave
    if (sizeof(T) * K <= 32 && ls.Kg > 64 * K) return hipErrorInvalidValue;
    int nblk = (ph.ny + R - 1) / R;
    if (bL > 0) {
        if (bnrt <= 0 || (long)bL * bnrt < ph.ny) return hipErrorInvalidValue;
        int most = 0;
        for (int x = 0; x < kNumXcd; ++x) {
            int r0, r1;
            band_rows(x, bnrt, bL, ph.ny, r0, r1);
            most = std::max(most, (r1 - r0 + R - 1) / R);
        }
        nblk = kNumXcd * std::max(most, 1);
    }
    const dim3 grid(nblk), block(G * R);
    if (G * R > xk_bound(K) || G % 64 || G / 64 > 16 || R > 8) return hipErrorInvalidValue;

    switch (K) {
        case 1: hipExtLaunchKernelGGL(k_x_scan<T, IMAG, 1, LOCAL, SCALE, xk_bound(1)>, grid, block, 0, st, e0, e1, 0, src, dst, sp, dp, ph, ls, scale, nin, G, R, bL, bnrt); break;
        case 2: hipExtLaunchKernelGGL(k_x_scan<T, IMAG, 2, LOCAL, SCALE, xk_bound(2)>, grid, block, 0, st, e0, e1, 0, src, dst, sp, dp, ph, ls, scale, nin, G, R, bL, bnrt); break;
        case 4: hipExtLaunchKernelGGL(k_x_scan<T, IMAG, 4, LOCAL, SCALE, xk_bound(4)>, grid, block, 0, st, e0, e1, 0, src, dst, sp, dp, ph, ls, scale, nin, G, R, bL, bnrt); break;
        case 8: hipExtLaunchKernelGGL(k_x_scan<T, IMAG, 8, LOCAL, SCALE, xk_bound(8)>, grid, block, 0, st, e0, e1, 0, src, dst, sp, dp, ph, ls, scale, nin, G, R, bL, bnrt); break;
        case 16: hipExtLaunchKernelGGL(k_x_scan<T, IMAG, 16, LOCAL, SCALE, xk_bound(16)>, grid, block, 0, st, e0, e1, 0, src, dst, sp, dp, ph, ls, scale, nin, G, R, bL, bnrt); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool IMAG, bool LOCAL, bool SCALE, int TI>
static hipError_t launch_xw_t(const XLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    constexpr YTile xt = ytile<T>(TI);
    const int ncs = (a.ph.nx + a.L - 1) / a.L;
    const int nrt = (a.ph.ny + 4 * xt.NW - 1) / (4 * xt.NW);
    const int nblk = ncs * nrt;
    const bool bands = a.order == 3 && a.bL > 0;
    int grid = xcd_grid(a.order ? 1 : 0, ncs, nrt);
    if (bands) {
        if (a.bnrt <= 0 || (long)a.bL * a.bnrt < a.ph.ny) return hipErrorInvalidValue;
        int most = 0;
        for (int x = 0; x < kNumXcd; ++x) {
            int r0, r1;
            band_rows(x, a.bnrt, a.bL, a.ph.ny, r0, r1);
            most = std::max(most, (r1 + 4 * xt.NW - 1) / (4 * xt.NW) - r0 / (4 * xt.NW));
        }
        grid = kNumXcd * std::max(most, 1) * ncs;
    }
    hipExtLaunchKernelGGL(k_x_window<T, IMAG, xt.KY, xt.NW, xt.SEQ, LOCAL, SCALE>, dim3(grid),
                          dim3(64 * xt.NW), 0, st, e0, e1, 0, a.src, a.dst, a.sp, a.dp, a.ph, a.ls, a.scale, a.L, a.h, ncs, nblk,
                          a.order, a.bL, a.bnrt);
    return hipGetLastError();
}

template <typename T, bool IMAG, bool LOCAL, bool SCALE>
static hipError_t launch_xw(const XLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    switch (a.tile) {
        case 0: return launch_xw_t<T, IMAG, LOCAL, SCALE, 0>(a, st, e0, e1);
        case 1: return launch_xw_t<T, IMAG, LOCAL, SCALE, 1>(a, st, e0, e1);
        case 2: return launch_xw_t<T, IMAG, LOCAL, SCALE, 2>(a, st, e0, e1);
        case 3: return launch_xw_t<T, IMAG, LOCAL, SCALE, 3>(a, st, e0, e1);
        case 4: return launch_xw_t<T, IMAG, LOCAL, SCALE, 4>(a, st, e0, e1);
        case 5: return launch_xw_t<T, IMAG, LOCAL, SCALE, 5>(a, st, e0, e1);
        case 6: return launch_xw_t<T, IMAG, LOCAL, SCALE, 6>(a, st, e0, e1);
        case 7: return launch_xw_t<T, IMAG, LOCAL, SCALE, 7>(a, st, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, bool IMAG, bool LOCAL, bool SCALE, int TI>
static hipError_t launch_xc_t(const XLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    constexpr ChainTile ct = xchain_tile<T>(TI);
    // the window (64 K points) writes L = 64 K - 2 h of them; the first window holds the corrected points
    if (a.h < 1 || a.L != 64 * ct.K - 2 * a.h || a.L <= 0 || a.ls.Kg > a.L) return hipErrorInvalidValue;
    const int nwin = (a.ph.nx + a.L - 1) / a.L;
    const long nwav = (long)nwin * a.ph.ny;
    if ((nwav + ct.NW - 1) / ct.NW > INT_MAX / 2) return hipErrorInvalidValue;
    const int nblk = (int)((nwav + ct.NW - 1) / ct.NW);
    const int grid = a.order ? xcd_blocks(nblk) : nblk;
    hipExtLaunchKernelGGL(k_x_chain<T, IMAG, ct.K, ct.NW, ct.SEQ, LOCAL, SCALE>, dim3(grid), dim3(64 * ct.NW), 0, st, e0,
                          e1, 0, a.src, a.dst, a.sp, a.dp, a.ph, a.ls, a.scale, a.nin, a.h, chain_lanes(a.h, ct.K), a.L,
                          nwin, nblk, a.order);
    return hipGetLastError();
}

template <typename T, bool IMAG, bool LOCAL, bool SCALE>
static hipError_t launch_xc(const XLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    switch (a.tile) {
        case 0: return launch_xc_t<T, IMAG, LOCAL, SCALE, 0>(a, st, e0, e1);
        case 1: return launch_xc_t<T, IMAG, LOCAL, SCALE, 1>(a, st, e0, e1);
        case 2: return launch_xc_t<T, IMAG, LOCAL, SCALE, 2>(a, st, e0, e1);
        case 3: return launch_xc_t<T, IMAG, LOCAL, SCALE, 3>(a, st, e0, e1);
        case 4: return launch_xc_t<T, IMAG, LOCAL, SCALE, 4>(a, st, e0, e1);
        case 5: return launch_xc_t<T, IMAG, LOCAL, SCALE, 5>(a, st, e0, e1);
        case 6: return launch_xc_t<T, IMAG, LOCAL, SCALE, 6>(a, st, e0, e1);
        case 7: return launch_xc_t<T, IMAG, LOCAL, SCALE, 7>(a, st, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_x(const XLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (a.chain) {
        // (the scale factors come from `scale`, or from a few norm partials
        // under the total-norm rule, summed by every wave)
        if (a.nin.partials != nullptr && (!a.imag || !a.local || a.nin.rule.fix_m || 3 * a.nin.n > 8 * 64))
            return hipErrorInvalidValue;
        if (a.imag) return a.local ? launch_xc<T, true, true, true>(a, st, e0, e1) : launch_xc<T, true, false, false>(a, st, e0, e1);
        return a.local ? launch_xc<T, false, true, false>(a, st, e0, e1) : launch_xc<T, false, false, false>(a, st, e0, e1);
    }
    if (a.window) {
        // the windowed kernel takes its scale factors from `scale` (the norm totals are formed beforehand)
        if (a.nin.partials != nullptr) return hipErrorInvalidValue;
        if (a.imag) return a.local ? launch_xw<T, true, true, true>(a, st, e0, e1) : launch_xw<T, true, false, false>(a, st, e0, e1);
        return a.local ? launch_xw<T, false, true, false>(a, st, e0, e1) : launch_xw<T, false, false, false>(a, st, e0, e1);
    }
    if (a.imag) {
        if (a.local) return launch_x_k<T, true, true, true>(a.K, a.src, a.dst, a.sp, a.dp, a.ph, a.ls, a.scale, a.nin, a.G, a.R, a.order == 3 ? a.bL : 0, a.bnrt, st, e0, e1);
        return launch_x_k<T, true, false, false>(a.K, a.src, a.dst, a.sp, a.dp, a.ph, a.ls, a.scale, a.nin, a.G, a.R, a.order == 3 ? a.bL : 0, a.bnrt, st, e0, e1);
    }
    if (a.local) return launch_x_k<T, false, true, false>(a.K, a.src, a.dst, a.sp, a.dp, a.ph, a.ls, a.scale, a.nin, a.G, a.R, a.order == 3 ? a.bL : 0, a.bnrt, st, e0, e1);
    return launch_x_k<T, false, false, false>(a.K, a.src, a.dst, a.sp, a.dp, a.ph, a.ls, a.scale, a.nin, a.G, a.R, a.order == 3 ? a.bL : 0, a.bnrt, st, e0, e1);
}

template <typename T, bool IMAG>
static hipError_t launch_x_batch_t(const XSlot<T>* slots, const unsigned* map, int nblk, int K, int block,
                                   hipStream_t st) {
    if (block > xk_bound(K) || block % 64 || block > 1024 || nblk <= 0) return hipErrorInvalidValue;
    const dim3 grid(nblk), blk(block);
    switch (K) {
        case 1: hipExtLaunchKernelGGL(k_x_batch<T, IMAG, 1, xk_bound(1)>, grid, blk, 0, st, nullptr, nullptr, 0, slots, map); break;
        case 2: hipExtLaunchKernelGGL(k_x_batch<T, IMAG, 2, xk_bound(2)>, grid, blk, 0, st, nullptr, nullptr, 0, slots, map); break;
        case 4: hipExtLaunchKernelGGL(k_x_batch<T, IMAG, 4, xk_bound(4)>, grid, blk, 0, st, nullptr, nullptr, 0, slots, map); break;
        case 8: hipExtLaunchKernelGGL(k_x_batch<T, IMAG, 8, xk_bound(8)>, grid, blk, 0, st, nullptr, nullptr, 0, slots, map); break;
        case 16: hipExtLaunchKernelGGL(k_x_batch<T, IMAG, 16, xk_bound(16)>, grid, blk, 0, st, nullptr, nullptr, 0, slots, map); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool IMAG, int TI>
static hipError_t launch_xc_batch_t(const XCSlot<T>* slots, const unsigned* map, int nblk, hipStream_t st) {
    constexpr ChainTile ct = xchain_tile<T>(TI);
    hipExtLaunchKernelGGL(k_x_chain_batch<T, IMAG, ct.K, ct.NW, ct.SEQ>, dim3(nblk), dim3(64 * ct.NW), 0, st, nullptr,
                          nullptr, 0, slots, map);
    return hipGetLastError();
}

template <typename T, bool IMAG>
static hipError_t launch_xc_batch_i(const XCSlot<T>* slots, const unsigned* map, int nblk, int tile, hipStream_t st) {
    if (nblk <= 0) return hipErrorInvalidValue;
    switch (tile) {
        case 0: return launch_xc_batch_t<T, IMAG, 0>(slots, map, nblk, st);
        case 1: return launch_xc_batch_t<T, IMAG, 1>(slots, map, nblk, st);
        case 2: return launch_xc_batch_t<T, IMAG, 2>(slots, map, nblk, st);
        case 3: return launch_xc_batch_t<T, IMAG, 3>(slots, map, nblk, st);
        case 4: return launch_xc_batch_t<T, IMAG, 4>(slots, map, nblk, st);
        case 5: return launch_xc_batch_t<T, IMAG, 5>(slots, map, nblk, st);
        case 6: return launch_xc_batch_t<T, IMAG, 6>(slots, map, nblk, st);
        case 7: return launch_xc_batch_t<T, IMAG, 7>(slots, map, nblk, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_xc_batch(const XCSlot<T>* slots, const unsigned* map, int nblk, int tile, bool imag, hipStream_t st) {
    return imag ? launch_xc_batch_i<T, true>(slots, map, nblk, tile, st)
                : launch_xc_batch_i<T, false>(slots, map, nblk, tile, st);
}

template <typename T>
hipError_t launch_x_batch(const XSlot<T>* slots, const unsigned* map, int nblk, int K, int block, bool imag,
                          hipStream_t st) {
    return imag ? launch_x_batch_t<T, true>(slots, map, nblk, K, block, st)
                : launch_x_batch_t<T, false>(slots, map, nblk, K, block, st);
}

template hipError_t launch_x<double>(const XLaunch<double>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_x<float>(const XLaunch<float>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_x_batch<double>(const XSlot<double>*, const unsigned*, int, int, int, bool, hipStream_t);
template hipError_t launch_x_batch<float>(const XSlot<float>*, const unsigned*, int, int, int, bool, hipStream_t);
template hipError_t launch_xc_batch<double>(const XCSlot<double>*, const unsigned*, int, int, bool, hipStream_t);
template hipError_t launch_xc_batch<float>(const XCSlot<float>*, const unsigned*, int, int, bool, hipStream_t);

}  // namespace gp
