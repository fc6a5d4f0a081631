// y sweep of the SSCN step on gfx950.
//
//   k_y_window   column tiles: 4 NW columns x 16 segments of KY rows; exact
//                partitioned Thomas inside the tile, windows overlapping by h
//                rows so that the truncated carries at the window ends decay
//                below the rounding level before the rows that are written.
//                Norm partials fused into the store.  k_y_batch: the same
//                over the tiles of many condensates in one launch.
//   k_y_thomas   exact per-thread Thomas down whole columns (one thread per
//                column, forward eliminations stored in place).
#include <hip/hip_ext.h>

#include "gp_chain.hpp"

namespace gp {

// ---------------------------------------------------------------------------
// y sweep, windowed partitioned Thomas over column tiles (increment form).
// Each wave holds 4 columns; each DPP row of 16 lanes holds the 16 segments of
// one column; each lane KY consecutive rows of its segment, so a window spans
// 16 KY rows.  The segment scans and the exchange of segment-end neighbours
// are DPP moves inside a row: no shared memory and no barrier (except for the
// norm reduction at the end).  Consecutive windows overlap by h rows on each
// side and write only their L = 16 KY - 2 h middle rows.
// ---------------------------------------------------------------------------
template <typename T, bool IMAG, int KY, int NW, bool SEQ, bool NORM, bool OUTL>
__device__ inline void y_window(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, size_t sp, size_t dp, const Phys& ph,
                                const LineSet<T>& ls, int L, int h, int ncs, NormOut no, int blk) {
    using C = cx<T>;
    constexpr int CPB = 4 * NW;  // columns per block
    __shared__ double shr[48];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int seg = lane & 15, cw = lane >> 4;
    const int cs = blk % ncs, rt = blk / ncs;
    const int i = cs * CPB + wv * 4 + cw;
    const bool col_ok = i < ph.nx;
    const int nx = ph.nx, ny = ph.ny;
    const int j0 = rt * L;
    const int g0 = j0 - h + seg * KY;  // first row of this lane
    C v[3][KY];
#pragma unroll
    for (int k = 0; k < KY; ++k) {
        const int g = g0 + k;
        const bool ok = col_ok && g >= 0 && g < ny;
        const size_t o = (size_t)(ok ? g : 0) * nx + (col_ok ? i : 0);
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m][k] = ok ? src[m * sp + o] : zero_c<C>();
    }
#pragma unroll
    for (int k = 0; k < KY; ++k) to_sx<C, T>(v[0][k], v[1][k], v[2][k]);
    const int il = col_ok ? i : 0;
    // the windows holding row 0 of their columns apply the line-start correction
    // (block-uniform: the first row tiles); row 0 sits h - j0 rows into the window
    // (under row bands a shortened row tile can leave row 0 inside the halo of
    // tiles after the first)
    const int off0 = h - j0;
    window_solve<T, KY, IMAG, SEQ>(v, ls, il * 3, g0, ny, off0 >= 0, off0 / KY, off0 % KY, lane);
#pragma unroll
    for (int k = 0; k < KY; ++k) from_sx<C, T>(v[0][k], v[1][k], v[2][k]);
    if (OUTL) {
        // Strang: the second half local substep, on the way out
        const T x = (T)(ph.x0 + il * ph.dx);
#pragma unroll
        for (int k = 0; k < KY; ++k) {
            const T y = (T)(ph.y0 + (g0 + k) * ph.dy);
            local_substep<T, IMAG>(v[0][k], v[1][k], v[2][k], trap_v<T>(ph, x, y), (T)ph.dtl, (T)ph.c0, (T)ph.c2,
                                   (T)ph.rabi);
        }
    }
    double acc[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < KY; ++k) {
        const int g = g0 + k;
        if (col_ok && g >= j0 && g < j0 + L && g < ny) {
            const size_t o = (size_t)g * nx + i;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                dst[m * dp + o] = v[m][k];
                if (NORM) acc[m] += (double)cnorm2(v[m][k]);
            }
        }
    }
    if (NORM) store_norm_partials(acc, shr, no, blk);
}

template <typename T, bool IMAG, int KY, int NW, bool SEQ, bool NORM, bool OUTL>
__global__ __launch_bounds__(64 * NW) void k_y_window(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst,
                                                      size_t sp, size_t dp, Phys ph, LineSet<T> ls, int L, int h, int ncs, NormOut no,
                                                      int nblk, int order) {
    const int lb = order_logical(order, (int)blockIdx.x, ncs, nblk / ncs);
    if (lb < 0) return;
    y_window<T, IMAG, KY, NW, SEQ, NORM, OUTL>(src, dst, sp, dp, ph, ls, L, h, ncs, no, lb);
}

// ---------------------------------------------------------------------------
// y sweep over chain windows (gp_chain.hpp): 4 columns per wave, 16 segments
// of KY rows per column (one DPP row of lanes), carries over nc segments
// within the DPP row; the window starting at row rt L - h writes the rows
// [rt L, rt L + L), L = 16 KY - 2 h.  Norm partials and the Strang half
// substep as in y_window.  Addresses are 32-bit byte offsets within a plane
// from the planes' base pointers (one offset per row serves all three
// components); the host keeps a plane below 2^32 bytes.
// ---------------------------------------------------------------------------
template <typename T, bool IMAG, int KY, int NW, bool SEQ, bool NORM, bool OUTL>
__global__ __launch_bounds__(64 * NW) void k_y_chain(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst,
                                                     size_t sp, size_t dp, Phys ph, LineSet<T> ls, int L, int h, int nc,
                                                     int ncs, NormOut no, int nblk, int order) {
    using C = cx<T>;
    constexpr int CPB = 4 * NW;  // columns per block
    __shared__ double shr[48];
    const int blk = order_logical(order, (int)blockIdx.x, ncs, nblk / ncs);
    if (blk < 0) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int seg = lane & 15, cw = lane >> 4;
    const int cs = blk % ncs, rt = blk / ncs;
    const int i = cs * CPB + wv * 4 + cw;
    const bool col_ok = i < ph.nx;
    const int nx = ph.nx, ny = ph.ny;
    const int j0 = rt * L;             // first row written
    const int s0 = j0 - h;             // first row of the window
    const int g0 = s0 + seg * KY;      // first row of this lane
    const bool edge = s0 < 0 || s0 + 16 * KY > ny;  // block-uniform
    const unsigned col = col_ok ? (unsigned)i : 0u;
    const unsigned pb = (unsigned)nx * (unsigned)ny * (unsigned)sizeof(C);  // bytes of a plane
    __amdgpu_buffer_rsrc_t rs[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) rs[m] = plane_rsrc(src + m * sp, pb);
    C v[3][KY];
#pragma unroll
    for (int k = 0; k < KY; ++k) {
        const int g = g0 + k;
        const bool ok = col_ok && (!edge || (g >= 0 && g < ny));
        const unsigned o = ((unsigned)(ok ? g : 0) * (unsigned)nx + col) * (unsigned)sizeof(C);
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m][k] = ok ? buf_load<C>(rs[m], o) : zero_c<C>();
    }
#pragma unroll
    for (int k = 0; k < KY; ++k) to_sx<C, T>(v[0][k], v[1][k], v[2][k]);
    const int line0 = (int)col * 3;
    if (!edge) chain_lines<T, KY, IMAG, false, false, SEQ>(v, ls, line0, nc, g0, ny, false, 0, 0);
    else chain_lines<T, KY, IMAG, false, true, SEQ>(v, ls, line0, nc, g0, ny, rt == 0, (lane & ~15) + h / KY, h % KY);
#pragma unroll
    for (int k = 0; k < KY; ++k) from_sx<C, T>(v[0][k], v[1][k], v[2][k]);
    if (OUTL) {
        // Strang: the second half local substep, on the way out
        const T x = (T)(ph.x0 + (int)col * ph.dx);
#pragma unroll
        for (int k = 0; k < KY; ++k) {
            const T y = (T)(ph.y0 + (g0 + k) * ph.dy);
            local_substep<T, IMAG>(v[0][k], v[1][k], v[2][k], trap_v<T>(ph, x, y), (T)ph.dtl, (T)ph.c0, (T)ph.c2,
                                   (T)ph.rabi);
        }
    }
    __amdgpu_buffer_rsrc_t rd[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) rd[m] = plane_rsrc(dst + m * dp, pb);
    const int j1 = min(j0 + L, ny);
    double acc[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < KY; ++k) {
        const int g = g0 + k;
        if (col_ok && g >= j0 && g < j1) {
            const unsigned o = ((unsigned)g * (unsigned)nx + col) * (unsigned)sizeof(C);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                buf_store(v[m][k], rd[m], o);
                if (NORM) acc[m] += (double)cnorm2(v[m][k]);
            }
        }
    }
    if (NORM) store_norm_partials(acc, shr, no, blk);
}

// ---------------------------------------------------------------------------
// y sweep over stacked chain windows: a block of NS / 4 waves takes 16
// consecutive columns (one per lane of a DPP row, so every load and store
// instruction reads or writes row pieces of 16 columns) and a window of NS KY
// rows, its NS segments (16 or 32) spread over the waves (4 per wave, lane =
// 16 segment + column).  The line solves are those of gp_chain.hpp, the
// carries and the segment-end neighbours passing through shared memory
// between the phases (each lane's carry from the nc segments before / after
// it).  Windows start at row rt L - h and write the rows [rt L, rt L + L).
// ---------------------------------------------------------------------------
// Shared memory of NQ lines at a time (3: the lines interleaved; 1: one after
// another, the buffers reused line by line).
template <typename T, int NS, int NQ> struct StackShm {
    cx<T> ends[2][NQ][NS][16];  // [first, last point][line][segment][column] (pre-solve values)
    cx<T> f[NQ][NS][16];        // forward value each segment passes on from a zero carry
    cx<T> b[NQ][NS][16];        // backward value each segment passes on from a zero carry
    cx<T> d0[3][16];            // increment at line point 0, per line and column
};

// Lines q0 .. q0 + NQ - 1 of the window (every thread of the block calls it:
// barriers inside).  Their segment-end values go to shared memory first (the
// previous group's last reads of it lie two barriers back).
template <typename T, int K, bool IMAG, bool EDGE, int NQ, int NS>
__device__ inline void stack_lines(cx<T> (&u)[3][K], int q0, const LineSet<T>& ls, int line0, int nc, int g0, int n,
                                   int seg, int cl, bool first, int seg0, int k0, StackShm<T, NS, NQ>& sh) {
    using C = cx<T>;
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq) {
        sh.ends[0][qq][seg][cl] = u[q0 + qq][0];
        sh.ends[1][qq][seg][cl] = u[q0 + qq][K - 1];
    }
    __syncthreads();
    C v[NQ][K];
    ChainLine<T> c[NQ];  // (P, R unused: formed where needed)
    // right-hand sides times -2 / w, and the forward value passed on from a zero carry
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq) {
        const int q = q0 + qq;
        c[qq] = chain_line<T, 1>(ls, line0 + q);
        // segment-end neighbours (pre-solve values; zeros beyond the window)
        const C um = seg > 0 ? sh.ends[1][qq][seg - 1][cl] : zero_c<C>();
        const C up = seg < NS - 1 ? sh.ends[0][qq][seg + 1][cl] : zero_c<C>();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const C l = k == 0 ? um : u[q][k - 1];
            const C r = k == K - 1 ? up : u[q][k + 1];
            C t = mul_bm1<T, IMAG>(ls.bm1, u[q][k]);
            t = cfma(l, c[qq].a, t);
            t = cfma(r, c[qq].e, t);
            v[qq][k] = cmul(c[qq].m2, t);
            if (EDGE && (g0 + k < 0 || g0 + k >= n)) v[qq][k] = zero_c<C>();
        }
        C f = v[qq][0];
#pragma unroll
        for (int k = 1; k < K; ++k) f = cfma(f, c[qq].nam, v[qq][k]);
        sh.f[qq][seg][cl] = f;
    }
    __syncthreads();
    // carry in from the nc segments before, forward values, backward value passed on
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq) {
        const int jm = seg < nc ? seg : nc;
        const C P = cpow_k<C, K>(c[qq].nam);  // (formed here: shorter live ranges)
        C x = zero_c<C>();
        for (int j = jm; j >= 1; --j) x = cfma(x, P, sh.f[qq][seg - j][cl]);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            x = cfma(x, c[qq].nam, v[qq][k]);
            if (EDGE && g0 + k >= n) x = zero_c<C>();
            v[qq][k] = x;
        }
        C b = v[qq][K - 1];
#pragma unroll
        for (int k = K - 2; k >= 0; --k) b = cfma(b, c[qq].ncp, v[qq][k]);
        sh.b[qq][seg][cl] = b;
    }
    __syncthreads();
    // carry in from the nc segments after, increments
    C d0[NQ];
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq) {
        const int q = q0 + qq;
        const int jm = NS - 1 - seg < nc ? NS - 1 - seg : nc;
        const C R = cpow_k<C, K>(c[qq].ncp);
        C x = zero_c<C>();
        for (int j = jm; j >= 1; --j) x = cfma(x, R, sh.b[qq][seg + j][cl]);
        d0[qq] = zero_c<C>();
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
            x = cfma(x, c[qq].ncp, v[qq][k]);
            if (first && seg == seg0 && k == k0) d0[qq] = x;
            u[q][k] = cadd(u[q][k], x);
        }
    }
    // the increment at line point 0 of each column, for the line-start correction
    // that the caller applies once every line is solved
    if (first && seg == seg0)
#pragma unroll
        for (int qq = 0; qq < NQ; ++qq) sh.d0[q0 + qq][cl] = d0[qq];
}

// One block's window: logical block blk takes column strip blk mod ncs of row
// tile blk / ncs.
template <typename T, bool IMAG, int KY, int NS, bool SEQ, bool NORM, bool OUTL>
__device__ __attribute__((always_inline)) inline void y_stack_block(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, size_t sp, size_t dp,
                                     const Phys& ph, const LineSet<T>& ls, int L, int h, int nc, int ncs, NormOut no,
                                     int blk, StackShm<T, NS, SEQ ? 1 : 3>& sh, double* shr) {
    using C = cx<T>;
    const int tid = threadIdx.x, lane = tid & 63;
    const int cl = lane & 15;                      // column within the block
    const int seg = (tid >> 6) * 4 + (lane >> 4);  // segment of the window, 0 .. NS - 1
    const int cs = blk % ncs, rt = blk / ncs;
    const int i = cs * 16 + cl;
    const bool col_ok = i < ph.nx;
    const int nx = ph.nx, ny = ph.ny;
    const int j0 = rt * L;          // first row written
    const int s0 = j0 - h;          // first row of the window
    const int g0 = s0 + seg * KY;   // first row of this lane
    const bool edge = s0 < 0 || s0 + NS * KY > ny;  // block-uniform
    const unsigned col = col_ok ? (unsigned)i : 0u;
    const unsigned pb = (unsigned)nx * (unsigned)ny * (unsigned)sizeof(C);
    __amdgpu_buffer_rsrc_t rs[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) rs[m] = plane_rsrc(src + m * sp, pb);
    C v[3][KY];
#pragma unroll
    for (int k = 0; k < KY; ++k) {
        const int g = g0 + k;
        const bool ok = col_ok && (!edge || (g >= 0 && g < ny));
        const unsigned o = ((unsigned)(ok ? g : 0) * (unsigned)nx + col) * (unsigned)sizeof(C);
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m][k] = ok ? buf_load<C>(rs[m], o) : zero_c<C>();
    }
#pragma unroll
    for (int k = 0; k < KY; ++k) to_sx<C, T>(v[0][k], v[1][k], v[2][k]);
    const int line0 = (int)col * 3;
    const bool first = rt == 0;  // the window holds row 0 (at segment h / KY, row h % KY)
    if constexpr (SEQ) {
        if (!edge) {
            stack_lines<T, KY, IMAG, false, 1, NS>(v, 0, ls, line0, nc, g0, ny, seg, cl, false, 0, 0, sh);
            stack_lines<T, KY, IMAG, false, 1, NS>(v, 1, ls, line0, nc, g0, ny, seg, cl, false, 0, 0, sh);
            stack_lines<T, KY, IMAG, false, 1, NS>(v, 2, ls, line0, nc, g0, ny, seg, cl, false, 0, 0, sh);
        } else {
            stack_lines<T, KY, IMAG, true, 1, NS>(v, 0, ls, line0, nc, g0, ny, seg, cl, first, h / KY, h % KY, sh);
            stack_lines<T, KY, IMAG, true, 1, NS>(v, 1, ls, line0, nc, g0, ny, seg, cl, first, h / KY, h % KY, sh);
            stack_lines<T, KY, IMAG, true, 1, NS>(v, 2, ls, line0, nc, g0, ny, seg, cl, first, h / KY, h % KY, sh);
        }
    } else {
        if (!edge) stack_lines<T, KY, IMAG, false, 3, NS>(v, 0, ls, line0, nc, g0, ny, seg, cl, false, 0, 0, sh);
        else stack_lines<T, KY, IMAG, true, 3, NS>(v, 0, ls, line0, nc, g0, ny, seg, cl, first, h / KY, h % KY, sh);
    }
    if (first) {
        // line-start correction (block-uniform branch)
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 3; ++q) line_start_fix<T, KY>(v[q], ls, line0 + q, sh.d0[q][cl], g0);
    }
#pragma unroll
    for (int k = 0; k < KY; ++k) from_sx<C, T>(v[0][k], v[1][k], v[2][k]);
    if (OUTL) {
        // Strang: the second half local substep, on the way out
        const T x = (T)(ph.x0 + (int)col * ph.dx);
#pragma unroll
        for (int k = 0; k < KY; ++k) {
            const T y = (T)(ph.y0 + (g0 + k) * ph.dy);
            local_substep<T, IMAG>(v[0][k], v[1][k], v[2][k], trap_v<T>(ph, x, y), (T)ph.dtl, (T)ph.c0, (T)ph.c2,
                                   (T)ph.rabi);
        }
    }
    __amdgpu_buffer_rsrc_t rd[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) rd[m] = plane_rsrc(dst + m * dp, pb);
    const int j1 = min(j0 + L, ny);
    double acc[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < KY; ++k) {
        const int g = g0 + k;
        if (col_ok && g >= j0 && g < j1) {
            const unsigned o = ((unsigned)g * (unsigned)nx + col) * (unsigned)sizeof(C);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                buf_store(v[m][k], rd[m], o);
                if (NORM) acc[m] += (double)cnorm2(v[m][k]);
            }
        }
    }
    if (NORM) store_norm_partials(acc, shr, no, blk);
}

// (16 NS threads; launch bound: 8 waves per CU, i.e. 256 registers per lane)
template <typename T, bool IMAG, int KY, int NS, bool SEQ, bool NORM, bool OUTL>
__global__ __launch_bounds__(16 * NS, 32 / NS) void k_y_stack(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst,
                                                             size_t sp, size_t dp, Phys ph, LineSet<T> ls, int L, int h,
                                                             int nc, int ncs, NormOut no, int nblk, int order) {
    __shared__ StackShm<T, NS, SEQ ? 1 : 3> sh;
    __shared__ double shr[48];
    const int blk = order_logical(order, (int)blockIdx.x, ncs, nblk / ncs);
    if (blk < 0) return;  // (the whole block)
    y_stack_block<T, IMAG, KY, NS, SEQ, NORM, OUTL>(src, dst, sp, dp, ph, ls, L, h, nc, ncs, no, blk, sh, shr);
}

// Many condensates in one launch: map entry b names the condensate and its
// window (imaginary time stores each condensate's norm partials).
template <typename T, bool IMAG, int KY, int NS, bool SEQ>
__global__ __launch_bounds__(16 * NS, 32 / NS) void k_y_stack_batch(const YSSlot<T>* __restrict__ slots,
                                                                   const unsigned* __restrict__ map) {
    __shared__ StackShm<T, NS, SEQ ? 1 : 3> sh;
    __shared__ double shr[48];
    const unsigned e = map[blockIdx.x];
    const YSSlot<T>& s = slots[e >> kMapShift];
    y_stack_block<T, IMAG, KY, NS, SEQ, IMAG, false>(s.src, s.dst, s.sp, s.dp, s.ph, s.ls, s.L, s.h, s.nc, s.ncs,
                                                     NormOut{s.partials}, (int)(e & kMapMask), sh, shr);
}

template <typename T, bool IMAG, int KY, int NW, bool SEQ>
__global__ __launch_bounds__(64 * NW) void k_y_batch(const YSlot<T>* __restrict__ slots, const unsigned* __restrict__ map) {
    const unsigned e = map[blockIdx.x];
    const YSlot<T>& s = slots[e >> kMapShift];
    y_window<T, IMAG, KY, NW, SEQ, IMAG, false>(s.src, s.dst, s.sp, s.dp, s.ph, s.ls, s.L, s.h, s.ncs, NormOut{s.partials},
                                                (int)(e & kMapMask));
}

// ---------------------------------------------------------------------------
// y sweep, exact per-thread Thomas down whole columns (increment form): the
// forward eliminations go to dst, the back substitution re-reads src.
// ---------------------------------------------------------------------------
template <typename T, bool IMAG, bool NORM, bool OUTL>
__global__ __launch_bounds__(256) void k_y_thomas(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, size_t sp,
                                                 size_t dp, Phys ph,
                                                 LineSet<T> ls, NormOut no) {
    using C = cx<T>;
    __shared__ double shr[48];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nx = ph.nx, ny = ph.ny;
    double acc[3] = {0, 0, 0};
    if (i < nx) {
        C a[3], e[3];
        Piv<T> lim[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            a[q] = ls.ae[2 * (i * 3 + q)];
            e[q] = ls.ae[2 * (i * 3 + q) + 1];
            lim[q] = ls.piv[(size_t)(i * 3 + q) * (ls.K + 1) + ls.K];
        }
        auto load_sx = [&](int g, C (&o)[3]) {
            if (g >= 0 && g < ny) {
#pragma unroll
                for (int m = 0; m < 3; ++m) o[m] = src[m * sp + (size_t)g * nx + i];
                to_sx<C, T>(o[0], o[1], o[2]);
            } else {
#pragma unroll
                for (int m = 0; m < 3; ++m) o[m] = zero_c<C>();
            }
        };
        C prev[3] = {zero_c<C>(), zero_c<C>(), zero_c<C>()}, cur[3], nxt[3], d[3];
        load_sx(0, cur);
        C carry[3] = {zero_c<C>(), zero_c<C>(), zero_c<C>()};
        for (int g = 0; g < ny; ++g) {
            load_sx(g + 1, nxt);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                C t = mul_bm1<T, IMAG>(ls.bm1, cur[q]);
                t = cfma(prev[q], a[q], t);
                t = cfma(nxt[q], e[q], t);
                const C rr = cscale(t, (T)-2);
                const Piv<T> pv = (g < ls.K) ? piv_at(ls, i * 3 + q, g) : lim[q];
                d[q] = cfma(carry[q], cneg(pv.am), cmul(pv.m, rr));
                carry[q] = d[q];
                prev[q] = cur[q];
                cur[q] = nxt[q];
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) dst[m * dp + (size_t)g * nx + i] = d[m];
        }
        C x[3] = {zero_c<C>(), zero_c<C>(), zero_c<C>()};
        for (int g = ny - 1; g >= 0; --g) {
            C o[3], uu[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) o[m] = dst[m * dp + (size_t)g * nx + i];
            load_sx(g, uu);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const Piv<T> pv = (g < ls.K) ? piv_at(ls, i * 3 + q, g) : lim[q];
                x[q] = csub(o[q], cmul(pv.cp, x[q]));
                o[q] = cadd(uu[q], x[q]);
            }
            from_sx<C, T>(o[0], o[1], o[2]);
            if (OUTL) {
                const T x = (T)(ph.x0 + i * ph.dx), y = (T)(ph.y0 + g * ph.dy);
                local_substep<T, IMAG>(o[0], o[1], o[2], trap_v<T>(ph, x, y), (T)ph.dtl, (T)ph.c0, (T)ph.c2,
                                       (T)ph.rabi);
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                dst[m * dp + (size_t)g * nx + i] = o[m];
                if (NORM) acc[m] += (double)cnorm2(o[m]);
            }
        }
    }
    if (NORM) store_norm_partials(acc, shr, no, (int)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <typename T, bool IMAG, bool NORM, bool OUTL, int TI>
static hipError_t launch_yw_t(const YLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    constexpr YTile yt = ytile<T>(TI);
    const int ncs = (a.ph.nx + 4 * yt.NW - 1) / (4 * yt.NW);
    const int nrt = (a.ph.ny + a.L - 1) / a.L;
    const int nblk = ncs * nrt;
    hipExtLaunchKernelGGL(k_y_window<T, IMAG, yt.KY, yt.NW, yt.SEQ, NORM, OUTL>, dim3(xcd_grid(a.order, ncs, nrt)),
                          dim3(64 * yt.NW), 0, st, e0, e1, 0, a.src, a.dst, a.sp, a.dp, a.ph, a.ls, a.L, a.h, ncs, a.no, nblk,
                          a.order);
    return hipGetLastError();
}

template <typename T, bool IMAG, bool NORM, bool OUTL>
static hipError_t launch_yw(const YLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    switch (a.tile) {
        case 0: return launch_yw_t<T, IMAG, NORM, OUTL, 0>(a, st, e0, e1);
        case 1: return launch_yw_t<T, IMAG, NORM, OUTL, 1>(a, st, e0, e1);
        case 2: return launch_yw_t<T, IMAG, NORM, OUTL, 2>(a, st, e0, e1);
        case 3: return launch_yw_t<T, IMAG, NORM, OUTL, 3>(a, st, e0, e1);
        case 4: return launch_yw_t<T, IMAG, NORM, OUTL, 4>(a, st, e0, e1);
        case 5: return launch_yw_t<T, IMAG, NORM, OUTL, 5>(a, st, e0, e1);
        case 6: return launch_yw_t<T, IMAG, NORM, OUTL, 6>(a, st, e0, e1);
        case 7: return launch_yw_t<T, IMAG, NORM, OUTL, 7>(a, st, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, bool IMAG, bool NORM, bool OUTL, int TI>
static hipError_t launch_yc_t(const YLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    constexpr ChainTile ct = ychain_tile<T>(TI);
    // the window (16 KY rows) writes L = 16 KY - 2 h rows; the first window holds the corrected rows;
    // byte offsets within a plane fit 32 bits
    if (a.h < 1 || a.L != 16 * ct.K - 2 * a.h || a.L <= 0 || a.ls.Kg > a.L ||
        (double)a.ph.nx * a.ph.ny * sizeof(cx<T>) >= 4294967296.0)
        return hipErrorInvalidValue;
    const int ncs = (a.ph.nx + 4 * ct.NW - 1) / (4 * ct.NW);
    const int nrt = (a.ph.ny + a.L - 1) / a.L;
    const int nblk = ncs * nrt;
    hipExtLaunchKernelGGL(k_y_chain<T, IMAG, ct.K, ct.NW, ct.SEQ, NORM, OUTL>, dim3(xcd_grid(a.order, ncs, nrt)),
                          dim3(64 * ct.NW), 0, st, e0, e1, 0, a.src, a.dst, a.sp, a.dp, a.ph, a.ls, a.L, a.h,
                          chain_lanes(a.h, ct.K), ncs, a.no, nblk, a.order);
    return hipGetLastError();
}

template <typename T, bool IMAG, bool NORM, bool OUTL>
static hipError_t launch_yc(const YLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (a.order == 3) return hipErrorInvalidValue;  // (row bands: scanned windows only)
    switch (a.tile) {
        case 0: return launch_yc_t<T, IMAG, NORM, OUTL, 0>(a, st, e0, e1);
        case 1: return launch_yc_t<T, IMAG, NORM, OUTL, 1>(a, st, e0, e1);
        case 2: return launch_yc_t<T, IMAG, NORM, OUTL, 2>(a, st, e0, e1);
        case 3: return launch_yc_t<T, IMAG, NORM, OUTL, 3>(a, st, e0, e1);
        case 4: return launch_yc_t<T, IMAG, NORM, OUTL, 4>(a, st, e0, e1);
        case 5: return launch_yc_t<T, IMAG, NORM, OUTL, 5>(a, st, e0, e1);
        case 6: return launch_yc_t<T, IMAG, NORM, OUTL, 6>(a, st, e0, e1);
        case 7: return launch_yc_t<T, IMAG, NORM, OUTL, 7>(a, st, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, bool IMAG, bool NORM, bool OUTL, int TI>
static hipError_t launch_ys_t(const YLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    constexpr ChainTile ct = ystack_tile<T>(TI);
    constexpr int NS = 4 * ct.NW;  // segments per window
    // the window (NS KY rows) writes L = NS KY - 2 h rows; the first window holds the corrected rows;
    // byte offsets within a plane fit 32 bits; the carries reach at most NS - 1 segments
    if (a.h < 1 || a.L != NS * ct.K - 2 * a.h || a.L <= 0 || a.ls.Kg > a.L || chain_lanes(a.h, ct.K) > NS - 1 ||
        (double)a.ph.nx * a.ph.ny * sizeof(cx<T>) >= 4294967296.0 || a.order == 3)
        return hipErrorInvalidValue;
    const int ncs = (a.ph.nx + 15) / 16;
    const int nrt = (a.ph.ny + a.L - 1) / a.L;
    const int nblk = ncs * nrt;
    hipExtLaunchKernelGGL(k_y_stack<T, IMAG, ct.K, NS, ct.SEQ, NORM, OUTL>, dim3(xcd_grid(a.order, ncs, nrt)),
                          dim3(16 * NS), 0, st, e0, e1, 0, a.src, a.dst, a.sp, a.dp, a.ph, a.ls, a.L, a.h,
                          chain_lanes(a.h, ct.K), ncs, a.no, nblk, a.order);
    return hipGetLastError();
}

template <typename T, bool IMAG, bool NORM, bool OUTL>
static hipError_t launch_ys(const YLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    switch (a.tile) {
        case 0: return launch_ys_t<T, IMAG, NORM, OUTL, 0>(a, st, e0, e1);
        case 1: return launch_ys_t<T, IMAG, NORM, OUTL, 1>(a, st, e0, e1);
        case 2: return launch_ys_t<T, IMAG, NORM, OUTL, 2>(a, st, e0, e1);
        case 3: return launch_ys_t<T, IMAG, NORM, OUTL, 3>(a, st, e0, e1);
        case 4: return launch_ys_t<T, IMAG, NORM, OUTL, 4>(a, st, e0, e1);
        case 5: return launch_ys_t<T, IMAG, NORM, OUTL, 5>(a, st, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
int y_blocks(const YLaunch<T>& a) {
    if (a.stack) return ((a.ph.nx + 15) / 16) * ((a.ph.ny + a.L - 1) / a.L);  // (any segment count)
    if (a.chain) {
        const ChainTile ct = ychain_tile<T>(a.tile);
        const int ncs = (a.ph.nx + 4 * ct.NW - 1) / (4 * ct.NW);
        return ncs * ((a.ph.ny + a.L - 1) / a.L);
    }
    if (a.window) {
        const YTile yt = ytile<T>(a.tile);
        const int ncs = (a.ph.nx + 4 * yt.NW - 1) / (4 * yt.NW);
        return ncs * ((a.ph.ny + a.L - 1) / a.L);
    }
    return (a.ph.nx + 255) / 256;
}

template <typename T, bool IMAG, bool NORM, bool OUTL>
static hipError_t launch_yt(const YLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const dim3 grid((a.ph.nx + 255) / 256), block(256);
    hipExtLaunchKernelGGL(k_y_thomas<T, IMAG, NORM, OUTL>, grid, block, 0, st, e0, e1, 0, a.src, a.dst, a.sp, a.dp, a.ph, a.ls, a.no);
    return hipGetLastError();
}

// (imag, norm, outl): the steps use (1, 1, *) and (0, 0, *); the substep calls (*, 0, 0).
template <typename T, bool IMAG, bool NORM, bool OUTL>
static hipError_t launch_y_v(const YLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (a.stack) return launch_ys<T, IMAG, NORM, OUTL>(a, st, e0, e1);
    if (a.chain) return launch_yc<T, IMAG, NORM, OUTL>(a, st, e0, e1);
    return a.window ? launch_yw<T, IMAG, NORM, OUTL>(a, st, e0, e1) : launch_yt<T, IMAG, NORM, OUTL>(a, st, e0, e1);
}

template <typename T>
hipError_t launch_y(const YLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (a.outl) {
        if (a.norm != a.imag) return hipErrorInvalidValue;
        return a.imag ? launch_y_v<T, true, true, true>(a, st, e0, e1) : launch_y_v<T, false, false, true>(a, st, e0, e1);
    }
    if (a.imag) return a.norm ? launch_y_v<T, true, true, false>(a, st, e0, e1) : launch_y_v<T, true, false, false>(a, st, e0, e1);
    return a.norm ? launch_y_v<T, false, true, false>(a, st, e0, e1) : launch_y_v<T, false, false, false>(a, st, e0, e1);
}

template <typename T, bool IMAG, int TI>
static hipError_t launch_y_batch_t(const YSlot<T>* slots, const unsigned* map, int nblk, hipStream_t st) {
    constexpr YTile yt = ytile<T>(TI);
    hipExtLaunchKernelGGL(k_y_batch<T, IMAG, yt.KY, yt.NW, yt.SEQ>, dim3(nblk), dim3(64 * yt.NW), 0, st, nullptr, nullptr, 0,
                          slots, map);
    return hipGetLastError();
}

template <typename T, bool IMAG>
static hipError_t launch_y_batch_i(const YSlot<T>* slots, const unsigned* map, int nblk, int tile, hipStream_t st) {
    if (nblk <= 0) return hipErrorInvalidValue;
    switch (tile) {
        case 0: return launch_y_batch_t<T, IMAG, 0>(slots, map, nblk, st);
        case 1: return launch_y_batch_t<T, IMAG, 1>(slots, map, nblk, st);
        case 2: return launch_y_batch_t<T, IMAG, 2>(slots, map, nblk, st);
        case 3: return launch_y_batch_t<T, IMAG, 3>(slots, map, nblk, st);
        case 4: return launch_y_batch_t<T, IMAG, 4>(slots, map, nblk, st);
        case 5: return launch_y_batch_t<T, IMAG, 5>(slots, map, nblk, st);
        case 6: return launch_y_batch_t<T, IMAG, 6>(slots, map, nblk, st);
        case 7: return launch_y_batch_t<T, IMAG, 7>(slots, map, nblk, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, bool IMAG, int TI>
static hipError_t launch_ys_batch_t(const YSSlot<T>* slots, const unsigned* map, int nblk, hipStream_t st) {
    constexpr ChainTile ct = ystack_tile<T>(TI);
    hipExtLaunchKernelGGL(k_y_stack_batch<T, IMAG, ct.K, 4 * ct.NW, ct.SEQ>, dim3(nblk), dim3(64 * ct.NW), 0, st,
                          nullptr, nullptr, 0, slots, map);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ys_batch(const YSSlot<T>* slots, const unsigned* map, int nblk, int tile, bool imag, hipStream_t st) {
    if (nblk <= 0) return hipErrorInvalidValue;
    switch (tile) {
        case 0: return imag ? launch_ys_batch_t<T, true, 0>(slots, map, nblk, st) : launch_ys_batch_t<T, false, 0>(slots, map, nblk, st);
        case 1: return imag ? launch_ys_batch_t<T, true, 1>(slots, map, nblk, st) : launch_ys_batch_t<T, false, 1>(slots, map, nblk, st);
        case 2: return imag ? launch_ys_batch_t<T, true, 2>(slots, map, nblk, st) : launch_ys_batch_t<T, false, 2>(slots, map, nblk, st);
        case 3: return imag ? launch_ys_batch_t<T, true, 3>(slots, map, nblk, st) : launch_ys_batch_t<T, false, 3>(slots, map, nblk, st);
        case 4: return imag ? launch_ys_batch_t<T, true, 4>(slots, map, nblk, st) : launch_ys_batch_t<T, false, 4>(slots, map, nblk, st);
        case 5: return imag ? launch_ys_batch_t<T, true, 5>(slots, map, nblk, st) : launch_ys_batch_t<T, false, 5>(slots, map, nblk, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_y_batch(const YSlot<T>* slots, const unsigned* map, int nblk, int tile, bool imag, hipStream_t st) {
    return imag ? launch_y_batch_i<T, true>(slots, map, nblk, tile, st) : launch_y_batch_i<T, false>(slots, map, nblk, tile, st);
}

template hipError_t launch_y<double>(const YLaunch<double>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_y<float>(const YLaunch<float>&, hipStream_t, hipEvent_t, hipEvent_t);
template int y_blocks<double>(const YLaunch<double>&);
template int y_blocks<float>(const YLaunch<float>&);
template hipError_t launch_y_batch<double>(const YSlot<double>*, const unsigned*, int, int, bool, hipStream_t);
template hipError_t launch_y_batch<float>(const YSlot<float>*, const unsigned*, int, int, bool, hipStream_t);
template hipError_t launch_ys_batch<double>(const YSSlot<double>*, const unsigned*, int, int, bool, hipStream_t);
template hipError_t launch_ys_batch<float>(const YSSlot<float>*, const unsigned*, int, int, bool, hipStream_t);

}  // namespace gp
