// gfx950 kernels of the SSCN step.
//
//   k_x_scan     local substep (+ pending renormalisation) fused into the x
//                Crank-Nicolson sweep; one row per thread group, K consecutive
//                points per thread in registers, exact partitioned Thomas
//                (local recurrences + wave/LDS scans of the block carries).
//   k_y_window   y sweep over column tiles: TW columns x (S segments of KY
//                rows); exact partitioned Thomas inside the tile, windows
//                overlapping by h rows so that the truncated carries at the
//                window ends decay below the rounding level before the rows
//                that are written.  Norm partials fused into the store.
//   k_y_thomas   exact per-thread Thomas down whole columns (one thread per
//                column, forward eliminations stored in place).
//   k_local, k_scale, k_set_scale, k_norm_finalize, k_obs, k_obs_finalize.
#include <hip/hip_ext.h>

#include "gp_kernels.hpp"
#include "gp_scan.hpp"

namespace gp {

// ---------------------------------------------------------------------------
// Crank-Nicolson line solve in increment form.  With A = I + alpha h the
// tridiagonal matrix (sub a, diagonal b, super e), the new values are
// u' = A^{-1} (2I - A) u = u + delta with A delta = -2 (A - I) u: the
// increment is small (of order alpha/dx^2 relative to u), so the rounding of
// the elimination is small relative to u and u + delta is rounded once.  (In
// FP32 the direct form drifts in norm by a few 1e-8 per sweep.)
//
// Partitioned Thomas on one line held as K consecutive values per thread
// (indices i0 .. i0+K-1 of a line of length n; indices outside [0, n) are
// padding), in place on u[]; left/right are the line values just outside the
// thread's block.  FS and BS are the forward and backward exclusive scans of
// the block transfer maps across the threads sharing the line; every thread
// must reach them (they contain barriers).
//
// Blocks entirely inside the line and past the tabulated transient of the
// pivots take a fast path with the converged pivots held in registers.
// ---------------------------------------------------------------------------
template <typename T, bool IMAG> __device__ inline cx<T> mul_bm1(cx<T> bm1, cx<T> u) {
    // b - 1 = alpha / dx^2: real in imaginary time, imaginary in real time
    return IMAG ? cscale(u, bm1.x) : cscale(ctimes_i(u), bm1.y);
}
template <typename C> __device__ inline C cneg(C a) { C z; z.x = -a.x; z.y = -a.y; return z; }
template <typename C, int K> __device__ inline C cpow_k(C a) {
    C r = one_c<C>(), b = a;
#pragma unroll
    for (int k = K; k > 0; k >>= 1) {
        if (k & 1) r = cmul(r, b);
        b = cmul(b, b);
    }
    return r;
}

template <typename T, int K, bool IMAG, typename FS, typename BS>
__device__ inline void block_solve(cx<T> (&u)[K], cx<T> left, cx<T> right, const LineSet<T>& ls, int line, int i0,
                                   int n, FS fscan, BS bscan) {
    using C = cx<T>;
    const C a = ls.ae[2 * line], e = ls.ae[2 * line + 1];
    const Piv<T> lim = ls.piv[(size_t)line * (ls.K + 1) + ls.K];
    const bool fast = i0 >= ls.K && i0 + K <= n;
    // right-hand side of the increment system: r = -2 ((b - 1) u_k + a u_{k-1} + e u_{k+1})
    C r[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const C um = (k == 0) ? left : u[k - 1];
        const C up = (k == K - 1) ? right : u[k + 1];
        C t = mul_bm1<T, IMAG>(ls.bm1, u[k]);
        t = cfma(um, a, t);
        t = cfma(up, e, t);
        r[k] = cscale(t, (T)-2);
    }
    const C nam = cneg(lim.am), ncp = cneg(lim.cp);
    // forward elimination over the block from a zero carry: E_k = m r_k - am E_{k-1}
    C E = zero_c<C>(), P;
    if (fast) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            E = cfma(E, nam, cmul(lim.m, r[k]));
            r[k] = E;
        }
        P = cpow_k<C, K>(nam);
    } else {
        P = one_c<C>();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = i0 + k;
            if (i >= 0 && i < n) {
                const Piv<T> pv = (i < ls.K) ? piv_at(ls, line, i) : lim;
                E = cfma(E, cneg(pv.am), cmul(pv.m, r[k]));
                P = cmul(cneg(pv.am), P);
            } else {
                E = zero_c<C>();
                P = zero_c<C>();
            }
            r[k] = E;
        }
    }
    const C din = fscan(P, E);
    // add the carry that enters the block, times the running product of -am
    if (fast) {
        C Q = one_c<C>();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            Q = cmul(Q, nam);
            r[k] = cfma(din, Q, r[k]);
        }
    } else {
        C Q = one_c<C>();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = i0 + k;
            if (i >= 0 && i < n) {
                const Piv<T> pv = (i < ls.K) ? piv_at(ls, line, i) : lim;
                Q = cmul(Q, cneg(pv.am));
                r[k] = cfma(din, Q, r[k]);
            }
        }
    }
    // back substitution over the block from a zero carry: G_k = r_k - cp G_{k+1}
    C G = zero_c<C>(), R;
    if (fast) {
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
            G = cfma(G, ncp, r[k]);
            r[k] = G;
        }
        R = cpow_k<C, K>(ncp);
    } else {
        R = one_c<C>();
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
            const int i = i0 + k;
            if (i >= 0 && i < n) {
                const Piv<T> pv = (i < ls.K) ? piv_at(ls, line, i) : lim;
                G = cfma(G, cneg(pv.cp), r[k]);
                R = cmul(cneg(pv.cp), R);
            } else {
                G = zero_c<C>();
                R = zero_c<C>();
            }
            r[k] = G;
        }
    }
    const C xin = bscan(R, G);
    if (fast) {
        C Sx = one_c<C>();
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
            Sx = cmul(Sx, ncp);
            u[k] = cadd(u[k], cfma(xin, Sx, r[k]));
        }
    } else {
        C Sx = one_c<C>();
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
            const int i = i0 + k;
            if (i >= 0 && i < n) {
                const Piv<T> pv = (i < ls.K) ? piv_at(ls, line, i) : lim;
                Sx = cmul(Sx, cneg(pv.cp));
                u[k] = cadd(u[k], cfma(xin, Sx, r[k]));
            }
        }
    }
}

template <typename T, int K, bool IMAG, typename FS, typename BS>
__device__ inline void block_solve3(cx<T> (&u)[3][K], const cx<T> (&left)[3], const cx<T> (&right)[3],
                                    const LineSet<T>& ls, int line0, int i0, int n, FS fscan, BS bscan) {
    using C = cx<T>;
    C a[3], e[3], nam[3], ncp[3], lm[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        a[q] = ls.ae[2 * (line0 + q)];
        e[q] = ls.ae[2 * (line0 + q) + 1];
        const Piv<T> lim = ls.piv[(size_t)(line0 + q) * (ls.K + 1) + ls.K];
        lm[q] = lim.m;
        nam[q] = cneg(lim.am);
        ncp[q] = cneg(lim.cp);
    }
    const bool fast = i0 >= ls.K && i0 + K <= n;
    // right-hand side of the increment system: r = -2 ((b - 1) u_k + a u_{k-1} + e u_{k+1})
    C r[3][K];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const C um = (k == 0) ? left[q] : u[q][k - 1];
            const C up = (k == K - 1) ? right[q] : u[q][k + 1];
            C t = mul_bm1<T, IMAG>(ls.bm1, u[q][k]);
            t = cfma(um, a[q], t);
            t = cfma(up, e[q], t);
            r[q][k] = cscale(t, (T)-2);
        }
    // forward elimination over the block from a zero carry: E_k = m r_k - am E_{k-1}
    C E[3], P[3], din[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) E[q] = zero_c<C>();
    if (fast) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                E[q] = cfma(E[q], nam[q], cmul(lm[q], r[q][k]));
                r[q][k] = E[q];
            }
#pragma unroll
        for (int q = 0; q < 3; ++q) P[q] = cpow_k<C, K>(nam[q]);
    } else {
#pragma unroll
        for (int q = 0; q < 3; ++q) P[q] = one_c<C>();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = i0 + k;
            const bool in = i >= 0 && i < n;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (in) {
                    const Piv<T> pv = piv_at(ls, line0 + q, i);
                    E[q] = cfma(E[q], cneg(pv.am), cmul(pv.m, r[q][k]));
                    P[q] = cmul(cneg(pv.am), P[q]);
                } else {
                    E[q] = zero_c<C>();
                    P[q] = zero_c<C>();
                }
                r[q][k] = E[q];
            }
        }
    }
    fscan(P, E, din);
    // add the carry that enters the block, times the running product of -am
    if (fast) {
        C Q[3] = {one_c<C>(), one_c<C>(), one_c<C>()};
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                Q[q] = cmul(Q[q], nam[q]);
                r[q][k] = cfma(din[q], Q[q], r[q][k]);
            }
    } else {
        C Q[3] = {one_c<C>(), one_c<C>(), one_c<C>()};
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = i0 + k;
            if (i >= 0 && i < n) {
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    Q[q] = cmul(Q[q], cneg(piv_at(ls, line0 + q, i).am));
                    r[q][k] = cfma(din[q], Q[q], r[q][k]);
                }
            }
        }
    }
    // back substitution over the block from a zero carry: G_k = r_k - cp G_{k+1}
    C G[3], R[3], xin[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) G[q] = zero_c<C>();
    if (fast) {
#pragma unroll
        for (int k = K - 1; k >= 0; --k)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                G[q] = cfma(G[q], ncp[q], r[q][k]);
                r[q][k] = G[q];
            }
#pragma unroll
        for (int q = 0; q < 3; ++q) R[q] = cpow_k<C, K>(ncp[q]);
    } else {
#pragma unroll
        for (int q = 0; q < 3; ++q) R[q] = one_c<C>();
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
            const int i = i0 + k;
            const bool in = i >= 0 && i < n;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (in) {
                    const C nc = cneg(piv_at(ls, line0 + q, i).cp);
                    G[q] = cfma(G[q], nc, r[q][k]);
                    R[q] = cmul(nc, R[q]);
                } else {
                    G[q] = zero_c<C>();
                    R[q] = zero_c<C>();
                }
                r[q][k] = G[q];
            }
        }
    }
    bscan(R, G, xin);
    if (fast) {
        C Sx[3] = {one_c<C>(), one_c<C>(), one_c<C>()};
#pragma unroll
        for (int k = K - 1; k >= 0; --k)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                Sx[q] = cmul(Sx[q], ncp[q]);
                u[q][k] = cadd(u[q][k], cfma(xin[q], Sx[q], r[q][k]));
            }
    } else {
        C Sx[3] = {one_c<C>(), one_c<C>(), one_c<C>()};
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
            const int i = i0 + k;
            if (i >= 0 && i < n) {
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    Sx[q] = cmul(Sx[q], cneg(piv_at(ls, line0 + q, i).cp));
                    u[q][k] = cadd(u[q][k], cfma(xin[q], Sx[q], r[q][k]));
                }
            }
        }
    }
}

template <typename T, bool IMAG, int K, bool LOCAL, bool SCALE, int LB>
__global__ __launch_bounds__(LB) void k_x_scan(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, Phys ph,
                                               LineSet<T> ls, const double* __restrict__ scale, int G, int R) {
    using C = cx<T>;
    __shared__ C shS[6 * 16];
    __shared__ C shN[2 * 3 * 16];
    const int tid = threadIdx.x;
    const int r = tid / G, t = tid - r * G;
    const int lane = t & 63, w = t >> 6, nw = G >> 6;
    const int j = blockIdx.x * R + r;
    const bool row_ok = j < ph.ny;
    const int nx = ph.nx;
    const size_t plane = (size_t)ph.nx * ph.ny;
    const int i0 = t * K;
    const size_t rowoff = (size_t)(row_ok ? j : 0) * nx;
    const C* rowp = src + rowoff;
    C* rowq = dst + rowoff;
    C v[3][K];
    if (row_ok && i0 + K <= nx) {
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k) v[m][k] = rowp[m * plane + i0 + k];
    } else {
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k)
                v[m][k] = (row_ok && i0 + k < nx) ? rowp[m * plane + i0 + k] : zero_c<C>();
    }
    if (SCALE) {
        const T s = (T)(*scale);
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k) v[m][k] = cscale(v[m][k], s);
    }
    if (LOCAL) {
        const T y = (T)(ph.y0 + (row_ok ? j : 0) * ph.dy);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T x = (T)(ph.x0 + (i0 + k) * ph.dx);
            local_substep<T, IMAG>(v[0][k], v[1][k], v[2][k], (T)0.5 * (x * x + y * y), (T)ph.dt, (T)ph.c0,
                                   (T)ph.c2, (T)ph.rabi);
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) to_sy<C, T>(v[0][k], v[1][k], v[2][k]);
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
    const int jl = row_ok ? j : 0;
    C* ss = shS + 6 * nrow;
    if constexpr (sizeof(T) * K <= 32) {
        // the three lines' chains interleaved (fits the register file for small blocks)
        auto fs = [&](const C (&P)[3], const C (&E)[3], C (&o)[3]) { row_scan3<true>(P, E, o, lane, w, nw, ss); };
        auto bs = [&](const C (&P)[3], const C (&E)[3], C (&o)[3]) { row_scan3<false>(P, E, o, lane, w, nw, ss); };
        block_solve3<T, K, IMAG>(v, left, right, ls, jl * 3, i0, nx, fs, bs);
    } else {
        // one line after the other
        auto fs = [&](C P, C E) { return row_scan<true>(P, E, lane, w, nw, ss, ss + nw); };
        auto bs = [&](C P, C E) { return row_scan<false>(P, E, lane, w, nw, ss, ss + nw); };
#pragma unroll
        for (int q = 0; q < 3; ++q) block_solve<T, K, IMAG>(v[q], left[q], right[q], ls, jl * 3 + q, i0, nx, fs, bs);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) from_sy<C, T>(v[0][k], v[1][k], v[2][k]);
    if (row_ok && i0 + K <= nx) {
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k) rowq[m * plane + i0 + k] = v[m][k];
    } else if (row_ok) {
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (i0 + k < nx) rowq[m * plane + i0 + k] = v[m][k];
    }
}

// ---------------------------------------------------------------------------
// Block reduction of one double (all threads call; result valid in thread 0).
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < nw; ++k) s += sh[k];
    __syncthreads();
    return s;
}

// Per-block partial sum of the imaginary-time norm, in block order; a one-block
// kernel launched next on the same stream forms the total (a device-wide
// release fence per block would write back the L2 of its XCD every time).
__device__ inline void store_norm_partial(double part, NormOut no) {
    if (threadIdx.x == 0) no.partials[blockIdx.x] = part;
}

// ---------------------------------------------------------------------------
// y sweep, windowed partitioned Thomas over column tiles (increment form).
// Each wave holds 4 columns; each DPP row of 16 lanes holds the 16 segments of
// one column; each lane KY consecutive rows of its segment, so a window spans
// 16 KY rows.  The segment scans and the exchange of segment-end neighbours
// are DPP moves inside a row: no shared memory and no barrier (except for the
// norm reduction at the end).  Consecutive windows overlap by h rows on each
// side and write only their L = 16 KY - 2 h middle rows.
// ---------------------------------------------------------------------------
template <typename T, bool IMAG, int KY, int NW, bool NORM>
__global__ __launch_bounds__(64 * NW) void k_y_window(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst,
                                                      Phys ph, LineSet<T> ls, int L, int h, int ncs, NormOut no) {
    using C = cx<T>;
    constexpr int CPB = 4 * NW;  // columns per block
    __shared__ double shr[16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int seg = lane & 15, cw = lane >> 4;
    const int cs = blockIdx.x % ncs, rt = blockIdx.x / ncs;
    const int i = cs * CPB + wv * 4 + cw;
    const bool col_ok = i < ph.nx;
    const int nx = ph.nx, ny = ph.ny;
    const size_t plane = (size_t)nx * ny;
    const int j0 = rt * L;
    const int g0 = j0 - h + seg * KY;  // first row of this lane
    C v[3][KY];
#pragma unroll
    for (int k = 0; k < KY; ++k) {
        const int g = g0 + k;
        const bool ok = col_ok && g >= 0 && g < ny;
        const size_t o = (size_t)(ok ? g : 0) * nx + (col_ok ? i : 0);
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m][k] = ok ? src[m * plane + o] : zero_c<C>();
    }
#pragma unroll
    for (int k = 0; k < KY; ++k) to_sx<C, T>(v[0][k], v[1][k], v[2][k]);
    // rows just above and below this lane's segment (zeros outside the window)
    C up[3], dn[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        up[q] = dpp_c<0x111>(zero_c<C>(), v[q][KY - 1]);  // row_shr:1
        dn[q] = dpp_c<0x101>(zero_c<C>(), v[q][0]);       // row_shl:1
    }
    const int il = col_ok ? i : 0;
    auto fs = [](const C (&P)[3], const C (&E)[3], C (&o)[3]) { seg16_scan3<true>(P, E, o); };
    auto bs = [](const C (&P)[3], const C (&E)[3], C (&o)[3]) { seg16_scan3<false>(P, E, o); };
    block_solve3<T, KY, IMAG>(v, up, dn, ls, il * 3, g0, ny, fs, bs);
#pragma unroll
    for (int k = 0; k < KY; ++k) from_sx<C, T>(v[0][k], v[1][k], v[2][k]);
    double acc = 0;
#pragma unroll
    for (int k = 0; k < KY; ++k) {
        const int g = g0 + k;
        if (col_ok && g >= j0 && g < j0 + L && g < ny) {
            const size_t o = (size_t)g * nx + i;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                dst[m * plane + o] = v[m][k];
                if (NORM) acc += (double)cnorm2(v[m][k]);
            }
        }
    }
    if (NORM) store_norm_partial(block_sum(acc, shr), no);
}

// ---------------------------------------------------------------------------
// y sweep, exact per-thread Thomas down whole columns (increment form): the
// forward eliminations go to dst, the back substitution re-reads src.
// ---------------------------------------------------------------------------
template <typename T, bool IMAG, bool NORM>
__global__ __launch_bounds__(256) void k_y_thomas(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, Phys ph,
                                                 LineSet<T> ls, NormOut no) {
    using C = cx<T>;
    __shared__ double shr[16];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nx = ph.nx, ny = ph.ny;
    const size_t plane = (size_t)nx * ny;
    double acc = 0;
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
                for (int m = 0; m < 3; ++m) o[m] = src[m * plane + (size_t)g * nx + i];
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
            for (int m = 0; m < 3; ++m) dst[m * plane + (size_t)g * nx + i] = d[m];
        }
        C x[3] = {zero_c<C>(), zero_c<C>(), zero_c<C>()};
        for (int g = ny - 1; g >= 0; --g) {
            C o[3], uu[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) o[m] = dst[m * plane + (size_t)g * nx + i];
            load_sx(g, uu);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const Piv<T> pv = (g < ls.K) ? piv_at(ls, i * 3 + q, g) : lim[q];
                x[q] = csub(o[q], cmul(pv.cp, x[q]));
                o[q] = cadd(uu[q], x[q]);
            }
            from_sx<C, T>(o[0], o[1], o[2]);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                dst[m * plane + (size_t)g * nx + i] = o[m];
                if (NORM) acc += (double)cnorm2(o[m]);
            }
        }
    }
    if (NORM) store_norm_partial(block_sum(acc, shr), no);
}

// ---------------------------------------------------------------------------
// Small kernels.
// ---------------------------------------------------------------------------
template <typename T, bool IMAG>
__global__ __launch_bounds__(256) void k_local(cx<T>* __restrict__ psi, Phys ph) {
    const size_t plane = (size_t)ph.nx * ph.ny;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < plane; idx += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % ph.nx), j = (int)(idx / ph.nx);
        const T x = (T)(ph.x0 + i * ph.dx), y = (T)(ph.y0 + j * ph.dy);
        cx<T> p = psi[idx], z = psi[plane + idx], m = psi[2 * plane + idx];
        local_substep<T, IMAG>(p, z, m, (T)0.5 * (x * x + y * y), (T)ph.dt, (T)ph.c0, (T)ph.c2, (T)ph.rabi);
        psi[idx] = p; psi[plane + idx] = z; psi[2 * plane + idx] = m;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scale(cx<T>* __restrict__ psi, size_t n, const double* __restrict__ scale) {
    const T s = (T)(*scale);
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x)
        psi[idx] = cscale(psi[idx], s);
}

template <typename T>
__global__ __launch_bounds__(256) void k_norm_partials(const cx<T>* __restrict__ psi, size_t n, double* __restrict__ partials) {
    __shared__ double shr[16];
    double acc = 0;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x)
        acc += (double)cnorm2(psi[idx]);
    const double tot = block_sum(acc, shr);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ void k_set_scale(double* scale, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *scale = v;
}

// Sum the per-block partial norms in a fixed order; scale = 1/sqrt(dx dy sum).
__global__ __launch_bounds__(256) void k_norm_finalize(const double* __restrict__ partials, int n, double dxdy,
                                                      double* __restrict__ scale, int* __restrict__ flag) {
    __shared__ double shr[16];
    double acc = 0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) acc += partials[k];
    const double tot = block_sum(acc, shr);
    if (threadIdx.x == 0) {
        const double nn = tot * dxdy;
        if (nn > 0.0 && isfinite(nn)) {
            *scale = 1.0 / sqrt(nn);
        } else {
            *scale = 1.0;
            *flag = 1;
        }
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
__global__ __launch_bounds__(256) void k_obs(const cx<T>* __restrict__ psi, Phys ph, ObsArgs oa,
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
        const cx<T> z = psi[m * plane + (size_t)j * nx + i];
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
        const double V = 0.5 * (x * x + y * y);
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
// Launchers.
// ---------------------------------------------------------------------------

template <typename T, bool IMAG, bool LOCAL, bool SCALE>
static hipError_t launch_x_k(int K, const cx<T>* src, cx<T>* dst, const Phys& ph, const LineSet<T>& ls,
                             const double* scale, int G, int R, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const int nblk = (ph.ny + R - 1) / R;
    const dim3 grid(nblk), block(G * R);
    if (G * R > xk_bound(K) || G % 64 || G / 64 > 16 || R > 8) return hipErrorInvalidValue;

    switch (K) {
        case 1: hipExtLaunchKernelGGL(k_x_scan<T, IMAG, 1, LOCAL, SCALE, xk_bound(1)>, grid, block, 0, st, e0, e1, 0, src, dst, ph, ls, scale, G, R); break;
        case 2: hipExtLaunchKernelGGL(k_x_scan<T, IMAG, 2, LOCAL, SCALE, xk_bound(2)>, grid, block, 0, st, e0, e1, 0, src, dst, ph, ls, scale, G, R); break;
        case 4: hipExtLaunchKernelGGL(k_x_scan<T, IMAG, 4, LOCAL, SCALE, xk_bound(4)>, grid, block, 0, st, e0, e1, 0, src, dst, ph, ls, scale, G, R); break;
        case 8: hipExtLaunchKernelGGL(k_x_scan<T, IMAG, 8, LOCAL, SCALE, xk_bound(8)>, grid, block, 0, st, e0, e1, 0, src, dst, ph, ls, scale, G, R); break;
        case 16: hipExtLaunchKernelGGL(k_x_scan<T, IMAG, 16, LOCAL, SCALE, xk_bound(16)>, grid, block, 0, st, e0, e1, 0, src, dst, ph, ls, scale, G, R); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_x(const XLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (a.imag) {
        if (a.local) return launch_x_k<T, true, true, true>(a.K, a.src, a.dst, a.ph, a.ls, a.scale, a.G, a.R, st, e0, e1);
        return launch_x_k<T, true, false, false>(a.K, a.src, a.dst, a.ph, a.ls, a.scale, a.G, a.R, st, e0, e1);
    }
    if (a.local) return launch_x_k<T, false, true, false>(a.K, a.src, a.dst, a.ph, a.ls, a.scale, a.G, a.R, st, e0, e1);
    return launch_x_k<T, false, false, false>(a.K, a.src, a.dst, a.ph, a.ls, a.scale, a.G, a.R, st, e0, e1);
}

template <typename T, bool IMAG, bool NORM, int TI>
static hipError_t launch_yw_t(const YLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    constexpr YTile yt = ytile<T>(TI);
    const int ncs = (a.ph.nx + 4 * yt.NW - 1) / (4 * yt.NW);
    const int nrt = (a.ph.ny + a.L - 1) / a.L;
    hipExtLaunchKernelGGL(k_y_window<T, IMAG, yt.KY, yt.NW, NORM>, dim3(ncs * nrt), dim3(64 * yt.NW), 0, st, e0, e1, 0,
                          a.src, a.dst, a.ph, a.ls, a.L, a.h, ncs, a.no);
    return hipGetLastError();
}

template <typename T, bool IMAG, bool NORM>
static hipError_t launch_yw(const YLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    switch (a.tile) {
        case 0: return launch_yw_t<T, IMAG, NORM, 0>(a, st, e0, e1);
        case 1: return launch_yw_t<T, IMAG, NORM, 1>(a, st, e0, e1);
        case 2: return launch_yw_t<T, IMAG, NORM, 2>(a, st, e0, e1);
        case 3: return launch_yw_t<T, IMAG, NORM, 3>(a, st, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
int y_blocks(const YLaunch<T>& a) {
    if (a.window) {
        const YTile yt = ytile<T>(a.tile);
        const int ncs = (a.ph.nx + 4 * yt.NW - 1) / (4 * yt.NW);
        return ncs * ((a.ph.ny + a.L - 1) / a.L);
    }
    return (a.ph.nx + 255) / 256;
}

template <typename T>
hipError_t launch_y(const YLaunch<T>& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (a.window) {
        if (a.imag) return a.norm ? launch_yw<T, true, true>(a, st, e0, e1) : launch_yw<T, true, false>(a, st, e0, e1);
        return a.norm ? launch_yw<T, false, true>(a, st, e0, e1) : launch_yw<T, false, false>(a, st, e0, e1);
    }
    const dim3 grid((a.ph.nx + 255) / 256), block(256);
    if (a.imag) {
        if (a.norm) hipExtLaunchKernelGGL(k_y_thomas<T, true, true>, grid, block, 0, st, e0, e1, 0, a.src, a.dst, a.ph, a.ls, a.no);
        else hipExtLaunchKernelGGL(k_y_thomas<T, true, false>, grid, block, 0, st, e0, e1, 0, a.src, a.dst, a.ph, a.ls, a.no);
    } else {
        if (a.norm) hipExtLaunchKernelGGL(k_y_thomas<T, false, true>, grid, block, 0, st, e0, e1, 0, a.src, a.dst, a.ph, a.ls, a.no);
        else hipExtLaunchKernelGGL(k_y_thomas<T, false, false>, grid, block, 0, st, e0, e1, 0, a.src, a.dst, a.ph, a.ls, a.no);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_local(cx<T>* psi, const Phys& ph, bool imag, hipStream_t st) {
    const size_t n = (size_t)ph.nx * ph.ny;
    const int nblk = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    if (imag) k_local<T, true><<<nblk, 256, 0, st>>>(psi, ph);
    else k_local<T, false><<<nblk, 256, 0, st>>>(psi, ph);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale(cx<T>* psi, size_t n, const double* scale, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const int nblk = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    hipExtLaunchKernelGGL(k_scale<T>, dim3(nblk), dim3(256), 0, st, e0, e1, 0, psi, n, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_norm_partials(const cx<T>* psi, size_t n, double* partials, int nblk, hipStream_t st) {
    k_norm_partials<T><<<nblk, 256, 0, st>>>(psi, n, partials);
    return hipGetLastError();
}

hipError_t launch_set_scale(double* scale, double v, hipStream_t st) {
    k_set_scale<<<1, 64, 0, st>>>(scale, v);
    return hipGetLastError();
}

hipError_t launch_norm_finalize(const double* partials, int n, double dxdy, double* scale, int* flag, hipStream_t st,
                                hipEvent_t e0, hipEvent_t e1) {
    hipExtLaunchKernelGGL(k_norm_finalize, dim3(1), dim3(256), 0, st, e0, e1, 0, partials, n, dxdy, scale, flag);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_obs(const cx<T>* psi, const Phys& ph, const ObsLaunch& o, T* dens, double* partials, int nblk,
                      hipStream_t st) {
    ObsArgs oa{o.c0, o.c2, o.rabi, o.gamma, o.omega, o.eta};
    k_obs<T><<<nblk, 256, 0, st>>>(psi, ph, oa, dens, partials);
    return hipGetLastError();
}

hipError_t launch_obs_finalize(const double* partials, int nblk, double* out, hipStream_t st) {
    k_obs_finalize<<<1, 256, 0, st>>>(partials, nblk, out);
    return hipGetLastError();
}

#define GP_INST(T)                                                                                             \
    template hipError_t launch_x<T>(const XLaunch<T>&, hipStream_t, hipEvent_t, hipEvent_t);                   \
    template hipError_t launch_y<T>(const YLaunch<T>&, hipStream_t, hipEvent_t, hipEvent_t);                   \
    template int y_blocks<T>(const YLaunch<T>&);                                                               \
    template hipError_t launch_local<T>(cx<T>*, const Phys&, bool, hipStream_t);                               \
    template hipError_t launch_scale<T>(cx<T>*, size_t, const double*, hipStream_t, hipEvent_t, hipEvent_t);   \
    template hipError_t launch_norm_partials<T>(const cx<T>*, size_t, double*, int, hipStream_t);              \
    template hipError_t launch_obs<T>(const cx<T>*, const Phys&, const ObsLaunch&, T*, double*, int, hipStream_t);
GP_INST(double)
GP_INST(float)

}  // namespace gp
