// Line solves and block reductions shared by the sweep kernels.
#pragma once

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
// Partitioned Thomas on NQ lines held as K consecutive values per thread
// (indices i0 .. i0+K-1 of lines of length n; indices outside [0, n) are
// padding), in place on u[][]; left/right are the line values just outside
// the thread's block.  FS and BS are the forward and backward exclusive scans
// of the block transfer maps across the threads sharing the lines; every
// thread must reach them (they may contain barriers).
//
// Every point uses the converged pivots (kept in registers): that factors the
// matrix A_inf whose first diagonal entry is the limit pivot instead of b.
// The carries are cut at the line ends (the forward carry into point 0, the
// backward carry into point n - 1), so the result is z = A_inf^{-1} r; the
// caller turns it into A^{-1} r with line_start_fix (a rank-one correction
// of the first LineSet::Kg points).  One code path for every thread: no
// divergence between the threads that hold the start of a line and the rest.
// ---------------------------------------------------------------------------
template <typename T, bool IMAG> __device__ inline cx<T> mul_bm1(cx<T> bm1, cx<T> u) {
    // b - 1 = alpha / dx^2: real in imaginary time, imaginary in real time
    return IMAG ? cscale(u, bm1.x) : cscale(ctimes_i(u), bm1.y);
}
template <typename C> __device__ inline C cneg(C a) { C z; z.x = -a.x; z.y = -a.y; return z; }

// Per-line coefficients of a solve: sub- and super-diagonal (a, e) and the
// converged pivots.  Loaded by the caller, so that a kernel can issue these
// loads together with its wave-function loads, ahead of any barrier.
template <typename T> struct LineCoef {
    cx<T> a, e;
    Piv<T> lim;
};
template <typename T, int NQ>
__device__ inline void line_coefs(const LineSet<T>& ls, int line0, LineCoef<T> (&cf)[NQ]) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int line = line0 + q;
        cf[q].a = ls.ae[2 * line];
        cf[q].e = ls.ae[2 * line + 1];
        cf[q].lim = ls.piv[(size_t)line * (ls.K + 1) + ls.K];
    }
}

template <typename C, int K> __device__ inline C cpow_k(C a) {
    C r = one_c<C>(), b = a;
#pragma unroll
    for (int k = K; k > 0; k >>= 1) {
        if (k & 1) r = cmul(r, b);
        b = cmul(b, b);
    }
    return r;
}

// dk: the increment at the thread's point kpick (the caller's index of line
// point 0, for the line-start correction; kpick < 0: none).
template <typename T, int K, bool IMAG, int NQ, typename FS, typename BS>
__device__ inline void block_solve(cx<T> (&u)[NQ][K], const cx<T> (&left)[NQ], const cx<T> (&right)[NQ],
                                   const LineSet<T>& ls, const LineCoef<T> (&cf)[NQ], int i0, int n, FS fscan,
                                   BS bscan, int kpick, cx<T> (&dk)[NQ]) {
    using C = cx<T>;
    C nam[NQ], ncp[NQ], lm[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        lm[q] = cf[q].lim.m;
        nam[q] = cneg(cf[q].lim.am);
        ncp[q] = cneg(cf[q].lim.cp);
        dk[q] = zero_c<C>();
    }
    // right-hand side of the increment system: r = -2 ((b - 1) u_k + a u_{k-1} + e u_{k+1})
    C r[NQ][K];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const C um = (k == 0) ? left[q] : u[q][k - 1];
            const C up = (k == K - 1) ? right[q] : u[q][k + 1];
            C t = mul_bm1<T, IMAG>(ls.bm1, u[q][k]);
            t = cfma(um, cf[q].a, t);
            t = cfma(up, cf[q].e, t);
            r[q][k] = cscale(t, (T)-2);
        }
    // forward elimination over the block from a zero carry: E_k = m r_k - am E_{k-1};
    // points i <= 0 take no carry (the line starts at 0)
    // (the block's product of -am: a running product for short blocks, fewer
    // registers; closed-form powers for K >= 8, a shorter dependent chain)
    C E[NQ], P[NQ], din[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) { E[q] = zero_c<C>(); P[q] = one_c<C>(); }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const bool cut = i0 + k <= 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const C na = cut ? zero_c<C>() : nam[q];
            E[q] = cfma(E[q], na, cmul(lm[q], r[q][k]));
            if constexpr (K < 8) P[q] = cmul(P[q], na);
            r[q][k] = E[q];
        }
    }
    if constexpr (K >= 8) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) P[q] = i0 <= 0 ? zero_c<C>() : cpow_k<C, K>(nam[q]);
    }
    fscan(P, E, din);
    // add the carry that enters the block, times the running product of -am
    {
        C Q[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) Q[q] = one_c<C>();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const bool cut = i0 + k <= 0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                Q[q] = cmul(Q[q], cut ? zero_c<C>() : nam[q]);
                r[q][k] = cfma(din[q], Q[q], r[q][k]);
            }
        }
    }
    // back substitution over the block from a zero carry: G_k = r_k - cp G_{k+1};
    // points i >= n - 1 take no carry (the line ends at n - 1)
    C G[NQ], R[NQ], xin[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) { G[q] = zero_c<C>(); R[q] = one_c<C>(); }
#pragma unroll
    for (int k = K - 1; k >= 0; --k) {
        const bool cut = i0 + k >= n - 1;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const C nc = cut ? zero_c<C>() : ncp[q];
            G[q] = cfma(G[q], nc, r[q][k]);
            if constexpr (K < 8) R[q] = cmul(nc, R[q]);
            r[q][k] = G[q];
        }
    }
    if constexpr (K >= 8) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) R[q] = i0 + K >= n ? zero_c<C>() : cpow_k<C, K>(ncp[q]);
    }
    bscan(R, G, xin);
    {
        C Sx[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) Sx[q] = one_c<C>();
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
            const bool cut = i0 + k >= n - 1;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                Sx[q] = cmul(Sx[q], cut ? zero_c<C>() : ncp[q]);
                const C d = cfma(xin[q], Sx[q], r[q][k]);
                if (k == kpick) dk[q] = d;
                u[q][k] = cadd(u[q][k], d);
            }
        }
    }
}


// Line-start correction (Sherman-Morrison, see LineSet): the points
// i0 .. i0 + K - 1 of line `line` lose gc d0 g_i, d0 being the increment the
// solve gave line point 0.
template <typename T, int K>
__device__ inline void line_start_fix(cx<T> (&u)[K], const LineSet<T>& ls, int line, cx<T> d0, int i0) {
    if (i0 >= ls.Kg || i0 + K <= 0) return;
    const cx<T> f = cmul(ls.gc[line], d0);
    const cx<T>* g = ls.g + (size_t)line * ls.Kg;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = i0 + k;
        if (i >= 0 && i < ls.Kg) u[k] = csub(u[k], cmul(f, g[i]));
    }
}

// The three eigen-lines of a window held by a DPP row of 16 lanes (K points
// per lane, lines line0 .. line0 + 2 of the LineSet), solved interleaved
// through one scan per direction, or (SEQ) one line after another, each with
// its own segment neighbours and line-start correction (so that only one
// line's extras are live at a time).  The scheduling barriers keep the
// compiler from re-interleaving the sequential solves, which would undo the
// register saving.  The points just before and after a lane's segment come
// from the neighbouring lanes of the DPP row (zeros outside the window).
// first: the window holds line point 0 (in segment seg0, at point k0 of that
// lane); then the line-start correction is applied with the increment at that
// point, gathered from its lane of the DPP row (every lane of the wave takes
// part in the gather).
template <typename T, int K, bool IMAG, int Q>
__device__ inline void window_line(cx<T> (&u)[3][K], const LineSet<T>& ls, int line0, int i0, int n, bool first,
                                   int seg0, int k0, int lane) {
    using C = cx<T>;
    auto fs = [](const C (&P)[1], const C (&E)[1], C (&o)[1]) { seg16_scan<true, 1>(P, E, o); };
    auto bs = [](const C (&P)[1], const C (&E)[1], C (&o)[1]) { seg16_scan<false, 1>(P, E, o); };
    const C l1[1] = {dpp_c<0x111>(zero_c<C>(), u[Q][K - 1])};  // row_shr:1
    const C r1[1] = {dpp_c<0x101>(zero_c<C>(), u[Q][0])};      // row_shl:1
    LineCoef<T> cf[1];
    line_coefs<T, 1>(ls, line0 + Q, cf);
    C d1[1];
    block_solve<T, K, IMAG, 1>(reinterpret_cast<C (&)[1][K]>(u[Q]), l1, r1, ls, cf, i0, n, fs, bs, first ? k0 : -1, d1);
    if (first) line_start_fix<T, K>(u[Q], ls, line0 + Q, bperm_c(d1[0], (lane & ~15) + seg0), i0);
}

template <typename T, int K, bool IMAG, bool SEQ>
__device__ inline void window_solve(cx<T> (&u)[3][K], const LineSet<T>& ls, int line0, int i0, int n, bool first,
                                    int seg0, int k0, int lane) {
    using C = cx<T>;
    if constexpr (SEQ) {
        window_line<T, K, IMAG, 0>(u, ls, line0, i0, n, first, seg0, k0, lane);
        __builtin_amdgcn_sched_barrier(0);
        window_line<T, K, IMAG, 1>(u, ls, line0, i0, n, first, seg0, k0, lane);
        __builtin_amdgcn_sched_barrier(0);
        window_line<T, K, IMAG, 2>(u, ls, line0, i0, n, first, seg0, k0, lane);
    } else {
        C lf[3], rg[3], d[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            lf[q] = dpp_c<0x111>(zero_c<C>(), u[q][K - 1]);  // row_shr:1
            rg[q] = dpp_c<0x101>(zero_c<C>(), u[q][0]);       // row_shl:1
        }
        auto fs = [](const C (&P)[3], const C (&E)[3], C (&o)[3]) { seg16_scan<true, 3>(P, E, o); };
        auto bs = [](const C (&P)[3], const C (&E)[3], C (&o)[3]) { seg16_scan<false, 3>(P, E, o); };
        LineCoef<T> cf[3];
        line_coefs<T, 3>(ls, line0, cf);
        block_solve<T, K, IMAG, 3>(u, lf, rg, ls, cf, i0, n, fs, bs, first ? k0 : -1, d);
        if (first) {
            // the increment at line point 0, from lane seg0 of this DPP row
            const int src = (lane & ~15) + seg0;
#pragma unroll
            for (int q = 0; q < 3; ++q) line_start_fix<T, K>(u[q], ls, line0 + q, bperm_c(d[q], src), i0);
        }
    }
}

// One line with K points per thread for long rows (K s > 32 bytes): the
// same elimination one line at a time, with the transient pivots read from
// the global table (keeps the register footprint of the long-row kernels).
template <typename T, int K, bool IMAG, typename FS, typename BS>
__device__ inline void block_solve1(cx<T> (&u)[K], cx<T> left, cx<T> right, const LineSet<T>& ls, int line, int i0,
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

// Block reduction of three doubles at once (all threads call; results valid
// in thread 0).
__device__ inline void block_sum3(double (&v)[3], double* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m] += __shfl_down(v[m], off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int m = 0; m < 3; ++m) sh[m * 16 + w] = v[m];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            double s = 0;
            for (int k = 0; k < nw; ++k) s += sh[m * 16 + k];
            v[m] = s;
        }
    __syncthreads();
}

// Per-block partial sums of the imaginary-time component norms, in block
// order; a one-block kernel launched next on the same stream forms the totals
// (a device-wide release fence per block would write back the L2 of its XCD
// every time).
__device__ inline void store_norm_partials(double (&acc)[3], double* sh, NormOut no, int blk) {
    block_sum3(acc, sh);
    if (threadIdx.x == 0)
#pragma unroll
        for (int m = 0; m < 3; ++m) no.partials[3 * blk + m] = acc[m];
}

// The total-norm branch of norm_scales alone (the same arithmetic), for
// kernels that must not hold the fixed-magnetisation branch's registers.
__device__ inline bool norm_scale_total(const double (&N)[3], double* s) {
    const double t = N[0] + N[1] + N[2];
    const double f = 1.0 / sqrt(t);
    const bool ok = isfinite(f) && f > 0.0;
    s[0] = s[1] = s[2] = ok ? f : 1.0;
    return ok;
}

// Scale factors of the three components from their norms N[m] (dx dy sum
// |psi_m|^2).  Total norm one: s_m = 1 / sqrt(N_{+1} + N_0 + N_{-1}).  Fixed
// magnetisation mag: the s_m that give total norm one, N_{+1} - N_{-1} = mag
// and s_{+1} s_{-1} = s_0^2 (normalised gradient flow of Bao and Lim):
// with u = s_0^2 the conditions give u = (1 - mag^2) / (N_0 + sqrt(mag^2 N_0^2
// + 4 (1 - mag^2) N_{+1} N_{-1})) and s_{+-1}^2 = (1 +- mag - u N_0) / (2 N_{+-1}).
// Returns false (and unit factors) when a factor is not a positive finite number.
__device__ inline bool norm_scales(const double (&N)[3], NormRule r, double* s) {
    double f0, f1, f2;
    if (r.fix_m) {
        const double m = r.mag, q = 1.0 - m * m;
        const double u = q / (N[1] + sqrt(m * m * N[1] * N[1] + 4.0 * q * N[0] * N[2]));
        f1 = sqrt(u);
        f0 = sqrt((1.0 + m - u * N[1]) / (2.0 * N[0]));
        f2 = sqrt((1.0 - m - u * N[1]) / (2.0 * N[2]));
    } else {
        const double t = N[0] + N[1] + N[2];
        f0 = f1 = f2 = 1.0 / sqrt(t);
    }
    const bool ok = isfinite(f0) && isfinite(f1) && isfinite(f2) && f0 > 0.0 && f1 > 0.0 && f2 > 0.0;
    s[0] = ok ? f0 : 1.0;
    s[1] = ok ? f1 : 1.0;
    s[2] = ok ? f2 : 1.0;
    return ok;
}

}  // namespace gp
