// Line solves with short-range carries ("chain" windows).
//
// The windowed sweeps solve each line (converged Thomas pivots, increment
// form; see gp_solve.hpp) over windows of lanes, K consecutive points per
// lane, with zero carries at the window ends; a window writes only the points
// at least h from both of its ends, h such that a carry decays below the
// rounding level of T over h points (decay^h).  The exact partitioned Thomas
// inside the window composes every lane's transfer map with all the maps
// before it (a scan).  But with the converged pivots a lane passes on
// P = (-a m)^K times the carry it receives (forward; R = (-e m)^K backward),
// so a lane more than nc = ceil((h - 1) / K) lanes away reaches a point only
// through nc whole lanes and at least one point of the receiving lane, i.e.
// through at least h points: below the rounding level, like the carries the
// window ends drop.  The carry entering lane l is therefore formed from the
// nc lanes before it,
//     c_in(l) = sum_{j=1..nc} P^{j-1} e(l - j),
// e(k) the value lane k passes on from a zero carry: nc shifts of one lane,
// each after a multiply-add (no scan, no shared memory), and every point at
// least h from both window ends is exact to the rounding level, as in the
// scanned windows.
//
// Each pass runs twice per lane: once from a zero carry for the value it
// passes on, once from the true carry for its points (no running products of
// the multipliers, fewer registers than keeping the zero-carry values).
//
// Lines that end inside a window (EDGE): points outside [0, n) hold zeros; their
// right-hand sides are zeroed, and past the line end the forward values are
// zeroed as well, so that no carry crosses the line ends in either direction.
#pragma once

#include "gp_solve.hpp"

namespace gp {

// One lane towards higher lanes (UP: lane l receives lane l - 1) or lower
// lanes, across the whole wave (WAVE) or within rows of 16 lanes; lanes
// without a source lane receive zero.
template <bool WAVE, bool UP, typename C> __device__ inline C lane_step(C v) {
    if constexpr (WAVE) return UP ? dpp_c<0x138>(zero_c<C>(), v) : dpp_c<0x130>(zero_c<C>(), v);  // wave_shr:1 / wave_shl:1
    else return UP ? dpp_c<0x111>(zero_c<C>(), v) : dpp_c<0x101>(zero_c<C>(), v);                 // row_shr:1 / row_shl:1
}

// sum_{j=1..nc} f^{j-1} e(l -+ j): nc shifts, each after a multiply-add.
template <bool WAVE, bool UP, typename C> __device__ inline C carry_chain(C e, C f, int nc) {
    C x = lane_step<WAVE, UP>(e);
    for (int t = 1; t < nc; ++t) x = lane_step<WAVE, UP>(cfma(x, f, e));
    return x;
}

// Buffer loads and stores of one complex value at a 32-bit byte offset from a
// plane's base (the base and size in scalar registers, the offset in one
// vector register that serves every plane); accesses past the plane's size
// read zeros and write nothing.
__device__ inline __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename C> __device__ inline C buf_load(__amdgpu_buffer_rsrc_t r, unsigned off);
template <> __device__ inline double2 buf_load<double2>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}
template <> __device__ inline float2 buf_load<float2>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ inline void buf_store(double2 v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    using V = __attribute__((ext_vector_type(4))) unsigned int;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V, v), r, (int)off, 0, 0);
}
__device__ inline void buf_store(float2 v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    using V = __attribute__((ext_vector_type(2))) unsigned int;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, (int)off, 0, 0);
}

// The factors of one line's converged elimination.
template <typename T> struct ChainLine {
    cx<T> a, e;    // sub- and super-diagonal
    cx<T> m2;      // -2 / w (w the converged pivot): the right-hand side's -2 folded into 1 / w
    cx<T> nam;     // -a / w
    cx<T> ncp;     // -e / w
    cx<T> P, R;    // nam^K, ncp^K: the carry a lane passes on per unit carry received
};

template <typename T, int K> __device__ inline ChainLine<T> chain_line(const LineSet<T>& ls, int line) {
    using C = cx<T>;
    ChainLine<T> c;
    c.a = ls.ae[2 * line];
    c.e = ls.ae[2 * line + 1];
    const Piv<T> lim = ls.piv[(size_t)line * (ls.K + 1) + ls.K];
    c.m2 = cscale(lim.m, (T)-2);
    c.nam = cneg(lim.am);
    c.ncp = cneg(lim.cp);
    c.P = cpow_k<C, K>(c.nam);
    c.R = cpow_k<C, K>(c.ncp);
    return c;
}

// One line, K points per lane at line indices g0 .. g0 + K - 1 (n points in
// the line), neighbours um / up of the lane's first and last point, nc lanes
// of carry.  In place on u (u += the increment).  kpick >= 0: the increment
// at the lane's point kpick goes to d0 (the line-start correction).
template <typename T, int K, bool IMAG, bool WAVE, bool EDGE>
__device__ inline void chain_solve(cx<T> (&u)[K], cx<T> um, cx<T> up, const ChainLine<T>& c, cx<T> bm1, int nc,
                                   int g0, int n, int kpick, cx<T>& d0) {
    using C = cx<T>;
    C v[K];
    // m r_k with r_k = -2 ((b - 1) u_k + a u_{k-1} + e u_{k+1})
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const C l = k == 0 ? um : u[k - 1];
        const C r = k == K - 1 ? up : u[k + 1];
        C t = mul_bm1<T, IMAG>(bm1, u[k]);
        t = cfma(l, c.a, t);
        t = cfma(r, c.e, t);
        v[k] = cmul(c.m2, t);
        if (EDGE && (g0 + k < 0 || g0 + k >= n)) v[k] = zero_c<C>();
    }
    // forward: the value passed on from a zero carry, the carry in, the values
    C f = v[0];
#pragma unroll
    for (int k = 1; k < K; ++k) f = cfma(f, c.nam, v[k]);
    C x = carry_chain<WAVE, true>(f, c.P, nc);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        x = cfma(x, c.nam, v[k]);
        if (EDGE && g0 + k >= n) x = zero_c<C>();
        v[k] = x;
    }
    // backward, the same way round from the line end
    C b = v[K - 1];
#pragma unroll
    for (int k = K - 2; k >= 0; --k) b = cfma(b, c.ncp, v[k]);
    x = carry_chain<WAVE, false>(b, c.R, nc);
#pragma unroll
    for (int k = K - 1; k >= 0; --k) {
        x = cfma(x, c.ncp, v[k]);
        if (k == kpick) d0 = x;
        u[k] = cadd(u[k], x);
    }
}

// The three eigen-lines of a window (lines line0 .. line0 + 2), one after
// another (SEQ: one line's temporaries live at a time) or interleaved.
// first: the window holds line point 0, at point k0 of lane src0; its
// increment there feeds the line-start correction (Sherman-Morrison, see
// LineSet) of the points g < Kg.  Every lane of the wave takes part in the
// gathers and shifts.
template <typename T, int K, bool IMAG, bool WAVE, bool EDGE, bool SEQ>
__device__ inline void chain_lines(cx<T> (&u)[3][K], const LineSet<T>& ls, int line0, int nc, int g0, int n,
                                   bool first, int src0, int k0) {
    using C = cx<T>;
    const int kpick = first ? k0 : -1;
    if constexpr (SEQ) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const C um = lane_step<WAVE, true>(u[q][K - 1]);
            const C up = lane_step<WAVE, false>(u[q][0]);
            const ChainLine<T> c = chain_line<T, K>(ls, line0 + q);
            C d0 = zero_c<C>();
            chain_solve<T, K, IMAG, WAVE, EDGE>(u[q], um, up, c, ls.bm1, nc, g0, n, kpick, d0);
            if (first) line_start_fix<T, K>(u[q], ls, line0 + q, bperm_c(d0, src0), g0);
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        C um[3], up[3], d0[3];
        ChainLine<T> c[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            um[q] = lane_step<WAVE, true>(u[q][K - 1]);
            up[q] = lane_step<WAVE, false>(u[q][0]);
            c[q] = chain_line<T, K>(ls, line0 + q);
            d0[q] = zero_c<C>();
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) chain_solve<T, K, IMAG, WAVE, EDGE>(u[q], um[q], up[q], c[q], ls.bm1, nc, g0, n, kpick, d0[q]);
        if (first) {
#pragma unroll
            for (int q = 0; q < 3; ++q) line_start_fix<T, K>(u[q], ls, line0 + q, bperm_c(d0[q], src0), g0);
        }
    }
}

}  // namespace gp
