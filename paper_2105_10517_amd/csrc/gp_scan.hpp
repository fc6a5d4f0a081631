// Scans of affine maps z -> P z + E over the threads that share one line.
//
// A tridiagonal line split into consecutive blocks (one block per thread) is
// solved exactly by Thomas elimination in three moves per direction: every
// thread runs the recurrence over its own block from a zero carry, the block
// transfer maps are composed across threads by a scan, and each thread adds
// the carry that enters its block times the running product of its
// multipliers.  The scans below return the exclusive prefix, i.e. the carry
// that enters each thread's block.
#pragma once

#include "gp_device.hpp"

namespace gp {

// Forward exclusive scan over the G = 64 * nw threads of one row (thread t =
// 64 w + lane).  shP/shE: >= nw entries of shared memory private to the row.
// Every thread of the block must call it (it contains barriers).
template <typename C>
__device__ inline C row_scan_fwd(C P, C E, int lane, int w, int nw, C* shP, C* shE) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const C Pp = shfl_up_c(P, off), Ep = shfl_up_c(E, off);
        if (lane >= off) { E = cfma(Ep, P, E); P = cmul(P, Pp); }
    }
    if (lane == 63) { shP[w] = P; shE[w] = E; }
    __syncthreads();
    C din = zero_c<C>();
    for (int v = 0; v < w; ++v) din = cfma(din, shP[v], shE[v]);
    const C incl = cfma(din, P, E);
    C ex = shfl_up_c(incl, 1);
    if (lane == 0) ex = din;
    __syncthreads();
    return ex;
}

// Backward exclusive scan: the carry entering thread t from the right is
// (g_{t+1} o g_{t+2} o ... o g_{G-1})(0).
template <typename C>
__device__ inline C row_scan_bwd(C P, C E, int lane, int w, int nw, C* shP, C* shE) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const C Pn = shfl_down_c(P, off), En = shfl_down_c(E, off);
        if (lane + off < 64) { E = cfma(En, P, E); P = cmul(P, Pn); }
    }
    if (lane == 0) { shP[w] = P; shE[w] = E; }
    __syncthreads();
    C din = zero_c<C>();
    for (int v = nw - 1; v > w; --v) din = cfma(din, shP[v], shE[v]);
    const C incl = cfma(din, P, E);
    C ex = shfl_down_c(incl, 1);
    if (lane == 63) ex = din;
    __syncthreads();
    return ex;
}

// Exclusive scan across the S segments of a column tile, thread (c, s) at
// index c + TW s; Kogge-Stone through shared memory (shP/shE: S*TW entries).
// REV = false: carry from segments 0..s-1; REV = true: from s+1..S-1.
template <typename C, int TW, int S, bool REV>
__device__ inline C seg_scan(C P, C E, int c, int s, C* shP, C* shE) {
    const int idx = c + TW * s;
#pragma unroll
    for (int off = 1; off < S; off <<= 1) {
        shP[idx] = P; shE[idx] = E;
        __syncthreads();
        const int o = REV ? s + off : s - off;
        if (REV ? (o < S) : (o >= 0)) {
            const C Po = shP[c + TW * o], Eo = shE[c + TW * o];
            E = cfma(Eo, P, E);
            P = cmul(P, Po);
        }
        __syncthreads();
    }
    // inclusive value -> exclusive: take the neighbour's inclusive map applied to 0
    shE[idx] = E;
    __syncthreads();
    const int o = REV ? s + 1 : s - 1;
    C ex = (REV ? (o < S) : (o >= 0)) ? shE[c + TW * o] : zero_c<C>();
    __syncthreads();
    return ex;
}

}  // namespace gp
