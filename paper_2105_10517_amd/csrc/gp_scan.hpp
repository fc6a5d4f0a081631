// Scans of affine maps z -> P z + E over the threads that share one line.
//
// A tridiagonal line split into consecutive blocks (one block per thread) is
// solved exactly by Thomas elimination in three moves per direction: every
// thread runs the recurrence over its own block from a zero carry, the block
// transfer maps are composed across threads by a scan, and each thread adds
// the carry that enters its block times the running product of its
// multipliers.  The scans below return the exclusive prefix, i.e. the carry
// that enters each thread's block.  Composition order: (f o g)(z) = f(g(z)),
// with g the map nearer the start of the scan direction.
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

// Exclusive scan across the S segments of a column tile.  Thread (c, s) sits
// at index c + TW s, so one wave holds SPW = 64/TW consecutive segments of the
// same TW columns: the scan runs by shuffles across lanes TW apart inside a
// wave, and through shared memory (shP/shE: (S/SPW) * TW entries) across waves.
// REV = false: carry from segments 0..s-1; REV = true: from s+1..S-1.
template <typename C, int TW, int S, bool REV>
__device__ inline C seg_scan(C P, C E, int c, int s, C* shP, C* shE) {
    constexpr int SPW = 64 / TW, NWV = S / SPW;
    const int sw = s % SPW, w = s / SPW;
#pragma unroll
    for (int off = 1; off < SPW; off <<= 1) {
        const C Po = REV ? shfl_down_c(P, off * TW) : shfl_up_c(P, off * TW);
        const C Eo = REV ? shfl_down_c(E, off * TW) : shfl_up_c(E, off * TW);
        if (REV ? (sw + off < SPW) : (sw >= off)) { E = cfma(Eo, P, E); P = cmul(P, Po); }
    }
    // wave totals: the inclusive map of the last segment of each wave in scan order
    if (REV ? (sw == 0) : (sw == SPW - 1)) { shP[w * TW + c] = P; shE[w * TW + c] = E; }
    __syncthreads();
    C din = zero_c<C>();
    if (!REV) {
        for (int v = 0; v < w; ++v) din = cfma(din, shP[v * TW + c], shE[v * TW + c]);
    } else {
        for (int v = NWV - 1; v > w; --v) din = cfma(din, shP[v * TW + c], shE[v * TW + c]);
    }
    const C incl = cfma(din, P, E);
    C ex = REV ? shfl_down_c(incl, TW) : shfl_up_c(incl, TW);
    if (REV ? (sw == SPW - 1) : (sw == 0)) ex = din;
    __syncthreads();
    return ex;
}

}  // namespace gp
