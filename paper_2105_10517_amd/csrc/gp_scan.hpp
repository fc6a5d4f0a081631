// Scans of affine maps z -> P z + E over the threads that share one line.
//
// A tridiagonal line split into consecutive blocks (one block per thread) is
// solved exactly by Thomas elimination in three moves per direction: every
// thread runs the recurrence over its own block from a zero carry, the block
// transfer maps are composed across threads by a scan, and each thread adds
// the carry that enters its block times the running product of its
// multipliers.  The scans below return the exclusive prefix, i.e. the carry
// that enters each thread's block.
//
// Inside a wave the scans use DPP lane moves (row_shr / row_shl within rows of
// 16 lanes, row broadcasts or ds_bpermute gathers across the four rows,
// wave_shr / wave_shl for the final shift); across the waves of a row they go
// through shared memory.
#pragma once

#include "gp_device.hpp"

namespace gp {

template <typename C> struct Aff { C P, E; };

// (f o g)(z) = f(g(z)): g applies first.
template <typename C> __device__ inline Aff<C> compose(const Aff<C>& f, const Aff<C>& g) {
    return Aff<C>{cmul(f.P, g.P), cfma(g.E, f.P, f.E)};
}
template <typename C> __device__ inline Aff<C> aff_id() { return Aff<C>{one_c<C>(), zero_c<C>()}; }

// --- DPP lane moves (lanes without a source lane keep `old`) ----------------
template <int CTRL, int RM> __device__ inline int dpp_i(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, RM, 0xF, false);
}
template <int CTRL, int RM> __device__ inline float dpp_r(float old, float v) {
    return __int_as_float(dpp_i<CTRL, RM>(__float_as_int(old), __float_as_int(v)));
}
template <int CTRL, int RM> __device__ inline double dpp_r(double old, double v) {
    const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
    const int lo = dpp_i<CTRL, RM>((int)o, (int)x);
    const int hi = dpp_i<CTRL, RM>((int)(o >> 32), (int)(x >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, int RM = 0xF, typename C> __device__ inline C dpp_c(C old, C v) {
    C z; z.x = dpp_r<CTRL, RM>(old.x, v.x); z.y = dpp_r<CTRL, RM>(old.y, v.y); return z;
}
template <int CTRL, int RM = 0xF, typename C> __device__ inline Aff<C> dpp_aff(const Aff<C>& a) {
    const Aff<C> id = aff_id<C>();
    return Aff<C>{dpp_c<CTRL, RM>(id.P, a.P), dpp_c<CTRL, RM>(id.E, a.E)};
}

// --- lane gathers through the LDS crossbar (ds_bpermute: no LDS memory) -----
__device__ inline int bperm_i(int v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }
__device__ inline float bperm_r(float v, int src) { return __int_as_float(bperm_i(__float_as_int(v), src)); }
__device__ inline double bperm_r(double v, int src) {
    const long long x = __double_as_longlong(v);
    const int lo = bperm_i((int)x, src), hi = bperm_i((int)(x >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename C> __device__ inline C bperm_c(C v, int src) {
    C z; z.x = bperm_r(v.x, src); z.y = bperm_r(v.y, src); return z;
}
template <typename C> __device__ inline Aff<C> bperm_aff(const Aff<C>& a, int src) {
    return Aff<C>{bperm_c(a.P, src), bperm_c(a.E, src)};
}

// Inclusive scans within each row of 16 lanes, NQ independent maps at once
// (their lane moves and compositions interleave).  FWD: lane l holds
// f_l o f_{l-1} o ... o f_{row start}; backward: f_l o f_{l+1} o ... o f_{row end}.
template <bool FWD, int NQ, typename C> __device__ inline void row16_incl(Aff<C> (&a)[NQ]) {
#define GP_STAGE(CTRL)                                                                \
    {                                                                                 \
        Aff<C> s[NQ];                                                                 \
        _Pragma("unroll") for (int q = 0; q < NQ; ++q) s[q] = dpp_aff<CTRL>(a[q]);   \
        _Pragma("unroll") for (int q = 0; q < NQ; ++q) a[q] = compose(a[q], s[q]);   \
    }
    if (FWD) {
        GP_STAGE(0x111) GP_STAGE(0x112) GP_STAGE(0x114) GP_STAGE(0x118)  // row_shr:1,2,4,8
    } else {
        GP_STAGE(0x101) GP_STAGE(0x102) GP_STAGE(0x104) GP_STAGE(0x108)  // row_shl:1,2,4,8
    }
#undef GP_STAGE
}

// Inclusive scan over the 64 lanes of a wave: the rows' scans, then two
// stages across rows.  Forward: DPP row broadcasts (row_bcast:15 into rows 1
// and 3, then row_bcast:31 into rows 2 and 3), the values stay in VGPRs.
// Backward (the maps of the rows above): two ds_bpermute gathers, from the
// first lane of the next row (rows 0 and 2), then from lane 32 (rows 0, 1).
template <bool FWD, int NQ, typename C> __device__ inline void wave_incl(Aff<C> (&a)[NQ], int lane) {
    row16_incl<FWD, NQ>(a);
    if (FWD) {
        Aff<C> s[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) s[q] = dpp_aff<0x142, 0xA>(a[q]);  // row_bcast:15, rows 1 and 3
#pragma unroll
        for (int q = 0; q < NQ; ++q) a[q] = compose(a[q], s[q]);
#pragma unroll
        for (int q = 0; q < NQ; ++q) s[q] = dpp_aff<0x143, 0xC>(a[q]);  // row_bcast:31, rows 2 and 3
#pragma unroll
        for (int q = 0; q < NQ; ++q) a[q] = compose(a[q], s[q]);
    } else {
        const int row = lane >> 4;
        const int src1 = (row & 1) ? lane : (lane & ~15) + 16;
        const int src2 = row >= 2 ? lane : 32;
        Aff<C> s[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) s[q] = bperm_aff(a[q], src1);
#pragma unroll
        for (int q = 0; q < NQ; ++q) a[q] = compose(a[q], (row & 1) ? aff_id<C>() : s[q]);
#pragma unroll
        for (int q = 0; q < NQ; ++q) s[q] = bperm_aff(a[q], src2);
#pragma unroll
        for (int q = 0; q < NQ; ++q) a[q] = compose(a[q], row >= 2 ? aff_id<C>() : s[q]);
    }
}

// Shared memory of one cross-wave scan: for line q, the transfer-map totals
// of the waves at P[q * 32 + w] and E[q * 32 + 16 + w] (w < 16).  Each scan
// of a launch gets a region of its own, so no barrier is needed after it.
template <typename C> struct ScanShm {
    C* base;
    __device__ C& P(int q, int w) const { return base[q * 32 + w]; }
    __device__ C& E(int q, int w) const { return base[q * 32 + 16 + w]; }
};

// Exclusive scan over the G = 64 * nw threads of one row (thread t = 64 w +
// lane), NQ lines: out[q] is the composite of the maps before this thread
// (FWD) or after it (backward) applied to a zero carry.  Every thread of the
// block must call it (one barrier when nw > 1).
template <bool FWD, int NQ, typename C>
__device__ inline void row_scan(const C (&P)[NQ], const C (&E)[NQ], C (&out)[NQ], int lane, int w, int nw,
                                ScanShm<C> sh) {
    Aff<C> a[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) a[q] = Aff<C>{P[q], E[q]};
    wave_incl<FWD, NQ>(a, lane);
    C din[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) din[q] = zero_c<C>();
    if (nw > 1) {
        if (lane == (FWD ? 63 : 0)) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) { sh.P(q, w) = a[q].P; sh.E(q, w) = a[q].E; }
        }
        __syncthreads();
        if (FWD) {
            for (int v = 0; v < w; ++v)
#pragma unroll
                for (int q = 0; q < NQ; ++q) din[q] = cfma(din[q], sh.P(q, v), sh.E(q, v));
        } else {
            for (int v = nw - 1; v > w; --v)
#pragma unroll
                for (int q = 0; q < NQ; ++q) din[q] = cfma(din[q], sh.P(q, v), sh.E(q, v));
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const C val = cfma(din[q], a[q].P, a[q].E);  // inclusive map applied to the carry into the wave
        out[q] = FWD ? dpp_c<0x138>(din[q], val) : dpp_c<0x130>(din[q], val);  // wave_shr:1 / wave_shl:1
    }
}

// Exclusive scans across the 16 lanes of a DPP row (segments of one column in
// the y sweep), NQ lines: no shared memory, no barrier.
template <bool FWD, int NQ, typename C> __device__ inline void seg16_scan(const C (&P)[NQ], const C (&E)[NQ], C (&out)[NQ]) {
    Aff<C> a[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) a[q] = Aff<C>{P[q], E[q]};
    row16_incl<FWD, NQ>(a);
#pragma unroll
    for (int q = 0; q < NQ; ++q) out[q] = FWD ? dpp_c<0x111>(zero_c<C>(), a[q].E) : dpp_c<0x101>(zero_c<C>(), a[q].E);
}

// Single-map forms used by the long-row x sweep (one line at a time; the
// trailing barrier lets the next line reuse shP / shE).
// Inclusive scan of one map over the wave.  FWD: lane l holds
// f_l o f_{l-1} o ... o f_0; backward: f_l o f_{l+1} o ... o f_63.
template <bool FWD, typename C> __device__ inline Aff<C> wave_incl1(Aff<C> a, int lane) {
    Aff<C> b[1] = {a};
    wave_incl<FWD, 1>(b, lane);
    return b[0];
}

// Exclusive scan over the G = 64 * nw threads of one row (thread t = 64 w +
// lane): the value of the composite of the maps before this thread (FWD) or
// after it (backward), applied to a zero carry.  shP/shE: >= nw entries of
// shared memory private to the row.  Every thread of the block must call it.
template <bool FWD, typename C>
__device__ inline C row_scan1(C P, C E, int lane, int w, int nw, C* shP, C* shE) {
    const Aff<C> a = wave_incl1<FWD>(Aff<C>{P, E}, lane);
    C din = zero_c<C>();
    if (nw > 1) {
        if (lane == (FWD ? 63 : 0)) { shP[w] = a.P; shE[w] = a.E; }
        __syncthreads();
        if (FWD) {
            for (int v = 0; v < w; ++v) din = cfma(din, shP[v], shE[v]);
        } else {
            for (int v = nw - 1; v > w; --v) din = cfma(din, shP[v], shE[v]);
        }
        __syncthreads();
    }
    const C val = cfma(din, a.P, a.E);  // this thread's inclusive map applied to the carry into the wave
    return FWD ? dpp_c<0x138>(din, val) : dpp_c<0x130>(din, val);  // wave_shr:1 / wave_shl:1
}

}  // namespace gp
