// Launch interface between the host runtime and the gfx950 kernels.
#pragma once

#include "gp_device.hpp"

namespace gp {

constexpr int kObsCount = 13;

// Tile shapes of the windowed sweeps: KY points per lane, NW waves (4 lines
// each) per block; a window spans 16 * KY points (16 segments per line).
// Shapes 0..3 solve the three eigen-lines of a window interleaved (one scan
// for all three); shapes 4..7 are the same shapes solving them one after
// another (SEQ: about half the registers, so more waves per SIMD, at the price
// of a longer dependent chain per wave).
constexpr int kNumYTiles = 8;
struct YTile { int KY, NW; bool SEQ; };
template <typename T> __host__ __device__ constexpr YTile ytile(int t);
template <> __host__ __device__ constexpr YTile ytile<double>(int t) {
    return (t & 3) == 0 ? YTile{8, 2, t > 3} : (t & 3) == 1 ? YTile{8, 4, t > 3}
                        : (t & 3) == 2 ? YTile{4, 4, t > 3} : YTile{4, 8, t > 3};
}
template <> __host__ __device__ constexpr YTile ytile<float>(int t) {
    return (t & 3) == 0 ? YTile{8, 4, t > 3} : (t & 3) == 1 ? YTile{4, 8, t > 3}
                        : (t & 3) == 2 ? YTile{4, 4, t > 3} : YTile{8, 8, t > 3};
}
__host__ __device__ constexpr int ywindow(YTile t) { return 16 * t.KY; }

// Tile shapes of the chain windows: K points per lane, NW waves per block,
// SEQ as for the scanned windows.  x windows: one row per wave (64 K
// points); y windows: four columns per wave, 16 segments each (16 K rows).
constexpr int kNumChainTiles = 8;
struct ChainTile { int K, NW; bool SEQ; };
template <typename T> __host__ __device__ constexpr ChainTile xchain_tile(int t);
template <> __host__ __device__ constexpr ChainTile xchain_tile<double>(int t) {
    return (t & 3) == 0 ? ChainTile{4, 4, t > 3} : (t & 3) == 1 ? ChainTile{8, 2, t > 3}
                        : (t & 3) == 2 ? ChainTile{2, 4, t > 3} : ChainTile{4, 2, t > 3};
}
template <> __host__ __device__ constexpr ChainTile xchain_tile<float>(int t) {
    return (t & 3) == 0 ? ChainTile{4, 4, t > 3} : (t & 3) == 1 ? ChainTile{8, 4, t > 3}
                        : (t & 3) == 2 ? ChainTile{8, 2, t > 3} : ChainTile{16, 2, t > 3};
}
template <typename T> __host__ __device__ constexpr ChainTile ychain_tile(int t);
template <> __host__ __device__ constexpr ChainTile ychain_tile<double>(int t) {
    return (t & 3) == 0 ? ChainTile{8, 2, t > 3} : (t & 3) == 1 ? ChainTile{8, 4, t > 3}
                        : (t & 3) == 2 ? ChainTile{4, 4, t > 3} : ChainTile{7, 4, t > 3};
}
template <> __host__ __device__ constexpr ChainTile ychain_tile<float>(int t) {
    return (t & 3) == 0 ? ChainTile{8, 4, t > 3} : (t & 3) == 1 ? ChainTile{8, 8, t > 3}
                        : (t & 3) == 2 ? ChainTile{4, 4, t > 3} : ChainTile{16, 2, t > 3};
}

// Carry lanes of a chain window for a halo of h points: nc = ceil((h - 1) / K),
// at least 1.  A carry from a lane farther away crosses nc whole lanes and at
// least one point of the receiving lane, nc K + 1 >= h points.
__host__ __device__ inline int chain_lanes(int h, int K) { return h <= K + 1 ? 1 : (h - 1 + K - 1) / K; }

// Stacked y windows (k_y_stack): 16 consecutive columns per block, one per
// lane of a DPP row, and the 4 NW segments of a window spread over the NW
// waves (4 per wave); carries pass through shared memory.  Tiles: K rows per
// segment, NW waves, SEQ as above; tiles 0-3 have 16 segments (windows of
// 16 K rows), tiles 4-5 32 segments (twice the rows per halo, one line at a
// time to keep the shared memory small).
constexpr int kNumStackTiles = 6;
template <typename T> __host__ __device__ constexpr ChainTile ystack_tile(int t);
template <> __host__ __device__ constexpr ChainTile ystack_tile<double>(int t) {
    return t >= 4 ? ChainTile{t == 4 ? 8 : 6, 8, true} : (t & 1) == 0 ? ChainTile{8, 4, t > 1} : ChainTile{6, 4, t > 1};
}
template <> __host__ __device__ constexpr ChainTile ystack_tile<float>(int t) {
    return t >= 4 ? ChainTile{t == 4 ? 8 : 16, 8, true} : (t & 1) == 0 ? ChainTile{8, 4, t > 1} : ChainTile{16, 4, t > 1};
}

// x sweep: K consecutive points per thread; the launch bound of each K.
constexpr int kNumXK = 5;
__host__ __device__ constexpr int xk_value(int idx) { return 1 << idx; }  // 1, 2, 4, 8, 16
__host__ __device__ constexpr int xk_bound(int K) { return K == 1 ? 1024 : 512; }

// Workgroups are dispatched to the 8 XCDs of the chip in turn (block b to XCD
// b mod 8), each with its own L2.  Block orders of the windowed sweeps (the
// window of logical block lb covers strip lb mod ncs of row tile lb / ncs):
//   0  hardware order: block b computes window b;
//   1  XCD-contiguous: XCD x takes the run of windows x ceil(n/8) .. , so
//      neighbouring windows along a strip, whose halos overlap, share an L2;
//   2  bands (y sweep): XCD x takes a contiguous range of strips and walks
//      them down kBand strips at a time, row tile by row tile, so that the
//      windows above and below each other are in flight together (the halo
//      rows are read through one L2) while the rows read stay contiguous;
//   3  row bands (both sweeps, small grids): XCD x owns the y row tiles
//      [x nrt / 8, (x + 1) nrt / 8) - all their windows, and in the x sweep
//      the rows they write.  The L2 keeps data across kernel boundaries, so
//      each sweep then reads what the previous one wrote on the same XCD
//      (measured: a 512^2 FP64 pass in 4 us instead of 9.5 us when the rows
//      come from another XCD), as long as a band of both wave functions fits
//      the 4 MB L2.
// Orders 1 to 3 launch more blocks than windows; the extra blocks exit at
// once (xcd_grid blocks in all, order_logical < 0).
constexpr int kNumXcd = 8;
constexpr int kBand = 8;
__host__ __device__ inline int xcd_blocks(int n) { return (n + kNumXcd - 1) / kNumXcd * kNumXcd; }
__host__ __device__ inline int xcd_grid(int order, int ncs, int nrt) {
    return order == 0 ? ncs * nrt
         : order == 1 ? xcd_blocks(ncs * nrt)
         : order == 2 ? kNumXcd * ((ncs + kNumXcd - 1) / kNumXcd) * nrt
                      : kNumXcd * ((nrt + kNumXcd - 1) / kNumXcd) * ncs;
}
// Rows [r0, r1) of XCD x under the row-band order (row tiles of L rows).
__host__ __device__ inline void band_rows(int x, int nrt, int L, int ny, int& r0, int& r1) {
    const int a = x * nrt / kNumXcd * L, b = (x + 1) * nrt / kNumXcd * L;
    r0 = a < ny ? a : ny;
    r1 = b < ny ? b : ny;
}
__device__ inline int order_logical(int order, int b, int ncs, int nrt) {
    const int n = ncs * nrt;
    if (order == 0) return b;
    const int x = b % kNumXcd, j = b / kNumXcd;
    if (order == 3) {
        const int t0 = x * nrt / kNumXcd, t1 = (x + 1) * nrt / kNumXcd;
        if (j >= (t1 - t0) * ncs) return -1;
        return (t0 + j / ncs) * ncs + j % ncs;
    }
    if (order == 1) {
        const int lb = x * ((n + kNumXcd - 1) / kNumXcd) + j;
        return lb < n ? lb : -1;
    }
    const int s0 = x * ncs / kNumXcd, sx = (x + 1) * ncs / kNumXcd - s0;  // this XCD's strips
    if (j >= sx * nrt) return -1;
    const int band = j / (kBand * nrt);
    const int gb = sx - band * kBand < kBand ? sx - band * kBand : kBand;  // strips in this band
    const int r = j - band * kBand * nrt;
    return (r / gb) * ncs + s0 + band * kBand + r % gb;
}

// Both sweeps run out of place (src -> dst): the y windows overlap, so a
// window's halo rows must not be rewritten by its neighbour while it reads.
// Where the y sweep leaves the imaginary-time norm: three partial sums per
// block, one per component (partials[3 blk + m]); launch_norm_finalize turns
// them into the three scale factors of the next step and the non-finite flag.
struct NormOut {
    double* partials;
};

// How the norm totals become scale factors: the total norm to one, or (fixed
// magnetisation) the component norms to total one and N_{+1} - N_{-1} = mag.
struct NormRule {
    int fix_m;
    double mag;
};

// The previous y sweep's norm partials, when the x sweep forms the scale
// factors itself (every block sums them in the same order); partials ==
// nullptr: the factors are read from `scale`.
struct NormIn {
    const double* partials;
    int n;
    double dxdy;
    NormRule rule;
    int* flag;
};

template <typename T> struct XLaunch {
    const cx<T>* src;
    cx<T>* dst;
    Phys ph;
    LineSet<T> ls;
    const double* scale;
    NormIn nin;
    int K, G, R;
    bool imag, local;
    bool window;    // truncated windows along the rows (tile shapes as the y sweep's) instead of whole rows
    bool chain = false;  // chain windows (gp_chain.hpp): one row segment of 64 K points per wave
    int L, h, tile;
    int order;      // block order: windows 0 hardware, 1 XCD-contiguous (2, 3 taken as 1); rows 0 or 3
    int bL, bnrt;   // order 3 on rows: the y sweep's row tile (rows) and number of row tiles
    size_t sp, dp;  // plane strides (elements between the component planes) of src and dst
};

template <typename T> struct YLaunch {
    const cx<T>* src;
    cx<T>* dst;
    Phys ph;
    LineSet<T> ls;
    NormOut no;
    int L, h, tile;
    bool window, imag, norm;
    bool chain = false;  // chain windows (gp_chain.hpp) instead of the scanned windows
    bool stack = false;  // stacked chain windows (k_y_stack; tile indexes ystack_tile)
    bool outl;  // second half local substep on the way out (Strang)
    int order;  // windows: block order (0 hardware, 1 XCD-contiguous, 2 bands, 3 row bands)
    size_t sp, dp;  // plane strides of src and dst
};

// Batched launches: one descriptor per condensate and one map entry per block,
// (condensate << kMapShift) | (block index within that condensate).
constexpr unsigned kMapShift = 20;
constexpr unsigned kMapMask = (1u << kMapShift) - 1;
constexpr int kMaxBatchSlots = 1 << (32 - kMapShift);
constexpr int kScaleChunk = 4096;  // values per block of the batched scale kernel

template <typename T> struct XSlot {
    const cx<T>* src;
    cx<T>* dst;
    Phys ph;
    LineSet<T> ls;
    const double* scale;
    int G, R;
    size_t sp, dp;
};

template <typename T> struct YSlot {
    const cx<T>* src;
    cx<T>* dst;
    Phys ph;
    LineSet<T> ls;
    double* partials;
    int L, h, ncs;
    size_t sp, dp;
};

// Batched chain windows (x) and stacked chain windows (y): per condensate,
// the windows of its own plan (halo h, carry lanes nc, points written L).
template <typename T> struct XCSlot {
    const cx<T>* src;
    cx<T>* dst;
    Phys ph;
    LineSet<T> ls;
    const double* scale;
    int h, nc, L, nwin;  // nwin windows per row
    size_t sp, dp;
};

template <typename T> struct YSSlot {
    const cx<T>* src;
    cx<T>* dst;
    Phys ph;
    LineSet<T> ls;
    double* partials;
    int L, h, nc, ncs;  // ncs strips of 16 columns
    size_t sp, dp;
};

struct NSlot {
    const double* partials;
    int n;
    double dxdy;
    double* scale;
    int* flag;
    NormRule rule;
};

template <typename T> struct SSlot {
    cx<T>* psi;
    size_t n;       // points per component plane
    size_t stride;  // elements between the planes
    const double* scale;
};

struct ObsLaunch {
    double c0, c2, rabi, gamma, omega;
    int eta;
};

// The sweep, scale and norm launchers take an optional event pair that the
// dispatch itself stamps at kernel start and end (per-kernel timing).
template <typename T>
hipError_t launch_x(const XLaunch<T>& a, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
template <typename T>
hipError_t launch_y(const YLaunch<T>& a, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
template <typename T> int y_blocks(const YLaunch<T>& a);
// The single-condensate kernels below address component m of point idx at
// psi[m sp + idx] (sp: the plane stride, at least nx ny).
template <typename T> hipError_t launch_local(cx<T>* psi, size_t sp, const Phys& ph, bool imag, hipStream_t st);
// psi[m][0 .. n) *= scale[m] (three factors, one per component)
template <typename T>
hipError_t launch_scale(cx<T>* psi, size_t n, size_t sp, const double* scale, hipStream_t st, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
template <typename T>
hipError_t launch_norm_partials(const cx<T>* psi, size_t n, size_t sp, double* partials, int nblk, hipStream_t st);
hipError_t launch_set_scale(double* scale, double v, hipStream_t st);
hipError_t launch_set_flag(int* flag, int v, hipStream_t st);  // a one-thread store (no memset node)
// n blocks' worth of partials (3 n values) -> scale[3], flag
hipError_t launch_norm_finalize(const double* partials, int n, double dxdy, NormRule rule, double* scale, int* flag,
                                hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
template <typename T>
hipError_t launch_obs(const cx<T>* psi, size_t sp, const Phys& ph, const ObsLaunch& o, T* dens, double* partials,
                      int nblk, hipStream_t st);
hipError_t launch_obs_finalize(const double* partials, int nblk, double* out, hipStream_t st);

// Batched forms: the x sweep (local substep fused; imaginary time also applies
// each condensate's pending scale) and the windowed y sweep (imaginary time
// stores norm partials) over the map's blocks, as whole-row scans and scanned
// windows or as chain x windows and stacked chain y windows (tile: the chain
// and stacked tile indices); per-condensate norm totals, scale resets and
// final scaling.
template <typename T>
hipError_t launch_x_batch(const XSlot<T>* slots, const unsigned* map, int nblk, int K, int block, bool imag,
                          hipStream_t st);
template <typename T>
hipError_t launch_y_batch(const YSlot<T>* slots, const unsigned* map, int nblk, int tile, bool imag, hipStream_t st);
template <typename T>
hipError_t launch_xc_batch(const XCSlot<T>* slots, const unsigned* map, int nblk, int tile, bool imag, hipStream_t st);
template <typename T>
hipError_t launch_ys_batch(const YSSlot<T>* slots, const unsigned* map, int nblk, int tile, bool imag, hipStream_t st);
hipError_t launch_set_scale_batch(const NSlot* slots, int n, double v, hipStream_t st);
hipError_t launch_norm_finalize_batch(const NSlot* slots, int n, hipStream_t st);
template <typename T>
hipError_t launch_scale_batch(const SSlot<T>* slots, const unsigned* map, int nblk, hipStream_t st);

}  // namespace gp
