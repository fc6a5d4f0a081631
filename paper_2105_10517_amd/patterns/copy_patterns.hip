// Copy kernels with the access patterns of the SSCN sweeps, on the 4096^2
// FP64 state (three planes of complex double, planes 4096^2 + 4160 elements
// apart as in the library's work buffer).  Each kernel copies src to dst and
// does nothing else: the bandwidth it reaches bounds what a sweep with that
// pattern can move.  A measurement program, not part of the library:
//
//   hipcc --offload-arch=gfx950 -O3 -std=c++17 -Xclang -target-feature -Xclang -packed-fp32-ops \
//       paper_2105_10517_amd/patterns/copy_patterns.hip -o /tmp/copy_patterns && /tmp/copy_patterns
//
// Patterns:
//   plain       coalesced, one element per thread per plane
//   x blocked K one row segment of 64 K points per wave, K consecutive points
//               per lane (the chain and window x sweeps)
//   x lds K     the same segment loaded coalesced (lane l: points l + 64 k),
//               every load issued first, transposed through shared memory to
//               the blocked layout and back, stored coalesced
//   x swz K4    the same, through a shared-memory region per wave (no block
//               barrier), slots rotated within 16-element chunks so that the
//               blocked reads and writes are free of bank conflicts; "in" stores
//               the blocked layout directly, "in+out" transposes back first
//   x pf K4     the blocked pattern from a fixed grid of waves, each looping
//               over segments and loading the next before storing the current
//   y 4-col K   4 columns per wave, 16 segments of K rows per column (one DPP
//               row of lanes each): the scanned and chain y windows
//   y stack K   16 consecutive columns per block, one per lane of a DPP row,
//               16 segments of K rows spread over 4 waves: the stacked y windows
#include <hip/hip_runtime.h>
#include <cstdio>

#define CK(x)                                                                                      \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) {                                                                    \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);             \
            return 1;                                                                              \
        }                                                                                          \
    } while (0)

typedef double2 C;
constexpr int NX = 4096, NY = 4096;
constexpr size_t PL = (size_t)NX * NY + 4160;

__global__ __launch_bounds__(256) void k_plain(const C* __restrict__ s, C* __restrict__ d) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;  // grid covers NX NY exactly
#pragma unroll
    for (int m = 0; m < 3; ++m) d[m * PL + i] = s[m * PL + i];
}

template <int K, int NW>
__global__ __launch_bounds__(64 * NW) void k_xblocked(const C* __restrict__ s, C* __restrict__ d) {
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * NW + (threadIdx.x >> 6);  // grid covers the segments exactly
    constexpr int nseg = NX / (64 * K);
    const size_t base = (size_t)(gw / nseg) * NX + (gw % nseg) * 64 * K + lane * K;
    C v[3][K];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m][k] = s[m * PL + base + k];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) d[m * PL + base + k] = v[m][k];
}

template <int K, int NW>
__global__ __launch_bounds__(64 * NW) void k_xlds(const C* __restrict__ s, C* __restrict__ d) {
    constexpr int W = 64 * K, WP = W + W / 4;  // one pad element per 4
    __shared__ C sh[NW][3][WP];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gw = blockIdx.x * NW + w;
    constexpr int nseg = NX / W;
    const size_t base = (size_t)(gw / nseg) * NX + (gw % nseg) * W;
    auto pad = [](int i) { return i + i / 4; };
    C t[3][K];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) t[m][k] = s[m * PL + base + lane + 64 * k];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int k = 0; k < K; ++k) sh[w][m][pad(lane + 64 * k)] = t[m][k];
    __syncthreads();
    C v[3][K];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int k = 0; k < K; ++k) v[m][k] = sh[w][m][pad(lane * K + k)];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int k = 0; k < K; ++k) sh[w][m][pad(lane * K + k)] = v[m][k];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int k = 0; k < K; ++k) t[m][k] = sh[w][m][pad(lane + 64 * k)];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) d[m * PL + base + lane + 64 * k] = t[m][k];
}

// Shared-memory slot of point p of a 256-point segment: a rotation within each
// chunk of 16 by the chunk index.  Lanes l and l + 16 j of a blocked access
// (points 4 l + k) then fall on different 16-byte bank groups.
__device__ inline int swz(int p) { return (p & ~15) | ((p + (p >> 4)) & 15); }
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NW, bool OUT>
__global__ __launch_bounds__(64 * NW) void k_xswz(const C* __restrict__ s, C* __restrict__ d) {
    __shared__ C sh[NW][3][256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gw = blockIdx.x * NW + w;  // grid covers the segments exactly
    constexpr int nseg = NX / 256;
    const size_t base = (size_t)(gw / nseg) * NX + (gw % nseg) * 256;
    C t[3][4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) t[m][k] = s[m * PL + base + 64 * k + lane];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) sh[w][m][swz(64 * k + lane)] = t[m][k];
    wave_sync();
    C v[3][4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m][k] = sh[w][m][swz(4 * lane + k)];
    if (!OUT) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int m = 0; m < 3; ++m) d[m * PL + base + 4 * lane + k] = v[m][k];
        return;
    }
    wave_sync();
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) sh[w][m][swz(4 * lane + k)] = v[m][k];
    wave_sync();
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) d[m * PL + base + 64 * k + lane] = sh[w][m][swz(64 * k + lane)];
}

// Blocked K = 4 from nw resident waves: wave w copies segments w, w + nw, ...,
// the next segment's loads issued before the current segment's stores.
__device__ inline size_t xpf_base(int gw, int lane) {
    constexpr int nseg = NX / 256;
    return (size_t)(gw / nseg) * NX + (gw % nseg) * 256 + lane * 4;
}
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_xpf(const C* __restrict__ s, C* __restrict__ d, int nw) {
    constexpr int total = NY * (NX / 256);
    const int lane = threadIdx.x & 63;
    int gw = blockIdx.x * NW + (threadIdx.x >> 6);
    if (gw >= total) return;
    C a[3][4], b[3][4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) a[m][k] = s[m * PL + xpf_base(gw, lane) + k];
    for (;;) {
        const int g1 = gw + nw;
        if (g1 < total) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int m = 0; m < 3; ++m) b[m][k] = s[m * PL + xpf_base(g1, lane) + k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int m = 0; m < 3; ++m) d[m * PL + xpf_base(gw, lane) + k] = a[m][k];
        if (g1 >= total) return;
        const int g2 = g1 + nw;
        if (g2 < total) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int m = 0; m < 3; ++m) a[m][k] = s[m * PL + xpf_base(g2, lane) + k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int m = 0; m < 3; ++m) d[m * PL + xpf_base(g1, lane) + k] = b[m][k];
        if (g2 >= total) return;
        gw = g2;
    }
}

template <int K, int NW>
__global__ __launch_bounds__(64 * NW) void k_y4col(const C* __restrict__ s, C* __restrict__ d) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    constexpr int ncs = NX / (4 * NW);
    const int rt = blockIdx.x / ncs, cs = blockIdx.x % ncs;  // grid covers the tiles exactly
    const int i = cs * 4 * NW + w * 4 + (lane >> 4);
    const int g0 = rt * 16 * K + (lane & 15) * K;
    C v[3][K];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m][k] = s[m * PL + (size_t)(g0 + k) * NX + i];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) d[m * PL + (size_t)(g0 + k) * NX + i] = v[m][k];
}

template <int K>
__global__ __launch_bounds__(256) void k_ystack(const C* __restrict__ s, C* __restrict__ d) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    constexpr int ncs = NX / 16;
    const int rt = blockIdx.x / ncs, cs = blockIdx.x % ncs;
    const int i = cs * 16 + (lane & 15);
    const int g0 = rt * 16 * K + (w * 4 + (lane >> 4)) * K;
    C v[3][K];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m][k] = s[m * PL + (size_t)(g0 + k) * NX + i];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) d[m * PL + (size_t)(g0 + k) * NX + i] = v[m][k];
}

// The stacked pattern with the windows of the 4096^2 FP64 y sweep: windows
// of 16 K rows starting at rt L - h, every row read, the middle L rows
// written (the halo rows are read twice, by neighbouring windows).
template <int K>
__global__ __launch_bounds__(256) void k_ystack_halo(const C* __restrict__ s, C* __restrict__ d, int h, int L) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    constexpr int ncs = NX / 16;
    const int rt = blockIdx.x / ncs, cs = blockIdx.x % ncs;
    const int i = cs * 16 + (lane & 15);
    const int j0 = rt * L, g0 = j0 - h + (w * 4 + (lane >> 4)) * K;
    C v[3][K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int g = g0 + k;
        const bool ok = g >= 0 && g < NY;
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m][k] = ok ? s[m * PL + (size_t)(ok ? g : 0) * NX + i] : C{0, 0};
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int g = g0 + k;
        if (g >= j0 && g < j0 + L && g < NY)
#pragma unroll
            for (int m = 0; m < 3; ++m) d[m * PL + (size_t)g * NX + i] = v[m][k];
    }
}

template <typename F>
float timeit(F f, int reps = 20) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    for (int i = 0; i < 3; ++i) f();
    (void)hipEventRecord(a);
    for (int i = 0; i < reps; ++i) f();
    (void)hipEventRecord(b);
    (void)hipEventSynchronize(b);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
}

int main() {
    C *s = nullptr, *d = nullptr;
    const size_t bytes = 3 * PL * sizeof(C);
    CK(hipMalloc(&s, bytes));
    CK(hipMalloc(&d, bytes));
    CK(hipMemset(s, 0, bytes));
    CK(hipMemset(d, 0, bytes));
    const double moved = 2.0 * 3 * (double)NX * NY * sizeof(C);
    auto rep = [&](const char* name, float ms) {
        std::printf("%-22s %8.1f us  %5.2f TB/s\n", name, ms * 1e3, moved / (ms * 1e-3) / 1e12);
        std::fflush(stdout);
    };
    const int npts = NX * NY;
    rep("hipMemcpy", timeit([&] { (void)hipMemcpyAsync(d, s, bytes, hipMemcpyDeviceToDevice, 0); }));
    rep("plain", timeit([&] { k_plain<<<npts / 256, 256>>>(s, d); }));
    rep("x blocked K2", timeit([&] { k_xblocked<2, 4><<<npts / 128 / 4, 256>>>(s, d); }));
    rep("x blocked K4", timeit([&] { k_xblocked<4, 2><<<npts / 256 / 2, 128>>>(s, d); }));
    rep("x blocked K8", timeit([&] { k_xblocked<8, 2><<<npts / 512 / 2, 128>>>(s, d); }));
    rep("x lds K4", timeit([&] { k_xlds<4, 2><<<npts / 256 / 2, 128>>>(s, d); }));
    rep("x lds K8", timeit([&] { k_xlds<8, 1><<<npts / 512, 64>>>(s, d); }));
    rep("x swz K4 in NW4", timeit([&] { k_xswz<4, false><<<npts / 256 / 4, 256>>>(s, d); }));
    rep("x swz K4 in+out NW4", timeit([&] { k_xswz<4, true><<<npts / 256 / 4, 256>>>(s, d); }));
    for (int wps : {2, 3, 4}) {
        const int nw = 256 * 4 * wps;  // resident waves: wps per SIMD
        char name[40];
        std::snprintf(name, sizeof name, "x pf K4 %d waves/SIMD", wps);
        rep(name, timeit([&] { k_xpf<2><<<nw / 2, 128>>>(s, d, nw); }));
    }
    rep("y 4-col K8 NW2", timeit([&] { k_y4col<8, 2><<<(NX / 8) * (NY / 128), 128>>>(s, d); }));
    rep("y 4-col K8 NW4", timeit([&] { k_y4col<8, 4><<<(NX / 16) * (NY / 128), 256>>>(s, d); }));
    rep("y stack K8", timeit([&] { k_ystack<8><<<(NX / 16) * (NY / 128), 256>>>(s, d); }));
    // h = 13, L = 102: the FP64 windows (41 row tiles)
    rep("y stack K8 halo 13", timeit([&] { k_ystack_halo<8><<<(NX / 16) * ((NY + 101) / 102), 256>>>(s, d, 13, 102); }));
    CK(hipGetLastError());
    CK(hipDeviceSynchronize());
    CK(hipFree(s));
    CK(hipFree(d));
    std::printf("done\n");
    return 0;
}
