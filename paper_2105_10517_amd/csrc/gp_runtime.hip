// Host runtime behind the C ABI of include/gp_spin1.h: parameter validation,
// Thomas pivot tables per line, stability checks, the launch plan and the
// step sequencing on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <thread>
#include <exception>
#include <vector>

#include "gp_kernels.hpp"
#include "gp_spin1.h"

using zd = std::complex<double>;
// |z|^2 from the parts (the library's std::norm goes through |z|, a hypot)
inline double nrm(zd z) { return z.real() * z.real() + z.imag() * z.imag(); }

namespace {

struct DirTable {
    int K = 0, lines = 0;
    zd b{1.0, 0.0};
    zd bm1{0.0, 0.0};
    double decay = 0.0;
    bool dominant = true;
    void* d_piv = nullptr;
    void* d_ae = nullptr;
    int Kg = 0;
    void* d_g = nullptr;   // line-start correction vectors [lines][Kg]
    void* d_gc = nullptr;  // and coefficients [lines]
};

struct ModeState {
    DirTable x, y;
    bool stable = false;
    std::string why;
    bool window = false;
    int hh = 0;        // halo the truncation bound asks for
    int h = 0, L = 0;  // halo and rows written per window for the chosen tile
    int xK = 2, xG = 64, xR = 1;  // x sweep: points per thread, threads per row, rows per block
    int ytile = 0;                // windowed y sweep tile shape (0-based)
    bool xwindow = false;         // x sweep over truncated windows
    int hhx = 0, hx = 0, Lx = 0, xtile = 0;
    int xorder = 1, yorder = 0;   // block orders (x windows 0/1, x rows 0/3; y windows 0..3), see gp_kernels.hpp
    bool xchain = false, ychain = false;  // chain windows (gp_chain.hpp) for the x / y sweep
    bool ystack = false;                  // y chain windows stacked over the waves (yctile indexes ystack_tile)
    int xctile = 0, hcx = 0, Lcx = 0;     // x chain tile, halo points, points written per window
    int yctile = 0, hcy = 0, Lcy = 0;     // y chain tile, halo rows, rows written per window
    gp_spin1_plan plan{};
};

}  // namespace

struct gp_spin1 {
    gp_spin1_params p{};
    hipStream_t stream = nullptr;
    int device = 0;
    ModeState mode[2];  // [0] real time, [1] imaginary time
    double* d_scale = nullptr;
    int* d_flag = nullptr;
    double* d_part = nullptr;
    size_t n_part = 0;
    double* d_obs = nullptr;
    int obs_blocks = 0;
    void* d_work = nullptr;  // a second wave function: the x sweep writes it, the y sweep reads it
    size_t psp = 0, wsp = 0;  // plane strides (elements) of the caller's wave functions and of d_work
    // optional per-kernel timing: pairs of events around launches of kind k
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_open;
    size_t ev_next = 0;
    int64_t t_launches[4] = {0, 0, 0, 0};
    double t_ms[4] = {0, 0, 0, 0};
    // step sequences captured as HIP graphs (gp_spin1_step_graph), newest last
    struct Graph {
        void* psi;
        int64_t n;
        bool imag;
        hipGraph_t g;
        hipGraphExec_t x;
    };
    std::vector<Graph> graphs;
    hipStream_t cap_stream = nullptr;  // the stream the captures are recorded on
    std::string err;
};

namespace {

constexpr double kNu[3] = {1.0, 0.0, -1.0};  // eigenvalue order of the basis changes (+1, 0, -1)
constexpr int kNumCu = 256;                    // compute units of the chip (one wave of blocks)
// Padding of the work buffer's component planes.  With planes exactly a
// power of two apart (every 2^k x 2^k grid), the three streams a sweep reads
// and the three it writes fall on the same HBM channels at the same time; a
// pad of 4160 elements (65 KiB in FP64, a multiple of 256 B) spreads them.
constexpr size_t kPlanePad = 4160;
size_t work_stride(const gp_spin1_params& p) { return (size_t)p.nx * p.ny + kPlanePad; }
size_t psi_stride(const gp_spin1_params& p) { return p.plane_stride > 0 ? (size_t)p.plane_stride : (size_t)p.nx * p.ny; }

int fail(gp_spin1* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

int hip_fail(gp_spin1* h, hipError_t e, const char* where) {
    return fail(h, GP_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Tridiagonal coefficients of (I + alpha h1) for h1 = -1/2 d^2 + c d on step s:
// sub a = alpha (-1/(2 s^2) - c/(2 s)), diag b = 1 + alpha/s^2, super e = alpha (-1/(2 s^2) + c/(2 s)).
void coeffs(zd alpha, double s, zd c, zd& a, zd& b, zd& e) {
    a = alpha * (-0.5 / (s * s) - c / (2.0 * s));
    b = 1.0 + alpha / (s * s);
    e = alpha * (-0.5 / (s * s) + c / (2.0 * s));
}

// Converged pivot: the root of w^2 - b w + a e = 0 of larger modulus (the
// attracting fixed point of w -> b - a e / w).
zd pivot_limit(zd a, zd b, zd e) {
    const zd d = std::sqrt(b * b - 4.0 * a * e);
    const zd w1 = 0.5 * (b + d), w2 = 0.5 * (b - d);
    return std::abs(w1) >= std::abs(w2) ? w1 : w2;
}

template <typename T>
gp::cx<T> to_dev(zd z) {
    return gp::mk<T>((T)z.real(), (T)z.imag());
}

// Pivot table of one direction, computed on the host in FP64: lines =
// nother * 3 (line index = other * 3 + eigenvalue index), line length n.
struct HostDir {
    int K = 1, lines = 0;
    zd b{1.0, 0.0};    // 1 + bm1, the diagonal whose pivots the table holds
    zd bm1{0.0, 0.0};  // b - 1 as the kernels see it (rounded to T)
    double decay = 0.0;
    bool dominant = true;
    std::vector<zd> A, E, W;
    int Kg = 1;            // points of the line-start correction
    std::vector<zd> G, GC; // [lines][Kg] and [lines]
};

// Round a complex coefficient to the storage precision T and back.
template <typename T>
zd round_to(zd z) {
    return zd((double)(T)z.real(), (double)(T)z.imag());
}

template <typename T, typename F>
void host_dir(HostDir& d, int n, int nother, zd alpha, double step, F coef) {
    const int lines = nother * 3;
    d.lines = lines;
    d.A.assign(lines, zd());
    d.E.assign(lines, zd());
    d.W.assign(lines, zd());
    // the finite-precision recurrence settles a few ulp from the exact fixed point
    const double tol = 32.0 * 1.1102230246251565e-16;
    int K = 1;
    d.dominant = true;
    d.decay = 0.0;
    for (int l = 0; l < lines; ++l) {
        zd a, e, b;
        coeffs(alpha, step, coef(l), a, b, e);
        // the kernels see a, e and b - 1 in precision T; the pivots are those of
        // the matrix with exactly these rounded entries
        a = round_to<T>(a); e = round_to<T>(e);
        d.bm1 = round_to<T>(alpha / (step * step));
        d.b = 1.0 + d.bm1;
        d.A[l] = a; d.E[l] = e;
        if (std::abs(d.b) < (std::abs(a) + std::abs(e)) * (1.0 - 1e-12)) d.dominant = false;
        const zd wl = pivot_limit(a, d.b, e);
        d.W[l] = wl;
        zd w = d.b;
        int k = 0;
        const double wl2 = tol * tol * nrm(wl);  // (squared moduli: no square roots in the loops)
        while (k < n - 1 && nrm(w - wl) > wl2) {
            w = d.b - a * e / w;
            ++k;
        }
        if (k + 1 > K) K = k + 1;
        d.decay = std::max(d.decay, std::max(std::abs(a / wl), std::abs(e / wl)));
    }
    d.K = std::min(K, n);
    // Line-start correction: g = A_inf^{-1} e0 on the n points of a line
    // (Thomas with the limit pivots throughout), kept while |g_k| is above
    // the rounding level of T relative to |g_0| (the same bound as the halo)
    const double tolg = sizeof(T) == 8 ? std::ldexp(1.0, -60) : std::ldexp(1.0, -32);
    // (every line's g in one buffer: no allocation per line)
    std::vector<zd> y, gall;
    std::vector<size_t> goff(lines + 1, 0);
    int Kg = 1;
    for (int l = 0; l < lines; ++l) {
        const zd w = d.W[l], m = 1.0 / w, am = d.A[l] * m, cp = d.E[l] * m;
        // y = L^{-1} e0 decays geometrically; past the point where it is far
        // below the rounding level it is taken as zero (exact for short lines)
        y.assign(1, m);
        const double ycut = 1e-54 * nrm(m);
        while ((int)y.size() < n && nrm(y.back()) > ycut) y.push_back(-am * y.back());
        const int M = (int)y.size();
        const size_t off = gall.size();
        gall.resize(off + M);
        zd* g = gall.data() + off;
        g[M - 1] = y[M - 1];
        for (int k = M - 2; k >= 0; --k) g[k] = y[k] - cp * g[k + 1];
        int kg = M;
        const double gcut = tolg * tolg * nrm(g[0]);
        while (kg > 1 && nrm(g[kg - 1]) < gcut) --kg;
        Kg = std::max(Kg, kg);
        goff[l + 1] = off + M;
    }
    d.Kg = Kg;
    d.G.assign((size_t)lines * Kg, zd());
    d.GC.assign(lines, zd());
    for (int l = 0; l < lines; ++l) {
        const zd* g = gall.data() + goff[l];
        const int M = (int)(goff[l + 1] - goff[l]);
        for (int k = 0; k < Kg && k < M; ++k) d.G[(size_t)l * Kg + k] = g[k];
        const zd bw = d.b - d.W[l];
        d.GC[l] = bw / (1.0 + bw * g[0]);
    }
}

template <typename T>
void set_piv(gp::Piv<T>& pv, zd a, zd e, zd w) {
    const zd m = 1.0 / w;
    pv.m = to_dev<T>(m);
    pv.am = to_dev<T>(a * m);
    pv.cp = to_dev<T>(e * m);
}

// Device memory for the line tables: hipMalloc, or (the entry point that
// allocates nothing) a bump allocator over the library's static scratch array.
// Arena copies go through the stream (ordered after earlier work on it).
struct Arena {
    unsigned char* base = nullptr;  // nullptr: allocate with hipMalloc
    size_t cap = 0, used = 0;
    hipStream_t stream = nullptr;
};

hipError_t dev_alloc(Arena* a, void** p, size_t bytes) {
    if (!a || !a->base) return hipMalloc(p, bytes);
    const size_t off = (a->used + 255) / 256 * 256;
    if (off > a->cap || bytes > a->cap - off) return hipErrorOutOfMemory;
    *p = a->base + off;
    a->used = off + bytes;
    return hipSuccess;
}

hipError_t dev_upload(Arena* a, void* dst, const void* src, size_t bytes) {
    if (!a || !a->base) return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, a->stream);
}

template <typename T>
int upload_dir(gp_spin1* h, const HostDir& hd, DirTable& d, Arena* arena = nullptr) {
    const int lines = hd.lines, K = hd.K;
    d.lines = lines; d.K = K; d.b = hd.b; d.bm1 = hd.bm1; d.decay = hd.decay; d.dominant = hd.dominant;
    std::vector<gp::Piv<T>> piv((size_t)lines * (K + 1));
    std::vector<gp::cx<T>> ae((size_t)lines * 2);
    for (int l = 0; l < lines; ++l) {
        zd w = hd.b;
        for (int k = 0; k < K; ++k) {
            if (k > 0) w = hd.b - hd.A[l] * hd.E[l] / w;
            set_piv<T>(piv[(size_t)l * (K + 1) + k], hd.A[l], hd.E[l], w);
        }
        set_piv<T>(piv[(size_t)l * (K + 1) + K], hd.A[l], hd.E[l], hd.W[l]);
        ae[2 * (size_t)l] = to_dev<T>(hd.A[l]);
        ae[2 * (size_t)l + 1] = to_dev<T>(hd.E[l]);
    }
    hipError_t e1 = dev_alloc(arena, &d.d_piv, piv.size() * sizeof(gp::Piv<T>));
    if (e1 != hipSuccess) return fail(h, GP_ENOMEM, "pivot table allocation failed");
    hipError_t e2 = dev_alloc(arena, &d.d_ae, ae.size() * sizeof(gp::cx<T>));
    if (e2 != hipSuccess) return fail(h, GP_ENOMEM, "coefficient table allocation failed");
    hipError_t e3 = dev_upload(arena, d.d_piv, piv.data(), piv.size() * sizeof(gp::Piv<T>));
    if (e3 != hipSuccess) return hip_fail(h, e3, "pivot table upload");
    hipError_t e4 = dev_upload(arena, d.d_ae, ae.data(), ae.size() * sizeof(gp::cx<T>));
    if (e4 != hipSuccess) return hip_fail(h, e4, "coefficient table upload");
    d.Kg = hd.Kg;
    std::vector<gp::cx<T>> g(hd.G.size()), gc(hd.GC.size());
    for (size_t i = 0; i < g.size(); ++i) g[i] = to_dev<T>(hd.G[i]);
    for (size_t i = 0; i < gc.size(); ++i) gc[i] = to_dev<T>(hd.GC[i]);
    if (dev_alloc(arena, &d.d_g, g.size() * sizeof(gp::cx<T>)) != hipSuccess ||
        dev_alloc(arena, &d.d_gc, gc.size() * sizeof(gp::cx<T>)) != hipSuccess)
        return fail(h, GP_ENOMEM, "correction table allocation failed");
    hipError_t e5 = dev_upload(arena, d.d_g, g.data(), g.size() * sizeof(gp::cx<T>));
    if (e5 != hipSuccess) return hip_fail(h, e5, "correction table upload");
    hipError_t e6 = dev_upload(arena, d.d_gc, gc.data(), gc.size() * sizeof(gp::cx<T>));
    if (e6 != hipSuccess) return hip_fail(h, e6, "correction table upload");
    // (arena uploads read the host vectors asynchronously: wait before they go)
    if (arena && arena->base) {
        hipError_t e7 = hipStreamSynchronize(arena->stream);
        if (e7 != hipSuccess) return hip_fail(h, e7, "table upload");
    }
    return GP_OK;
}

template <typename T>
gp::LineSet<T> lineset(const DirTable& d) {
    gp::LineSet<T> ls;
    ls.piv = (const gp::Piv<T>*)d.d_piv;
    ls.ae = (const gp::cx<T>*)d.d_ae;
    ls.bm1 = to_dev<T>(d.bm1);
    ls.K = d.K;
    ls.g = (const gp::cx<T>*)d.d_g;
    ls.gc = (const gp::cx<T>*)d.d_gc;
    ls.Kg = d.Kg;
    return ls;
}

gp::Phys phys(const gp_spin1_params& p) {
    gp::Phys ph;
    ph.nx = p.nx; ph.ny = p.ny;
    ph.dx = p.dx; ph.dy = p.dy; ph.x0 = p.x0; ph.y0 = p.y0; ph.dt = p.dt;
    ph.c0 = p.c0; ph.c2 = p.c2; ph.rabi = p.rabi;
    ph.dtl = p.split == GP_SPLIT_STRANG ? 0.5 * p.dt : p.dt;
    const double gx = p.trap_gx == 0.0 ? 1.0 : p.trap_gx, gy = p.trap_gy == 0.0 ? 1.0 : p.trap_gy;
    ph.gx2 = gx * gx;
    ph.gy2 = gy * gy;
    return ph;
}

gp::NormRule norm_rule(const gp_spin1_params& p) {
    return gp::NormRule{p.fix_magnetization, p.magnetization};
}

// x launch shape for K points per thread: G threads per row (a multiple of
// 64), R rows per block; false if this K cannot hold a row of nx points.
bool x_shape(int nx, int K, int& G, int& R) {
    G = ((nx + K - 1) / K + 63) / 64 * 64;
    if (G > gp::xk_bound(K) || G > 1024) return false;
    R = std::max(1, std::min(8, 256 / G));
    while (G * R > gp::xk_bound(K)) --R;
    return true;
}

// Whether the whole-row x sweep can run K points per thread: the row fits a
// block, and where the three lines are solved together (K s <= 32 bytes,
// s = sizeof(T)) the line-start correction of Kg points lies in the row's
// first wave (the long-row path with K s > 32 takes the tabulated transient
// pivots itself and needs no correction).
bool x_shape_ok(int nx, int K, int Kg, size_t s, int& G, int& R) {
    return x_shape(nx, K, G, R) && (s * K > 32 || Kg <= 64 * K);
}

// Default x shape before any tuning: the fewest points per thread (at least
// two) that keep a row within 512 threads.
int x_default_k(int nx, int Kg, size_t s) {
    for (int idx = 1; idx < gp::kNumXK; ++idx) {
        const int K = gp::xk_value(idx);
        int G, R;
        if (x_shape_ok(nx, K, Kg, s, G, R) && G <= 512) return K;
    }
    return 16;
}

// Line tables, stability checks and the launch plan of one propagation mode,
// all on the host.
struct HostMode {
    HostDir x, y;
    bool stable = true;
    std::string why;
    bool window = false;
    int hh = 0, h = 0, L = 0;
    int xK = 2, xG = 64, xR = 1, ytile = 0;
    bool xwindow = false;
    int hhx = 0, hx = 0, Lx = 0, xtile = 0;
    int xorder = 1, yorder = 0;  // block orders of the windowed sweeps
    bool xchain = false, ychain = false, ystack = false;
    int xctile = 0, hcx = 0, Lcx = 0, yctile = 0, hcy = 0, Lcy = 0;
};

// Halo that makes decay^h fall below the rounding level of T.
template <typename T> int halo_for(double decay) {
    const double tolw = sizeof(T) == 8 ? std::ldexp(1.0, -60) : std::ldexp(1.0, -32);
    if (decay <= 0.0) return 1;
    if (decay >= 1.0) return 1 << 20;
    return (int)std::ceil(std::log(tolw) / std::log(decay)) + 1;
}

// Window of a y tile shape: the whole column fits one window (no halo), or
// windows of W rows overlap by the halo hh on each side and write W - 2 hh
// rows (accepted while the halo is at most a quarter of the window).
bool tile_window(int ny, int hh, int W, int& h, int& L) {
    if (ny <= W) { h = 0; L = W; return true; }
    if (2 * hh <= W / 2) { h = hh; L = W - 2 * hh; return true; }
    return false;
}

// Chain windows (gp_chain.hpp): a window of W points (64 K along x, 16 K
// along y) writes L = W - 2 h of them, h the halo the decay bound asks for;
// the first window writes every point of the line-start correction.  Along y
// the kernels address a plane with 32-bit byte offsets.
template <typename T> bool xchain_fits(int hh, int Kg, int t, int& h, int& L) {
    const gp::ChainTile ct = gp::xchain_tile<T>(t);
    h = std::max(hh, 1);
    L = 64 * ct.K - 2 * h;
    return L > 0 && Kg <= L;
}
template <typename T> bool ychain_fits(int nx, int ny, int hh, int Kg, int t, int& h, int& L) {
    const gp::ChainTile ct = gp::ychain_tile<T>(t);
    h = std::max(hh, 1);
    L = 16 * ct.K - 2 * h;
    return L > 0 && Kg <= L && (double)nx * ny * sizeof(gp::cx<T>) < 4294967296.0;
}

template <typename T> bool ystack_fits(int nx, int ny, int hh, int Kg, int t, int& h, int& L) {
    const gp::ChainTile ct = gp::ystack_tile<T>(t);
    const int ns = 4 * ct.NW;  // segments per window
    h = std::max(hh, 1);
    L = ns * ct.K - 2 * h;
    return L > 0 && Kg <= L && gp::chain_lanes(h, ct.K) <= ns - 1 && (double)nx * ny * sizeof(gp::cx<T>) < 4294967296.0;
}

// Row tile of the y windows as launched.  Under row bands (order 3) each XCD
// owns a contiguous range of row tiles, and ny / L tiles rarely split evenly
// over the 8 XCDs (512 rows of 42: 13 tiles, so some XCDs hold twice the
// rows of others, in both sweeps).  There the tile shrinks to the height that
// gives 8 m tiles, m = ceil(nrt / 8); the window keeps its span W, and the rows
// it no longer writes widen its halo on both sides.
void band_tile(int ny, int order, int W, int h, int L, int& hb, int& Lb) {
    hb = h;
    Lb = L;
    if (order != 3 || ny <= W) return;
    const int nrt = (ny + L - 1) / L;
    const int m = (nrt + gp::kNumXcd - 1) / gp::kNumXcd;
    const int Le = (ny + gp::kNumXcd * m - 1) / (gp::kNumXcd * m);
    if (Le >= L) return;
    Lb = Le;
    hb = (W - Le) / 2;  // >= h, as Le < L = W - 2 h; the lower halo is W - Le - hb >= hb
}

template <typename T>
void host_mode(const gp_spin1_params& p, bool imag, HostMode& hm) {
    const zd alpha = imag ? zd(0.5 * p.dt, 0.0) : zd(0.0, 0.5 * p.dt);
    auto xdir = [&] {
        host_dir<T>(hm.x, p.nx, p.ny, alpha, p.dx, [&](int l) {
            const double y = p.y0 + (l / 3) * p.dy;
            return zd(0.0, -(p.omega * y - p.gamma * kNu[l % 3]));  // c = -i (Omega y - gamma nu)
        });
    };
    auto ydir = [&] {
        host_dir<T>(hm.y, p.ny, p.nx, alpha, p.dy, [&](int l) {
            const double x = p.x0 + (l / 3) * p.dx;
            return zd(0.0, p.omega * x - p.eta * p.gamma * kNu[l % 3]);  // c = i (Omega x - eta gamma mu)
        });
    };
    if ((long)p.nx + p.ny < 1024) {
        xdir();
        ydir();
    } else {
        // large grids: the y tables on a second thread (an exception there is
        // passed on after the join)
        std::exception_ptr err;
        std::thread ty([&] {
            try { ydir(); } catch (...) { err = std::current_exception(); }
        });
        try { xdir(); } catch (...) { ty.join(); throw; }
        ty.join();
        if (err) std::rethrow_exception(err);
    }
    hm.stable = true;
    hm.why.clear();
    if (!hm.x.dominant || !hm.y.dominant) {
        hm.stable = false;
        hm.why = "line systems are not diagonally dominant (dt too large for dx, dy and the rotation/SO terms)";
    }
    if (imag) {
        const double Lmax = std::max(std::max(std::fabs(p.x0), std::fabs(p.x0 + (p.nx - 1) * p.dx)),
                                     std::max(std::fabs(p.y0), std::fabs(p.y0 + (p.ny - 1) * p.dy)));
        const double cm = std::fabs(p.omega) * Lmax + std::fabs(p.gamma);
        if (0.25 * p.dt * cm * cm >= 1.0) {
            hm.stable = false;
            hm.why = "imaginary-time Cayley bound (dt/4)(|Omega| L_max + |gamma|)^2 < 1 fails";
        }
    }
    // y plan: windows overlapping by h rows on each side, where the truncated
    // carries decay by decay^h below the rounding level of T.
    const double tolw = sizeof(T) == 8 ? std::ldexp(1.0, -60) : std::ldexp(1.0, -32);
    if (hm.y.decay <= 0.0) hm.hh = 1;
    else if (hm.y.decay >= 1.0) hm.hh = 1 << 20;
    else hm.hh = (int)std::ceil(std::log(tolw) / std::log(hm.y.decay)) + 1;
    // the first window must write every point the line-start correction touches
    hm.hh = std::max(hm.hh, hm.y.Kg);
    hm.window = false;
    hm.h = 0;
    hm.L = 0;
    hm.ytile = 0;
    if (p.y_solver != GP_YSOLVER_THOMAS) {
        if (p.y_tile > 0 && p.y_solver != GP_YSOLVER_CHAIN && p.y_solver != GP_YSOLVER_STACK) {
            hm.ytile = p.y_tile - 1;
            hm.window = tile_window(p.ny, hm.hh, gp::ywindow(gp::ytile<T>(hm.ytile)), hm.h, hm.L);
        } else {
            for (int t = 0; t < gp::kNumYTiles && !hm.window; ++t)
                if (tile_window(p.ny, hm.hh, gp::ywindow(gp::ytile<T>(t)), hm.h, hm.L)) { hm.window = true; hm.ytile = t; }
        }
    }
    // launch shapes requested in p, else the defaults (autotuning may replace them)
    hm.xK = p.x_points > 0 ? p.x_points : x_default_k(p.nx, hm.x.Kg, sizeof(T));
    x_shape(p.nx, hm.xK, hm.xG, hm.xR);
    // x windows: only when asked for (autotuning may also choose them)
    hm.hhx = std::max(halo_for<T>(hm.x.decay), hm.x.Kg);
    hm.xwindow = false;
    hm.hx = hm.Lx = hm.xtile = 0;
    if (p.x_solver == GP_XSOLVER_WINDOW) {
        if (p.x_tile > 0) {
            hm.xtile = p.x_tile - 1;
            hm.xwindow = tile_window(p.nx, hm.hhx, gp::ywindow(gp::ytile<T>(hm.xtile)), hm.hx, hm.Lx);
        } else {
            for (int t = 0; t < gp::kNumYTiles && !hm.xwindow; ++t)
                if (tile_window(p.nx, hm.hhx, gp::ywindow(gp::ytile<T>(t)), hm.hx, hm.Lx)) { hm.xwindow = true; hm.xtile = t; }
        }
    }
    // chain windows: when asked for, and by default on large grids and long
    // rows (below); autotuning may also choose them
    hm.xchain = hm.ychain = false;
    if (p.x_solver == GP_XSOLVER_CHAIN) {
        for (int t = p.x_tile > 0 ? p.x_tile - 1 : 0; t < gp::kNumChainTiles && !hm.xchain; ++t) {
            if (xchain_fits<T>(hm.hhx, hm.x.Kg, t, hm.hcx, hm.Lcx)) { hm.xchain = true; hm.xctile = t; }
            if (p.x_tile > 0) break;
        }
    }
    const bool large = (double)p.nx * p.ny >= 1048576.0;  // 1024^2 points and up
    if (p.x_solver == GP_XSOLVER_AUTO && p.x_points == 0 && (hm.xK == 16 || large)) {
        // rows longer than 512 threads of eight points: the whole-row solve
        // would hold sixteen points per thread and spill; the chain windows
        // take rows of any length, and on large grids they are the faster
        // sweep (4096^2 FP64: 316 against 777 us).  FP64: two points per
        // lane, one line at a time, while the window writes at least 3/4 of
        // the points it loads (4096^2: 316-320 against 371-385 us for four
        // points per lane).  Then four points per lane (the fastest FP32
        // tiles), one line at a time first; where no such tile fits, the tile
        // that writes the largest share of the points it loads (sixteen
        // points per lane spill with the local substep fused)
        if (sizeof(T) == 8) {
            constexpr int t2 = 6;  // {K = 2, 4 waves, one line at a time}
            int h2, L2;
            if (xchain_fits<T>(hm.hhx, hm.x.Kg, t2, h2, L2) && 4 * L2 >= 3 * 64 * gp::xchain_tile<T>(t2).K) {
                hm.xchain = true;
                hm.xctile = t2;
                hm.hcx = h2;
                hm.Lcx = L2;
            }
        }
        for (int i = 0; i < gp::kNumChainTiles && !hm.xchain; ++i) {
            const int t = gp::kNumChainTiles - 1 - i;  // (one line at a time first: fewer registers)
            if (gp::xchain_tile<T>(t).K == 4 && xchain_fits<T>(hm.hhx, hm.x.Kg, t, hm.hcx, hm.Lcx)) {
                hm.xchain = true;
                hm.xctile = t;
            }
        }
        double best = 0.0;
        for (int i = 0; i < gp::kNumChainTiles && !hm.xchain; ++i) {
            const int t = (i + 4) % gp::kNumChainTiles;
            int h, L;
            if (gp::xchain_tile<T>(t).K > 8 || !xchain_fits<T>(hm.hhx, hm.x.Kg, t, h, L)) continue;
            const double eff = (double)L / (64.0 * gp::xchain_tile<T>(t).K);
            if (eff > best) { best = eff; hm.xctile = t; hm.hcx = h; hm.Lcx = L; }
        }
        if (best > 0.0) hm.xchain = true;
    }
    if (p.y_solver == GP_YSOLVER_CHAIN) {
        for (int t = p.y_tile > 0 ? p.y_tile - 1 : 0; t < gp::kNumChainTiles && !hm.ychain; ++t) {
            if (ychain_fits<T>(p.nx, p.ny, hm.hh, hm.y.Kg, t, hm.hcy, hm.Lcy)) { hm.ychain = true; hm.yctile = t; }
            if (p.y_tile > 0) break;
        }
    }
    hm.ystack = false;
    if (p.y_solver == GP_YSOLVER_AUTO && p.y_tile == 0 && large) {
        // large grids: the stacked chain windows (4096^2 FP64: 362 against
        // 480 us for the scanned windows), the first tile that fits
        for (int t = 0; t < gp::kNumStackTiles && !hm.ychain; ++t)
            if (ystack_fits<T>(p.nx, p.ny, hm.hh, hm.y.Kg, t, hm.hcy, hm.Lcy)) { hm.ychain = hm.ystack = true; hm.yctile = t; }
    }
    if (p.y_solver == GP_YSOLVER_STACK) {
        for (int t = p.y_tile > 0 ? p.y_tile - 1 : 0; t < gp::kNumStackTiles && !hm.ychain; ++t) {
            if (ystack_fits<T>(p.nx, p.ny, hm.hh, hm.y.Kg, t, hm.hcy, hm.Lcy)) { hm.ychain = hm.ystack = true; hm.yctile = t; }
            if (p.y_tile > 0) break;
        }
    }
    // block orders: grouping the x windows by XCD has measured as fast or
    // faster at every size; the y windows gain from it only while the grid is
    // about one wave of blocks (on larger grids the eight separate HBM streams
    // cost more than the shared halos save)
    hm.xorder = 1;
    hm.yorder = 0;
    if (p.block_order != GP_ORDER_AUTO) {
        hm.xorder = p.block_order == GP_ORDER_HARDWARE ? 0 : p.block_order == GP_ORDER_ROWS ? 3 : 1;
        hm.yorder = p.block_order == GP_ORDER_HARDWARE ? 0 : p.block_order == GP_ORDER_XCD ? 1
                  : p.block_order == GP_ORDER_BANDS ? 2 : 3;
    } else if (hm.window) {
        const gp::YTile yt = gp::ytile<T>(hm.ytile);
        const long nblk = (long)((p.nx + 4 * yt.NW - 1) / (4 * yt.NW)) * ((p.ny + hm.L - 1) / hm.L);
        hm.yorder = nblk <= 2 * kNumCu ? 1 : 0;
    }
}

// The plan a mode's launches follow (gp_spin1_get_plan).
template <typename T>
void fill_plan(const gp_spin1_params& p, ModeState& ms) {
    gp_spin1_plan* out = &ms.plan;
    std::memset(out, 0, sizeof *out);
    out->x_points_per_thread = ms.xchain ? gp::xchain_tile<T>(ms.xctile).K : ms.xK;
    out->x_threads_per_row = ms.xG;
    out->x_rows_per_block = ms.xR;
    const gp::YTile yt = gp::ytile<T>(ms.ytile);
    if (ms.ychain) {
        const gp::ChainTile ct = ms.ystack ? gp::ystack_tile<T>(ms.yctile) : gp::ychain_tile<T>(ms.yctile);
        out->y_solver = ms.ystack ? GP_YSOLVER_STACK : GP_YSOLVER_CHAIN;
        out->y_halo = ms.hcy;
        out->y_rows_out = ms.Lcy;
        out->y_tile = ms.yctile + 1;
        out->y_tile_cols = ms.ystack ? 16 : 4 * ct.NW;
        out->y_rows_per_thread = ct.K;
    } else {
        out->y_solver = ms.window ? GP_YSOLVER_WINDOW : GP_YSOLVER_THOMAS;
        band_tile(p.ny, ms.window ? ms.yorder : 0, gp::ywindow(yt), ms.h, ms.L, out->y_halo, out->y_rows_out);
        out->y_tile = ms.ytile + 1;
        out->y_tile_cols = 4 * yt.NW;
        out->y_rows_per_thread = yt.KY;
    }
    out->y_segments = ms.ystack ? 4 * gp::ystack_tile<T>(ms.yctile).NW : 16;
    out->pivots_x = ms.x.K;
    out->pivots_y = ms.y.K;
    out->decay_x = ms.x.decay;
    out->decay_y = ms.y.decay;
    out->stable = ms.stable ? 1 : 0;
    if (ms.xchain) {
        out->x_solver = GP_XSOLVER_CHAIN;
        out->x_halo = ms.hcx;
        out->x_points_out = ms.Lcx;
        out->x_tile = ms.xctile + 1;
        out->x_block_order = ms.xorder ? 1 : 0;
    } else {
        out->x_solver = ms.xwindow ? GP_XSOLVER_WINDOW : GP_XSOLVER_SCAN;
        out->x_halo = ms.xwindow ? ms.hx : 0;
        out->x_points_out = ms.xwindow ? ms.Lx : 0;
        out->x_tile = ms.xwindow ? ms.xtile + 1 : 0;
        out->x_block_order = ms.xorder == 3 && !ms.window ? (ms.xwindow ? 1 : 0) : ms.xwindow || ms.xorder == 3 ? ms.xorder : 0;
    }
    out->y_block_order = ms.window || ms.ychain ? ms.yorder : 0;
}

template <typename T>
void copy_plan(const gp_spin1_params& p, const HostMode& hm, ModeState& ms);

template <typename T>
int build_mode(gp_spin1* h, ModeState& ms, bool imag, Arena* arena = nullptr) {
    const gp_spin1_params& p = h->p;
    HostMode hm;
    host_mode<T>(p, imag, hm);
    int rc = upload_dir<T>(h, hm.x, ms.x, arena);
    if (rc) return rc;
    rc = upload_dir<T>(h, hm.y, ms.y, arena);
    if (rc) return rc;
    copy_plan<T>(p, hm, ms);
    return GP_OK;
}

// The launch choices of a host-side mode (tables excepted), and the plan.
template <typename T>
void copy_plan(const gp_spin1_params& p, const HostMode& hm, ModeState& ms) {
    ms.x.K = hm.x.K; ms.x.decay = hm.x.decay; ms.x.Kg = hm.x.Kg;
    ms.y.K = hm.y.K; ms.y.decay = hm.y.decay; ms.y.Kg = hm.y.Kg;
    ms.stable = hm.stable;
    ms.why = hm.why;
    ms.window = hm.window;
    ms.hh = hm.hh;
    ms.h = hm.h;
    ms.L = hm.L;
    ms.xK = hm.xK; ms.xG = hm.xG; ms.xR = hm.xR;
    ms.ytile = hm.ytile;
    ms.xwindow = hm.xwindow;
    ms.hhx = hm.hhx; ms.hx = hm.hx; ms.Lx = hm.Lx; ms.xtile = hm.xtile;
    ms.xorder = hm.xorder; ms.yorder = hm.yorder;
    ms.xchain = hm.xchain; ms.xctile = hm.xctile; ms.hcx = hm.hcx; ms.Lcx = hm.Lcx;
    ms.ychain = hm.ychain; ms.ystack = hm.ystack; ms.yctile = hm.yctile; ms.hcy = hm.hcy; ms.Lcy = hm.Lcy;
    fill_plan<T>(p, ms);
}

// Blocks of the y sweep for the largest grid of any tile shape (partials).
template <typename T>
size_t max_y_blocks(const gp_spin1_params& p, const ModeState& ms) {
    size_t best = (size_t)(p.nx + 255) / 256;  // per-column Thomas
    // chain tiles (any may be chosen by the autotuner)
    for (int t = 0; t < gp::kNumChainTiles; ++t) {
        int h, L;
        if (!ychain_fits<T>(p.nx, p.ny, ms.hh, ms.y.Kg, t, h, L)) continue;
        const gp::ChainTile ct = gp::ychain_tile<T>(t);
        best = std::max(best, (size_t)((p.nx + 4 * ct.NW - 1) / (4 * ct.NW)) * ((p.ny + L - 1) / L));
    }
    for (int t = 0; t < gp::kNumStackTiles; ++t) {
        int h, L;
        if (!ystack_fits<T>(p.nx, p.ny, ms.hh, ms.y.Kg, t, h, L)) continue;
        best = std::max(best, (size_t)((p.nx + 15) / 16) * ((p.ny + L - 1) / L));
    }
    if (!ms.window) return best;
    for (int t = 0; t < gp::kNumYTiles; ++t) {
        const gp::YTile yt = gp::ytile<T>(t);
        int h, L;
        if (!tile_window(p.ny, ms.hh, gp::ywindow(yt), h, L)) continue;
        // (+7: the row-band tiles, at most 8 ceil(nrt / 8) of them)
        best = std::max(best, (size_t)((p.nx + 4 * yt.NW - 1) / (4 * yt.NW)) * ((p.ny + L - 1) / L + 7));
    }
    return best;
}

void free_dir(DirTable& d) {
    if (d.d_piv) (void)hipFree(d.d_piv);
    if (d.d_ae) (void)hipFree(d.d_ae);
    if (d.d_g) (void)hipFree(d.d_g);
    if (d.d_gc) (void)hipFree(d.d_gc);
    d.d_piv = d.d_ae = nullptr;
}

void destroy_all(gp_spin1* h) {
    if (!h->graphs.empty()) (void)hipStreamSynchronize(h->stream);
    for (auto& g : h->graphs) {
        (void)hipGraphExecDestroy(g.x);
        (void)hipGraphDestroy(g.g);
    }
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (auto& m : h->mode) { free_dir(m.x); free_dir(m.y); }
    if (h->d_scale) (void)hipFree(h->d_scale);
    if (h->d_flag) (void)hipFree(h->d_flag);
    if (h->d_part) (void)hipFree(h->d_part);
    if (h->d_obs) (void)hipFree(h->d_obs);
    if (h->d_work) (void)hipFree(h->d_work);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    delete h;
}

bool finite(double v) { return std::isfinite(v); }

int validate(const gp_spin1_params* p, std::string& why) {
    if (!p) { why = "params is NULL"; return GP_EINVAL; }
    if (p->nx < 3 || p->ny < 3) { why = "nx and ny must be >= 3"; return GP_EINVAL; }
    if (!(p->dx > 0) || !(p->dy > 0) || !finite(p->dx) || !finite(p->dy)) { why = "dx, dy must be finite and > 0"; return GP_EINVAL; }
    if (!(p->dt > 0) || !finite(p->dt)) { why = "dt must be finite and > 0"; return GP_EINVAL; }
    if (!finite(p->c0) || !finite(p->c2) || !finite(p->gamma) || !finite(p->rabi) || !finite(p->omega)) {
        why = "c0, c2, gamma, rabi, omega must be finite";
        return GP_EINVAL;
    }
    if ((!std::isnan(p->x0) && !finite(p->x0)) || (!std::isnan(p->y0) && !finite(p->y0))) {
        why = "x0, y0 must be finite (or NaN for the default)";
        return GP_EINVAL;
    }
    if (p->plane_stride != 0 && (p->plane_stride < (int64_t)p->nx * p->ny || p->plane_stride > ((int64_t)1 << 40))) {
        why = "plane_stride must be 0 or at least nx * ny";
        return GP_EINVAL;
    }
    if (p->eta != 1 && p->eta != -1) { why = "eta must be +1 (Rashba) or -1 (Dresselhaus)"; return GP_EINVAL; }
    if (p->precision != GP_FP64 && p->precision != GP_FP32) { why = "precision must be GP_FP64 or GP_FP32"; return GP_EINVAL; }
    if (p->y_solver < GP_YSOLVER_AUTO || p->y_solver > GP_YSOLVER_STACK) { why = "unknown y_solver"; return GP_EINVAL; }
    const int nmax = 8192;
    if (p->nx > nmax) { why = "nx above the longest row the library handles (8192)"; return GP_EUNSUPPORTED; }
    if ((double)p->nx * (double)p->ny * 3.0 > 4.0e9) { why = "grid too large"; return GP_EUNSUPPORTED; }
    if (!finite(p->trap_gx) || !finite(p->trap_gy) || p->trap_gx < 0 || p->trap_gy < 0) {
        why = "trap_gx, trap_gy must be finite and >= 0 (0 selects 1)";
        return GP_EINVAL;
    }
    if (p->x_solver < GP_XSOLVER_AUTO || p->x_solver > GP_XSOLVER_CHAIN) { why = "unknown x_solver"; return GP_EINVAL; }
    if (p->block_order < GP_ORDER_AUTO || p->block_order > GP_ORDER_ROWS) { why = "unknown block_order"; return GP_EINVAL; }
    if (p->x_tile < 0 || p->x_tile > gp::kNumYTiles) { why = "x_tile must be 0..8"; return GP_EINVAL; }
    if (p->y_tile < 0 || p->y_tile > gp::kNumYTiles) { why = "y_tile must be 0..8"; return GP_EINVAL; }
    if (p->x_tile > 0 && p->x_solver != GP_XSOLVER_WINDOW && p->x_solver != GP_XSOLVER_CHAIN) {
        why = "x_tile needs x_solver = GP_XSOLVER_WINDOW or GP_XSOLVER_CHAIN";
        return GP_EINVAL;
    }
    if (p->split != GP_SPLIT_LIE && p->split != GP_SPLIT_STRANG) { why = "split must be GP_SPLIT_LIE or GP_SPLIT_STRANG"; return GP_EINVAL; }
    if (p->fix_magnetization != 0 && p->fix_magnetization != 1) { why = "fix_magnetization must be 0 or 1"; return GP_EINVAL; }
    if (p->fix_magnetization) {
        if (!(std::fabs(p->magnetization) < 1.0)) { why = "fixed magnetisation must lie in (-1, 1)"; return GP_EINVAL; }
        if (p->gamma != 0.0 || p->rabi != 0.0) {
            why = "fixed magnetisation needs gamma = 0 and rabi = 0 (otherwise the flow does not conserve it)";
            return GP_EINVAL;
        }
    }
    return GP_OK;
}

template <typename T>
gp::XLaunch<T> xlaunch(gp_spin1* h, const void* src, void* dst, bool imag, bool local, size_t sp, size_t dp);
template <typename T>
gp::YLaunch<T> ylaunch(gp_spin1* h, const void* src, void* dst, bool imag, bool norm, size_t sp, size_t dp);

// Mean duration in ms of `reps` launches of f() after two warm-up launches.
template <typename F>
int time_launches(gp_spin1* h, F f, int reps, float& ms, int batches = 3, float batch_ms = 0.5f) {
    // two untimed launches, then timed batches of at least batch_ms each (the
    // first batch sizes the others); the fastest batch counts, which keeps
    // clock ramps and neighbours' noise out of the comparison
    hipEvent_t a, b;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess) return hip_fail(h, e, "autotune");
    if ((e = hipEventCreate(&b)) != hipSuccess) { (void)hipEventDestroy(a); return hip_fail(h, e, "autotune"); }
    int rc = GP_OK;
    for (int w = 0; w < 2 && rc == GP_OK; ++w)
        if ((e = f()) != hipSuccess) rc = hip_fail(h, e, "autotune launch");
    float best = 1e30f;
    for (int batch = 0; batch < batches && rc == GP_OK; ++batch) {
        if ((e = hipEventRecord(a, h->stream)) != hipSuccess) { rc = hip_fail(h, e, "autotune"); break; }
        for (int r = 0; r < reps && rc == GP_OK; ++r)
            if ((e = f()) != hipSuccess) rc = hip_fail(h, e, "autotune launch");
        if (rc != GP_OK) break;
        float el = 0.f;
        if ((e = hipEventRecord(b, h->stream)) != hipSuccess || (e = hipEventSynchronize(b)) != hipSuccess ||
            (e = hipEventElapsedTime(&el, a, b)) != hipSuccess) {
            rc = hip_fail(h, e, "autotune");
            break;
        }
        el /= reps;
        if (el < best) best = el;
        if (batch == 0 && el > 0.f) reps = std::min(1000, std::max(reps, (int)std::ceil(batch_ms / el)));
    }
    ms = best;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return rc;
}

// Time every admissible x points-per-thread and y tile shape on a scratch
// wave function of this grid, per propagation mode, and keep the fastest
// (fields fixed in the parameters are left as given).
template <typename T>
int autotune_t(gp_spin1* h) {
    const gp_spin1_params& p = h->p;
    const size_t bytes = (2 * h->psp + (size_t)p.nx * p.ny) * sizeof(gp::cx<T>);  // laid out as the caller's
    void* tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, bytes);
    if (e != hipSuccess) return fail(h, GP_ENOMEM, "autotune buffer allocation failed");
    int rc = GP_OK;
    if ((e = hipMemsetAsync(tmp, 0, bytes, h->stream)) != hipSuccess) rc = hip_fail(h, e, "autotune");
    const int reps = 5;
    // bring the clocks up before the first comparison
    if (rc == GP_OK) {
        const gp::XLaunch<T> xa = xlaunch<T>(h, tmp, h->d_work, false, true, h->psp, h->wsp);
        float warm = 0.f;
        rc = time_launches(h, [&] { return gp::launch_x<T>(xa, h->stream); }, reps, warm);
    }
    // block orders to time (x windows: hardware, XCD-contiguous; y windows: also bands), unless p fixes one
    int o0 = 0, o1 = 2, p0 = 0, p1 = 3;
    if (p.block_order != GP_ORDER_AUTO) {
        o0 = p.block_order == GP_ORDER_HARDWARE ? 0 : 1; o1 = o0 + 1;
        p0 = p.block_order == GP_ORDER_HARDWARE ? 0 : p.block_order == GP_ORDER_XCD ? 1
           : p.block_order == GP_ORDER_BANDS ? 2 : 3;
        p1 = p0 + 1;
    }
    for (int m = 0; m < 2 && rc == GP_OK; ++m) {
        ModeState& ms = h->mode[m];
        const bool imag = m == 1;
        // every candidate is timed inside x + y pairs with the current choice
        // for the other sweep, as in a step: a sweep's speed depends on where
        // the previous kernel left its input (which L2, written back or not)
        auto pair = [&](float& t, int batches = 3, float batch_ms = 0.5f) {
            const gp::XLaunch<T> xa = xlaunch<T>(h, tmp, h->d_work, imag, true, h->psp, h->wsp);
            const gp::YLaunch<T> ya = ylaunch<T>(h, h->d_work, tmp, imag, imag, h->wsp, h->psp);
            return time_launches(h, [&] {
                const hipError_t ex = gp::launch_x<T>(xa, h->stream);
                return ex != hipSuccess ? ex : gp::launch_y<T>(ya, h->stream);
            }, reps, t, batches, batch_ms);
        };
        if (p.x_points == 0 && p.x_solver != GP_XSOLVER_WINDOW && p.x_solver != GP_XSOLVER_CHAIN) {
            float best = 1e30f;
            int bestK = ms.xK;
            for (int idx = 0; idx < gp::kNumXK && rc == GP_OK; ++idx) {
                const int K = gp::xk_value(idx);
                int G, R;
                if (!x_shape_ok(p.nx, K, ms.x.Kg, sizeof(T), G, R)) continue;
                ms.xK = K; ms.xG = G; ms.xR = R;
                float t = 0.f;
                rc = pair(t);
                if (rc == GP_OK && t < best) { best = t; bestK = K; }
            }
            ms.xK = bestK;
            x_shape(p.nx, bestK, ms.xG, ms.xR);
            // windows along the rows, where the decay bound fits a window
            ms.xwindow = false;
            if (p.x_solver == GP_XSOLVER_AUTO) {
                int bestT = -1, bestO = ms.xorder;
                for (int t = 0; t < gp::kNumYTiles && rc == GP_OK; ++t) {
                    if (!tile_window(p.nx, ms.hhx, gp::ywindow(gp::ytile<T>(t)), ms.hx, ms.Lx)) continue;
                    for (int o = o0; o < o1 && rc == GP_OK; ++o) {
                        ms.xwindow = true;
                        ms.xtile = t;
                        ms.xorder = o;
                        float tt = 0.f;
                        rc = pair(tt);
                        if (rc == GP_OK && tt < best) { best = tt; bestT = t; bestO = o; }
                    }
                }
                ms.xwindow = bestT >= 0;
                ms.xorder = bestO;
                if (ms.xwindow) {
                    ms.xtile = bestT;
                    tile_window(p.nx, ms.hhx, gp::ywindow(gp::ytile<T>(bestT)), ms.hx, ms.Lx);
                }
            }
        }
        if (p.x_solver == GP_XSOLVER_WINDOW && p.x_tile == 0) {
            // windows asked for: the fastest tile
            float best = 1e30f;
            int bestT = ms.xtile, bestO = ms.xorder;
            for (int t = 0; t < gp::kNumYTiles && rc == GP_OK; ++t) {
                if (!tile_window(p.nx, ms.hhx, gp::ywindow(gp::ytile<T>(t)), ms.hx, ms.Lx)) continue;
                for (int o = o0; o < o1 && rc == GP_OK; ++o) {
                    ms.xtile = t;
                    ms.xorder = o;
                    float tt = 0.f;
                    rc = pair(tt);
                    if (rc == GP_OK && tt < best) { best = tt; bestT = t; bestO = o; }
                }
            }
            ms.xtile = bestT;
            ms.xorder = bestO;
            tile_window(p.nx, ms.hhx, gp::ywindow(gp::ytile<T>(bestT)), ms.hx, ms.Lx);
        }
        // x chain windows: against the choice above (AUTO), or the fastest chain tile (CHAIN)
        if (rc == GP_OK && ((p.x_solver == GP_XSOLVER_AUTO && p.x_points == 0) ||
                            (p.x_solver == GP_XSOLVER_CHAIN && p.x_tile == 0))) {
            float best = 1e30f;
            if (p.x_solver == GP_XSOLVER_AUTO) {
                ms.xchain = false;
                rc = pair(best);
            }
            const bool k0 = ms.xchain;
            const int kt = ms.xctile, ko = ms.xorder;
            bool bestC = k0;
            int bestT = kt, bestO = ko;
            for (int t = 0; t < gp::kNumChainTiles && rc == GP_OK; ++t) {
                if (!xchain_fits<T>(ms.hhx, ms.x.Kg, t, ms.hcx, ms.Lcx)) continue;
                for (int o = o0; o < o1 && rc == GP_OK; ++o) {
                    ms.xchain = true;
                    ms.xctile = t;
                    ms.xorder = o;
                    float tt = 0.f;
                    rc = pair(tt);
                    if (rc == GP_OK && tt < best) { best = tt; bestC = true; bestT = t; bestO = o; }
                }
            }
            ms.xchain = bestC;
            ms.xctile = bestT;
            ms.xorder = bestO;
            if (ms.xchain) xchain_fits<T>(ms.hhx, ms.x.Kg, bestT, ms.hcx, ms.Lcx);
        }
        if (p.y_tile == 0 && ms.window && p.y_solver != GP_YSOLVER_CHAIN && p.y_solver != GP_YSOLVER_STACK) {
            float best = 1e30f;
            int bestT = ms.ytile, bestO = ms.yorder;
            for (int t = 0; t < gp::kNumYTiles && rc == GP_OK; ++t) {
                if (!tile_window(p.ny, ms.hh, gp::ywindow(gp::ytile<T>(t)), ms.h, ms.L)) continue;
                for (int o = p0; o < p1 && rc == GP_OK; ++o) {
                    ms.ytile = t;
                    ms.yorder = o;
                    float tt = 0.f;
                    rc = pair(tt);
                    if (rc == GP_OK && tt < best) { best = tt; bestT = t; bestO = o; }
                }
            }
            ms.ytile = bestT;
            ms.yorder = bestO;
            tile_window(p.ny, ms.hh, gp::ywindow(gp::ytile<T>(bestT)), ms.h, ms.L);
        }
        // y chain windows: against the choice above (AUTO), or the fastest chain tile (CHAIN)
        if (rc == GP_OK && p.y_tile == 0 &&
            (p.y_solver == GP_YSOLVER_AUTO || p.y_solver == GP_YSOLVER_CHAIN || p.y_solver == GP_YSOLVER_STACK)) {
            float best = 1e30f;
            if (p.y_solver == GP_YSOLVER_AUTO) {
                ms.ychain = ms.ystack = false;
                rc = pair(best);
            }
            bool bestC = ms.ychain;
            int bestT = ms.yctile, bestO = ms.yorder;
            bool bestS = ms.ystack;
            // large grids: the hardware order only, unless one is asked for (there
            // the eight XCDs' separate streams through HBM cost more than the shared
            // halos save; short autotuning pairs have measured otherwise, 4096^2 FP32:
            // bands chosen, 198 against 190 us over a run)
            const int pe = p.block_order == GP_ORDER_AUTO && (double)p.nx * p.ny >= 1048576.0 ? 1 : std::min(p1, 3);
            for (int st = 0; st < 2 && rc == GP_OK; ++st) {
                if ((p.y_solver == GP_YSOLVER_CHAIN && st == 1) || (p.y_solver == GP_YSOLVER_STACK && st == 0)) continue;
                for (int t = 0; t < (st ? gp::kNumStackTiles : gp::kNumChainTiles) && rc == GP_OK; ++t) {
                    if (st ? !ystack_fits<T>(p.nx, p.ny, ms.hh, ms.y.Kg, t, ms.hcy, ms.Lcy)
                           : !ychain_fits<T>(p.nx, p.ny, ms.hh, ms.y.Kg, t, ms.hcy, ms.Lcy))
                        continue;
                    for (int o = p0; o < pe && rc == GP_OK; ++o) {
                        ms.ychain = true;
                        ms.ystack = st == 1;
                        ms.yctile = t;
                        ms.yorder = o;
                        float tt = 0.f;
                        rc = pair(tt);
                        if (rc == GP_OK && tt < best) { best = tt; bestC = true; bestS = st == 1; bestT = t; bestO = o; }
                    }
                }
            }
            ms.ychain = bestC;
            ms.ystack = bestC && bestS;
            ms.yctile = bestT;
            ms.yorder = bestO;
            if (ms.ystack) ystack_fits<T>(p.nx, p.ny, ms.hh, ms.y.Kg, bestT, ms.hcy, ms.Lcy);
            else if (ms.ychain) ychain_fits<T>(p.nx, p.ny, ms.hh, ms.y.Kg, bestT, ms.hcy, ms.Lcy);
        }
        if (p.block_order == GP_ORDER_ROWS) ms.xorder = 3;
        // row bands for both sweeps (only as a pair: each sweep then reads what the
        // other wrote on the same XCD), where the y sweep has windows
        if (rc == GP_OK && ms.window && !ms.ychain && !ms.xchain && p.block_order == GP_ORDER_AUTO) {
            const int kx = ms.xorder, ky = ms.yorder;
            const bool kw = ms.xwindow;
            // (the final choice: longer measurements than the sweeps above)
            float best = 0.f;
            rc = pair(best, 5, 2.0f);
            int bx = kx, by = ky;
            bool bw = kw;
            // with the chosen x sweep, and (where windows won) with the fastest whole-row shape
            for (int v = 0; v < 2 && rc == GP_OK; ++v) {
                if (v == 1 && (!kw || p.x_solver == GP_XSOLVER_WINDOW)) continue;
                ms.xwindow = v == 0 ? kw : false;
                ms.xorder = 3;
                ms.yorder = 3;
                float tb = 0.f;
                rc = pair(tb, 5, 2.0f);
                if (rc == GP_OK && tb < best) { best = tb; bx = 3; by = 3; bw = ms.xwindow; }
            }
            ms.xorder = bx;
            ms.yorder = by;
            ms.xwindow = bw;
        }
        fill_plan<T>(p, ms);
    }
    const double one = 1.0;
    const int zero = 0;
    if (rc == GP_OK && (e = hipStreamSynchronize(h->stream)) != hipSuccess) rc = hip_fail(h, e, "autotune");
    const double ones[3] = {one, one, one};
    if (rc == GP_OK && (e = hipMemcpy(h->d_scale, ones, sizeof ones, hipMemcpyHostToDevice)) != hipSuccess) rc = hip_fail(h, e, "autotune");
    if (rc == GP_OK && (e = hipMemcpy(h->d_flag, &zero, sizeof zero, hipMemcpyHostToDevice)) != hipSuccess) rc = hip_fail(h, e, "autotune");
    (void)hipFree(tmp);
    return rc;
}

template <typename T>
int create_t(gp_spin1* h) {
    const gp_spin1_params& p = h->p;
    if (p.x_points > 0) {
        int G, R;
        if ((p.x_points & (p.x_points - 1)) || p.x_points > 16 || !x_shape(p.nx, p.x_points, G, R))
            return fail(h, GP_EUNSUPPORTED, "x_points must be 1, 2, 4, 8 or 16 and hold a row in one block");
    }
    if (p.y_tile < 0 || p.y_tile > gp::kNumYTiles) return fail(h, GP_EINVAL, "y_tile must be 0..8");
    for (int m = 0; m < 2; ++m) {
        int rc = build_mode<T>(h, h->mode[m], m == 1);
        if (rc) return rc;
        int G, R;
        if (p.x_points > 0 && !h->mode[m].xwindow &&
            !x_shape_ok(p.nx, p.x_points, h->mode[m].x.Kg, sizeof(T), G, R))
            return fail(h, GP_EUNSUPPORTED, "x_points too small for the line-start correction of these lines");
        if (p.x_solver == GP_XSOLVER_WINDOW && !h->mode[m].xwindow)
            return fail(h, GP_EUNSUPPORTED, "x windows asked for, but the decay of the x lines fits no window");
        if (p.x_solver == GP_XSOLVER_CHAIN && !h->mode[m].xchain)
            return fail(h, GP_EUNSUPPORTED, "x chain windows asked for, but the decay of the x lines fits no such tile");
        if ((p.y_solver == GP_YSOLVER_CHAIN || p.y_solver == GP_YSOLVER_STACK) && !h->mode[m].ychain)
            return fail(h, GP_EUNSUPPORTED, "y chain windows asked for, but no such tile fits these columns");
    }
    // a handle that no propagation can use is refused here; one stable in real
    // time only is kept, and gp_spin1_step_imag reports the failed bound
    if (!h->mode[0].stable && !h->mode[1].stable) return fail(h, GP_EUNSTABLE, h->mode[0].why);
    size_t need = 1;
    for (auto& m : h->mode) need = std::max(need, max_y_blocks<T>(p, m));
    const size_t npts = (size_t)p.nx * p.ny;
    h->obs_blocks = (int)std::min<size_t>(1024, (npts + 255) / 256);
    need *= 3;  // three component partials per y block
    need = std::max(need, (size_t)h->obs_blocks * gp::kObsCount);
    need = std::max(need, (size_t)1024);
    h->n_part = need;
    if (hipMalloc(&h->d_part, need * sizeof(double)) != hipSuccess) return fail(h, GP_ENOMEM, "scratch allocation failed");
    if (hipMalloc(&h->d_scale, 3 * sizeof(double)) != hipSuccess) return fail(h, GP_ENOMEM, "scratch allocation failed");
    if (hipMalloc(&h->d_flag, sizeof(int)) != hipSuccess) return fail(h, GP_ENOMEM, "scratch allocation failed");
    if (hipMalloc(&h->d_obs, gp::kObsCount * sizeof(double)) != hipSuccess) return fail(h, GP_ENOMEM, "scratch allocation failed");
    h->psp = psi_stride(p);
    h->wsp = work_stride(p);
    if (hipMalloc(&h->d_work, (2 * h->wsp + npts) * sizeof(gp::cx<T>)) != hipSuccess)
        return fail(h, GP_ENOMEM, "work buffer allocation failed");
    const double one = 1.0;
    const int zero = 0;
    hipError_t e;
    const double ones[3] = {one, one, one};
    if ((e = hipMemcpy(h->d_scale, ones, sizeof ones, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(h, e, "init");
    if ((e = hipMemcpy(h->d_flag, &zero, sizeof zero, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(h, e, "init");
    if (p.autotune) {
        int rc = autotune_t<T>(h);
        if (rc) return rc;
    }
    return GP_OK;
}

template <typename T>
gp::XLaunch<T> xlaunch(gp_spin1* h, const void* src, void* dst, bool imag, bool local, size_t sp, size_t dp) {
    gp::XLaunch<T> a;
    a.src = (const gp::cx<T>*)src;
    a.dst = (gp::cx<T>*)dst;
    a.sp = sp;
    a.dp = dp;
    a.ph = phys(h->p);
    a.ls = lineset<T>(h->mode[imag].x);
    a.scale = h->d_scale;
    a.nin = gp::NormIn{nullptr, 0, 0.0, gp::NormRule{0, 0.0}, nullptr};
    const ModeState& ms = h->mode[imag];
    a.K = ms.xK; a.G = ms.xG; a.R = ms.xR;
    a.imag = imag; a.local = local;
    a.window = ms.xwindow; a.L = ms.Lx; a.h = ms.hx; a.tile = ms.xtile;
    a.order = ms.xorder;
    a.chain = ms.xchain;
    if (ms.xchain) { a.window = false; a.L = ms.Lcx; a.h = ms.hcx; a.tile = ms.xctile; }
    // row bands follow the y sweep's row tiles (none without y windows)
    int hb = 0, Lb = 0;
    if (ms.window) band_tile(h->p.ny, ms.yorder, gp::ywindow(gp::ytile<T>(ms.ytile)), ms.h, ms.L, hb, Lb);
    a.bL = Lb;
    a.bnrt = ms.window ? (h->p.ny + Lb - 1) / Lb : 0;
    return a;
}

template <typename T>
gp::YLaunch<T> ylaunch(gp_spin1* h, const void* src, void* dst, bool imag, bool norm, size_t sp, size_t dp) {
    const ModeState& ms = h->mode[imag];
    gp::YLaunch<T> a;
    a.src = (const gp::cx<T>*)src;
    a.dst = (gp::cx<T>*)dst;
    a.ph = phys(h->p);
    a.ls = lineset<T>(ms.y);
    a.no.partials = h->d_part;
    a.L = ms.L; a.h = ms.h; a.tile = ms.ytile;
    if (ms.window) band_tile(h->p.ny, ms.yorder, gp::ywindow(gp::ytile<T>(ms.ytile)), ms.h, ms.L, a.h, a.L);
    a.window = ms.window; a.imag = imag; a.norm = norm;
    a.outl = false;
    a.order = ms.yorder;
    a.chain = ms.ychain && !ms.ystack;
    a.stack = ms.ystack;
    if (ms.ychain) { a.L = ms.Lcy; a.h = ms.hcy; a.tile = ms.yctile; }
    a.sp = sp;
    a.dp = dp;
    return a;
}

// Timing: fold finished event pairs into the per-kind sums.
hipError_t timing_drain(gp_spin1* h) {
    if (h->ev_open.empty()) return hipSuccess;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return e;
    for (auto& o : h->ev_open) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, o.second.first, o.second.second);
        if (e != hipSuccess) return e;
        h->t_ms[o.first] += ms;
        h->t_launches[o.first] += 1;
    }
    h->ev_open.clear();
    h->ev_next = 0;
    return hipSuccess;
}

// Launch f(start, stop) with an event pair of kind k that the dispatch stamps
// at kernel start and end when timing is on (null events otherwise).
template <typename F>
hipError_t timed(gp_spin1* h, int k, F f) {
    if (!h->timing) return f(nullptr, nullptr);
    if (h->ev_next + 2 > 4096) {
        hipError_t e = timing_drain(h);
        if (e != hipSuccess) return e;
    }
    while (h->ev_pool.size() < h->ev_next + 2) {
        hipEvent_t ev;
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) return e;
        h->ev_pool.push_back(ev);
    }
    hipEvent_t a = h->ev_pool[h->ev_next], b = h->ev_pool[h->ev_next + 1];
    h->ev_next += 2;
    hipError_t e = f(a, b);
    if (e != hipSuccess) return e;
    h->ev_open.push_back({k, {a, b}});
    return hipSuccess;
}

template <typename T>
int steps_t(gp_spin1* h, void* psi, int64_t n, bool imag) {
    const ModeState& ms = h->mode[imag];
    if (!ms.stable) return fail(h, GP_EUNSTABLE, ms.why);
    if (n == 0) return GP_OK;
    hipStream_t st = h->stream;
    const gp::XLaunch<T> xa = xlaunch<T>(h, psi, h->d_work, imag, true, h->psp, h->wsp);
    gp::YLaunch<T> ya = ylaunch<T>(h, h->d_work, psi, imag, imag, h->wsp, h->psp);
    ya.outl = h->p.split == GP_SPLIT_STRANG;
    const int nyb = gp::y_blocks<T>(ya);
    const double dxdy = h->p.dx * h->p.dy;
    const gp::NormRule rule = norm_rule(h->p);
    hipError_t e;
    if (imag && (e = gp::launch_set_scale(h->d_scale, 1.0, st)) != hipSuccess) return hip_fail(h, e, "set_scale");
    // Imaginary time: the y sweep leaves per-block norm partials.  Where they are
    // few, every block (whole rows) or wave (chain windows, total norm one) of
    // the next x sweep sums them itself (no launch in between); otherwise one
    // block sums them into the scale factors.  The last step's partials always go through that
    // block (for the final scaling).
    gp::XLaunch<T> xn = xa;
    const bool fold = imag && !xa.window &&
                      (xa.chain ? !rule.fix_m && 3 * nyb <= 8 * 64 : 3 * nyb <= 8 * xa.G * xa.R);
    if (fold) xn.nin = gp::NormIn{h->d_part, nyb, dxdy, rule, h->d_flag};
    for (int64_t s = 0; s < n; ++s) {
        const gp::XLaunch<T>& x = s > 0 ? xn : xa;
        if ((e = timed(h, 0, [&](hipEvent_t a, hipEvent_t b) { return gp::launch_x<T>(x, st, a, b); })) != hipSuccess) return hip_fail(h, e, "x sweep launch");
        if ((e = timed(h, 1, [&](hipEvent_t a, hipEvent_t b) { return gp::launch_y<T>(ya, st, a, b); })) != hipSuccess) return hip_fail(h, e, "y sweep launch");
        if (imag && (!fold || s == n - 1) &&
            (e = timed(h, 2, [&](hipEvent_t a, hipEvent_t b) { return gp::launch_norm_finalize(h->d_part, nyb, dxdy, rule, h->d_scale, h->d_flag, st, a, b); })) != hipSuccess)
            return hip_fail(h, e, "norm launch");
    }
    if (imag) {
        const size_t npts = (size_t)h->p.nx * h->p.ny;
        if ((e = timed(h, 3, [&](hipEvent_t a, hipEvent_t b) { return gp::launch_scale<T>((gp::cx<T>*)psi, npts, h->psp, h->d_scale, st, a, b); })) != hipSuccess)
            return hip_fail(h, e, "scale launch");
    }
    return GP_OK;
}

// The launch sequence of n steps on psi, captured once as a HIP graph (on a
// stream of the handle's own, with per-kernel timing off: event records would
// become graph nodes) and replayed on the handle's stream.  The sequence holds
// kernels only (scale and flag resets are one-thread kernels, no memset
// nodes).  Up to kMaxGraphs captures are kept per handle, the oldest dropped.
constexpr size_t kMaxGraphs = 8;

template <typename T>
int graph_steps_t(gp_spin1* h, void* psi, int64_t n, bool imag) {
    const ModeState& ms = h->mode[imag];
    if (!ms.stable) return fail(h, GP_EUNSTABLE, ms.why);
    if (n == 0) return GP_OK;
    hipError_t e;
    size_t k = 0;
    while (k < h->graphs.size() && !(h->graphs[k].psi == psi && h->graphs[k].n == n && h->graphs[k].imag == imag)) ++k;
    if (k == h->graphs.size()) {
        if (!h->cap_stream && (e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(h, e, "capture stream");
        const hipStream_t st = h->stream;
        const bool timing = h->timing;
        if ((e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(h, e, "begin capture");
        h->stream = h->cap_stream;
        h->timing = false;
        const int rc = steps_t<T>(h, psi, n, imag);
        h->stream = st;
        h->timing = timing;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(h->cap_stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(h, e, "end capture");
        hipGraphExec_t x = nullptr;
        if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_fail(h, e, "graph instantiate");
        }
        if (h->graphs.size() == kMaxGraphs) {
            // (the oldest may still run on the stream)
            if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_fail(h, e, "graph eviction");
            (void)hipGraphExecDestroy(h->graphs.front().x);
            (void)hipGraphDestroy(h->graphs.front().g);
            h->graphs.erase(h->graphs.begin());
        }
        h->graphs.push_back(gp_spin1::Graph{psi, n, imag, g, x});
        k = h->graphs.size() - 1;
    }
    if ((e = hipGraphLaunch(h->graphs[k].x, h->stream)) != hipSuccess) return hip_fail(h, e, "graph launch");
    return GP_OK;
}

template <typename T>
int substep_t(gp_spin1* h, void* psi, int which, bool imag) {
    hipStream_t st = h->stream;
    hipError_t e = hipSuccess;
    const size_t npts = (size_t)h->p.nx * h->p.ny;
    const size_t cs = sizeof(gp::cx<T>);
    switch (which) {
        case 0: e = gp::launch_local<T>((gp::cx<T>*)psi, h->psp, phys(h->p), imag, st); break;
        case 1:
        case 2: {
            // out of place into the work buffer, then back plane by plane
            if (which == 1) e = gp::launch_x<T>(xlaunch<T>(h, psi, h->d_work, imag, false, h->psp, h->wsp), st);
            else e = gp::launch_y<T>(ylaunch<T>(h, psi, h->d_work, imag, false, h->psp, h->wsp), st);
            if (e != hipSuccess) break;
            e = hipMemcpy2DAsync(psi, h->psp * cs, h->d_work, h->wsp * cs, npts * cs, 3, hipMemcpyDeviceToDevice, st);
            break;
        }
        case 3: {
            const int nblk = (int)std::min<size_t>(1024, (3 * npts + 255) / 256);
            if ((e = gp::launch_norm_partials<T>((const gp::cx<T>*)psi, npts, h->psp, h->d_part, nblk, st)) != hipSuccess) break;
            if ((e = gp::launch_norm_finalize(h->d_part, nblk, h->p.dx * h->p.dy, norm_rule(h->p), h->d_scale, h->d_flag,
                                              st)) != hipSuccess)
                break;
            e = gp::launch_scale<T>((gp::cx<T>*)psi, npts, h->psp, h->d_scale, st);
            break;
        }
        default: return fail(h, GP_EINVAL, "substep: which must be 0..3");
    }
    if (e != hipSuccess) return hip_fail(h, e, "substep launch");
    return GP_OK;
}

template <typename T>
int obs_t(gp_spin1* h, const void* psi, gp_spin1_obs* out, void* dens) {
    hipStream_t st = h->stream;
    gp::ObsLaunch o{h->p.c0, h->p.c2, h->p.rabi, h->p.gamma, h->p.omega, h->p.eta};
    hipError_t e;
    if ((e = gp::launch_obs<T>((const gp::cx<T>*)psi, h->psp, phys(h->p), o, (T*)dens, h->d_part, h->obs_blocks, st)) != hipSuccess)
        return hip_fail(h, e, "observables launch");
    if ((e = gp::launch_obs_finalize(h->d_part, h->obs_blocks, h->d_obs, st)) != hipSuccess)
        return hip_fail(h, e, "observables finalize launch");
    double q[gp::kObsCount];
    if ((e = hipMemcpyAsync(q, h->d_obs, sizeof q, hipMemcpyDeviceToHost, st)) != hipSuccess) return hip_fail(h, e, "observables copy");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(h, e, "observables sync");
    const double w = h->p.dx * h->p.dy;
    for (double& v : q) v *= w;
    out->norm[0] = q[0]; out->norm[1] = q[1]; out->norm[2] = q[2];
    out->norm_total = q[0] + q[1] + q[2];
    out->magnetization = q[0] - q[2];
    out->e_kin = q[3]; out->e_trap = q[4]; out->e_int = q[5]; out->e_rot = q[6];
    out->e_so = q[7]; out->e_rabi = q[8]; out->lz = q[9];
    out->energy = q[3] + q[4] + q[5] + q[6] + q[7] + q[8];
    // an empty component (norm exactly 0) has no chemical potential of its own: reported as 0
    for (int m = 0; m < 3; ++m) out->mu[m] = q[m] > 0.0 ? q[10 + m] / q[m] : 0.0;
    out->mu_total = (q[10] + q[11] + q[12]) / out->norm_total;
    for (double v : q)
        if (!std::isfinite(v)) return fail(h, GP_ENONFINITE, "non-finite value in the observables");
    return GP_OK;
}


// A handle from validated parameters (also the slots of a batch).
int make_handle(const gp_spin1_params* p, hipStream_t st, gp_spin1** out) {
    if (!out) return GP_EINVAL;
    std::string why;
    int rc = validate(p, why);
    if (rc) return rc;
    gp_spin1* h = new (std::nothrow) gp_spin1();
    if (!h) return GP_ENOMEM;
    h->p = *p;
    if (std::isnan(h->p.x0)) h->p.x0 = -0.5 * h->p.nx * h->p.dx;
    if (std::isnan(h->p.y0)) h->p.y0 = -0.5 * h->p.ny * h->p.dy;
    h->stream = st;
    if (hipGetDevice(&h->device) != hipSuccess) { destroy_all(h); return GP_EHIP; }
    try {
        rc = h->p.precision == GP_FP64 ? create_t<double>(h) : create_t<float>(h);
    } catch (...) {
        destroy_all(h);
        throw;
    }
    if (rc) { destroy_all(h); return rc; }
    *out = h;
    return GP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Stepping without allocation (gp_spin1_step_static).  The call keeps
// everything beyond the caller's wave function - the line tables, the work
// wave function, the norm partials, the scale factors and the non-finite flag
// - in this array: one copy per GPU, held until the process ends, shared by
// every such call on that GPU.  On the host the array's name is no device
// address; its address on each device comes from hipGetSymbolAddress.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[GP_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The array's address on the current device (looked up on the first call there).
int scratch_base(gp_spin1* h, unsigned char** out) {
    if (h->device < 0 || h->device >= kMaxDevices) return fail(h, GP_EUNSUPPORTED, "device index beyond the static table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[h->device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(h, e, "scratch address");
        if (!p) return fail(h, GP_EHIP, "scratch address: null");
        g_scratch_ptr[h->device] = p;
    }
    *out = (unsigned char*)g_scratch_ptr[h->device];
    return GP_OK;
}

template <typename T>
int step_static_t(gp_spin1* h, void* psi, int64_t n, bool imag) {
    const gp_spin1_params& p = h->p;
    if (p.x_points > 0) {
        int G, R;
        if ((p.x_points & (p.x_points - 1)) || p.x_points > 16 || !x_shape(p.nx, p.x_points, G, R))
            return fail(h, GP_EUNSUPPORTED, "x_points must be 1, 2, 4, 8 or 16 and hold a row in one block");
    }
    unsigned char* base = nullptr;
    int rc = scratch_base(h, &base);
    if (rc) return rc;
    Arena a;
    a.base = base;
    a.cap = GP_STATIC_SCRATCH_BYTES;
    a.stream = h->stream;
    ModeState& ms = h->mode[imag];
    if ((rc = build_mode<T>(h, ms, imag, &a)) != GP_OK) return rc;
    int G, R;
    if (p.x_points > 0 && !ms.xwindow && !x_shape_ok(p.nx, p.x_points, ms.x.Kg, sizeof(T), G, R))
        return fail(h, GP_EUNSUPPORTED, "x_points too small for the line-start correction of these lines");
    if (p.x_solver == GP_XSOLVER_WINDOW && !ms.xwindow)
        return fail(h, GP_EUNSUPPORTED, "x windows asked for, but the decay of the x lines fits no window");
    const size_t npts = (size_t)p.nx * p.ny;
    h->psp = psi_stride(p);
    h->wsp = work_stride(p);
    h->n_part = std::max<size_t>(3 * max_y_blocks<T>(p, ms), 1024);
    const size_t work_bytes = (2 * h->wsp + npts) * sizeof(gp::cx<T>);
    hipError_t e;
    if (dev_alloc(&a, (void**)&h->d_part, h->n_part * sizeof(double)) != hipSuccess ||
        dev_alloc(&a, (void**)&h->d_scale, 3 * sizeof(double)) != hipSuccess ||
        dev_alloc(&a, (void**)&h->d_flag, sizeof(int)) != hipSuccess ||
        dev_alloc(&a, &h->d_work, work_bytes) != hipSuccess) {
        char msg[200];
        std::snprintf(msg, sizeof msg, "grid needs more than the %zu bytes of the static scratch (work wave function alone: %zu)",
                      (size_t)GP_STATIC_SCRATCH_BYTES, work_bytes);
        return fail(h, GP_ENOMEM, msg);
    }
    // start values (kernels, not memsets: a captured memset node misbehaves on replays)
    if ((e = gp::launch_set_scale(h->d_scale, 1.0, h->stream)) != hipSuccess) return hip_fail(h, e, "scale reset");
    if ((e = gp::launch_set_flag(h->d_flag, 0, h->stream)) != hipSuccess) return hip_fail(h, e, "flag reset");
    if ((rc = steps_t<T>(h, psi, n, imag)) != GP_OK) return rc;
    int flag = 0;
    if ((e = hipMemcpyAsync(&flag, h->d_flag, sizeof flag, hipMemcpyDeviceToHost, h->stream)) != hipSuccess)
        return hip_fail(h, e, "flag read");
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_fail(h, e, "sync");
    if (flag) return fail(h, GP_ENONFINITE, "an imaginary-time norm was not finite");
    return GP_OK;
}

// Message of the calling thread's last gp_spin1_step_static failure.
std::string& static_err() {
    thread_local std::string err;
    return err;
}

// One call: a handle on the stack whose device memory is the static array
// (nothing to free afterwards).
int step_static(const gp_spin1_params* p, void* psi, int64_t n, int32_t mode, hipStream_t st, std::string* err) {
    std::string why;
    int rc = validate(p, why);
    if (rc) { if (err) *err = why; return rc; }
    if (p->autotune) { if (err) *err = "autotune needs an allocation: give autotune = 0"; return GP_EINVAL; }
    if (!psi || n < 0 || (mode != 0 && mode != 1)) { if (err) *err = "psi is NULL, nsteps < 0 or mode not 0/1"; return GP_EINVAL; }
    gp_spin1 h;
    h.p = *p;
    if (std::isnan(h.p.x0)) h.p.x0 = -0.5 * h.p.nx * h.p.dx;
    if (std::isnan(h.p.y0)) h.p.y0 = -0.5 * h.p.ny * h.p.dy;
    h.stream = st;
    if (hipGetDevice(&h.device) != hipSuccess) return GP_EHIP;
    const bool imag = mode == 0;
    rc = h.p.precision == GP_FP64 ? step_static_t<double>(&h, psi, n, imag) : step_static_t<float>(&h, psi, n, imag);
    if (rc && err) *err = h.err;
    return rc;
}

}  // namespace

// ---------------------------------------------------------------------------
// Batches: independent condensates (own grid, couplings, time step and mode)
// advanced together.  Every sweep is one launch over the rows / column tiles
// of all condensates that share the batch's launch shape; a condensate whose
// y windows do not fit the batch tile runs on its own handle (same stream).
// ---------------------------------------------------------------------------
struct gp_spin1_batch {
    int n = 0;
    int precision = GP_FP64;
    hipStream_t stream = nullptr;
    std::vector<gp_spin1*> slot;  // nullptr: empty slot
    void* h_stage = nullptr;      // pinned host staging of descriptors and block maps
    size_t h_cap = 0;
    void* d_stage = nullptr;
    size_t d_cap = 0;
    hipEvent_t staged = nullptr;  // recorded after the last upload from h_stage
    bool staged_pending = false;
    gp_spin1_batch_info info{};
    std::string err;
};

namespace {

int bfail(gp_spin1_batch* b, int code, const std::string& msg) {
    b->err = msg;
    return code;
}
int bhip(gp_spin1_batch* b, hipError_t e, const std::string& where) {
    b->err = where + ": " + hipGetErrorString(e);
    return GP_EHIP;
}

void batch_free(gp_spin1_batch* b) {
    for (gp_spin1* h : b->slot)
        if (h) destroy_all(h);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    if (b->d_stage) (void)hipFree(b->d_stage);
    if (b->staged) (void)hipEventDestroy(b->staged);
    delete b;
}

// Append a POD array to the staging image at a 256-byte boundary; returns its offset.
template <typename V>
size_t stage_put(std::vector<unsigned char>& img, const std::vector<V>& v) {
    size_t off = (img.size() + 255) / 256 * 256;
    img.resize(off + v.size() * sizeof(V));
    if (!v.empty()) std::memcpy(img.data() + off, v.data(), v.size() * sizeof(V));
    return off;
}

// The launch shape shared by a group: x points per thread and block size
// from the widest row, the y tile that the most condensates can window.
struct BatchShape {
    int K = 2, block = 64, tile = 0;
    bool chain = false;     // chain x windows and stacked chain y windows
    int xtile = 0, ytile = 0;  // their tiles
};

// The chain shapes of a group, when every condensate of it that can be
// grouped (Lie splitting) leaves both solvers to the library or asks for
// these, and fits one x chain tile and one stacked y tile: the tiles with the
// fewest lane-points over the group.
template <typename T>
bool batch_chain_shape(const std::vector<gp_spin1*>& hs, bool imag, BatchShape& bs) {
    std::vector<gp_spin1*> g;
    for (gp_spin1* h : hs) {
        if (h->p.split != GP_SPLIT_LIE) continue;
        if (h->p.x_solver != GP_XSOLVER_AUTO && h->p.x_solver != GP_XSOLVER_CHAIN) return false;
        if (h->p.y_solver != GP_YSOLVER_AUTO && h->p.y_solver != GP_YSOLVER_STACK) return false;
        g.push_back(h);
    }
    if (g.empty()) return false;
    double bx = -1.0, by = -1.0;
    for (int i = 0; i < gp::kNumChainTiles; ++i) {
        const int t = (i + 4) % gp::kNumChainTiles;  // (one line at a time first: fewer registers)
        if (gp::xchain_tile<T>(t).K > 8) continue;   // (spills with the local substep fused)
        double cost = 0.0;
        bool all = true;
        for (gp_spin1* h : g) {
            const ModeState& ms = h->mode[imag];
            int hh, L;
            if (!xchain_fits<T>(ms.hhx, ms.x.Kg, t, hh, L)) { all = false; break; }
            cost += (double)((h->p.nx + L - 1) / L) * h->p.ny * 64.0 * gp::xchain_tile<T>(t).K;
        }
        if (all && (bx < 0 || cost < bx)) { bx = cost; bs.xtile = t; }
    }
    for (int t = 0; t < gp::kNumStackTiles; ++t) {
        double cost = 0.0;
        bool all = true;
        for (gp_spin1* h : g) {
            const ModeState& ms = h->mode[imag];
            int hh, L;
            if (!ystack_fits<T>(h->p.nx, h->p.ny, ms.hh, ms.y.Kg, t, hh, L)) { all = false; break; }
            cost += (double)((h->p.nx + 15) / 16) * ((h->p.ny + L - 1) / L) * 64.0 * gp::ystack_tile<T>(t).NW *
                    gp::ystack_tile<T>(t).K;
        }
        if (all && (by < 0 || cost < by)) { by = cost; bs.ytile = t; }
    }
    if (bx < 0 || by < 0) return false;
    bs.chain = true;
    bs.K = gp::xchain_tile<T>(bs.xtile).K;
    bs.block = 64 * gp::xchain_tile<T>(bs.xtile).NW;
    return true;
}

template <typename T>
BatchShape batch_shape(const std::vector<gp_spin1*>& hs, bool imag) {
    BatchShape bs;
    int nxmax = 3;
    int kgmax = 1;
    for (gp_spin1* h : hs) {
        nxmax = std::max(nxmax, h->p.nx);
        kgmax = std::max(kgmax, h->mode[imag].x.Kg);
    }
    bs.K = x_default_k(nxmax, kgmax, sizeof(T));
    int G, R;
    x_shape(nxmax, bs.K, G, R);
    bs.block = G;
    int best = -1;
    for (int t = 0; t < gp::kNumYTiles; ++t) {
        int cnt = 0;
        for (gp_spin1* h : hs) {
            const ModeState& ms = h->mode[imag];
            int hh, L;
            if (ms.window && tile_window(h->p.ny, ms.hh, gp::ywindow(gp::ytile<T>(t)), hh, L)) ++cnt;
        }
        if (cnt > best) { best = cnt; bs.tile = t; }
    }
    return bs;
}

// Descriptors and block maps of the chain-shaped group for one phase (the
// condensates with steps left after `done`), appended to the staging image.
template <typename T>
void chain_tables(gp_spin1_batch* b, const std::vector<int>& grouped, void* const* psi, const int64_t* nsteps,
                  int64_t done, bool imag, const BatchShape& bs, std::vector<unsigned char>& img, size_t& o_xs,
                  size_t& o_ys, size_t& o_ns, size_t& o_ss, size_t& o_xm, size_t& o_ym, size_t& o_sm, int& nslot,
                  int& xblk, int& yblk, int& sblk) {
    using C = gp::cx<T>;
    std::vector<gp::XCSlot<T>> xs;
    std::vector<gp::YSSlot<T>> ys;
    std::vector<gp::NSlot> ns;
    std::vector<gp::SSlot<T>> ss;
    std::vector<unsigned> xm, ym, sm;
    const gp::ChainTile xt = gp::xchain_tile<T>(bs.xtile);
    const gp::ChainTile yt = gp::ystack_tile<T>(bs.ytile);
    for (int s : grouped) {
        if (nsteps[s] <= done) continue;
        gp_spin1* h = b->slot[s];
        const ModeState& ms = h->mode[imag];
        const unsigned id = (unsigned)xs.size();
        int hx, Lx, hy, Ly;
        xchain_fits<T>(ms.hhx, ms.x.Kg, bs.xtile, hx, Lx);
        ystack_fits<T>(h->p.nx, h->p.ny, ms.hh, ms.y.Kg, bs.ytile, hy, Ly);
        const int nwin = (h->p.nx + Lx - 1) / Lx;
        const int xb = (int)(((int64_t)nwin * h->p.ny + xt.NW - 1) / xt.NW);
        const int ncs = (h->p.nx + 15) / 16;
        const int nyb = ncs * ((h->p.ny + Ly - 1) / Ly);
        const size_t n3 = (size_t)3 * h->p.nx * h->p.ny;
        const int nsb = (int)((n3 + gp::kScaleChunk - 1) / gp::kScaleChunk);
        xs.push_back(gp::XCSlot<T>{(const C*)psi[s], (C*)h->d_work, phys(h->p), lineset<T>(ms.x), h->d_scale, hx,
                                   gp::chain_lanes(hx, xt.K), Lx, nwin, h->psp, h->wsp});
        ys.push_back(gp::YSSlot<T>{(const C*)h->d_work, (C*)psi[s], phys(h->p), lineset<T>(ms.y), h->d_part, Ly, hy,
                                   gp::chain_lanes(hy, yt.K), ncs, h->wsp, h->psp});
        ns.push_back(gp::NSlot{h->d_part, nyb, h->p.dx * h->p.dy, h->d_scale, h->d_flag, norm_rule(h->p)});
        ss.push_back(gp::SSlot<T>{(C*)psi[s], n3 / 3, h->psp, h->d_scale});
        for (int k = 0; k < xb; ++k) xm.push_back((id << gp::kMapShift) | (unsigned)k);
        for (int k = 0; k < nyb; ++k) ym.push_back((id << gp::kMapShift) | (unsigned)k);
        for (int k = 0; k < nsb; ++k) sm.push_back((id << gp::kMapShift) | (unsigned)k);
    }
    nslot = (int)xs.size();
    if (!nslot) return;
    xblk = (int)xm.size();
    yblk = (int)ym.size();
    sblk = (int)sm.size();
    o_xs = stage_put(img, xs);
    o_ys = stage_put(img, ys);
    o_ns = stage_put(img, ns);
    o_ss = stage_put(img, ss);
    o_xm = stage_put(img, xm);
    o_ym = stage_put(img, ym);
    o_sm = stage_put(img, sm);
}

template <typename T>
int batch_step_t(gp_spin1_batch* b, void* const* psi, const int64_t* nsteps, const int32_t* mode,
                 const uint8_t* active) {
    using C = gp::cx<T>;
    hipStream_t st = b->stream;
    std::vector<int> act;
    for (int s = 0; s < b->n; ++s) {
        if (active && !active[s]) continue;
        if (nsteps[s] < 0) return bfail(b, GP_EINVAL, "slot " + std::to_string(s) + ": nsteps < 0");
        if (nsteps[s] == 0) continue;
        if (!b->slot[s]) return bfail(b, GP_EINVAL, "slot " + std::to_string(s) + " is empty");
        if (!psi[s]) return bfail(b, GP_EINVAL, "slot " + std::to_string(s) + ": psi is NULL");
        if (mode[s] != 0 && mode[s] != 1) return bfail(b, GP_EINVAL, "slot " + std::to_string(s) + ": mode must be 0 or 1");
        const ModeState& ms = b->slot[s]->mode[mode[s] == 0];
        if (!ms.stable) return bfail(b, GP_EUNSTABLE, "slot " + std::to_string(s) + ": " + ms.why);
        act.push_back(s);
    }
    b->info = gp_spin1_batch_info{};
    if (act.empty()) return GP_OK;
    // launch shape per mode (index 1 = imaginary time) and the grouped / individual split
    BatchShape shape[2];
    std::vector<int> grouped[2];
    for (int im = 0; im < 2; ++im) {
        std::vector<gp_spin1*> hs;
        for (int s : act)
            if ((mode[s] == 0) == (im == 1)) hs.push_back(b->slot[s]);
        if (hs.empty()) continue;
        if (!batch_chain_shape<T>(hs, im == 1, shape[im])) shape[im] = batch_shape<T>(hs, im == 1);
    }
    int64_t maxn = 0;
    for (int s : act) {
        const bool im = mode[s] == 0;
        gp_spin1* h = b->slot[s];
        const ModeState& ms = h->mode[im];
        int hh, L, G, R;
        // Strang slots need the y sweep's output substep, which the batched kernel does not carry
        bool ok;
        if (shape[im].chain) {
            const gp::ChainTile xt = gp::xchain_tile<T>(shape[im].xtile);
            int hx, Lx;
            ok = h->p.split == GP_SPLIT_LIE && xchain_fits<T>(ms.hhx, ms.x.Kg, shape[im].xtile, hx, Lx) &&
                 ystack_fits<T>(h->p.nx, h->p.ny, ms.hh, ms.y.Kg, shape[im].ytile, hh, L);
            if (ok) {
                const int64_t xb = ((int64_t)((h->p.nx + Lx - 1) / Lx) * h->p.ny + xt.NW - 1) / xt.NW;
                const int64_t yb = (int64_t)((h->p.nx + 15) / 16) * ((h->p.ny + L - 1) / L);
                const int64_t sb = ((int64_t)3 * h->p.nx * h->p.ny + gp::kScaleChunk - 1) / gp::kScaleChunk;
                const int64_t lim = (int64_t)gp::kMapMask + 1;
                ok = xb <= lim && yb <= lim && sb <= lim;
            }
        } else {
            ok = h->p.split == GP_SPLIT_LIE && ms.window &&
                 tile_window(h->p.ny, ms.hh, gp::ywindow(gp::ytile<T>(shape[im].tile)), hh, L) &&
                 x_shape_ok(h->p.nx, shape[im].K, ms.x.Kg, sizeof(T), G, R) && G <= shape[im].block;
            if (ok) {
                // every block of a grouped condensate is named by a map entry with
                // kMapShift bits of block index: larger condensates run alone
                const gp::YTile yt = gp::ytile<T>(shape[im].tile);
                const int64_t rb = std::max(1, std::min(8, shape[im].block / G));
                const int64_t xb = (h->p.ny + rb - 1) / rb;
                const int64_t yb = (int64_t)((h->p.nx + 4 * yt.NW - 1) / (4 * yt.NW)) * ((h->p.ny + L - 1) / L);
                const int64_t sb = ((int64_t)3 * h->p.nx * h->p.ny + gp::kScaleChunk - 1) / gp::kScaleChunk;
                const int64_t lim = (int64_t)gp::kMapMask + 1;
                ok = xb <= lim && yb <= lim && sb <= lim;
            }
        }
        // and the map names at most kMaxBatchSlots condensates per launch
        if (ok && (int)grouped[im].size() >= gp::kMaxBatchSlots) ok = false;
        if (ok) {
            grouped[im].push_back(s);
            maxn = std::max(maxn, nsteps[s]);
        } else {
            // on its own handle, with its own plan
            int rc = steps_t<T>(h, psi[s], nsteps[s], im);
            if (rc) return bfail(b, rc, "slot " + std::to_string(s) + ": " + h->err);
            b->info.individual += 1;
        }
    }
    b->info.grouped = (int)(grouped[0].size() + grouped[1].size());
    for (int md = 0; md < 2; ++md) {
        const int im = md == 0 ? 1 : 0;  // info index is the ABI mode (0 imaginary)
        if (grouped[im].empty()) continue;
        b->info.x_points[md] = shape[im].K;
        b->info.x_block[md] = shape[im].block;
        b->info.y_tile[md] = (shape[im].chain ? shape[im].ytile : shape[im].tile) + 1;
        b->info.x_solver[md] = shape[im].chain ? GP_XSOLVER_CHAIN : GP_XSOLVER_SCAN;
        b->info.y_solver[md] = shape[im].chain ? GP_YSOLVER_STACK : GP_YSOLVER_WINDOW;
        b->info.x_tile[md] = shape[im].chain ? shape[im].xtile + 1 : 0;
    }
    // phases: the grouped condensates still running share each launch
    int64_t done = 0;
    while (done < maxn) {
        int64_t next = maxn;
        for (int im = 0; im < 2; ++im)
            for (int s : grouped[im])
                if (nsteps[s] > done) next = std::min(next, nsteps[s]);
        const int64_t c = next - done;
        // descriptors and block maps of this phase
        std::vector<unsigned char> img;
        struct GroupTables {
            size_t xs = 0, ys = 0, ns = 0, ss = 0, xm = 0, ym = 0, sm = 0;
            int nslot = 0, xblk = 0, yblk = 0, sblk = 0;
        } tb[2];
        for (int im = 0; im < 2; ++im) {
            if (shape[im].chain) {
                chain_tables<T>(b, grouped[im], psi, nsteps, done, im == 1, shape[im], img, tb[im].xs, tb[im].ys,
                                tb[im].ns, tb[im].ss, tb[im].xm, tb[im].ym, tb[im].sm, tb[im].nslot, tb[im].xblk,
                                tb[im].yblk, tb[im].sblk);
                continue;
            }
            std::vector<gp::XSlot<T>> xs;
            std::vector<gp::YSlot<T>> ys;
            std::vector<gp::NSlot> ns;
            std::vector<gp::SSlot<T>> ss;
            std::vector<unsigned> xm, ym, sm;
            const gp::YTile yt = gp::ytile<T>(shape[im].tile);
            for (int s : grouped[im]) {
                if (nsteps[s] <= done) continue;
                gp_spin1* h = b->slot[s];
                const ModeState& ms = h->mode[im];
                const unsigned id = (unsigned)xs.size();
                int G, R, hh, L;
                x_shape(h->p.nx, shape[im].K, G, R);
                R = std::max(1, std::min(8, shape[im].block / G));
                tile_window(h->p.ny, ms.hh, gp::ywindow(yt), hh, L);
                const int ncs = (h->p.nx + 4 * yt.NW - 1) / (4 * yt.NW);
                const int nyb = ncs * ((h->p.ny + L - 1) / L);
                const size_t n3 = (size_t)3 * h->p.nx * h->p.ny;
                const int nsb = (int)((n3 + gp::kScaleChunk - 1) / gp::kScaleChunk);
                xs.push_back(gp::XSlot<T>{(const C*)psi[s], (C*)h->d_work, phys(h->p), lineset<T>(ms.x), h->d_scale, G, R,
                                          h->psp, h->wsp});
                ys.push_back(gp::YSlot<T>{(const C*)h->d_work, (C*)psi[s], phys(h->p), lineset<T>(ms.y), h->d_part, L, hh, ncs,
                                          h->wsp, h->psp});
                ns.push_back(gp::NSlot{h->d_part, nyb, h->p.dx * h->p.dy, h->d_scale, h->d_flag, norm_rule(h->p)});
                ss.push_back(gp::SSlot<T>{(C*)psi[s], n3 / 3, h->psp, h->d_scale});
                for (int k = 0; k < (h->p.ny + R - 1) / R; ++k) xm.push_back((id << gp::kMapShift) | (unsigned)k);
                for (int k = 0; k < nyb; ++k) ym.push_back((id << gp::kMapShift) | (unsigned)k);
                for (int k = 0; k < nsb; ++k) sm.push_back((id << gp::kMapShift) | (unsigned)k);
            }
            tb[im].nslot = (int)xs.size();
            if (!tb[im].nslot) continue;
            if (tb[im].nslot > gp::kMaxBatchSlots) return bfail(b, GP_EUNSUPPORTED, "too many condensates in one launch");
            tb[im].xblk = (int)xm.size();
            tb[im].yblk = (int)ym.size();
            tb[im].sblk = (int)sm.size();
            tb[im].xs = stage_put(img, xs);
            tb[im].ys = stage_put(img, ys);
            tb[im].ns = stage_put(img, ns);
            tb[im].ss = stage_put(img, ss);
            tb[im].xm = stage_put(img, xm);
            tb[im].ym = stage_put(img, ym);
            tb[im].sm = stage_put(img, sm);
        }
        // upload through pinned staging (wait until the previous upload has left it)
        hipError_t e;
        if (b->staged_pending) {
            if ((e = hipEventSynchronize(b->staged)) != hipSuccess) return bhip(b, e, "batch staging");
            b->staged_pending = false;
        }
        if (img.size() > b->h_cap) {
            if (b->h_stage) (void)hipHostFree(b->h_stage);
            b->h_stage = nullptr;
            b->h_cap = 0;
            if ((e = hipHostMalloc(&b->h_stage, img.size())) != hipSuccess) return bhip(b, e, "batch staging");
            b->h_cap = img.size();
        }
        if (img.size() > b->d_cap) {
            // the stream may still read the old tables
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return bhip(b, e, "batch staging");
            if (b->d_stage) (void)hipFree(b->d_stage);
            b->d_stage = nullptr;
            b->d_cap = 0;
            if ((e = hipMalloc(&b->d_stage, img.size())) != hipSuccess) return bfail(b, GP_ENOMEM, "batch tables");
            b->d_cap = img.size();
        }
        std::memcpy(b->h_stage, img.data(), img.size());
        if ((e = hipMemcpyAsync(b->d_stage, b->h_stage, img.size(), hipMemcpyHostToDevice, st)) != hipSuccess)
            return bhip(b, e, "batch upload");
        if ((e = hipEventRecord(b->staged, st)) != hipSuccess) return bhip(b, e, "batch upload");
        b->staged_pending = true;
        auto at = [&](size_t off) { return (void*)((unsigned char*)b->d_stage + off); };
        // imaginary-time scales start at one
        if (tb[1].nslot &&
            (e = gp::launch_set_scale_batch((const gp::NSlot*)at(tb[1].ns), tb[1].nslot, 1.0, st)) != hipSuccess)
            return bhip(b, e, "batch set_scale");
        for (int64_t k = 0; k < c; ++k) {
            for (int im = 1; im >= 0; --im) {
                if (!tb[im].nslot) continue;
                const GroupTables& g = tb[im];
                if (shape[im].chain) {
                    if ((e = gp::launch_xc_batch<T>((const gp::XCSlot<T>*)at(g.xs), (const unsigned*)at(g.xm), g.xblk,
                                                    shape[im].xtile, im == 1, st)) != hipSuccess)
                        return bhip(b, e, "batch x sweep");
                    if ((e = gp::launch_ys_batch<T>((const gp::YSSlot<T>*)at(g.ys), (const unsigned*)at(g.ym), g.yblk,
                                                    shape[im].ytile, im == 1, st)) != hipSuccess)
                        return bhip(b, e, "batch y sweep");
                } else {
                    if ((e = gp::launch_x_batch<T>((const gp::XSlot<T>*)at(g.xs), (const unsigned*)at(g.xm), g.xblk,
                                                   shape[im].K, shape[im].block, im == 1, st)) != hipSuccess)
                        return bhip(b, e, "batch x sweep");
                    if ((e = gp::launch_y_batch<T>((const gp::YSlot<T>*)at(g.ys), (const unsigned*)at(g.ym), g.yblk,
                                                   shape[im].tile, im == 1, st)) != hipSuccess)
                        return bhip(b, e, "batch y sweep");
                }
                if (im == 1 && (e = gp::launch_norm_finalize_batch((const gp::NSlot*)at(g.ns), g.nslot, st)) != hipSuccess)
                    return bhip(b, e, "batch norm");
                b->info.launches += im == 1 ? 3 : 2;
            }
        }
        if (tb[1].nslot &&
            (e = gp::launch_scale_batch<T>((const gp::SSlot<T>*)at(tb[1].ss), (const unsigned*)at(tb[1].sm), tb[1].sblk,
                                           st)) != hipSuccess)
            return bhip(b, e, "batch scale");
        b->info.phases += 1;
        done = next;
    }
    return GP_OK;
}


// ---------------------------------------------------------------------------
// Serving: a trace of requests (arrival time, parameters, steps, mode, a
// device wave function each) replayed against the clock.  Requests are
// admitted in arrival order into the slots of one batch while a slot is free
// and the device-memory budget allows; every round advances all admitted
// condensates together by the steps left to the nearest completion (at most
// chunk_steps), so requests join and leave between rounds (continuous
// batching).
//
// The host keeps up to two rounds in flight on a stream of its own (one that
// does not wait for the null stream, so the table uploads of an admission run
// beside the rounds): while the GPU runs round r, the host admits arrivals
// and enqueues round r + 1.  The condensates that a round completes are known
// when it is enqueued (the step counts are), so their slots take new
// requests for the next round at once; their tables are released only when
// the GPU is idle (freeing device memory waits for the whole device) or at
// the end.  A request's completion time is read from the event recorded after
// its last round, and its latency runs from its arrival to that time.
// ---------------------------------------------------------------------------
// Device bytes a condensate holds while admitted: its wave function, the
// work copy and the per-line tables (pivots + coefficients, both directions).
size_t request_bytes(const gp_spin1_params& p) {
    const size_t s = p.precision == GP_FP64 ? 16 : 8;
    const size_t n = (size_t)p.nx * p.ny;
    const size_t state = (2 * psi_stride(p) + n) * s, work = (2 * work_stride(p) + n) * s;
    const size_t tables = (size_t)2 * 3 * ((size_t)p.nx + p.ny) * 72 * s;  // generous bound
    return state + work + tables + (1u << 16);
}

double seconds_since(const std::chrono::steady_clock::time_point& t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// A round in flight: its events and the requests it completes.
struct Round {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<int> finishing;   // request indices
    std::vector<gp_spin1*> dead;  // their slot handles (released later)
    double bytes = 0.0;           // their budget charge
};

// Everything the serving loop owns (released on every exit path).
struct ServeState {
    hipStream_t sst = nullptr;
    gp_spin1_batch* b = nullptr;
    std::vector<hipEvent_t> events;  // pool
    std::vector<Round> flight;       // rounds in flight, oldest first
    std::vector<gp_spin1*> graveyard;
    hipEvent_t origin = nullptr;
    ~ServeState() {
        if (sst) (void)hipStreamSynchronize(sst);
        for (Round& r : flight) {
            for (gp_spin1* h : r.dead) graveyard.push_back(h);
            if (r.e0) events.push_back(r.e0);
            if (r.e1) events.push_back(r.e1);
        }
        for (gp_spin1* h : graveyard) destroy_all(h);
        if (b) (void)gp_spin1_batch_destroy(b);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        if (origin) (void)hipEventDestroy(origin);
        if (sst) (void)hipStreamDestroy(sst);
    }
    hipError_t event(hipEvent_t* e) {
        if (!events.empty()) {
            *e = events.back();
            events.pop_back();
            return hipSuccess;
        }
        return hipEventCreate(e);
    }
};

int serve_run(const gp_spin1_request* req, int n, const gp_spin1_serve_config& cfg, hipStream_t st,
              gp_spin1_request_result* out, gp_spin1_serve_stats* stats, std::string& err) {
    const int prec = req[0].p.precision;
    for (int k = 0; k < n; ++k) {
        if (req[k].p.precision != prec) { err = "requests differ in precision"; return GP_EINVAL; }
        if (req[k].nsteps < 1 || (req[k].mode != 0 && req[k].mode != 1) || !req[k].psi_dev) {
            err = "request " + std::to_string(k) + ": nsteps < 1, bad mode or NULL psi";
            return GP_EINVAL;
        }
        if (k && req[k].arrival < req[k - 1].arrival) { err = "requests must be sorted by arrival"; return GP_EINVAL; }
        if ((double)request_bytes(req[k].p) > cfg.hbm_budget_bytes) {
            err = "request " + std::to_string(k) + " alone exceeds the memory budget";
            return GP_EINVAL;
        }
    }
    ServeState S;
    hipError_t e;
    auto hfail = [&](hipError_t x, const char* where) {
        err = std::string("serve: ") + where + ": " + hipGetErrorString(x);
        return GP_EHIP;
    };
    if ((e = hipStreamCreateWithFlags(&S.sst, hipStreamNonBlocking)) != hipSuccess) return hfail(e, "stream");
    // the rounds start after the caller's work on st (the wave functions' uploads)
    if ((e = S.event(&S.origin)) != hipSuccess) return hfail(e, "event");
    if ((e = hipEventRecord(S.origin, st)) != hipSuccess) return hfail(e, "event");
    if ((e = hipStreamWaitEvent(S.sst, S.origin, 0)) != hipSuccess) return hfail(e, "event");
    if ((e = hipEventSynchronize(S.origin)) != hipSuccess) return hfail(e, "event");
    const int ns = cfg.max_slots;
    std::vector<gp_spin1_params> empty(ns);
    for (auto& x : empty) { std::memset(&x, 0, sizeof x); x.precision = prec; }
    int rc = gp_spin1_batch_create(empty.data(), ns, (void*)S.sst, &S.b);
    if (rc) { err = "batch create failed"; return rc; }
    gp_spin1_batch* b = S.b;
    // the clock starts just before the origin event, which the idle stream
    // passes at once (so a GPU time after the origin never runs ahead of the
    // host clock: a request admitted after the host saw a round end starts
    // no earlier than that round's end)
    const auto t0 = std::chrono::steady_clock::now();
    if ((e = hipEventRecord(S.origin, S.sst)) != hipSuccess) return hfail(e, "event");
    if ((e = hipEventSynchronize(S.origin)) != hipSuccess) return hfail(e, "event");
    auto arrival = [&](int k) { return req[k].arrival * cfg.time_scale; };
    auto gpu_time = [&](hipEvent_t ev) {  // seconds after the origin, on the GPU's clock
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, S.origin, ev);
        return 1e-3 * ms;
    };
    std::vector<int> who(ns, -1);
    std::vector<int64_t> left(ns, 0);
    std::vector<void*> psi(ns, nullptr);
    std::vector<int64_t> nst(ns, 0);
    std::vector<int32_t> md(ns, 0);
    std::vector<uint8_t> on(ns, 0);
    std::vector<double> lat;
    lat.reserve(n);
    std::vector<Round>& flight = S.flight;
    double in_use = 0.0, dead_bytes = 0.0, active_sum = 0.0, pts = 0.0, busy = 0.0, admit_s = 0.0;
    int next = 0, done = 0, active = 0, max_active = 0, rounds = 0;
    const double dead_cap = std::max(1e9, 0.25 * cfg.hbm_budget_bytes);
    // retire the oldest round (waits for it)
    auto retire = [&]() -> int {
        Round& r = flight.front();
        if ((e = hipEventSynchronize(r.e1)) != hipSuccess) return hfail(e, "round");
        const double fin = gpu_time(r.e1);
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) busy += 1e-3 * ms;
        for (int k : r.finishing) {
            out[k].finish = fin;
            lat.push_back(fin - arrival(k));
            ++done;
        }
        in_use -= r.bytes;
        for (gp_spin1* h : r.dead) S.graveyard.push_back(h);
        S.events.push_back(r.e0);
        S.events.push_back(r.e1);
        flight.erase(flight.begin());
        return GP_OK;
    };
    // release the tables of finished requests (only when nothing is in flight)
    auto bury = [&]() {
        for (gp_spin1* h : S.graveyard) destroy_all(h);
        S.graveyard.clear();
        dead_bytes = 0.0;
    };
    while (done < n) {
        // rounds that have ended
        while (!flight.empty() && hipEventQuery(flight.front().e1) == hipSuccess)
            if ((rc = retire())) return rc;
        // admission, first come first served
        const auto ta = std::chrono::steady_clock::now();
        double now = seconds_since(t0);
        for (int sl = 0; sl < ns && next < n; ++sl) {
            if (who[sl] >= 0) continue;
            if (arrival(next) > now) break;
            const double need = (double)request_bytes(req[next].p);
            if (in_use + need > cfg.hbm_budget_bytes) break;
            gp_spin1* h = nullptr;
            rc = make_handle(&req[next].p, S.sst, &h);
            if (rc) { err = "request " + std::to_string(next) + ": invalid or unsupported parameters"; return rc; }
            b->slot[sl] = h;
            who[sl] = next;
            left[sl] = req[next].nsteps;
            psi[sl] = req[next].psi_dev;
            md[sl] = req[next].mode;
            out[next].start = now;
            in_use += need;
            ++active;
            ++next;
        }
        admit_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - ta).count();
        if (active == 0) {
            if (!flight.empty()) {
                if ((rc = retire())) return rc;
                continue;
            }
            // idle until the next arrival: a good time to release tables
            bury();
            if (next < n) {
                const double wait = arrival(next) - seconds_since(t0);
                if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
            }
            continue;
        }
        if (flight.size() >= 2) {
            if ((rc = retire())) return rc;
            continue;
        }
        if (dead_bytes > dead_cap) {
            // too much held for finished requests: drain and release
            while (!flight.empty())
                if ((rc = retire())) return rc;
            bury();
        }
        // enqueue the next round
        max_active = std::max(max_active, active);
        int64_t c = cfg.chunk_steps > 0 ? cfg.chunk_steps : INT64_MAX;
        for (int sl = 0; sl < ns; ++sl)
            if (who[sl] >= 0) c = std::min(c, left[sl]);
        for (int sl = 0; sl < ns; ++sl) {
            on[sl] = who[sl] >= 0;
            nst[sl] = on[sl] ? c : 0;
        }
        flight.emplace_back();
        Round& r = flight.back();
        if ((e = S.event(&r.e0)) != hipSuccess || (e = S.event(&r.e1)) != hipSuccess) return hfail(e, "event");
        if ((e = hipEventRecord(r.e0, S.sst)) != hipSuccess) return hfail(e, "event");
        rc = gp_spin1_batch_step(b, psi.data(), nst.data(), md.data(), on.data());
        if (rc) { err = b->err; return rc; }
        if ((e = hipEventRecord(r.e1, S.sst)) != hipSuccess) return hfail(e, "event");
        ++rounds;
        active_sum += active;
        for (int sl = 0; sl < ns; ++sl) {
            if (who[sl] < 0) continue;
            const int k = who[sl];
            pts += (double)c * req[k].p.nx * req[k].p.ny;
            left[sl] -= c;
            if (left[sl] > 0) continue;
            // done with this round: the slot takes a new request for the next one
            r.finishing.push_back(k);
            r.dead.push_back(b->slot[sl]);
            r.bytes += (double)request_bytes(req[k].p);
            dead_bytes += (double)request_bytes(req[k].p);
            b->slot[sl] = nullptr;
            who[sl] = -1;
            --active;
        }
    }
    while (!flight.empty())
        if ((rc = retire())) return rc;
    // (the batch's own stream is idle now)
    rc = gp_spin1_batch_sync(b);
    if (rc) { err = b->err; return rc; }
    // the caller's stream continues after the rounds
    if ((e = hipEventRecord(S.origin, S.sst)) != hipSuccess || (e = hipStreamWaitEvent(st, S.origin, 0)) != hipSuccess)
        return hfail(e, "event");
    const double wall = seconds_since(t0);
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double q) {
        if (lat.empty()) return 0.0;
        const double pos = q * (lat.size() - 1);
        const size_t i = (size_t)pos;
        const double f = pos - i;
        return i + 1 < lat.size() ? lat[i] * (1 - f) + lat[i + 1] * f : lat[i];
    };
    double offered = 0.0;
    for (int k = 0; k < n; ++k) offered += (double)req[k].nsteps * req[k].p.nx * req[k].p.ny;
    const double span = n > 1 ? arrival(n - 1) - arrival(0) : 0.0;
    std::memset(stats, 0, sizeof *stats);
    stats->wall_s = wall;
    stats->pt_steps = pts;
    stats->served_rate = wall > 0 ? pts / wall : 0.0;
    stats->offered_rate = span > 0 ? offered / span : 0.0;
    stats->p50_latency = pct(0.50);
    stats->p99_latency = pct(0.99);
    double sum = 0.0;
    for (double v : lat) sum += v;
    stats->mean_latency = lat.empty() ? 0.0 : sum / lat.size();
    stats->max_latency = lat.empty() ? 0.0 : lat.back();
    stats->completed = done;
    stats->max_active = max_active;
    stats->rounds = rounds;
    stats->mean_active = rounds ? active_sum / rounds : 0.0;
    stats->gpu_busy = wall > 0 ? busy / wall : 0.0;
    stats->admit_ms = 1e3 * admit_s;
    return GP_OK;
}

// No C++ exception leaves the library: a failed host allocation (tables,
// launch maps, messages) becomes GP_ENOMEM, anything else GP_EUNSUPPORTED.
// err: where the handle keeps its last message (nullable).
template <typename F>
int no_throw(F&& f, std::string* err = nullptr) noexcept {
    int rc;
    const char* what;
    try {
        return f();
    } catch (const std::bad_alloc&) {
        rc = GP_ENOMEM;
        what = "host allocation failed";
    } catch (const std::length_error&) {
        rc = GP_ENOMEM;
        what = "host allocation failed (size beyond a container's limit)";
    } catch (...) {
        rc = GP_EUNSUPPORTED;
        what = "unexpected C++ exception";
    }
    if (err) {
        try {
            *err = what;
        } catch (...) {
        }
    }
    return rc;
}

}  // namespace

extern "C" {

int gp_spin1_create(const gp_spin1_params* p, void* hip_stream, gp_spin1_t** out) {
    return no_throw([&]() -> int {
        return make_handle(p, (hipStream_t)hip_stream, out);
    });
}

int gp_spin1_step_static(const gp_spin1_params* p, void* psi, int64_t nsteps, int32_t mode, void* hip_stream) {
    std::string& err = static_err();
    err.clear();
    return no_throw([&]() -> int { return step_static(p, psi, nsteps, mode, (hipStream_t)hip_stream, &err); }, &err);
}

const char* gp_spin1_static_last_error(void) { return static_err().c_str(); }

int gp_spin1_destroy(gp_spin1_t* h) {
    if (!h) return GP_EINVAL;
    destroy_all(h);
    return GP_OK;
}

int gp_spin1_step_imag(gp_spin1_t* h, void* psi, int64_t nsteps) {
    return no_throw([&]() -> int {
        if (!h) return GP_EINVAL;
        if (!psi || nsteps < 0) return fail(h, GP_EINVAL, "psi is NULL or nsteps < 0");
        return h->p.precision == GP_FP64 ? steps_t<double>(h, psi, nsteps, true) : steps_t<float>(h, psi, nsteps, true);
    }, h ? &h->err : nullptr);
}

int gp_spin1_step_real(gp_spin1_t* h, void* psi, int64_t nsteps) {
    return no_throw([&]() -> int {
        if (!h) return GP_EINVAL;
        if (!psi || nsteps < 0) return fail(h, GP_EINVAL, "psi is NULL or nsteps < 0");
        return h->p.precision == GP_FP64 ? steps_t<double>(h, psi, nsteps, false) : steps_t<float>(h, psi, nsteps, false);
    }, h ? &h->err : nullptr);
}

int gp_spin1_step_graph(gp_spin1_t* h, void* psi, int64_t nsteps, int32_t mode) {
    return no_throw([&]() -> int {
        if (!h) return GP_EINVAL;
        if (!psi || nsteps < 0) return fail(h, GP_EINVAL, "psi is NULL or nsteps < 0");
        if (mode != 0 && mode != 1) return fail(h, GP_EINVAL, "mode must be 0 (imaginary time) or 1 (real time)");
        return h->p.precision == GP_FP64 ? graph_steps_t<double>(h, psi, nsteps, mode == 0)
                                         : graph_steps_t<float>(h, psi, nsteps, mode == 0);
    }, h ? &h->err : nullptr);
}

int gp_spin1_substep(gp_spin1_t* h, void* psi, int32_t which, int32_t imag) {
    return no_throw([&]() -> int {
        if (!h) return GP_EINVAL;
        if (!psi) return fail(h, GP_EINVAL, "psi is NULL");
        return h->p.precision == GP_FP64 ? substep_t<double>(h, psi, which, imag != 0)
                                         : substep_t<float>(h, psi, which, imag != 0);
    }, h ? &h->err : nullptr);
}

int gp_spin1_observables(gp_spin1_t* h, const void* psi, gp_spin1_obs* out, void* dens) {
    return no_throw([&]() -> int {
        if (!h) return GP_EINVAL;
        if (!psi || !out) return fail(h, GP_EINVAL, "psi or out is NULL");
        return h->p.precision == GP_FP64 ? obs_t<double>(h, psi, out, dens) : obs_t<float>(h, psi, out, dens);
    }, h ? &h->err : nullptr);
}

int gp_spin1_sync(gp_spin1_t* h) {
    return no_throw([&]() -> int {
        if (!h) return GP_EINVAL;
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "sync");
        int flag = 0;
        if ((e = hipMemcpy(&flag, h->d_flag, sizeof flag, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(h, e, "flag read");
        if (flag) {
            const int zero = 0;
            if ((e = hipMemcpy(h->d_flag, &zero, sizeof zero, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(h, e, "flag clear");
            return fail(h, GP_ENONFINITE, "an imaginary-time norm was not finite");
        }
        return GP_OK;
    }, h ? &h->err : nullptr);
}

int gp_spin1_get_plan(const gp_spin1_t* h, int32_t imag, gp_spin1_plan* out) {
    if (!h || !out) return GP_EINVAL;
    *out = h->mode[imag ? 1 : 0].plan;
    return GP_OK;
}

int gp_spin1_plan_query(const gp_spin1_params* p, int32_t imag, gp_spin1_plan* out) {
    return no_throw([&]() -> int {
        if (!out) return GP_EINVAL;
        std::string why;
        int rc = validate(p, why);
        if (rc) return rc;
        gp_spin1_params q = *p;
        if (std::isnan(q.x0)) q.x0 = -0.5 * q.nx * q.dx;
        if (std::isnan(q.y0)) q.y0 = -0.5 * q.ny * q.dy;
        HostMode hm;
        ModeState ms;
        if (q.precision == GP_FP64) {
            host_mode<double>(q, imag != 0, hm);
            copy_plan<double>(q, hm, ms);
        } else {
            host_mode<float>(q, imag != 0, hm);
            copy_plan<float>(q, hm, ms);
        }
        *out = ms.plan;
        return GP_OK;
    });
}

int gp_spin1_timing_enable(gp_spin1_t* h, int32_t enable) {
    return no_throw([&]() -> int {
        if (!h) return GP_EINVAL;
        hipError_t e = timing_drain(h);
        if (e != hipSuccess) return hip_fail(h, e, "timing");
        h->timing = enable != 0;
        for (int k = 0; k < 4; ++k) { h->t_launches[k] = 0; h->t_ms[k] = 0.0; }
        return GP_OK;
    }, h ? &h->err : nullptr);
}

int gp_spin1_timing_read(gp_spin1_t* h, gp_spin1_timing* out) {
    return no_throw([&]() -> int {
        if (!h || !out) return GP_EINVAL;
        hipError_t e = timing_drain(h);
        if (e != hipSuccess) return hip_fail(h, e, "timing");
        for (int k = 0; k < 4; ++k) { out->launches[k] = h->t_launches[k]; out->ms[k] = h->t_ms[k]; }
        return GP_OK;
    }, h ? &h->err : nullptr);
}

const char* gp_spin1_strerror(int status) {
    switch (status) {
        case GP_OK: return "success";
        case GP_EINVAL: return "invalid argument";
        case GP_EUNSTABLE: return "parameters fail the stability checks for this propagation";
        case GP_ENOMEM: return "allocation failed (device or host memory)";
        case GP_EHIP: return "HIP runtime error";
        case GP_ENONFINITE: return "non-finite value";
        case GP_EUNSUPPORTED: return "unsupported size or option";
        default: return "unknown status";
    }
}

const char* gp_spin1_last_error(const gp_spin1_t* h) {
    if (!h) return "";
    return h->err.c_str();
}


int gp_spin1_batch_create(const gp_spin1_params* p, int32_t n, void* hip_stream, gp_spin1_batch_t** out) {
    return no_throw([&]() -> int {
        if (!out || !p || n < 1 || n > 65536) return GP_EINVAL;
        for (int s = 1; s < n; ++s)
            if (p[s].precision != p[0].precision) return GP_EINVAL;
        if (p[0].precision != GP_FP64 && p[0].precision != GP_FP32) return GP_EINVAL;
        gp_spin1_batch* b = new (std::nothrow) gp_spin1_batch();
        if (!b) return GP_ENOMEM;
        b->n = n;
        b->precision = p[0].precision;
        b->stream = (hipStream_t)hip_stream;
        b->slot.assign(n, nullptr);
        if (hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) { batch_free(b); return GP_EHIP; }
        try {
            for (int s = 0; s < n; ++s) {
                if (p[s].nx == 0) continue;  // empty slot
                int rc = make_handle(&p[s], b->stream, &b->slot[s]);
                if (rc) { batch_free(b); return rc; }
            }
        } catch (...) {
            batch_free(b);
            throw;
        }
        *out = b;
        return GP_OK;
    });
}

int gp_spin1_batch_set_slot(gp_spin1_batch_t* b, int32_t slot, const gp_spin1_params* p) {
    return no_throw([&]() -> int {
        if (!b) return GP_EINVAL;
        if (slot < 0 || slot >= b->n) return bfail(b, GP_EINVAL, "slot out of range");
        if (p && p->nx != 0 && p->precision != b->precision) return bfail(b, GP_EINVAL, "precision differs from the batch");
        gp_spin1* h = nullptr;
        if (p && p->nx != 0) {
            int rc = make_handle(p, b->stream, &h);
            if (rc) return bfail(b, rc, "slot " + std::to_string(slot) + ": invalid or unsupported parameters");
        }
        if (b->slot[slot]) {
            // the stream may still use the old slot's tables
            hipError_t e = hipStreamSynchronize(b->stream);
            if (e != hipSuccess) {
                if (h) destroy_all(h);
                return bhip(b, e, "set_slot");
            }
            destroy_all(b->slot[slot]);
        }
        b->slot[slot] = h;
        return GP_OK;
    }, b ? &b->err : nullptr);
}

int gp_spin1_batch_step(gp_spin1_batch_t* b, void* const* psi_dev, const int64_t* nsteps, const int32_t* mode,
                        const uint8_t* active) {
    return no_throw([&]() -> int {
        if (!b) return GP_EINVAL;
        if (!psi_dev || !nsteps || !mode) return bfail(b, GP_EINVAL, "psi_dev, nsteps and mode are required");
        return b->precision == GP_FP64 ? batch_step_t<double>(b, psi_dev, nsteps, mode, active)
                                       : batch_step_t<float>(b, psi_dev, nsteps, mode, active);
    }, b ? &b->err : nullptr);
}

int gp_spin1_batch_sync(gp_spin1_batch_t* b) {
    return no_throw([&]() -> int {
        if (!b) return GP_EINVAL;
        hipError_t e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return bhip(b, e, "sync");
        for (int s = 0; s < b->n; ++s) {
            if (!b->slot[s]) continue;
            int rc = gp_spin1_sync(b->slot[s]);
            if (rc) return bfail(b, rc, "slot " + std::to_string(s) + ": " + b->slot[s]->err);
        }
        return GP_OK;
    }, b ? &b->err : nullptr);
}

int gp_spin1_batch_observables(gp_spin1_batch_t* b, int32_t slot, const void* psi, gp_spin1_obs* out, void* dens) {
    return no_throw([&]() -> int {
        if (!b) return GP_EINVAL;
        if (slot < 0 || slot >= b->n || !b->slot[slot]) return bfail(b, GP_EINVAL, "slot out of range or empty");
        int rc = gp_spin1_observables(b->slot[slot], psi, out, dens);
        if (rc) return bfail(b, rc, "slot " + std::to_string(slot) + ": " + b->slot[slot]->err);
        return GP_OK;
    }, b ? &b->err : nullptr);
}

int gp_spin1_batch_info_read(const gp_spin1_batch_t* b, gp_spin1_batch_info* out) {
    if (!b || !out) return GP_EINVAL;
    *out = b->info;
    return GP_OK;
}

int gp_spin1_batch_destroy(gp_spin1_batch_t* b) {
    if (!b) return GP_EINVAL;
    (void)hipStreamSynchronize(b->stream);
    batch_free(b);
    return GP_OK;
}

const char* gp_spin1_batch_last_error(const gp_spin1_batch_t* b) {
    return b ? b->err.c_str() : "null batch";
}


int gp_spin1_serve(const gp_spin1_request* req, int32_t n, const gp_spin1_serve_config* cfg, void* hip_stream,
                   gp_spin1_request_result* out, gp_spin1_serve_stats* stats) {
    return no_throw([&]() -> int {
        if (!req || n < 1 || !cfg || !out || !stats) return GP_EINVAL;
        if (cfg->max_slots < 1 || cfg->max_slots > gp::kMaxBatchSlots || !(cfg->hbm_budget_bytes > 0) ||
            !(cfg->time_scale >= 0) || cfg->chunk_steps < 0)
            return GP_EINVAL;
        for (int k = 0; k < n; ++k) out[k].start = out[k].finish = -1.0;
        std::string err;
        const int rc = serve_run(req, n, *cfg, (hipStream_t)hip_stream, out, stats, err);
        if (rc) std::fprintf(stderr, "gp_spin1_serve: %s\n", err.c_str());
        return rc;
    });
}

}  // extern "C"
