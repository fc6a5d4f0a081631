// Launch interface between the host runtime and the gfx950 kernels.
#pragma once

#include "gp_device.hpp"

namespace gp {

constexpr int kObsCount = 13;

// Tile geometry of the windowed y sweep per precision: TW columns (a
// contiguous run of each row) x S segments of KY rows per thread; a window
// spans S * KY = 128 rows.
template <typename T> struct YCfg;
template <> struct YCfg<double> { static constexpr int KY = 4, TW = 16, S = 32; };
template <> struct YCfg<float> { static constexpr int KY = 8, TW = 32, S = 16; };

// Both sweeps run out of place (src -> dst): the y windows overlap, so a
// window's halo rows must not be rewritten by its neighbour while it reads.
// Where the y sweep leaves the imaginary-time norm: per-block partial sums,
// a ticket counter (zero between launches), the resulting scale factor and the
// non-finite flag.
struct NormOut {
    double* partials;
    unsigned int* ticket;
    double* scale;
    int* flag;
    double dxdy;
};

template <typename T> struct XLaunch {
    const cx<T>* src;
    cx<T>* dst;
    Phys ph;
    LineSet<T> ls;
    const double* scale;
    int K, G, R;
    bool imag, local;
};

template <typename T> struct YLaunch {
    const cx<T>* src;
    cx<T>* dst;
    Phys ph;
    LineSet<T> ls;
    NormOut no;
    int L, h;
    bool window, imag, norm;
};

struct ObsLaunch {
    double c0, c2, rabi, gamma, omega;
    int eta;
};

template <typename T> hipError_t launch_x(const XLaunch<T>& a, hipStream_t st);
template <typename T> hipError_t launch_y(const YLaunch<T>& a, hipStream_t st);
template <typename T> int y_blocks(const YLaunch<T>& a);
template <typename T> hipError_t launch_local(cx<T>* psi, const Phys& ph, bool imag, hipStream_t st);
template <typename T> hipError_t launch_scale(cx<T>* psi, size_t n, const double* scale, hipStream_t st);
template <typename T>
hipError_t launch_norm_partials(const cx<T>* psi, size_t n, double* partials, int nblk, hipStream_t st);
hipError_t launch_set_scale(double* scale, double v, hipStream_t st);
hipError_t launch_norm_finalize(const double* partials, int n, double dxdy, double* scale, int* flag, hipStream_t st);
template <typename T>
hipError_t launch_obs(const cx<T>* psi, const Phys& ph, const ObsLaunch& o, T* dens, double* partials, int nblk,
                      hipStream_t st);
hipError_t launch_obs_finalize(const double* partials, int nblk, double* out, hipStream_t st);

}  // namespace gp
