/*
 * gp_spin1.h -- C ABI of the MI355X (gfx950) split-step Crank-Nicolson (SSCN)
 * solver for the quasi-2D rotating spin-1 Gross-Pitaevskii equation with
 * Rashba or Dresselhaus spin-orbit (SO) coupling and Rabi coupling.
 *
 * The equations are Eqs. (S.1)-(S.3) of the Supplementary Material of
 * arXiv:2105.10517 (Muruganandam, Balaz, Adhikari):
 *   i d_t psi_{+-1} = [H + c2 (rho_{+-1} - rho_{-+1} + rho_0)] psi_{+-1}
 *                     + c2 psi_0^2 psi_{-+1}^* + R/sqrt2 psi_0 + gamma f_{+-1}
 *   i d_t psi_0     = [H + c2 (rho_{+1} + rho_{-1})] psi_0
 *                     + 2 c2 psi_{+1} psi_{-1} psi_0^* + R/sqrt2 (psi_{+1} + psi_{-1}) + gamma f_0
 *   H = -1/2 grad^2 + V + c0 rho - Omega L_z,   V = (x^2 + y^2)/2,
 *   gamma f = gamma (eta p_y Sigma_x - p_x Sigma_y)   (eta = +1 Rashba, -1 Dresselhaus),
 * with Sigma_x, Sigma_y the spin-1 matrices of Eq. (S.5), lengths in l0, time
 * in 1/omega.  The paper's solution method is the SSCN scheme in imaginary time
 * (stationary states) and in real time (dynamics).
 *
 * One time step (Lie splitting) is
 *   1. local substep   psi <- exp(-i dt H_loc) psi      (real time)
 *                      psi <- exp(-dt H_loc) psi        (imaginary time)
 *      H_loc = (V + c0 rho) I + c2 F.Sigma + R Sigma_x, F = psi^+ Sigma psi,
 *      frozen at the substep input;
 *   2. x sweep  (I + a H_x) psi' = (I - a H_x) psi,  H_x = -1/2 d_x^2 - i Omega y d_x + i gamma Sigma_y d_x;
 *   3. y sweep  (I + a H_y) psi' = (I - a H_y) psi,  H_y = -1/2 d_y^2 + i Omega x d_y - i eta gamma Sigma_x d_y;
 *   4. imaginary time only: psi <- psi / sqrt(dx dy sum |psi|^2)
 *      (normalisation condition stated after Eq. (S.5));
 * with a = i dt/2 in real time and a = dt/2 in imaginary time, 3-point
 * second differences, central first differences and psi = 0 on the ghost
 * points just outside the grid.
 *
 * Wave-function layout (every entry point): psi[3][ny][nx], x fastest, the
 * component planes plane_stride elements apart (nx ny, i.e. C-contiguous,
 * unless the parameters set a larger stride), components ordered m = +1, 0, -1, interleaved complex
 * (complex128 for GP_FP64, complex64 for GP_FP32).  Grid: x_i = x0 + i dx,
 * y_j = y0 + j dy.  psi lives in caller-owned device memory; the library
 * borrows it for the duration of a call and never frees it.
 *
 * Status: every function returns a gp_status (0 = success).  No exception
 * crosses this boundary.  A handle is not thread-safe: use one handle per
 * stream.  Device work is enqueued on the stream given at creation; the step
 * and substep calls return without waiting, gp_spin1_observables and
 * gp_spin1_sync wait for the stream.
 */
#ifndef GP_SPIN1_H
#define GP_SPIN1_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GP_OK = 0,
    GP_EINVAL = -1,        /* bad argument: non-finite value, n < 3, d <= 0, dt <= 0, |eta| != 1, NULL */
    GP_EUNSTABLE = -2,     /* the requested propagation fails the create-time stability checks */
    GP_ENOMEM = -3,        /* a device or host allocation failed */
    GP_EHIP = -4,          /* a HIP runtime call failed; gp_spin1_last_error has the message */
    GP_ENONFINITE = -5,    /* a NaN or Inf was met in a norm or an observable */
    GP_EUNSUPPORTED = -6   /* a size or option the library does not handle  */
} gp_status;

typedef enum { GP_FP64 = 0, GP_FP32 = 1 } gp_precision; /* FP32: bulk in FP32, reductions in FP64 */

/* Choice of the y-sweep line solver. */
typedef enum {
    GP_YSOLVER_AUTO = 0,   /* grids of 1024^2 points and up: stacked chain windows when a tile fits;
                              otherwise the windowed scan when its truncation bound holds, else
                              per-column Thomas (autotuning may choose any of them)                */
    GP_YSOLVER_WINDOW = 1, /* windowed partitioned scan over column tiles (2 HBM passes per step) */
    GP_YSOLVER_THOMAS = 2, /* exact per-thread Thomas down whole columns (one thread per column) */
    GP_YSOLVER_CHAIN = 3,  /* windows as GP_YSOLVER_WINDOW, each segment's carry formed from the ceil((h - 1) / K)
                              segments before and after it instead of a scan of the whole window (their
                              carries are attenuated below the same rounding bound as the window ends);
                              y_tile then names a chain tile */
    GP_YSOLVER_STACK = 4   /* chain windows with 16 consecutive columns per block and the window's segments
                              stacked over its waves (carries through shared memory); y_tile 1..4 with
                              16 segments per window, 5..6 with 32                                      */
} gp_ysolver;

/* Choice of the x-sweep line solver. */
typedef enum {
    GP_XSOLVER_AUTO = 0,   /* whole-row partitioned Thomas, or the windows when autotuning finds them faster;
                              grids of 1024^2 points and up, and rows above 4096 points, take the chain
                              windows when a chain tile fits (FP64: two points per lane while a window
                              writes at least 3/4 of what it loads, else four; FP32: four)               */
    GP_XSOLVER_SCAN = 1,   /* exact partitioned Thomas over whole rows (scans across the row's threads)     */
    GP_XSOLVER_WINDOW = 2, /* truncated overlapping windows along the rows (the y sweep's scheme); refused
                              (GP_EUNSUPPORTED) when the decay bound does not fit any window            */
    GP_XSOLVER_CHAIN = 3   /* windows of one row segment per wave (64 K points) with carries over ceil((h - 1) / K)
                              lanes (as GP_YSOLVER_CHAIN); x_tile then names a chain tile               */
} gp_xsolver;

/* Block order of the windowed sweeps.  The chip hands workgroups to its 8
 * XCDs (each with its own L2) in turn; grouping gives each XCD a contiguous
 * run of windows instead, so that overlapping halos are read through one L2. */
typedef enum {
    GP_ORDER_AUTO = 0,     /* x windows grouped, y windows grouped only on grids of about one wave of blocks;
                              with autotune, both timed and the faster kept per sweep                       */
    GP_ORDER_HARDWARE = 1, /* block b processes window b                                                    */
    GP_ORDER_XCD = 2,      /* block b processes window (b mod 8) ceil(n/8) + b div 8 (n windows)            */
    GP_ORDER_BANDS = 3,    /* y windows: XCD x takes a contiguous range of column strips and walks them down
                              8 strips at a time (windows above and below each other in flight together);
                              x windows as GP_ORDER_XCD                                                    */
    GP_ORDER_ROWS = 4      /* row bands for small grids: XCD x owns the y row tiles [x nrt/8, (x+1) nrt/8)
                              (nrt row tiles) in both sweeps - their y windows and the x rows they cover -
                              so that each sweep reads from its own L2 what the other wrote; needs y
                              windows (else x windows as GP_ORDER_XCD, whole rows in hardware order)    */
} gp_block_order;

/* Order of the substeps within one step. */
typedef enum {
    GP_SPLIT_LIE = 0,    /* local substep (dt), x sweep, y sweep: the order the paper's scheme name implies */
    GP_SPLIT_STRANG = 1  /* local substep (dt/2), x sweep, y sweep, local substep (dt/2): symmetric in the
                            local / linear split (second order in dt where the sweeps commute, i.e.
                            Omega = gamma = 0, and the frozen local exponential is exact) */
} gp_split;

typedef struct {
    int32_t nx, ny;    /* grid points, each >= 3; nx <= 8192 (one row is held on chip)        */
    double dx, dy;     /* grid steps, > 0 (lengths in l0)                                      */
    double x0, y0;     /* coordinate of index 0; NaN selects the default -n*d/2                */
    double dt;         /* time step, > 0 (same meaning in imaginary and real time)             */
    double c0, c2;     /* density and spin-exchange couplings of Eq. (S.4)                     */
    double gamma;      /* SO strength gamma                                                    */
    int32_t eta;       /* +1 Rashba, -1 Dresselhaus (term gamma (eta p_y Sigma_x - p_x Sigma_y)) */
    double rabi;       /* Rabi coupling R                                                      */
    double omega;      /* rotation frequency Omega (in units of the trap frequency)            */
    int32_t precision; /* gp_precision                                                         */
    int32_t y_solver;  /* gp_ysolver                                                           */
    int32_t x_points;  /* points per thread of the x sweep: 0 = chosen by the library, else 1, 2, 4, 8 or 16 */
    int32_t y_tile;    /* tile shape of the windowed y sweep: 0 = chosen by the library, else 1..8            */
    int32_t autotune;  /* != 0: time the candidate x and y launch shapes at creation and keep the fastest
                          (only for the fields left at 0); the choice depends on the grid shape only        */
    double trap_gx, trap_gy; /* trap V = (gx^2 x^2 + gy^2 y^2)/2 (Eq. (S.3) with the harmonic trap, optionally
                                anisotropic); 0 selects 1, the paper's isotropic trap                        */
    int32_t split;           /* gp_split                                                                   */
    int32_t fix_magnetization; /* imaginary time: != 0 renormalises to total norm 1 AND magnetisation
                                  N_{+1} - N_{-1} = magnetization (the two conditions stated after Eq. (S.5)),
                                  with the third condition s_{+1} s_{-1} = s_0^2 on the component scale
                                  factors of the normalised gradient flow (Bao and Lim, SIAM J. Sci.
                                  Comput. 30, 2008); needs gamma = rabi = 0 and |magnetization| < 1     */
    double magnetization;
    int32_t x_solver;        /* gp_xsolver                                                                  */
    int32_t block_order;     /* gp_block_order: how the windowed sweeps number their blocks (no effect on
                                results, which are bit-identical in every order)                         */
    int32_t x_tile;          /* tile shape of the windowed x sweep: 0 = chosen by the library, else 1..8
                                (the y_tile shapes turned along the rows; chain tiles with
                                GP_XSOLVER_CHAIN)                                                        */
    int64_t plane_stride;    /* elements between the component planes of every wave function passed to this
                                handle (psi_m starts at psi + m plane_stride; rows nx apart, points
                                contiguous); 0 = nx ny (a contiguous [3][ny][nx] array).  A stride that is
                                not a power of two apart (e.g. nx ny + 4160) keeps the sweeps' three
                                streams off the same HBM channels; the gaps are never read or written  */
} gp_spin1_params;

/* Observables of one wave function (all FP64, rectangle-rule quadrature
 * dx dy sum):
 *   norm[m] = int rho_m, norm_total, magnetization = norm[+1] - norm[-1]
 *   (conditions after Eq. (S.5));
 *   energy = e_kin + e_trap + e_int + e_rot + e_so + e_rabi, the terms of the
 *   Eq. (S.6) functional (e_kin from forward differences over the ghost-padded
 *   grid, i.e. <psi| -grad^2/2 |psi>; e_int = 1/2 int (c0 rho^2 + c2 |F|^2));
 *   lz = <L_z> summed over components;
 *   mu[m] = Re <psi_m | (H psi)_m> / norm[m] with (H psi) the right-hand sides
 *   of Eqs. (S.1)-(S.2) (0 for a component whose norm is exactly 0),
 *   mu_total = sum_m Re <psi_m|(H psi)_m> / norm_total. */
typedef struct {
    double norm[3], norm_total, magnetization;
    double energy, e_kin, e_trap, e_int, e_rot, e_so, e_rabi, lz;
    double mu[3], mu_total;
} gp_spin1_obs;

/* What gp_spin1_create chose for one propagation mode (introspection). */
typedef struct {
    int32_t x_points_per_thread; /* K of the x kernel: each thread holds K consecutive points   */
    int32_t x_threads_per_row;   /* threads cooperating on one row                               */
    int32_t x_rows_per_block;
    int32_t y_solver;            /* GP_YSOLVER_WINDOW, _CHAIN, _STACK or _THOMAS                  */
    int32_t y_halo;              /* rows read above a y window's output (at least as many below) */
    int32_t y_rows_out;          /* rows written per y window                                    */
    int32_t y_tile;              /* 1..8, the tile shape below (5..8: lines solved one at a time)  */
    int32_t y_tile_cols;         /* columns per y block (4 per wave; 16 for stacked windows)      */
    int32_t y_segments;          /* segments per column and window (16: one DPP row of lanes;
                                    stacked windows 16 or 32)                                     */
    int32_t y_rows_per_thread;   /* a window spans y_segments * y_rows_per_thread rows            */
    int32_t pivots_x, pivots_y;  /* tabulated Thomas pivots per line before the constant limit  */
    double decay_x, decay_y;     /* largest |a m| or |c'| of the converged pivots per direction  */
    int32_t stable;              /* 1 if the mode passed the stability checks                    */
    int32_t x_solver;            /* GP_XSOLVER_SCAN, GP_XSOLVER_WINDOW or GP_XSOLVER_CHAIN        */
    int32_t x_halo;              /* windows: points of overlap on each side                       */
    int32_t x_points_out;        /* windows: points written per window                            */
    int32_t x_tile;              /* windows: 1..8, same shapes as y_tile (rows per block = 4 per wave) */
    int32_t x_block_order;       /* 0 blocks in hardware order, 1 XCD-contiguous windows (each of   */
    int32_t y_block_order;       /*   the 8 XCDs a contiguous run), 2 bands (y), 3 row bands        */
} gp_spin1_plan;

typedef struct gp_spin1 gp_spin1_t;

/* Create a solver handle.  p is copied.  hip_stream is a hipStream_t (NULL =
 * the default stream).  Validates p (GP_EINVAL), tabulates the Thomas pivots
 * of every x line (row j, Sigma_y eigenvalue) and y line (column i, Sigma_x
 * eigenvalue) for both propagation modes, and allocates small device tables
 * and reduction scratch.  GP_EUNSTABLE when the line systems of real time
 * are not diagonally dominant (then neither propagation can run); parameters
 * that fail only the imaginary-time bound give a handle whose
 * gp_spin1_step_imag returns GP_EUNSTABLE.  *out is set only on success. */
int gp_spin1_create(const gp_spin1_params* p, void* hip_stream, gp_spin1_t** out);
int gp_spin1_destroy(gp_spin1_t* h);

/* nsteps >= 0 imaginary-time SSCN steps on psi (device), renormalised to unit
 * norm after each step.  GP_EUNSTABLE if the imaginary-time Cayley bound
 * (dt/4)(|Omega| L_max + |gamma|)^2 < 1 or the diagonal dominance of the line
 * systems fails.  Asynchronous; a non-finite norm is reported by the next
 * gp_spin1_sync or gp_spin1_observables as GP_ENONFINITE. */
int gp_spin1_step_imag(gp_spin1_t* h, void* psi_dev, int64_t nsteps);

/* nsteps >= 0 real-time SSCN steps on psi (device); no renormalisation.
 * GP_EUNSTABLE if the line systems lose diagonal dominance.  Asynchronous. */
int gp_spin1_step_real(gp_spin1_t* h, void* psi_dev, int64_t nsteps);

/* nsteps steps in mode 0 (imaginary time, as gp_spin1_step_imag) or 1 (real
 * time, as gp_spin1_step_real), replayed from a HIP graph: the launch
 * sequence of nsteps steps on psi_dev is captured once (on a stream of the
 * handle's own; it holds kernels only) and kept per (psi_dev, nsteps, mode),
 * up to 8 per handle (the oldest is dropped, after a wait for the stream);
 * every call then launches the graph on the handle's stream.  Results equal
 * those of gp_spin1_step_imag / step_real bit for bit.  For runs of many
 * short steps, where the host's launch cost could leave the GPU idle.
 * Per-kernel timing (gp_spin1_timing_enable) does not see
 * the kernels of a graph.  The captured sequence holds psi_dev's address: a
 * graph must not outlive the wave function it was captured on (free it with
 * the handle, or call with other arguments).  Asynchronous. */
int gp_spin1_step_graph(gp_spin1_t* h, void* psi_dev, int64_t nsteps, int32_t mode);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): nsteps SSCN steps of
 * psi_dev (caller-owned, layout as for gp_spin1_create) in imaginary time
 * (mode 0, renormalised each step) or real time (mode 1), with the launch
 * plan gp_spin1_create picks without autotuning, computed exactly as by a
 * handle with the same parameters.  No handle: the line tables, the work wave
 * function, the norm partials and the scale factors live in a static device
 * array of GP_STATIC_SCRATCH_BYTES per GPU (held until the process ends; the
 * grid must fit it: the work wave function takes (3 nx ny + 8320) s bytes,
 * s = 16 or 8, so up to about 690 thousand points in FP64 and 1.38 million
 * in FP32).  No device memory is allocated or freed; the tables are built on
 * the host and copied on hip_stream.  Blocks until the steps are done.
 * Every call on one GPU uses the same array: calls that overlap on one GPU
 * (several host threads, or several streams) race and must not be issued.
 * Returns GP_EINVAL for invalid parameters, autotune != 0, a NULL psi_dev,
 * nsteps < 0 or a bad mode; GP_ENOMEM when the grid exceeds the array
 * (message from gp_spin1_static_last_error); GP_EUNSTABLE and GP_ENONFINITE
 * as the handle calls. */
#define GP_STATIC_SCRATCH_BYTES ((size_t)32 << 20)
int gp_spin1_step_static(const gp_spin1_params* p, void* psi_dev, int64_t nsteps, int32_t mode, void* hip_stream);
/* Message of the calling thread's last failed gp_spin1_step_static ("" after success). */
const char* gp_spin1_static_last_error(void);

/* One substep alone (diagnostics and per-kernel parity checks):
 * which = 0 local substep, 1 x sweep, 2 y sweep, 3 renormalise to unit norm;
 * imag != 0 selects the imaginary-time form.  Asynchronous. */
int gp_spin1_substep(gp_spin1_t* h, void* psi_dev, int32_t which, int32_t imag);

/* Observables of psi (device).  Blocks until out_host is written.  If dens_dev
 * is not NULL it receives rho_m = |psi_m|^2 as a real [3][ny][nx] array of the
 * handle's precision (device).  GP_ENONFINITE if any sum is not finite. */
int gp_spin1_observables(gp_spin1_t* h, const void* psi_dev, gp_spin1_obs* out_host, void* dens_dev);

/* Wait for the handle's stream; returns GP_ENONFINITE if an imaginary-time
 * norm was not finite since the last check (and clears the flag). */
int gp_spin1_sync(gp_spin1_t* h);

/* Plan chosen for imag != 0 (imaginary time) or imag == 0 (real time). */
int gp_spin1_get_plan(const gp_spin1_t* h, int32_t imag, gp_spin1_plan* out);

/* The same plan computed on the host alone, without a handle or any device
 * call: validates p (GP_EINVAL / GP_EUNSUPPORTED as gp_spin1_create) and
 * reports the pivot tables, decay factors, y solver and stability flag that
 * gp_spin1_create would choose. */
int gp_spin1_plan_query(const gp_spin1_params* p, int32_t imag, gp_spin1_plan* out);

/* Per-kernel timing (diagnostics).  While enabled, the step calls bracket
 * every kernel launch with a HIP event pair on the handle's stream; gp_spin1_timing_read
 * waits for the stream and returns, per kernel kind, the number of launches
 * and their summed duration in milliseconds since the last enable (which
 * resets the counters).  Kinds: 0 x sweep (with the fused local substep and
 * the pending renormalisation), 1 y sweep (with the fused norm partial sums),
 * 2 imaginary-time norm total (one block, after each y sweep), 3 final
 * renormalisation at the end of an imaginary-time call.  The events are
 * stamped by the kernel dispatches themselves (kernel durations only). */
typedef struct {
    int64_t launches[4];
    double ms[4];
} gp_spin1_timing;
int gp_spin1_timing_enable(gp_spin1_t* h, int32_t enable);
int gp_spin1_timing_read(gp_spin1_t* h, gp_spin1_timing* out);

const char* gp_spin1_strerror(int status);
const char* gp_spin1_last_error(const gp_spin1_t* h); /* per-handle message of the last failure */

/* ---------------------------------------------------------------------------
 * Batches of independent condensates.  The paper's workflows run many
 * separate SSCN solutions (parameter scans of Omega, couplings and SO type,
 * imaginary- then real-time runs, Sec. "Numerical results" of the
 * Supplementary Material); a batch advances such condensates together, each
 * with its own grid, spacings, time step, couplings and propagation mode, in
 * one kernel launch per sweep over the rows and column tiles of all of them.
 * Each condensate follows exactly the step of gp_spin1_step_imag /
 * gp_spin1_step_real; results equal those of a single handle created with
 * the batch's launch shape (gp_spin1_batch_info: x_solver and x_tile or
 * x_points, y_solver and y_tile) to the last bit or two.
 *
 * Launch shape per propagation mode: chain x windows and stacked chain y
 * windows when every condensate of that mode that can be grouped (Lie
 * splitting) leaves x_solver / y_solver at AUTO (or asks for CHAIN / STACK)
 * and fits one chain tile and one stacked tile (those with the fewest
 * lane-points over the group); otherwise whole-row scans and scanned windows.
 *
 * gp_spin1_batch_create: p is an array of n parameter sets (1 <= n <= 65536),
 *   one per slot; an entry with nx == 0 leaves its slot empty.  Every entry carries
 *   the same precision.  Each slot owns the tables and scratch of a single
 *   handle (allocated here, freed by set_slot / destroy).  Work runs on
 *   hip_stream.  GP_EINVAL / GP_EUNSUPPORTED as gp_spin1_create.
 * gp_spin1_batch_set_slot: replaces the condensate of one slot (admission of a
 *   new request); p == NULL or p->nx == 0 empties it.  Waits for the stream
 *   when it frees the old slot's tables.
 * gp_spin1_batch_step: psi_dev[s] is the device wave function of slot s in
 *   the layout above (complex128 / complex64 by the batch precision);
 *   nsteps[s] >= 0 steps in mode[s] (0 imaginary time, renormalised every
 *   step; 1 real time); active (nullable) masks slots out.  Slots with
 *   Strang splitting, whose windows do not fit the batch tiles, that need
 *   more than 2^20 blocks in a sweep, or beyond the first 4096 of one mode,
 *   run on their own, on the same stream.  Asynchronous like gp_spin1_step_*; psi_dev arrays may be
 *   reused as soon as the call returns.  Calls that overlap on one batch are
 *   not allowed (a batch is not thread-safe).
 * gp_spin1_batch_sync: waits for the stream; GP_ENONFINITE names the slot
 *   whose imaginary-time norm was not finite.
 * gp_spin1_batch_observables: gp_spin1_observables for one slot.
 * gp_spin1_batch_info_read: the launch shape of the last batch_step call. */
typedef struct gp_spin1_batch gp_spin1_batch_t;
typedef struct {                 /* [0] imaginary-time launches, [1] real-time launches (0 if none) */
    int32_t x_points[2]; /* points per thread of the batched x sweep */
    int32_t x_block[2];  /* threads per block of the batched x sweep */
    int32_t y_tile[2];   /* 1-based y tile of the batched y sweep */
    int32_t grouped;     /* condensates that ran in the batched launches */
    int32_t individual;  /* condensates that ran on their own plan */
    int32_t phases;      /* groups of steps with a fixed set of condensates */
    int64_t launches;    /* batched sweep and norm launches */
    int32_t x_solver[2]; /* GP_XSOLVER_CHAIN (chain x windows) or GP_XSOLVER_SCAN (whole-row scans) */
    int32_t y_solver[2]; /* GP_YSOLVER_STACK (stacked chain windows; y_tile a stacked tile) or
                            GP_YSOLVER_WINDOW (scanned windows)                                  */
    int32_t x_tile[2];   /* 1-based chain tile of the batched x sweep (0: whole-row scans)      */
} gp_spin1_batch_info;
int gp_spin1_batch_create(const gp_spin1_params* p, int32_t n, void* hip_stream, gp_spin1_batch_t** out);
int gp_spin1_batch_set_slot(gp_spin1_batch_t* b, int32_t slot, const gp_spin1_params* p);
int gp_spin1_batch_step(gp_spin1_batch_t* b, void* const* psi_dev, const int64_t* nsteps, const int32_t* mode,
                        const uint8_t* active);
int gp_spin1_batch_sync(gp_spin1_batch_t* b);
int gp_spin1_batch_observables(gp_spin1_batch_t* b, int32_t slot, const void* psi_dev, gp_spin1_obs* out_host,
                               void* dens_dev);
int gp_spin1_batch_info_read(const gp_spin1_batch_t* b, gp_spin1_batch_info* out);
int gp_spin1_batch_destroy(gp_spin1_batch_t* b);
const char* gp_spin1_batch_last_error(const gp_spin1_batch_t* b);

/* ---------------------------------------------------------------------------
 * Serving loop.  Replays a trace of independent solve requests against the
 * clock on one batch: requests are admitted in arrival order while a slot is
 * free and the device-memory budget allows (an admitted condensate is charged
 * (2 P + nx ny) s bytes for its wave function, P its plane stride, (2 W + nx ny) s
 * for the work copy, W = nx ny + 4160, 432 (nx + ny) s for its line tables and
 * 64 KiB of scratch, s = 16 or 8); each round advances every admitted
 * condensate together by the steps left to the nearest completion (at most
 * chunk_steps), so requests join and leave between rounds.  A request's
 * latency runs from its arrival to the end of the round that completes it
 * (read from an event recorded after that round).  The rounds run on a stream
 * of the loop's own (non-blocking, default priority; it starts after the
 * work queued on hip_stream, which resumes after the last round), up to two
 * at a time: while the GPU runs one round the host admits arrivals (building
 * their tables) and enqueues the next.  A finished request's tables and work
 * copy leave the budget with its round but stay allocated until they are
 * released (freeing waits for the device): while the GPU idles, at the end,
 * or once such held memory exceeds max(1 GB, a quarter of the budget), after
 * the rounds in flight have drained.
 *
 * req[n]: sorted by arrival (seconds after the start of the trace, scaled by
 *   time_scale; 0 replays every request as arriving at once); p as for
 *   gp_spin1_create, the same precision for all; nsteps >= 1 steps in mode
 *   (0 imaginary time, 1 real time) advance psi_dev (caller-owned device
 *   memory in the usual layout) in place.
 * out[n]: admission and completion times (seconds after the start).
 * stats: wall time, pt-steps served, served and offered pt-steps per second,
 *   latency percentiles (p50, p99; linear interpolation), rounds and mean /
 *   maximum condensates in flight.
 * Blocks until every request is done.  Allocates the slot tables as requests
 * are admitted and frees them after they complete.  GP_EINVAL for unsorted or
 * malformed requests or a request larger than the budget; errors of the
 * batch calls otherwise (message on stderr). */
typedef struct {
    double arrival;        /* seconds after the start of the trace */
    gp_spin1_params p;
    int64_t nsteps;
    int32_t mode;          /* 0 imaginary time, 1 real time */
    void* psi_dev;
} gp_spin1_request;
typedef struct {
    int32_t max_slots;        /* condensates in flight at most (1 .. 4096) */
    double hbm_budget_bytes;  /* device bytes the admitted condensates may hold */
    int64_t chunk_steps;      /* steps per round at most (0: to the nearest completion) */
    double time_scale;        /* factor on the arrival times (1 = real time) */
} gp_spin1_serve_config;
typedef struct {
    double start, finish;     /* seconds after the start of the trace */
} gp_spin1_request_result;
typedef struct {
    double wall_s, pt_steps, served_rate, offered_rate;
    double p50_latency, p99_latency, mean_latency, max_latency;
    int32_t completed, max_active, rounds;
    double mean_active;
    double gpu_busy;          /* fraction of the wall time the GPU spent in rounds */
    double admit_ms;          /* host time spent admitting requests (tables, uploads) */
} gp_spin1_serve_stats;
int gp_spin1_serve(const gp_spin1_request* req, int32_t n, const gp_spin1_serve_config* cfg, void* hip_stream,
                   gp_spin1_request_result* out, gp_spin1_serve_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* GP_SPIN1_H */
