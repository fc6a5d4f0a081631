/*
 * Plain FP64 CPU oracle for the split-step Crank-Nicolson (SSCN) time step of
 * the quasi-2D rotating spin-1 Gross-Pitaevskii equation with Rashba or
 * Dresselhaus spin-orbit (SO) coupling and Rabi coupling
 * (Muruganandam, Balaz, Adhikari, arXiv:2105.10517, Supplementary Material,
 * Eqs. (S.1)-(S.6)).
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the GPU library; it is
 * never called by the product path.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header or
 * table with the HIP kernels.
 *
 * Everything is written in the original spin basis (m = +1, 0, -1), with
 * generic 3x3 complex linear algebra: a generic matrix exponential for the
 * local substep and block-tridiagonal Thomas elimination (3x3 blocks, partial
 * pivoting inside each block) for the two Crank-Nicolson line sweeps.  No
 * eigenbasis tricks, no closed forms, no blocking beyond the scheme itself.
 *
 * Readings of points the paper leaves open (each one is listed, with its
 * reason, in the design notes of the repository):
 *   - Lie splitting, in the order local -> x sweep -> y sweep (-> renormalise
 *     in imaginary time).                     [Solution method; Eqs. S.1-S.3]
 *   - The x parts of -Omega L_z and of the SO term go in the x sweep, the y
 *     parts in the y sweep; L_z = -i (x d/dy - y d/dx).           [Eq. S.3]
 *   - 3-point second difference, central first difference, psi = 0 on the
 *     ghost points just outside the grid.
 *   - V = (x^2 + y^2)/2 (isotropic harmonic trap, lengths in l0).  [Eq. S.3]
 *     Optionally anisotropic, V = (gx^2 x^2 + gy^2 y^2)/2 (the paper calls
 *     V "the confining trap" without fixing its shape).
 *   - The local substep applies the exact exponential of the 3x3 Hermitian
 *     matrix H_loc = (V + c0 rho) I + c2 F.Sigma + R Sigma_x, frozen at the
 *     substep input; H_loc psi reproduces every non-derivative term of
 *     Eqs. (S.1)-(S.2).
 *   - Imaginary time: t -> -i tau, CN with alpha = dt/2, local factor
 *     exp(-dt H_loc), then psi <- psi / sqrt(dx dy sum |psi|^2).
 *   - Real time: CN with alpha = i dt/2, local factor exp(-i dt H_loc).
 *   - Rectangle-rule quadrature; kinetic energy from forward differences over
 *     the ghost-padded range (equal to <psi| -D2/2 |psi>).
 *   - Optional Strang order: half local substep, x sweep, y sweep, half local
 *     substep (second order in dt for the same substeps).
 *   - Optional fixed magnetisation in imaginary time (gamma = R = 0): after
 *     each step the components are rescaled so that the total norm is 1 and
 *     N_{+1} - N_{-1} = m (normalisation and magnetisation conditions stated
 *     with Eq. (S.5)), with the third condition s_{+1} s_{-1} = s_0^2 of the
 *     normalised gradient flow of Bao and Lim (SIAM J. Sci. Comput. 30, 2008).
 *
 * Layout of every wave function: psi[(m * ny + j) * nx + i], m = 0 (+1),
 * 1 (0), 2 (-1); x_i = x0 + i dx, y_j = y0 + j dy.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (see build.py).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

typedef struct {
    int32_t nx, ny;
    double dx, dy, x0, y0, dt;
    double c0, c2, gamma;
    int32_t eta; /* +1 Rashba, -1 Dresselhaus */
    double rabi, omega;
    double gx, gy;        /* trap V = (gx^2 x^2 + gy^2 y^2)/2; 1, 1 is the paper's isotropic trap */
    int32_t split;        /* 0 Lie: local, x, y; 1 Strang: local(dt/2), x, y, local(dt/2) */
    int32_t fix_m;        /* imaginary time: project to norm 1 and magnetisation `magnetization` */
    double magnetization;
} orc_params;

typedef struct {
    double norm[3], norm_total, magnetization;
    double energy, e_kin, e_trap, e_int, e_rot, e_so, e_rabi, lz;
    double mu[3], mu_total;
} orc_obs;

#define IDX(p, m, j, i) (((size_t)(m) * (size_t)(p)->ny + (size_t)(j)) * (size_t)(p)->nx + (size_t)(i))

/* ---------------------------------------------------------------------------
 * Spin-1 matrices.  Sigma_x and Sigma_y as printed in Eq. (S.5); Sigma_z is
 * the diagonal diag(+1, 0, -1) of the F_z = +-1, 0 components (its expectation
 * gives rho_{+1} - rho_{-1}, the magnetisation density of the paper).
 * Row-major 3x3, index [r*3 + c].
 * ------------------------------------------------------------------------- */
static void spin_x(cplx S[9]) {
    const double s = 1.0 / sqrt(2.0);
    cplx t[9] = {0, s, 0, s, 0, s, 0, s, 0};
    memcpy(S, t, sizeof t);
}
static void spin_y(cplx S[9]) {
    const double s = 1.0 / sqrt(2.0);
    /* (i/sqrt2) * [[0,-1,0],[1,0,-1],[0,1,0]] */
    cplx t[9] = {0, -I * s, 0, I * s, 0, -I * s, 0, I * s, 0};
    memcpy(S, t, sizeof t);
}
static void spin_z(cplx S[9]) {
    cplx t[9] = {1, 0, 0, 0, 0, 0, 0, 0, -1};
    memcpy(S, t, sizeof t);
}

/* ---------------------------------------------------------------------------
 * Small dense 3x3 complex helpers.
 * ------------------------------------------------------------------------- */
static void m3_zero(cplx A[9]) { for (int k = 0; k < 9; ++k) A[k] = 0; }
static void m3_eye(cplx A[9]) { m3_zero(A); A[0] = A[4] = A[8] = 1; }
static void m3_mul(const cplx A[9], const cplx B[9], cplx C[9]) {
    cplx T[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += A[r * 3 + k] * B[k * 3 + c];
            T[r * 3 + c] = s;
        }
    memcpy(C, T, sizeof T);
}
static void m3_vec(const cplx A[9], const cplx v[3], cplx w[3]) {
    cplx t[3];
    for (int r = 0; r < 3; ++r) t[r] = A[r * 3 + 0] * v[0] + A[r * 3 + 1] * v[1] + A[r * 3 + 2] * v[2];
    memcpy(w, t, sizeof t);
}
static double m3_norm1(const cplx A[9]) {
    double best = 0;
    for (int c = 0; c < 3; ++c) {
        double s = cabs(A[c]) + cabs(A[3 + c]) + cabs(A[6 + c]);
        if (s > best) best = s;
    }
    return best;
}

/* LU factorisation with partial pivoting of a 3x3 complex matrix. */
typedef struct { cplx lu[9]; int piv[3]; } lu3;

static void lu3_factor(const cplx M[9], lu3 *f) {
    memcpy(f->lu, M, sizeof f->lu);
    for (int k = 0; k < 3; ++k) f->piv[k] = k;
    for (int k = 0; k < 3; ++k) {
        int p = k;
        double best = cabs(f->lu[k * 3 + k]);
        for (int r = k + 1; r < 3; ++r)
            if (cabs(f->lu[r * 3 + k]) > best) { best = cabs(f->lu[r * 3 + k]); p = r; }
        if (p != k) {
            for (int c = 0; c < 3; ++c) {
                cplx t = f->lu[k * 3 + c]; f->lu[k * 3 + c] = f->lu[p * 3 + c]; f->lu[p * 3 + c] = t;
            }
            int t = f->piv[k]; f->piv[k] = f->piv[p]; f->piv[p] = t;
        }
        for (int r = k + 1; r < 3; ++r) {
            cplx l = f->lu[r * 3 + k] / f->lu[k * 3 + k];
            f->lu[r * 3 + k] = l;
            for (int c = k + 1; c < 3; ++c) f->lu[r * 3 + c] -= l * f->lu[k * 3 + c];
        }
    }
}
static void lu3_solve(const lu3 *f, const cplx b[3], cplx x[3]) {
    cplx y[3];
    for (int r = 0; r < 3; ++r) y[r] = b[f->piv[r]];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < r; ++c) y[r] -= f->lu[r * 3 + c] * y[c];
    for (int r = 2; r >= 0; --r) {
        for (int c = r + 1; c < 3; ++c) y[r] -= f->lu[r * 3 + c] * y[c];
        y[r] /= f->lu[r * 3 + r];
    }
    memcpy(x, y, sizeof y);
}
/* X = M^{-1} B for a 3x3 right-hand side B. */
static void lu3_solve_mat(const lu3 *f, const cplx B[9], cplx X[9]) {
    cplx T[9];
    for (int c = 0; c < 3; ++c) {
        cplx col[3] = {B[c], B[3 + c], B[6 + c]}, sol[3];
        lu3_solve(f, col, sol);
        T[c] = sol[0]; T[3 + c] = sol[1]; T[6 + c] = sol[2];
    }
    memcpy(X, T, sizeof T);
}

/* Generic matrix exponential by scaling and squaring with a truncated Taylor
 * series (Moler & Van Loan, "Nineteen dubious ways...", method 3): scale A by
 * 2^-s so that ||A||_1 <= 1/2, sum 24 Taylor terms, square s times. */
static void m3_expm(const cplx A[9], cplx E[9]) {
    int s = 0;
    double nrm = m3_norm1(A);
    while (nrm > 0.5) { nrm *= 0.5; ++s; }
    const double scale = ldexp(1.0, -s);
    cplx B[9], term[9], sum[9];
    for (int k = 0; k < 9; ++k) B[k] = A[k] * scale;
    m3_eye(sum);
    m3_eye(term);
    for (int n = 1; n <= 24; ++n) {
        m3_mul(term, B, term);
        for (int k = 0; k < 9; ++k) term[k] /= (double)n;
        for (int k = 0; k < 9; ++k) sum[k] += term[k];
    }
    for (int q = 0; q < s; ++q) m3_mul(sum, sum, sum);
    memcpy(E, sum, sizeof sum);
}

/* ---------------------------------------------------------------------------
 * Local (non-derivative) operator.
 *   H_loc = (V + c0 rho) I + c2 (F_x Sigma_x + F_y Sigma_y + F_z Sigma_z)
 *           + R Sigma_x,       F_a = psi^dagger Sigma_a psi,
 * which reproduces the bracketed c2 terms, the {} spin-mixing terms and the
 * Rabi terms of Eqs. (S.1)-(S.2), with the trap and c0 rho of H in Eq. (S.3).
 * ------------------------------------------------------------------------- */
/* Trap potential V(x, y) (Eq. S.3, harmonic, optionally anisotropic). */
static double orc_trap(const orc_params *p, double x, double y) {
    return 0.5 * (p->gx * p->gx * x * x + p->gy * p->gy * y * y);
}

void orc_local_matrix(const orc_params *p, const cplx v[3], double x, double y, cplx H[9]) {
    cplx Sx[9], Sy[9], Sz[9], w[3];
    spin_x(Sx); spin_y(Sy); spin_z(Sz);
    const double rho = creal(conj(v[0]) * v[0] + conj(v[1]) * v[1] + conj(v[2]) * v[2]);
    double F[3];
    const cplx *S[3] = {Sx, Sy, Sz};
    for (int a = 0; a < 3; ++a) {
        m3_vec(S[a], v, w);
        F[a] = creal(conj(v[0]) * w[0] + conj(v[1]) * w[1] + conj(v[2]) * w[2]);
    }
    const double V = orc_trap(p, x, y);
    m3_eye(H);
    for (int k = 0; k < 9; ++k)
        H[k] = H[k] * (V + p->c0 * rho) + p->c2 * (F[0] * Sx[k] + F[1] * Sy[k] + F[2] * Sz[k]) + p->rabi * Sx[k];
}

/* Local substep: psi <- exp(-i dt H_loc) psi (real time) or
 * exp(-dt H_loc) psi (imaginary time), H_loc frozen at the input. */
void orc_pointwise(const orc_params *p, cplx *psi, int imag) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < p->ny; ++j) {
        const double y = p->y0 + j * p->dy;
        for (int i = 0; i < p->nx; ++i) {
            const double x = p->x0 + i * p->dx;
            cplx v[3] = {psi[IDX(p, 0, j, i)], psi[IDX(p, 1, j, i)], psi[IDX(p, 2, j, i)]};
            cplx H[9], A[9], E[9];
            orc_local_matrix(p, v, x, y, H);
            const cplx f = imag ? -p->dt : -I * p->dt;
            for (int k = 0; k < 9; ++k) A[k] = f * H[k];
            m3_expm(A, E);
            m3_vec(E, v, v);
            for (int m = 0; m < 3; ++m) psi[IDX(p, m, j, i)] = v[m];
        }
    }
}

/* ---------------------------------------------------------------------------
 * SO coupling matrices, read off the explicit Rashba/Dresselhaus terms printed
 * after Eq. (S.5):
 *   gamma f_{+-1} = -i g~ [eta d_y psi_0 +- i d_x psi_0]
 *   gamma f_0     = -i g~ [-i d_x psi_{+1} + i d_x psi_{-1}
 *                          + eta d_y psi_{+1} + eta d_y psi_{-1}],
 * g~ = gamma/sqrt2.  Written as K_x d_x psi + K_y d_y psi with 3x3 K's.
 * ------------------------------------------------------------------------- */
static void so_kx(const orc_params *p, cplx K[9]) {
    const double g = p->gamma / sqrt(2.0);
    m3_zero(K);
    K[0 * 3 + 1] = -I * g * (I);   /* f_{+1}: -i g (+i d_x psi_0) */
    K[2 * 3 + 1] = -I * g * (-I);  /* f_{-1}: -i g (-i d_x psi_0) */
    K[1 * 3 + 0] = -I * g * (-I);  /* f_0:    -i g (-i d_x psi_{+1}) */
    K[1 * 3 + 2] = -I * g * (I);   /* f_0:    -i g (+i d_x psi_{-1}) */
}
static void so_ky(const orc_params *p, cplx K[9]) {
    const double g = p->gamma / sqrt(2.0);
    const double e = (double)p->eta;
    m3_zero(K);
    K[0 * 3 + 1] = -I * g * e;  /* f_{+1}: -i g eta d_y psi_0 */
    K[2 * 3 + 1] = -I * g * e;  /* f_{-1}: -i g eta d_y psi_0 */
    K[1 * 3 + 0] = -I * g * e;  /* f_0:    -i g eta d_y psi_{+1} */
    K[1 * 3 + 2] = -I * g * e;  /* f_0:    -i g eta d_y psi_{-1} */
}

/* Block-tridiagonal Thomas elimination for a line of n unknown 3-vectors with
 * constant blocks:  A u_{k-1} + B u_k + C u_{k+1} = r_k,  u_{-1} = u_n = 0.
 * On entry u holds r (n*3), on exit the solution.  work: n*9 complex. */
static void block_thomas(int n, const cplx A[9], const cplx B[9], const cplx C[9], cplx *u, cplx *Cp) {
    lu3 f;
    cplx M[9], T[9], t3[3];
    lu3_factor(B, &f);
    lu3_solve_mat(&f, C, Cp);
    lu3_solve(&f, &u[0], &u[0]);
    for (int k = 1; k < n; ++k) {
        m3_mul(A, &Cp[(size_t)(k - 1) * 9], T);
        for (int q = 0; q < 9; ++q) M[q] = B[q] - T[q];
        lu3_factor(M, &f);
        lu3_solve_mat(&f, C, &Cp[(size_t)k * 9]);
        m3_vec(A, &u[(size_t)(k - 1) * 3], t3);
        for (int q = 0; q < 3; ++q) t3[q] = u[(size_t)k * 3 + q] - t3[q];
        lu3_solve(&f, t3, &u[(size_t)k * 3]);
    }
    for (int k = n - 2; k >= 0; --k) {
        m3_vec(&Cp[(size_t)k * 9], &u[(size_t)(k + 1) * 3], t3);
        for (int q = 0; q < 3; ++q) u[(size_t)k * 3 + q] -= t3[q];
    }
}

/* One Crank-Nicolson line solve (I + alpha H1) u' = (I - alpha H1) u for a
 * 1-D operator H1 u_k = L u_{k-1} + D u_k + U u_{k+1}. */
static void cn_line(int n, cplx alpha, const cplx L[9], const cplx D[9], const cplx U[9], cplx *u, cplx *rhs,
                    cplx *work) {
    cplx A[9], B[9], C[9];
    for (int q = 0; q < 9; ++q) {
        A[q] = alpha * L[q];
        B[q] = (q % 4 == 0 ? 1.0 : 0.0) + alpha * D[q];
        C[q] = alpha * U[q];
    }
    for (int k = 0; k < n; ++k) {
        cplx h[3] = {0, 0, 0}, t[3];
        if (k > 0) { m3_vec(L, &u[(size_t)(k - 1) * 3], t); for (int q = 0; q < 3; ++q) h[q] += t[q]; }
        m3_vec(D, &u[(size_t)k * 3], t);
        for (int q = 0; q < 3; ++q) h[q] += t[q];
        if (k + 1 < n) { m3_vec(U, &u[(size_t)(k + 1) * 3], t); for (int q = 0; q < 3; ++q) h[q] += t[q]; }
        for (int q = 0; q < 3; ++q) rhs[(size_t)k * 3 + q] = u[(size_t)k * 3 + q] - alpha * h[q];
    }
    block_thomas(n, A, B, C, rhs, work);
    memcpy(u, rhs, (size_t)n * 3 * sizeof(cplx));
}

/* Stencil blocks of a 1-D operator  -1/2 d2 + s d + K d  on step h, where s is
 * a scalar coefficient of d (the rotation part) and K the SO matrix:
 *   L = -1/(2h^2) I - s/(2h) I - K/(2h),  D = 1/h^2 I,
 *   U = -1/(2h^2) I + s/(2h) I + K/(2h). */
static void line_blocks(double h, cplx s, const cplx K[9], cplx L[9], cplx D[9], cplx U[9]) {
    for (int q = 0; q < 9; ++q) {
        const double id = (q % 4 == 0) ? 1.0 : 0.0;
        L[q] = id * (-0.5 / (h * h) - s / (2 * h)) - K[q] / (2 * h);
        D[q] = id * (1.0 / (h * h));
        U[q] = id * (-0.5 / (h * h) + s / (2 * h)) + K[q] / (2 * h);
    }
}

/* x sweep.  H_x = -1/2 d_x^2 - i Omega y d_x + K_x d_x : the x parts of the
 * kinetic term, of -Omega L_z = i Omega (x d_y - y d_x) and of the SO term. */
void orc_sweep_x(const orc_params *p, cplx *psi, int imag) {
    const cplx alpha = imag ? 0.5 * p->dt : 0.5 * I * p->dt;
    cplx K[9];
    so_kx(p, K);
#pragma omp parallel
    {
        cplx *u = malloc((size_t)p->nx * 3 * sizeof(cplx));
        cplx *rhs = malloc((size_t)p->nx * 3 * sizeof(cplx));
        cplx *work = malloc((size_t)p->nx * 9 * sizeof(cplx));
#pragma omp for schedule(static)
        for (int j = 0; j < p->ny; ++j) {
            const double y = p->y0 + j * p->dy;
            cplx L[9], D[9], U[9];
            line_blocks(p->dx, -I * p->omega * y, K, L, D, U);
            for (int i = 0; i < p->nx; ++i)
                for (int m = 0; m < 3; ++m) u[(size_t)i * 3 + m] = psi[IDX(p, m, j, i)];
            cn_line(p->nx, alpha, L, D, U, u, rhs, work);
            for (int i = 0; i < p->nx; ++i)
                for (int m = 0; m < 3; ++m) psi[IDX(p, m, j, i)] = u[(size_t)i * 3 + m];
        }
        free(u); free(rhs); free(work);
    }
}

/* y sweep.  H_y = -1/2 d_y^2 + i Omega x d_y + K_y d_y. */
void orc_sweep_y(const orc_params *p, cplx *psi, int imag) {
    const cplx alpha = imag ? 0.5 * p->dt : 0.5 * I * p->dt;
    cplx K[9];
    so_ky(p, K);
#pragma omp parallel
    {
        cplx *u = malloc((size_t)p->ny * 3 * sizeof(cplx));
        cplx *rhs = malloc((size_t)p->ny * 3 * sizeof(cplx));
        cplx *work = malloc((size_t)p->ny * 9 * sizeof(cplx));
#pragma omp for schedule(static)
        for (int i = 0; i < p->nx; ++i) {
            const double x = p->x0 + i * p->dx;
            cplx L[9], D[9], U[9];
            line_blocks(p->dy, I * p->omega * x, K, L, D, U);
            for (int j = 0; j < p->ny; ++j)
                for (int m = 0; m < 3; ++m) u[(size_t)j * 3 + m] = psi[IDX(p, m, j, i)];
            cn_line(p->ny, alpha, L, D, U, u, rhs, work);
            for (int j = 0; j < p->ny; ++j)
                for (int m = 0; m < 3; ++m) psi[IDX(p, m, j, i)] = u[(size_t)j * 3 + m];
        }
        free(u); free(rhs); free(work);
    }
}

/* Total norm dx dy sum_m sum_ij |psi_m|^2 (normalisation condition after
 * Eq. (S.5)); summed per row, then rows in order. */
double orc_norm(const orc_params *p, const cplx *psi) {
    double *row = calloc((size_t)p->ny, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int j = 0; j < p->ny; ++j) {
        double s = 0;
        for (int m = 0; m < 3; ++m)
            for (int i = 0; i < p->nx; ++i) {
                const cplx v = psi[IDX(p, m, j, i)];
                s += creal(v) * creal(v) + cimag(v) * cimag(v);
            }
        row[j] = s;
    }
    double s = 0;
    for (int j = 0; j < p->ny; ++j) s += row[j];
    free(row);
    return s * p->dx * p->dy;
}

/* Norm of one component, N_m = dx dy sum |psi_m|^2. */
static double orc_component_norm(const orc_params *p, const cplx *psi, int m) {
    double s = 0.0;
    for (int j = 0; j < p->ny; ++j) {
        double r = 0.0;
        for (int i = 0; i < p->nx; ++i) {
            const cplx v = psi[IDX(p, m, j, i)];
            r += creal(v) * creal(v) + cimag(v) * cimag(v);
        }
        s += r;
    }
    return s * p->dx * p->dy;
}

/* Imaginary-time normalisation.  Total norm: psi <- psi / sqrt(N).  Fixed
 * magnetisation m: psi_j <- s_j psi_j with
 *   s_{+1}^2 N_{+1} + s_0^2 N_0 + s_{-1}^2 N_{-1} = 1,
 *   s_{+1}^2 N_{+1} - s_{-1}^2 N_{-1} = m,
 *   s_{+1} s_{-1} = s_0^2.
 * The first two give s_{+-1}^2 = (1 +- m - u N_0) / (2 N_{+-1}) with
 * u = s_0^2; the third then reads
 *   (N_0^2 - 4 N_{+1} N_{-1}) u^2 - 2 N_0 u + (1 - m^2) = 0,
 * whose root that stays finite as N_0^2 -> 4 N_{+1} N_{-1} is
 *   u = (1 - m^2) / (N_0 + sqrt(m^2 N_0^2 + 4 (1 - m^2) N_{+1} N_{-1})). */
void orc_normalize(const orc_params *p, cplx *psi) {
    double f[3];
    if (p->fix_m) {
        const double n1 = orc_component_norm(p, psi, 0), n0 = orc_component_norm(p, psi, 1),
                     nm = orc_component_norm(p, psi, 2), m = p->magnetization;
        const double u = (1.0 - m * m) / (n0 + sqrt(m * m * n0 * n0 + 4.0 * (1.0 - m * m) * n1 * nm));
        f[1] = sqrt(u);
        f[0] = sqrt((1.0 + m - u * n0) / (2.0 * n1));
        f[2] = sqrt((1.0 - m - u * n0) / (2.0 * nm));
    } else {
        f[0] = f[1] = f[2] = 1.0 / sqrt(orc_norm(p, psi));
    }
    const size_t plane = (size_t)p->nx * p->ny;
    for (int c = 0; c < 3; ++c)
        for (size_t k = 0; k < plane; ++k) psi[c * plane + k] *= f[c];
}

/* One SSCN step.  Lie: local substep, x sweep, y sweep; Strang: half local
 * substep, x sweep, y sweep, half local substep; then (imaginary time) the
 * normalisation. */
void orc_step(const orc_params *p, cplx *psi, int64_t nsteps, int imag) {
    orc_params half = *p;
    half.dt = 0.5 * p->dt;
    for (int64_t s = 0; s < nsteps; ++s) {
        orc_pointwise(p->split ? &half : p, psi, imag);
        orc_sweep_x(p, psi, imag);
        orc_sweep_y(p, psi, imag);
        if (p->split) orc_pointwise(&half, psi, imag);
        if (imag) orc_normalize(p, psi);
    }
}

/* ---------------------------------------------------------------------------
 * Right-hand sides of Eqs. (S.1)-(S.2), term by term as printed, on the grid:
 *   out_m = [H + c2 (...)] psi_m + {c2 spin-mixing} + R/sqrt2 (...) + gamma f_m,
 *   H = -1/2 (D_xx + D_yy) + V + c0 rho - Omega L_z,
 *   L_z = -i (x D_y - y D_x).
 * ------------------------------------------------------------------------- */
static inline cplx at(const orc_params *p, const cplx *psi, int m, int j, int i) {
    if (i < 0 || i >= p->nx || j < 0 || j >= p->ny) return 0;
    return psi[IDX(p, m, j, i)];
}

void orc_apply_h(const orc_params *p, const cplx *psi, cplx *out) {
    const double gt = p->gamma / sqrt(2.0), eta = (double)p->eta, r2 = p->rabi / sqrt(2.0);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < p->ny; ++j) {
        const double y = p->y0 + j * p->dy;
        for (int i = 0; i < p->nx; ++i) {
            const double x = p->x0 + i * p->dx;
            cplx v[3], lap[3], ddx[3], ddy[3];
            for (int m = 0; m < 3; ++m) {
                v[m] = at(p, psi, m, j, i);
                lap[m] = (at(p, psi, m, j, i + 1) - 2.0 * v[m] + at(p, psi, m, j, i - 1)) / (p->dx * p->dx)
                       + (at(p, psi, m, j + 1, i) - 2.0 * v[m] + at(p, psi, m, j - 1, i)) / (p->dy * p->dy);
                ddx[m] = (at(p, psi, m, j, i + 1) - at(p, psi, m, j, i - 1)) / (2 * p->dx);
                ddy[m] = (at(p, psi, m, j + 1, i) - at(p, psi, m, j - 1, i)) / (2 * p->dy);
            }
            const double rp = creal(v[0] * conj(v[0])), r0 = creal(v[1] * conj(v[1])), rm = creal(v[2] * conj(v[2]));
            const double rho = rp + r0 + rm;
            const double V = orc_trap(p, x, y);
            cplx Hv[3];
            for (int m = 0; m < 3; ++m) {
                const cplx Lz = -I * (x * ddy[m] - y * ddx[m]);
                Hv[m] = -0.5 * lap[m] + (V + p->c0 * rho) * v[m] - p->omega * Lz;
            }
            /* gamma f terms (after Eq. (S.5)) */
            const cplx fp = -I * gt * (eta * ddy[1] + I * ddx[1]);
            const cplx fm = -I * gt * (eta * ddy[1] - I * ddx[1]);
            const cplx f0 = -I * gt * (-I * ddx[0] + I * ddx[2] + eta * ddy[0] + eta * ddy[2]);
            /* Eq. (S.1), upper sign (+1) and lower sign (-1); Eq. (S.2) for 0 */
            out[IDX(p, 0, j, i)] = Hv[0] + p->c2 * (rp - rm + r0) * v[0] + p->c2 * v[1] * v[1] * conj(v[2]) + r2 * v[1] + fp;
            out[IDX(p, 2, j, i)] = Hv[2] + p->c2 * (rm - rp + r0) * v[2] + p->c2 * v[1] * v[1] * conj(v[0]) + r2 * v[1] + fm;
            out[IDX(p, 1, j, i)] = Hv[1] + p->c2 * (rp + rm) * v[1] + 2.0 * p->c2 * v[0] * v[2] * conj(v[1])
                                 + r2 * (v[0] + v[2]) + f0;
        }
    }
}

/* ---------------------------------------------------------------------------
 * Observables: norms and magnetisation (conditions after Eq. (S.5)), the
 * energy functional of Eq. (S.6) term by term, <L_z>, and chemical potentials
 *   mu_m = Re <psi_m | (H psi)_m> / N_m,  mu = sum_m Re<psi_m|(H psi)_m> / sum N_m,
 * with (H psi) the right-hand sides of Eqs. (S.1)-(S.2).
 * Every sum is accumulated per row, then over rows in order.
 * ------------------------------------------------------------------------- */
enum { Q_N0, Q_N1, Q_N2, Q_KIN, Q_TRAP, Q_INT, Q_ROT, Q_SO, Q_RABI, Q_LZ, Q_HM0, Q_HM1, Q_HM2, Q_COUNT };

void orc_observables(const orc_params *p, const cplx *psi, orc_obs *o) {
    const size_t n = (size_t)3 * p->nx * p->ny;
    cplx *hpsi = malloc(n * sizeof(cplx));
    orc_apply_h(p, psi, hpsi);
    double *rows = calloc((size_t)p->ny * Q_COUNT, sizeof(double));
    const double gt = p->gamma / sqrt(2.0), eta = (double)p->eta;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < p->ny; ++j) {
        double *q = &rows[(size_t)j * Q_COUNT];
        const double y = p->y0 + j * p->dy;
        /* kinetic: forward differences over the ghost-padded range; the
           i = -1 and j = -1 terms (|psi_0 - 0|^2) are assigned to i = 0 / j = 0 */
        for (int m = 0; m < 3; ++m)
            for (int i = 0; i < p->nx; ++i) {
                const cplx v = at(p, psi, m, j, i);
                const cplx gx = at(p, psi, m, j, i + 1) - v, gy = at(p, psi, m, j + 1, i) - v;
                double k = creal(gx * conj(gx)) / (p->dx * p->dx) + creal(gy * conj(gy)) / (p->dy * p->dy);
                if (i == 0) k += creal(v * conj(v)) / (p->dx * p->dx);
                if (j == 0) k += creal(v * conj(v)) / (p->dy * p->dy);
                q[Q_KIN] += 0.5 * k;
            }
        for (int i = 0; i < p->nx; ++i) {
            const double x = p->x0 + i * p->dx;
            cplx v[3], ddx[3], ddy[3];
            for (int m = 0; m < 3; ++m) {
                v[m] = at(p, psi, m, j, i);
                ddx[m] = (at(p, psi, m, j, i + 1) - at(p, psi, m, j, i - 1)) / (2 * p->dx);
                ddy[m] = (at(p, psi, m, j + 1, i) - at(p, psi, m, j - 1, i)) / (2 * p->dy);
            }
            const double rp = creal(v[0] * conj(v[0])), r0 = creal(v[1] * conj(v[1])), rm = creal(v[2] * conj(v[2]));
            const double rho = rp + r0 + rm;
            const double V = orc_trap(p, x, y);
            q[Q_N0] += rp; q[Q_N1] += r0; q[Q_N2] += rm;
            q[Q_TRAP] += V * rho;
            /* 1/2 { c0 rho^2 + c2 [ ... ] } of Eq. (S.6) */
            const cplx mix = conj(v[2]) * v[1] * v[1] * conj(v[0]) + v[2] * conj(v[1]) * conj(v[1]) * v[0];
            q[Q_INT] += 0.5 * (p->c0 * rho * rho
                               + p->c2 * (rp * rp + rm * rm + 2.0 * (rp * r0 + rm * r0 - rp * rm + creal(mix))));
            /* -Omega sum_j psi_j^* L_z psi_j */
            for (int m = 0; m < 3; ++m) {
                const cplx Lz = -I * (x * ddy[m] - y * ddx[m]);
                const double lz = creal(conj(v[m]) * Lz);
                q[Q_LZ] += lz;
                q[Q_ROT] += -p->omega * lz;
            }
            /* 1/2 sqrt2 R [ (psi_{+1}^* + psi_{-1}^*) psi_0 + psi_0^* (psi_{+1} + psi_{-1}) ] */
            q[Q_RABI] += 0.5 * sqrt(2.0) * p->rabi * creal((conj(v[0]) + conj(v[2])) * v[1] + conj(v[1]) * (v[0] + v[2]));
            /* 1/2 * 2 [psi_{+1}^* (gamma f_{+1}) + psi_{-1}^* (gamma f_{-1}) + psi_0^* (gamma f_0)] */
            const cplx fp = -I * gt * (eta * ddy[1] + I * ddx[1]);
            const cplx fm = -I * gt * (eta * ddy[1] - I * ddx[1]);
            const cplx f0 = -I * gt * (-I * ddx[0] + I * ddx[2] + eta * ddy[0] + eta * ddy[2]);
            q[Q_SO] += creal(conj(v[0]) * fp + conj(v[2]) * fm + conj(v[1]) * f0);
            for (int m = 0; m < 3; ++m) q[Q_HM0 + m] += creal(conj(v[m]) * hpsi[IDX(p, m, j, i)]);
        }
    }
    double tot[Q_COUNT] = {0};
    for (int j = 0; j < p->ny; ++j)
        for (int k = 0; k < Q_COUNT; ++k) tot[k] += rows[(size_t)j * Q_COUNT + k];
    const double w = p->dx * p->dy;
    for (int k = 0; k < Q_COUNT; ++k) tot[k] *= w;
    o->norm[0] = tot[Q_N0]; o->norm[1] = tot[Q_N1]; o->norm[2] = tot[Q_N2];
    o->norm_total = tot[Q_N0] + tot[Q_N1] + tot[Q_N2];
    o->magnetization = tot[Q_N0] - tot[Q_N2];
    o->e_kin = tot[Q_KIN]; o->e_trap = tot[Q_TRAP]; o->e_int = tot[Q_INT]; o->e_rot = tot[Q_ROT];
    o->e_so = tot[Q_SO]; o->e_rabi = tot[Q_RABI]; o->lz = tot[Q_LZ];
    o->energy = o->e_kin + o->e_trap + o->e_int + o->e_rot + o->e_so + o->e_rabi;
    double hs = 0;
    for (int m = 0; m < 3; ++m) {
        /* an empty component (N_m = 0) has no chemical potential of its own: 0 */
        o->mu[m] = o->norm[m] > 0.0 ? tot[Q_HM0 + m] / o->norm[m] : 0.0;
        hs += tot[Q_HM0 + m];
    }
    o->mu_total = hs / o->norm_total;
    free(rows);
    free(hpsi);
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
