/*
 * she_oracle.c -- plain FP64 CPU oracle for the finite-volume stochastic heat
 * equation (SHE) and the Dean-Kawasaki (DK) species-diffusion equation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP library.
 *
 * What it computes (Garcia, Bell, Nonaka, Srivastava, Ladiges, Kim,
 * "An Introduction to Computational Fluctuating Hydrodynamics"):
 *   - cell-centred grid x_i = (i+1/2) dx, faces at half-integers (Sec. 3);
 *   - forward-Euler (Euler-Maruyama) step: T += r*(second difference)
 *     + divergence of the stochastic face flux (Sec. 3, FE scheme);
 *   - predictor-corrector step: trapezoidal corrector that re-uses the
 *     predictor's Gaussian numbers (Sec. 3, PC scheme and its footnote);
 *   - face temperature = arithmetic mean of the two cells (Sec. 3);
 *   - face noise = N(0,1) / sqrt(dV dt) per face per step (Sec. 3, discrete
 *     noise variance); combined with alpha*dt/dx this is sigma*T_face*N with
 *     sigma = sqrt(2 r eps), eps = k_B/(rho c_V dV), r = kappa dt/dx^2;
 *   - Dirichlet walls: ghost stencil (T_1 - 3 T_0 + 2 T_L) and wall-face noise
 *     sqrt(2) T_L Z (Sec. 3, Dirichlet boundary paragraph);
 *   - Dean-Kawasaki flux: D grad n + sqrt(2 D n) Z (Sec. 4, eq. DK), i.e.
 *     sigma*sqrt(n_face)*N with sigma = sqrt(2 r / dV);
 *   - time averages after a relaxation period (Sec. 3, time-average formula),
 *     variance, two-point correlation, and the structure factor
 *     S_k = <|sum_j T_j exp(-2 pi i j k/N)|^2> (Sec. 3, structure factor);
 *   - 1D time correlation <dT_i^n dT_i^(n-m)> over sample lags m (the first
 *     of the suggested exercises, Sec. 6): sums over samples n >= m of
 *     delta_i(n) delta_i(n-m), with the last L samples kept in a ring;
 *   - stochastic Burgers equation (Sec. 5, menagerie):
 *     dc/dt = -d/dx( a c (1-c) - D dc/dx + sqrt(2 D c (1-c)) Z ), in the same
 *     face-flux form: the face value is the arithmetic mean c_f, the flux
 *     gains -nu c_f (1 - c_f) (nu = a dt/dx, centred) and the noise amplitude
 *     is sqrt(max(c_f (1 - c_f), 0)); the paper gives no scheme for it, so
 *     this is the SHE/DK framework of Sec. 3 applied to it (1D);
 *   - implicit diffusion (the implicit-scheme exercise, Sec. 6), 1D: backward
 *     Euler (theta = 1) or Crank-Nicolson (theta = 1/2) for the deterministic
 *     flux with the noise explicit (face amplitude of U^n):
 *       (I - theta W A) U' = U + (1 - theta) W (A U + b) + theta W b + noise,
 *     W (A U + b) being the noise-free divergence (b: Dirichlet wall terms);
 *     solved with the Thomas algorithm, periodic rods with the
 *     Sherman-Morrison correction of the cyclic system;
 *   - 1D materials that vary along the rod (the composite-rod exercise,
 *     Sec. 6): the conservative form rho c_V dT/dt = -d/dx(flux) of eq. SHE
 *     with a conductance r_f and noise factor s_f per face and a factor
 *     w_i = (rho c_V)_ref / (rho c_V)_i per cell, T_i += w_i (F_(i+1) - F_i).
 *
 * Gaussian numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11) and the Box-Muller transform
 * (Box and Muller 1958).  The paper draws from an unseeded NumPy generator, so
 * any reproducible counter layout is a reading; the one used here is:
 *   key     = (seed mod 2^32, seed div 2^32)
 *   counter = (face >> 2, step mod 2^32, ((step >> 32) & 0xFFFF) | tag << 16,
 *              realisation)
 *   lane    = face & 3; lanes (0,1) and (2,3) form Box-Muller pairs,
 *   u_a     = ((word_a >> 9) + 1/2) * 2^-23 in (0, 1) (the radius needs u_a > 0),
 *   u_b     = (word_b >> 9) * 2^-23 in [0, 1) (the angle; exact in FP32 and FP64),
 *   even lane: sqrt(-2 ln u_a) cos(2 pi u_b), odd lane: ... sin(2 pi u_b).
 * tag 0 = step noise, tag 1 = initial perturbation (one number per cell).
 *
 * Face numbering: 1D face f is the low (left) face of cell f, f = 0..N-1
 * (periodic) or 0..N (Dirichlet, face N = right wall).  In 2D/3D the low face
 * of cell (x,y,z) in direction e is  f = ((z*Ny + y)*dim + e)*Nx + x.
 *
 * Compiled with -ffp-contract=off; everything in IEEE double.  Loops whose
 * iterations are independent (one Philox block, one face flux, one cell
 * update, one DFT line each) run on OpenMP threads; every sum over cells or
 * samples stays a sequential loop, so the results do not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    int32_t dim;         /* 1, 2 or 3                                         */
    int32_t n[3];        /* cells per axis (unused axes = 1)                  */
    int32_t eq;          /* 0 = heat (T), 1 = species number density (DK),
                            2 = stochastic Burgers (c, 1D)                     */
    int32_t bc;          /* 0 = periodic, 1 = Dirichlet walls in x (1D only)  */
    int32_t scheme;      /* 0 = forward Euler, 1 = predictor-corrector,
                            2 = backward Euler, 3 = Crank-Nicolson (1D)       */
    int32_t noise;       /* 0 = instantaneous face value, 1 = deterministic
                            (steady-profile) face value, 2 = no noise         */
    double r;            /* kappa dt / dx^2 (heat) or D dt / dx^2 (species)  */
    double sigma;        /* noise factor sqrt(2 r eps)                        */
    double u0;           /* uniform initial / reference value (periodic)      */
    double u_left;       /* Dirichlet wall value at x = 0                     */
    double u_right;      /* Dirichlet wall value at x = L                     */
    double init_sd;      /* std. dev. of the initial per-cell perturbation    */
    uint64_t seed;
    uint32_t realisation;
    uint32_t pad_;
    const double *face_r;  /* 1D, optional: conductance per face (replaces r)  */
    const double *face_s;  /* 1D, optional: noise factor per face (replaces sigma) */
    const double *cell_w;  /* 1D, optional: capacity factor per cell (else 1)  */
    double nu;             /* Burgers: Courant number a dt / dx               */
} or_desc;

typedef struct {
    int64_t burn_in;     /* sample after completed step t if t > burn_in ... */
    int64_t every;       /* ... and t % every == 0                            */
    int64_t n_samples;
    double *s1, *s2;     /* per-cell sums of delta, delta^2 (delta = U - ref) */
    double *m2;          /* 1D: N*N sums of delta_i delta_j, or NULL          */
    double *sk;          /* 1D: N sums of |DFT(U)_k|^2; nD: radial bin sums  */
    int32_t n_bins;
    int32_t pad_;
    double sp_mean;      /* sum over samples of the spatial mean of delta     */
    double sp_sq;        /* ... of the spatial mean of delta^2                */
    double sp_var;       /* ... of the spatial variance                       */
    int64_t clamp_count; /* DK: faces whose mean density was negative         */
    int32_t nonfinite;
    int32_t pad2_;
    int64_t nonfinite_step;
    int64_t tc_lags;     /* 1D: lags L of the time correlation (0 = off)      */
    double *tc;          /* L*N sums over samples n >= m of d_i(n) d_i(n-m)   */
    double *tc_hist;     /* L*N ring of the last L samples' delta             */
    /* batch means (Sec. 3 time averages, split into consecutive batches):
     * sample n (0-based) belongs to batch n / batch_len; each batch keeps
     * its own sums of the same quantities as the totals above           */
    int64_t batch_len;   /* samples per batch (0: no batch sums)              */
    int64_t batch_cap;   /* batches the arrays below hold                     */
    double *b_s1, *b_s2; /* [batch_cap][nc] sums of delta, delta^2, or NULL   */
    double *b_sk;        /* [batch_cap][n_bins (nD) or N (1D)], or NULL       */
    double *b_sp;        /* [batch_cap][3]: spatial mean, mean square, variance */
} or_stats;

/* ---------------------------------------------------------------- Philox */

/* Philox4x32 with 10 rounds, written from the SC'11 definition: each round
 * multiplies words 0 and 2 by the two round multipliers, takes the 64-bit
 * products apart into high and low halves, and permutes/xors them with the
 * other two words and the round key; the key is bumped by the two Weyl
 * constants between rounds. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void block_words(uint64_t seed, uint32_t realisation, uint32_t tag,
                        uint64_t step, uint64_t block, uint32_t x[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = (uint32_t)block;
    ctr[1] = (uint32_t)(step & 0xFFFFFFFFu);
    ctr[2] = (uint32_t)((step >> 32) & 0xFFFFu) | (tag << 16);
    ctr[3] = realisation;
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
    or_philox4x32_10(ctr, key, x);
}

static double unit_open(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * 0x1p-23;
}

static double unit_angle(uint32_t w)
{
    return (double)(w >> 9) * 0x1p-23;
}

/* Box-Muller on one Philox block: out[lane] for lanes 0..3. */
static void block_normals(const uint32_t x[4], double out[4])
{
    for (int p = 0; p < 4; p += 2) {
        double ua = unit_open(x[p]);
        double ub = unit_angle(x[p + 1]);
        double rho = sqrt(-2.0 * log(ua));
        double ang = 2.0 * M_PI * ub;
        out[p] = rho * cos(ang);
        out[p + 1] = rho * sin(ang);
    }
}

/* The Gaussian number of one face (the definition every other draw follows). */
double or_normal(uint64_t seed, uint32_t realisation, uint32_t tag,
                 uint64_t step, uint64_t face)
{
    uint32_t x[4];
    double z[4];
    block_words(seed, realisation, tag, step, face >> 2, x);
    block_normals(x, z);
    return z[face & 3];
}

/* count consecutive face numbers starting at face0 */
void or_normals(uint64_t seed, uint32_t realisation, uint32_t tag, uint64_t step,
                uint64_t face0, int64_t count, double *out)
{
    for (int64_t i = 0; i < count; ++i)
        out[i] = or_normal(seed, realisation, tag, step, face0 + (uint64_t)i);
}

/* Threads of the parallel loops (n < 1: all the runtime offers). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* loops shorter than this run on one thread (fork/join costs more) */
#define OR_PAR_MIN 4096

/* All faces 0..nfaces-1 of one step: each Philox block is evaluated once and
 * its four lanes handed to the four faces it covers. */
static void draw_faces(const or_desc *d, uint32_t tag, uint64_t step,
                       int64_t nfaces, double *z)
{
    int64_t nblocks = (nfaces + 3) / 4;
#pragma omp parallel for schedule(static) if (nfaces >= OR_PAR_MIN)
    for (int64_t b = 0; b < nblocks; ++b) {
        uint32_t x[4];
        double g[4];
        block_words(d->seed, d->realisation, tag, step, (uint64_t)b, x);
        block_normals(x, g);
        for (int l = 0; l < 4; ++l)
            if (4 * b + l < nfaces) z[4 * b + l] = g[l];
    }
}

/* ---------------------------------------------------------------- grid */

int64_t or_ncells(const or_desc *d)
{
    return (int64_t)d->n[0] * d->n[1] * d->n[2];
}

int64_t or_nfaces(const or_desc *d)
{
    if (d->dim == 1) return d->bc == 1 ? d->n[0] + 1 : d->n[0];
    return (int64_t)d->dim * or_ncells(d);
}

static int check_desc(const or_desc *d)
{
    if (d->dim < 1 || d->dim > 3) return -1;
    for (int a = 0; a < 3; ++a) {
        if (d->n[a] < 1) return -1;
        if (a >= d->dim && d->n[a] != 1) return -1;
    }
    if (d->bc == 1 && d->dim != 1) return -1;
    if (d->bc != 0 && d->bc != 1) return -1;
    if (d->eq != 0 && d->eq != 1 && d->eq != 2) return -1;
    if (d->eq == 2 && d->dim != 1) return -1;
    if (d->scheme < 0 || d->scheme > 3) return -1;
    if (d->scheme >= 2 && (d->dim != 1 || d->eq == 2)) return -1;
    if (d->scheme >= 2 && d->bc == 0 && d->n[0] < 3) return -1;
    if (d->noise < 0 || d->noise > 2) return -1;
    if (d->dim == 1 && d->bc == 0 && d->n[0] < 2) return -1;
    if ((d->face_r || d->face_s || d->cell_w) && d->dim != 1) return -1;
    if ((d->face_r != NULL) != (d->face_s != NULL)) return -1;
    return 0;
}

/* Steady deterministic profile at cell centres: uniform u0 (periodic), or the
 * linear profile between the walls (Dirichlet), x_i = (i + 1/2) dx. */
void or_reference(const or_desc *d, double *ref)
{
    int64_t nc = or_ncells(d);
    for (int64_t i = 0; i < nc; ++i) {
        if (d->bc == 1)
            ref[i] = d->u_left + (d->u_right - d->u_left) * ((double)i + 0.5) / d->n[0];
        else
            ref[i] = d->u0;
    }
}

/* Initial state: the steady profile plus, if init_sd > 0, init_sd * N per
 * cell from tag 1 at step 0 with face number = cell number. */
int or_init(const or_desc *d, double *u)
{
    if (check_desc(d)) return -1;
    or_reference(d, u);
    if (d->init_sd > 0.0) {
        int64_t nc = or_ncells(d);
        double *z = (double *)malloc(sizeof(double) * (size_t)nc);
        if (!z) return -2;
        draw_faces(d, 1u, 0u, nc, z);
        for (int64_t i = 0; i < nc; ++i) u[i] += d->init_sd * z[i];
        free(z);
    }
    return 0;
}

/* Noise amplitude of a face whose (mean or deterministic) value is v. */
static double amplitude(const or_desc *d, double v, int64_t *clamps)
{
    if (d->eq == 0) return v;
    const double q = d->eq == 2 ? v * (1.0 - v) : v;   /* Burgers: c (1 - c) */
    if (q < 0.0) {
        if (clamps) ++*clamps;
        return 0.0;
    }
    return sqrt(q);
}

/* out[i] = sum over directions of (flux through the high face of i) minus
 * (flux through the low face of i), where the flux through the face between
 * cells a (low side) and b (high side) is r (U_b - U_a) + sigma A(U_face) Z. */
static void divergence(const or_desc *d, const double *u, const double *z,
                       double *flux, double *out, int64_t *clamps)
{
    const double r = d->r, s = d->sigma;
    const int noisy = d->noise != 2;
    if (d->dim == 1) {
        const int64_t N = d->n[0];
        /* per-face conductance and noise factor (uniform unless given) */
#define RF(f) (d->face_r ? d->face_r[f] : r)
#define SF(f) (d->face_s ? d->face_s[f] : s)
        /* Burgers hyperbolic flux through a face with value c (times nu) */
#define HYP(c) (d->eq == 2 ? d->nu * (c) * (1.0 - (c)) : 0.0)
        if (d->bc == 1) {
            const double wall = sqrt(2.0);
            for (int64_t f = 0; f <= N; ++f) {
                double fl;
                if (f == 0) {
                    fl = 2.0 * RF(0) * (u[0] - d->u_left) - HYP(d->u_left);
                    if (noisy) fl += wall * SF(0) * amplitude(d, d->u_left, clamps) * z[0];
                } else if (f == N) {
                    fl = 2.0 * RF(N) * (d->u_right - u[N - 1]) - HYP(d->u_right);
                    if (noisy) fl += wall * SF(N) * amplitude(d, d->u_right, clamps) * z[N];
                } else {
                    fl = RF(f) * (u[f] - u[f - 1]) - HYP(0.5 * (u[f - 1] + u[f]));
                    if (noisy) {
                        double v = d->noise == 1
                                       ? d->u_left + (d->u_right - d->u_left) * (double)f / N
                                       : 0.5 * (u[f - 1] + u[f]);
                        fl += SF(f) * amplitude(d, v, clamps) * z[f];
                    }
                }
                flux[f] = fl;
            }
            for (int64_t i = 0; i < N; ++i) out[i] = flux[i + 1] - flux[i];
        } else {
            for (int64_t f = 0; f < N; ++f) {
                int64_t a = (f + N - 1) % N;
                double fl = RF(f) * (u[f] - u[a]) - HYP(0.5 * (u[a] + u[f]));
                if (noisy) {
                    double v = d->noise == 1 ? d->u0 : 0.5 * (u[a] + u[f]);
                    fl += SF(f) * amplitude(d, v, clamps) * z[f];
                }
                flux[f] = fl;
            }
            for (int64_t i = 0; i < N; ++i) out[i] = flux[(i + 1) % N] - flux[i];
        }
#undef RF
#undef SF
#undef HYP
        if (d->cell_w)
            for (int64_t i = 0; i < N; ++i) out[i] = d->cell_w[i] * out[i];
        return;
    }
    /* 2D / 3D periodic */
    const int dim = d->dim;
    const int64_t nx = d->n[0], ny = d->n[1], nz = d->n[2];
    const int64_t nc = nx * ny * nz;
    int64_t ncl = 0;   /* clamps of this call (integer sum: order-free) */
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : ncl) if (nc >= OR_PAR_MIN)
    for (int64_t zc = 0; zc < nz; ++zc)
        for (int64_t yc = 0; yc < ny; ++yc)
            for (int64_t xc = 0; xc < nx; ++xc) {
                int64_t c = (zc * ny + yc) * nx + xc;
                for (int e = 0; e < dim; ++e) {
                    int64_t xa = xc, ya = yc, za = zc;
                    if (e == 0) xa = (xc + nx - 1) % nx;
                    if (e == 1) ya = (yc + ny - 1) % ny;
                    if (e == 2) za = (zc + nz - 1) % nz;
                    int64_t a = (za * ny + ya) * nx + xa;
                    double fl = r * (u[c] - u[a]);
                    if (noisy) {
                        int64_t face = ((zc * ny + yc) * dim + e) * nx + xc;
                        double v = d->noise == 1 ? d->u0 : 0.5 * (u[a] + u[c]);
                        fl += s * amplitude(d, v, clamps ? &ncl : NULL) * z[face];
                    }
                    flux[c * dim + e] = fl;
                }
            }
    if (clamps) *clamps += ncl;
#pragma omp parallel for collapse(2) schedule(static) if (nc >= OR_PAR_MIN)
    for (int64_t zc = 0; zc < nz; ++zc)
        for (int64_t yc = 0; yc < ny; ++yc)
            for (int64_t xc = 0; xc < nx; ++xc) {
                int64_t c = (zc * ny + yc) * nx + xc;
                double acc = 0.0;
                for (int e = 0; e < dim; ++e) {
                    int64_t xb = xc, yb = yc, zb = zc;
                    if (e == 0) xb = (xc + 1) % nx;
                    if (e == 1) yb = (yc + 1) % ny;
                    if (e == 2) zb = (zc + 1) % nz;
                    int64_t b = (zb * ny + yb) * nx + xb;
                    acc += flux[b * dim + e] - flux[c * dim + e];
                }
                out[c] = acc;
            }
    (void)nc;
}

/* ---------------------------------------------------------------- statistics */

int32_t or_n_bins(const or_desc *d)
{
    double kmax2 = 0.0;
    for (int a = 0; a < d->dim; ++a) kmax2 += 0.25 * (double)d->n[a] * (double)d->n[a];
    return (int32_t)floor(sqrt(kmax2) + 0.5) + 1;
}

static int64_t signed_k(int64_t k, int64_t n)
{
    return 2 * k < n ? k : k - n;
}

/* Radial shell of a Fourier mode: round(|k|) with signed wavenumbers in
 * [-N/2, N/2). */
static int64_t mode_bin(const or_desc *d, int64_t kx, int64_t ky, int64_t kz)
{
    double sx = (double)signed_k(kx, d->n[0]);
    double sy = (double)signed_k(ky, d->n[1]);
    double sz = (double)signed_k(kz, d->n[2]);
    return (int64_t)floor(sqrt(sx * sx + sy * sy + sz * sz) + 0.5);
}

/* Number of Fourier modes in each radial shell (n_bins entries). */
void or_bin_modes(const or_desc *d, double *modes)
{
    int32_t nb = or_n_bins(d);
    for (int32_t b = 0; b < nb; ++b) modes[b] = 0.0;
    for (int64_t kz = 0; kz < d->n[2]; ++kz)
        for (int64_t ky = 0; ky < d->n[1]; ++ky)
            for (int64_t kx = 0; kx < d->n[0]; ++kx) {
                int64_t b = mode_bin(d, kx, ky, kz);
                if (b < nb) modes[b] += 1.0;
            }
}

/* In-place DFT X_k = sum_j x_j exp(-2 pi i j k / n) along one axis of a
 * complex field (re, im), evaluated by its definition. */
static void dft_axis(const or_desc *d, int axis, double *re, double *im)
{
    const int64_t nx = d->n[0], ny = d->n[1], nz = d->n[2];
    const int64_t n = d->n[axis];
    const int64_t stride = axis == 0 ? 1 : (axis == 1 ? nx : nx * ny);
    const int64_t l0 = axis == 2 ? 1 : nz, l1 = axis == 1 ? 1 : ny, l2 = axis == 0 ? 1 : nx;
#pragma omp parallel if (l0 * l1 * l2 * n >= OR_PAR_MIN)
    {
        double *tr = (double *)malloc(sizeof(double) * (size_t)n);
        double *ti = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for collapse(3) schedule(static)
        for (int64_t zc = 0; zc < l0; ++zc)
            for (int64_t yc = 0; yc < l1; ++yc)
                for (int64_t xc = 0; xc < l2; ++xc) {
                    int64_t base = (zc * ny + yc) * nx + xc;
                    for (int64_t k = 0; k < n; ++k) {
                        double sr = 0.0, si = 0.0;
                        for (int64_t j = 0; j < n; ++j) {
                            double ang = -2.0 * M_PI * (double)((j * k) % n) / (double)n;
                            double c = cos(ang), s = sin(ang);
                            double xr = re[base + j * stride], xi = im[base + j * stride];
                            sr += xr * c - xi * s;
                            si += xr * s + xi * c;
                        }
                        tr[k] = sr;
                        ti[k] = si;
                    }
                    for (int64_t k = 0; k < n; ++k) {
                        re[base + k * stride] = tr[k];
                        im[base + k * stride] = ti[k];
                    }
                }
        free(tr);
        free(ti);
    }
}

/* Returns 1 if the state holds a non-finite value (then nothing is added). */
static int take_sample(const or_desc *d, const double *u, const double *ref,
                       or_stats *st, int64_t t)
{
    const int64_t nc = or_ncells(d);
    for (int64_t i = 0; i < nc; ++i)
        if (!isfinite(u[i])) {
            st->nonfinite = 1;
            st->nonfinite_step = t;
            return 1;
        }
    /* the batch this sample belongs to (-1: none kept) */
    int64_t bs = -1;
    if (st->batch_len > 0 && st->n_samples / st->batch_len < st->batch_cap) bs = st->n_samples / st->batch_len;
    double a = 0.0, b = 0.0;
    for (int64_t i = 0; i < nc; ++i) {
        double del = u[i] - ref[i];
        if (st->s1) st->s1[i] += del;
        if (st->s2) st->s2[i] += del * del;
        if (bs >= 0 && st->b_s1) st->b_s1[bs * nc + i] += del;
        if (bs >= 0 && st->b_s2) st->b_s2[bs * nc + i] += del * del;
        a += del;
        b += del * del;
    }
    a /= (double)nc;
    b /= (double)nc;
    st->sp_mean += a;
    st->sp_sq += b;
    st->sp_var += b - a * a;
    if (bs >= 0 && st->b_sp) {
        st->b_sp[bs * 3 + 0] += a;
        st->b_sp[bs * 3 + 1] += b;
        st->b_sp[bs * 3 + 2] += b - a * a;
    }
    if (st->m2 && d->dim == 1) {
        for (int64_t i = 0; i < nc; ++i)
            for (int64_t j = 0; j < nc; ++j)
                st->m2[i * nc + j] += (u[i] - ref[i]) * (u[j] - ref[j]);
    }
    if (st->tc && st->tc_lags > 0 && d->dim == 1) {
        /* this sample is number n; sample n - m sits in ring slot (n - m) mod L */
        const int64_t L = st->tc_lags, n = st->n_samples;
        double *now = st->tc_hist + (n % L) * nc;
        for (int64_t i = 0; i < nc; ++i) now[i] = u[i] - ref[i];
        for (int64_t m = 0; m < L && m <= n; ++m) {
            const double *past = st->tc_hist + ((n - m) % L) * nc;
            for (int64_t i = 0; i < nc; ++i) st->tc[m * nc + i] += now[i] * past[i];
        }
    }
    if (st->sk) {
        double *re = (double *)calloc((size_t)nc, sizeof(double));
        double *im = (double *)calloc((size_t)nc, sizeof(double));
        for (int64_t i = 0; i < nc; ++i) re[i] = u[i];
        for (int axis = 0; axis < d->dim; ++axis) dft_axis(d, axis, re, im);
        double *bsk = (bs >= 0 && st->b_sk) ? st->b_sk + bs * (d->dim == 1 ? nc : st->n_bins) : NULL;
        if (d->dim == 1) {
            for (int64_t k = 0; k < nc; ++k) {
                st->sk[k] += re[k] * re[k] + im[k] * im[k];
                if (bsk) bsk[k] += re[k] * re[k] + im[k] * im[k];
            }
        } else {
            for (int64_t kz = 0; kz < d->n[2]; ++kz)
                for (int64_t ky = 0; ky < d->n[1]; ++ky)
                    for (int64_t kx = 0; kx < d->n[0]; ++kx) {
                        int64_t b2 = mode_bin(d, kx, ky, kz);
                        int64_t i = (kz * d->n[1] + ky) * d->n[0] + kx;
                        if (b2 < st->n_bins) {
                            st->sk[b2] += re[i] * re[i] + im[i] * im[i];
                            if (bsk) bsk[b2] += re[i] * re[i] + im[i] * im[i];
                        }
                    }
        }
        free(re); free(im);
    }
    st->n_samples += 1;
    return 0;
}

/* ---------------------------------------------------------------- stepping */

/* Rows of M = I - theta W A for the 1D implicit schemes: lo[i], di[i], up[i]
 * multiply U_(i-1), U_i, U_(i+1) (cyclic for periodic rods).  A U is the
 * noise-free flux divergence without the wall terms: face conductances r_f,
 * a Dirichlet wall face 2 r_f on the diagonal. */
static void implicit_rows(const or_desc *d, double theta, double *lo, double *di, double *up)
{
    const int64_t N = d->n[0];
    const int dir = d->bc == 1;
    for (int64_t i = 0; i < N; ++i) {
        const int64_t fl = i, fh = dir ? i + 1 : (i + 1) % N;
        const double rl = d->face_r ? d->face_r[fl] : d->r;
        const double rh = d->face_r ? d->face_r[fh] : d->r;
        const double w = d->cell_w ? d->cell_w[i] : 1.0;
        const double dl = (dir && i == 0) ? 2.0 * rl : rl;
        const double dh = (dir && i == N - 1) ? 2.0 * rh : rh;
        di[i] = 1.0 + theta * w * (dl + dh);
        lo[i] = (dir && i == 0) ? 0.0 : -theta * w * rl;
        up[i] = (dir && i == N - 1) ? 0.0 : -theta * w * rh;
    }
}

/* Thomas algorithm for lo[i] x_(i-1) + di[i] x_i + up[i] x_(i+1) = rhs[i],
 * lo[0] and up[N-1] unused.  work: N doubles. */
static void thomas(int64_t N, const double *lo, const double *di, const double *up, const double *rhs,
                   double *x, double *work)
{
    double den = di[0];
    x[0] = rhs[0] / den;
    for (int64_t i = 1; i < N; ++i) {
        work[i] = up[i - 1] / den;
        den = di[i] - lo[i] * work[i];
        x[i] = (rhs[i] - lo[i] * x[i - 1]) / den;
    }
    for (int64_t i = N - 2; i >= 0; --i) x[i] -= work[i + 1] * x[i + 1];
}

/* Cyclic system (lo[0] couples x_(N-1), up[N-1] couples x_0): write it as a
 * tridiagonal T plus the rank-one u v^T with u = (g, 0, .., 0, up[N-1]),
 * v = (1, 0, .., 0, lo[0]/g), g = -di[0], and apply Sherman-Morrison:
 * x = y - (v.y / (1 + v.z)) z with T y = rhs, T z = u.  work: 4N doubles. */
static void cyclic_thomas(int64_t N, const double *lo, const double *di, const double *up, const double *rhs,
                          double *x, double *work)
{
    double *dt = work, *uu = work + N, *zz = work + 2 * N, *w = work + 3 * N;
    const double g = -di[0], alpha = up[N - 1], beta = lo[0];
    for (int64_t i = 0; i < N; ++i) {
        dt[i] = di[i];
        uu[i] = 0.0;
    }
    dt[0] -= g;
    dt[N - 1] -= alpha * beta / g;
    uu[0] = g;
    uu[N - 1] = alpha;
    thomas(N, lo, dt, up, rhs, x, w);
    thomas(N, lo, dt, up, uu, zz, w);
    const double f = (x[0] + beta * x[N - 1] / g) / (1.0 + zz[0] + beta * zz[N - 1] / g);
    for (int64_t i = 0; i < N; ++i) x[i] -= f * zz[i];
}

/* Advance u by nsteps steps; the step taken from completed-step count t uses
 * the noise of step t (tag 0).  With st != NULL the state is sampled after
 * every completed step t with t > burn_in and t % every == 0.  Returns 0, or
 * 1 if a sample met a non-finite value (the state is left as it was then),
 * or a negative number for an invalid description / allocation failure. */
int or_advance(const or_desc *d, double *u, int64_t step0, int64_t nsteps, or_stats *st)
{
    if (check_desc(d)) return -1;
    const int64_t nc = or_ncells(d), nf = or_nfaces(d);
    double *z = (double *)calloc((size_t)nf, sizeof(double));
    double *flux = (double *)calloc((size_t)(nf > d->dim * nc ? nf : d->dim * nc), sizeof(double));
    double *div = (double *)malloc(sizeof(double) * (size_t)nc);
    double *us = (double *)malloc(sizeof(double) * (size_t)nc);
    double *ref = (double *)malloc(sizeof(double) * (size_t)nc);
    if (!z || !flux || !div || !us || !ref) return -2;
    /* implicit schemes: matrix rows, noise-free divergence, right-hand side */
    const int impl = d->scheme >= 2;
    const double theta = d->scheme == 2 ? 1.0 : 0.5;
    double *lo = NULL, *di = NULL, *up = NULL, *det = NULL, *work = NULL;
    or_desc dq = *d;
    dq.noise = 2;
    if (impl) {
        lo = (double *)malloc(sizeof(double) * (size_t)nc);
        di = (double *)malloc(sizeof(double) * (size_t)nc);
        up = (double *)malloc(sizeof(double) * (size_t)nc);
        det = (double *)malloc(sizeof(double) * (size_t)nc);
        work = (double *)malloc(sizeof(double) * 4 * (size_t)nc);
        if (!lo || !di || !up || !det || !work) return -2;
        implicit_rows(d, theta, lo, di, up);
    }
    or_reference(d, ref);
    int64_t *clamps = st ? &st->clamp_count : NULL;
    int rc = 0;
    for (int64_t k = 0; k < nsteps; ++k) {
        const uint64_t n = (uint64_t)(step0 + k);
        if (d->noise != 2) draw_faces(d, 0u, n, nf, z);
        divergence(d, u, z, flux, div, clamps);
        if (impl) {
            /* rhs = U + full - theta det + theta W b (W b: the wall terms of det) */
            const int64_t N = nc;
            divergence(&dq, u, z, flux, det, NULL);
            for (int64_t i = 0; i < N; ++i) us[i] = u[i] + div[i] - theta * det[i];
            if (d->bc == 1) {
                const double r0 = d->face_r ? d->face_r[0] : d->r, rN = d->face_r ? d->face_r[N] : d->r;
                us[0] += theta * (d->cell_w ? d->cell_w[0] : 1.0) * 2.0 * r0 * d->u_left;
                us[N - 1] += theta * (d->cell_w ? d->cell_w[N - 1] : 1.0) * 2.0 * rN * d->u_right;
                thomas(N, lo, di, up, us, u, work);
            } else {
                cyclic_thomas(N, lo, di, up, us, u, work);
            }
        } else if (d->scheme == 0) {
#pragma omp parallel for schedule(static) if (nc >= OR_PAR_MIN)
            for (int64_t i = 0; i < nc; ++i) u[i] = u[i] + div[i];
        } else {
#pragma omp parallel for schedule(static) if (nc >= OR_PAR_MIN)
            for (int64_t i = 0; i < nc; ++i) us[i] = u[i] + div[i];
            divergence(d, us, z, flux, div, clamps);
#pragma omp parallel for schedule(static) if (nc >= OR_PAR_MIN)
            for (int64_t i = 0; i < nc; ++i) u[i] = 0.5 * (u[i] + us[i] + div[i]);
        }
        const int64_t t = step0 + k + 1;
        if (st && t > st->burn_in && st->every > 0 && t % st->every == 0) {
            if (take_sample(d, u, ref, st, t)) {
                rc = 1;
                break;
            }
        }
    }
    free(z); free(flux); free(div); free(us); free(ref);
    free(lo); free(di); free(up); free(det); free(work);
    return rc;
}
