/*
 * she.h -- C ABI of the MI355X (gfx950) library for the finite-volume
 * stochastic heat equation (SHE) and its Dean-Kawasaki (DK) species analogue.
 *
 * Method (Garcia, Bell, Nonaka, Srivastava, Ladiges, Kim, "An Introduction to
 * Computational Fluctuating Hydrodynamics"):
 *   - Sec. 3, FE scheme:  U_i += r (U_{i+1} - 2U_i + U_{i-1})
 *                              + sigma (A_{i+1/2} N_{i+1/2} - A_{i-1/2} N_{i-1/2})
 *     with sigma = sqrt(2 r eps), r = kappa dt/dx^2, eps = k_B/(rho c_V dV),
 *     face amplitude A = T_face = (T_i + T_{i+1})/2 (SHE, Sec. 3) or
 *     A = sqrt(max(n_face, 0)) with eps = 1/dV (DK, Sec. 4 eq. DK), and one
 *     standard normal N per face per step (Sec. 3 discrete noise);
 *   - Sec. 3, PC scheme: FE predictor U*, then
 *     U^{n+1} = (U^n + U* + Delta(U*; same N)) / 2;
 *   - Sec. 3, Dirichlet walls: ghost stencil (U_1 - 3U_0 + 2U_L) and wall-face
 *     noise sqrt(2) A(U_L) N (1D only; 2D/3D grids are periodic);
 *   - Sec. 3, statistics: time averages after a relaxation period, variance,
 *     two-point correlation <dU_i dU_j>, structure factor <|U_k|^2>.
 *   In 2D/3D every direction has its own independent face numbers (white noise
 *   with independent Cartesian components, Sec. 2 eq. GWN) and the cells are
 *   cubes of volume dV.
 *
 * Noise: Philox4x32-10 (Salmon et al., SC'11) + Box-Muller.  Counter of the
 * block holding face f at step n with stream tag g and realisation q:
 *     (f >> 2, n mod 2^32, ((n >> 32) & 0xFFFF) | g << 16, q),
 * key (seed mod 2^32, seed div 2^32); lane f & 3; lanes (0,1) and (2,3) are
 * Box-Muller pairs with u = ((word >> 9) + 1/2) 2^-23, even lane
 * sqrt(-2 ln u_a) cos(2 pi u_b), odd lane ... sin(2 pi u_b).  Tag 0 = step
 * noise, tag 1 = initial perturbation (face number = cell number).
 * Face numbers: 1D f = low (left) face of cell f, f = 0..N-1 periodic,
 * 0..N Dirichlet (f = N is the right wall); 2D/3D the low face of cell
 * (x,y,z) in direction e is ((z*Ny + y)*dim + e)*Nx + x.
 *
 * Conventions for every call:
 *   - every function returns she_status (0 = SHE_OK, < 0 = error);
 *     she_last_error() gives a message; no exception crosses the ABI;
 *   - all GPU work is enqueued on the stream given in she_config (NULL = the
 *     null stream); she_step / she_run return without waiting; she_stats,
 *     she_read_field, she_get_state synchronise that stream;
 *   - host pointers are caller-owned and only read/written during the call;
 *   - one handle must not be used from two host threads at once;
 *   - device memory is allocated at she_create and freed at she_destroy,
 *     or carved from a caller-owned device arena (she_config.arena), which the
 *     caller keeps alive until she_destroy.
 */
#ifndef SHE_H
#define SHE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct she_handle she_handle;

typedef enum {
    SHE_OK = 0,
    SHE_EINVAL = -1,       /* invalid argument or configuration               */
    SHE_EUNSTABLE = -2,    /* r above the explicit stability limit 1/(2 dim)  */
    SHE_ENOMEM = -3,       /* device allocation failed / arena too small      */
    SHE_EDEVICE = -4,      /* HIP runtime error                               */
    SHE_ENONFINITE = -5,   /* a sample met a non-finite value; state frozen   */
    SHE_ESTATE = -6,       /* checkpoint blob does not match this handle      */
    SHE_EUNSUPPORTED = -7  /* valid in the method, not provided by a kernel   */
} she_status;

/* equation: SHE (Sec. 2 eq. SHE), Dean-Kawasaki species diffusion (Sec. 4
 * eq. DK), stochastic Burgers (Sec. 5, 1D: hyperbolic flux a c (1-c), noise
 * sqrt(2 D c (1-c)); the same face-flux scheme with the arithmetic face value) */
enum { SHE_HEAT = 0, SHE_SPECIES = 1, SHE_BURGERS = 2 };
enum { SHE_PERIODIC = 0, SHE_DIRICHLET = 1 };                 /* x boundary    */
/* scheme: forward Euler, predictor-corrector (Sec. 3); backward Euler and
 * Crank-Nicolson for the deterministic flux with the noise explicit (1D heat /
 * species; the implicit-scheme exercise, Sec. 6): no stability limit on r */
enum { SHE_EM = 0, SHE_HEUN = 1, SHE_BE = 2, SHE_CN = 3 };
enum { SHE_NOISE_INSTANT = 0, SHE_NOISE_FROZEN = 1, SHE_NOISE_OFF = 2 };
enum { SHE_F32 = 0, SHE_F64 = 1 };                            /* state type    */

/* statistics selected in she_config.stats_mask */
enum {
    SHE_STAT_MOMENTS = 1,  /* 1D: per-cell FP64 sums of dU and dU^2           */
    SHE_STAT_CORR = 2,     /* 1D: full N x N covariance (MFMA X^T X blocks)   */
    SHE_STAT_SK = 4,       /* nD: radially binned S(k) (FFT per sample);
                              1D: S_k comes from the covariance (needs CORR)  */
    SHE_STAT_SPATIAL = 8,  /* per-instance spatial mean / variance per sample */
    SHE_STAT_TCORR = 16    /* 1D: time correlation <dU_i^n dU_i^(n-m)> over
                              sample lags m < tcorr_lags (first suggested
                              exercise, Sec. 6); implies MOMENTS             */
};

/* she_config.tuning_flags: launch-order choices (results are identical) */
enum {
    SHE_TUNE_XCD_ORDER = 1,       /* 2D/3D: give each XCD a contiguous range of
                                     workgroups (neighbouring chunks share an
                                     L2) instead of the plain order; measured
                                     no faster on MI355X, so off by default   */
    SHE_TUNE_SEARCH = 2,          /* she_create runs she_tune first and uses
                                     its choice (not with an arena)          */
    SHE_TUNE_SINGLE_STEP = 4      /* 2D FE: one step per launch.  By default
                                     direct (not graph-replayed) steps go two
                                     per launch, the intermediate field kept
                                     on chip, wherever at most one of the two
                                     samples (the first only for FP32 states,
                                     and with SHE_STAT_SK only where the step
                                     kernel transforms the rows: Nx 512 or
                                     1024); fields and S(k) are the same bits,
                                     spatial moments the same to rounding    */
};

/* she_config.flags */
enum {
    SHE_ALLOW_UNSTABLE = 1        /* create instances whose second moment grows
                                     without bound (see she_create); their runs
                                     end in a non-finite sample, SHE_ENONFINITE
                                     and a frozen state.  For tests of that
                                     path.                                    */
};

/* One instance (realisation) of the scheme.  Dirichlet walls only in 1D. */
typedef struct {
    int32_t dim;          /* 1, 2, 3                                          */
    int32_t n[3];         /* cells per axis, unused axes = 1.  2D/3D: n[0] a
                             power of two in [8, 1024]                         */
    int32_t eq;           /* SHE_HEAT, SHE_SPECIES or SHE_BURGERS (1D)        */
    int32_t bc;           /* SHE_PERIODIC or SHE_DIRICHLET (dim == 1)         */
    int32_t scheme;       /* SHE_EM, SHE_HEUN, SHE_BE or SHE_CN (1D)          */
    int32_t noise;        /* SHE_NOISE_*: face amplitude from the current
                             state (paper's practice), from the deterministic
                             profile (footnote of Sec. 2), or no noise        */
    double r;             /* kappa dt/dx^2 (SHE) or D dt/dx^2 (DK)            */
    double eps;           /* k_B/(rho c_V dV) (SHE) or 1/dV (DK)               */
    double u0;            /* periodic: initial and reference value             */
    double u_left;        /* Dirichlet wall values (x = 0 and x = L)           */
    double u_right;
    double init_sd;       /* std. dev. of the initial perturbation (tag 1)     */
    uint64_t seed;        /* Philox key                                        */
    uint32_t realisation; /* Philox counter word 3                             */
    uint32_t reserved;    /* must be 0                                         */
    const double *cond;   /* 1D, optional (NULL = uniform): N conductivity
                             ratios lambda_i / lambda_ref > 0 per cell, for a
                             material that varies along the rod (composite
                             rod exercise, Sec. 6).  r refers to lambda_ref;
                             a face conducts like its two half cells in
                             series, a wall face like its cell.  Read during
                             she_create / she_arena_bytes only.              */
    const double *cap;    /* 1D, optional: N heat-capacity ratios
                             (rho c_V)_i / (rho c_V)_ref > 0; eps refers to
                             the reference material.  With cond or cap the
                             step is U_i += (F_(i+1) - F_i) / cap_i, F_f =
                             r_f dU + sqrt(2 r_f eps) A_f N_f (r_f = r times
                             the face conductivity ratio); FE stability needs
                             max_i (sum of the conductances of row i) /
                             cap_i <= 2, else SHE_EUNSTABLE.  Deterministic
                             face values (SHE_NOISE_FROZEN) need
                             u_left == u_right.                              */
    double nu;            /* SHE_BURGERS: Courant number a dt / dx (the flux
                             gains -nu c_f (1 - c_f)); must be 0 otherwise.
                             SHE_EUNSTABLE unless every mode's one-step factor
                             of the linearised scheme, at the steepest slope
                             |1 - 2c| = 1, has modulus <= 1.                 */
} she_instance_desc;

typedef struct {
    int32_t n_instances;
    int32_t precision;            /* SHE_F32 or SHE_F64 for the state         */
    const she_instance_desc *inst;/* n_instances entries, copied at create.
                                     1D instances may differ in every field;
                                     2D/3D instances must share the grid,
                                     eq, scheme, noise and seed (r, u0, eps,
                                     init_sd and realisation may differ;
                                     otherwise SHE_EUNSUPPORTED)             */
    int64_t burn_in;              /* sample after completed step t when
                                     t > burn_in and t % sample_every == 0    */
    int32_t sample_every;         /* >= 1                                      */
    uint32_t stats_mask;          /* SHE_STAT_* bits                           */
    int32_t block_threads;        /* tuning: 1D threads per workgroup: 0 (auto),
                                     64, 256 or 512, or 1024 for an FP32
                                     batch of FE/PC heat instances with
                                     instantaneous noise, uniform material
                                     and stats_mask 0; an instance
                                     takes whole waves of a workgroup, small
                                     instances share one                    */
    int32_t rows_per_block;       /* tuning: 2D/3D march length (0 auto)      */
    int32_t rows_per_group;       /* tuning: 3D rows per workgroup (0 auto)   */
    int32_t tuning_flags;         /* SHE_TUNE_* bits (0 = defaults)           */
    int32_t graph_steps;          /* 2D/3D: record K >= 1 steps into a HIP
                                     graph and replay it (K is rounded up to a
                                     multiple of 2, and of sample_every for
                                     she_run); 0 launches every step directly.
                                     Results are identical.  Ignored in 1D.  */
    int32_t tcorr_lags;           /* TCORR: lags L in sampling intervals,
                                     1..1024 (0 without TCORR)               */
    int32_t batch_samples;        /* batch-means error bars: samples per batch
                                     L >= 1 (0: none).  Samples 1..L form batch
                                     0, L+1..2L batch 1, ...; each statistic is
                                     also formed per complete batch, and its
                                     standard error is the standard deviation
                                     of the B batch values (divisor B - 1) over
                                     sqrt(B) (time averages after relaxation,
                                     Sec. 3).  Needs stats_mask != 0.         */
    uint32_t flags;               /* SHE_ALLOW_UNSTABLE, or 0                 */
    void *stream;                 /* hipStream_t (e.g. torch's current stream)*/
    void *arena;                  /* optional device memory for all buffers   */
    size_t arena_bytes;
} she_config;

/* Results of one instance; caller-owned arrays with their capacities (in
 * elements).  A NULL array is skipped; a too small capacity is SHE_EINVAL. */
typedef struct {
    int64_t n_samples;            /* samples taken since create / reset       */
    int64_t steps;                /* completed steps                           */
    double *mean;   int64_t mean_cap;  /* 1D: N time-averaged U_i;
                                          nD: 1, time-averaged spatial mean   */
    double *var;    int64_t var_cap;   /* 1D: N population variances;
                                          nD: 1, time-averaged spatial var.   */
    double *corr;   int64_t corr_cap;  /* 1D + CORR: N*N covariance, row-major */
    double *sk;     int64_t sk_cap;    /* 1D + CORR: N values <|U_k|^2>;
                                          nD + SK: shell averages, shell
                                          round(|k|), signed k in [-N/2,N/2)  */
    double *sk_modes; int64_t sk_modes_cap; /* nD: modes per shell            */
    double sum_u;                 /* current sum of U over the cells (FP64)   */
    int32_t nonfinite;            /* 1 if a sample met a non-finite value      */
    int32_t reserved;
    int64_t clamp_count;          /* DK: face evaluations with negative mean  */
    double *tcorr;  int64_t tcorr_cap; /* 1D + TCORR: L*N values [m][i],
                                          C_i(m) = S_i(m)/(M-m) - mu_i^2 with
                                          S_i(m) the sum over sample pairs
                                          (n, n-m) of dU_i(n) dU_i(n-m),
                                          mu_i = S1_i/M, M samples; NaN for
                                          m >= M                              */
    /* Batch-means standard errors (she_config.batch_samples = L > 0): B =
     * floor(M / L) complete batches, SE = sqrt(sum_b (x_b - xbar)^2 /
     * (B (B - 1))) over the batch values x_b of the statistic, each formed
     * like the statistic itself from the L samples of its batch; NaN while
     * B < 2.  The statistics above use all M samples, the error bars the
     * complete batches. */
    int64_t n_batches;
    double *mean_se; int64_t mean_se_cap; /* 1D + MOMENTS: N; nD: 1           */
    double *var_se;  int64_t var_se_cap;  /* 1D + MOMENTS: N; nD: 1           */
    double *sk_se;   int64_t sk_se_cap;   /* 1D + CORR: N; nD + SK: shells     */
    double spatial_var;           /* time average over the samples of the
                                     spatial variance of U (every dim; nD: =
                                     var[0]): (1/n) sum_i dU_i^2 - ((1/n)
                                     sum_i dU_i)^2 per sample, n cells       */
    double spatial_var_se;        /* its standard error (NaN: no batches)      */
} she_stats_out;

/* Validate cfg, allocate device buffers, write the initial state (steady
 * profile + init_sd * N(tag 1)).  Errors:
 *   - r > 1/(2 dim) (explicit schemes): SHE_EUNSTABLE;
 *   - a periodic FE heat instance with instantaneous noise whose second
 *     moment has no stationary value, eps * beta >= 1 with beta = (1/n)
 *     sum over the modes k != 0 of h_k cos^2(pi k_x / n_x), h_k = 1 / (1 -
 *     x_k / 2), x_k = 4 r sum_d sin^2(pi k_d / n_d) (n cells; the face
 *     temperature's variance feeds the noise, stationary variance eps m^2
 *     gamma / (1 - eps beta): FE scheme and noise of Sec. 3):
 *     SHE_EUNSTABLE unless flags has SHE_ALLOW_UNSTABLE (other schemes and
 *     boundaries are not checked; their divergence ends in SHE_ENONFINITE);
 *   - periodic with u_left != u_right, or Dirichlet in 2D/3D: SHE_EINVAL
 *     (the paper's program refuses a gradient with periodic walls). */
she_status she_create(const she_config *cfg, she_handle **out);

/* Bytes of device memory she_create needs for cfg (for a caller arena). */
she_status she_arena_bytes(const she_config *cfg, size_t *bytes);

/* Autotuner: time the launch shapes valid for cfg and write cfg with the
 * fastest into *tuned (block_threads for 1D; rows_per_block for 2D;
 * rows_per_block x rows_per_group for 3D).  Each candidate is a trial handle
 * (she_create without cfg->arena: it allocates), warmed up and then timed
 * over `steps` steps of she_step with events on cfg->stream (steps <= 0:
 * 2000 in 1D, 20 in 2D/3D); shapes the batch rejects are skipped.  Results
 * are identical for every shape; only the time differs.  A choice is cached
 * for the process, keyed by precision, stats_mask, the XCD-order and
 * single-step flags and each instance's sizes, boundary, scheme, equation,
 * noise mode and material; a cached key returns
 * at once.  Synchronises cfg->stream.  SHE_EUNSUPPORTED if no shape runs. */
she_status she_tune(const she_config *cfg, int32_t steps, she_config *tuned);

/* Advance every instance by nsteps time steps of its scheme (Sec. 3: the FE
 * update and the PC predictor / corrector on the face fluxes, with one fresh
 * standard normal per face per step from the counters (seed, face block,
 * step, realisation); Sec. 4 for DK) without taking samples.  h: a handle
 * from she_create; nsteps >= 0 (0: no work).  Enqueued on the handle's
 * stream and returns without waiting.  SHE_EINVAL for a NULL handle or
 * nsteps < 0; SHE_EDEVICE if a launch fails (she_last_error names the call).
 * An instance whose state turns non-finite is frozen and reported by
 * she_stats (SHE_ENONFINITE). */
she_status she_step(she_handle *h, int64_t nsteps);

/* As she_step, sampling the statistics of stats_mask after each completed
 * step t with t > burn_in and t a multiple of sample_every (Sec. 3: time
 * averages after a relaxation period, samples taken every few steps so they
 * are less correlated).  Same arguments, asynchrony and errors as she_step. */
she_status she_run(she_handle *h, int64_t nsteps);

/* Finalised statistics of one instance in FP64 (mean = ref + S1/M,
 * var = S2/M - (S1/M)^2 with the population normalisation of the paper's
 * program, cov = M2/M - m m^T, S_k).  Synchronises the stream.  Returns
 * SHE_ENONFINITE (after filling out) if a sample met a non-finite value. */
she_status she_stats(she_handle *h, int32_t instance, she_stats_out *out);

/* Zero every statistics accumulator, batch means included (the step count
 * is kept): a new relaxation period starts (Sec. 3).  Ordered on the stream;
 * SHE_EINVAL for a NULL handle. */
she_status she_reset_stats(she_handle *h);

/* Copy the current field of one instance to / from host FP64 (n = cells,
 * x fastest).  read synchronises the stream; write is ordered on it. */
she_status she_read_field(she_handle *h, int32_t instance, double *host, int64_t n);
she_status she_write_field(she_handle *h, int32_t instance, const double *host, int64_t n);

/* Completed step count of the handle. */
she_status she_get_step(const she_handle *h, int64_t *steps);

/* Checkpoint: state + step count + every statistics accumulator, as one
 * host blob.  Resuming from it reproduces the uninterrupted run bit for bit:
 * the noise of Sec. 3 (one normal per face per step) is a function of the
 * seed, face, step and realisation, not of a generator state.
 * she_state_bytes: the blob size for this handle (SHE_EINVAL for NULL).
 * she_get_state: copies the blob into caller-owned host memory of at least
 * that size; synchronises the stream (SHE_EINVAL for NULL or a short buffer).
 * she_set_state: loads a blob taken from a handle of the same layout (same
 * dimension, precision, instance count and sizes, statistics and batch
 * length); SHE_ESTATE if it is short or of another layout, and then the
 * handle is unchanged.  Synchronises the stream. */
she_status she_state_bytes(const she_handle *h, size_t *bytes);
she_status she_get_state(she_handle *h, void *host, size_t bytes);
she_status she_set_state(she_handle *h, const void *host, size_t bytes);

/* Message of the last failed call on h (h == NULL: last she_create failure
 * of this thread).  Valid until the next call on h. */
const char *she_last_error(const she_handle *h);

void she_destroy(she_handle *h);

/* Verification entry points (same kernels' device functions):
 * raw Philox4x32-10 words for count counters (host array 4*count, word 0
 * first) under key (seed lo, seed hi) -> host out[4*count]; and count
 * consecutive face normals in FP32 (precision SHE_F32) or FP64, as the step
 * kernels draw them.  Both run on `stream` and synchronise it. */
she_status she_debug_philox(uint64_t seed, const uint32_t *ctr, int64_t count,
                            uint32_t *out, void *stream);
she_status she_debug_normals(uint64_t seed, uint32_t realisation, uint32_t tag,
                             uint64_t step, uint64_t face0, int64_t count,
                             int32_t precision, double *out, void *stream);

/* she_debug_normals without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the numbers are staged in a fixed device array of
 * SHE_NOALLOC_MAX_NORMALS doubles that the library holds on each GPU it runs
 * on until the process ends, instead of a buffer allocated per call.  Same
 * arguments, same values bit for bit; count > SHE_NOALLOC_MAX_NORMALS is
 * SHE_EINVAL.  Every call on one GPU shares that array (the last call's
 * numbers stay in it): calls that overlap on one GPU, from several threads
 * or on several streams, race; serialise them.  Synchronises `stream`. */
#define SHE_NOALLOC_MAX_NORMALS (1 << 20)
she_status she_debug_normals_noalloc(uint64_t seed, uint32_t realisation, uint32_t tag,
                                     uint64_t step, uint64_t face0, int64_t count,
                                     int32_t precision, double *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SHE_H */
