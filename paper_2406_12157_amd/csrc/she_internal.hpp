// Internal types shared by the host runtime and the kernels of libshe.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace she {

constexpr int kCorrBlock = 256;  // snapshots per X^T X block (MFMA K dimension)

// One 1D instance in the ragged batch (device table entry).
struct Inst1D {
    int64_t off;        // first cell in the state pool / per-cell statistics
    int64_t x_off;      // first element of this instance's 256 x N X block, -1: none
    int64_t c_off;      // first element of this instance's N x N FP64 sum, -1: none
    int64_t h_off;      // first element of this instance's sample history ring, -1: none
    int64_t tc_off;     // first element of this instance's L x N FP64 lag sums, -1: none
    int64_t k_off;      // material coefficients r_f[nf], s_f[nf] (wall sqrt 2 included), w_i[N]
                        // in the state type, -1: uniform rod
    int32_t n;          // cells
    int32_t bc;         // 0 periodic, 1 Dirichlet
    int32_t scheme;     // 0 FE, 1 PC, 2 backward Euler, 3 Crank-Nicolson
    int32_t noise;      // 0 instantaneous, 1 frozen, 2 off
    int32_t eq;         // 0 heat, 1 species, 2 Burgers
    uint32_t realisation;
    uint64_t seed;
    double r, sigma, u0, uL, uR;
    double nu;          // Burgers: Courant number
    // implicit schemes: FP64 parallel-cyclic-reduction factors of M = I - theta W A
    // at p_off of the reduction buffer: k1[L][N], k2[L][N], 1/b[N], then (periodic)
    // the Sherman-Morrison vector z[N] and the scalars q, 1/(1 + z_0 + q z_(N-1))
    int64_t p_off;
    int32_t pcr_levels;
    int32_t pad_;
    double theta;
};

// Per-instance accumulators that are not per cell (device).
struct InstAcc {
    int64_t n_samples;
    int64_t clamp_count;
    double sum_u;       // sum of U over the cells at the last sample / step
    double sp_mean;     // sum over samples of the spatial mean of dU
    double sp_sq;       // ... of the spatial mean of dU^2
    double sp_var;      // ... of the spatial variance
    int32_t nonfinite;
    int32_t pad;
    // batch means (samples per batch L): complete batches folded so far, the
    // spatial sums at the end of the last folded batch, the FP64 Welford
    // mean / M2 over batches of the batch's spatial mean and spatial
    // variance, and the spatial-mean sum of the batch folded last
    int64_t n_batches;
    double bsp_mean, bsp_var;
    double wm_mean, wm_m2;
    double wv_mean, wv_m2;
    double batch_sp_mean;
};

// One step of Welford's update of (mean, M2) with the b-th value x (b >= 1):
// M2 / (b - 1) is the sample variance of the b values.
__host__ __device__ inline void welford(double x, double b, double &mean, double &m2)
{
    const double d = x - mean;
    mean += d / b;
    m2 += d * (x - mean);
}

// Fold a completed batch of `len` samples into an instance's spatial
// batch-means accumulators (the batch statistic is the sum over its samples
// divided by len; the sums at its start are the snapshots).
__host__ __device__ inline void fold_spatial(InstAcc &q, int32_t len)
{
    const double b = static_cast<double>(q.n_batches + 1);
    const double bm = q.sp_mean - q.bsp_mean;
    welford(bm / len, b, q.wm_mean, q.wm_m2);
    welford((q.sp_var - q.bsp_var) / len, b, q.wv_mean, q.wv_m2);
    q.batch_sp_mean = bm;
    q.bsp_mean = q.sp_mean;
    q.bsp_var = q.sp_var;
    q.n_batches += 1;
}

// Per-instance reduction of the FP64 spatial partials of a sample launch:
// the partials of instance inst summed in a fixed order by one wave (lane
// l adds pairs l, l + 64, ..., then a butterfly over the wave), then lane 0
// updates the sums (or marks the instance non-finite) and folds a completed
// batch.  Run by k_reduce_parts, and on 2D batches with S(k) by the first
// column-transform block of each instance.
struct SpatialParts {
    const double *part;  // [n_inst][nparts][2]
    InstAcc *acc;
    double inv_cells;
    int32_t nparts;
    int32_t batch_len;
};

__device__ __forceinline__ void reduce_spatial_wave(const SpatialParts &sp, int inst, int lane)
{
    if (sp.acc[inst].nonfinite) return;
    const double *pp = sp.part + 2 * static_cast<int64_t>(inst) * sp.nparts;
    double a = 0.0, b = 0.0;
    // pairs lane, lane + 64, ... in order; four pairs loaded ahead of their adds
    int i = lane;
    for (; i + 192 < sp.nparts; i += 256) {
        double x[4], y[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[k] = pp[2 * (i + 64 * k)];
            y[k] = pp[2 * (i + 64 * k) + 1];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a += x[k];
            b += y[k];
        }
    }
    for (; i < sp.nparts; i += 64) {
        a += pp[2 * i];
        b += pp[2 * i + 1];
    }
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    if (lane == 0) {
        if (!isfinite(a) || !isfinite(b)) {
            sp.acc[inst].nonfinite = 1;
            return;
        }
        a *= sp.inv_cells;
        b *= sp.inv_cells;
        InstAcc q = sp.acc[inst];
        q.sp_mean += a;
        q.sp_sq += b;
        q.sp_var += b - a * a;
        q.n_samples += 1;
        // a sample that completes a batch folds it
        if (sp.batch_len > 0 && q.n_samples % sp.batch_len == 0) fold_spatial(q, sp.batch_len);
        sp.acc[inst] = q;
    }
}

// Batch-means arrays of a 1D batch (device; null when not kept).  cell:
// [6][total_cells] = snapshots of s1 and s2 at the end of the last folded
// batch, Welford (mean, M2) of the batch means of dU, of the batch
// variances; csnap: the covariance sums at that point (c_off layout); skw:
// [2][total_cells] Welford (mean, M2) of the batch S_k (at the instance's off).
struct Batch1D {
    double *cell;
    double *csnap;
    double *skw;
    int64_t total_cells;
    int32_t len;
    int32_t pad;
};

struct InstND;

// Batch-means arrays of the 2D structure factor (device; null when not
// kept): the shell sums at the end of the last folded batch and the Welford
// (mean, M2) of the batch shell averages, n_inst x nbins each.
struct BatchSk {
    double *snap;
    double *wmean;
    double *wm2;
    const double *modes;
    const InstND *ip;       // per-instance u0 (the k = 0 mode)
    double cells;
    int32_t len;
    int32_t pad;
};

// Statistics buffers of the 1D kernel.
struct Stats1D {
    double *s1;         // per cell, or nullptr
    double *s2;
    void *xblk;         // X blocks (state type), 256 x N per instance
    double *c;          // N x N per instance
    InstAcc *acc;       // per instance
    void *hist;         // sample history rings (state type), hist_rows x N per instance
    int32_t hist_rows;
    int32_t pad;
};

// One wave's place in a 1D launch: waves [w0, w0 + nw) of a workgroup serve
// instance `inst` (-1: the wave is idle and exits); the instance's LDS region
// starts `lds` bytes into the workgroup's dynamic LDS.  Several instances
// can share a workgroup; each keeps to its own waves and region.
struct Seg1D {
    int32_t inst;
    int32_t w0;
    int32_t nw;
    int32_t lds;
};

// LDS region of one 1D instance (byte offsets, 16-byte aligned parts):
// exchange arrays [2 buffers][first value, last value, face-0 number][nfg
// rounded up to 4] of the state type; the wave sums of a sample (3 x 16
// doubles); with material arrays (mode 1 or 2) r_f and s_f [nf + 4]
// and w_i [n + 4] of the state type; for implicit schemes (mode 2) an FP64
// array [n] for the reduction.
struct SegLds {
    int32_t xch, red, rf, sf, wc, pd, total;
};

__host__ __device__ inline int32_t lds_align16(int32_t b) { return (b + 15) & ~15; }

__host__ __device__ inline SegLds seg_lds(int32_t n, int32_t nf, int32_t es, int32_t mode)
{
    SegLds l{};
    const int32_t nfg = (nf + 3) >> 2, nfgp = (nfg + 3) & ~3;
    int32_t o = 0;
    l.xch = o;
    o = lds_align16(o + 6 * nfgp * es);
    l.red = o;
    o = lds_align16(o + 3 * 16 * 8);
    l.rf = l.sf = l.wc = l.pd = -1;
    if (mode == 1 || mode == 2) {
        l.rf = o;
        o = lds_align16(o + (nf + 4) * es);
        l.sf = o;
        o = lds_align16(o + (nf + 4) * es);
        l.wc = o;
        o = lds_align16(o + (n + 4) * es);
    }
    if (mode == 2) {
        l.pd = o;
        o = lds_align16(o + n * 8);
    }
    l.total = o;
    return l;
}

// Per-instance parameters of a 2D/3D batch (device table).
struct InstND {
    double ns;              // factor folded into the drawn numbers: sigma/2 (SHE),
                            // sigma/sqrt(2) (DK), sigma A(u0) (deterministic face
                            // value), 0 without noise; sigma = sqrt(2 r eps)
    double init_sd;         // std. dev. of the initial perturbation
    double r;               // mesh ratio of the instance
    double u0;              // its reference value (start, statistics shift)
    uint32_t realisation;   // Philox counter word 3
    uint32_t pad;
};

// Parameters of a 2D/3D batch: one grid, equation, scheme, noise mode and
// seed; r, u0, eps, init_sd and the realisation per instance (InstND).
struct ParamsND {
    int32_t nx, ny, nz;     // nz = 1 in 2D
    int32_t dim;
    int32_t eq, scheme, noise;
    int32_t n_inst;
    int32_t chunk;          // rows (2D, along y) or planes (3D, along z) per march
    int32_t xcd_order;      // 1: give each XCD a contiguous range of workgroups
    uint64_t seed;
    const InstND *ip;       // device, n_inst
};

// Step index and sampling decision of one 2D/3D step.  Launched directly,
// `step` is the step index and `sample` says whether it is a sample step.
// Inside a captured graph (`base` != nullptr) the index is *base + step, read
// from device memory so that replays advance, and `sample` says whether the
// step may sample; the kernels then decide with the burn-in / period rule.
struct StepArg {
    int64_t step;
    const int64_t *base;
    int64_t burn_in;
    int32_t every;
    int32_t sample;
};

__device__ __forceinline__ void resolve_step(const StepArg &a, int64_t &step, int &sample)
{
    if (a.base) {
        step = *a.base + a.step;
        const int64_t t = step + 1;
        sample = a.sample && t > a.burn_in && a.every > 0 && t % a.every == 0;
    } else {
        step = a.step;
        sample = a.sample;
    }
}

}  // namespace she

namespace she {

// ---- launchers (defined next to their kernels) ----
// mode 0: uniform explicit batch; 3: the same with every instance a heat
// equation with instantaneous noise (only that face path compiled);
// 1: some instance has material coefficients
// (k_off >= 0 in `coef`; r_f, s_f, w_i of every instance staged in LDS);
// 2: some instance is implicit (reduction factors in `pcr`; mode 1 included).
// segs: n_blocks * block / 64 wave entries.
hipError_t launch_step1d(int prec, int block, int maxg, bool stats, int mode, int n_blocks, size_t smem,
                         hipStream_t s, const Inst1D *tab, const Seg1D *segs, void *pool,
                         const void *coef, const double *pcr, int64_t step0, int32_t nsteps, int64_t burn_in,
                         int32_t every, uint32_t mask, Stats1D st);
// Initial state of 1D instances: steady profile + init_sd * N(tag 1, step 0, face = cell).
hipError_t launch_init1d(int prec, int n_inst, int nmax, hipStream_t s, const Inst1D *tab,
                         const double *init_sd, void *pool);
// 1D finalisation of one instance into out (FP64):
//   out[0..N) mean, [N..2N) var, [2N..2N+N^2) cov, then N S_k values, then
//   N^2 scratch, then 1 value sum(U).
hipError_t launch_fin1d(int prec, hipStream_t s, const Inst1D *tab, int inst, int n,
                        const void *pool, const double *s1, const double *s2, const void *xblk,
                        const double *c, int64_t n_samples, int partial_rows, bool corr,
                        double *out);

// Where a sample launch of the two-step 2D FE march puts the row transforms
// of the rows it writes (the first stage of the structure factor).
struct SkRows {
    void *half;             // column-tiled half spectrum (half_index), complex state type
    const void *tw;         // natural twiddles exp(-2 pi i t / nx), complex state type
    int32_t ltc;            // log2 of the columns per tile
    int32_t nkb;            // tiles per instance
};

// Whether the two-step march can transform its sample rows itself: one row
// per wave (nx = 512 or 1024) and the LDS of four waves' transforms within
// 64 KB (FP32, or FP64 at nx = 512).
inline bool sk_rows_fusable(int prec, int nx) { return nx == 512 || (nx == 1024 && prec == 0); }

// scheme: 0 FE, 1 PC, 2 two FE steps in one pass (steps st.step and
// st.step + 1; the spatial partials are those of the second).  skr
// (scheme 2, a sample launch, sk_rows_fusable, even march chunks): also
// write the row transforms of the sampled field.
hipError_t launch_step2d(int prec, int cx, int eq, int scheme, int n_blocks, hipStream_t s,
                         const ParamsND &p, const void *src, void *dst, const StepArg &st,
                         double *part, InstAcc *acc, const SkRows *skr = nullptr);
// stage 0: dst = src + Delta(src) (FE, or the PC predictor); stage 1: the PC
// corrector dst = (base + src + Delta(src)) / 2 with src the predictor.
hipError_t launch_step3d(int prec, int cx, int eq, int stage, int ty, int n_blocks, size_t smem,
                         hipStream_t s, const ParamsND &p, const void *src, const void *base, void *dst,
                         const StepArg &st, double *part, InstAcc *acc);
// With batch_len > 0 a sample that completes a batch also folds it
// (fold_spatial).
hipError_t launch_reduce_parts(int n_inst, hipStream_t s, const StepArg &st, const double *part,
                               int32_t nparts, double inv_cells, int32_t batch_len, InstAcc *acc);
// Device step counter of captured graphs: *ctr = value, *ctr += k.
hipError_t launch_set_step(hipStream_t s, int64_t *ctr, int64_t value);
hipError_t launch_add_step(hipStream_t s, int64_t *ctr, int64_t k);
// nD initial state: u0 + init_sd * N(tag 1, step 0, face = cell) per instance.
hipError_t launch_initnd(int prec, hipStream_t s, const ParamsND &p, int64_t cells, void *field);
// nD finalisation of one instance: out[0] spatial mean, out[1] spatial variance,
// out[2] sum(U), then (nbins > 0) out[3 + b] the shell average of <|U_k|^2>.
hipError_t launch_finnd(int prec, hipStream_t s, const ParamsND &p, int inst, int64_t cells,
                        const void *field, const InstAcc *acc, const double *sk_sums,
                        const double *sk_modes, int nbins, double *out);

// 1D time correlation: lag sums tc[m][i] += sum over the samples n in
// [n0, min(n0 + count, n_samples)) with n >= m of h[n][i] h[n-m][i] (FP64),
// rows of the history ring h taken mod hist_rows.
hipError_t launch_tcorr1d(int prec, int n_inst, int nmax, int lags, hipStream_t s, const Inst1D *tab,
                          const void *hist, int32_t hist_rows, int64_t n0, int64_t count, double *tc,
                          const InstAcc *acc);
// Fold the batch that the last launch completed (acc n_samples = (n_batches
// + 1) len) into the 1D batch-means arrays: S_k (instances with CORR), the
// per-cell means and variances (bk.cell), then the spatial sums and
// n_batches.  Instances that have not completed the batch (frozen) are left.
hipError_t launch_fold1d(int prec, int n_inst, int nmax, hipStream_t s, const Inst1D *tab, const void *xblk,
                         const double *c, const double *s1, const double *s2, InstAcc *acc, const Batch1D &bk);
// C_i(m) = tc[m][i]/(M-m) - (s1[i]/M)^2 (NaN for m >= M) of one instance into out[L*N].
hipError_t launch_fin_tc(hipStream_t s, int n, int lags, const double *s1, const double *tc, int64_t M,
                         double *out);

// Verification: raw Philox words / face normals on the device.
hipError_t launch_debug_philox(hipStream_t s, uint64_t seed, const uint32_t *ctr, int64_t count,
                               uint32_t *out);
hipError_t launch_debug_normals(hipStream_t s, int prec, uint64_t seed, uint32_t realisation,
                                uint32_t tag, uint64_t step, uint64_t face0, int64_t count,
                                double *out);

// Column-tiled half spectrum of 2D fields: the columns kx = 0..nx/2 of each
// instance in tiles of 2^ltc (nkb tiles, the last one padded); a tile holds
// rows y = 0..ny-1 of its columns row-major, so a row's piece of a tile is
// one contiguous run and a tile is one contiguous block.
__host__ __device__ inline int64_t half_index(int inst, int y, int kx, int ny, int ltc, int nkb)
{
    return (((static_cast<int64_t>(inst) * nkb + (kx >> ltc)) * ny + y) << ltc) | (kx & ((1 << ltc) - 1));
}
// log2 of the columns per tile (those the column transform takes at once)
int half_tile_log2(int prec, int ny);
inline int half_tiles(int nx, int ltc) { return (nx / 2 + 1 + (1 << ltc) - 1) >> ltc; }

// 2D structure factor on a sample step: row FFTs into the column-tiled half
// spectrum (skipped with rows_done: the step kernel wrote it), column FFTs +
// shell binning into per-block partials, fixed-order reduction into sums
// (n_inst x nbins FP64).  half: n_inst * ny * (half_tiles << ltc) complex of
// the state type.
hipError_t launch_sk2d(int prec, hipStream_t s, const StepArg &st, int n_inst, int nx, int ny, const InstND *ip,
                       const void *field, void *half, const void *twx, const void *twy, const uint16_t *shells,
                       double *part, int nbins, double *sums, InstAcc *acc, const BatchSk &bk, bool rows_done,
                       const SpatialParts &sp);
// shells[kx (nbins + 1) + b], kx = 0..nx/2, b = 0..nbins: the first |ky| of
// shell b in column kx (the range of |ky| in shell b is [first(b), first(b+1)))
hipError_t launch_shell_table(hipStream_t s, int nx, int ny, int nbins, uint16_t *shells);
// exp(-2 pi i t/n), t < n/2, as complex pairs of the state type
hipError_t launch_twiddles(int prec, hipStream_t s, int n, void *tw);
int sk2d_groups(int prec, int nx, int ny, int n_inst);

}  // namespace she
