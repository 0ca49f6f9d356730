// Radially binned static structure factor of 2D fields on sample steps.
//
// S(k) = <|U_k|^2> with U_k = sum_j U_j exp(-2 pi i (j.k)/N) (Garcia et al.,
// Sec. 3, structure factor), averaged over the modes of each shell
// round(|k|), signed k in [-N/2, N/2).  The transform is taken of the shifted
// field dU = U - u0 (which changes only the k = 0 mode; the finalisation
// restores that mode exactly from the spatial sums), in the state's precision.
//
// 1. Row transforms: two real rows are packed as one complex sequence
//    (dU_a + i dU_b) and transformed along x by one wave; the two half spectra,
//    doubled (2 A_k = Z_k + conj Z_-k, 2 B_k = (Z_k - conj Z_-k)/i,
//    kx = 0..Nx/2; the shell sums take the exact 1/4 back), are stored
//    column-tiled: tiles of the columns one column-transform block takes, each
//    tile Ny rows of its columns, row-major and contiguous.  On the sample
//    launches of the two-step 2D FE march the step kernel does this itself for
//    the rows it has just written (she_step_nd.hpp); otherwise k_sk_rows reads
//    the field back.
// 2. k_sk_colt: a block streams a tile of columns of the half spectrum into
//    its waves' LDS regions (the transpose), and each wave transforms its
//    columns along y.  The power |X|^2 gets weight 2 for 0 < kx < Nx/2 (the
//    mirrored half of the spectrum), times the 1/4 of the doubled rows, and
//    is binned without atomics: per column the wave forms the FP64 prefix sum
//    P(m) of the power over |ky| <= m (fixed-order scan), and lane b adds
//    P(hi-1) - P(lo-1) over the range [lo(kx, b), lo(kx, b+1)) of |ky|, with
//    lo(kx, b) the first |ky| in shell b: (2b-1)^2 <= 4(kx^2 + ky^2), exact in
//    integers (a table built once per handle).  Only shells
//    kx .. round(sqrt(kx^2 + (Ny/2)^2)) meet column kx.  The waves' shell sums
//    are added in a fixed order into one partial per block.  The first block
//    of each instance also does the sample's spatial reduction (one wave, the
//    same fixed-order sum as k_reduce_parts); k_bins_reduce, which follows,
//    reads the sample counts it updates.
// 3. k_bins_reduce: per instance and shell, the partials are added in a fixed
//    order to the FP64 running sums.
//
// Transforms: Stockham autosort (decimation in frequency, natural order in
// and out), radix 8 with a final radix 4 or 2, one wave per sequence (or per
// group of short sequences).  A lane holds P points in registers; between
// passes the wave exchanges them through its own LDS region, so a transform
// needs no workgroup barrier.  The twiddle table exp(-2 pi i t/n) is
// precomputed once per handle and staged in LDS.
#include "she_fft.hpp"
#include "she_internal.hpp"
#include "she_wave.hpp"

#include <algorithm>
#include <cmath>

namespace she {

// twiddle table exp(-2 pi i t/n), t < n, in the transform's precision
template <typename T>
__global__ void __launch_bounds__(256) k_twiddles(int n, cplx<T> *__restrict__ tw)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    double sn, cs;
    sincospi(-2.0 * static_cast<double>(t) / static_cast<double>(n), &sn, &cs);
    tw[t] = cplx<T>{static_cast<T>(cs), static_cast<T>(sn)};
}

constexpr int kLdsBudget = 64 * 1024;  // bytes of LDS per block

// Waves per block of the row transform: as many as fit the LDS budget, up to
// 8 (a block's 16 rows of a tile are one contiguous run of the store).
template <typename T, int LG>
constexpr int row_waves()
{
    using F = WaveFft<LG>;
    constexpr int es = static_cast<int>(sizeof(cplx<T>));
    return es * (F::tw + 8 * F::lds) <= kLdsBudget ? 8 : es * (F::tw + 4 * F::lds) <= kLdsBudget ? 4 : 2;
}

#define SHE_SAMPLE_GATE()                                                                          \
    do {                                                                                           \
        int64_t step_;                                                                             \
        int sample_;                                                                               \
        resolve_step(sarg, step_, sample_);                                                        \
        if (!sample_) return; /* a non-sample step of a captured graph */                           \
    } while (0)

// grid: (ceil(ny/2 / (W S)), n_inst); block 64 W; LDS: pass twiddles + W regions.
template <typename T, int LGX>
__global__ void __launch_bounds__(512)
    k_sk_rows(StepArg sarg, const T *__restrict__ field, int ny, const InstND *__restrict__ ip,
              const cplx<T> *__restrict__ twx,
              cplx<T> *__restrict__ half, int ltc, int nkb)
{
    SHE_SAMPLE_GATE();
    using F = WaveFft<LGX>;
    constexpr int n = F::n, P = F::P, S = F::S, W = row_waves<T, LGX>();
    constexpr int LR = PassRadix<LGX>::LR, R = 1 << LR;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *tw = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *reg = tw + F::tw;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int inst = blockIdx.y;
    const int pair0 = blockIdx.x * (W * S);
    const int npairs = min(W * S, ny / 2 - pair0);
    const T *f = field + static_cast<int64_t>(inst) * n * ny;
    const T su0 = static_cast<T>(ip[inst].u0);
    cplx<T> v[P];
#pragma unroll
    for (int i = 0; i < P / R; ++i) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            int seq, x;
            pass_input<LGX, LR>(lane, i, k, seq, x);
            const int pair = wave * S + seq;
            if (pair < npairs) {
                const T *ra = f + static_cast<int64_t>(2 * (pair0 + pair)) * n;
                v[i * R + k] = cplx<T>{ra[x] - su0, ra[n + x] - su0};
            } else {
                v[i * R + k] = cplx<T>{T(0), T(0)};
            }
        }
    }
    fill_pass_twiddles<T, LGX>(tw, twx);
    __syncthreads();
    wave_fft<T, LGX, LGX>(v, reg + wave * F::lds, tw, lane);
    __syncthreads();
    // column-tiled store: the block's rows of one tile are one contiguous run
    constexpr int nh = n / 2 + 1;
    const int nrow = 2 * npairs, tcw = 1 << ltc;
    constexpr int lS = 31 - __builtin_clz(S);
    for (int e = threadIdx.x; e < nkb * nrow * tcw; e += blockDim.x) {
        const int t = e / (nrow * tcw), rest = e - t * (nrow * tcw);
        const int rr = rest >> ltc, k = (t << ltc) + (rest & (tcw - 1));
        if (k >= nh) continue;
        const int pair = rr >> 1;
        const cplx<T> *z0 = reg + (pair >> lS) * F::lds;
        const int sb = (pair & (S - 1)) << LGX;
        const cplx<T> z = z0[pidx(sb + k)];
        const cplx<T> zm = z0[pidx(sb + ((n - k) & (n - 1)))];
        // 2A = z + conj zm (row 2q), 2B = (z - conj zm)/i (row 2q+1)
        half[half_index(inst, 2 * pair0 + rr, k, ny, ltc, nkb)] = (rr & 1) ? unpack2_b(z, zm) : unpack2_a(z, zm);
    }
}

// LDS bytes per column group of the column transform: its transform region
// and the FP64 prefix sums of one column (ppad layout).  A group of one
// column (S = 1) holds the prefix sums in its transform region once the
// transform has left it, so they need no room of their own.
constexpr int col_region(int es, int lg)
{
    return es * wave_lds(lg) + (wave_seqs(lg) == 1 ? 0 : 8 * (((1 << lg) / 2 + 1) * 5 / 4 + 1));
}

// Index of |ky| = m in a column's prefix sums: one pad entry per four, so the
// lanes' runs of four consecutive m fall in distinct banks.
__device__ __forceinline__ int ppad(int m)
{
    return m + (m >> 2);
}

// Shape of the tiled column transform: a tile of TC = CW CPW S columns by Ny
// rows holds up to 32 KB of points, at most eight column groups (of S
// columns); a block has CW <= 4 waves and each wave transforms CPW groups of
// the tile in turn.  Wide tiles keep the row runs of the column-tiled half
// spectrum at 64 bytes and more; small blocks keep the barriers cheap.
template <typename T, int LGY>
constexpr int colt_groups()
{
    constexpr int w = 32768 / (64 * WaveFft<LGY>::P * static_cast<int>(sizeof(cplx<T>)));
    return w >= 8 ? 8 : (w >= 4 ? 4 : (w >= 2 ? 2 : 1));
}

template <typename T, int LGY>
constexpr int colt_waves()
{
    return colt_groups<T, LGY>() >= 4 ? 4 : colt_groups<T, LGY>();
}

constexpr int kMaxBinIters = 12;  // shells per lane: nbins <= 64 * 12

// First |ky| of shell b in column kx, clipped to [0, hy + 1]: the smallest
// m >= 0 with 4 (kx^2 + m^2) >= (2b - 1)^2 (b = 0: m = 0), given kx4 = 4 kx^2.
// The native single precision root is within one of the answer and the
// integer tests settle it.  The factors are below 2^24 (b <= 768, m <= 769),
// and masked to say so, which lets the products use 24-bit multiplies.
__device__ __forceinline__ unsigned sq24(int v)
{
    const unsigned u = static_cast<unsigned>(v) & 0xffffffu;
    return u * u;
}

__device__ __forceinline__ int shell_first(int kx4, int b, int hy)
{
    const int need = static_cast<int>(sq24(2 * b - 1)) - kx4;
    int m = static_cast<int>(ceilf(0.5f * __builtin_amdgcn_sqrtf(static_cast<float>(max(need, 0)))));
    if (4 * static_cast<int>(sq24(m)) < need) ++m;
    else if (m > 0 && 4 * static_cast<int>(sq24(m - 1)) >= need) --m;
    return (b == 0 || need <= 0) ? 0 : min(m, hy + 1);
}

// The shell table: first(b) for every column kx = 0..Nx/2 and shell
// b = 0..nbins (the same for every instance and sample; built once).
__global__ void __launch_bounds__(256) k_shell_table(int nh, int nbins, int hy, uint16_t *__restrict__ tab)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e >= static_cast<int64_t>(nh) * (nbins + 1)) return;
    const int kx = static_cast<int>(e / (nbins + 1)), b = static_cast<int>(e - static_cast<int64_t>(kx) * (nbins + 1));
    tab[e] = static_cast<uint16_t>(shell_first(4 * kx * kx, b, hy));
}

// Power spectrum of one column folded onto |ky| and its FP64 prefix sums, from
// a transform held in registers (one sequence per wave: lane l holds
// X(l + 64 j), j < P, slot i R + k for j = i + k P/R with R the last pass's
// radix).  e(m) = |X(m)|^2 + |X(n - m)|^2 for 0 < m < n/2, |X(m)|^2 at m = 0
// and m = n/2 (powers in T, their sum in FP64); pre[ppad(m)] = e(0) + ... + e(m).
// The mirror X(n - m) of m = l + 64 j is X((64 - l) + 64 (P - 1 - j)) for
// l > 0 (another lane, read with a lane permute) and X(64 (P - j)) for l = 0
// (this lane).  The e(m) go through pre so that lane l sums the Q = P/2
// consecutive m = Q l .. Q l + Q - 1 (lane 63 also m = n/2) in order, and the
// lane totals are scanned once over the wave.
template <typename T, int LG>
__device__ __forceinline__ void col_power_prefix(const cplx<T> (&v)[WaveFft<LG>::P], double *pre, int lane)
{
    using F = WaveFft<LG>;
    static_assert(F::S == 1, "one sequence per wave");
    constexpr int P = F::P, n = F::n, hy = n / 2, Q = P / 2;
    constexpr int LR = LG - 3 * ((LG - 1) / 3), R = 1 << LR;  // radix 8 passes, then this one
    T pw[P];
#pragma unroll
    for (int i = 0; i < P / R; ++i) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const cplx<T> x = v[i * R + k];
            pw[i + k * (P / R)] = x.re * x.re + x.im * x.im;
        }
    }
    const int src = ((64 - lane) & 63) << 2;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        T mir;
        if constexpr (sizeof(T) == 4) {
            mir = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(pw[P - 1 - j])));
        } else {
            const long long u = __double_as_longlong(pw[P - 1 - j]);
            const int lo = __builtin_amdgcn_ds_bpermute(src, static_cast<int>(u & 0xffffffffLL));
            const int hi = __builtin_amdgcn_ds_bpermute(src, static_cast<int>(u >> 32));
            mir = __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
        }
        if (lane == 0) mir = j == 0 ? T(0) : pw[P - j];
        pre[ppad(lane + 64 * j)] = static_cast<double>(pw[j]) + static_cast<double>(mir);
    }
    if (lane == 0) pre[ppad(hy)] = static_cast<double>(pw[Q]);
    wave_sync();
    double loc[Q + 1];
    double run = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        run += pre[ppad(Q * lane + i)];
        loc[i] = run;
    }
    loc[Q] = lane == 63 ? run + pre[ppad(hy)] : 0.0;
    // exclusive prefix of the lane totals: the inclusive scan moved one lane up
    const long long u = __double_as_longlong(wave_inclusive_sum(run));
    const int elo = __builtin_amdgcn_update_dpp(0, static_cast<int>(u & 0xffffffffLL), 0x138, 0xf, 0xf, false);
    const int ehi = __builtin_amdgcn_update_dpp(0, static_cast<int>(u >> 32), 0x138, 0xf, 0xf, false);
    const double excl = __longlong_as_double((static_cast<long long>(ehi) << 32) | static_cast<unsigned>(elo));
    wave_sync();
#pragma unroll
    for (int i = 0; i < Q; ++i) pre[ppad(Q * lane + i)] = excl + loc[i];
    if (lane == 63) pre[ppad(hy)] = excl + loc[Q];
}

// Adds column kx's power to the shell sums: lane b of group j takes shell
// b = lane + 64 j, the range [first(b), first(b + 1)) of |ky| (from the shell
// table, col = its row for kx), as pre[first(b + 1) - 1] - pre[first(b) - 1],
// weighted 1/4 (the row stage stores doubled half spectra, so the powers are
// 4 |X|^2), and twice that off the kx = 0 and Nx/2 columns (the mirrored half
// of the spectrum); both scalings are exact.  first(b) and its prefix value are lane
// b - 1's, moved one lane up; lane 0 takes those of lane 63 of the previous
// group, and 0 for the first group met (its shells lie below kx, first = 0).
// Only shells kx .. round(sqrt(kx^2 + hy^2)) (bound by excess) meet the column.
template <int NBJ>
__device__ __forceinline__ void bin_column(double (&acc)[NBJ], const double *pre, const uint16_t *__restrict__ col,
                                           int kx, int nx, int nbins, int nbj, int hy, int lane)
{
    const double w = (kx == 0 || 2 * kx == nx) ? 0.25 : 0.5;
    const int jlo = kx >> 6;
    const int jhi = static_cast<int>(__builtin_amdgcn_sqrtf(static_cast<float>(kx * kx + hy * hy)) + 1.5f) >> 6;
    int m1s[NBJ];
#pragma unroll
    for (int j = 0; j < NBJ; ++j) {
        const int b = lane + 64 * j;
        m1s[j] = (j >= jlo && j <= jhi && j < nbj && b < nbins) ? static_cast<int>(col[b + 1]) : hy + 1;
    }
    int carry = 0, clo = 0, chi = 0;
#pragma unroll
    for (int j = 0; j < NBJ; ++j) {
        if (j >= jlo && j <= jhi && j < nbj) {
            const int b = lane + 64 * j;
            const int m1 = m1s[j];
            const int m0 = __builtin_amdgcn_update_dpp(carry, m1, 0x138, 0xf, 0xf, false);  // wave_shr:1
            const double p1 = m1 > 0 ? pre[ppad(m1 - 1)] : 0.0;
            const long long u = __double_as_longlong(p1);
            const int ulo = static_cast<int>(u & 0xffffffffLL), uhi = static_cast<int>(u >> 32);
            const int plo = __builtin_amdgcn_update_dpp(clo, ulo, 0x138, 0xf, 0xf, false);
            const int phi = __builtin_amdgcn_update_dpp(chi, uhi, 0x138, 0xf, 0xf, false);
            const double p0 = __longlong_as_double((static_cast<long long>(phi) << 32) | static_cast<unsigned>(plo));
            carry = __builtin_amdgcn_readlane(m1, 63);
            clo = __builtin_amdgcn_readlane(ulo, 63);
            chi = __builtin_amdgcn_readlane(uhi, 63);
            if (b < nbins && m1 > m0) acc[j] += w * (p1 - p0);
        }
    }
}

// grid: (groups, n_inst); block 64 CW.  Block b takes `iters` consecutive
// tiles of TC columns from tile b iters.  The block copies a tile (one
// contiguous block of the column-tiled half spectrum) through registers into
// the LDS regions of its NG column groups (the transpose), and wave w
// transforms groups w CPW .. w CPW + CPW - 1 in turn.  LDS: pass twiddles,
// then per group `rs` bytes: its columns' transform region, the FP64 prefix
// sums of one column (within the transform region when S = 1), and (after
// the loop, the first CW) the waves' shell sums.
// Compiled for four waves per SIMD (128 VGPRs) where the FP32 transform fits
// without spilling, else two.
template <typename T, int LGY, int NBJ>
__global__ void __launch_bounds__(256, (sizeof(T) == 4 && LGY <= 9) ? 4 : 2)
    k_sk_colt(StepArg sarg, const cplx<T> *__restrict__ half, int nx, int nkb, int iters, int rs, int nbins,
              const cplx<T> *__restrict__ twy, const uint16_t *__restrict__ shells, double *__restrict__ part,
              SpatialParts sp)
{
    SHE_SAMPLE_GATE();
    // the sample's spatial reduction of this instance, when it rides along
    // (one wave of the instance's first block; the shell reduction that
    // follows reads what it wrote)
    if (sp.part && blockIdx.x == 0 && threadIdx.x < 64) reduce_spatial_wave(sp, blockIdx.y, threadIdx.x);
    using F = WaveFft<LGY>;
    constexpr int n = F::n, P = F::P, S = F::S, hy = n / 2;
    constexpr int LR = PassRadix<LGY>::LR, R = 1 << LR;
    constexpr int CW = colt_waves<T, LGY>(), NG = colt_groups<T, LGY>(), CPW = NG / CW, TC = NG * S;
    constexpr int per = (hy + 1 + 63) >> 6;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *tw = reinterpret_cast<cplx<T> *>(smem_raw);
    unsigned char *regions = smem_raw + sizeof(cplx<T>) * F::tw;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int inst = blockIdx.y;
    const int nh = nx / 2 + 1;
    const cplx<T> *hi = half + static_cast<int64_t>(inst) * nkb * n * TC;
    fill_pass_twiddles<T, LGY>(tw, twy);
    // a tile (contiguous: n rows of TC columns) has n TC = 64 CW CPW P
    // points, CPW P per thread.  Entry e is row e / TC, column e % TC, and
    // goes to the region of column group e % TC / S.  FP64: point j of thread
    // t is entry t + 64 CW j.  FP32 points move two at a time, in 16-byte
    // loads of two adjacent columns of a row: points 2 j and 2 j + 1 are
    // entries 2 e and 2 e + 1, e = t + 64 CW j.
    constexpr int lTC = 31 - __builtin_clz(TC), PT = CPW * P;
    const int tc = threadIdx.x & (TC - 1);
    cplx<T> pf[PT];
    constexpr bool V2 = sizeof(T) == 4 && TC >= 2;
    auto fetch = [&](int cb) {
        const cplx<T> *tile = hi + static_cast<unsigned>(cb * n);  // tile cb / TC
        if constexpr (V2) {
            typedef float f4v __attribute__((ext_vector_type(4)));
            const f4v *t4 = reinterpret_cast<const f4v *>(tile);
            if (cb + TC <= nh) {
                // a full tile (all but an instance's last): no column to mask
#pragma unroll
                for (int j = 0; j < PT / 2; ++j) {
                    const f4v q = t4[threadIdx.x + 64 * CW * j];
                    pf[2 * j] = cplx<T>{q.x, q.y};
                    pf[2 * j + 1] = cplx<T>{q.z, q.w};
                }
                return;
            }
            const int c0 = (2 * threadIdx.x) & (TC - 1);
            const bool in0 = cb + c0 < nh, in1 = cb + c0 + 1 < nh;
#pragma unroll
            for (int j = 0; j < PT / 2; ++j) {
                const f4v q = t4[threadIdx.x + 64 * CW * j];
                pf[2 * j] = in0 ? cplx<T>{q.x, q.y} : cplx<T>{T(0), T(0)};
                pf[2 * j + 1] = in1 ? cplx<T>{q.z, q.w} : cplx<T>{T(0), T(0)};
            }
        } else {
            const bool in = cb + tc < nh;
#pragma unroll
            for (int j = 0; j < PT; ++j)
                pf[j] = in ? tile[threadIdx.x + 64 * CW * j] : cplx<T>{T(0), T(0)};
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const int e = V2 ? 2 * (threadIdx.x + 64 * CW * (j >> 1)) + (j & 1) : threadIdx.x + 64 * CW * j;
            const int y = e >> lTC, c = e & (TC - 1);
            cplx<T> *dst = reinterpret_cast<cplx<T> *>(regions + static_cast<size_t>(c / S) * rs);
            dst[pidx(((c & (S - 1)) << LGY) + y)] = pf[j];
        }
    };
    const int nbj = (nbins + 63) >> 6;
    double acc[NBJ];
#pragma unroll
    for (int j = 0; j < NBJ; ++j) acc[j] = 0.0;
    const int t0 = blockIdx.x * iters;
    for (int it = 0; it < iters; ++it) {
        const int cb = (t0 + it) * TC;
        if (cb >= nh) break;  // block-uniform
        fetch(cb);
        stash();
        __syncthreads();
        for (int cg = 0; cg < CPW; ++cg) {
            const int r = wave * CPW + cg;  // the column group's region
            cplx<T> *buf = reinterpret_cast<cplx<T> *>(regions + static_cast<size_t>(r) * rs);
            double *pre = S == 1 ? reinterpret_cast<double *>(buf) : reinterpret_cast<double *>(buf + F::lds);
            const int g = cb + S * r;
            if (g < nh) {  // wave-uniform
                cplx<T> v[P];
#pragma unroll
                for (int i = 0; i < P / R; ++i) {
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        int seq, y;
                        pass_input<LGY, LR>(lane, i, k, seq, y);
                        v[i * R + k] = buf[pidx((seq << LGY) + y)];
                    }
                }
                wave_sync();
                if constexpr (S == 1) {
                    // the transform stays in registers: lane l holds X(l + 64 j)
                    wave_fft<T, LGY, LGY, true>(v, buf, tw, lane);
                    col_power_prefix<T, LGY>(v, pre, lane);
                    wave_sync();
                    bin_column<NBJ>(acc, pre, shells + g * (nbins + 1), g, nx, nbins, nbj, hy, lane);
                } else {
                    wave_fft<T, LGY, LGY>(v, buf, tw, lane);
                    for (int c = 0; c < S && g + c < nh; ++c) {
                        const int kx = g + c;
                        const cplx<T> *col = buf;
                        const int cbase = c << LGY;
                        double loc[per];
                        double run = 0.0;
#pragma unroll
                        for (int j = 0; j < per; ++j) {
                            // power at |ky| = m: X(m), plus X(-m) for 0 < m < hy; m > hy
                            // is padding (both reads stay inside the column, masked after)
                            const int m = lane * per + j;
                            const cplx<T> a = col[pidx(cbase + min(m, hy))];
                            const cplx<T> b = col[pidx(cbase + ((n - m) & (n - 1)))];
                            const T ea = m <= hy ? a.re * a.re + a.im * a.im : T(0);
                            const T eb = (m != 0 && m < hy) ? b.re * b.re + b.im * b.im : T(0);
                            run += static_cast<double>(ea) + static_cast<double>(eb);
                            loc[j] = run;
                        }
                        const double excl = wave_inclusive_sum(run) - run;
#pragma unroll
                        for (int j = 0; j < per; ++j) {
                            const int m = lane * per + j;
                            if (m <= hy) pre[ppad(m)] = excl + loc[j];
                        }
                        wave_sync();
                        bin_column<NBJ>(acc, pre, shells + kx * (nbins + 1), kx, nx, nbins, nbj, hy, lane);
                        wave_sync();
                    }
                }
            }
        }
        __syncthreads();  // the regions take the next tile
    }
    double *mine = reinterpret_cast<double *>(regions + static_cast<size_t>(wave) * rs);
#pragma unroll
    for (int j = 0; j < NBJ; ++j) {
        const int b = lane + 64 * j;
        if (j < nbj && b < nbins) mine[b] = acc[j];
    }
    __syncthreads();
    double *pp = part + (static_cast<int64_t>(inst) * gridDim.x + blockIdx.x) * nbins;
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < CW; ++w) s += reinterpret_cast<const double *>(regions + static_cast<size_t>(w) * rs)[b];
        pp[b] = s;
    }
}

__global__ void __launch_bounds__(256)
    k_bins_reduce(StepArg sarg, const double *__restrict__ part, int ngroups, int nbins, int n_inst,
                  double *__restrict__ sums, const InstAcc *__restrict__ acc, BatchSk bk)
{
    SHE_SAMPLE_GATE();
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e >= static_cast<int64_t>(n_inst) * nbins) return;
    const int inst = static_cast<int>(e / nbins), b = static_cast<int>(e - static_cast<int64_t>(inst) * nbins);
    const InstAcc q = acc[inst];
    if (q.nonfinite) return;
    const double *pp = part + static_cast<int64_t>(inst) * ngroups * nbins + b;
    // in group order; four loads issued ahead of their adds
    double s = 0.0;
    int g = 0;
    for (; g + 4 <= ngroups; g += 4) {
        const double a0 = pp[static_cast<int64_t>(g) * nbins], a1 = pp[static_cast<int64_t>(g + 1) * nbins];
        const double a2 = pp[static_cast<int64_t>(g + 2) * nbins], a3 = pp[static_cast<int64_t>(g + 3) * nbins];
        s += a0;
        s += a1;
        s += a2;
        s += a3;
    }
    for (; g < ngroups; ++g) s += pp[static_cast<int64_t>(g) * nbins];
    const double tot = sums[e] + s;
    sums[e] = tot;
    // The sample reduction ran first and folded the spatial sums of a batch
    // this sample completed; fold the shells' batch averages too (the k = 0
    // shell restored from the batch's spatial-mean sum, as at finalisation).
    if (bk.len > 0 && q.n_samples % bk.len == 0) {
        const double L = static_cast<double>(bk.len), N = bk.cells;
        double v = tot - bk.snap[e];
        const double u0 = bk.ip[inst].u0;
        if (b == 0) v += L * N * N * u0 * u0 + 2.0 * N * u0 * (N * q.batch_sp_mean);
        const double x = bk.modes[b] > 0 ? v / (L * bk.modes[b]) : 0.0;
        welford(x, static_cast<double>(q.n_batches), bk.wmean[e], bk.wm2[e]);
        bk.snap[e] = tot;
    }
}

// ------------------------------------------------------------------ host side

namespace {

int ilog2(int v)
{
    return 31 - __builtin_clz(v);
}

// LDS bytes of a column-transform block (nbins shell sums fit each wave's
// region after the transforms)
template <typename T, int LGY>
size_t colt_lds(int nbins, size_t *rs_out)
{
    size_t rs = col_region(static_cast<int>(sizeof(cplx<T>)), LGY);
    rs = std::max(rs, sizeof(double) * static_cast<size_t>(nbins));
    // regions an odd multiple of 32 bytes apart: the eight regions then
    // start 32 bytes apart modulo the 256 bytes of the 64 LDS banks (in some
    // order), so the tile copy's half-wave stores (four rows of eight columns,
    // or eight rows of four even or odd columns) meet each bank once
    rs = ((rs + 31) & ~static_cast<size_t>(63)) + 32;
    if (rs_out) *rs_out = rs;
    return ((sizeof(cplx<T>) * WaveFft<LGY>::tw + 15) & ~static_cast<size_t>(15)) + colt_groups<T, LGY>() * rs;
}

int tile_cols(int prec, int lgy)
{
#define SHE_TC(L)                                                                            \
    case L:                                                                                  \
        return prec == 0 ? colt_groups<float, L>() * WaveFft<L>::S : colt_groups<double, L>() * WaveFft<L>::S;
    switch (lgy) {
        SHE_TC(1) SHE_TC(2) SHE_TC(3) SHE_TC(4) SHE_TC(5) SHE_TC(6) SHE_TC(7) SHE_TC(8) SHE_TC(9) SHE_TC(10)
    default: return 1;
    }
#undef SHE_TC
}

// Tiles per column-transform block: at least about 4096 blocks over the
// batch (four resident per CU, so about four rounds).  Measured at
// 512 x 512 x 256 (8448 tiles), us per sample: 1 tile per block 103.4, 2
// 101.4, 3 102.0, 4 106.7, 5 107.6, 6 115.2, 8 118.8.
int colt_iters(int prec, int nx, int ny, int n_inst)
{
    const int tc = tile_cols(prec, ilog2(ny));
    const int64_t tiles = static_cast<int64_t>((nx / 2 + 1 + tc - 1) / tc) * n_inst;
    int it = 1;
    while (it < 8 && tiles / (2 * it) >= 4096) it *= 2;
    return it;
}

}  // namespace

int half_tile_log2(int prec, int ny) { return ilog2(tile_cols(prec, ilog2(ny))); }

int sk2d_groups(int prec, int nx, int ny, int n_inst)
{
    const int tc = tile_cols(prec, ilog2(ny));
    const int tiles = (nx / 2 + 1 + tc - 1) / tc, it = colt_iters(prec, nx, ny, n_inst);
    return (tiles + it - 1) / it;
}

hipError_t launch_shell_table(hipStream_t s, int nx, int ny, int nbins, uint16_t *shells)
{
    const int64_t tot = static_cast<int64_t>(nx / 2 + 1) * (nbins + 1);
    hipLaunchKernelGGL(k_shell_table, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, s, nx / 2 + 1,
                       nbins, ny / 2, shells);
    return hipGetLastError();
}

hipError_t launch_twiddles(int prec, hipStream_t s, int n, void *tw)
{
    const dim3 g((n + 255) / 256);
    if (prec == 0)
        hipLaunchKernelGGL(k_twiddles<float>, g, dim3(256), 0, s, n, static_cast<cplx<float> *>(tw));
    else
        hipLaunchKernelGGL(k_twiddles<double>, g, dim3(256), 0, s, n, static_cast<cplx<double> *>(tw));
    return hipGetLastError();
}

namespace {

template <typename T, int LGX>
void rows_t(hipStream_t s, const StepArg &sa, int n_inst, int ny, const InstND *ip, const void *field, const void *twx,
            void *half, int ltc, int nkb)
{
    using F = WaveFft<LGX>;
    constexpr int W = row_waves<T, LGX>();
    const int pairs = W * F::S;
    const dim3 grid((ny / 2 + pairs - 1) / pairs, n_inst);
    const size_t smem = sizeof(cplx<T>) * (F::tw + static_cast<size_t>(W) * F::lds);
    static_assert(sizeof(cplx<T>) * (F::tw + W * F::lds) <= kLdsBudget, "row transform exceeds the LDS budget");
    hipLaunchKernelGGL((k_sk_rows<T, LGX>), grid, dim3(64 * W), smem, s, sa, static_cast<const T *>(field), ny, ip,
                       static_cast<const cplx<T> *>(twx), static_cast<cplx<T> *>(half), ltc, nkb);
}

template <typename T, int LGY>
bool cols_t(hipStream_t s, const StepArg &sa, int n_inst, int nx, int nkb, int nbins, const void *half, const void *twy,
            const uint16_t *shells, double *part, int groups, int iters, const SpatialParts &sp)
{
    size_t rs = 0;
    const size_t smem = colt_lds<T, LGY>(nbins, &rs);
    if (smem > kLdsBudget) return false;
    const dim3 grid(groups, n_inst), block(64 * colt_waves<T, LGY>());
    if (nbins <= 64 * (kMaxBinIters / 2))
        hipLaunchKernelGGL((k_sk_colt<T, LGY, kMaxBinIters / 2>), grid, block, smem, s, sa,
                           static_cast<const cplx<T> *>(half), nx, nkb, iters, static_cast<int>(rs), nbins,
                           static_cast<const cplx<T> *>(twy), shells, part, sp);
    else
        hipLaunchKernelGGL((k_sk_colt<T, LGY, kMaxBinIters>), grid, block, smem, s, sa,
                           static_cast<const cplx<T> *>(half), nx, nkb, iters, static_cast<int>(rs), nbins,
                           static_cast<const cplx<T> *>(twy), shells, part, sp);
    return true;
}

template <typename T>
bool rows_dispatch(int lgx, hipStream_t s, const StepArg &sa, int n_inst, int ny, const InstND *ip, const void *field,
                   const void *twx, void *half, int ltc, int nkb)
{
#define SHE_ROWS(L)                                                        \
    case L:                                                                \
        rows_t<T, L>(s, sa, n_inst, ny, ip, field, twx, half, ltc, nkb);  \
        return true;
    switch (lgx) {
        SHE_ROWS(3) SHE_ROWS(4) SHE_ROWS(5) SHE_ROWS(6) SHE_ROWS(7) SHE_ROWS(8) SHE_ROWS(9) SHE_ROWS(10)
    default: return false;
    }
#undef SHE_ROWS
}

template <typename T>
bool cols_dispatch(int lgy, hipStream_t s, const StepArg &sa, int n_inst, int nx, int nkb, int nbins, const void *half,
                   const void *twy, const uint16_t *shells, double *part, int groups, int iters,
                   const SpatialParts &sp)
{
#define SHE_COLS(L)                                                                              \
    case L:                                                                                      \
        return cols_t<T, L>(s, sa, n_inst, nx, nkb, nbins, half, twy, shells, part, groups, iters, sp);
    switch (lgy) {
        SHE_COLS(1) SHE_COLS(2) SHE_COLS(3) SHE_COLS(4) SHE_COLS(5) SHE_COLS(6) SHE_COLS(7) SHE_COLS(8)
        SHE_COLS(9) SHE_COLS(10)
    default: return false;
    }
#undef SHE_COLS
}

}  // namespace

hipError_t launch_sk2d(int prec, hipStream_t s, const StepArg &sa, int n_inst, int nx, int ny, const InstND *ip,
                       const void *field, void *half, const void *twx, const void *twy, const uint16_t *shells,
                       double *part, int nbins, double *sums, InstAcc *acc, const BatchSk &bk, bool rows_done,
                       const SpatialParts &sp)
{
    if (nbins > 64 * kMaxBinIters) return hipErrorInvalidValue;
    const int lgx = ilog2(nx), lgy = ilog2(ny);
    const int ltc = half_tile_log2(prec, ny), nkb = half_tiles(nx, ltc);
    const int groups = sk2d_groups(prec, nx, ny, n_inst), iters = colt_iters(prec, nx, ny, n_inst);
    bool ok;
    if (prec == 0) {
        ok = (rows_done || rows_dispatch<float>(lgx, s, sa, n_inst, ny, ip, field, twx, half, ltc, nkb)) &&
             cols_dispatch<float>(lgy, s, sa, n_inst, nx, nkb, nbins, half, twy, shells, part, groups, iters, sp);
    } else {
        ok = (rows_done || rows_dispatch<double>(lgx, s, sa, n_inst, ny, ip, field, twx, half, ltc, nkb)) &&
             cols_dispatch<double>(lgy, s, sa, n_inst, nx, nkb, nbins, half, twy, shells, part, groups, iters, sp);
    }
    if (!ok) return hipErrorInvalidValue;
    const int64_t tot = static_cast<int64_t>(n_inst) * nbins;
    hipLaunchKernelGGL(k_bins_reduce, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, s, sa, part,
                       groups, nbins, n_inst, sums, acc, bk);
    return hipGetLastError();
}

}  // namespace she
