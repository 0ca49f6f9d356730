// Radially binned static structure factor of 2D fields on sample steps.
//
// S(k) = <|U_k|^2> with U_k = sum_j U_j exp(-2 pi i (j.k)/N) (Garcia et al.,
// Sec. 3, structure factor), averaged over the modes of each shell
// round(|k|), signed k in [-N/2, N/2).  The transform is taken of the shifted
// field dU = U - u0 (which changes only the k = 0 mode; the finalisation
// restores that mode exactly from the spatial sums), in the state's precision.
//
// 1. k_sk_rows: two real rows are packed as one complex sequence
//    (dU_a + i dU_b) and transformed along x by one wave; the two half spectra
//    A_k = (Z_k + conj Z_-k)/2, B_k = (Z_k - conj Z_-k)/(2i) are stored
//    kx-major (y fastest), so that the waves of a block, which hold
//    consecutive row pairs, write runs of consecutive y per kx.
// 2. k_sk_cols: each wave transforms half-spectrum columns (contiguous in
//    memory) along y, looping over the block's columns and loading the next
//    column while it transforms the current one.  The power |X|^2 gets weight
//    2 for 0 < kx < Nx/2 (the mirrored half of the spectrum) and is binned
//    without atomics: per column the wave forms the FP64 prefix sum P(m) of
//    the power over |ky| <= m (fixed-order scan), and lane b adds
//    P(hi-1) - P(lo-1) over the range [lo(kx, b), lo(kx, b+1)) of |ky|, with
//    lo(kx, b) the first |ky| in shell b: (2b-1)^2 <= 4(kx^2 + ky^2), exact in
//    integers.  Only shells kx .. round(sqrt(kx^2 + (Ny/2)^2)) meet column kx.
//    The waves' shell sums are added in a fixed order into one partial per
//    block.
// 3. k_bins_reduce: per instance and shell, the partials are added in a fixed
//    order to the FP64 running sums.
//
// Transforms: Stockham autosort (decimation in frequency, natural order in
// and out), radix 8 with a final radix 4 or 2, one wave per sequence (or per
// group of short sequences).  A lane holds P points in registers; between
// passes the wave exchanges them through its own LDS region, so a transform
// needs no workgroup barrier.  The twiddle table exp(-2 pi i t/n) is
// precomputed once per handle and staged in LDS.
#include "she_internal.hpp"
#include "she_wave.hpp"

#include <algorithm>

namespace she {

// Aligned to its size, so that one lane's point moves in one 64-bit (FP32)
// or 128-bit (FP64) LDS access; at the alignment of T every exchange store
// and load splits into two, and the transforms are bound by the LDS.
template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b)
{
    return cplx<T>{a.re + b.re, a.im + b.im};
}

template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b)
{
    return cplx<T>{a.re - b.re, a.im - b.im};
}

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> w)
{
    return cplx<T>{a.re * w.re - a.im * w.im, a.re * w.im + a.im * w.re};
}

// Shape of the per-wave transform of length n = 2^lg: P points per lane,
// S sequences per wave (64 P = S n), padded LDS entries per wave region.
constexpr int wave_points(int lg)
{
    return (1 << lg) >= 512 ? (1 << lg) / 64 : ((1 << lg) >= 8 ? 8 : (1 << lg));
}

constexpr int wave_seqs(int lg)
{
    return (64 * wave_points(lg)) >> lg;
}

constexpr int wave_lds(int lg)
{
    return (wave_seqs(lg) << lg) + (((wave_seqs(lg) << lg) - 1) >> 4) + 1;
}

// log2 of the radix of the pass at sub-transform length 2^rem: 8, then 4 or 2
constexpr int pass_lr(int rem)
{
    return rem >= 3 ? 3 : rem;
}

// Twiddles per pass, laid out [p][k-1] (k = 1..R-1) so that the lanes of a
// pass, which differ in p, read R-1 consecutive entries each (odd stride: no
// bank conflicts).  A pass at sub-length 2^rem has 2^(rem - lr) values of p
// and none when it is the last one.  Entries of the passes from 2^rem down:
constexpr int tw_entries(int rem)
{
    return rem <= 0 ? 0
                    : (rem > pass_lr(rem) ? (1 << (rem - pass_lr(rem))) * ((1 << pass_lr(rem)) - 1) : 0) +
                          tw_entries(rem - pass_lr(rem));
}

template <int LG>
struct WaveFft {
    static constexpr int n = 1 << LG;
    static constexpr int P = wave_points(LG);
    static constexpr int S = wave_seqs(LG);
    static constexpr int lds = wave_lds(LG);
    static constexpr int tw = tw_entries(LG) > 0 ? tw_entries(LG) : 1;  // per-pass twiddle entries
};

// one pad entry per 16 spreads the strided exchange accesses over the banks
__device__ __forceinline__ int pidx(int i)
{
    return i + (i >> 4);
}

// Order the LDS accesses of one wave (a wave's LDS operations complete in
// issue order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// In-register DFTs of length 2, 4, 8 (natural order in and out).
template <typename T>
__device__ __forceinline__ void dft2(cplx<T> *a)
{
    const cplx<T> t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
}

template <typename T>
__device__ __forceinline__ void dft4(cplx<T> &a0, cplx<T> &a1, cplx<T> &a2, cplx<T> &a3)
{
    const cplx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3);
    const cplx<T> d = csub(a1, a3);
    const cplx<T> t3{d.im, -d.re};  // -i (a1 - a3)
    a0 = cadd(t0, t2);
    a1 = cadd(t1, t3);
    a2 = csub(t0, t2);
    a3 = csub(t1, t3);
}

template <typename T>
__device__ __forceinline__ void dft8(cplx<T> *a)
{
    // even and odd halves, then w8^k on the odd outputs
    dft4(a[0], a[2], a[4], a[6]);
    dft4(a[1], a[3], a[5], a[7]);
    const T c = static_cast<T>(0.70710678118654752440);
    const cplx<T> o1{c * (a[3].re + a[3].im), c * (a[3].im - a[3].re)};  // (1 - i)/sqrt2
    const cplx<T> o2{a[5].im, -a[5].re};                                 // -i
    const cplx<T> o3{c * (a[7].im - a[7].re), -c * (a[7].re + a[7].im)}; // (-1 - i)/sqrt2
    const cplx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6], o0 = a[1];
    a[0] = cadd(e0, o0);
    a[4] = csub(e0, o0);
    a[1] = cadd(e1, o1);
    a[5] = csub(e1, o1);
    a[2] = cadd(e2, o2);
    a[6] = csub(e2, o2);
    a[3] = cadd(e3, o3);
    a[7] = csub(e3, o3);
}

template <int REM>
struct PassRadix {
    static constexpr int LR = pass_lr(REM);
};

// Inputs of a pass of radix R = 2^LR: lane slot i*R + k holds element
// t + k n/R of sequence seq, for butterfly b = lane + 64 i = seq (n/R) + t.
template <int LG, int LR>
__device__ __forceinline__ void pass_input(int lane, int i, int k, int &seq, int &idx)
{
    constexpr int n = 1 << LG;
    const int b = lane + 64 * i;
    seq = b >> (LG - LR);
    idx = (b & ((n >> LR) - 1)) + k * (n >> LR);
}

// Remaining passes of the wave transform from sub-transform length 2^REM.
// Butterfly t = q + s p (s = 2^(LG-REM), q < s) forms the R-point DFT of its
// inputs, multiplies output k by exp(-2 pi i k p s / n) and writes it to
// element q + s (R p + k).  After the last pass the wave's LDS region holds
// the transforms in natural order.
template <typename T, int LG, int REM>
__device__ __forceinline__ void wave_fft(cplx<T> (&v)[WaveFft<LG>::P], cplx<T> *buf, const cplx<T> *tw, int lane)
{
    using F = WaveFft<LG>;
    constexpr int LR = PassRadix<REM>::LR, R = 1 << LR, B = F::P / R, n = F::n;
    constexpr int ls = LG - REM, s = 1 << ls;
    // this pass's twiddles first, all of them: read between the region
    // stores they would each wait for the stores before them
    constexpr int NW = REM > LR ? R - 1 : 0;
    cplx<T> wt[B][NW > 0 ? NW : 1];
    if constexpr (NW > 0) {
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const int p = ((lane + 64 * i) & ((n >> LR) - 1)) >> ls;
#pragma unroll
            for (int k = 0; k < NW; ++k) wt[i][k] = tw[(tw_entries(LG) - tw_entries(REM)) + p * NW + k];
        }
    }
#pragma unroll
    for (int i = 0; i < B; ++i) {
        const int b = lane + 64 * i;
        const int seq = b >> (LG - LR), t = b & ((n >> LR) - 1);
        const int q = t & (s - 1), p = t >> ls;
        cplx<T> *a = &v[i * R];
        if constexpr (R == 8) dft8(a);
        else if constexpr (R == 4) dft4(a[0], a[1], a[2], a[3]);
        else dft2(a);
        const int base = (seq << LG) + q + s * R * p;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            cplx<T> o = a[k];
            if constexpr (NW > 0) {
                if (k > 0) o = cmul(o, wt[i][k - 1]);
            }
            buf[pidx(base + s * k)] = o;
        }
    }
    wave_sync();
    if constexpr (REM > LR) {
        constexpr int REM2 = REM - LR, LR2 = PassRadix<REM2>::LR, R2 = 1 << LR2;
#pragma unroll
        for (int i = 0; i < F::P / R2; ++i) {
#pragma unroll
            for (int k = 0; k < R2; ++k) {
                int seq, idx;
                pass_input<LG, LR2>(lane, i, k, seq, idx);
                v[i * R2 + k] = buf[pidx((seq << LG) + idx)];
            }
        }
        wave_sync();
        wave_fft<T, LG, REM2>(v, buf, tw, lane);
    }
}

// Per-pass twiddle tables of a length-2^LG transform from the natural table
// exp(-2 pi i t/n): pass at sub-length 2^rem, stride s = 2^(LG-rem), entry
// (p, k) = exp(-2 pi i k p s / n).  Block-cooperative.
template <typename T, int LG>
__device__ __forceinline__ void fill_pass_twiddles(cplx<T> *dst, const cplx<T> *__restrict__ nat)
{
    constexpr int n = 1 << LG;
    int off = 0;
    for (int rem = LG; rem > 0;) {
        const int lr = pass_lr(rem), r = 1 << lr;
        if (rem > lr) {
            const int m = 1 << (rem - lr), s = 1 << (LG - rem);
            for (int e = threadIdx.x; e < m * (r - 1); e += blockDim.x) {
                const int p = e / (r - 1), k = e - p * (r - 1) + 1;
                dst[off + e] = nat[(k * p * s) & (n - 1)];
            }
            off += m * (r - 1);
        }
        rem -= lr;
    }
}

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
// 8 (8 row pairs give 128-byte runs per kx in the kx-major store).
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
    k_sk_rows(StepArg sarg, const T *__restrict__ field, int ny, double u0, const cplx<T> *__restrict__ twx,
              cplx<T> *__restrict__ half)
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
    const T su0 = static_cast<T>(u0);
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
    // kx-major store: per kx a run of 2*npairs consecutive y (rows fastest)
    constexpr int nh = n / 2 + 1;
    const int nrow = 2 * npairs;  // a power of two (ny and W S are)
    const int lrow = 31 - __builtin_clz(nrow);
    constexpr int lS = 31 - __builtin_clz(S);
    cplx<T> *h = half + static_cast<int64_t>(inst) * nh * ny + 2 * pair0;
    for (int e = threadIdx.x; e < nrow * nh; e += blockDim.x) {
        const int k = e >> lrow, rr = e & (nrow - 1);
        const int pair = rr >> 1;
        const cplx<T> *z0 = reg + (pair >> lS) * F::lds;
        const int sb = (pair & (S - 1)) << LGX;
        const cplx<T> z = z0[pidx(sb + k)];
        const cplx<T> zm = z0[pidx(sb + ((n - k) & (n - 1)))];
        // A = (z + conj zm)/2 (row 2q), B = (z - conj zm)/(2i) (row 2q+1)
        const cplx<T> o = (rr & 1) ? cplx<T>{T(0.5) * (z.im + zm.im), T(-0.5) * (z.re - zm.re)}
                                   : cplx<T>{T(0.5) * (z.re + zm.re), T(0.5) * (z.im - zm.im)};
        h[static_cast<int64_t>(k) * ny + rr] = o;
    }
}

// LDS bytes per wave of the column transform: its transform region and the
// FP64 prefix sums of one column.  A wave that holds one column per
// transform (S = 1) writes the prefix sums over that column once it has read
// it, so they need no room of their own.
constexpr int col_region(int es, int lg)
{
    return es * wave_lds(lg) + (wave_seqs(lg) == 1 ? 0 : 8 * ((1 << lg) / 2 + 1));
}

// Waves per block of the column transform: 4, or 2 where 4 regions and the
// twiddles exceed the LDS budget (the largest FP64 columns).
constexpr int col_waves(int es, int lg)
{
    return es * tw_entries(lg) + 4 * col_region(es, lg) <= kLdsBudget ? 4 : 2;
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

// Loads the column group of one wave iteration (S columns from `g`) in the
// first pass's order; columns beyond nh are zero.
template <typename T, int LGY>
__device__ __forceinline__ void load_cols(cplx<T> (&v)[WaveFft<LGY>::P], const cplx<T> *__restrict__ hc, int g,
                                          int nh, int lane)
{
    using F = WaveFft<LGY>;
    constexpr int LR = PassRadix<LGY>::LR, R = 1 << LR;
#pragma unroll
    for (int i = 0; i < F::P / R; ++i) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            int seq, y;
            pass_input<LGY, LR>(lane, i, k, seq, y);
            v[i * R + k] = g + seq < nh ? hc[(static_cast<int64_t>(g + seq) << LGY) + y] : cplx<T>{T(0), T(0)};
        }
    }
}

// grid: (groups, n_inst); block 64 CW; wave w handles, in iteration it, the
// S columns from cb + S (it CW + w).  LDS: pass twiddles, then
// per wave `rs` bytes: the transform region, the FP64 prefix sums of one
// column (within the transform region when S = 1), and (after the loop) the
// wave's shell sums.
template <typename T, int LGY, int NBJ>
__global__ void __launch_bounds__(256)
    k_sk_cols(StepArg sarg, const cplx<T> *__restrict__ half, int nx, int iters, int rs, int nbins,
              const cplx<T> *__restrict__ twy, double *__restrict__ part)
{
    SHE_SAMPLE_GATE();
    using F = WaveFft<LGY>;
    constexpr int n = F::n, P = F::P, S = F::S, hy = n / 2;
    constexpr int CW = col_waves(static_cast<int>(sizeof(cplx<T>)), LGY);
    constexpr int per = (hy + 1 + 63) >> 6;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *tw = reinterpret_cast<cplx<T> *>(smem_raw);
    unsigned char *regions = smem_raw + sizeof(cplx<T>) * F::tw;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    cplx<T> *buf = reinterpret_cast<cplx<T> *>(regions + static_cast<size_t>(wave) * rs);
    double *pre = S == 1 ? reinterpret_cast<double *>(buf) : reinterpret_cast<double *>(buf + F::lds);
    const int inst = blockIdx.y;
    const int nh = nx / 2 + 1;
    const int cb = blockIdx.x * (CW * S * iters);
    const cplx<T> *hc = half + static_cast<int64_t>(inst) * nh * n;
    fill_pass_twiddles<T, LGY>(tw, twy);
    const int nbj = (nbins + 63) >> 6;
    double acc[NBJ];
#pragma unroll
    for (int j = 0; j < NBJ; ++j) acc[j] = 0.0;
    cplx<T> nxt[P];
    load_cols<T, LGY>(nxt, hc, cb + S * wave, nh, lane);
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
        const int g = cb + S * (it * CW + wave);
        if (g >= nh) break;  // wave-uniform; later iterations are further right
        cplx<T> v[P];
#pragma unroll
        for (int j = 0; j < P; ++j) v[j] = nxt[j];
        if (it + 1 < iters) load_cols<T, LGY>(nxt, hc, g + S * CW, nh, lane);
        wave_fft<T, LGY, LGY>(v, buf, tw, lane);
        for (int c = 0; c < S && g + c < nh; ++c) {
            const int kx = g + c;
            // mirrored half of the spectrum: weight 2 off the kx = 0 and Nx/2
            // columns, applied to the shell sums (an exact scaling)
            const double w = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
            const cplx<T> *col = buf;
            const int cbase = c << LGY;
            double loc[per];
            double run = 0.0;
#pragma unroll
            for (int j = 0; j < per; ++j) {
                // power at |ky| = m: X(m), plus X(-m) for 0 < m < hy; m > hy is
                // padding (both reads stay inside the column, masked after)
                const int m = lane * per + j;
                const cplx<T> a = col[pidx(cbase + min(m, hy))];
                const cplx<T> b = col[pidx(cbase + ((n - m) & (n - 1)))];
                const T ea = m <= hy ? a.re * a.re + a.im * a.im : T(0);
                const T eb = (m != 0 && m < hy) ? b.re * b.re + b.im * b.im : T(0);
                run += static_cast<double>(ea) + static_cast<double>(eb);
                loc[j] = run;
            }
            const double excl = wave_inclusive_sum(run) - run;
            if (S == 1) wave_sync();  // the prefix sums overwrite the column just read
#pragma unroll
            for (int j = 0; j < per; ++j) {
                const int m = lane * per + j;
                if (m <= hy) pre[m] = excl + loc[j];
            }
            wave_sync();
            // shells met by this column: kx .. round(sqrt(kx^2 + hy^2)) (bound by
            // excess).  Lane b takes the end of its shell, first(b + 1); the start,
            // first(b), is the end of lane b - 1 (a whole-wave shift by one lane),
            // and for lane 0 the end of lane 63 in the previous group (0 for the
            // first group met: its shells lie below kx).
            const int kx4 = 4 * kx * kx;
            const int jlo = kx >> 6;
            const int jhi = static_cast<int>(__builtin_amdgcn_sqrtf(static_cast<float>(kx * kx + hy * hy)) + 1.5f) >> 6;
            int carry = 0;
#pragma unroll
            for (int j = 0; j < NBJ; ++j) {
                if (j >= jlo && j <= jhi && j < nbj) {
                    const int b = lane + 64 * j;
                    const int m1 = shell_first(kx4, b + 1, hy);
                    const int m0 = __builtin_amdgcn_update_dpp(carry, m1, 0x138, 0xf, 0xf, false);  // wave_shr:1
                    carry = __builtin_amdgcn_readlane(m1, 63);
                    if (b < nbins && m1 > m0) acc[j] += w * (pre[m1 - 1] - (m0 > 0 ? pre[m0 - 1] : 0.0));
                }
            }
            wave_sync();
        }
    }
    __syncthreads();
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
    double s = 0.0;
    for (int g = 0; g < ngroups; ++g) s += pp[static_cast<int64_t>(g) * nbins];
    const double tot = sums[e] + s;
    sums[e] = tot;
    // The sample reduction ran first and folded the spatial sums of a batch
    // this sample completed; fold the shells' batch averages too (the k = 0
    // shell restored from the batch's spatial-mean sum, as at finalisation).
    if (bk.len > 0 && q.n_samples % bk.len == 0) {
        const double L = static_cast<double>(bk.len), N = bk.cells;
        double v = tot - bk.snap[e];
        if (b == 0) v += L * N * N * bk.u0 * bk.u0 + 2.0 * N * bk.u0 * (N * q.batch_sp_mean);
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

int elem_bytes(int prec)
{
    return prec == 0 ? static_cast<int>(sizeof(cplx<float>)) : static_cast<int>(sizeof(cplx<double>));
}

// column iterations per wave: about 2048 blocks in flight over the batch
int col_iters(int prec, int nx, int ny, int n_inst)
{
    const int nh = nx / 2 + 1;
    const int per_iter = col_waves(elem_bytes(prec), ilog2(ny)) * wave_seqs(ilog2(ny));
    const int64_t groups = static_cast<int64_t>((nh + per_iter - 1) / per_iter) * n_inst;
    int it = 1;
    while (it < 8 && groups / (2 * it) >= 2048) it *= 2;
    return it;
}

}  // namespace

int sk2d_groups(int prec, int nx, int ny, int n_inst)
{
    const int nh = nx / 2 + 1;
    const int per_block =
        col_waves(elem_bytes(prec), ilog2(ny)) * wave_seqs(ilog2(ny)) * col_iters(prec, nx, ny, n_inst);
    return (nh + per_block - 1) / per_block;
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
void rows_t(hipStream_t s, const StepArg &sa, int n_inst, int ny, double u0, const void *field, const void *twx,
            void *half)
{
    using F = WaveFft<LGX>;
    constexpr int W = row_waves<T, LGX>();
    const int pairs = W * F::S;
    const dim3 grid((ny / 2 + pairs - 1) / pairs, n_inst);
    const size_t smem = sizeof(cplx<T>) * (F::tw + static_cast<size_t>(W) * F::lds);
    static_assert(sizeof(cplx<T>) * (F::tw + W * F::lds) <= kLdsBudget, "row transform exceeds the LDS budget");
    hipLaunchKernelGGL((k_sk_rows<T, LGX>), grid, dim3(64 * W), smem, s, sa, static_cast<const T *>(field), ny, u0,
                       static_cast<const cplx<T> *>(twx), static_cast<cplx<T> *>(half));
}

template <typename T, int LGY>
bool cols_t(hipStream_t s, const StepArg &sa, int n_inst, int nx, int nbins, const void *half, const void *twy,
            double *part, int groups, int iters)
{
    using F = WaveFft<LGY>;
    constexpr int CW = col_waves(static_cast<int>(sizeof(cplx<T>)), LGY);
    size_t rs = col_region(static_cast<int>(sizeof(cplx<T>)), LGY);
    rs = std::max(rs, sizeof(double) * static_cast<size_t>(nbins));
    rs = (rs + 15) & ~static_cast<size_t>(15);
    const size_t smem = sizeof(cplx<T>) * F::tw + CW * rs;
    if (smem > kLdsBudget) return false;
    if (nbins <= 64 * (kMaxBinIters / 2))
        hipLaunchKernelGGL((k_sk_cols<T, LGY, kMaxBinIters / 2>), dim3(groups, n_inst), dim3(64 * CW), smem, s, sa,
                           static_cast<const cplx<T> *>(half), nx, iters, static_cast<int>(rs), nbins,
                           static_cast<const cplx<T> *>(twy), part);
    else
        hipLaunchKernelGGL((k_sk_cols<T, LGY, kMaxBinIters>), dim3(groups, n_inst), dim3(64 * CW), smem, s, sa,
                           static_cast<const cplx<T> *>(half), nx, iters, static_cast<int>(rs), nbins,
                           static_cast<const cplx<T> *>(twy), part);
    return true;
}

template <typename T>
bool rows_dispatch(int lgx, hipStream_t s, const StepArg &sa, int n_inst, int ny, double u0, const void *field,
                   const void *twx, void *half)
{
#define SHE_ROWS(L)                                                 \
    case L:                                                         \
        rows_t<T, L>(s, sa, n_inst, ny, u0, field, twx, half);      \
        return true;
    switch (lgx) {
        SHE_ROWS(3) SHE_ROWS(4) SHE_ROWS(5) SHE_ROWS(6) SHE_ROWS(7) SHE_ROWS(8) SHE_ROWS(9) SHE_ROWS(10)
    default: return false;
    }
#undef SHE_ROWS
}

template <typename T>
bool cols_dispatch(int lgy, hipStream_t s, const StepArg &sa, int n_inst, int nx, int nbins, const void *half,
                   const void *twy, double *part, int groups, int iters)
{
#define SHE_COLS(L)                                                                      \
    case L:                                                                              \
        return cols_t<T, L>(s, sa, n_inst, nx, nbins, half, twy, part, groups, iters);
    switch (lgy) {
        SHE_COLS(1) SHE_COLS(2) SHE_COLS(3) SHE_COLS(4) SHE_COLS(5) SHE_COLS(6) SHE_COLS(7) SHE_COLS(8)
        SHE_COLS(9) SHE_COLS(10)
    default: return false;
    }
#undef SHE_COLS
}

}  // namespace

hipError_t launch_sk2d(int prec, hipStream_t s, const StepArg &sa, int n_inst, int nx, int ny, double u0,
                       const void *field, void *half, const void *twx, const void *twy, double *part, int nbins,
                       double *sums, const InstAcc *acc, const BatchSk &bk)
{
    if (nbins > 64 * kMaxBinIters) return hipErrorInvalidValue;
    const int lgx = ilog2(nx), lgy = ilog2(ny);
    const int iters = col_iters(prec, nx, ny, n_inst);
    const int groups = sk2d_groups(prec, nx, ny, n_inst);
    bool ok;
    if (prec == 0) {
        ok = rows_dispatch<float>(lgx, s, sa, n_inst, ny, u0, field, twx, half) &&
             cols_dispatch<float>(lgy, s, sa, n_inst, nx, nbins, half, twy, part, groups, iters);
    } else {
        ok = rows_dispatch<double>(lgx, s, sa, n_inst, ny, u0, field, twx, half) &&
             cols_dispatch<double>(lgy, s, sa, n_inst, nx, nbins, half, twy, part, groups, iters);
    }
    if (!ok) return hipErrorInvalidValue;
    const int64_t tot = static_cast<int64_t>(n_inst) * nbins;
    hipLaunchKernelGGL(k_bins_reduce, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, s, sa, part,
                       groups, nbins, n_inst, sums, acc, bk);
    return hipGetLastError();
}

}  // namespace she
