// Wave-level FFT building blocks shared by the structure-factor kernels and
// the sample launches of the 2D step kernel: complex arithmetic, the shape of
// a per-wave transform, radix-8/4/2 Stockham passes through the wave's own LDS
// region, and the per-pass twiddle tables.
#pragma once

#include <hip/hip_runtime.h>

namespace she {

// Aligned to its size, so that one lane's point moves in one 64-bit (FP32)
// or 128-bit (FP64) LDS access; at the alignment of T every exchange store
// and load splits into two, and the transforms are bound by the LDS.
template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T re, im;
};

// Every function below states its rounding: multiply-adds are written out as
// fma and nothing else is contracted, so a transform gives the same bits in
// every kernel it is inlined into.

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
#pragma clang fp contract(off)
    return cplx<T>{fma(a.re, w.re, -(a.im * w.im)), fma(a.re, w.im, a.im * w.re)};
}

// Half spectra of two real sequences a, b transformed together as z = a + i b,
// doubled: from Z_k and Z_(-k), 2 A_k = Z_k + conj Z_(-k) and
// 2 B_k = (Z_k - conj Z_(-k)) / i.  The factor 2 is exact, and the power sums
// take the 1/4 back once per column.
template <typename T>
__device__ __forceinline__ cplx<T> unpack2_a(cplx<T> z, cplx<T> zm)
{
    return cplx<T>{z.re + zm.re, z.im - zm.im};
}

template <typename T>
__device__ __forceinline__ cplx<T> unpack2_b(cplx<T> z, cplx<T> zm)
{
    return cplx<T>{z.im + zm.im, zm.re - z.re};
}

// Shape of the per-wave transform of length n = 2^lg: P points per lane,
// S sequences per wave (64 P = S n), padded LDS entries per wave region
// (three pad entries per 32, see pidx).
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
    return (wave_seqs(lg) << lg) + 3 * (((wave_seqs(lg) << lg) - 1) >> 5) + 1;
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

// Three pad entries after every 32.  A 64-bit access of a wave is served 32
// lanes at a time by the 64 four-byte banks, so 32 lanes touching 32
// distinct entries modulo 32 are conflict-free.  With this padding the
// exchanges of the 512-point transform, entries l + 64 k and 8 l + k for lane
// l, are; those of the middle pass, (l & 7) + 64 (l >> 3) + 8 k, conflict
// two-way (a pad of one per 16 made all three two-way).  The pad of an entry
// is a multiple of the lane's part plus one of k, so every access is a
// per-lane base plus a constant offset.
__device__ __forceinline__ int pidx(int i)
{
    return i + 3 * (i >> 5);
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
#pragma clang fp contract(off)
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
// the transforms in natural order; with KEEP the last pass stores nothing and
// its outputs stay in v: for one sequence per wave (S = 1), slot i R + k
// holds element lane + 64 (i + k P/R).
template <typename T, int LG, int REM, bool KEEP = false>
__device__ __forceinline__ void wave_fft(cplx<T> (&v)[WaveFft<LG>::P], cplx<T> *buf, const cplx<T> *tw, int lane)
{
#pragma clang fp contract(off)
    using F = WaveFft<LG>;
    constexpr int LR = PassRadix<REM>::LR, R = 1 << LR, B = F::P / R, n = F::n;
    constexpr int ls = LG - REM, s = 1 << ls;
    // this pass's twiddles first, all of them: read between the region
    // stores they would each wait for the stores before them
    constexpr int NW = REM > LR ? R - 1 : 0;
    constexpr bool store = !KEEP || REM > LR;
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
        if constexpr (store) {
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
    }
    if constexpr (!store) return;
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
        wave_fft<T, LG, REM2, KEEP>(v, buf, tw, lane);
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

}  // namespace she
