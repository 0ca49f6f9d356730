// Radially binned static structure factor of 2D fields on sample steps.
//
// S(k) = <|U_k|^2> with U_k = sum_j U_j exp(-2 pi i (j.k)/N) (Garcia et al.,
// Sec. 3, structure factor), averaged over the modes of each shell
// round(|k|), signed k in [-N/2, N/2).  The transform is taken of the shifted
// field dU = U - u0 (which changes only the k = 0 mode; the finalisation
// restores that mode exactly from the spatial sums), in the state's precision.
//
// 1. k_fft_rows: two real rows are packed as one complex sequence
//    (dU_a + i dU_b), transformed along x in LDS, separated into the two half
//    spectra A_k = (Z_k + conj Z_-k)/2, B_k = (Z_k - conj Z_-k)/(2i), and
//    stored column-major (kx-major, y fastest) so that a block of 2*RP rows
//    writes runs of 2*RP consecutive y per kx.
// 2. k_fft_cols: CW half-spectrum columns (contiguous in memory) are
//    transformed along y in LDS, the power |X|^2 is formed with weight 2 for
//    0 < kx < Nx/2 (the mirrored half of the spectrum), and binned without
//    atomics: per column a wave forms the FP64 prefix sum P(m) of the power
//    over |ky| <= m (fixed-order scan), and thread b adds, column by column,
//    P(hi-1) - P(lo-1) over the range [lo(kx, b), lo(kx, b+1)) of |ky| read
//    from an integer table built from (2b-1)^2 <= 4(kx^2 + ky^2) < (2b+1)^2.
//    The per-block shell sums go to a partial buffer.
// 3. k_bins_reduce: per instance and shell, the partials are added in a fixed
//    order to the FP64 running sums.
//
// The transforms are Stockham autosort passes (radix 4, a final radix 2 for
// odd log2 n; natural order in and out, so the LDS reads of a pass are
// contiguous), with the twiddle table exp(-2 pi i t/n) precomputed once per
// handle.
#include "she_internal.hpp"

namespace she {

template <typename T>
struct cplx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> w)
{
    return cplx<T>{a.re * w.re - a.im * w.im, a.re * w.im + a.im * w.re};
}

// One pass of the Stockham autosort FFT (decimation in frequency, radix
// R = 2^LR) over `count` sequences of length n = 2^lg stored contiguously in
// LDS, natural order in and out.  Current sub-transform length 2^rem, stride
// s = 2^(lg - rem), m = 2^(rem - LR): butterfly t = q + s p (q < s, p < m)
// reads x[t + k n/R], forms the R-point DFT, multiplies output k by
// exp(-2 pi i k p s / n) and writes it to x[q + s (R p + k)].  All reads of a
// pass are staged in registers between two barriers, so one buffer serves.
// tw holds exp(-2 pi i t/n), t < n.  At most kPts/R butterflies per thread.
constexpr int kPts = 16;  // points staged per thread and pass

template <typename T, int LG, int REM, int LR>
__device__ __forceinline__ void stockham_pass(cplx<T> *buf, int count, const cplx<T> *tw)
{
    constexpr int R = 1 << LR;
    constexpr int MAXB = kPts / R;
    constexpr int lg = LG;
    constexpr int n = 1 << lg;
    constexpr int ls = lg - REM;
    const int nbf = count << (lg - LR);
    cplx<T> v[MAXB][R];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * blockDim.x;
        if (b < nbf) {
            const int seq = b >> (lg - LR), t = b & ((n >> LR) - 1);
            const cplx<T> *x = buf + (seq << lg);
            cplx<T> a[R];
#pragma unroll
            for (int k = 0; k < R; ++k) a[k] = x[t + k * (n >> LR)];
            const int p = t >> ls;
            if constexpr (R == 4) {
                const cplx<T> t0{a[0].re + a[2].re, a[0].im + a[2].im};
                const cplx<T> t1{a[0].re - a[2].re, a[0].im - a[2].im};
                const cplx<T> t2{a[1].re + a[3].re, a[1].im + a[3].im};
                const cplx<T> t3{a[1].im - a[3].im, a[3].re - a[1].re};  // -i (a1 - a3)
                v[i][0] = cplx<T>{t0.re + t2.re, t0.im + t2.im};
                v[i][1] = cmul(cplx<T>{t1.re + t3.re, t1.im + t3.im}, tw[p << ls]);
                v[i][2] = cmul(cplx<T>{t0.re - t2.re, t0.im - t2.im}, tw[(2 * p) << ls]);
                v[i][3] = cmul(cplx<T>{t1.re - t3.re, t1.im - t3.im}, tw[(3 * p) << ls]);
            } else {
                v[i][0] = cplx<T>{a[0].re + a[1].re, a[0].im + a[1].im};
                v[i][1] = cmul(cplx<T>{a[0].re - a[1].re, a[0].im - a[1].im}, tw[p << ls]);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * blockDim.x;
        if (b < nbf) {
            const int seq = b >> (lg - LR), t = b & ((n >> LR) - 1);
            const int q = t & ((1 << ls) - 1), p = t >> ls;
            cplx<T> *x = buf + (seq << lg);
#pragma unroll
            for (int k = 0; k < R; ++k) x[q + ((R * p + k) << ls)] = v[i][k];
        }
    }
    __syncthreads();
}

// FFTs of `count` contiguous sequences of length 2^LG in LDS, natural order
// in and out; count << LG must not exceed kPts * blockDim.x.
template <typename T, int LG, int REM = LG>
__device__ __forceinline__ void fft_stockham(cplx<T> *buf, int count, const cplx<T> *tw)
{
    if constexpr (REM >= 2) {
        stockham_pass<T, LG, REM, 2>(buf, count, tw);
        fft_stockham<T, LG, REM - 2>(buf, count, tw);
    } else if constexpr (REM == 1) {
        stockham_pass<T, LG, 1, 1>(buf, count, tw);
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

// grid: (ceil(ny/2 / rp), n_inst); block 256; LDS: rp*nx complex + nx twiddles.
// Output: half[inst][kx][y], kx = 0..nx/2.
template <typename T, int LGX>
__global__ void __launch_bounds__(256)
    k_fft_rows(StepArg sarg, const T *__restrict__ field, int ny, int rp, double u0, const cplx<T> *__restrict__ twx,
               cplx<T> *__restrict__ half)
{
    {
        int64_t step;
        int sample;
        resolve_step(sarg, step, sample);
        if (!sample) return;  // a non-sample step of a captured graph
    }
    constexpr int nx = 1 << LGX;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *tw = buf + rp * nx;
    const int inst = blockIdx.y;
    const int pair0 = blockIdx.x * rp;
    const int npairs = min(rp, ny / 2 - pair0);
    constexpr int bits = LGX;
    constexpr int nh = nx / 2 + 1;
    for (int t = threadIdx.x; t < nx; t += blockDim.x) tw[t] = twx[t];
    const T *f = field + static_cast<int64_t>(inst) * nx * ny;
    const T su0 = static_cast<T>(u0);
    for (int e = threadIdx.x; e < npairs * nx; e += blockDim.x) {
        const int q = e >> bits, j = e & (nx - 1);
        const int ya = 2 * (pair0 + q);
        const T a = f[static_cast<int64_t>(ya) * nx + j] - su0;
        const T b = f[static_cast<int64_t>(ya + 1) * nx + j] - su0;
        buf[q * nx + j] = cplx<T>{a, b};
    }
    __syncthreads();
    fft_stockham<T, LGX>(buf, npairs, tw);
    cplx<T> *h = half + static_cast<int64_t>(inst) * nh * ny;
    const int nrow = 2 * npairs;  // a power of two (ny and rp are)
    const int lrow = 31 - __builtin_clz(nrow);
    // thread e -> (k, row within the block), rows fastest: runs of nrow y per kx
    for (int e = threadIdx.x; e < nrow * nh; e += blockDim.x) {
        const int k = e >> lrow, rr = e & (nrow - 1);
        const int q = rr >> 1;
        const cplx<T> z = buf[q * nx + k];
        const cplx<T> zm = buf[q * nx + ((nx - k) & (nx - 1))];
        // A = (z + conj zm)/2 (row 2q), B = (z - conj zm)/(2i) (row 2q+1)
        const cplx<T> v = (rr & 1) ? cplx<T>{T(0.5) * (z.im + zm.im), T(-0.5) * (z.re - zm.re)}
                                   : cplx<T>{T(0.5) * (z.re + zm.re), T(0.5) * (z.im - zm.im)};
        h[static_cast<int64_t>(k) * ny + 2 * pair0 + rr] = v;
    }
}

// grid: (ceil(nh / cw), n_inst); block 256; LDS: cw*ny complex + ny twiddles.
// lo: nh x (nbins + 1) table of the first |ky| of each shell per column.
template <typename T, int LGY>
__global__ void __launch_bounds__(256)
    k_fft_cols(StepArg sarg, const cplx<T> *__restrict__ half, int nx, int cw, int nbins,
               const cplx<T> *__restrict__ twy, const int32_t *__restrict__ lo, double *__restrict__ part)
{
    {
        int64_t step;
        int sample;
        resolve_step(sarg, step, sample);
        if (!sample) return;  // a non-sample step of a captured graph
    }
    constexpr int ny = 1 << LGY;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *tw = buf + cw * ny;
    const int inst = blockIdx.y;
    const int nh = nx / 2 + 1;
    const int c0 = blockIdx.x * cw;
    const int ncol = min(cw, nh - c0);
    constexpr int bits = LGY;
    for (int t = threadIdx.x; t < ny; t += blockDim.x) tw[t] = twy[t];
    const cplx<T> *h = half + (static_cast<int64_t>(inst) * nh + c0) * ny;
    for (int e = threadIdx.x; e < ncol * ny; e += blockDim.x) buf[e] = h[e];
    __syncthreads();
    fft_stockham<T, LGY>(buf, ncol, tw);
    // power with the mirror weight, in place (re := |X|^2 w)
    for (int e = threadIdx.x; e < ncol * ny; e += blockDim.x) {
        const int kx = c0 + (e >> bits);
        const T w = (kx == 0 || kx == nx / 2) ? T(1) : T(2);
        const cplx<T> v = buf[e];
        buf[e].re = w * (v.re * v.re + v.im * v.im);
    }
    __syncthreads();
    // Per column, P(m) = sum over |ky| <= m of the power (the +ky and -ky modes
    // together), as an FP64 prefix sum: each wave scans one column at a time,
    // lane l holding |ky| = l*per .. l*per + per - 1 (fixed order, no atomics).
    // The column's prefix sums overwrite the column's own storage (the wave has
    // read all of it into registers first; LDS accesses of a wave are ordered).
    constexpr int hy = ny / 2;
    {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
        constexpr int per = (hy + 1 + 63) >> 6;
        for (int c = wave; c < ncol; c += nwave) {
            const T *col = &buf[c * ny].re;
            double loc[per];
            double run = 0.0;
#pragma unroll
            for (int j = 0; j < per; ++j) {
                const int m = lane * per + j;
                double v = 0.0;
                if (m <= hy) {
                    v = static_cast<double>(col[2 * m]);
                    if (m != 0 && m != hy) v += static_cast<double>(col[2 * (ny - m)]);
                }
                run += v;
                loc[j] = run;
            }
            double incl = run;
            for (int d = 1; d < 64; d <<= 1) {
                const double o = __shfl_up(incl, d, 64);
                if (lane >= d) incl += o;
            }
            const double excl = incl - run;
            double *pref = reinterpret_cast<double *>(&buf[c * ny]);
#pragma unroll
            for (int j = 0; j < per; ++j) {
                const int m = lane * per + j;
                if (m <= hy) pref[m] = excl + loc[j];
            }
        }
    }
    __syncthreads();
    double *pp = part + (static_cast<int64_t>(inst) * gridDim.x + blockIdx.x) * nbins;
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
        double acc = 0.0;
        for (int c = 0; c < ncol; ++c) {
            const int32_t *lc = lo + static_cast<int64_t>(c0 + c) * (nbins + 1);
            const int m0 = lc[b], m1 = lc[b + 1];
            if (m1 > m0) {
                const double *pc = reinterpret_cast<const double *>(&buf[c * ny]);
                acc += pc[m1 - 1] - (m0 > 0 ? pc[m0 - 1] : 0.0);
            }
        }
        pp[b] = acc;
    }
}

__global__ void __launch_bounds__(256)
    k_bins_reduce(StepArg sarg, const double *__restrict__ part, int ngroups, int nbins, int n_inst,
                  double *__restrict__ sums, const InstAcc *__restrict__ acc)
{
    {
        int64_t step;
        int sample;
        resolve_step(sarg, step, sample);
        if (!sample) return;  // a non-sample step of a captured graph
    }
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e >= static_cast<int64_t>(n_inst) * nbins) return;
    const int inst = static_cast<int>(e / nbins), b = static_cast<int>(e - static_cast<int64_t>(inst) * nbins);
    if (acc[inst].nonfinite) return;
    const double *pp = part + static_cast<int64_t>(inst) * ngroups * nbins + b;
    double s = 0.0;
    for (int g = 0; g < ngroups; ++g) s += pp[static_cast<int64_t>(g) * nbins];
    sums[e] += s;
}

// LDS-fitting shapes: row pairs per block and columns per block; each block
// transforms at most kPts * 256 points (the registers of one pass).
void sk2d_shape(int prec, int nx, int ny, int *rp, int *cw)
{
    const size_t es = prec == 0 ? 2 * sizeof(float) : 2 * sizeof(double);
    const size_t budget = 64 * 1024;
    int r = 1;
    while (r < 8 && r * 2 <= ny / 2 && 2 * r * nx <= kPts * 256 &&
           (static_cast<size_t>(2 * r) * nx + nx) * es <= budget)
        r *= 2;
    int c = 1;
    while (c < 64 && c * 2 <= nx / 2 + 1 && 2 * c * ny <= kPts * 256 &&
           (static_cast<size_t>(2 * c) * ny + ny) * es <= budget)
        c *= 2;
    *rp = r;
    *cw = c;
}

int sk2d_groups(int prec, int nx, int ny)
{
    int rp, cw;
    sk2d_shape(prec, nx, ny, &rp, &cw);
    return (nx / 2 + 1 + cw - 1) / cw;
}

// First |ky| of shell b in column kx (b = 0..nbins), clipped to [0, ny/2 + 1]:
// the smallest m >= 0 with 4 (kx^2 + m^2) >= (2b - 1)^2 (b = 0: m = 0).
void sk2d_shell_table(int nx, int ny, int nbins, int32_t *lo)
{
    const int nh = nx / 2 + 1, hy = ny / 2;
    for (int kx = 0; kx < nh; ++kx) {
        for (int b = 0; b <= nbins; ++b) {
            int m = 0;
            if (b > 0) {
                const long long need = static_cast<long long>(2 * b - 1) * (2 * b - 1) - 4LL * kx * kx;
                while (m <= hy && 4LL * m * m < need) ++m;
            }
            lo[static_cast<int64_t>(kx) * (nbins + 1) + b] = m > hy + 1 ? hy + 1 : m;
        }
    }
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

template <typename T, int LGX, int LGY>
static void sk2d_launch_t(hipStream_t s, const StepArg &sa, dim3 g1, dim3 g2, size_t sm1, size_t sm2, int nx, int ny, int rp, int cw,
                          int nbins, double u0, const void *field, void *half, const void *twx, const void *twy,
                          const int32_t *lo, double *part)
{
    using C = cplx<T>;
    hipLaunchKernelGGL((k_fft_rows<T, LGX>), g1, dim3(256), sm1, s, sa, static_cast<const T *>(field), ny, rp, u0,
                       static_cast<const C *>(twx), static_cast<C *>(half));
    hipLaunchKernelGGL((k_fft_cols<T, LGY>), g2, dim3(256), sm2, s, sa, static_cast<const C *>(half), nx, cw, nbins,
                       static_cast<const C *>(twy), lo, part);
}

template <typename T, int LGX>
static bool sk2d_launch_y(int lgy, hipStream_t s, const StepArg &sa, dim3 g1, dim3 g2, size_t sm1, size_t sm2, int nx, int ny, int rp,
                          int cw, int nbins, double u0, const void *field, void *half, const void *twx,
                          const void *twy, const int32_t *lo, double *part)
{
#define SHE_SK_Y(L)                                                                                             \
    case L:                                                                                                     \
        sk2d_launch_t<T, LGX, L>(s, sa, g1, g2, sm1, sm2, nx, ny, rp, cw, nbins, u0, field, half, twx, twy, lo, part); \
        return true;
    switch (lgy) {
        SHE_SK_Y(1) SHE_SK_Y(2) SHE_SK_Y(3) SHE_SK_Y(4) SHE_SK_Y(5) SHE_SK_Y(6) SHE_SK_Y(7) SHE_SK_Y(8)
        SHE_SK_Y(9) SHE_SK_Y(10)
    default: return false;
    }
#undef SHE_SK_Y
}

template <typename T>
static bool sk2d_launch(int lgx, int lgy, hipStream_t s, const StepArg &sa, dim3 g1, dim3 g2, size_t sm1, size_t sm2, int nx, int ny,
                        int rp, int cw, int nbins, double u0, const void *field, void *half, const void *twx,
                        const void *twy, const int32_t *lo, double *part)
{
#define SHE_SK_X(L)                                                                                               \
    case L:                                                                                                       \
        return sk2d_launch_y<T, L>(lgy, s, sa, g1, g2, sm1, sm2, nx, ny, rp, cw, nbins, u0, field, half, twx, twy, lo, \
                                   part);
    switch (lgx) {
        SHE_SK_X(3) SHE_SK_X(4) SHE_SK_X(5) SHE_SK_X(6) SHE_SK_X(7) SHE_SK_X(8) SHE_SK_X(9) SHE_SK_X(10)
    default: return false;
    }
#undef SHE_SK_X
}

hipError_t launch_sk2d(int prec, hipStream_t s, const StepArg &sa, int n_inst, int nx, int ny, double u0, const void *field, void *half,
                       const void *twx, const void *twy, const int32_t *lo, double *part, int nbins, double *sums,
                       const InstAcc *acc)
{
    int rp, cw;
    sk2d_shape(prec, nx, ny, &rp, &cw);
    const int nh = nx / 2 + 1;
    const int ngroups = (nh + cw - 1) / cw;
    const int lgx = 31 - __builtin_clz(nx), lgy = 31 - __builtin_clz(ny);
    const dim3 g1((ny / 2 + rp - 1) / rp, n_inst), g2(ngroups, n_inst);
    bool ok;
    if (prec == 0) {
        const size_t es = sizeof(cplx<float>);
        const size_t sm1 = (static_cast<size_t>(rp) * nx + nx) * es;
        const size_t sm2 = (static_cast<size_t>(cw) * ny + ny) * es;
        ok = sk2d_launch<float>(lgx, lgy, s, sa, g1, g2, sm1, sm2, nx, ny, rp, cw, nbins, u0, field, half, twx, twy, lo,
                                part);
    } else {
        const size_t es = sizeof(cplx<double>);
        const size_t sm1 = (static_cast<size_t>(rp) * nx + nx) * es;
        const size_t sm2 = (static_cast<size_t>(cw) * ny + ny) * es;
        ok = sk2d_launch<double>(lgx, lgy, s, sa, g1, g2, sm1, sm2, nx, ny, rp, cw, nbins, u0, field, half, twx, twy, lo,
                                 part);
    }
    if (!ok) return hipErrorInvalidValue;
    const int64_t tot = static_cast<int64_t>(n_inst) * nbins;
    hipLaunchKernelGGL(k_bins_reduce, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, s, sa, part, ngroups,
                       nbins, n_inst, sums, acc);
    return hipGetLastError();
}

}  // namespace she
