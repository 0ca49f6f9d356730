// Radially binned static structure factor of 2D fields on sample steps.
//
// S(k) = <|U_k|^2> with U_k = sum_j U_j exp(-2 pi i (j.k)/N) (Garcia et al.,
// Sec. 3, structure factor), averaged over the modes of each shell
// round(|k|), signed k in [-N/2, N/2).  The transform is taken of the shifted
// field dU = U - u0 (which changes only the k = 0 mode; the host corrects that
// mode exactly from the spatial sums), in the state's precision.
//
// 1. k_fft_rows: two real rows are packed as one complex sequence
//    (dU_a + i dU_b), transformed along x (radix-2, in LDS), separated into the
//    two half spectra A_k = (Z_k + conj Z_-k)/2, B_k = (Z_k - conj Z_-k)/(2i)
//    and stored for k = 0..Nx/2.
// 2. k_fft_cols: CW half-spectrum columns are transformed along y in LDS, the
//    power |X|^2 is formed with weight 2 for 0 < kx < Nx/2 (the mirrored half
//    of the spectrum), and binned without atomics: thread b owns shell b and
//    sums, column by column, the exact integer range of |ky| with
//    (2b-1)^2 <= 4(kx^2 + ky^2) < (2b+1)^2, in a fixed order.  The per-block
//    shell sums go to a partial buffer.
// 3. k_bins_reduce: per instance and shell, the partials are added in a fixed
//    order to the FP64 running sums.
#include "she_internal.hpp"

namespace she {

template <typename T>
struct cplx {
    T re, im;
};

__device__ __forceinline__ unsigned bitrev(unsigned v, int bits)
{
    return __builtin_bitreverse32(v) >> (32 - bits);
}

template <typename T>
__device__ __forceinline__ void twiddle(int t, int n, T &c, T &s)
{
    double sn, cs;
    sincospi(-2.0 * static_cast<double>(t) / static_cast<double>(n), &sn, &cs);
    c = static_cast<T>(cs);
    s = static_cast<T>(sn);
}

// In-place radix-2 FFTs of `count` sequences of length n (power of two) held
// in bit-reversed order in LDS (sequence q at buf + q*stride), all threads of
// the block cooperating.  tw holds exp(-2 pi i t/n), t < n/2.
template <typename T>
__device__ void fft_lds(cplx<T> *buf, int count, int n, int stride, const cplx<T> *tw)
{
    const int half = n >> 1;
    for (int len = 2; len <= n; len <<= 1) {
        const int hl = len >> 1, step = n / len;
        const int total = count * half;
        for (int b = threadIdx.x; b < total; b += blockDim.x) {
            const int q = b / half, r = b - q * half;
            const int grp = r / hl, j = r - grp * hl;
            cplx<T> *base = buf + q * stride + grp * len;
            const cplx<T> w = tw[j * step];
            const cplx<T> u = base[j], v0 = base[j + hl];
            const cplx<T> v{v0.re * w.re - v0.im * w.im, v0.re * w.im + v0.im * w.re};
            base[j] = cplx<T>{u.re + v.re, u.im + v.im};
            base[j + hl] = cplx<T>{u.re - v.re, u.im - v.im};
        }
        __syncthreads();
    }
}

// grid: (ceil(ny/2 / RP), n_inst); block 256; LDS: RP*nx complex + nx/2 twiddles
template <typename T>
__global__ void __launch_bounds__(256)
    k_fft_rows(const T *__restrict__ field, int nx, int ny, int rp, double u0, cplx<T> *__restrict__ half)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *tw = buf + rp * nx;
    const int inst = blockIdx.y;
    const int pair0 = blockIdx.x * rp;
    const int npairs = min(rp, ny / 2 - pair0);
    const int bits = 31 - __builtin_clz(nx);
    const int nh = nx / 2 + 1;
    for (int t = threadIdx.x; t < nx / 2; t += blockDim.x) twiddle<T>(t, nx, tw[t].re, tw[t].im);
    const T *f = field + static_cast<int64_t>(inst) * nx * ny;
    const T su0 = static_cast<T>(u0);
    for (int e = threadIdx.x; e < npairs * nx; e += blockDim.x) {
        const int q = e / nx, j = e - q * nx;
        const int ya = 2 * (pair0 + q);
        const T a = f[static_cast<int64_t>(ya) * nx + j] - su0;
        const T b = f[static_cast<int64_t>(ya + 1) * nx + j] - su0;
        buf[q * nx + bitrev(j, bits)] = cplx<T>{a, b};
    }
    __syncthreads();
    fft_lds<T>(buf, npairs, nx, nx, tw);
    cplx<T> *h = half + static_cast<int64_t>(inst) * ny * nh;
    for (int e = threadIdx.x; e < npairs * nh; e += blockDim.x) {
        const int q = e / nh, k = e - q * nh;
        const cplx<T> z = buf[q * nx + k];
        const cplx<T> zm = buf[q * nx + ((nx - k) & (nx - 1))];
        // A = (z + conj zm)/2, B = (z - conj zm)/(2i)
        const cplx<T> A{T(0.5) * (z.re + zm.re), T(0.5) * (z.im - zm.im)};
        const cplx<T> B{T(0.5) * (z.im + zm.im), T(-0.5) * (z.re - zm.re)};
        const int ya = 2 * (pair0 + q);
        h[static_cast<int64_t>(ya) * nh + k] = A;
        h[static_cast<int64_t>(ya + 1) * nh + k] = B;
    }
}

// smallest m >= 0 with 4 m^2 >= v (v may be <= 0)
__device__ __forceinline__ int ceil_half_sqrt(long long v)
{
    if (v <= 0) return 0;
    long long m = static_cast<long long>(sqrt(static_cast<double>(v)) * 0.5);
    while (4 * m * m < v) ++m;
    while (m > 0 && 4 * (m - 1) * (m - 1) >= v) --m;
    return static_cast<int>(m);
}

// grid: (ceil(nh / cw), n_inst); block 256; LDS: cw*ny complex + ny/2 twiddles
template <typename T>
__global__ void __launch_bounds__(256)
    k_fft_cols(const cplx<T> *__restrict__ half, int nx, int ny, int cw, int nbins, double *__restrict__ part)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *tw = buf + cw * ny;
    const int inst = blockIdx.y;
    const int nh = nx / 2 + 1;
    const int c0 = blockIdx.x * cw;
    const int ncol = min(cw, nh - c0);
    const int bits = 31 - __builtin_clz(ny);
    for (int t = threadIdx.x; t < ny / 2; t += blockDim.x) twiddle<T>(t, ny, tw[t].re, tw[t].im);
    const cplx<T> *h = half + static_cast<int64_t>(inst) * ny * nh;
    for (int e = threadIdx.x; e < ncol * ny; e += blockDim.x) {
        const int y = e / ncol, c = e - y * ncol;
        buf[c * ny + bitrev(y, bits)] = h[static_cast<int64_t>(y) * nh + c0 + c];
    }
    __syncthreads();
    fft_lds<T>(buf, ncol, ny, ny, tw);
    // power with the mirror weight, in place (re := |X|^2 w)
    for (int e = threadIdx.x; e < ncol * ny; e += blockDim.x) {
        const int c = e / ny;
        const int kx = c0 + c;
        const T w = (kx == 0 || kx == nx / 2) ? T(1) : T(2);
        const cplx<T> v = buf[e];
        buf[e].re = w * (v.re * v.re + v.im * v.im);
    }
    __syncthreads();
    double *pp = part + (static_cast<int64_t>(inst) * gridDim.x + blockIdx.x) * nbins;
    const int hy = ny / 2;
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
        double acc = 0.0;
        for (int c = 0; c < ncol; ++c) {
            const long long kx = c0 + c;
            const long long lo2 = static_cast<long long>(2 * b - 1) * (2 * b - 1) - 4 * kx * kx;
            const long long hi2 = static_cast<long long>(2 * b + 1) * (2 * b + 1) - 4 * kx * kx;
            const int lo = b == 0 ? 0 : ceil_half_sqrt(lo2);
            const int hi = min(ceil_half_sqrt(hi2), hy + 1);
            const T *col = &buf[c * ny].re;
            for (int m = lo; m < hi; ++m) {
                if (m == 0 || m == hy) {
                    acc += static_cast<double>(col[2 * m]);
                } else {
                    acc += static_cast<double>(col[2 * m]);
                    acc += static_cast<double>(col[2 * (ny - m)]);
                }
            }
        }
        pp[b] = acc;
    }
}

__global__ void __launch_bounds__(256)
    k_bins_reduce(const double *__restrict__ part, int ngroups, int nbins, int n_inst, double *__restrict__ sums,
                  const InstAcc *__restrict__ acc)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e >= static_cast<int64_t>(n_inst) * nbins) return;
    const int inst = static_cast<int>(e / nbins), b = static_cast<int>(e - static_cast<int64_t>(inst) * nbins);
    if (acc[inst].nonfinite) return;
    const double *pp = part + static_cast<int64_t>(inst) * ngroups * nbins + b;
    double s = 0.0;
    for (int g = 0; g < ngroups; ++g) s += pp[static_cast<int64_t>(g) * nbins];
    sums[e] += s;
}

// LDS-fitting shapes: row pairs per block and columns per block.
void sk2d_shape(int prec, int nx, int ny, int *rp, int *cw)
{
    const size_t es = prec == 0 ? 2 * sizeof(float) : 2 * sizeof(double);
    const size_t budget = 48 * 1024;
    int r = 1;
    while (r < 8 && r * 2 <= ny / 2 && (static_cast<size_t>(2 * r) * nx + nx / 2) * es <= budget) r *= 2;
    int c = 1;
    while (c < 64 && c * 2 <= nx / 2 + 1 && (static_cast<size_t>(2 * c) * ny + ny / 2) * es <= budget) c *= 2;
    *rp = r;
    *cw = c;
}

int sk2d_groups(int prec, int nx, int ny)
{
    int rp, cw;
    sk2d_shape(prec, nx, ny, &rp, &cw);
    return (nx / 2 + 1 + cw - 1) / cw;
}

hipError_t launch_sk2d(int prec, hipStream_t s, int n_inst, int nx, int ny, double u0, const void *field, void *half,
                       double *part, int nbins, double *sums, const InstAcc *acc)
{
    int rp, cw;
    sk2d_shape(prec, nx, ny, &rp, &cw);
    const int nh = nx / 2 + 1;
    const int ngroups = (nh + cw - 1) / cw;
    const dim3 g1((ny / 2 + rp - 1) / rp, n_inst), g2(ngroups, n_inst);
    if (prec == 0) {
        const size_t sm1 = (static_cast<size_t>(rp) * nx + nx / 2) * sizeof(cplx<float>);
        const size_t sm2 = (static_cast<size_t>(cw) * ny + ny / 2) * sizeof(cplx<float>);
        hipLaunchKernelGGL(k_fft_rows<float>, g1, dim3(256), sm1, s, static_cast<const float *>(field), nx, ny, rp,
                           u0, static_cast<cplx<float> *>(half));
        hipLaunchKernelGGL(k_fft_cols<float>, g2, dim3(256), sm2, s, static_cast<const cplx<float> *>(half), nx, ny,
                           cw, nbins, part);
    } else {
        const size_t sm1 = (static_cast<size_t>(rp) * nx + nx / 2) * sizeof(cplx<double>);
        const size_t sm2 = (static_cast<size_t>(cw) * ny + ny / 2) * sizeof(cplx<double>);
        hipLaunchKernelGGL(k_fft_rows<double>, g1, dim3(256), sm1, s, static_cast<const double *>(field), nx, ny,
                           rp, u0, static_cast<cplx<double> *>(half));
        hipLaunchKernelGGL(k_fft_cols<double>, g2, dim3(256), sm2, s, static_cast<const cplx<double> *>(half), nx,
                           ny, cw, nbins, part);
    }
    const int64_t tot = static_cast<int64_t>(n_inst) * nbins;
    hipLaunchKernelGGL(k_bins_reduce, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, s, part, ngroups,
                       nbins, n_inst, sums, acc);
    return hipGetLastError();
}

}  // namespace she
