// 2D / 3D periodic grids: launch dispatch, sample reductions, initial state
// and finalisation.  The step kernels themselves are in she_step_nd.hpp.
#include "she_internal.hpp"
#include "she_rng.hpp"

namespace she {

// Typed launchers, instantiated in she_k2d_*.hip / she_k3d_*.hip.
template <typename T, int CX>
hipError_t step2d_e(int eq, int scheme, int n_blocks, hipStream_t s, const ParamsND &p, const void *src,
                    void *dst, const StepArg &sa, double *part, InstAcc *acc, const SkRows *skr);
template <typename T, int CX>
hipError_t step3d_e(int eq, int stage, int ty, int n_blocks, size_t smem, hipStream_t s, const ParamsND &p,
                    const void *src, const void *base, void *dst, const StepArg &sa, double *part, InstAcc *acc);

template <typename T>
static hipError_t step2d_c(int cx, int eq, int scheme, int n_blocks, hipStream_t s, const ParamsND &p,
                           const void *src, void *dst, const StepArg &sa, double *part, InstAcc *acc,
                           const SkRows *skr)
{
    switch (cx) {
    case 4: return step2d_e<T, 4>(eq, scheme, n_blocks, s, p, src, dst, sa, part, acc, skr);
    case 8: return step2d_e<T, 8>(eq, scheme, n_blocks, s, p, src, dst, sa, part, acc, skr);
    case 16: return step2d_e<T, 16>(eq, scheme, n_blocks, s, p, src, dst, sa, part, acc, skr);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step2d(int prec, int cx, int eq, int scheme, int n_blocks, hipStream_t s, const ParamsND &p,
                         const void *src, void *dst, const StepArg &sa, double *part, InstAcc *acc,
                         const SkRows *skr)
{
    if (prec == 0) return step2d_c<float>(cx, eq, scheme, n_blocks, s, p, src, dst, sa, part, acc, skr);
    return step2d_c<double>(cx, eq, scheme, n_blocks, s, p, src, dst, sa, part, acc, skr);
}

hipError_t launch_step3d(int prec, int cx, int eq, int stage, int ty, int n_blocks, size_t smem, hipStream_t s,
                         const ParamsND &p, const void *src, const void *base, void *dst, const StepArg &sa,
                         double *part, InstAcc *acc)
{
    if (prec == 0) {
        if (cx == 4) return step3d_e<float, 4>(eq, stage, ty, n_blocks, smem, s, p, src, base, dst, sa, part, acc);
        if (cx == 8) return step3d_e<float, 8>(eq, stage, ty, n_blocks, smem, s, p, src, base, dst, sa, part, acc);
        if (cx == 16) return step3d_e<float, 16>(eq, stage, ty, n_blocks, smem, s, p, src, base, dst, sa, part, acc);
    } else {
        if (cx == 4) return step3d_e<double, 4>(eq, stage, ty, n_blocks, smem, s, p, src, base, dst, sa, part, acc);
        if (cx == 8) return step3d_e<double, 8>(eq, stage, ty, n_blocks, smem, s, p, src, base, dst, sa, part, acc);
        if (cx == 16)
            return step3d_e<double, 16>(eq, stage, ty, n_blocks, smem, s, p, src, base, dst, sa, part, acc);
    }
    return hipErrorInvalidValue;
}

// Per-instance reduction of the sample partials, fixed order.
__global__ void __launch_bounds__(64)
    k_reduce_parts(StepArg sarg, SpatialParts sp)
{
    int64_t step;
    int sample;
    resolve_step(sarg, step, sample);
    if (!sample) return;
    reduce_spatial_wave(sp, blockIdx.x, threadIdx.x);
}

// ------------------------------------------------------------------ init / finalisation

template <typename T>
__global__ void __launch_bounds__(256)
    k_initnd(ParamsND p, int64_t cells, T *__restrict__ field)
{
    const int inst = blockIdx.y;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (c >= cells) return;
    const InstND ipar = p.ip[inst];
    double v = ipar.u0;
    if (ipar.init_sd > 0.0) {
        const Normals4<double> nz = block_normals<double>(static_cast<uint32_t>(c >> 2), 0u, ctr_word2(0, 1u),
                                                          ipar.realisation, make_key(p.seed));
        v += ipar.init_sd * nz.z[c & 3];
    }
    field[static_cast<int64_t>(inst) * cells + c] = static_cast<T>(v);
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_finnd(ParamsND p, int inst, int64_t cells, const T *__restrict__ field, const InstAcc *__restrict__ acc,
            const double *__restrict__ sk_sums, const double *__restrict__ sk_modes, int nbins,
            double *__restrict__ out)
{
    __shared__ double red[256];
    const T *f = field + static_cast<int64_t>(inst) * cells;
    double a = 0.0;
    for (int64_t c = threadIdx.x; c < cells; c += 256) a += static_cast<double>(f[c]);
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double u0 = p.ip[inst].u0;
    if (threadIdx.x == 0) {
        const InstAcc q = acc[inst];
        const double M = q.n_samples > 0 ? static_cast<double>(q.n_samples) : 1.0;
        out[0] = u0 + q.sp_mean / M;
        out[1] = q.sp_var / M;
        out[2] = red[0];
    }
    // shell averages; the k = 0 mode of U = u0 + dU is
    // sum_samples (N u0 + sum dU)^2 = M N^2 u0^2 + 2 N u0 (N sp_mean) + sum (sum dU)^2
    if (nbins > 0) {
        const InstAcc q = acc[inst];
        const double M = q.n_samples > 0 ? static_cast<double>(q.n_samples) : 1.0;
        const double N = static_cast<double>(cells);
        const double *ss = sk_sums + static_cast<int64_t>(inst) * nbins;
        for (int b = threadIdx.x; b < nbins; b += 256) {
            double v = ss[b];
            if (b == 0) v += M * N * N * u0 * u0 + 2.0 * N * u0 * (N * q.sp_mean);
            out[3 + b] = sk_modes[b] > 0 ? v / (M * sk_modes[b]) : 0.0;
        }
    }
}

// ------------------------------------------------------------------ launchers

hipError_t launch_reduce_parts(int n_inst, hipStream_t s, const StepArg &sa, const double *part, int32_t nparts,
                               double inv_cells, int32_t batch_len, InstAcc *acc)
{
    const SpatialParts sp{part, acc, inv_cells, nparts, batch_len};
    hipLaunchKernelGGL(k_reduce_parts, dim3(n_inst), dim3(64), 0, s, sa, sp);
    return hipGetLastError();
}

__global__ void k_set_step(int64_t *ctr, int64_t value)
{
    if (threadIdx.x == 0) *ctr = value;
}

__global__ void k_add_step(int64_t *ctr, int64_t k)
{
    if (threadIdx.x == 0) *ctr += k;
}

hipError_t launch_set_step(hipStream_t s, int64_t *ctr, int64_t value)
{
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, ctr, value);
    return hipGetLastError();
}

hipError_t launch_add_step(hipStream_t s, int64_t *ctr, int64_t k)
{
    hipLaunchKernelGGL(k_add_step, dim3(1), dim3(64), 0, s, ctr, k);
    return hipGetLastError();
}

hipError_t launch_initnd(int prec, hipStream_t s, const ParamsND &p, int64_t cells, void *field)
{
    const dim3 grid(static_cast<unsigned>((cells + 255) / 256), p.n_inst);
    if (prec == 0)
        hipLaunchKernelGGL(k_initnd<float>, grid, dim3(256), 0, s, p, cells, static_cast<float *>(field));
    else
        hipLaunchKernelGGL(k_initnd<double>, grid, dim3(256), 0, s, p, cells, static_cast<double *>(field));
    return hipGetLastError();
}

hipError_t launch_finnd(int prec, hipStream_t s, const ParamsND &p, int inst, int64_t cells, const void *field,
                        const InstAcc *acc, const double *sk_sums, const double *sk_modes, int nbins, double *out)
{
    if (prec == 0)
        hipLaunchKernelGGL(k_finnd<float>, dim3(1), dim3(256), 0, s, p, inst, cells,
                           static_cast<const float *>(field), acc, sk_sums, sk_modes, nbins, out);
    else
        hipLaunchKernelGGL(k_finnd<double>, dim3(1), dim3(256), 0, s, p, inst, cells,
                           static_cast<const double *>(field), acc, sk_sums, sk_modes, nbins, out);
    return hipGetLastError();
}

}  // namespace she
