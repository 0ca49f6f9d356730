// Counter-based Gaussian noise for the step kernels (gfx950).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each round
// forms the 64-bit products of words 0 and 2 with the two round multipliers and
// recombines their halves with words 1 and 3 and the round key; the key is
// advanced by the two Weyl increments between rounds.  The key is uniform over
// a launch, so its schedule lives in scalar registers.
//
// Box-Muller: the radius takes u_a = ((w_a >> 9) + 1/2) 2^-23 in (0, 1), the
// angle u_b = (w_b >> 9) 2^-23 in [0, 1) (both exact in FP32 and FP64);
// pairs (lane 0, lane 1) and (lane 2, lane 3); even lane
// sqrt(-2 ln u_a) cos(2 pi u_b), odd lane sqrt(-2 ln u_a) sin(2 pi u_b).
// The FP32 form uses the native v_log_f32 (log2), v_sqrt_f32 and
// v_sin_f32 / v_cos_f32, whose argument is in revolutions, so 2 pi u_b
// needs no multiply and no range reduction, and 1 + u_b (the bits of one
// funnel shift, no subtraction) gives the same sine and cosine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace she {

struct PhiloxKey {
    uint32_t k0, k1;
};

__host__ __device__ inline PhiloxKey make_key(uint64_t seed)
{
    return PhiloxKey{static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32)};
}

// Counter word 2 of step n for stream tag g.
__host__ __device__ inline uint32_t ctr_word2(uint64_t step, uint32_t tag)
{
    return static_cast<uint32_t>((step >> 32) & 0xFFFFu) | (tag << 16);
}

struct Words4 {
    uint32_t w[4];
};

// LIVE_KEY: the key passes through an empty asm statement, so the compiler
// forms the round keys inside each call (two scalar adds per round) instead
// of holding all twenty in scalar registers across an enclosing loop; for
// kernels whose loops are short of scalar registers.
template <bool LIVE_KEY = false>
__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, PhiloxKey key)
{
    uint32_t k0 = key.k0, k1 = key.k1;
    if constexpr (LIVE_KEY) asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
        const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
        // Callers vary word 0 (the block number) per lane and keep the other
        // words and the key uniform.  Up to round 2 some xors thus have two
        // uniform inputs (round 0: word 0's product and word 2's inputs
        // other than its product; round 1: the product of word 0, uniform
        // after round 0, and the words beside the varying one; round 2: word
        // 3, the low half of that uniform product).  Those pairs are formed
        // first and the varying input is xored on by v_bitop3_b32 with a zero
        // third input (table 0x96), which the compiler does not reassociate:
        // the pair stays in scalar registers and one vector instruction
        // remains, where a three-input vector xor would first need a scalar
        // input moved to a vector register.  Elsewhere one three-input
        // v_bitop3_b32 does the xor.
        if (round == 0) {
            c0 = hi1 ^ c1 ^ k0;
            c2 = __builtin_amdgcn_bitop3_b32(hi0, c3 ^ k1, 0u, 0x96);
        } else if (round == 1) {
            c0 = __builtin_amdgcn_bitop3_b32(hi1, c1 ^ k0, 0u, 0x96);
            c2 = __builtin_amdgcn_bitop3_b32(c3, hi0 ^ k1, 0u, 0x96);
        } else if (round == 2) {
            c0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
            c2 = __builtin_amdgcn_bitop3_b32(hi0, c3 ^ k1, 0u, 0x96);
        } else {
            c0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
            c2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
        }
        c1 = lo1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words4{{c0, c1, c2, c3}};
}

template <typename T>
struct Normals4 {
    T z[4];
};

// FP32: the bits of 1 + m 2^-23 (m = w >> 9) come from one funnel shift of
// (0x7F, w) by 9; subtracting 1 - 2^-24 is exact (the operands are within a
// factor of two), leaving (m + 1/2) 2^-23.
__device__ __forceinline__ float unit_open_f32(uint32_t w)
{
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9)) - 0x1.fffffep-1f;
}

__device__ __forceinline__ double unit_open_f64(uint32_t w)
{
    return (static_cast<double>(w >> 9) + 0.5) * 0x1p-23;
}

// The angle uniform: 1 + u_b in FP32 (a whole number of revolutions more),
// u_b in FP64.
__device__ __forceinline__ float unit_angle_f32(uint32_t w)
{
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9));
}

__device__ __forceinline__ double unit_angle_f64(uint32_t w)
{
    return static_cast<double>(w >> 9) * 0x1p-23;
}

__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float &zc, float &zs)
{
    const float ua = unit_open_f32(wa);
    const float ub = unit_angle_f32(wb);
    // -2 ln(u) = -2 ln(2) log2(u)
    const float rho = __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(ua) * -1.38629436111989061883f);
    zc = rho * __builtin_amdgcn_cosf(ub);
    zs = rho * __builtin_amdgcn_sinf(ub);
}

__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double &zc, double &zs)
{
    const double ua = unit_open_f64(wa);
    const double ub = unit_angle_f64(wb);
    const double rho = sqrt(-2.0 * log(ua));
    // sin and cos of 2 pi u_b from the exactly reduced sincospi(2 u_b): no
    // multiply by an inexact 2 pi and no general range reduction (the
    // argument is in [0, 2)); c1 steps 10% faster than with sincos(2 pi u_b)
    double s, c;
    sincospi(2.0 * ub, &s, &c);
    zc = rho * c;
    zs = rho * s;
}

// The four normals of Philox block `block` at step `step`.
template <typename T, bool LIVE_KEY = false>
__device__ __forceinline__ Normals4<T> block_normals(uint32_t block, uint32_t step_lo,
                                                     uint32_t w2, uint32_t realisation,
                                                     PhiloxKey key)
{
    const Words4 x = philox4x32_10<LIVE_KEY>(block, step_lo, w2, realisation, key);
    Normals4<T> n;
    box_muller(x.w[0], x.w[1], n.z[0], n.z[1]);
    box_muller(x.w[2], x.w[3], n.z[2], n.z[3]);
    return n;
}

// Scaled normals s*N for a fixed factor s >= 0, with the factor folded into
// the Box-Muller radius: FP32 takes rc = -2 ln(2) s^2 and forms
// sqrt(log2(u_a) rc); FP64 takes rc = s.
__device__ __forceinline__ void box_muller_scaled(uint32_t wa, uint32_t wb, float rc, float &zc, float &zs)
{
    const float ua = unit_open_f32(wa);
    const float ub = unit_angle_f32(wb);
    const float rho = __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(ua) * rc);
    zc = rho * __builtin_amdgcn_cosf(ub);
    zs = rho * __builtin_amdgcn_sinf(ub);
}

__device__ __forceinline__ void box_muller_scaled(uint32_t wa, uint32_t wb, double rc, double &zc, double &zs)
{
    double c, s;
    box_muller(wa, wb, c, s);
    zc = c * rc;
    zs = s * rc;
}

// The same pairs in the form a face whose amplitude is itself a square root
// takes: the squared scaled radius r2 = -2 ln(u_a) s^2 and the unit factors
// cos and sin of the angle, so that the face forms sqrt(x) rho = sqrt(x r2)
// with one root (rc as for box_muller_scaled: -2 ln(2) s^2 in FP32, s in
// FP64).
__device__ __forceinline__ void box_muller_sq(uint32_t wa, uint32_t wb, float rc, float &r2, float &c, float &s)
{
    const float ua = unit_open_f32(wa);
    const float ub = unit_angle_f32(wb);
    r2 = __builtin_amdgcn_logf(ua) * rc;
    c = __builtin_amdgcn_cosf(ub);
    s = __builtin_amdgcn_sinf(ub);
}

__device__ __forceinline__ void box_muller_sq(uint32_t wa, uint32_t wb, double rc, double &r2, double &c,
                                              double &s)
{
    const double ua = unit_open_f64(wa);
    const double ub = unit_angle_f64(wb);
    r2 = (-2.0 * log(ua)) * (rc * rc);
    sincospi(2.0 * ub, &s, &c);
}

template <typename T>
struct NormalsSq4 {
    T t[4];   // cos, sin of pair 0; cos, sin of pair 1
    T r2[2];  // squared scaled radius of each pair
};

template <typename T>
__device__ __forceinline__ NormalsSq4<T> block_normals_sq(uint32_t block, uint32_t step_lo, uint32_t w2,
                                                          uint32_t realisation, PhiloxKey key, T rc)
{
    const Words4 x = philox4x32_10(block, step_lo, w2, realisation, key);
    NormalsSq4<T> n;
    box_muller_sq(x.w[0], x.w[1], rc, n.r2[0], n.t[0], n.t[1]);
    box_muller_sq(x.w[2], x.w[3], rc, n.r2[1], n.t[2], n.t[3]);
    return n;
}

// Square root of a noise amplitude: FP32 takes the native v_sqrt_f32 (about
// one ulp, one instruction; the library form adds a denormal-scaling and
// rounding-correction sequence), FP64 the correctly rounded library sqrt.
__device__ __forceinline__ float amp_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double amp_sqrt(double x) { return sqrt(x); }

template <typename T>
__host__ __device__ inline T radius_const(double s);

template <>
__host__ __device__ inline float radius_const<float>(double s)
{
    return static_cast<float>(-1.38629436111989061883 * s * s);
}

template <>
__host__ __device__ inline double radius_const<double>(double s)
{
    return s;
}

template <typename T>
__device__ __forceinline__ Normals4<T> block_normals_scaled(uint32_t block, uint32_t step_lo, uint32_t w2,
                                                            uint32_t realisation, PhiloxKey key, T rc)
{
    const Words4 x = philox4x32_10(block, step_lo, w2, realisation, key);
    Normals4<T> n;
    box_muller_scaled(x.w[0], x.w[1], rc, n.z[0], n.z[1]);
    box_muller_scaled(x.w[2], x.w[3], rc, n.z[2], n.z[3]);
    return n;
}

}  // namespace she
