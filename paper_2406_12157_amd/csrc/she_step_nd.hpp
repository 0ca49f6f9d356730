#pragma once

// Step kernels of the 2D / 3D periodic grids and their typed launchers.
// Included by the translation units that instantiate them (one per state
// type and cells per lane, so the kernels compile in parallel).
//
// Scheme (Garcia et al., Sec. 3, applied per direction with independent face
// numbers, Sec. 2 eq. GWN): the low face of cell c in direction e carries
// F = r (U_c - U_{c-e}) + sigma A N, A = (U_{c-e} + U_c)/2 (SHE) or
// sqrt(max(., 0)) of it (Dean-Kawasaki, Sec. 4); U_c += sum_e F(c+e) - F(c).
// PC (2D): U* = FE step, U = (U + U* + Delta(U*; same N)) / 2.
//
// The constant factors of the noise term are folded into the Box-Muller
// radius: the kernels draw z = s N with s = sigma/2 (SHE: A z = (U_l + U_r) z),
// s = sigma/sqrt(2) (DK: sqrt(U_l + U_r) z) or s = sigma A(u0) (deterministic
// face value: the noise term is z), so a face costs sub, add, mul, fma.
//
// Layout: realisation-major, x fastest, FP32 or FP64.  Face numbers
// ((z*Ny + y)*dim + e)*Nx + x make the four faces of one Philox block four
// consecutive x-cells of one direction, so a lane that owns CX consecutive
// cells of a row needs CX/4 Philox calls per direction and uses every number.
//
// 2D: a "row group" of LX = Nx/CX lanes owns a full x-row and marches along y
// over a chunk of rows.  The x-neighbours come from the adjacent lanes
// (ds_bpermute shuffles inside the group, periodic wrap within the group);
// the y-neighbours stay in registers from the previous row, and the row two
// ahead is prefetched, so each cell is read once and written once per step;
// only the first row of a chunk (FE) or its first three rows (PC) are
// computed twice.
//
// 3D: a workgroup of TY row groups owns TY consecutive rows in y and marches
// along z.  Low y-face fluxes are exchanged between the rows through LDS (one
// barrier per plane, double-buffered); the tile's top row computes the flux
// through its high y-face itself (one extra Philox call per plane for that
// row).  z-neighbours stay in registers; the plane two ahead is prefetched.
// PC runs as two passes of the same kernel: the predictor U* = U + Delta(U)
// into a scratch field, then the corrector (U + U* + Delta(U*)) / 2, whose
// numbers are drawn again from the same counters.
//
// Sample steps: every lane adds dU = U - u0 and dU^2 of its output cells in
// FP64; the group / workgroup sum is written to a per-chunk partial; a small
// kernel reduces the partials per instance in a fixed order.
//
// Structure factor rows (SK, sample launches of the two-step FE march with
// one row per wave, nx = 512 or 1024): the wave keeps each even output row
// and, once the odd row after it is out, transforms the pair along x as one
// complex row (dU_even + i dU_odd) with the wave FFT of she_fft.hpp (the
// lane's CX consecutive cells are first transposed through the wave's LDS
// region into the transform's input order) and stores both half spectra,
// kx = 0..nx/2, as two rows of the column-tiled half spectrum.  This is the row
// stage of the S(k) transform of the field the launch writes, done while the
// rows are still in registers instead of reading the field back.  A two-step
// launch whose first step samples (kernel variant SCHEME 3) takes the
// statistics and transforms of its intermediate rows instead, as the march
// forms them: that field never reaches memory.
#include <type_traits>

#include "she_fft.hpp"
#include "she_internal.hpp"
#include "she_rng.hpp"

namespace she {

// max(x, 0) for a face density.  FP32 compares the bits as signed integers
// (every negative float, -0 included, is a negative integer), one integer
// max with no NaN canonicalisation; a NaN density stays NaN either way
// through the difference term of the flux.
__device__ __forceinline__ float clamp_nonneg(float x)
{
    return __int_as_float(max(__float_as_int(x), 0));
}

__device__ __forceinline__ double clamp_nonneg(double x)
{
    return fmax(x, 0.0);
}

// The numbers of one face.  Most forms carry the scaled normal zs.  The
// Dean-Kawasaki face with instantaneous noise (SQ) carries instead the unit
// factor t (cosine or sine of its Box-Muller angle) and the squared scaled
// radius r2 of its pair: its amplitude sqrt(max(s, 0)) rho is then formed as
// sqrt(max(s, 0) r2), one root per face and none for the radius.
template <typename T, bool SQ>
struct FaceNoise {
    T zs;
};

template <typename T>
struct FaceNoise<T, true> {
    T t, r2;
};

// Flux through a face between cells with values lo (low side) and hi, for
// its numbers z (see above), in noise mode NZ (0 instantaneous,
// 1 deterministic face value, 2 off); neg tells whether the Dean-Kawasaki
// face density was negative and clamped to zero.
template <typename T, int EQ, int NZ, bool SQ>
__device__ __forceinline__ T face_flux(T lo, T hi, FaceNoise<T, SQ> z, bool &neg)
{
    // The face flux divided by r: the difference hi - lo plus the noise term,
    // whose scale carries 1/r (the caller multiplies the divergence by r once
    // per cell, which saves a multiply per face).  The multiply-add is written
    // out so that every copy of this code rounds alike: a face computed in two
    // places gets one value.
    const T d = hi - lo;
    neg = false;
    if constexpr (NZ == 0) {
        const T s = lo + hi;
        if constexpr (EQ == 0) {
            return fma(s, z.zs, d);
        } else {
            // the root of max(s, 0): the compare only counts the clamp
            neg = s < T(0);
            if constexpr (SQ)
                return fma(amp_sqrt(clamp_nonneg(s) * z.r2), z.t, d);
            else
                return fma(amp_sqrt(clamp_nonneg(s)), z.zs, d);
        }
    } else if constexpr (NZ == 1) {
        return d + z.zs;
    } else {
        return d;
    }
}

template <typename T, int EQ, int NZ, bool SQ>
__device__ __forceinline__ T face_flux(T lo, T hi, FaceNoise<T, SQ> z, uint32_t &clamps)
{
    bool neg;
    const T f = face_flux<T, EQ, NZ>(lo, hi, z, neg);
    clamps += neg ? 1u : 0u;
    return f;
}

// Number of lanes of the wave for which b holds (wave-uniform).  Called in
// control flow that all lanes of the wave take, it lets a count of rare
// events live in one scalar register: no per-lane select and add.
__device__ __forceinline__ uint32_t wave_count(bool b)
{
    return static_cast<uint32_t>(__builtin_popcountll(__builtin_amdgcn_ballot_w64(b)));
}

// Box-Muller radius constant of the normals a face flux takes: the noise
// scale ns of the instance over r (the fluxes are carried divided by r; r = 0
// has no noise).
template <typename T>
__device__ __forceinline__ T flux_radius(const InstND &ip)
{
    return radius_const<T>(ip.r > 0.0 ? ip.ns / ip.r : 0.0);
}

__device__ __forceinline__ int wrap(int i, int n)
{
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

template <typename T, int CX>
__device__ __forceinline__ void load_row(const T *__restrict__ p, T (&v)[CX])
{
#pragma unroll
    for (int j = 0; j < CX; ++j) v[j] = p[j];
}

template <typename T, int CX>
__device__ __forceinline__ void store_row(T *__restrict__ p, const T (&v)[CX])
{
#pragma unroll
    for (int j = 0; j < CX; ++j) p[j] = v[j];
}

template <typename T, int CX>
__device__ __forceinline__ void copy_row(T (&d)[CX], const T (&s)[CX])
{
#pragma unroll
    for (int j = 0; j < CX; ++j) d[j] = s[j];
}

// Numbers of one lane's CX faces of direction-row `drow` (= row*dim + e).
template <typename T, int CX, int NZ, bool SQ>
__device__ __forceinline__ void row_normals(FaceNoise<T, SQ> (&z)[CX], uint32_t drow, uint32_t nq, uint32_t q0,
                                            uint32_t slo, uint32_t w2, uint32_t real, PhiloxKey key, T rc)
{
    if constexpr (NZ == 2) {
        static_assert(!SQ, "no numbers in noise mode 2");
#pragma unroll
        for (int j = 0; j < CX; ++j) z[j].zs = T(0);
        return;
    }
#pragma unroll
    for (int c = 0; c < CX / 4; ++c) {
        if constexpr (SQ) {
            const NormalsSq4<T> nz = block_normals_sq<T>(drow * nq + q0 + c, slo, w2, real, key, rc);
#pragma unroll
            for (int l = 0; l < 4; ++l) z[4 * c + l] = FaceNoise<T, true>{nz.t[l], nz.r2[l >> 1]};
        } else {
            const Normals4<T> nz = block_normals_scaled<T>(drow * nq + q0 + c, slo, w2, real, key, rc);
#pragma unroll
            for (int l = 0; l < 4; ++l) z[4 * c + l].zs = nz.z[l];
        }
    }
}

// x-fluxes of one row held by a group of LX lanes: Flo[j] is the flux through
// the low face of the lane's cell j, Fhi the flux through the high face of its
// last cell (= the next lane's Flo[0]).  count(neg) is called once per face.
template <typename T, int CX, int EQ, int NZ, bool SQ, typename Count>
__device__ __forceinline__ void row_xflux(const T (&v)[CX], const FaceNoise<T, SQ> (&z)[CX], T (&Flo)[CX], T &Fhi,
                                          int lx, int LX, Count &&count)
{
    const int lane = threadIdx.x & 63;
    const int gbase = lane - lx;
    const int left = gbase + (lx == 0 ? LX - 1 : lx - 1);
    const int right = gbase + (lx == LX - 1 ? 0 : lx + 1);
    const T vleft = __shfl(v[CX - 1], left, 64);
    bool neg;
    Flo[0] = face_flux<T, EQ, NZ>(vleft, v[0], z[0], neg);
    count(neg);
#pragma unroll
    for (int j = 1; j < CX; ++j) {
        Flo[j] = face_flux<T, EQ, NZ>(v[j - 1], v[j], z[j], neg);
        count(neg);
    }
    Fhi = __shfl(Flo[0], right, 64);
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// On request (SHE_TUNE_XCD_ORDER) they are renumbered so that XCD x runs a
// contiguous range of logical blocks: neighbouring march chunks, which read
// each other's halo rows, then share an L2.  A bijection on the first
// 8*floor(n/8) blocks; the rest keep their index.  On MI355X this measured no
// faster than the plain order, which is the default.
__device__ __forceinline__ int xcd_block(int b, int n)
{
    constexpr int kXcd = 8;
    const int per = n / kXcd;
    if (b >= per * kXcd) return b;
    return (b % kXcd) * per + b / kXcd;
}

template <typename T, int CX>
__device__ __forceinline__ T xdiv(const T (&Flo)[CX], T Fhi, int j)
{
    return (j + 1 < CX ? Flo[j + 1] : Fhi) - Flo[j];
}

template <typename T, int CX>
__device__ __forceinline__ void accumulate(const T (&out)[CX], double u0, double &sa, double &sb)
{
#pragma unroll
    for (int j = 0; j < CX; ++j) {
        const double dl = static_cast<double>(out[j]) - u0;
        sa += dl;
        sb += dl * dl;
    }
}

// ------------------------------------------------------------------ 2D

// RW: one row per wave (Nx = 64 CX, i.e. every grid from Nx = 256 on).  The
// wave's chunk, instance and rows are then wave-uniform: instance parameters,
// row offsets and counter words live in scalar registers.
template <typename T, int CX, int EQ, int SCHEME, bool SK, bool RW>
__global__ void __launch_bounds__(256)
    k_step2d(ParamsND p, const T *__restrict__ src, T *__restrict__ dst, StepArg sarg, double *__restrict__ part,
             InstAcc *__restrict__ acc, SkRows skr)
{
    int64_t step;
    int sample;
    resolve_step(sarg, step, sample);
    // SK: pass twiddles of the row transform in LDS, then one transform
    // region per wave (= per row group)
    constexpr int LGX = CX == 16 ? 10 : 9;
    using FX = WaveFft<LGX>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *twl = reinterpret_cast<cplx<T> *>(smem_raw);
    if constexpr (SK) {
        fill_pass_twiddles<T, LGX>(twl, static_cast<const cplx<T> *>(skr.tw));
        __syncthreads();
    }
    const int LX = RW ? 64 : p.nx / CX;
    const int lx = RW ? static_cast<int>(threadIdx.x & 63) : static_cast<int>(threadIdx.x) % LX;
    const int grp = RW ? __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6))
                       : static_cast<int>(threadIdx.x) / LX;
    const int gpb = RW ? static_cast<int>(blockDim.x >> 6) : static_cast<int>(blockDim.x) / LX;
    const int nchunks = (p.ny + p.chunk - 1) / p.chunk;
    const int gchunk = (p.xcd_order ? xcd_block(blockIdx.x, gridDim.x) : static_cast<int>(blockIdx.x)) * gpb + grp;
    if (gchunk >= p.n_inst * nchunks) return;
    const int inst = gchunk / nchunks, ch = gchunk - inst * nchunks;
    const int y0 = ch * p.chunk, y1 = min(y0 + p.chunk, p.ny);
    const int64_t plane = static_cast<int64_t>(p.nx) * p.ny;
    const T *S = src + inst * plane + CX * lx;
    T *D = dst + inst * plane + CX * lx;

    if (acc[inst].nonfinite) {  // frozen: carry the state over unchanged
        for (int y = y0; y < y1; ++y) {
            T v[CX];
            load_row<T, CX>(S + static_cast<int64_t>(y) * p.nx, v);
            store_row<T, CX>(D + static_cast<int64_t>(y) * p.nx, v);
        }
        return;
    }

    const InstND ipar = p.ip[inst];
    const T r = static_cast<T>(ipar.r);
    const T rc = flux_radius<T>(ipar);
    uint32_t clamps = 0;
    const int noise = p.noise;
    const uint32_t real = ipar.realisation;
    const PhiloxKey key = make_key(p.seed);
    const uint32_t slo = static_cast<uint32_t>(step), w2 = ctr_word2(static_cast<uint64_t>(step), 0u);
    // counter words of the following step (the second stage of a two-step march)
    const uint32_t slo1 = static_cast<uint32_t>(step + 1), w21 = ctr_word2(static_cast<uint64_t>(step + 1), 0u);
    const uint32_t nq = static_cast<uint32_t>(p.nx / 4), q0 = static_cast<uint32_t>((CX / 4) * lx);
    const int ny = p.ny;
    auto rowp = [&](int y) { return S + static_cast<int64_t>(wrap(y, ny)) * p.nx; };
    auto drow = [&](int y, int e) { return static_cast<uint32_t>(wrap(y, ny) * 2 + e); };

    double sa = 0.0, sb = 0.0;
    const double u0d = ipar.u0;

    // The march loops are unrolled over the period of their register window
    // (FE: three rows and two flux rows, period 6; PC: four rows and pairs,
    // period 4); each unrolled copy names the buffers in rotated roles, so rows
    // move through the window without register copies.
    auto march = [&](auto nzc) __attribute__((always_inline)) {
        constexpr int NZ = decltype(nzc)::value;
        // Dean-Kawasaki faces with instantaneous noise take their amplitude
        // with one root (FaceNoise)
        constexpr bool SQ = EQ == 1 && NZ == 0;
        using Z = FaceNoise<T, SQ>;
        auto normals = [&](Z (&z)[CX], uint32_t dr) __attribute__((always_inline)) {
            row_normals<T, CX, NZ, SQ>(z, dr, nq, q0, slo, w2, real, key, rc);
        };
        // Density clamps are counted once per face and stage, by the chunk that
        // owns the face (the low faces of its rows); faces a chunk recomputes
        // for its halo (own = false) are not counted.
        auto flux = [&](T lo, T hi, Z z, bool own = true) __attribute__((always_inline)) {
            uint32_t c = 0;
            const T f = face_flux<T, EQ, NZ>(lo, hi, z, c);
            clamps += own ? c : 0u;
            return f;
        };
        auto xflux = [&](const T (&v)[CX], const Z (&z)[CX], T (&fx)[CX], T &fxh,
                         bool own = true) __attribute__((always_inline)) {
            uint32_t c = 0;
            row_xflux<T, CX, EQ, NZ, SQ>(v, z, fx, fxh, lx, LX, [&](bool neg) { c += neg ? 1u : 0u; });
            clamps += own ? c : 0u;
        };
        // The sampling of a finished row of the sampled field: its spatial
        // moments and, on sample launches with S(k), its transform along x.
        auto take = [&](const T (&out)[CX], int y) __attribute__((always_inline)) {
            if (sample) accumulate<T, CX>(out, u0d, sa, sb);
            if constexpr (SK) {
                // the pair's complex row: the even row's dU goes to the real
                // parts of the wave's region at once (the transpose), the odd
                // row's to the imaginary parts
                const T su0 = static_cast<T>(u0d);
                constexpr int n = FX::n, LR = PassRadix<LGX>::LR, R = 1 << LR;
                cplx<T> *wreg = twl + FX::tw + grp * FX::lds;
                if ((y & 1) == 0) {
#pragma unroll
                    for (int j = 0; j < CX; ++j) wreg[pidx(CX * lx + j)].re = out[j] - su0;
                } else {
#pragma unroll
                    for (int j = 0; j < CX; ++j) wreg[pidx(CX * lx + j)].im = out[j] - su0;
                    wave_sync();
                    cplx<T> v[FX::P];
#pragma unroll
                    for (int i = 0; i < FX::P / R; ++i) {
#pragma unroll
                        for (int k = 0; k < R; ++k) {
                            int seq, x;
                            pass_input<LGX, LR>(lx, i, k, seq, x);
                            v[i * R + k] = wreg[pidx(x)];
                        }
                    }
                    wave_sync();
                    wave_fft<T, LGX, LGX>(v, wreg, twl, lx);
                    // 32-bit offsets from the instance's base: entry (y - 1, k)
                    // of the column-tiled layout, and row y at +TC in the same tile
                    cplx<T> *hb = static_cast<cplx<T> *>(skr.half) + half_index(inst, 0, 0, p.ny, skr.ltc, skr.nkb);
                    const uint32_t ltc = static_cast<uint32_t>(skr.ltc), tcm = (1u << ltc) - 1u;
                    const uint32_t yoff = static_cast<uint32_t>(y - 1) << ltc;
                    const uint32_t uny = static_cast<uint32_t>(p.ny);
                    if (ltc <= 6) {
                        // tiles of at most 64 columns: lane l's columns l + 64 i lie
                        // 64/TC tiles apart, i.e. 64 ny entries, from its first one
                        const uint32_t ul = static_cast<uint32_t>(lx);
                        cplx<T> *hl = hb + ((((ul >> ltc) * uny) << ltc) + yoff + (ul & tcm));
                        const size_t s64 = static_cast<size_t>(uny) << 6;
#pragma unroll
                        for (int i = 0; i <= n / 128; ++i) {
                            if (i == n / 128 && lx != 0) break;  // kx = n/2: lane 0 only
                            const int k = lx + 64 * i;
                            const cplx<T> z = wreg[pidx(k)], zm = wreg[pidx((n - k) & (n - 1))];
                            hl[i * s64] = unpack2_a(z, zm);
                            hl[i * s64 + tcm + 1u] = unpack2_b(z, zm);
                        }
                    } else {
                        for (int k = lx; k <= n / 2; k += 64) {
                            const cplx<T> z = wreg[pidx(k)], zm = wreg[pidx((n - k) & (n - 1))];
                            const uint32_t uk = static_cast<uint32_t>(k);
                            const uint32_t e = (((uk >> ltc) * uny) << ltc) + yoff + (uk & tcm);
                            hb[e] = unpack2_a(z, zm);
                            hb[e + tcm + 1u] = unpack2_b(z, zm);
                        }
                    }
                    wave_sync();  // the next pair's transpose overwrites the region
                }
            }
        };
        auto emit = [&](const T (&out)[CX], int y) __attribute__((always_inline)) {
            store_row<T, CX>(D + static_cast<int64_t>(y) * p.nx, out);
            take(out, y);
        };
        const int rows = y1 - y0;
        if constexpr (SCHEME == 0) {
            T ra[CX], rb[CX], rq[CX], fa[CX], fb[CX];
            // rows of the window: ra, rb, rq; flux rows: fa, fb
            auto by6 = [&](auto &&row) __attribute__((always_inline)) {
                for (int i = 0; i < rows; i += 6) {
                    row(ra, rb, rq, fa, fb, i);
                    if (i + 1 >= rows) break;
                    row(rb, rq, ra, fb, fa, i + 1);
                    if (i + 2 >= rows) break;
                    row(rq, ra, rb, fa, fb, i + 2);
                    if (i + 3 >= rows) break;
                    row(ra, rb, rq, fb, fa, i + 3);
                    if (i + 4 >= rows) break;
                    row(rb, rq, ra, fa, fb, i + 4);
                    if (i + 5 >= rows) break;
                    row(rq, ra, rb, fb, fa, i + 5);
                }
            };
            if ((ch & 1) == 0) {
                // upward march: the low-y flux of row y is carried from row y-1
                {
                    T tp[CX];
                    Z z[CX];
                    load_row<T, CX>(rowp(y0 - 1), tp);
                    load_row<T, CX>(rowp(y0), ra);
                    load_row<T, CX>(rowp(y0 + 1), rb);
                    normals(z, drow(y0, 1));
#pragma unroll
                    for (int j = 0; j < CX; ++j) fa[j] = flux(tp[j], ra[j], z[j]);
                }
                // tc, tn: rows y, y+1; tq receives row y+2; flo: low-y flux of row y
                by6([&](const T (&tc)[CX], const T (&tn)[CX], T (&tq)[CX], const T (&flo)[CX], T (&fhi)[CX],
                        int i) __attribute__((always_inline)) {
                    const int y = y0 + i;
                    if (y + 2 <= y1) load_row<T, CX>(rowp(y + 2), tq);
                    Z z[CX];
                    T fx[CX], fxh, out[CX];
                    normals(z, drow(y + 1, 1));
#pragma unroll
                    for (int j = 0; j < CX; ++j) fhi[j] = flux(tc[j], tn[j], z[j], y + 1 < y1);
                    normals(z, drow(y, 0));
                    xflux(tc, z, fx, fxh);
#pragma unroll
                    for (int j = 0; j < CX; ++j) out[j] = fma(r, xdiv<T, CX>(fx, fxh, j) + (fhi[j] - flo[j]), tc[j]);
                    emit(out, y);
                });
            } else {
                // downward march (odd chunks): each chunk boundary is then read by
                // both neighbours at the same end of their marches, so the second
                // read of its rows can hit the cache.  The high-y flux of row y is
                // carried from row y+1; every face gets the same value either way.
                {
                    T tu[CX];
                    Z z[CX];
                    load_row<T, CX>(rowp(y1), tu);
                    load_row<T, CX>(rowp(y1 - 1), ra);
                    load_row<T, CX>(rowp(y1 - 2), rb);
                    normals(z, drow(y1, 1));
#pragma unroll
                    for (int j = 0; j < CX; ++j) fa[j] = flux(ra[j], tu[j], z[j], false);
                }
                // tc, tn: rows y, y-1; tq receives row y-2; fhi: high-y flux of row y
                by6([&](const T (&tc)[CX], const T (&tn)[CX], T (&tq)[CX], const T (&fhi)[CX], T (&flo)[CX],
                        int i) __attribute__((always_inline)) {
                    const int y = y1 - 1 - i;
                    if (y - 2 >= y0 - 1) load_row<T, CX>(rowp(y - 2), tq);
                    Z z[CX];
                    T fx[CX], fxh, out[CX];
                    normals(z, drow(y, 1));
#pragma unroll
                    for (int j = 0; j < CX; ++j) flo[j] = flux(tn[j], tc[j], z[j]);
                    normals(z, drow(y, 0));
                    xflux(tc, z, fx, fxh);
#pragma unroll
                    for (int j = 0; j < CX; ++j) out[j] = fma(r, xdiv<T, CX>(fx, fxh, j) + (fhi[j] - flo[j]), tc[j]);
                    emit(out, y);
                });
            }
        } else if constexpr (SCHEME == 2 || SCHEME == 3) {
            // Two FE steps in one pass (steps n and n+1 of the counter): the
            // intermediate field U1 lives only in registers.  Iteration k forms
            // row k of U1 = FE(U0) and row k-1 of U2 = FE(U1), with the same
            // face and update expressions as the one-step march, so U2 is the
            // field two single steps give, bit for bit.  tc, tn: U0 rows k,
            // k+1, tq receiving row k+2; sc, sn: U1 rows k-1, k; fpc, fpn: the
            // step-n low-y fluxes of rows k, k+1; fcm, fcc: the step-(n+1)
            // low-y fluxes of U1 rows k-1, k.  Each chunk recomputes the U1
            // rows on both sides of it.  SCHEME 3, a launch whose first step
            // samples, takes the chunk's own U1 rows as they are formed and
            // only stores U2 (a variant of its own: one sampling site per
            // kernel keeps the row transforms' registers out of the other).
            constexpr bool first = SCHEME == 3;
            auto normals1 = [&](Z (&z)[CX], uint32_t dr) __attribute__((always_inline)) {
                row_normals<T, CX, NZ, SQ>(z, dr, nq, q0, slo1, w21, real, key, rc);
            };
            T ta[CX], tb[CX], tcc[CX], sa_[CX], sb_[CX], pa[CX], pb[CX], ma[CX], mb[CX];
            const int k0 = y0 - 1;
            {
                T tp[CX];
                Z z[CX];
                load_row<T, CX>(rowp(k0 - 1), tp);
                load_row<T, CX>(rowp(k0), ta);
                load_row<T, CX>(rowp(k0 + 1), tb);
                normals(z, drow(k0, 1));
#pragma unroll
                for (int j = 0; j < CX; ++j) pa[j] = flux(tp[j], ta[j], z[j], false);
            }
            auto row = [&](const T (&tc)[CX], const T (&tn)[CX], T (&tq)[CX], const T (&sc)[CX], T (&sn)[CX],
                           const T (&fpc)[CX], T (&fpn)[CX], const T (&fcm)[CX], T (&fcc)[CX],
                           int i) __attribute__((always_inline)) {
                const int k = k0 + i;
                load_row<T, CX>(rowp(k + 2), tq);
                Z z[CX];
                T fx[CX], fxh;
                normals(z, drow(k + 1, 1));
#pragma unroll
                for (int j = 0; j < CX; ++j) fpn[j] = flux(tc[j], tn[j], z[j], k + 1 < y1);
                normals(z, drow(k, 0));
                xflux(tc, z, fx, fxh, k >= y0 && k < y1);
#pragma unroll
                for (int j = 0; j < CX; ++j) sn[j] = fma(r, xdiv<T, CX>(fx, fxh, j) + (fpn[j] - fpc[j]), tc[j]);
                if constexpr (first) {
                    if (k >= y0 && k < y1) take(sn, k);
                }
                if (i >= 1) {
                    normals1(z, drow(k, 1));
#pragma unroll
                    for (int j = 0; j < CX; ++j) fcc[j] = flux(sc[j], sn[j], z[j], k < y1);
                }
                if (i >= 2) {
                    normals1(z, drow(k - 1, 0));
                    xflux(sc, z, fx, fxh);
                    T out[CX];
#pragma unroll
                    for (int j = 0; j < CX; ++j) out[j] = fma(r, xdiv<T, CX>(fx, fxh, j) + (fcc[j] - fcm[j]), sc[j]);
                    if constexpr (first)
                        store_row<T, CX>(D + static_cast<int64_t>(k - 1) * p.nx, out);
                    else
                        emit(out, k - 1);
                }
            };
            const int iters = rows + 2;  // k = y0-1 .. y1
            for (int i = 0; i < iters; i += 6) {
                row(ta, tb, tcc, sa_, sb_, pa, pb, ma, mb, i);
                if (i + 1 >= iters) break;
                row(tb, tcc, ta, sb_, sa_, pb, pa, mb, ma, i + 1);
                if (i + 2 >= iters) break;
                row(tcc, ta, tb, sa_, sb_, pa, pb, ma, mb, i + 2);
                if (i + 3 >= iters) break;
                row(ta, tb, tcc, sb_, sa_, pb, pa, mb, ma, i + 3);
                if (i + 4 >= iters) break;
                row(tb, tcc, ta, sa_, sb_, pa, pb, ma, mb, i + 4);
                if (i + 5 >= iters) break;
                row(tcc, ta, tb, sb_, sa_, pb, pa, mb, ma, i + 5);
            }
        } else {
            // Predictor-corrector.  Iteration k produces the predictor row k and
            // the corrected row k-1.  Per iteration: tm, tc, tn rows k-1..k+1 and
            // tq receiving row k+2; sc the predictor row k-1, sn receiving row k;
            // zyc, zyn the y numbers of rows k, k+1; zxm, zxc the x numbers of
            // rows k-1, k; fpc, fpn the predictor low-y fluxes of rows k, k+1;
            // fcm, fcc the corrector low-y fluxes of rows k-1, k.
            T ta[CX], tb[CX], tcc[CX], td[CX], sa_[CX], sb_[CX], pa[CX], pb[CX], ma[CX], mb[CX];
            Z ya[CX], yb[CX], xa[CX], xb[CX];
            const int k0 = y0 - 1;
            load_row<T, CX>(rowp(k0 - 1), ta);
            load_row<T, CX>(rowp(k0), tb);
            load_row<T, CX>(rowp(k0 + 1), tcc);
            normals(ya, drow(k0, 1));
#pragma unroll
            for (int j = 0; j < CX; ++j) pa[j] = flux(ta[j], tb[j], ya[j], false);
            auto row = [&](const T (&tm)[CX], const T (&tc)[CX], const T (&tn)[CX], T (&tq)[CX], const T (&sc)[CX],
                           T (&sn)[CX], const Z (&zyc)[CX], Z (&zyn)[CX], const Z (&zxm)[CX], Z (&zxc)[CX],
                           const T (&fpc)[CX], T (&fpn)[CX], const T (&fcm)[CX], T (&fcc)[CX],
                           int i) __attribute__((always_inline)) {
                const int k = k0 + i;
                load_row<T, CX>(rowp(k + 2), tq);
                normals(zyn, drow(k + 1, 1));
#pragma unroll
                for (int j = 0; j < CX; ++j) fpn[j] = flux(tc[j], tn[j], zyn[j], k + 1 >= y0 && k + 1 < y1);
                normals(zxc, drow(k, 0));
                T fx[CX], fxh;
                xflux(tc, zxc, fx, fxh, k >= y0 && k < y1);
#pragma unroll
                for (int j = 0; j < CX; ++j) sn[j] = fma(r, xdiv<T, CX>(fx, fxh, j) + (fpn[j] - fpc[j]), tc[j]);
                if (i >= 1) {
#pragma unroll
                    for (int j = 0; j < CX; ++j) fcc[j] = flux(sc[j], sn[j], zyc[j], k < y1);
                }
                if (i >= 2) {
                    // corrected row k-1 from predictor rows k-2 (fcm), k-1 (sc), k (sn)
                    xflux(sc, zxm, fx, fxh);
                    T out[CX];
#pragma unroll
                    for (int j = 0; j < CX; ++j)
                        out[j] = T(0.5) * fma(r, xdiv<T, CX>(fx, fxh, j) + (fcc[j] - fcm[j]), tm[j] + sc[j]);
                    emit(out, k - 1);
                }
            };
            const int iters = rows + 2;  // k = y0-1 .. y1
            for (int i = 0; i < iters; i += 4) {
                row(ta, tb, tcc, td, sa_, sb_, ya, yb, xa, xb, pa, pb, ma, mb, i);
                if (i + 1 >= iters) break;
                row(tb, tcc, td, ta, sb_, sa_, yb, ya, xb, xa, pb, pa, mb, ma, i + 1);
                if (i + 2 >= iters) break;
                row(tcc, td, ta, tb, sa_, sb_, ya, yb, xa, xb, pa, pb, ma, mb, i + 2);
                if (i + 3 >= iters) break;
                row(td, ta, tb, tcc, sb_, sa_, yb, ya, xb, xa, pb, pa, mb, ma, i + 3);
            }
        }
    };
    if (noise == 0) march(std::integral_constant<int, 0>{});
    else if (noise == 1) march(std::integral_constant<int, 1>{});
    else march(std::integral_constant<int, 2>{});
    if (sample) {
        for (int off = 1; off < LX; off <<= 1) {
            sa += __shfl_xor(sa, off, 64);
            sb += __shfl_xor(sb, off, 64);
        }
        if (lx == 0) {
            part[2 * static_cast<int64_t>(gchunk)] = sa;
            part[2 * static_cast<int64_t>(gchunk) + 1] = sb;
        }
    }
    if (clamps) atomicAdd(reinterpret_cast<unsigned long long *>(&acc[inst].clamp_count),
                          static_cast<unsigned long long>(clamps));
}

// ------------------------------------------------------------------ 3D (FE; PC in two passes)

// STAGE 0: FE step (or a PC predictor) dst = src + Delta(src);
// STAGE 1: PC corrector dst = (base + src + Delta(src)) / 2, with src the
// predictor and base the state it was taken from (same step, same numbers).
// RW: one row per wave (Nx = 64 CX).  The row, its plane offsets and its
// counter words are then the same for the whole wave and live in scalar
// registers; otherwise several rows share a wave.
template <typename T, int CX, int EQ, int STAGE, bool RW>
__global__ void __launch_bounds__(256)
    k_step3d(ParamsND p, int32_t ty, const T *__restrict__ src, const T *__restrict__ base, T *__restrict__ dst,
             StepArg sarg, double *__restrict__ part, InstAcc *__restrict__ acc)
{
    int64_t step;
    int sample;
    resolve_step(sarg, step, sample);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int LX = RW ? 64 : p.nx / CX;
    const int lx = RW ? static_cast<int>(threadIdx.x & 63) : static_cast<int>(threadIdx.x) % LX;
    // row within the tile
    const int g = RW ? __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6)) : static_cast<int>(threadIdx.x) / LX;
    const int nyt = p.ny / ty, nzc = (p.nz + p.chunk - 1) / p.chunk;
    const int tiles = nyt * nzc;
    const int lblock = p.xcd_order ? xcd_block(blockIdx.x, gridDim.x) : static_cast<int>(blockIdx.x);
    const int inst = lblock / tiles;
    const int tile = lblock - inst * tiles;
    const int yt = tile % nyt, zc = tile / nyt;
    const int y = yt * ty + g;
    const int z0 = zc * p.chunk, z1 = min(z0 + p.chunk, p.nz);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int64_t vol = static_cast<int64_t>(nx) * ny * nz;
    const T *S = src + inst * vol + CX * lx;
    const T *B = STAGE == 1 ? base + inst * vol + CX * lx : nullptr;
    T *D = dst + inst * vol + CX * lx;
    auto rowp = [&](int yy, int zz) {
        return static_cast<int64_t>(wrap(zz, nz) * ny + wrap(yy, ny)) * nx;
    };

    if (acc[inst].nonfinite) {  // frozen: carry the state over unchanged
        const T *F = STAGE == 1 ? B : S;
        for (int zz = z0; zz < z1; ++zz) {
            T v[CX];
            load_row<T, CX>(F + rowp(y, zz), v);
            store_row<T, CX>(D + rowp(y, zz), v);
        }
        return;
    }

    // LDS: T rows of the current plane and low-y fluxes, both double-buffered
    T *tsh = reinterpret_cast<T *>(smem_raw);            // [2][ty][nx]
    T *fsh = tsh + 2 * ty * nx;                           // [2][ty][nx]
    const int cell0 = CX * lx;

    const InstND ipar = p.ip[inst];
    const T r = static_cast<T>(ipar.r);
    const T rc = flux_radius<T>(ipar);
    // density clamps of the wave: every count is taken in control flow that
    // the whole wave follows, so the total is wave-uniform (lane 0 reports it)
    uint32_t clamps = 0;
    const int noise = p.noise;
    const uint32_t real = ipar.realisation;
    const PhiloxKey key = make_key(p.seed);
    const uint32_t slo = static_cast<uint32_t>(step), w2 = ctr_word2(static_cast<uint64_t>(step), 0u);
    const uint32_t nq = static_cast<uint32_t>(nx / 4), q0 = static_cast<uint32_t>((CX / 4) * lx);
    auto drow = [&](int yy, int zz, int e) {
        return static_cast<uint32_t>((wrap(zz, nz) * ny + wrap(yy, ny)) * 3 + e);
    };

    double sa = 0.0, sb = 0.0;
    const double u0d = ipar.u0;

    // As in 2D, the march is unrolled over the period of its register window
    // (three planes of the row and two z-flux rows: period 6) and the noise
    // mode is fixed per copy.
    auto march = [&](auto nzc) __attribute__((always_inline)) {
        constexpr int NZ = decltype(nzc)::value;
        // Dean-Kawasaki faces with instantaneous noise take their amplitude
        // with one root (FaceNoise)
        constexpr bool SQ = EQ == 1 && NZ == 0;
        using Z = FaceNoise<T, SQ>;
        auto normals = [&](Z (&z)[CX], uint32_t dr) __attribute__((always_inline)) {
            row_normals<T, CX, NZ, SQ>(z, dr, nq, q0, slo, w2, real, key, rc);
        };
        // Each face's clamp is counted once: x- and low y-faces by the row
        // they belong to, z-faces by the chunk below them (its planes' high
        // z-faces, the last one included; so not the low z-faces of a chunk's
        // first plane), and not the high y-faces a tile's top row recomputes
        // (own = false, in a branch only that row takes).
        auto flux = [&](T lo, T hi, Z z, bool own = true) __attribute__((always_inline)) {
            bool neg;
            const T f = face_flux<T, EQ, NZ>(lo, hi, z, neg);
            if constexpr (EQ == 1 && NZ == 0) {
                if (own) clamps += wave_count(neg);
            }
            return f;
        };
        auto count = [&](bool neg) __attribute__((always_inline)) {
            if constexpr (EQ == 1 && NZ == 0) clamps += wave_count(neg);
        };
        T ra[CX], rb[CX], rq[CX], fa[CX], fb[CX];
        {
            T tp[CX];
            Z z[CX];
            load_row<T, CX>(S + rowp(y, z0 - 1), tp);
            load_row<T, CX>(S + rowp(y, z0), ra);
            load_row<T, CX>(S + rowp(y, z0 + 1), rb);
            normals(z, drow(y, z0, 2));
#pragma unroll
            for (int j = 0; j < CX; ++j) fa[j] = flux(tp[j], ra[j], z[j], false);
            T *dstp = tsh + ((z0 & 1) * ty + g) * nx + cell0;
#pragma unroll
            for (int j = 0; j < CX; ++j) dstp[j] = ra[j];
        }
        __syncthreads();
        // tc, tn: planes zi, zi+1 of the row; tq receives plane zi+2; fzlo: the
        // low-z flux of plane zi
        auto plane = [&](const T (&tc)[CX], const T (&tn)[CX], T (&tq)[CX], const T (&fzlo)[CX], T (&fzhi)[CX],
                         int zi) __attribute__((always_inline)) {
            const int buf = zi & 1;
            load_row<T, CX>(S + rowp(y, zi + 2), tq);
            Z z[CX];
            normals(z, drow(y, zi + 1, 2));
#pragma unroll
            for (int j = 0; j < CX; ++j) fzhi[j] = flux(tc[j], tn[j], z[j]);

            T fxlo[CX], fxhi;
            normals(z, drow(y, zi, 0));
            row_xflux<T, CX, EQ, NZ, SQ>(tc, z, fxlo, fxhi, lx, LX, count);

            T ylo[CX], fylo[CX];
            normals(z, drow(y, zi, 1));
            if (g > 0) {
                const T *q = tsh + (buf * ty + g - 1) * nx + cell0;
#pragma unroll
                for (int j = 0; j < CX; ++j) ylo[j] = q[j];
            } else {
                load_row<T, CX>(S + rowp(y - 1, zi), ylo);
            }
#pragma unroll
            for (int j = 0; j < CX; ++j) fylo[j] = flux(ylo[j], tc[j], z[j]);
            {
                T *fp = fsh + (buf * ty + g) * nx + cell0;
#pragma unroll
                for (int j = 0; j < CX; ++j) fp[j] = fylo[j];
                T *tp = tsh + (((zi + 1) & 1) * ty + g) * nx + cell0;
#pragma unroll
                for (int j = 0; j < CX; ++j) tp[j] = tn[j];
            }
            __syncthreads();
            T fyhi[CX];
            if (g + 1 < ty) {
                const T *fp = fsh + (buf * ty + g + 1) * nx + cell0;
#pragma unroll
                for (int j = 0; j < CX; ++j) fyhi[j] = fp[j];
            } else {
                T yhi[CX];
                load_row<T, CX>(S + rowp(y + 1, zi), yhi);
                normals(z, drow(y + 1, zi, 1));
#pragma unroll
                for (int j = 0; j < CX; ++j) fyhi[j] = flux(tc[j], yhi[j], z[j], false);
            }
            T out[CX];
            if constexpr (STAGE == 0) {
#pragma unroll
                for (int j = 0; j < CX; ++j)
                    out[j] = fma(r, (xdiv<T, CX>(fxlo, fxhi, j) + (fyhi[j] - fylo[j])) + (fzhi[j] - fzlo[j]), tc[j]);
            } else {
                T ub[CX];
                load_row<T, CX>(B + rowp(y, zi), ub);
#pragma unroll
                for (int j = 0; j < CX; ++j)
                    out[j] = T(0.5) * fma(r, (xdiv<T, CX>(fxlo, fxhi, j) + (fyhi[j] - fylo[j])) + (fzhi[j] - fzlo[j]),
                                          ub[j] + tc[j]);
            }
            if (sample) accumulate<T, CX>(out, u0d, sa, sb);
            store_row<T, CX>(D + rowp(y, zi), out);
        };
        const int planes = z1 - z0;
        for (int i = 0; i < planes; i += 6) {
            plane(ra, rb, rq, fa, fb, z0 + i);
            if (i + 1 >= planes) break;
            plane(rb, rq, ra, fb, fa, z0 + i + 1);
            if (i + 2 >= planes) break;
            plane(rq, ra, rb, fa, fb, z0 + i + 2);
            if (i + 3 >= planes) break;
            plane(ra, rb, rq, fb, fa, z0 + i + 3);
            if (i + 4 >= planes) break;
            plane(rb, rq, ra, fa, fb, z0 + i + 4);
            if (i + 5 >= planes) break;
            plane(rq, ra, rb, fb, fa, z0 + i + 5);
        }
    };
    if (noise == 0) march(std::integral_constant<int, 0>{});
    else if (noise == 1) march(std::integral_constant<int, 1>{});
    else march(std::integral_constant<int, 2>{});
    if (sample) {
        for (int off = 1; off < LX; off <<= 1) {
            sa += __shfl_xor(sa, off, 64);
            sb += __shfl_xor(sb, off, 64);
        }
        __syncthreads();
        double *red = reinterpret_cast<double *>(smem_raw);
        if (lx == 0) {
            red[2 * g] = sa;
            red[2 * g + 1] = sb;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double ta = 0.0, tb = 0.0;
            for (int w = 0; w < ty; ++w) {
                ta += red[2 * w];
                tb += red[2 * w + 1];
            }
            part[2 * static_cast<int64_t>(lblock)] = ta;
            part[2 * static_cast<int64_t>(lblock) + 1] = tb;
        }
    }
    if (clamps && (threadIdx.x & 63) == 0)
        atomicAdd(reinterpret_cast<unsigned long long *>(&acc[inst].clamp_count),
                  static_cast<unsigned long long>(clamps));
}

// ------------------------------------------------------------------ typed launchers

// The two-step launch that samples its first step (SCHEME 3) is compiled for
// FP32 only; the planner does not ask for it in FP64.
template <typename T>
constexpr bool kFirstStepVariant = std::is_same<T, float>::value;

template <typename T, int CX, int EQ>
static hipError_t step2d_s(int scheme, int n_blocks, hipStream_t s, const ParamsND &p, const void *src, void *dst,
                           const StepArg &sa, double *part, InstAcc *acc, const SkRows *skr)
{
    const SkRows none{nullptr, nullptr, 0, 0};
    const T *in = static_cast<const T *>(src);
    T *out = static_cast<T *>(dst);
    // one row per wave from Nx = 64 CX on; the planner takes CX = 8 and 16
    // only there, so those have no other form
    const bool rw = p.nx == 64 * CX;
    if (!rw) {
        if constexpr (CX == 4) {
            if (scheme == 0)
                hipLaunchKernelGGL((k_step2d<T, CX, EQ, 0, false, false>), dim3(n_blocks), dim3(256), 0, s, p, in,
                                   out, sa, part, acc, none);
            else if (scheme == 1)
                hipLaunchKernelGGL((k_step2d<T, CX, EQ, 1, false, false>), dim3(n_blocks), dim3(256), 0, s, p, in,
                                   out, sa, part, acc, none);
            else if (!skr && sa.sample == 2) {
                if constexpr (kFirstStepVariant<T>)
                    hipLaunchKernelGGL((k_step2d<T, CX, EQ, 3, false, false>), dim3(n_blocks), dim3(256), 0, s, p,
                                       in, out, sa, part, acc, none);
                else
                    return hipErrorInvalidValue;
            }
            else if (!skr)
                hipLaunchKernelGGL((k_step2d<T, CX, EQ, 2, false, false>), dim3(n_blocks), dim3(256), 0, s, p, in,
                                   out, sa, part, acc, none);
            else
                return hipErrorInvalidValue;
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (scheme == 0)
        hipLaunchKernelGGL((k_step2d<T, CX, EQ, 0, false, true>), dim3(n_blocks), dim3(256), 0, s, p, in, out, sa,
                           part, acc, none);
    else if (scheme == 1)
        hipLaunchKernelGGL((k_step2d<T, CX, EQ, 1, false, true>), dim3(n_blocks), dim3(256), 0, s, p, in, out, sa,
                           part, acc, none);
    else if (!skr && sa.sample == 2) {
        if constexpr (kFirstStepVariant<T>)
            hipLaunchKernelGGL((k_step2d<T, CX, EQ, 3, false, true>), dim3(n_blocks), dim3(256), 0, s, p, in, out,
                               sa, part, acc, none);
        else
            return hipErrorInvalidValue;
    }
    else if (!skr)
        hipLaunchKernelGGL((k_step2d<T, CX, EQ, 2, false, true>), dim3(n_blocks), dim3(256), 0, s, p, in, out, sa,
                           part, acc, none);
    else {
        if constexpr (CX == 8 || CX == 16) {
            using FX = WaveFft<CX == 16 ? 10 : 9>;
            const size_t smem = sizeof(cplx<T>) * (FX::tw + 4 * static_cast<size_t>(FX::lds));
            if (smem > 64 * 1024) return hipErrorInvalidValue;
            if (sa.sample == 2) {
                if constexpr (kFirstStepVariant<T>)
                    hipLaunchKernelGGL((k_step2d<T, CX, EQ, 3, true, true>), dim3(n_blocks), dim3(256), smem, s, p,
                                       in, out, sa, part, acc, *skr);
                else
                    return hipErrorInvalidValue;
            } else
                hipLaunchKernelGGL((k_step2d<T, CX, EQ, 2, true, true>), dim3(n_blocks), dim3(256), smem, s, p, in,
                                   out, sa, part, acc, *skr);
        } else {
            return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

template <typename T, int CX>
hipError_t step2d_e(int eq, int scheme, int n_blocks, hipStream_t s, const ParamsND &p, const void *src,
                           void *dst, const StepArg &sa, double *part, InstAcc *acc, const SkRows *skr)
{
    if (eq == 0) return step2d_s<T, CX, 0>(scheme, n_blocks, s, p, src, dst, sa, part, acc, skr);
    return step2d_s<T, CX, 1>(scheme, n_blocks, s, p, src, dst, sa, part, acc, skr);
}

template <typename T, int CX, int EQ>
static hipError_t step3d_s(int stage, int ty, int n_blocks, size_t smem, hipStream_t s, const ParamsND &p,
                           const void *src, const void *base, void *dst, const StepArg &sa, double *part,
                           InstAcc *acc)
{
    const dim3 block((p.nx / CX) * ty);
    const T *in = static_cast<const T *>(src), *bs = static_cast<const T *>(base);
    T *out = static_cast<T *>(dst);
    // as in 2D: CX = 8 and 16 only with one row per wave
    const bool rw = p.nx == 64 * CX;
    if (!rw) {
        if constexpr (CX == 4) {
            if (stage == 0)
                hipLaunchKernelGGL((k_step3d<T, CX, EQ, 0, false>), dim3(n_blocks), block, smem, s, p, ty, in, bs,
                                   out, sa, part, acc);
            else
                hipLaunchKernelGGL((k_step3d<T, CX, EQ, 1, false>), dim3(n_blocks), block, smem, s, p, ty, in, bs,
                                   out, sa, part, acc);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (stage == 0)
        hipLaunchKernelGGL((k_step3d<T, CX, EQ, 0, true>), dim3(n_blocks), block, smem, s, p, ty, in, bs, out, sa,
                           part, acc);
    else
        hipLaunchKernelGGL((k_step3d<T, CX, EQ, 1, true>), dim3(n_blocks), block, smem, s, p, ty, in, bs, out, sa,
                           part, acc);
    return hipGetLastError();
}

template <typename T, int CX>
hipError_t step3d_e(int eq, int stage, int ty, int n_blocks, size_t smem, hipStream_t s, const ParamsND &p,
                           const void *src, const void *base, void *dst, const StepArg &sa, double *part,
                           InstAcc *acc)
{
    if (eq == 0) return step3d_s<T, CX, 0>(stage, ty, n_blocks, smem, s, p, src, base, dst, sa, part, acc);
    return step3d_s<T, CX, 1>(stage, ty, n_blocks, smem, s, p, src, base, dst, sa, part, acc);
}

}  // namespace she
