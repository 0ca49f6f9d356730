// 1D step kernel: one workgroup owns one instance of a (possibly ragged) batch
// and keeps its whole state in LDS for a chunk of steps.
//
// Scheme (Garcia et al., Sec. 3): face flux F_f = r (U_f - U_{f-1}) + w sigma A N_f
// through the low face f of cell f, update U_i += F_{i+1} - F_i (FE), or the
// predictor-corrector U = (U + U* + Delta(U*; same N)) / 2 (PC).  Dirichlet
// walls: F_0 = 2 r (U_0 - U_L) + sqrt(2) sigma A(U_L) N_0 and mirrored at the
// right wall (ghost stencil U_1 - 3U_0 + 2U_L of the Dirichlet paragraph).
//
// Implicit schemes (backward Euler theta = 1, Crank-Nicolson theta = 1/2;
// the implicit-scheme exercise, Sec. 6): the flux pass weights the
// state-dependent deterministic flux by 1 - theta, giving the right-hand side
// U + W [(1 - theta) A U + b + noise]; M = I - theta W A is constant, so the
// host precomputes in FP64 the factors of parallel cyclic reduction (log2 N
// levels of d_i -= k1 d_(i-s) + k2 d_(i+s), then d_i / b_i) and, for periodic
// rods, the Sherman-Morrison vector of the cyclic part.  The reduction runs in
// FP64 for either state type (an FP64 array over the flux and scratch LDS),
// so only the final state is rounded: rounded factors would bias the
// conserved sum a little every step.
//
// Material varying along the rod (composite-rod exercise, Sec. 6; VARC): the
// conservative form with a conductance r_f and noise factor s_f per face and
// a factor w_i = (rho c_V)_ref / (rho c_V)_i per cell, U_i += w_i (F_(i+1) -
// F_i), staged in LDS next to the state.  Uniform instances of such a batch
// get uniform arrays (bit-identical to the uniform kernel).
//
// Work split: an instance is served by a run of whole waves of a workgroup
// (small instances share a workgroup, each with its own waves and LDS
// region); its thread t owns Philox blocks g = t, t + TS, ... (TS threads);
// block g holds faces 4g..4g+3, which are the low faces of cells 4g..4g+3,
// so one Philox call and two Box-Muller pairs serve four cells and PC re-uses
// the numbers from registers.  The state stays in registers for the whole
// launch; one LDS exchange and one barrier per FE step, two per PC step.
//
// Statistics on sample steps: per-cell FP64 sums of dU and dU^2 kept in
// registers for the whole launch, spatial sums reduced over the workgroup,
// and (optionally) the shifted state written as one row of a 256-row X block;
// a full block is contracted on the matrix cores, C += X^T X, with
// v_mfma_f32_16x16x4f32 (FP32 state) or v_mfma_f64_16x16x4f64 (FP64 state),
// and added to the FP64 N x N sum.  For the time correlation each sample row
// also goes to a per-instance history ring; after the launch, k_tcorr adds the
// lag products of the new rows (one thread per cell and lag, FP64).
#include <type_traits>

#include "she_internal.hpp"
#include "she_rng.hpp"
#include "she_wave.hpp"

namespace she {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Noise amplitude of a face with value v: v (SHE), sqrt(v) (DK),
// sqrt(v (1 - v)) (Burgers); a negative radicand is clamped and counted.
template <typename T>
__device__ __forceinline__ T face_amp(int eq, T v, uint32_t &clamps)
{
    if (eq == 0) return v;
    const T q = eq == 2 ? v * (T(1) - v) : v;
    if (q < T(0)) {
        ++clamps;
        return T(0);
    }
    return amp_sqrt(q);
}

// Value of the last of the first `m` (1..4) entries, chosen among values
// (a select of array elements as lvalues would become an address select and
// move the array to private memory).
template <typename T>
__device__ __forceinline__ T last_of(int m, T a0, T a1, T a2, T a3)
{
    return m >= 4 ? a3 : (m == 3 ? a2 : (m == 2 ? a1 : a0));
}

__device__ __forceinline__ f32x4 mfma16x16x4(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f64x4 mfma16x16x4(double a, double b, f64x4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// C[N x N] += X^T X for a full block X[256 x N] (row = snapshot).  Tiles of
// 16 x 16 over the upper triangle are spread over the instance's waves
// (wave = 0 .. nwave-1); each lane accumulates four outputs of its tile over
// K = 256 in the matrix-core accumulator type and adds them to the FP64 sum
// (both triangles).
// Operand layout of the 16x16x4 instructions: lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; output element v of lane l is D[4(l/16)+v][l%16] for
// the FP32 form and D[(l/16)+4v][l%16] for the FP64 form.
template <typename T>
__device__ void xtx_block(const T *__restrict__ X, double *__restrict__ Cm, int N, int wave, int nwave)
{
    using acc_t = typename std::conditional<std::is_same<T, float>::value, f32x4, f64x4>::type;
    const int lane = threadIdx.x & 63;
    const int nt = (N + 15) >> 4;
    const int ntiles = nt * (nt + 1) / 2;
    for (int t = wave; t < ntiles; t += nwave) {
        int ti = 0, rem = t;
        while (rem >= nt - ti) {
            rem -= nt - ti;
            ++ti;
        }
        const int tj = ti + rem;
        const int i = 16 * ti + (lane & 15), j = 16 * tj + (lane & 15);
        acc_t acc = {0, 0, 0, 0};
        // eight K-steps of operands are loaded before their eight products, so
        // the loads overlap instead of each product waiting for its own
        constexpr int kB = 8;
        for (int k0 = 0; k0 < kCorrBlock; k0 += 4 * kB) {
            T a[kB], b[kB];
#pragma unroll
            for (int q = 0; q < kB; ++q) {
                const int k = k0 + 4 * q + (lane >> 4);
                a[q] = i < N ? X[(int64_t)k * N + i] : T(0);
                b[q] = j < N ? X[(int64_t)k * N + j] : T(0);
            }
#pragma unroll
            for (int q = 0; q < kB; ++q) acc = mfma16x16x4(a[q], b[q], acc);
        }
        const int col = 16 * tj + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            // output rows: FP32 form 4(l/16)+v, FP64 form (l/16)+4v (measured on gfx950)
            const int row = 16 * ti + (std::is_same<T, float>::value ? 4 * (lane >> 4) + v : (lane >> 4) + 4 * v);
            if (row < N && col < N) {
                const double val = static_cast<double>(acc[v]);
                Cm[(int64_t)row * N + col] += val;
                if (ti != tj) Cm[(int64_t)col * N + row] += val;
            }
        }
    }
}

// MODE 0: uniform explicit batch; 3: the same with every instance a heat
// equation with instantaneous noise (only that face path is compiled: fewer
// registers and a shorter loop); 1: material coefficients (VARC); 2: some
// instance is implicit (material arrays available as well).  Each mode is
// compiled separately so that a batch pays only for the paths it uses.
//
// Thread t of an instance's waves owns Philox blocks g = t + s TS (s < MAXG,
// TS the instance's thread count): the faces 4g..4g+3 and the cells 4g..4g+3,
// whose values stay in registers.  A stage (the FE step, or either half of a
// PC step) publishes each block's first and last cell value (and, once per
// step, the number of its face 4g) in LDS, passes one barrier, reads the
// values next to its block and computes five fluxes: its own four faces and
// the face after its last cell, which the next block computes as its face 0
// as well (same inputs, same code, so the two agree bit for bit and the sum
// is conserved).  The exchange arrays alternate between two buffers, so one
// barrier per stage suffices.
template <typename T, int BLOCK, int MAXG, bool STATS, int MODE>
__device__ __forceinline__ void step1d_body(const Inst1D *__restrict__ tab, const Seg1D *__restrict__ segs,
                                            T *__restrict__ pool, const T *__restrict__ coef,
                                            const double *__restrict__ pcr, int64_t step0, int32_t nsteps,
                                            int64_t burn_in, int32_t every, uint32_t mask, Stats1D st)
{
    constexpr bool VARC = MODE == 1 || MODE == 2;
    constexpr bool HEAT_ONLY = MODE == 3;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const Seg1D seg = segs[static_cast<int64_t>(blockIdx.x) * (BLOCK / 64) + wave];
    if (seg.inst < 0) return;  // idle wave (barriers count the waves still running)
    const int inst = seg.inst;
    const Inst1D d = tab[inst];
    InstAcc *acc = st.acc + inst;
    if (acc->nonfinite) return;  // frozen after a non-finite sample

    const int N = d.n;
    const bool dir = d.bc == 1;
    const int nf = dir ? N + 1 : N;
    const int nfg = (nf + 3) >> 2, nfgp = (nfg + 3) & ~3;
    const int glast = (N - 1) >> 2;  // block of the last cell
    const int TS = 64 * seg.nw;
    const int t = static_cast<int>(threadIdx.x) - 64 * seg.w0;
    const int lw = wave - seg.w0;
    const SegLds lay = seg_lds(N, nf, static_cast<int32_t>(sizeof(T)), MODE);
    unsigned char *base = smem_raw + seg.lds;
    T *xch = reinterpret_cast<T *>(base + lay.xch);
    double *red = reinterpret_cast<double *>(base + lay.red);  // [3][16] wave sums of a sample
    T *Rf = reinterpret_cast<T *>(base + lay.rf);  // VARC: conductance per face (periodic: [N] = [0])
    T *Sf = reinterpret_cast<T *>(base + lay.sf);  // VARC: noise factor per face (walls: sqrt 2 included)
    T *Wc = reinterpret_cast<T *>(base + lay.wc);  // VARC: capacity factor per cell
    double *PD = reinterpret_cast<double *>(base + lay.pd);  // implicit: FP64 reduction array

    const T r = static_cast<T>(d.r);
    const T sg = static_cast<T>(d.sigma);
    const T sgw = static_cast<T>(d.sigma * 1.41421356237309504880);
    const T uL = static_cast<T>(d.uL), uR = static_cast<T>(d.uR), u0 = static_cast<T>(d.u0);
    const int eq = d.eq, noise = d.noise;
    const T nu = static_cast<T>(eq == 2 ? d.nu : 0.0);  // Burgers hyperbolic flux nu c_f (1 - c_f)
    const PhiloxKey key = make_key(d.seed);
    T *gU = pool + d.off;

    T u[MAXG][4];
#pragma unroll
    for (int s = 0; s < MAXG; ++s)
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int i = 4 * (t + s * TS) + l;
            u[s][l] = i < N ? gU[i] : T(0);
        }
    if constexpr (VARC) {
        if (d.k_off >= 0) {
            const T *k = coef + d.k_off;
            for (int f = t; f < nf; f += TS) {
                Rf[f] = k[f];
                Sf[f] = k[nf + f];
            }
            for (int i = t; i < N; i += TS) Wc[i] = k[2 * nf + i];
            if (!dir && t == 0) {
                Rf[N] = k[0];
                Sf[N] = k[nf];
            }
        } else {
            for (int f = t; f < nf; f += TS) {
                Rf[f] = r;
                Sf[f] = (dir && (f == 0 || f == N)) ? sgw : sg;
            }
            for (int i = t; i < N; i += TS) Wc[i] = T(1);
            if (!dir && t == 0) {
                Rf[N] = r;
                Sf[N] = sg;
            }
        }
    }

    // wall amplitudes (deterministic)
    uint32_t clamps = 0;
    const T amp_uL = face_amp<T>(eq, uL, clamps);
    const T amp_uR = face_amp<T>(eq, uR, clamps);
    clamps = 0;

    // Per-cell sums of dU and dU^2: in registers for the launch with one
    // Philox block per thread; with more, updated in memory on each sample
    // (registers for the stage matter more there: they set how many
    // workgroups of a packed batch are resident at once).
    constexpr bool kRegSums = MAXG == 1;
    double s1[MAXG][4], s2[MAXG][4];
    const bool moments = STATS && (mask & 1u) && st.s1 != nullptr;
    const bool corr = STATS && (mask & 2u) && d.x_off >= 0;
    const bool tcorr = STATS && (mask & 16u) && d.h_off >= 0;
    int64_t nsamp = STATS ? acc->n_samples : 0;
    // spatial sums of the instance, carried in registers over the launch
    double sp_mean = STATS ? acc->sp_mean : 0.0, sp_sq = STATS ? acc->sp_sq : 0.0,
           sp_var = STATS ? acc->sp_var : 0.0;
    // first sample of the launch: the smallest t > burn_in, t > step0 with
    // t % every == 0 (t = steps completed); later ones follow every `every`
    int64_t t_next = -1;
    if (STATS && every > 0) {
        const int64_t a0 = (step0 > burn_in ? step0 : burn_in) + 1;
        const int64_t rm = a0 % every;
        t_next = rm == 0 ? a0 : a0 + (every - rm);
    }
    // reference profile of the deviations: u0, or the linear wall profile
    const double ref0 = dir ? d.uL : d.u0, ref_slope = dir ? (d.uR - d.uL) / N : 0.0;
#pragma unroll
    for (int s = 0; s < MAXG; ++s)
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int i = 4 * (t + s * TS) + l;
            s1[s][l] = (kRegSums && moments && i < N) ? st.s1[d.off + i] : 0.0;
            s2[s][l] = (kRegSums && moments && i < N) ? st.s2[d.off + i] : 0.0;
        }
    __syncthreads();

    // implicit schemes: weight of the state-dependent deterministic flux
    const bool impl = MODE == 2 && d.scheme >= 2;
    const T ex = static_cast<T>(impl ? 1.0 - d.theta : 1.0);
    const T rex = r * ex;
    // face kinds: 0 heat with instantaneous noise; 1 deterministic or no
    // noise (any equation); 2 Dean-Kawasaki; 3 Burgers (both instantaneous)
    const int kind = noise != 0 ? 1 : (eq == 0 ? 0 : eq + 1);

    int ph = 0;  // exchange buffer of the next stage
    // Flux divergence dv of the state V (registers) for every owned cell.
    // first: the stage that also exchanges the face-0 numbers (rnz: the
    // number of the face after each block, kept for the second PC stage).
    auto stage = [&](const T (&V)[MAXG][4], const T (&z)[MAXG][4], T (&rnz)[MAXG], T (&dv)[MAXG][4],
                     bool first) __attribute__((always_inline)) {
        T *Uf = xch + (3 * ph) * nfgp, *Ul = Uf + nfgp, *Zf = Ul + nfgp;
        ph ^= 1;
#pragma unroll
        for (int s = 0; s < MAXG; ++s) {
            const int g = t + s * TS;
            if (g < nfg) {
                const int nc = N - 4 * g;
                Uf[g] = V[s][0];
                Ul[g] = last_of<T>(nc, V[s][0], V[s][1], V[s][2], V[s][3]);
                if (first) Zf[g] = z[s][0];
            }
        }
        __syncthreads();
        auto faces = [&](auto kc) __attribute__((always_inline)) {
            constexpr int K = decltype(kc)::value;
#pragma unroll
            for (int s = 0; s < MAXG; ++s) {
                const int g = t + s * TS;
                const int nc = N - 4 * g;  // cells from this block's first on
                if (nc <= 0) continue;     // no cells (a Dirichlet block holding only face N)
                const bool inner = nc > 4;
                const T lnb = Ul[g == 0 ? glast : g - 1];
                const T left = (dir && g == 0) ? uL : lnb;
                const T rnb = Uf[inner ? g + 1 : 0];
                const T right = (dir && !inner) ? uR : rnb;
                if (first) {
                    const T zn = Zf[inner || (dir && nc == 4) ? g + 1 : 0];
                    // Dirichlet, N not a multiple of 4: face N is this block's own
                    rnz[s] = (dir && nc < 4) ? last_of<T>(nc + 1, z[s][0], z[s][1], z[s][2], z[s][3]) : zn;
                }
                T lo[5], hi[5], zz[5];
                lo[0] = left;
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    lo[l + 1] = V[s][l];
                    hi[l] = V[s][l];
                    zz[l] = z[s][l];
                }
                hi[4] = right;
                zz[4] = rnz[s];
                if (nc < 4) {  // the block of the last cell when 4 does not divide N
#pragma unroll
                    for (int l = 1; l < 4; ++l)
                        if (l >= nc) {
                            hi[l] = right;
                            zz[l] = rnz[s];
                        }
                }
                T F[5];
#pragma unroll
                for (int l = 0; l < 5; ++l) {
                    const int f = 4 * g + l;
                    const T rf = VARC ? Rf[f] * ex : rex;
                    const T sf = VARC ? Sf[f] : sg;
                    const T df = hi[l] - lo[l];
                    const T cf = T(0.5) * (lo[l] + hi[l]);
                    // clamps are counted on the faces this block owns
                    const bool own = l < 4 && l < nc && !(dir && f == 0);
                    if constexpr (K == 0) {
                        F[l] = fma(sf * cf, zz[l], rf * df);
                    } else if constexpr (K == 1) {
                        T am = T(0);
                        if (noise == 1) {
                            const T v = dir ? uL + (uR - uL) * static_cast<T>(f) / static_cast<T>(N) : u0;
                            uint32_t c = 0;
                            am = face_amp<T>(eq, v, c);
                            if (own) clamps += c;
                        }
                        F[l] = fma(sf * am, zz[l], fma(-nu * cf, T(1) - cf, rf * df));
                    } else if constexpr (K == 2) {
                        const bool neg = cf < T(0);
                        if (own && neg) ++clamps;
                        const T am = neg ? T(0) : amp_sqrt(cf);
                        F[l] = fma(sf * am, zz[l], rf * df);
                    } else {
                        const T q = cf * (T(1) - cf);
                        const bool neg = q < T(0);
                        if (own && neg) ++clamps;
                        const T am = neg ? T(0) : amp_sqrt(q);
                        F[l] = fma(sf * am, zz[l], fma(-nu, q, rf * df));
                    }
                }
                if (dir) {
                    // walls: F_0 = 2 r (U_0 - U_L) + sqrt 2 sigma A(U_L) N_0, mirrored at
                    // face N (the state term weighted by 1 - theta in implicit schemes)
                    if (g == 0) {
                        const T rw = VARC ? Rf[0] : r;
                        const T sw = VARC ? Sf[0] : sgw;
                        const T dwl = fma(-nu * uL, T(1) - uL, T(2) * rw * (ex * V[s][0] - uL));
                        F[0] = noise != 2 ? fma(sw * amp_uL, zz[0], dwl) : dwl;
                    }
                    if (!inner) {
                        const int m = nc < 4 ? nc : 4;
                        const T vl = last_of<T>(m, V[s][0], V[s][1], V[s][2], V[s][3]);
                        const T rw = VARC ? Rf[N] : r;
                        const T sw = VARC ? Sf[N] : sgw;
                        const T dwr = fma(-nu * uR, T(1) - uR, T(2) * rw * (uR - ex * vl));
                        const T w = noise != 2 ? fma(sw * amp_uR, rnz[s], dwr) : dwr;
#pragma unroll
                        for (int l = 1; l < 5; ++l)
                            if (l == m) F[l] = w;
                    }
                }
#pragma unroll
                for (int l = 0; l < 4; ++l) dv[s][l] = VARC ? Wc[4 * g + l] * (F[l + 1] - F[l]) : F[l + 1] - F[l];
            }
        };
        if constexpr (HEAT_ONLY) {
            faces(std::integral_constant<int, 0>{});
        } else {
            switch (kind) {
            case 0: faces(std::integral_constant<int, 0>{}); break;
            case 1: faces(std::integral_constant<int, 1>{}); break;
            case 2: faces(std::integral_constant<int, 2>{}); break;
            default: faces(std::integral_constant<int, 3>{}); break;
            }
        }
    };

    for (int k = 0; k < nsteps; ++k) {
        const uint64_t n = static_cast<uint64_t>(step0 + k);
        T z[MAXG][4];
#pragma unroll
        for (int s = 0; s < MAXG; ++s) {
            const int g = t + s * TS;
            if (noise != 2 && g < nfg) {
                const Normals4<T> nz = block_normals<T, true>(static_cast<uint32_t>(g), static_cast<uint32_t>(n),
                                                              ctr_word2(n, 0u), d.realisation, key);
#pragma unroll
                for (int l = 0; l < 4; ++l) z[s][l] = nz.z[l];
            } else {
#pragma unroll
                for (int l = 0; l < 4; ++l) z[s][l] = T(0);
            }
        }
        T rnz[MAXG], dv[MAXG][4];
#pragma unroll
        for (int s = 0; s < MAXG; ++s) rnz[s] = T(0);
        stage(u, z, rnz, dv, true);
        if (MODE == 2 && impl) {
            // right-hand side in FP64, then M U' = rhs by parallel cyclic
            // reduction in the FP64 LDS array (same cells per thread)
            double x[MAXG][4];
#pragma unroll
            for (int s = 0; s < MAXG; ++s)
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    const int i = 4 * (t + s * TS) + l;
                    x[s][l] = static_cast<double>(u[s][l] + dv[s][l]);
                    if (i < N) PD[i] = x[s][l];
                }
            const double *P = pcr + d.p_off;
            const int L = d.pcr_levels;
            // factors of the current level in registers; the next level's are
            // loaded before this level's barriers so their latency overlaps
            double f1[MAXG][4], f2[MAXG][4];
            auto load_level = [&](int lv, double (&a)[MAXG][4], double (&b)[MAXG][4]) __attribute__((always_inline)) {
                const double *k1 = P + static_cast<int64_t>(lv) * N, *k2 = P + static_cast<int64_t>(L + lv) * N;
#pragma unroll
                for (int s = 0; s < MAXG; ++s)
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        const int i = 4 * (t + s * TS) + l;
                        a[s][l] = i < N ? k1[i] : 0.0;
                        b[s][l] = i < N ? k2[i] : 0.0;
                    }
            };
            if (L > 0) load_level(0, f1, f2);
            __syncthreads();
            for (int lv = 0; lv < L; ++lv) {
                const int sh = 1 << lv;
#pragma unroll
                for (int s = 0; s < MAXG; ++s)
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        const int i = 4 * (t + s * TS) + l;
                        if (i < N) {
                            double v = PD[i];
                            if (i >= sh) v -= f1[s][l] * PD[i - sh];
                            if (i + sh < N) v -= f2[s][l] * PD[i + sh];
                            x[s][l] = v;
                        }
                    }
                if (lv + 1 < L) load_level(lv + 1, f1, f2);
                __syncthreads();
#pragma unroll
                for (int s = 0; s < MAXG; ++s)
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        const int i = 4 * (t + s * TS) + l;
                        if (i < N) PD[i] = x[s][l];
                    }
                __syncthreads();
            }
            const double *invb = P + static_cast<int64_t>(2 * L) * N;
#pragma unroll
            for (int s = 0; s < MAXG; ++s)
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    const int i = 4 * (t + s * TS) + l;
                    if (i < N) x[s][l] *= invb[i];
                }
            if (!dir) {
                // cyclic part: x = y - f z, f = (y_0 + q y_(N-1)) / (1 + z_0 + q z_(N-1))
#pragma unroll
                for (int s = 0; s < MAXG; ++s)
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        const int i = 4 * (t + s * TS) + l;
                        if (i < N) PD[i] = x[s][l];
                    }
                __syncthreads();
                const double *zv = invb + N;
                const double f = (PD[0] + zv[N] * PD[N - 1]) * zv[N + 1];
#pragma unroll
                for (int s = 0; s < MAXG; ++s)
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        const int i = 4 * (t + s * TS) + l;
                        if (i < N) x[s][l] -= f * zv[i];
                    }
            }
#pragma unroll
            for (int s = 0; s < MAXG; ++s)
#pragma unroll
                for (int l = 0; l < 4; ++l) u[s][l] = static_cast<T>(x[s][l]);
        } else if (d.scheme == 0) {
#pragma unroll
            for (int s = 0; s < MAXG; ++s)
#pragma unroll
                for (int l = 0; l < 4; ++l) u[s][l] = u[s][l] + dv[s][l];
        } else {
            T us[MAXG][4];
#pragma unroll
            for (int s = 0; s < MAXG; ++s)
#pragma unroll
                for (int l = 0; l < 4; ++l) us[s][l] = u[s][l] + dv[s][l];
            stage(us, z, rnz, dv, false);
#pragma unroll
            for (int s = 0; s < MAXG; ++s)
#pragma unroll
                for (int l = 0; l < 4; ++l) u[s][l] = T(0.5) * ((u[s][l] + us[s][l]) + dv[s][l]);
        }

        if (STATS) {
            if (step0 + k + 1 == t_next) {
                t_next += every;
                double a = 0.0, b = 0.0;
                int bad = 0;
                double del[MAXG][4];
                const int row = static_cast<int>(nsamp % kCorrBlock);
                T *X = corr ? static_cast<T *>(st.xblk) + d.x_off : nullptr;
                T *Hrow = tcorr ? static_cast<T *>(st.hist) + d.h_off + (nsamp % st.hist_rows) * N : nullptr;
#pragma unroll
                for (int s = 0; s < MAXG; ++s)
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        const int i = 4 * (t + s * TS) + l;
                        del[s][l] = 0.0;
                        if (i < N) {
                            const T v = u[s][l];
                            if (!isfinite(v)) bad = 1;
                            const double dl = static_cast<double>(v) - fma(ref_slope, i + 0.5, ref0);
                            del[s][l] = dl;
                            if (kRegSums) {
                                s1[s][l] += dl;
                                s2[s][l] += dl * dl;
                            }
                            a += dl;
                            b += dl * dl;
                            if (corr) X[(int64_t)row * N + i] = static_cast<T>(dl);
                            if (tcorr) Hrow[i] = static_cast<T>(dl);
                        }
                    }
                // sums over the instance (fixed order): DPP within each wave,
                // then (several waves) the wave sums through LDS, added by every
                // thread in the same order
                a = wave_total(a);
                b = wave_total(b);
                bad = __any(bad) ? 1 : 0;
                if (seg.nw > 1) {
                    if ((t & 63) == 0) {
                        red[lw] = a;
                        red[16 + lw] = b;
                        red[32 + lw] = static_cast<double>(bad);
                    }
                    __syncthreads();
                    a = b = 0.0;
                    bad = 0;
                    for (int w = 0; w < seg.nw; ++w) {
                        a += red[w];
                        b += red[16 + w];
                        bad |= red[32 + w] != 0.0;
                    }
                }
                if (bad) {
                    // a non-finite sample: keep the statistics as they were
                    // before it and freeze the state
#pragma unroll
                    for (int s = 0; s < MAXG; ++s)
#pragma unroll
                        for (int l = 0; l < 4; ++l) {
                            const int i = 4 * (t + s * TS) + l;
                            if (i < N) gU[i] = u[s][l];
                        }
                    if (t == 0) {
                        acc->nonfinite = 1;
                        acc->n_samples = nsamp;
                        acc->sp_mean = sp_mean;
                        acc->sp_sq = sp_sq;
                        acc->sp_var = sp_var;
                    }
                    return;
                }
                a /= N;
                b /= N;
                sp_mean += a;
                sp_sq += b;
                sp_var += b - a * a;
                if (!kRegSums && moments) {
#pragma unroll
                    for (int s = 0; s < MAXG; ++s)
#pragma unroll
                        for (int l = 0; l < 4; ++l) {
                            const int i = 4 * (t + s * TS) + l;
                            if (i < N) {
                                st.s1[d.off + i] += del[s][l];
                                st.s2[d.off + i] += del[s][l] * del[s][l];
                            }
                        }
                }
                ++nsamp;
                if (corr && row == kCorrBlock - 1) {
                    __threadfence_block();
                    __syncthreads();
                    xtx_block<T>(X, st.c + d.c_off, N, lw, seg.nw);
                    __syncthreads();
                }
            }
        }
    }

#pragma unroll
    for (int s = 0; s < MAXG; ++s)
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int i = 4 * (t + s * TS) + l;
            if (i < N) gU[i] = u[s][l];
        }
    if (kRegSums && moments) {
#pragma unroll
        for (int s = 0; s < MAXG; ++s)
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                const int i = 4 * (t + s * TS) + l;
                if (i < N) {
                    st.s1[d.off + i] = s1[s][l];
                    st.s2[d.off + i] = s2[s][l];
                }
            }
    }
    if (STATS) {
        if (clamps) atomicAdd(reinterpret_cast<unsigned long long *>(&acc->clamp_count),
                              static_cast<unsigned long long>(clamps));
        if (t == 0) {
            acc->n_samples = nsamp;
            acc->sp_mean = sp_mean;
            acc->sp_sq = sp_sq;
            acc->sp_var = sp_var;
        }
    }
}

template <typename T, int BLOCK, int MAXG, bool STATS, int MODE>
__global__ void __launch_bounds__(BLOCK)
    k_step1d(const Inst1D *__restrict__ tab, const Seg1D *__restrict__ segs, T *__restrict__ pool,
             const T *__restrict__ coef, const double *__restrict__ pcr, int64_t step0, int32_t nsteps,
             int64_t burn_in, int32_t every, uint32_t mask, Stats1D st)
{
    step1d_body<T, BLOCK, MAXG, STATS, MODE>(tab, segs, pool, coef, pcr, step0, nsteps, burn_in, every, mask, st);
}

// 1024 threads with one Philox block each, for a uniform explicit FP32 batch
// of heat instances with instantaneous noise and no statistics (only that
// face path is compiled), held to 64 VGPRs so that two workgroups (32 waves) fit on a
// CU: a packed batch of instances up to 4096 Philox blocks stays resident in
// one round while its largest instances keep one block per thread.
template <typename T>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
    k_step1d_wide(const Inst1D *__restrict__ tab, const Seg1D *__restrict__ segs, T *__restrict__ pool,
                  const T *__restrict__ coef, const double *__restrict__ pcr, int64_t step0, int32_t nsteps,
                  int64_t burn_in, int32_t every, uint32_t mask, Stats1D st)
{
    step1d_body<T, 1024, 1, false, 3>(tab, segs, pool, coef, pcr, step0, nsteps, burn_in, every, mask, st);
}

// ------------------------------------------------------------------ time correlation

// grid: (ceil(nmax L / 256), n_inst); thread (m, i) with i fastest, so the
// ring rows are read coalesced.  Sample n sits in ring row n mod hist_rows;
// the host keeps each launch's new samples plus L - 1 older ones in the ring.
template <typename T>
__global__ void __launch_bounds__(256)
    k_tcorr(const Inst1D *__restrict__ tab, const T *__restrict__ hist, int32_t hist_rows, int32_t lags, int64_t n0,
            int64_t count, double *__restrict__ tc, const InstAcc *__restrict__ acc)
{
    const int inst = blockIdx.y;
    const Inst1D d = tab[inst];
    if (d.h_off < 0) return;
    const int N = d.n;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e >= static_cast<int64_t>(N) * lags) return;
    const int i = static_cast<int>(e % N), m = static_cast<int>(e / N);
    const int64_t n1 = min(n0 + count, acc[inst].n_samples);  // a frozen instance stopped sampling
    const int64_t nb = max(n0, static_cast<int64_t>(m));
    if (nb >= n1) return;
    const T *h = hist + d.h_off + i;
    int64_t a = nb % hist_rows, b = (nb - m) % hist_rows;
    double sum = 0.0;
    for (int64_t n = nb; n < n1; ++n) {
        sum += static_cast<double>(h[a * N]) * static_cast<double>(h[b * N]);
        if (++a == hist_rows) a = 0;
        if (++b == hist_rows) b = 0;
    }
    tc[d.tc_off + static_cast<int64_t>(m) * N + i] += sum;
}

__global__ void __launch_bounds__(256)
    k_fin_tc(int n, int lags, const double *__restrict__ s1, const double *__restrict__ tc, int64_t M,
             double *__restrict__ out)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e >= static_cast<int64_t>(n) * lags) return;
    const int i = static_cast<int>(e % n), m = static_cast<int>(e / n);
    if (M <= m) {
        out[e] = __builtin_nan("");
        return;
    }
    const double mu = s1[i] / static_cast<double>(M);
    out[e] = tc[e] / static_cast<double>(M - m) - mu * mu;
}

hipError_t launch_tcorr1d(int prec, int n_inst, int nmax, int lags, hipStream_t s, const Inst1D *tab,
                          const void *hist, int32_t hist_rows, int64_t n0, int64_t count, double *tc,
                          const InstAcc *acc)
{
    const dim3 grid(static_cast<unsigned>((static_cast<int64_t>(nmax) * lags + 255) / 256), n_inst);
    if (prec == 0)
        hipLaunchKernelGGL(k_tcorr<float>, grid, dim3(256), 0, s, tab, static_cast<const float *>(hist), hist_rows,
                           lags, n0, count, tc, acc);
    else
        hipLaunchKernelGGL(k_tcorr<double>, grid, dim3(256), 0, s, tab, static_cast<const double *>(hist),
                           hist_rows, lags, n0, count, tc, acc);
    return hipGetLastError();
}

hipError_t launch_fin_tc(hipStream_t s, int n, int lags, const double *s1, const double *tc, int64_t M,
                         double *out)
{
    const int64_t tot = static_cast<int64_t>(n) * lags;
    hipLaunchKernelGGL(k_fin_tc, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, s, n, lags, s1, tc, M,
                       out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ init

template <typename T>
__global__ void __launch_bounds__(256)
    k_init1d(const Inst1D *__restrict__ tab, const double *__restrict__ init_sd, T *__restrict__ pool)
{
    const int inst = blockIdx.x;
    const Inst1D d = tab[inst];
    const int i = blockIdx.y * 256 + threadIdx.x;
    if (i >= d.n) return;
    const double ref = d.bc == 1 ? d.uL + (d.uR - d.uL) * (i + 0.5) / d.n : d.u0;
    double v = ref;
    const double sd = init_sd[inst];
    if (sd > 0.0) {
        const Normals4<double> nz = block_normals<double>(static_cast<uint32_t>(i >> 2), 0u, ctr_word2(0, 1u),
                                                          d.realisation, make_key(d.seed));
        v = ref + sd * nz.z[i & 3];
    }
    pool[d.off + i] = static_cast<T>(v);
}

// ------------------------------------------------------------------ finalisation

// m2[i][j] = (C[i][j] + sum over the rows of the open block X_b,i X_b,j) / M
template <typename T>
__global__ void __launch_bounds__(256)
    k_fin_m2(const T *__restrict__ X, int rows, const double *__restrict__ C, int N, int64_t M,
             double *__restrict__ m2)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e >= static_cast<int64_t>(N) * N) return;
    const int i = static_cast<int>(e / N), j = static_cast<int>(e - static_cast<int64_t>(i) * N);
    double acc = C[e];
    for (int b = 0; b < rows; ++b)
        acc += static_cast<double>(X[static_cast<int64_t>(b) * N + i]) * static_cast<double>(X[static_cast<int64_t>(b) * N + j]);
    m2[e] = acc / static_cast<double>(M);
}

// mean, variance per cell, sum(U) of the current field, covariance
template <typename T>
__global__ void __launch_bounds__(256)
    k_fin_cells(const Inst1D *__restrict__ tab, int inst, const T *__restrict__ pool,
                const double *__restrict__ s1, const double *__restrict__ s2, int64_t M, bool corr,
                double *__restrict__ out)
{
    const Inst1D d = tab[inst];
    const int N = d.n;
    double *mean = out, *var = out + N, *cov = out + 2 * N, *m2 = out + 3 * N + static_cast<int64_t>(N) * N;
    double *sum = m2 + static_cast<int64_t>(N) * N;
    const double inv = M > 0 ? 1.0 / static_cast<double>(M) : 0.0;
    for (int i = threadIdx.x; i < N; i += 256) {
        const double ref = d.bc == 1 ? d.uL + (d.uR - d.uL) * (i + 0.5) / N : d.u0;
        const double m = s1 ? s1[d.off + i] * inv : 0.0;
        mean[i] = ref + m;
        var[i] = s2 ? s2[d.off + i] * inv - m * m : 0.0;
    }
    if (corr) {
        for (int64_t e = threadIdx.x; e < static_cast<int64_t>(N) * N; e += 256) {
            const int i = static_cast<int>(e / N), j = static_cast<int>(e - static_cast<int64_t>(i) * N);
            cov[e] = m2[e] - (s1[d.off + i] * inv) * (s1[d.off + j] * inv);
        }
    }
    __shared__ double red[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < N; i += 256) a += static_cast<double>(pool[d.off + i]);
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *sum = red[0];
}

// <|U_k|^2> = |R_k|^2 + 2 Re(conj(R_k) sum_j m_j w^{jk}) + sum_ij m2_ij cos(2 pi k (i-j)/N),
// R_k = DFT of the reference profile, m = E[dU], m2 = E[dU dU^T].
__global__ void __launch_bounds__(256)
    k_fin_sk(const Inst1D *__restrict__ tab, int inst, const double *__restrict__ s1, int64_t M,
             double *__restrict__ out)
{
    const Inst1D d = tab[inst];
    const int N = d.n;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= N) return;
    const double *m2 = out + 3 * N + static_cast<int64_t>(N) * N;
    double *sk = out + 2 * N + static_cast<int64_t>(N) * N;
    const double inv = 1.0 / static_cast<double>(M);
    double rr = 0.0, ri = 0.0, mr = 0.0, mi = 0.0;
    for (int j = 0; j < N; ++j) {
        const int64_t idx = (static_cast<int64_t>(j) * k) % N;
        double sn, cs;
        sincospi(-2.0 * static_cast<double>(idx) / N, &sn, &cs);
        const double ref = d.bc == 1 ? d.uL + (d.uR - d.uL) * (j + 0.5) / N : d.u0;
        const double m = s1[d.off + j] * inv;
        rr += ref * cs;
        ri += ref * sn;
        mr += m * cs;
        mi += m * sn;
    }
    double q = 0.0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            int64_t idx = (static_cast<int64_t>(k) * (i - j)) % N;
            if (idx < 0) idx += N;
            q += m2[static_cast<int64_t>(i) * N + j] * cospi(2.0 * static_cast<double>(idx) / N);
        }
    sk[k] = (rr * rr + ri * ri) + 2.0 * (rr * mr + ri * mi) + q;
}

// ------------------------------------------------------------------ batch means

// Whether the last launch completed batch n_batches + 1 of this instance.
__device__ __forceinline__ bool batch_done(const InstAcc &q, int32_t len)
{
    return len > 0 && !q.nonfinite && q.n_samples >= (q.n_batches + 1) * static_cast<int64_t>(len);
}

// S_k of the batch, from its covariance sums: Cb = (C + the open X rows) -
// csnap, its circulant sums c(d) = sum_i Cb[i][(i - d) mod N] (so that
// sum_ij Cb_ij cos(2 pi k (i - j)/N) = sum_d c(d) cos(2 pi k d/N)), and the
// batch mean m_b of dU: S_k = |R_k|^2 + 2 Re(conj(R_k) DFT(m_b)_k) +
// sum_d c(d) cos(2 pi k d/N) / L, R the DFT of the reference profile (the
// formula of k_fin_sk for one batch).  Then csnap takes the current sums.
// One block per instance; runs before k_fold_cells1d (it reads the s1
// snapshot that kernel moves on).
template <typename T>
__global__ void __launch_bounds__(256)
    k_fold_sk1d(const Inst1D *__restrict__ tab, const T *__restrict__ xblk, const double *__restrict__ c,
                const double *__restrict__ s1, const InstAcc *__restrict__ acc, Batch1D bk)
{
    const int inst = blockIdx.x;
    const Inst1D d = tab[inst];
    const InstAcc q = acc[inst];
    if (d.c_off < 0 || !batch_done(q, bk.len)) return;
    __shared__ double cd[1024], mb[1024];
    const int N = d.n;
    const int rows = static_cast<int>(q.n_samples % kCorrBlock);  // open rows of the X block
    const T *X = xblk + d.x_off;
    const double *C = c + d.c_off;
    double *Cs = bk.csnap + d.c_off;
    const double *s1s = bk.cell;
    const double L = static_cast<double>(bk.len);
    auto ctot = [&](int i, int j) {
        double v = C[static_cast<int64_t>(i) * N + j];
        for (int r = 0; r < rows; ++r)
            v += static_cast<double>(X[static_cast<int64_t>(r) * N + i]) * static_cast<double>(X[static_cast<int64_t>(r) * N + j]);
        return v;
    };
    for (int dd = threadIdx.x; dd < N; dd += 256) {
        double a = 0.0;
        for (int i = 0; i < N; ++i) {
            const int j = i - dd < 0 ? i - dd + N : i - dd;
            a += ctot(i, j) - Cs[static_cast<int64_t>(i) * N + j];
        }
        cd[dd] = a;
    }
    for (int i = threadIdx.x; i < N; i += 256) mb[i] = (s1[d.off + i] - s1s[d.off + i]) / L;
    __syncthreads();
    for (int64_t e = threadIdx.x; e < static_cast<int64_t>(N) * N; e += 256) {
        const int i = static_cast<int>(e / N), j = static_cast<int>(e - static_cast<int64_t>(i) * N);
        Cs[e] = ctot(i, j);
    }
    const double b = static_cast<double>(q.n_batches + 1);
    for (int k = threadIdx.x; k < N; k += 256) {
        double rr = 0.0, ri = 0.0, mr = 0.0, mi = 0.0, qq = 0.0;
        for (int j = 0; j < N; ++j) {
            const int64_t idx = (static_cast<int64_t>(j) * k) % N;
            double sn, cs;
            sincospi(-2.0 * static_cast<double>(idx) / N, &sn, &cs);
            const double ref = d.bc == 1 ? d.uL + (d.uR - d.uL) * (j + 0.5) / N : d.u0;
            rr += ref * cs;
            ri += ref * sn;
            mr += mb[j] * cs;
            mi += mb[j] * sn;
            qq += cd[j] * cs;   // cos(2 pi k d / N) for d = j
        }
        const double x = (rr * rr + ri * ri) + 2.0 * (rr * mr + ri * mi) + qq / L;
        welford(x, b, bk.skw[d.off + k], bk.skw[bk.total_cells + d.off + k]);
    }
}

// Per-cell batch mean and variance of dU, folded into their Welford sums;
// the s1 / s2 snapshots move to the current sums.
__global__ void __launch_bounds__(256)
    k_fold_cells1d(const Inst1D *__restrict__ tab, const double *__restrict__ s1, const double *__restrict__ s2,
                   const InstAcc *__restrict__ acc, Batch1D bk)
{
    const int inst = blockIdx.x;
    const Inst1D d = tab[inst];
    const InstAcc q = acc[inst];
    const int i = blockIdx.y * 256 + threadIdx.x;
    if (i >= d.n || !batch_done(q, bk.len)) return;
    const int64_t tc = bk.total_cells, e = d.off + i;
    double *cl = bk.cell;
    const double L = static_cast<double>(bk.len), b = static_cast<double>(q.n_batches + 1);
    const double m = (s1[e] - cl[e]) / L;
    const double v = (s2[e] - cl[tc + e]) / L - m * m;
    welford(m, b, cl[2 * tc + e], cl[3 * tc + e]);
    welford(v, b, cl[4 * tc + e], cl[5 * tc + e]);
    cl[e] = s1[e];
    cl[tc + e] = s2[e];
}

// Spatial statistics of the batch and the batch count (last of the folds).
__global__ void __launch_bounds__(64) k_fold_acc1d(int n_inst, InstAcc *__restrict__ acc, int32_t len)
{
    const int inst = blockIdx.x * 64 + threadIdx.x;
    if (inst >= n_inst) return;
    InstAcc q = acc[inst];
    if (!batch_done(q, len)) return;
    fold_spatial(q, len);
    acc[inst] = q;
}

hipError_t launch_fold1d(int prec, int n_inst, int nmax, hipStream_t s, const Inst1D *tab, const void *xblk,
                         const double *c, const double *s1, const double *s2, InstAcc *acc, const Batch1D &bk)
{
    if (bk.csnap) {
        if (prec == 0)
            hipLaunchKernelGGL(k_fold_sk1d<float>, dim3(n_inst), dim3(256), 0, s, tab,
                               static_cast<const float *>(xblk), c, s1, acc, bk);
        else
            hipLaunchKernelGGL(k_fold_sk1d<double>, dim3(n_inst), dim3(256), 0, s, tab,
                               static_cast<const double *>(xblk), c, s1, acc, bk);
    }
    if (bk.cell)
        hipLaunchKernelGGL(k_fold_cells1d, dim3(n_inst, (nmax + 255) / 256), dim3(256), 0, s, tab, s1, s2, acc, bk);
    hipLaunchKernelGGL(k_fold_acc1d, dim3((n_inst + 63) / 64), dim3(64), 0, s, n_inst, acc, bk.len);
    return hipGetLastError();
}

// ------------------------------------------------------------------ launchers

struct Step1DLaunch {
    int n_blocks;
    size_t smem;
    hipStream_t s;
    const Inst1D *tab;
    const Seg1D *segs;
    void *pool;
    const void *coef;
    const double *pcr;
    int64_t step0;
    int32_t nsteps;
    int64_t burn_in;
    int32_t every;
    uint32_t mask;
    Stats1D st;
};

template <typename T, int BLOCK, int MAXG, bool STATS, int MODE>
static hipError_t step1d_k(const Step1DLaunch &a)
{
    hipLaunchKernelGGL((k_step1d<T, BLOCK, MAXG, STATS, MODE>), dim3(a.n_blocks), dim3(BLOCK), a.smem, a.s, a.tab,
                       a.segs, static_cast<T *>(a.pool), static_cast<const T *>(a.coef), a.pcr, a.step0, a.nsteps,
                       a.burn_in, a.every, a.mask, a.st);
    return hipGetLastError();
}

template <typename T, int BLOCK, int MAXG, bool STATS>
static hipError_t step1d_m(int mode, const Step1DLaunch &a)
{
    switch (mode) {
    case 0: return step1d_k<T, BLOCK, MAXG, STATS, 0>(a);
    case 1: return step1d_k<T, BLOCK, MAXG, STATS, 1>(a);
    case 2: return step1d_k<T, BLOCK, MAXG, STATS, 2>(a);
    case 3: return step1d_k<T, BLOCK, MAXG, STATS, 3>(a);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int BLOCK, int MAXG>
static hipError_t step1d_t(bool stats, int mode, const Step1DLaunch &a)
{
    return stats ? step1d_m<T, BLOCK, MAXG, true>(mode, a) : step1d_m<T, BLOCK, MAXG, false>(mode, a);
}

// Launch shapes (threads per workgroup, Philox blocks per thread) the
// planner chooses: 64 x {1, 2}, 256 x {1, 2}, 512 x {1, 2, 4}, and 1024 x 1
// for uniform explicit batches without statistics.
template <typename T>
static hipError_t step1d_p(int block, int maxg, bool stats, int mode, const Step1DLaunch &a)
{
    if (block == 64 && maxg == 1) return step1d_t<T, 64, 1>(stats, mode, a);
    if (block == 64 && maxg == 2) return step1d_t<T, 64, 2>(stats, mode, a);
    if (block == 256 && maxg == 1) return step1d_t<T, 256, 1>(stats, mode, a);
    if (block == 256 && maxg == 2) return step1d_t<T, 256, 2>(stats, mode, a);
    if (block == 512 && maxg == 1) return step1d_t<T, 512, 1>(stats, mode, a);
    if (block == 512 && maxg == 2) return step1d_t<T, 512, 2>(stats, mode, a);
    if (block == 512 && maxg == 4) return step1d_t<T, 512, 4>(stats, mode, a);
    if constexpr (std::is_same<T, float>::value) {
        if (block == 1024 && maxg == 1 && !stats && mode == 3) {
            hipLaunchKernelGGL((k_step1d_wide<T>), dim3(a.n_blocks), dim3(1024), a.smem, a.s, a.tab, a.segs,
                               static_cast<T *>(a.pool), static_cast<const T *>(a.coef), a.pcr, a.step0,
                               a.nsteps, a.burn_in, a.every, a.mask, a.st);
            return hipGetLastError();
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step1d(int prec, int block, int maxg, bool stats, int mode, int n_blocks, size_t smem,
                         hipStream_t s, const Inst1D *tab, const Seg1D *segs, void *pool, const void *coef,
                         const double *pcr, int64_t step0, int32_t nsteps, int64_t burn_in, int32_t every,
                         uint32_t mask, Stats1D st)
{
    const Step1DLaunch a{n_blocks, smem, s, tab, segs, pool, coef, pcr, step0, nsteps, burn_in, every, mask, st};
    if (prec == 0) return step1d_p<float>(block, maxg, stats, mode, a);
    return step1d_p<double>(block, maxg, stats, mode, a);
}

hipError_t launch_init1d(int prec, int n_inst, int nmax, hipStream_t s, const Inst1D *tab, const double *init_sd,
                         void *pool)
{
    const dim3 grid(n_inst, (nmax + 255) / 256);
    if (prec == 0)
        hipLaunchKernelGGL(k_init1d<float>, grid, dim3(256), 0, s, tab, init_sd, static_cast<float *>(pool));
    else
        hipLaunchKernelGGL(k_init1d<double>, grid, dim3(256), 0, s, tab, init_sd, static_cast<double *>(pool));
    return hipGetLastError();
}

hipError_t launch_fin1d(int prec, hipStream_t s, const Inst1D *tab, int inst, int n, const void *pool,
                        const double *s1, const double *s2, const void *xblk, const double *c, int64_t n_samples,
                        int partial_rows, bool corr, double *out)
{
    const int64_t nn = static_cast<int64_t>(n) * n;
    double *m2 = out + 3 * n + nn;
    const int64_t M = n_samples > 0 ? n_samples : 1;
    if (corr) {
        const int nb = static_cast<int>((nn + 255) / 256);
        if (prec == 0)
            hipLaunchKernelGGL(k_fin_m2<float>, dim3(nb), dim3(256), 0, s, static_cast<const float *>(xblk),
                               partial_rows, c, n, M, m2);
        else
            hipLaunchKernelGGL(k_fin_m2<double>, dim3(nb), dim3(256), 0, s, static_cast<const double *>(xblk),
                               partial_rows, c, n, M, m2);
    }
    if (prec == 0)
        hipLaunchKernelGGL(k_fin_cells<float>, dim3(1), dim3(256), 0, s, tab, inst, static_cast<const float *>(pool),
                           s1, s2, M, corr, out);
    else
        hipLaunchKernelGGL(k_fin_cells<double>, dim3(1), dim3(256), 0, s, tab, inst,
                           static_cast<const double *>(pool), s1, s2, M, corr, out);
    if (corr) hipLaunchKernelGGL(k_fin_sk, dim3((n + 255) / 256), dim3(256), 0, s, tab, inst, s1, M, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ verification

__global__ void __launch_bounds__(256)
    k_debug_philox(uint64_t seed, const uint32_t *__restrict__ ctr, int64_t count, uint32_t *__restrict__ out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= count) return;
    const Words4 w = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], make_key(seed));
    for (int l = 0; l < 4; ++l) out[4 * i + l] = w.w[l];
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_debug_normals(uint64_t seed, uint32_t real, uint32_t tag, uint64_t step, uint64_t face0, int64_t count,
                    double *__restrict__ out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= count) return;
    const uint64_t f = face0 + static_cast<uint64_t>(i);
    const Normals4<T> nz = block_normals<T>(static_cast<uint32_t>(f >> 2), static_cast<uint32_t>(step),
                                            ctr_word2(step, tag), real, make_key(seed));
    out[i] = static_cast<double>(nz.z[f & 3]);
}

hipError_t launch_debug_philox(hipStream_t s, uint64_t seed, const uint32_t *ctr, int64_t count, uint32_t *out)
{
    hipLaunchKernelGGL(k_debug_philox, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s, seed, ctr,
                       count, out);
    return hipGetLastError();
}

hipError_t launch_debug_normals(hipStream_t s, int prec, uint64_t seed, uint32_t realisation, uint32_t tag,
                                uint64_t step, uint64_t face0, int64_t count, double *out)
{
    const dim3 grid(static_cast<unsigned>((count + 255) / 256));
    if (prec == 0)
        hipLaunchKernelGGL(k_debug_normals<float>, grid, dim3(256), 0, s, seed, realisation, tag, step, face0, count,
                           out);
    else
        hipLaunchKernelGGL(k_debug_normals<double>, grid, dim3(256), 0, s, seed, realisation, tag, step, face0, count,
                           out);
    return hipGetLastError();
}

}  // namespace she
