// Host runtime behind include/she.h: validation, device memory plan, launch
// schedule, finalisation and checkpoints.  No arithmetic of the method lives
// here beyond the FP64 coefficient sigma = sqrt(2 r eps) (Sec. 3: the face
// noise alpha dt/dx * N/sqrt(dV dt) of the SHE; Sec. 4 eq. DK with eps = 1/dV).
#include "she.h"
#include "she_internal.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

using namespace she;

struct she_handle {
    std::string err;
    int dim = 1, prec = 0;
    size_t esz = 4;
    int n_inst = 0;
    std::vector<she_instance_desc> inst;
    int64_t burn_in = 0;
    int32_t every = 1;
    uint32_t mask = 0;
    hipStream_t stream = nullptr;
    int64_t steps = 0;
    int device = 0;

    // device memory
    bool own = false;
    char *base = nullptr;
    size_t bytes = 0;

    InstAcc *d_acc = nullptr;
    double *d_fin = nullptr;      // finalisation scratch
    size_t fin_len = 0;
    double *d_init_sd = nullptr;

    // 1D
    Inst1D *d_tab = nullptr;
    Seg1D *d_segs = nullptr;      // per wave of the 1D launch
    std::vector<Seg1D> segs_host;
    int blocks1d = 0;             // workgroups of the 1D launch
    int mode1d = 0;               // kernel mode (see launch_step1d)
    void *d_pool = nullptr;
    std::vector<Inst1D> tab;
    int64_t total_cells = 0;
    double *d_s1 = nullptr, *d_s2 = nullptr;
    void *d_x = nullptr;
    double *d_c = nullptr;
    int64_t x_elems = 0, c_elems = 0;
    int block1d = 64, maxg = 1, nmax = 0;
    // time correlation: history ring of hist_rows sample rows, L x N lag sums
    int tc_lags = 0;
    int32_t hist_rows = 0;
    int64_t samples = 0;          // 1D: samples since create / reset (equal on every instance still sampling)
    void *d_hist = nullptr;
    double *d_tc = nullptr;
    int64_t hist_elems = 0, tc_elems = 0;
    // material varying along the rod: r_f, s_f, w_i per instance (state type)
    bool varc = false;
    std::vector<double> coef_host;
    void *d_coef = nullptr;
    std::vector<double> pcr_host;     // implicit schemes: FP64 reduction factors
    double *d_pcr = nullptr;
    size_t smem1d = 0;

    // batch means: samples per batch (0: none) and their arrays
    int32_t batch_len = 0;
    double *d_bcell = nullptr, *d_csnap = nullptr, *d_skw1 = nullptr;      // 1D (Batch1D)
    double *d_sksnap = nullptr, *d_skwm = nullptr, *d_skwm2 = nullptr;     // 2D S(k) (BatchSk)

    // 2D / 3D
    ParamsND pnd{};
    int64_t cells = 0;            // per instance
    void *d_a = nullptr, *d_b = nullptr;
    void *d_pred = nullptr;       // 3D PC: predictor field
    int cur = 0;                  // 0: state in d_a
    InstND *d_ip = nullptr;       // per-instance parameters
    std::vector<InstND> ip_host;
    double *d_part = nullptr;
    int nparts = 0, cx = 4, ty = 1, nd_blocks = 0;
    size_t smem3d = 0;
    // 2D structure factor
    int nbins = 0, sk_groups = 0;
    void *d_half = nullptr, *d_twx = nullptr, *d_twy = nullptr;
    uint16_t *d_shells = nullptr;  // first |ky| of each shell per column (shell_table)
    double *d_skpart = nullptr, *d_sksum = nullptr, *d_skmodes = nullptr;
    std::vector<double> skmodes;
    // captured step loops: [0] without, [1] with sample steps
    int64_t *d_step = nullptr;    // device step counter read by replayed kernels
    int64_t dev_step = -1;        // value *d_step holds once the stream is idle
    int32_t graph_steps = 0;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int64_t gk[2] = {0, 0};
    // 2D FE: two steps per launch where no sample falls between them, in
    // march chunks of chunk2 rows
    bool two_step = false;
    int chunk2 = 0, nparts2 = 0, nd_blocks2 = 0;
    // 2D FE with S(k): the two-step sample launches transform their rows
    // themselves (one row per wave, even march chunks)
    bool sk_fused = false;

    void *field() const { return dim == 1 ? d_pool : (cur == 0 ? d_a : d_b); }
    // 1D: per-cell sums are kept (and so per-cell batch means)
    bool d_s1_planned() const { return (mask & (SHE_STAT_MOMENTS | SHE_STAT_CORR | SHE_STAT_TCORR)) != 0; }
};

static thread_local std::string g_create_err;

namespace {

she_status fail(she_handle *h, she_status st, const std::string &msg)
{
    if (h)
        h->err = msg;
    else
        g_create_err = msg;
    return st;
}

she_status hipfail(she_handle *h, hipError_t e, const char *what)
{
    return fail(h, SHE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define SHE_HIP(h, call)                                   \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hipfail((h), e_, #call); \
    } while (0)

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Face conductivity ratios of a 1D rod with cell ratios cond (NULL: 1): an
// interior face conducts like its two half cells in series (harmonic mean),
// a Dirichlet wall face like its cell.  Faces 0..N-1 (periodic) or 0..N.
std::vector<double> face_conductivity(const she_instance_desc &d)
{
    const int N = d.n[0];
    const bool dir = d.bc == SHE_DIRICHLET;
    auto lam = [&](int i) { return d.cond ? d.cond[i] : 1.0; };
    std::vector<double> lf(dir ? N + 1 : N);
    for (int f = 0; f < static_cast<int>(lf.size()); ++f) {
        if (dir && f == 0) lf[f] = lam(0);
        else if (dir && f == N) lf[f] = lam(N - 1);
        else {
            const double a = lam((f - 1 + N) % N), b = lam(f % N);
            lf[f] = 2.0 * a * b / (a + b);
        }
    }
    return lf;
}

// Rows of M = I - theta W A of an implicit 1D step: lo[i], di[i], up[i]
// multiply U_(i-1), U_i, U_(i+1) (cyclic for periodic rods); A is the
// noise-free flux divergence with face conductances r_f (a Dirichlet wall
// face twice on the diagonal), W the per-cell capacity factors.
void implicit_rows(const she_instance_desc &d, double theta, std::vector<double> &lo, std::vector<double> &di,
                   std::vector<double> &up)
{
    const int N = d.n[0];
    const bool dir = d.bc == SHE_DIRICHLET;
    const std::vector<double> lf = face_conductivity(d);
    lo.assign(N, 0.0);
    di.assign(N, 0.0);
    up.assign(N, 0.0);
    for (int i = 0; i < N; ++i) {
        const double rl = d.r * lf[i], rh = d.r * lf[dir ? i + 1 : (i + 1) % N];
        const double w = d.cap ? 1.0 / d.cap[i] : 1.0;
        const double dl = (dir && i == 0) ? 2.0 * rl : rl, dh = (dir && i == N - 1) ? 2.0 * rh : rh;
        di[i] = 1.0 + theta * w * (dl + dh);
        lo[i] = (dir && i == 0) ? 0.0 : -theta * w * rl;
        up[i] = (dir && i == N - 1) ? 0.0 : -theta * w * rh;
    }
}

// Factors of parallel cyclic reduction for a x_(i-1) + b x_i + c x_(i+1) = d
// with a_0 = c_(N-1) = 0: level l (stride s = 2^l) replaces row i by itself
// minus k1 times row i-s minus k2 times row i+s (k1 = a_i / b_(i-s),
// k2 = c_i / b_(i+s)), which leaves it coupled to rows i -+ 2s; after
// ceil(log2 N) levels every row holds one unknown.  Appends k1[L][N],
// k2[L][N], 1/b[N] to out and returns L.
int pcr_factors(std::vector<double> a, std::vector<double> b, std::vector<double> c, std::vector<double> &out)
{
    const int N = static_cast<int>(b.size());
    int L = 0;
    while ((1 << L) < N) ++L;
    std::vector<double> k1(static_cast<size_t>(L) * N), k2(static_cast<size_t>(L) * N);
    for (int l = 0; l < L; ++l) {
        const int s = 1 << l;
        std::vector<double> na(N, 0.0), nb(N), nc(N, 0.0);
        for (int i = 0; i < N; ++i) {
            const double f1 = i - s >= 0 ? a[i] / b[i - s] : 0.0;
            const double f2 = i + s < N ? c[i] / b[i + s] : 0.0;
            nb[i] = b[i] - (i - s >= 0 ? f1 * c[i - s] : 0.0) - (i + s < N ? f2 * a[i + s] : 0.0);
            if (i - s >= 0) na[i] = -f1 * a[i - s];
            if (i + s < N) nc[i] = -f2 * c[i + s];
            k1[static_cast<size_t>(l) * N + i] = f1;
            k2[static_cast<size_t>(l) * N + i] = f2;
        }
        a.swap(na);
        b.swap(nb);
        c.swap(nc);
    }
    out.insert(out.end(), k1.begin(), k1.end());
    out.insert(out.end(), k2.begin(), k2.end());
    for (int i = 0; i < N; ++i) out.push_back(1.0 / b[i]);
    return L;
}

// Thomas algorithm (host, FP64) for the Sherman-Morrison vector.
std::vector<double> thomas_solve(const std::vector<double> &a, const std::vector<double> &b,
                                 const std::vector<double> &c, std::vector<double> d)
{
    const int N = static_cast<int>(b.size());
    std::vector<double> cp(N, 0.0);
    double den = b[0];
    d[0] /= den;
    for (int i = 1; i < N; ++i) {
        cp[i] = c[i - 1] / den;
        den = b[i] - a[i] * cp[i];
        d[i] = (d[i] - a[i] * d[i - 1]) / den;
    }
    for (int i = N - 2; i >= 0; --i) d[i] -= cp[i + 1] * d[i + 1];
    return d;
}

// Largest modulus over wavenumbers theta of the one-step factor of the
// linearised Burgers scheme at the steepest slope |1 - 2c| = 1:
// L = -4 r sin^2(theta/2) - i nu sin(theta), G = 1 + L (FE), 1 + L + L^2/2 (PC).
double burgers_growth(double r, double nu, int scheme)
{
    double worst = 0.0;
    for (int j = 0; j <= 4096; ++j) {
        const double th = M_PI * j / 4096.0;
        const double lr = -4.0 * r * std::sin(0.5 * th) * std::sin(0.5 * th), li = -nu * std::sin(th);
        double gr = 1.0 + lr, gi = li;
        if (scheme == SHE_HEUN) {
            gr += 0.5 * (lr * lr - li * li);
            gi += lr * li;
        }
        worst = std::max(worst, std::sqrt(gr * gr + gi * gi));
    }
    return worst;
}

// Gershgorin bound of the FE operator w_i (sum of row i's conductances, the
// Dirichlet wall face counted twice on the diagonal); the step is stable
// when it is at most 2.
double varc_row_bound(const she_instance_desc &d)
{
    const int N = d.n[0];
    const bool dir = d.bc == SHE_DIRICHLET;
    const std::vector<double> lf = face_conductivity(d);
    double worst = 0.0;
    for (int i = 0; i < N; ++i) {
        const int hi = dir ? i + 1 : (i + 1) % N;
        const double lo_c = (dir && i == 0) ? 2.0 * lf[0] : lf[i];
        const double hi_c = (dir && i == N - 1) ? 2.0 * lf[N] : lf[hi];
        const double lo_g = (dir && i == 0) ? 0.0 : lf[i];
        const double hi_g = (dir && i == N - 1) ? 0.0 : lf[hi];
        const double w = d.cap ? 1.0 / d.cap[i] : 1.0;
        worst = std::max(worst, w * d.r * (lo_c + hi_c + lo_g + hi_g));
    }
    return worst;
}

// beta = (1/n) sum over the modes k != 0 of h_k cos^2(pi k_x / n_x) of a
// periodic grid, h_k = 1 / (1 - x_k / 2), x_k = 4 r sum_d sin^2(pi k_d / n_d):
// the face temperature's share of the FE stationary spectrum N eps m^2 h_k /
// (1 - eps beta) that feeds the instantaneous noise back into itself (the
// face value is the mean of the two cells, whose spectrum weight is
// cos^2(pi k_x / n_x) for an x-face).  Modes k and n - k give the same
// terms, so each axis runs over k <= n/2 with multiplicity 1 or 2.  Infinite
// when a mode has x_k >= 2 (FE amplification -1: no damping at all).
double fe_beta(const she_instance_desc &d)
{
    std::vector<double> s2[3], mult[3];
    for (int a = 0; a < 3; ++a) {
        const int n = a < d.dim ? d.n[a] : 1;
        for (int k = 0; 2 * k <= n; ++k) {
            const double s = std::sin(M_PI * k / n);
            s2[a].push_back(s * s);
            mult[a].push_back((k == 0 || 2 * k == n) ? 1.0 : 2.0);
        }
    }
    double sum = 0.0;
    for (size_t kz = 0; kz < s2[2].size(); ++kz)
        for (size_t ky = 0; ky < s2[1].size(); ++ky)
            for (size_t kx = 0; kx < s2[0].size(); ++kx) {
                if (kx == 0 && ky == 0 && kz == 0) continue;
                const double x = 4.0 * d.r * (s2[0][kx] + s2[1][ky] + s2[2][kz]);
                if (x >= 2.0) return HUGE_VAL;
                sum += mult[0][kx] * mult[1][ky] * mult[2][kz] * (1.0 - s2[0][kx]) / (1.0 - 0.5 * x);
            }
    return sum / (static_cast<double>(d.n[0]) * d.n[1] * d.n[2]);
}

size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

// Memory plan: a list of (pointer slot, bytes); carved in order from one block.
struct Plan {
    std::vector<std::pair<void **, size_t>> items;
    size_t total = 0;
    void add(void **slot, size_t bytes)
    {
        items.emplace_back(slot, bytes);
        total += align256(bytes);
    }
    void carve(char *base)
    {
        size_t off = 0;
        for (auto &it : items) {
            *it.first = it.second ? base + off : nullptr;
            off += align256(it.second);
        }
    }
};

she_status validate(const she_config *cfg, she_handle *h)
{
    if (!cfg) return fail(nullptr, SHE_EINVAL, "config is NULL");
    if (cfg->n_instances < 1 || !cfg->inst) return fail(nullptr, SHE_EINVAL, "need at least one instance");
    if (cfg->precision != SHE_F32 && cfg->precision != SHE_F64)
        return fail(nullptr, SHE_EINVAL, "precision must be SHE_F32 or SHE_F64");
    if (cfg->sample_every < 1) return fail(nullptr, SHE_EINVAL, "sample_every must be >= 1");
    if (cfg->burn_in < 0) return fail(nullptr, SHE_EINVAL, "burn_in must be >= 0");
    if (cfg->tuning_flags & ~(SHE_TUNE_XCD_ORDER | SHE_TUNE_SEARCH | SHE_TUNE_SINGLE_STEP))
        return fail(nullptr, SHE_EINVAL, "unknown tuning_flags bits");
    if ((cfg->tuning_flags & SHE_TUNE_SEARCH) && cfg->arena)
        return fail(nullptr, SHE_EINVAL, "SHE_TUNE_SEARCH allocates trial handles: tune with she_tune, then "
                                         "size the arena for the tuned configuration");
    if (cfg->graph_steps < 0 || cfg->graph_steps > (1 << 16))
        return fail(nullptr, SHE_EINVAL, "graph_steps must be in [0, 65536]");
    if (cfg->flags & ~static_cast<uint32_t>(SHE_ALLOW_UNSTABLE)) return fail(nullptr, SHE_EINVAL, "unknown flags bits");
    if (cfg->batch_samples < 0) return fail(nullptr, SHE_EINVAL, "batch_samples must be >= 0");
    if (cfg->batch_samples > 0 && cfg->stats_mask == 0)
        return fail(nullptr, SHE_EINVAL, "batch_samples needs statistics (stats_mask != 0)");
    if (cfg->stats_mask & ~0x1Fu) return fail(nullptr, SHE_EINVAL, "unknown stats_mask bits");
    if (cfg->stats_mask & SHE_STAT_TCORR) {
        if (cfg->inst[0].dim != 1) return fail(nullptr, SHE_EUNSUPPORTED, "SHE_STAT_TCORR is provided for 1D");
        if (cfg->tcorr_lags < 1 || cfg->tcorr_lags > 1024)
            return fail(nullptr, SHE_EINVAL, "tcorr_lags must be in [1, 1024] with SHE_STAT_TCORR");
    } else if (cfg->tcorr_lags != 0) {
        return fail(nullptr, SHE_EINVAL, "tcorr_lags must be 0 without SHE_STAT_TCORR");
    }
    const int dim = cfg->inst[0].dim;
    double beta_r = -1.0, beta_v = 0.0;     // last fe_beta: instances of a batch often share r and n
    int beta_n[3] = {0, 0, 0};
    for (int i = 0; i < cfg->n_instances; ++i) {
        const she_instance_desc &d = cfg->inst[i];
        char buf[160];
        std::snprintf(buf, sizeof buf, "instance %d: ", i);
        const std::string pre(buf);
        if (d.dim != dim) return fail(nullptr, SHE_EINVAL, pre + "all instances must have the same dim");
        if (d.dim < 1 || d.dim > 3) return fail(nullptr, SHE_EINVAL, pre + "dim must be 1, 2 or 3");
        for (int a = 0; a < 3; ++a) {
            if (a < d.dim && d.n[a] < 1) return fail(nullptr, SHE_EINVAL, pre + "cell counts must be >= 1");
            if (a >= d.dim && d.n[a] != 1) return fail(nullptr, SHE_EINVAL, pre + "unused axes must have n = 1");
        }
        if (d.eq != SHE_HEAT && d.eq != SHE_SPECIES && d.eq != SHE_BURGERS)
            return fail(nullptr, SHE_EINVAL, pre + "bad equation");
        if (!std::isfinite(d.nu) || (d.nu != 0.0 && d.eq != SHE_BURGERS))
            return fail(nullptr, SHE_EINVAL, pre + "nu must be finite, and 0 unless eq = SHE_BURGERS");
        if (d.eq == SHE_BURGERS) {
            if (d.dim != 1) return fail(nullptr, SHE_EUNSUPPORTED, pre + "SHE_BURGERS is provided for 1D");
            if (d.cond || d.cap) return fail(nullptr, SHE_EUNSUPPORTED, pre + "SHE_BURGERS with cond / cap");
            if (burgers_growth(d.r, d.nu, d.scheme) > 1.0 + 1e-12)
                return fail(nullptr, SHE_EUNSTABLE, pre + "Burgers step amplifies a mode (reduce nu or r)");
        }
        if (d.bc != SHE_PERIODIC && d.bc != SHE_DIRICHLET) return fail(nullptr, SHE_EINVAL, pre + "bad boundary");
        if (d.scheme < SHE_EM || d.scheme > SHE_CN) return fail(nullptr, SHE_EINVAL, pre + "bad scheme");
        const bool implicit = d.scheme == SHE_BE || d.scheme == SHE_CN;
        if (implicit && (d.dim != 1 || d.eq == SHE_BURGERS))
            return fail(nullptr, SHE_EUNSUPPORTED, pre + "implicit schemes are provided for 1D heat / species");
        if (implicit && d.bc == SHE_PERIODIC && d.n[0] < 3)
            return fail(nullptr, SHE_EINVAL, pre + "implicit periodic rods need N >= 3");
        if (d.noise < 0 || d.noise > 2) return fail(nullptr, SHE_EINVAL, pre + "bad noise mode");
        if (d.reserved != 0) return fail(nullptr, SHE_EINVAL, pre + "reserved field must be 0");
        if (!(d.r >= 0.0) || !(d.eps >= 0.0) || !(d.init_sd >= 0.0) || !std::isfinite(d.u0) ||
            !std::isfinite(d.u_left) || !std::isfinite(d.u_right))
            return fail(nullptr, SHE_EINVAL, pre + "r, eps, init_sd must be >= 0 and values finite");
        if (!implicit && d.r > 0.5 / d.dim)
            return fail(nullptr, SHE_EUNSTABLE, pre + "r above the explicit stability limit 1/(2 dim)");
        if (d.eq == SHE_HEAT && d.scheme == SHE_EM && d.bc == SHE_PERIODIC && d.noise == SHE_NOISE_INSTANT &&
            d.eps > 0.0 && !d.cond && !d.cap && !(cfg->flags & SHE_ALLOW_UNSTABLE)) {
            if (d.r != beta_r || d.n[0] != beta_n[0] || d.n[1] != beta_n[1] || d.n[2] != beta_n[2]) {
                beta_v = fe_beta(d);
                beta_r = d.r;
                for (int a = 0; a < 3; ++a) beta_n[a] = d.n[a];
            }
            const double eb = d.eps * beta_v;
            if (!(eb < 1.0)) {
                char buf[200];
                std::snprintf(buf, sizeof buf,
                              "eps * beta = %.4g >= 1: the second moment of the FE scheme with instantaneous "
                              "noise grows without bound (SHE_ALLOW_UNSTABLE to run it anyway)", eb);
                return fail(nullptr, SHE_EUNSTABLE, pre + buf);
            }
        }
        if (d.bc == SHE_DIRICHLET && d.dim != 1)
            return fail(nullptr, SHE_EINVAL, pre + "Dirichlet walls are provided in 1D only");
        // the 2D predictor-corrector march reads two rows beyond its chunk and
        // the 3D march one plane beyond the next: the periodic wrap of one
        // period must reach them
        if (d.dim == 2 && d.scheme == SHE_HEUN && d.n[1] < 3)
            return fail(nullptr, SHE_EUNSUPPORTED, pre + "2D predictor-corrector needs n[1] >= 3");
        if (d.dim == 3 && d.n[2] < 2) return fail(nullptr, SHE_EUNSUPPORTED, pre + "3D needs n[2] >= 2");
        if (d.bc == SHE_PERIODIC && d.u_left != d.u_right)
            return fail(nullptr, SHE_EINVAL, pre + "a wall gradient needs Dirichlet walls, not periodic");
        if (d.dim == 1 && d.bc == SHE_PERIODIC && d.n[0] < 2)
            return fail(nullptr, SHE_EINVAL, pre + "periodic 1D needs N >= 2");
        if (d.cond || d.cap) {
            if (d.dim != 1) return fail(nullptr, SHE_EUNSUPPORTED, pre + "cond / cap are provided for 1D rods");
            for (int c = 0; c < d.n[0]; ++c)
                if ((d.cond && !(d.cond[c] > 0.0 && std::isfinite(d.cond[c]))) ||
                    (d.cap && !(d.cap[c] > 0.0 && std::isfinite(d.cap[c]))))
                    return fail(nullptr, SHE_EINVAL, pre + "cond / cap must be finite and > 0");
            if (d.noise == SHE_NOISE_FROZEN && d.u_left != d.u_right)
                return fail(nullptr, SHE_EUNSUPPORTED,
                            pre + "deterministic face values on a composite rod need u_left == u_right");
            if (!implicit && varc_row_bound(d) > 2.0)
                return fail(nullptr, SHE_EUNSTABLE, pre + "composite rod above the explicit stability limit");
        }
    }
    (void)h;
    return SHE_OK;
}

}  // namespace

// ------------------------------------------------------------------ create

// Instances take whole waves (as many as they have Philox blocks, up to the
// workgroup) and are packed first-fit, largest first, into workgroups of
// block / 64 waves and at most 64 KB of LDS.  Returns an error text, or null.
static const char *pack_1d(const std::vector<Inst1D> &tab, int block, int32_t es, int mode,
                           std::vector<Seg1D> &segs, int &n_blocks, size_t &smem, int cus)
{
    const int W = block / 64;
    constexpr int kLdsCap = 64 * 1024;
    const int n_inst = static_cast<int>(tab.size());
    std::vector<int> nw(n_inst), bytes(n_inst), idx(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const int n = tab[i].n, nf = tab[i].bc == SHE_DIRICHLET ? n + 1 : n;
        const int nfg = (nf + 3) / 4;
        nw[i] = std::min(W, (nfg + 63) / 64);
        bytes[i] = seg_lds(n, nf, es, mode).total;
        if (bytes[i] > kLdsCap) return "1D instance too large for LDS (64 KB per workgroup)";
        idx[i] = i;
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        if (nw[a] != nw[b]) return nw[a] > nw[b];
        const int64_t wa = static_cast<int64_t>(tab[a].n) * (1 + tab[a].scheme);
        const int64_t wb = static_cast<int64_t>(tab[b].n) * (1 + tab[b].scheme);
        return wa > wb;
    });
    std::vector<int> used_w, used_b;
    segs.clear();
    for (int i : idx) {
        size_t bin = 0;
        while (bin < used_w.size() && (used_w[bin] + nw[i] > W || used_b[bin] + bytes[i] > kLdsCap)) ++bin;
        if (bin == used_w.size()) {
            used_w.push_back(0);
            used_b.push_back(0);
            segs.resize(segs.size() + W, Seg1D{-1, 0, 0, 0});
        }
        for (int w = 0; w < nw[i]; ++w) segs[bin * W + used_w[bin] + w] = Seg1D{i, used_w[bin], nw[i], used_b[bin]};
        used_w[bin] += nw[i];
        used_b[bin] += bytes[i];
    }
    n_blocks = static_cast<int>(used_w.size());
    smem = static_cast<size_t>(*std::max_element(used_b.begin(), used_b.end()));
    // Between one and two workgroups per CU: workgroup p and p + C (C CUs)
    // are dispatched to the same CU, so the order pairs loads.  The heaviest
    // workgroups (work ~ cells x stages per step) run alone, and the others
    // go in pairs of a heavier with a lighter one.  Measured on the
    // 1000-rod batch of log-uniform lengths (64..4096, FE and PC): 2.03-2.10
    // against 2.16-2.17 us per step in packing order.
    if (n_blocks > cus && n_blocks <= 2 * cus) {
        std::vector<int64_t> wt(n_blocks, 0);
        for (int b = 0; b < n_blocks; ++b)
            for (int w = 0; w < W; ++w) {
                const Seg1D &sg = segs[static_cast<size_t>(b) * W + w];
                if (sg.inst >= 0 && sg.w0 == w) wt[b] += static_cast<int64_t>(tab[sg.inst].n) * (1 + tab[sg.inst].scheme);
            }
        std::vector<int> ord(n_blocks);
        for (int b = 0; b < n_blocks; ++b) ord[b] = b;
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return wt[a] > wt[b]; });
        const int pairs = n_blocks - cus, singles = cus - pairs;
        std::vector<int> pos(n_blocks);
        for (int k = 0; k < singles; ++k) pos[pairs + k] = ord[k];        // alone on their CU
        for (int k = 0; k < pairs; ++k) pos[k] = ord[singles + k];        // heavier of a pair
        for (int k = 0; k < pairs; ++k) pos[cus + k] = ord[n_blocks - 1 - k];  // lighter partner
        std::vector<Seg1D> moved(segs.size());
        for (int p = 0; p < n_blocks; ++p)
            for (int w = 0; w < W; ++w)
                moved[static_cast<size_t>(p) * W + w] = segs[static_cast<size_t>(pos[p]) * W + w];
        segs.swap(moved);
    }
    return nullptr;
}

// Compute units of the current device (the planner also runs without one:
// then 256, MI355X's count).
static int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
        (void)hipGetLastError();
        return 256;
    }
    return cus;
}

static she_status plan_1d(she_handle *h, const she_config *cfg, Plan &plan)
{
    const size_t es = h->esz;
    h->tab.resize(h->n_inst);
    int64_t off = 0, xo = 0, co = 0;
    int nfg_max = 0;
    const bool corr = (h->mask & SHE_STAT_CORR) != 0;
    const bool tcorr = (h->mask & SHE_STAT_TCORR) != 0;
    int64_t cells = 0;
    for (int i = 0; i < h->n_inst; ++i) cells += h->inst[i].n[0];
    if (tcorr) {
        // samples per launch: up to 4096, fewer for large batches (ring <= ~4 Mi
        // cells x samples), plus the L - 1 older rows the lags reach back to
        h->tc_lags = cfg->tcorr_lags;
        const int64_t per = std::max<int64_t>(64, std::min<int64_t>(4096, (int64_t(1) << 22) / std::max<int64_t>(1, cells)));
        h->hist_rows = static_cast<int32_t>(per + h->tc_lags);
    }
    int64_t ho = 0, to = 0;
    std::map<std::vector<double>, std::pair<int64_t, int32_t>> pcr_shared;  // matrix rows -> factor block
    for (int i = 0; i < h->n_inst; ++i) {
        const she_instance_desc &d = h->inst[i];
        Inst1D &t = h->tab[i];
        t.off = off;
        t.n = d.n[0];
        t.bc = d.bc;
        t.scheme = d.scheme;
        t.noise = d.noise;
        t.eq = d.eq;
        t.realisation = d.realisation;
        t.seed = d.seed;
        t.r = d.r;
        t.sigma = std::sqrt(2.0 * d.r * d.eps);
        t.u0 = d.u0;
        t.uL = d.bc == SHE_DIRICHLET ? d.u_left : d.u0;
        t.uR = d.bc == SHE_DIRICHLET ? d.u_right : d.u0;
        t.nu = d.nu;
        if (corr) {
            if (d.n[0] > 1024) return fail(nullptr, SHE_EUNSUPPORTED, "SHE_STAT_CORR needs N <= 1024");
            t.x_off = xo;
            t.c_off = co;
            xo += static_cast<int64_t>(kCorrBlock) * d.n[0];
            co += static_cast<int64_t>(d.n[0]) * d.n[0];
        } else {
            t.x_off = -1;
            t.c_off = -1;
        }
        if (d.cond || d.cap) {
            // r_f, s_f (wall faces with their sqrt 2), w_i
            const std::vector<double> lf = face_conductivity(d);
            const int nf = static_cast<int>(lf.size());
            t.k_off = static_cast<int64_t>(h->coef_host.size());
            for (int f = 0; f < nf; ++f) h->coef_host.push_back(d.r * lf[f]);
            for (int f = 0; f < nf; ++f) {
                const bool wall = d.bc == SHE_DIRICHLET && (f == 0 || f == d.n[0]);
                h->coef_host.push_back(std::sqrt(2.0 * d.r * lf[f] * d.eps) * (wall ? std::sqrt(2.0) : 1.0));
            }
            for (int c = 0; c < d.n[0]; ++c) h->coef_host.push_back(d.cap ? 1.0 / d.cap[c] : 1.0);
            h->varc = true;
        } else {
            t.k_off = -1;
        }
        t.p_off = -1;
        t.pcr_levels = 0;
        t.theta = 0.0;
        if (d.scheme == SHE_BE || d.scheme == SHE_CN) {
            // M = I - theta W A; periodic: M = T + u v^T with u = (g, 0.., up_(N-1)),
            // v = (1, 0.., lo_0 / g), g = -di_0 (Sherman-Morrison), T tridiagonal
            t.theta = d.scheme == SHE_BE ? 1.0 : 0.5;
            std::vector<double> lo, di, up;
            implicit_rows(d, t.theta, lo, di, up);
            const int N = d.n[0];
            const bool per = d.bc == SHE_PERIODIC;
            // instances with the same matrix share one block of factors (the
            // reduction reads them every level; a shared block stays in L2)
            std::vector<double> key(lo);
            key.insert(key.end(), di.begin(), di.end());
            key.insert(key.end(), up.begin(), up.end());
            key.push_back(per ? 1.0 : 0.0);
            const auto hit = pcr_shared.find(key);
            if (hit != pcr_shared.end()) {
                t.p_off = hit->second.first;
                t.pcr_levels = hit->second.second;
            } else {
                const double g = -di[0], alpha = up[N - 1], beta = lo[0];
                if (per) {
                    di[0] -= g;
                    di[N - 1] -= alpha * beta / g;
                    lo[0] = 0.0;
                    up[N - 1] = 0.0;
                }
                t.p_off = static_cast<int64_t>(h->pcr_host.size());
                t.pcr_levels = pcr_factors(lo, di, up, h->pcr_host);
                if (per) {
                    std::vector<double> u(N, 0.0);
                    u[0] = g;
                    u[N - 1] = alpha;
                    const std::vector<double> z = thomas_solve(lo, di, up, u);
                    h->pcr_host.insert(h->pcr_host.end(), z.begin(), z.end());
                    const double q = beta / g;
                    h->pcr_host.push_back(q);
                    h->pcr_host.push_back(1.0 / (1.0 + z[0] + q * z[N - 1]));
                }
                pcr_shared.emplace(std::move(key), std::make_pair(t.p_off, t.pcr_levels));
            }
        }
        if (tcorr) {
            t.h_off = ho;
            t.tc_off = to;
            ho += static_cast<int64_t>(h->hist_rows) * d.n[0];
            to += static_cast<int64_t>(h->tc_lags) * d.n[0];
        } else {
            t.h_off = -1;
            t.tc_off = -1;
        }
        off += d.n[0];
        h->nmax = std::max(h->nmax, d.n[0]);
        const int nf = d.bc == SHE_DIRICHLET ? d.n[0] + 1 : d.n[0];
        nfg_max = std::max(nfg_max, (nf + 3) / 4);
    }
    h->total_cells = off;
    h->x_elems = xo;
    h->c_elems = co;
    h->hist_elems = ho;
    h->tc_elems = to;
    // Launch shape: threads per workgroup and Philox blocks per thread.  Auto:
    // the smallest shape whose workgroup holds the largest instance with at
    // most one block per thread up to 512 threads (64 x 1, 64 x 2, 256 x 1,
    // 512 x 1), then 512 threads with 2 or 4 blocks each.
    bool heat_only = true;
    for (int i = 0; i < h->n_inst; ++i)
        heat_only = heat_only && h->tab[i].eq == SHE_HEAT && h->tab[i].noise == SHE_NOISE_INSTANT;
    const int mode = !h->pcr_host.empty() ? 2 : (h->varc ? 1 : (heat_only ? 3 : 0));
    h->mode1d = mode;
    // A uniform explicit FP32 batch of heat instances with instantaneous noise
    // and no statistics whose largest instance has 513..1024 blocks may take
    // 1024 threads with one block each (a kernel compiled for that face path
    // only, 38 VGPRs, two workgroups per CU).
    const bool wide_ok = h->prec == SHE_F32 && mode == 3 && h->mask == 0;
    int block = cfg->block_threads, maxg = 1;
    if (block == 0) {
        if (nfg_max <= 64) block = 64;
        else if (nfg_max <= 128) block = 64, maxg = 2;
        else if (nfg_max <= 256) block = 256;
        else if (nfg_max <= 512) block = 512;
        else block = 512, maxg = nfg_max <= 1024 ? 2 : 4;
        if (wide_ok && nfg_max > 512 && nfg_max <= 1024) {
            // 1024 x 1 halves the largest instances' chain, but its workgroups
            // are resident together only up to one per CU (measured: a c4-like
            // batch of 282 such workgroups ran slower than 471 of 512 x 2)
            std::vector<Seg1D> sg;
            int nb = 0;
            size_t sm = 0;
            const int cus = device_cus();
            if (!pack_1d(h->tab, 1024, static_cast<int32_t>(es), mode, sg, nb, sm, cus) && nb <= cus)
                block = 1024, maxg = 1;
        }
    } else {
        if (block != 64 && block != 256 && block != 512 && !(block == 1024 && wide_ok))
            return fail(nullptr, SHE_EINVAL,
                        "block_threads must be 0, 64, 256, 512, or 1024 (FP32 heat with instantaneous noise, "
                        "uniform material, explicit, no statistics)");
        const int g = (nfg_max + block - 1) / block;
        while (maxg < g) maxg *= 2;
    }
    if (maxg > (block == 512 ? 4 : (block == 1024 ? 1 : 2)))
        return fail(nullptr, SHE_EUNSUPPORTED, "1D instance too large for the resident kernel at this block size");
    h->block1d = block;
    h->maxg = maxg;
    {
        const char *why =
            pack_1d(h->tab, block, static_cast<int32_t>(es), mode, h->segs_host, h->blocks1d, h->smem1d, device_cus());
        if (why) return fail(nullptr, SHE_EUNSUPPORTED, why);
    }

    plan.add(reinterpret_cast<void **>(&h->d_tab), sizeof(Inst1D) * h->n_inst);
    plan.add(reinterpret_cast<void **>(&h->d_segs), sizeof(Seg1D) * h->segs_host.size());
    plan.add(&h->d_pool, es * off);
    if (h->mask & (SHE_STAT_MOMENTS | SHE_STAT_CORR | SHE_STAT_TCORR)) {
        plan.add(reinterpret_cast<void **>(&h->d_s1), sizeof(double) * off);
        plan.add(reinterpret_cast<void **>(&h->d_s2), sizeof(double) * off);
    }
    if (corr) {
        plan.add(&h->d_x, es * xo);
        plan.add(reinterpret_cast<void **>(&h->d_c), sizeof(double) * co);
    }
    if (!h->coef_host.empty()) plan.add(&h->d_coef, es * h->coef_host.size());
    if (!h->pcr_host.empty()) plan.add(reinterpret_cast<void **>(&h->d_pcr), sizeof(double) * h->pcr_host.size());
    if (tcorr) {
        plan.add(&h->d_hist, es * ho);
        plan.add(reinterpret_cast<void **>(&h->d_tc), sizeof(double) * to);
    }
    if (h->batch_len > 0 && h->d_s1_planned()) {
        plan.add(reinterpret_cast<void **>(&h->d_bcell), sizeof(double) * 6 * off);
        if (corr) {
            plan.add(reinterpret_cast<void **>(&h->d_csnap), sizeof(double) * co);
            plan.add(reinterpret_cast<void **>(&h->d_skw1), sizeof(double) * 2 * off);
        }
    }
    h->fin_len = 4 * static_cast<size_t>(h->nmax) + 2 * static_cast<size_t>(h->nmax) * h->nmax + 8 +
                 static_cast<size_t>(h->tc_lags) * h->nmax;
    return SHE_OK;
}

static she_status plan_nd(she_handle *h, const she_config *cfg, Plan &plan)
{
    const she_instance_desc &d0 = h->inst[0];
    for (int i = 1; i < h->n_inst; ++i) {
        const she_instance_desc &d = h->inst[i];
        if (d.n[0] != d0.n[0] || d.n[1] != d0.n[1] || d.n[2] != d0.n[2] || d.eq != d0.eq || d.scheme != d0.scheme ||
            d.noise != d0.noise || d.seed != d0.seed)
            return fail(nullptr, SHE_EUNSUPPORTED,
                        "2D/3D batches must share the grid, equation, scheme, noise mode and seed "
                        "(r, u0, eps, init_sd and the realisation may differ)");
    }
    const int nx = d0.n[0];
    if (!is_pow2(nx) || nx < 8 || nx > 1024)
        return fail(nullptr, SHE_EUNSUPPORTED, "2D/3D kernels need n[0] a power of two in [8, 1024]");
    if (h->mask & (SHE_STAT_CORR | SHE_STAT_MOMENTS))
        return fail(nullptr, SHE_EUNSUPPORTED, "2D/3D statistics are SHE_STAT_SPATIAL (and SHE_STAT_SK)");
    if (h->mask & SHE_STAT_SK) {
        if (d0.dim != 2 || !is_pow2(d0.n[1]) || d0.n[1] < 2 || d0.n[1] > 1024)
            return fail(nullptr, SHE_EUNSUPPORTED,
                        "SHE_STAT_SK is provided for 2D grids with n[1] a power of two in [2, 1024]");
        h->mask |= SHE_STAT_SPATIAL;
    }
    int cx = 4;
    while (nx / cx > 64) cx *= 2;
    h->cx = cx;
    const int LX = nx / cx;
    ParamsND &p = h->pnd;
    p.nx = nx;
    p.ny = d0.n[1];
    p.nz = d0.n[2];
    p.dim = d0.dim;
    p.eq = d0.eq;
    p.scheme = d0.scheme;
    p.noise = d0.noise;
    p.n_inst = h->n_inst;
    p.xcd_order = (cfg->tuning_flags & SHE_TUNE_XCD_ORDER) ? 1 : 0;
    p.seed = d0.seed;
    h->ip_host.resize(h->n_inst);
    for (int i = 0; i < h->n_inst; ++i) {
        const she_instance_desc &d = h->inst[i];
        const double sigma = std::sqrt(2.0 * d.r * d.eps);
        InstND &q = h->ip_host[i];
        if (d.noise == SHE_NOISE_FROZEN)
            q.ns = sigma * (d.eq == SHE_HEAT ? d.u0 : std::sqrt(std::max(d.u0, 0.0)));
        else if (d.noise == SHE_NOISE_INSTANT)
            q.ns = d.eq == SHE_HEAT ? 0.5 * sigma : sigma * std::sqrt(0.5);
        else
            q.ns = 0.0;
        q.init_sd = d.init_sd;
        q.r = d.r;
        q.u0 = d.u0;
        q.realisation = d.realisation;
        q.pad = 0;
    }
    h->cells = static_cast<int64_t>(p.nx) * p.ny * p.nz;
    if (d0.dim == 2) {
        // Default march length.  FE: about 16384 row groups in flight, 1..8 rows
        // each (short marches keep more loads in flight; the halo row a chunk
        // re-reads mostly hits the cache).  PC recomputes three rows per chunk
        // and its kernel holds three waves per SIMD, so it takes as few groups
        // as fill that once, 12 per CU, of up to 64 rows.  Measured at
        // 512 x 512 x 256 (ms per step without statistics): 43 rows (3072
        // groups, one round) 0.1222; 32 rows (4096) 0.1263; 64 rows 0.1238;
        // 40 rows (3328, a short second round) 0.1422.
        int chunk = cfg->rows_per_block;
        const int64_t rows_all = static_cast<int64_t>(h->n_inst) * p.ny;
        if (chunk <= 0) {
            const int64_t pc_groups = 12 * static_cast<int64_t>(device_cus());
            chunk = d0.scheme == SHE_EM
                        ? static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(8, rows_all / 16384)))
                        : static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(64, (rows_all + pc_groups - 1) /
                                                                                             pc_groups)));
        }
        chunk = std::min(chunk, p.ny);
        p.chunk = chunk;
        const int nchunks = (p.ny + chunk - 1) / chunk;
        h->nparts = nchunks;
        const int gpb = 256 / LX;
        h->nd_blocks = (h->n_inst * nchunks + gpb - 1) / gpb;
    } else {
        if (d0.scheme != SHE_EM && d0.scheme != SHE_HEUN)
            return fail(nullptr, SHE_EUNSUPPORTED, "3D provides the FE and PC schemes");
        int ty = cfg->rows_per_group;
        if (ty == 0) {
            ty = 1;
            for (int c = 1; c <= p.ny; ++c)
                if (p.ny % c == 0 && LX * c <= 256) ty = c;
        }
        if (ty < 1 || p.ny % ty != 0 || LX * ty > 256)
            return fail(nullptr, SHE_EINVAL, "rows_per_group must divide n[1] with (n[0]/cx)*rows <= 256");
        h->ty = ty;
        int chunk = cfg->rows_per_block > 0 ? cfg->rows_per_block : 8;
        chunk = std::min(chunk, p.nz);
        p.chunk = chunk;
        const int nzc = (p.nz + chunk - 1) / chunk;
        h->nparts = (p.ny / ty) * nzc;
        h->nd_blocks = h->n_inst * h->nparts;
        h->smem3d = std::max(4 * static_cast<size_t>(ty) * nx * h->esz, 2 * sizeof(double) * ty);
        if (h->smem3d > 64 * 1024) return fail(nullptr, SHE_EUNSUPPORTED, "3D tile exceeds 64 KB of LDS");
    }
    const size_t es = h->esz;
    const size_t fbytes = es * static_cast<size_t>(h->cells) * h->n_inst;
    plan.add(&h->d_a, fbytes);
    plan.add(&h->d_b, fbytes);
    if (d0.dim == 3 && d0.scheme == SHE_HEUN) plan.add(&h->d_pred, fbytes);
    plan.add(reinterpret_cast<void **>(&h->d_ip), sizeof(InstND) * h->n_inst);
    plan.add(reinterpret_cast<void **>(&h->d_part), 2 * sizeof(double) * h->nparts * h->n_inst);
    plan.add(reinterpret_cast<void **>(&h->d_step), sizeof(int64_t));
    h->graph_steps = cfg->graph_steps;
    h->fin_len = 8;
    if (h->mask & SHE_STAT_SK) {
        // shells round(|k|), signed k in [-N/2, N/2); mode counts per shell
        const double kmax = std::sqrt(0.25 * nx * nx + 0.25 * p.ny * p.ny);
        h->nbins = static_cast<int>(std::floor(kmax + 0.5)) + 1;
        h->skmodes.assign(h->nbins, 0.0);
        for (int ky = 0; ky < p.ny; ++ky)
            for (int kx = 0; kx < nx; ++kx) {
                const double sx = 2 * kx < nx ? kx : kx - nx, sy = 2 * ky < p.ny ? ky : ky - p.ny;
                const int b = static_cast<int>(std::floor(std::sqrt(sx * sx + sy * sy) + 0.5));
                if (b < h->nbins) h->skmodes[b] += 1.0;
            }
        h->sk_groups = sk2d_groups(h->prec, nx, p.ny, h->n_inst);
        const int ltc = half_tile_log2(h->prec, p.ny);
        plan.add(&h->d_half, 2 * es * (static_cast<size_t>(half_tiles(nx, ltc)) << ltc) * p.ny * h->n_inst);
        plan.add(&h->d_twx, 2 * es * nx);
        plan.add(&h->d_twy, 2 * es * p.ny);
        plan.add(reinterpret_cast<void **>(&h->d_shells),
                 sizeof(uint16_t) * static_cast<size_t>(nx / 2 + 1) * (h->nbins + 1));
        plan.add(reinterpret_cast<void **>(&h->d_skpart), sizeof(double) * h->n_inst * h->sk_groups * h->nbins);
        plan.add(reinterpret_cast<void **>(&h->d_sksum), sizeof(double) * h->n_inst * h->nbins);
        plan.add(reinterpret_cast<void **>(&h->d_skmodes), sizeof(double) * h->nbins);
        if (h->batch_len > 0) {
            const size_t nb = sizeof(double) * h->n_inst * h->nbins;
            plan.add(reinterpret_cast<void **>(&h->d_sksnap), nb);
            plan.add(reinterpret_cast<void **>(&h->d_skwm), nb);
            plan.add(reinterpret_cast<void **>(&h->d_skwm2), nb);
        }
        h->fin_len = 3 + h->nbins;
    }
    return SHE_OK;
}

static she_status build_plan(she_handle *h, const she_config *cfg, Plan &plan)
{
    h->dim = cfg->inst[0].dim;
    h->prec = cfg->precision;
    h->esz = cfg->precision == SHE_F32 ? 4 : 8;
    h->n_inst = cfg->n_instances;
    h->inst.assign(cfg->inst, cfg->inst + cfg->n_instances);
    h->burn_in = cfg->burn_in;
    h->every = cfg->sample_every;
    h->mask = cfg->stats_mask;
    if (h->mask & (SHE_STAT_CORR | SHE_STAT_TCORR)) h->mask |= SHE_STAT_MOMENTS;
    h->batch_len = cfg->batch_samples;
    h->stream = static_cast<hipStream_t>(cfg->stream);
    she_status st = h->dim == 1 ? plan_1d(h, cfg, plan) : plan_nd(h, cfg, plan);
    for (she_instance_desc &d : h->inst) d.cond = d.cap = nullptr;  // caller memory, read during planning only
    if (st != SHE_OK) return st;
    if (h->dim == 2 && h->pnd.scheme == SHE_EM && h->pnd.ny >= 3 && !(cfg->tuning_flags & SHE_TUNE_SINGLE_STEP)) {
        // Two FE steps per launch (n[1] >= 3: the march reads two rows beyond
        // its chunk).  Each march chunk recomputes the intermediate rows on
        // both sides of it, so the chunks are longer: about 2048 of up to 32
        // rows.  Measured on 512 x 512 fields, ms per step, one step per launch
        // vs two: 256 realisations 0.1113 vs 0.0855, 64: 0.0326 vs 0.0232,
        // 16: 0.0131 vs 0.0090, 1: 0.0041 vs 0.0033.  Never shorter than
        // the one-step chunks, whose partials buffer this reuses.
        const ParamsND &p = h->pnd;
        const int64_t rows_all = static_cast<int64_t>(h->n_inst) * p.ny;
        const int c2 = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(32, rows_all / 2048)));
        h->chunk2 = std::min(std::max(c2, p.chunk), p.ny);
        h->nparts2 = (p.ny + h->chunk2 - 1) / h->chunk2;
        const int gpb = 256 / (p.nx / h->cx);
        h->nd_blocks2 = (h->n_inst * h->nparts2 + gpb - 1) / gpb;
        h->two_step = true;
        if ((h->mask & SHE_STAT_SK) && sk_rows_fusable(h->prec, p.nx) && p.ny % 2 == 0) {
            // row pairs must not straddle march chunks
            h->chunk2 += h->chunk2 & 1;
            h->nparts2 = (p.ny + h->chunk2 - 1) / h->chunk2;
            h->nd_blocks2 = (h->n_inst * h->nparts2 + gpb - 1) / gpb;
            h->sk_fused = true;
        }
    }
    plan.add(reinterpret_cast<void **>(&h->d_acc), sizeof(InstAcc) * h->n_inst);
    plan.add(reinterpret_cast<void **>(&h->d_init_sd), sizeof(double) * h->n_inst);
    plan.add(reinterpret_cast<void **>(&h->d_fin), sizeof(double) * h->fin_len);
    return SHE_OK;
}

extern "C" she_status she_arena_bytes(const she_config *cfg, size_t *bytes)
{
    if (!bytes) return fail(nullptr, SHE_EINVAL, "bytes is NULL");
    she_status st = validate(cfg, nullptr);
    if (st != SHE_OK) return st;
    she_handle tmp;
    Plan plan;
    st = build_plan(&tmp, cfg, plan);
    if (st != SHE_OK) return st;
    *bytes = plan.total;
    return SHE_OK;
}

static she_status zero_stats(she_handle *h)
{
    hipStream_t s = h->stream;
    SHE_HIP(h, hipMemsetAsync(h->d_acc, 0, sizeof(InstAcc) * h->n_inst, s));
    if (h->d_s1) SHE_HIP(h, hipMemsetAsync(h->d_s1, 0, sizeof(double) * h->total_cells, s));
    if (h->d_s2) SHE_HIP(h, hipMemsetAsync(h->d_s2, 0, sizeof(double) * h->total_cells, s));
    if (h->d_x) SHE_HIP(h, hipMemsetAsync(h->d_x, 0, h->esz * h->x_elems, s));
    if (h->d_c) SHE_HIP(h, hipMemsetAsync(h->d_c, 0, sizeof(double) * h->c_elems, s));
    if (h->d_sksum) SHE_HIP(h, hipMemsetAsync(h->d_sksum, 0, sizeof(double) * h->n_inst * h->nbins, s));
    if (h->d_tc) SHE_HIP(h, hipMemsetAsync(h->d_tc, 0, sizeof(double) * h->tc_elems, s));
    if (h->d_bcell) SHE_HIP(h, hipMemsetAsync(h->d_bcell, 0, sizeof(double) * 6 * h->total_cells, s));
    if (h->d_csnap) SHE_HIP(h, hipMemsetAsync(h->d_csnap, 0, sizeof(double) * h->c_elems, s));
    if (h->d_skw1) SHE_HIP(h, hipMemsetAsync(h->d_skw1, 0, sizeof(double) * 2 * h->total_cells, s));
    for (double *p : {h->d_sksnap, h->d_skwm, h->d_skwm2})
        if (p) SHE_HIP(h, hipMemsetAsync(p, 0, sizeof(double) * h->n_inst * h->nbins, s));
    h->samples = 0;
    return SHE_OK;
}

// ------------------------------------------------------------------ autotuning

// Choices measured before in this process, keyed by what decides the launch
// shapes: precision, statistics mask, and per instance the sizes, boundary,
// scheme, equation, noise mode and whether material arrays are given.
struct TuneChoice {
    int32_t block_threads, rows_per_block, rows_per_group;
};
static std::mutex g_tune_mu;
static std::map<std::string, TuneChoice> g_tune_cache;

static std::string tune_key(const she_config *cfg)
{
    std::string k;
    char buf[128];
    std::snprintf(buf, sizeof buf, "p%d m%u f%d|", cfg->precision, cfg->stats_mask,
                  cfg->tuning_flags & (SHE_TUNE_XCD_ORDER | SHE_TUNE_SINGLE_STEP));
    k += buf;
    for (int i = 0; i < cfg->n_instances; ++i) {
        const she_instance_desc &d = cfg->inst[i];
        std::snprintf(buf, sizeof buf, "%d:%dx%dx%d:%d%d%d%d%d;", d.dim, d.n[0], d.n[1], d.n[2], d.bc, d.scheme, d.eq,
                      d.noise, (d.cond || d.cap) ? 1 : 0);
        k += buf;
    }
    return k;
}

extern "C" she_status she_tune(const she_config *cfg, int32_t steps, she_config *tuned)
{
    if (!tuned) return fail(nullptr, SHE_EINVAL, "tuned is NULL");
    she_status st = validate(cfg, nullptr);
    if (st != SHE_OK) return st;
    *tuned = *cfg;
    tuned->tuning_flags &= ~SHE_TUNE_SEARCH;
    const std::string key = tune_key(cfg);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        const auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            tuned->block_threads = it->second.block_threads;
            tuned->rows_per_block = it->second.rows_per_block;
            tuned->rows_per_group = it->second.rows_per_group;
            return SHE_OK;
        }
    }
    const int dim = cfg->inst[0].dim;
    std::vector<TuneChoice> cand;
    if (dim == 1) {
        for (int b : {64, 256, 512, 1024}) cand.push_back({b, cfg->rows_per_block, cfg->rows_per_group});
    } else if (dim == 2) {
        for (int c : {4, 8, 16, 32, 64}) cand.push_back({cfg->block_threads, c, cfg->rows_per_group});
    } else {
        for (int c : {4, 8, 16})
            for (int g : {1, 2, 4, 8}) cand.push_back({cfg->block_threads, c, g});
    }
    if (steps <= 0) steps = dim == 1 ? 2000 : 20;
    hipStream_t s = static_cast<hipStream_t>(cfg->stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(nullptr, SHE_EDEVICE, "she_tune: hipEventCreate failed");
    }
    double best = 1e300;
    TuneChoice pick{};
    bool any = false;
    for (const TuneChoice &c : cand) {
        she_config t = *tuned;
        t.block_threads = c.block_threads;
        t.rows_per_block = c.rows_per_block;
        t.rows_per_group = c.rows_per_group;
        t.arena = nullptr;
        t.arena_bytes = 0;
        she_handle *h = nullptr;
        if (she_create(&t, &h) != SHE_OK) continue;  // shape not valid for this batch
        float ms = 0.0f;
        const bool ok = she_step(h, std::max(1, steps / 4)) == SHE_OK && hipEventRecord(e0, s) == hipSuccess &&
                        she_step(h, steps) == SHE_OK && hipEventRecord(e1, s) == hipSuccess &&
                        hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        she_destroy(h);
        if (ok && ms < best) {
            best = ms;
            pick = c;
            any = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!any) return fail(nullptr, SHE_EUNSUPPORTED, "she_tune: no candidate launch shape ran for this configuration");
    tuned->block_threads = pick.block_threads;
    tuned->rows_per_block = pick.rows_per_block;
    tuned->rows_per_group = pick.rows_per_group;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = pick;
    return SHE_OK;
}

extern "C" she_status she_create(const she_config *cfg, she_handle **out)
{
    if (!out) return fail(nullptr, SHE_EINVAL, "out is NULL");
    *out = nullptr;
    she_status st = validate(cfg, nullptr);
    if (st != SHE_OK) return st;
    if (cfg->tuning_flags & SHE_TUNE_SEARCH) {
        she_config tuned;
        st = she_tune(cfg, 0, &tuned);
        if (st != SHE_OK) return st;
        return she_create(&tuned, out);
    }
    she_handle *h = new she_handle();
    Plan plan;
    st = build_plan(h, cfg, plan);
    if (st != SHE_OK) {
        delete h;
        return st;
    }
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return fail(nullptr, SHE_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    if (cfg->arena) {
        if (cfg->arena_bytes < plan.total) {
            char buf[128];
            std::snprintf(buf, sizeof buf, "arena too small: %zu bytes needed", plan.total);
            delete h;
            return fail(nullptr, SHE_ENOMEM, buf);
        }
        if (reinterpret_cast<uintptr_t>(cfg->arena) % 256 != 0) {
            delete h;
            return fail(nullptr, SHE_EINVAL, "arena must be 256-byte aligned");
        }
        h->base = static_cast<char *>(cfg->arena);
        h->own = false;
    } else {
        e = hipMalloc(reinterpret_cast<void **>(&h->base), plan.total);
        if (e != hipSuccess) {
            delete h;
            return fail(nullptr, SHE_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        h->own = true;
    }
    h->bytes = plan.total;
    plan.carve(h->base);

    hipStream_t s = h->stream;
    // host sources of the asynchronous copies below; they live until the
    // stream synchronisation at the end of creation
    std::vector<double> sd(h->n_inst);
    std::vector<float> coef32;
    for (int i = 0; i < h->n_inst; ++i) sd[i] = h->inst[i].init_sd;
#define CREATE_HIP(call)                                          \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) {                                   \
            std::string m_ = std::string(#call) + ": " + hipGetErrorString(e_); \
            she_destroy(h);                                       \
            return fail(nullptr, SHE_EDEVICE, m_);                \
        }                                                         \
    } while (0)
    CREATE_HIP(hipMemcpyAsync(h->d_init_sd, sd.data(), sizeof(double) * h->n_inst, hipMemcpyHostToDevice, s));
    if (h->dim == 1) {
        CREATE_HIP(hipMemcpyAsync(h->d_tab, h->tab.data(), sizeof(Inst1D) * h->n_inst, hipMemcpyHostToDevice, s));
        CREATE_HIP(hipMemcpyAsync(h->d_segs, h->segs_host.data(), sizeof(Seg1D) * h->segs_host.size(),
                                  hipMemcpyHostToDevice, s));
        if (!h->pcr_host.empty())
            CREATE_HIP(hipMemcpyAsync(h->d_pcr, h->pcr_host.data(), sizeof(double) * h->pcr_host.size(),
                                      hipMemcpyHostToDevice, s));
        if (!h->coef_host.empty()) {
            if (h->prec == SHE_F32) {
                coef32.assign(h->coef_host.begin(), h->coef_host.end());
                CREATE_HIP(hipMemcpyAsync(h->d_coef, coef32.data(), sizeof(float) * coef32.size(),
                                          hipMemcpyHostToDevice, s));
            } else {
                CREATE_HIP(hipMemcpyAsync(h->d_coef, h->coef_host.data(), sizeof(double) * h->coef_host.size(),
                                          hipMemcpyHostToDevice, s));
            }
        }
        CREATE_HIP(launch_init1d(h->prec, h->n_inst, h->nmax, s, h->d_tab, h->d_init_sd, h->d_pool));
    } else {
        CREATE_HIP(hipMemcpyAsync(h->d_ip, h->ip_host.data(), sizeof(InstND) * h->n_inst, hipMemcpyHostToDevice, s));
        h->pnd.ip = h->d_ip;
        if (h->d_skmodes) {
            CREATE_HIP(hipMemcpyAsync(h->d_skmodes, h->skmodes.data(), sizeof(double) * h->nbins,
                                      hipMemcpyHostToDevice, s));
            CREATE_HIP(launch_twiddles(h->prec, s, h->pnd.nx, h->d_twx));
            CREATE_HIP(launch_twiddles(h->prec, s, h->pnd.ny, h->d_twy));
            CREATE_HIP(launch_shell_table(s, h->pnd.nx, h->pnd.ny, h->nbins, h->d_shells));
        }
        CREATE_HIP(launch_initnd(h->prec, s, h->pnd, h->cells, h->d_a));
        h->cur = 0;
    }
    // staged host copies must stay valid until the stream has consumed them
    CREATE_HIP(hipStreamSynchronize(s));
#undef CREATE_HIP
    if (zero_stats(h) != SHE_OK) {
        std::string m = h->err;
        she_destroy(h);
        return fail(nullptr, SHE_EDEVICE, m);
    }
    *out = h;
    return SHE_OK;
}

extern "C" void she_destroy(she_handle *h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    for (hipGraphExec_t &g : h->gexec)
        if (g) (void)hipGraphExecDestroy(g);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->own && h->base) (void)hipFree(h->base);
    delete h;
}

extern "C" const char *she_last_error(const she_handle *h)
{
    return h ? h->err.c_str() : g_create_err.c_str();
}

// ------------------------------------------------------------------ stepping

// Enqueue one 2D/3D step from buffer `cur` (two 2D FE steps when `two`)
// and, when it may sample, the reduction of its partials and the structure
// factor of its output.
static hipError_t nd_enqueue(she_handle *h, hipStream_t s, const StepArg &sa, int cur, bool may_sample,
                             bool two = false)
{
    const void *src = cur == 0 ? h->d_a : h->d_b;
    void *dst = cur == 0 ? h->d_b : h->d_a;
    hipError_t e;
    const bool fused = two && may_sample && h->sk_fused;
    if (two) {
        // the handle's parameters (with their device pointers) and the
        // two-step march length; on sample launches with S(k), the row
        // transforms of the new field as well
        ParamsND p2 = h->pnd;
        p2.chunk = h->chunk2;
        const int ltc = half_tile_log2(h->prec, p2.ny);
        const SkRows skr{h->d_half, h->d_twx, ltc, half_tiles(p2.nx, ltc)};
        e = launch_step2d(h->prec, h->cx, p2.eq, 2, h->nd_blocks2, s, p2, src, dst, sa, h->d_part, h->d_acc,
                          fused ? &skr : nullptr);
    }
    else if (h->dim == 2)
        e = launch_step2d(h->prec, h->cx, h->pnd.eq, h->pnd.scheme, h->nd_blocks, s, h->pnd, src, dst, sa, h->d_part,
                          h->d_acc);
    else if (h->pnd.scheme == SHE_EM)
        e = launch_step3d(h->prec, h->cx, h->pnd.eq, 0, h->ty, h->nd_blocks, h->smem3d, s, h->pnd, src, nullptr, dst,
                          sa, h->d_part, h->d_acc);
    else {
        // PC: predictor into the scratch field (no sampling), then the corrector
        StepArg pa = sa;
        pa.sample = 0;
        e = launch_step3d(h->prec, h->cx, h->pnd.eq, 0, h->ty, h->nd_blocks, h->smem3d, s, h->pnd, src, nullptr,
                          h->d_pred, pa, h->d_part, h->d_acc);
        if (e == hipSuccess)
            e = launch_step3d(h->prec, h->cx, h->pnd.eq, 1, h->ty, h->nd_blocks, h->smem3d, s, h->pnd, h->d_pred,
                              src, dst, sa, h->d_part, h->d_acc);
    }
    if (e != hipSuccess || !may_sample) return e;
    const SpatialParts sp{h->d_part, h->d_acc, 1.0 / static_cast<double>(h->cells), two ? h->nparts2 : h->nparts,
                          h->batch_len};
    // with S(k), the first column-transform block of each instance does the
    // spatial reduction (one launch fewer per sample)
    if (!(h->mask & SHE_STAT_SK))
        return launch_reduce_parts(h->n_inst, s, sa, sp.part, sp.nparts, sp.inv_cells, sp.batch_len, sp.acc);
    const BatchSk bk{h->d_sksnap, h->d_skwm, h->d_skwm2, h->d_skmodes, h->d_ip, static_cast<double>(h->cells),
                     h->d_sksnap ? h->batch_len : 0, 0};
    return launch_sk2d(h->prec, s, sa, h->n_inst, h->pnd.nx, h->pnd.ny, h->d_ip, dst, h->d_half, h->d_twx, h->d_twy,
                       h->d_shells, h->d_skpart, h->nbins, h->d_sksum, h->d_acc, bk, fused, sp);
}

// Whether completed step t samples.
static bool samples_at(const she_handle *h, bool samp, int64_t t)
{
    return samp && t > h->burn_in && t % h->every == 0;
}

// Whether a two-step launch can sample its first step: the intermediate
// field never reaches memory, so its statistics are taken in the kernel as
// its rows are formed, which S(k) allows only with the row transforms there.
// That kernel variant is compiled for FP32 states only.
static bool first_step_samples_ok(const she_handle *h)
{
    return h->prec == SHE_F32 && (!(h->mask & SHE_STAT_SK) || h->sk_fused);
}

// One direct step, or two in one launch when `pair` allows it and at most
// one of them samples (the first only where first_step_samples_ok).  The
// launch's sample flag: 1 its last step samples, 2 its first, 0 none.
static she_status nd_direct(she_handle *h, bool samp, bool pair = false)
{
    const bool s1 = samples_at(h, samp, h->steps + 1), s2 = samples_at(h, samp, h->steps + 2);
    const bool two = pair && h->two_step && !(s1 && (s2 || !first_step_samples_ok(h)));
    const int64_t t = h->steps + (two ? 2 : 1);
    const int sample = two ? (s2 ? 1 : (s1 ? 2 : 0)) : (s1 ? 1 : 0);
    const StepArg sa{h->steps, nullptr, h->burn_in, h->every, sample};
    SHE_HIP(h, nd_enqueue(h, h->stream, sa, h->cur, sample != 0, two));
    h->cur ^= 1;
    h->steps = t;
    return SHE_OK;
}

// Record K steps that start at a step index s0 = *d_step with s0 % L == 0 and
// buffer 0 current (kind 1: s0 >= burn_in, positions with (j+1) % every == 0
// sample; kind 0: none does), then *d_step += K.  Kernels of a replay read the
// counter, so one graph serves every aligned start.
static she_status record_graph(she_handle *h, int kind, int64_t K)
{
    if (h->gexec[kind]) {
        SHE_HIP(h, hipGraphExecDestroy(h->gexec[kind]));
        h->gexec[kind] = nullptr;
    }
    if (!h->cap_stream) SHE_HIP(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    SHE_HIP(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int64_t j = 0; j < K && e == hipSuccess; ++j) {
        const int may = kind == 1 && (j + 1) % h->every == 0;
        const StepArg sa{j, h->d_step, h->burn_in, h->every, may};
        e = nd_enqueue(h, h->cap_stream, sa, static_cast<int>(j & 1), may != 0);
    }
    if (e == hipSuccess) e = launch_add_step(h->cap_stream, h->d_step, K);
    hipGraph_t g = nullptr;
    const hipError_t e_end = hipStreamEndCapture(h->cap_stream, &g);
    if (e == hipSuccess) e = e_end;
    if (e == hipSuccess) e = hipGraphInstantiate(&h->gexec[kind], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        h->gexec[kind] = nullptr;
        return hipfail(h, e, "recording the step graph");
    }
    h->gk[kind] = K;
    return SHE_OK;
}

static she_status advance(she_handle *h, int64_t nsteps, bool sampling)
{
    if (!h) return fail(nullptr, SHE_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(h, SHE_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return SHE_OK;
    hipStream_t s = h->stream;
    if (h->dim == 1) {
        Stats1D st{h->d_s1, h->d_s2, h->d_x, h->d_c, h->d_acc, h->d_hist, h->hist_rows, 0};
        const bool stats = sampling && h->mask != 0;
        const bool tc = stats && (h->mask & SHE_STAT_TCORR);
        const int64_t chunk = 1 << 16;
        // samples taken after completed steps (0, T]: multiples of `every` above burn_in
        auto sampled_by = [&](int64_t T) -> int64_t {
            return T > h->burn_in ? T / h->every - h->burn_in / h->every : 0;
        };
        for (int64_t done = 0; done < nsteps;) {
            int64_t k = std::min<int64_t>(chunk, nsteps - done);
            if (tc) {
                // at most hist_rows - L new samples per launch, so the ring still
                // holds the older rows the lags of the new ones reach
                const int64_t room = h->hist_rows - h->tc_lags;
                const int64_t j0 = std::max(h->steps, h->burn_in) / h->every;
                k = std::min<int64_t>(k, h->every * (j0 + room + 1) - 1 - h->steps);
            }
            // batch means: a launch ends at the step whose sample completes the
            // current batch, and the fold kernels follow it.  The j-th sample
            // after step t completes at every * (max(t, burn_in) / every + j).
            bool fold = false;
            if (stats && h->batch_len > 0) {
                const int64_t need = (h->samples / h->batch_len + 1) * h->batch_len - h->samples;
                const int64_t t_end = h->every * (std::max(h->steps, h->burn_in) / h->every + need);
                if (t_end - h->steps <= k) {
                    k = t_end - h->steps;
                    fold = true;
                }
            }
            SHE_HIP(h, launch_step1d(h->prec, h->block1d, h->maxg, stats, h->mode1d, h->blocks1d, h->smem1d, s,
                                     h->d_tab, h->d_segs, h->d_pool, h->d_coef, h->d_pcr, h->steps,
                                     static_cast<int32_t>(k),
                                     h->burn_in, h->every, h->mask, st));
            const int64_t cnt = stats ? sampled_by(h->steps + k) - sampled_by(h->steps) : 0;
            if (tc && cnt > 0)
                SHE_HIP(h, launch_tcorr1d(h->prec, h->n_inst, h->nmax, h->tc_lags, s, h->d_tab, h->d_hist,
                                          h->hist_rows, h->samples, cnt, h->d_tc, h->d_acc));
            h->samples += cnt;
            if (fold) {
                const Batch1D bk{h->d_bcell, h->d_csnap, h->d_skw1, h->total_cells, h->batch_len, 0};
                SHE_HIP(h, launch_fold1d(h->prec, h->n_inst, h->nmax, s, h->d_tab, h->d_x, h->d_c, h->d_s1, h->d_s2,
                                         h->d_acc, bk));
            }
            h->steps += k;
            done += k;
        }
        return SHE_OK;
    }
    const bool samp = sampling && (h->mask & SHE_STAT_SPATIAL);
    if (h->graph_steps > 0) {
        // replay chunks of K steps that start at a step index aligned to L (so
        // the buffers and the sample positions inside the chunk are those the
        // graph was recorded with); direct steps before, between and after
        const int64_t L = samp ? std::lcm<int64_t>(h->every, 2) : 2;
        const int64_t K = (h->graph_steps + L - 1) / L * L;
        while (nsteps > 0) {
            int kind = -1;
            if (h->steps % L == 0 && h->cur == 0 && nsteps >= K) {
                if (!samp || h->steps + K <= h->burn_in) kind = 0;  // no step of the chunk samples
                else if (h->steps >= h->burn_in) kind = 1;          // every aligned position samples
            }
            if (kind < 0) {
                she_status st = nd_direct(h, samp);
                if (st != SHE_OK) return st;
                --nsteps;
                continue;
            }
            if (!h->gexec[kind] || h->gk[kind] != K) {
                she_status st = record_graph(h, kind, K);
                if (st != SHE_OK) return st;
            }
            if (h->dev_step != h->steps) SHE_HIP(h, launch_set_step(s, h->d_step, h->steps));
            SHE_HIP(h, hipGraphLaunch(h->gexec[kind], s));
            h->steps += K;
            h->dev_step = h->steps;
            nsteps -= K;
        }
        return SHE_OK;
    }
    for (const int64_t end = h->steps + nsteps; h->steps < end;) {
        // Where a pair of steps may not start with a sample step, an odd
        // distance to the next sample step inside the run is bridged by one
        // single step first: the pairs that follow then end on the sample
        // step, and the sample launch is a two-step one.
        bool pair = end - h->steps >= 2;
        if (pair && samp && !first_step_samples_ok(h)) {
            const int64_t t = (std::max(h->steps, h->burn_in) / h->every + 1) * h->every;  // next sample step
            if (t <= end && ((t - h->steps) & 1)) pair = false;
        }
        she_status st = nd_direct(h, samp, pair);
        if (st != SHE_OK) return st;
    }
    return SHE_OK;
}

extern "C" she_status she_step(she_handle *h, int64_t nsteps) { return advance(h, nsteps, false); }

extern "C" she_status she_run(she_handle *h, int64_t nsteps) { return advance(h, nsteps, true); }

extern "C" she_status she_get_step(const she_handle *h, int64_t *steps)
{
    if (!h || !steps) return SHE_EINVAL;
    *steps = h->steps;
    return SHE_OK;
}

extern "C" she_status she_reset_stats(she_handle *h)
{
    if (!h) return fail(nullptr, SHE_EINVAL, "handle is NULL");
    return zero_stats(h);
}

// ------------------------------------------------------------------ results

static she_status copy_out(she_handle *h, double *dst, int64_t cap, const double *src, int64_t n, const char *what)
{
    if (!dst) return SHE_OK;
    if (cap < n) return fail(h, SHE_EINVAL, std::string("capacity too small for ") + what);
    std::memcpy(dst, src, sizeof(double) * n);
    return SHE_OK;
}

extern "C" she_status she_stats(she_handle *h, int32_t instance, she_stats_out *out)
{
    if (!h || !out) return fail(h, SHE_EINVAL, "NULL argument");
    if (instance < 0 || instance >= h->n_inst) return fail(h, SHE_EINVAL, "instance out of range");
    hipStream_t s = h->stream;
    InstAcc acc;
    SHE_HIP(h, hipMemcpyAsync(&acc, h->d_acc + instance, sizeof(InstAcc), hipMemcpyDeviceToHost, s));
    SHE_HIP(h, hipStreamSynchronize(s));
    out->n_samples = acc.n_samples;
    out->steps = h->steps;
    out->nonfinite = acc.nonfinite;
    out->clamp_count = acc.clamp_count;
    // batch-means error bars: SE = sqrt(M2 / (B (B - 1))) from the Welford
    // M2 of the B complete batches' values; NaN while B < 2
    out->n_batches = acc.n_batches;
    const double nbat = static_cast<double>(acc.n_batches);
    auto se_of = [&](double m2) { return acc.n_batches >= 2 ? std::sqrt(m2 / (nbat * (nbat - 1.0))) : NAN; };
    out->spatial_var = acc.n_samples > 0 ? acc.sp_var / static_cast<double>(acc.n_samples) : 0.0;
    out->spatial_var_se = se_of(acc.wv_m2);
    // n values into dst from the device M2 array m2 (null: no batch arrays: NaN)
    auto se_array = [&](double *dst, int64_t cap, int64_t n, const double *m2, const char *what) -> she_status {
        if (!dst) return SHE_OK;
        if (cap < n) return fail(h, SHE_EINVAL, std::string("capacity too small for ") + what);
        if (!m2) {
            for (int64_t i = 0; i < n; ++i) dst[i] = NAN;
            return SHE_OK;
        }
        SHE_HIP(h, hipMemcpyAsync(dst, m2, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        SHE_HIP(h, hipStreamSynchronize(s));
        for (int64_t i = 0; i < n; ++i) dst[i] = se_of(dst[i]);
        return SHE_OK;
    };
    {
        she_status st;
        if (h->dim == 1) {
            const int64_t N = h->tab[instance].n, off = h->tab[instance].off, tc = h->total_cells;
            if ((st = se_array(out->mean_se, out->mean_se_cap, N, h->d_bcell ? h->d_bcell + 3 * tc + off : nullptr,
                               "mean_se")) != SHE_OK)
                return st;
            if ((st = se_array(out->var_se, out->var_se_cap, N, h->d_bcell ? h->d_bcell + 5 * tc + off : nullptr,
                               "var_se")) != SHE_OK)
                return st;
            const bool corr_i = h->tab[instance].c_off >= 0;
            if ((st = se_array(out->sk_se, out->sk_se_cap, N, (h->d_skw1 && corr_i) ? h->d_skw1 + tc + off : nullptr,
                               "sk_se")) != SHE_OK)
                return st;
        } else {
            if (out->mean_se) {
                if (out->mean_se_cap < 1) return fail(h, SHE_EINVAL, "capacity too small for mean_se");
                out->mean_se[0] = se_of(acc.wm_m2);
            }
            if (out->var_se) {
                if (out->var_se_cap < 1) return fail(h, SHE_EINVAL, "capacity too small for var_se");
                out->var_se[0] = se_of(acc.wv_m2);
            }
            if ((st = se_array(out->sk_se, out->sk_se_cap, h->nbins,
                               h->d_skwm2 ? h->d_skwm2 + static_cast<int64_t>(instance) * h->nbins : nullptr,
                               "sk_se")) != SHE_OK)
                return st;
        }
    }
    if (h->dim == 1) {
        const int N = h->tab[instance].n;
        const bool corr = h->tab[instance].x_off >= 0;
        const int rows = static_cast<int>(acc.n_samples % kCorrBlock);
        SHE_HIP(h, launch_fin1d(h->prec, s, h->d_tab, instance, N, h->d_pool, h->d_s1, h->d_s2,
                                corr ? static_cast<char *>(h->d_x) + h->esz * h->tab[instance].x_off : nullptr,
                                corr ? h->d_c + h->tab[instance].c_off : nullptr, acc.n_samples, rows, corr,
                                h->d_fin));
        const size_t len = 4 * static_cast<size_t>(N) + 2 * static_cast<size_t>(N) * N + 1;
        std::vector<double> host(len);
        SHE_HIP(h, hipMemcpyAsync(host.data(), h->d_fin, sizeof(double) * len, hipMemcpyDeviceToHost, s));
        SHE_HIP(h, hipStreamSynchronize(s));
        const int64_t nn = static_cast<int64_t>(N) * N;
        she_status st;
        if (h->d_s1 == nullptr && (out->mean || out->var))
            return fail(h, SHE_EINVAL, "per-cell mean/var need SHE_STAT_MOMENTS");
        if ((st = copy_out(h, out->mean, out->mean_cap, host.data(), N, "mean")) != SHE_OK) return st;
        if ((st = copy_out(h, out->var, out->var_cap, host.data() + N, N, "var")) != SHE_OK) return st;
        if ((out->corr || out->sk) && !corr) return fail(h, SHE_EINVAL, "corr / sk need SHE_STAT_CORR");
        if ((st = copy_out(h, out->corr, out->corr_cap, host.data() + 2 * N, nn, "corr")) != SHE_OK) return st;
        if ((st = copy_out(h, out->sk, out->sk_cap, host.data() + 2 * N + nn, N, "sk")) != SHE_OK) return st;
        out->sum_u = host[3 * N + 2 * nn];
        if (out->tcorr) {
            if (!h->d_tc) return fail(h, SHE_EINVAL, "tcorr needs SHE_STAT_TCORR");
            const int64_t ln = static_cast<int64_t>(h->tc_lags) * N;
            if (out->tcorr_cap < ln) return fail(h, SHE_EINVAL, "capacity too small for tcorr");
            SHE_HIP(h, launch_fin_tc(s, N, h->tc_lags, h->d_s1 + h->tab[instance].off, h->d_tc + h->tab[instance].tc_off,
                                     acc.n_samples, h->d_fin));
            SHE_HIP(h, hipMemcpyAsync(out->tcorr, h->d_fin, sizeof(double) * ln, hipMemcpyDeviceToHost, s));
            SHE_HIP(h, hipStreamSynchronize(s));
        }
    } else {
        SHE_HIP(h, launch_finnd(h->prec, s, h->pnd, instance, h->cells, h->field(), h->d_acc, h->d_sksum,
                                h->d_skmodes, h->nbins, h->d_fin));
        std::vector<double> host(3 + h->nbins);
        SHE_HIP(h, hipMemcpyAsync(host.data(), h->d_fin, sizeof(double) * host.size(), hipMemcpyDeviceToHost, s));
        SHE_HIP(h, hipStreamSynchronize(s));
        she_status st;
        if ((st = copy_out(h, out->mean, out->mean_cap, host.data(), 1, "mean")) != SHE_OK) return st;
        if ((st = copy_out(h, out->var, out->var_cap, host.data() + 1, 1, "var")) != SHE_OK) return st;
        if (out->corr || out->tcorr) return fail(h, SHE_EINVAL, "corr / tcorr are 1D only");
        if ((out->sk || out->sk_modes) && h->nbins == 0) return fail(h, SHE_EINVAL, "sk needs SHE_STAT_SK (2D)");
        if ((st = copy_out(h, out->sk, out->sk_cap, host.data() + 3, h->nbins, "sk")) != SHE_OK) return st;
        if ((st = copy_out(h, out->sk_modes, out->sk_modes_cap, h->skmodes.data(), h->nbins, "sk_modes")) != SHE_OK)
            return st;
        out->sum_u = host[2];
    }
    if (acc.nonfinite) return fail(h, SHE_ENONFINITE, "a sample met a non-finite value; state frozen");
    return SHE_OK;
}

static int64_t inst_cells(const she_handle *h, int i)
{
    return h->dim == 1 ? h->tab[i].n : h->cells;
}

static char *inst_field(const she_handle *h, int i)
{
    const int64_t off = h->dim == 1 ? h->tab[i].off : static_cast<int64_t>(i) * h->cells;
    return static_cast<char *>(h->field()) + h->esz * off;
}

extern "C" she_status she_read_field(she_handle *h, int32_t instance, double *host, int64_t n)
{
    if (!h || !host) return fail(h, SHE_EINVAL, "NULL argument");
    if (instance < 0 || instance >= h->n_inst) return fail(h, SHE_EINVAL, "instance out of range");
    const int64_t nc = inst_cells(h, instance);
    if (n != nc) return fail(h, SHE_EINVAL, "n must equal the instance's cell count");
    std::vector<char> buf(h->esz * nc);
    SHE_HIP(h, hipMemcpyAsync(buf.data(), inst_field(h, instance), buf.size(), hipMemcpyDeviceToHost, h->stream));
    SHE_HIP(h, hipStreamSynchronize(h->stream));
    for (int64_t i = 0; i < nc; ++i)
        host[i] = h->prec == SHE_F32 ? static_cast<double>(reinterpret_cast<float *>(buf.data())[i])
                                     : reinterpret_cast<double *>(buf.data())[i];
    return SHE_OK;
}

extern "C" she_status she_write_field(she_handle *h, int32_t instance, const double *host, int64_t n)
{
    if (!h || !host) return fail(h, SHE_EINVAL, "NULL argument");
    if (instance < 0 || instance >= h->n_inst) return fail(h, SHE_EINVAL, "instance out of range");
    const int64_t nc = inst_cells(h, instance);
    if (n != nc) return fail(h, SHE_EINVAL, "n must equal the instance's cell count");
    std::vector<char> buf(h->esz * nc);
    for (int64_t i = 0; i < nc; ++i) {
        if (h->prec == SHE_F32)
            reinterpret_cast<float *>(buf.data())[i] = static_cast<float>(host[i]);
        else
            reinterpret_cast<double *>(buf.data())[i] = host[i];
    }
    SHE_HIP(h, hipMemcpyAsync(inst_field(h, instance), buf.data(), buf.size(), hipMemcpyHostToDevice, h->stream));
    SHE_HIP(h, hipStreamSynchronize(h->stream));
    return SHE_OK;
}

// ------------------------------------------------------------------ checkpoints

namespace {
struct Blob {
    uint64_t magic;
    uint64_t version;
    int64_t steps;
    int64_t dim, prec, n_inst, cells, x_elems, c_elems, stat_cells;
    int64_t cur;
    int64_t hist_elems, tc_elems, tc_samples;
    int64_t batch_len;
};
constexpr uint64_t kMagic = 0x3153544b50454853ull;  // "SHEPKTS1"

struct Section {
    void *dev;
    size_t bytes;
};

std::vector<Section> sections(const she_handle *h)
{
    std::vector<Section> v;
    if (h->dim == 1) {
        v.push_back({h->d_pool, h->esz * h->total_cells});
        if (h->d_s1) v.push_back({h->d_s1, sizeof(double) * h->total_cells});
        if (h->d_s2) v.push_back({h->d_s2, sizeof(double) * h->total_cells});
        if (h->d_x) v.push_back({h->d_x, h->esz * h->x_elems});
        if (h->d_c) v.push_back({h->d_c, sizeof(double) * h->c_elems});
        if (h->d_hist) v.push_back({h->d_hist, h->esz * h->hist_elems});
        if (h->d_tc) v.push_back({h->d_tc, sizeof(double) * h->tc_elems});
        if (h->d_bcell) v.push_back({h->d_bcell, sizeof(double) * 6 * h->total_cells});
        if (h->d_csnap) v.push_back({h->d_csnap, sizeof(double) * h->c_elems});
        if (h->d_skw1) v.push_back({h->d_skw1, sizeof(double) * 2 * h->total_cells});
    } else {
        v.push_back({h->field(), h->esz * h->cells * h->n_inst});
        if (h->d_sksum) v.push_back({h->d_sksum, sizeof(double) * h->n_inst * h->nbins});
        for (double *p : {h->d_sksnap, h->d_skwm, h->d_skwm2})
            if (p) v.push_back({p, sizeof(double) * h->n_inst * h->nbins});
    }
    v.push_back({h->d_acc, sizeof(InstAcc) * h->n_inst});
    return v;
}

Blob header(const she_handle *h)
{
    Blob b{};
    b.magic = kMagic;
    b.version = 3;
    b.batch_len = h->batch_len;
    b.steps = h->steps;
    b.dim = h->dim;
    b.prec = h->prec;
    b.n_inst = h->n_inst;
    b.cells = h->dim == 1 ? h->total_cells : h->cells;
    b.x_elems = h->x_elems;
    b.c_elems = h->c_elems;
    b.stat_cells = h->d_s1 ? h->total_cells : 0;
    b.cur = 0;
    b.hist_elems = h->hist_elems;
    b.tc_elems = h->tc_elems;
    b.tc_samples = h->samples;
    return b;
}
}  // namespace

extern "C" she_status she_state_bytes(const she_handle *h, size_t *bytes)
{
    if (!h || !bytes) return SHE_EINVAL;
    size_t t = sizeof(Blob);
    for (const Section &s : sections(h)) t += s.bytes;
    *bytes = t;
    return SHE_OK;
}

extern "C" she_status she_get_state(she_handle *h, void *host, size_t bytes)
{
    size_t need = 0;
    if (!h || !host) return fail(h, SHE_EINVAL, "NULL argument");
    she_state_bytes(h, &need);
    if (bytes < need) return fail(h, SHE_EINVAL, "buffer too small for the checkpoint");
    Blob b = header(h);
    char *p = static_cast<char *>(host);
    std::memcpy(p, &b, sizeof b);
    p += sizeof b;
    for (const Section &s : sections(h)) {
        SHE_HIP(h, hipMemcpyAsync(p, s.dev, s.bytes, hipMemcpyDeviceToHost, h->stream));
        p += s.bytes;
    }
    SHE_HIP(h, hipStreamSynchronize(h->stream));
    return SHE_OK;
}

extern "C" she_status she_set_state(she_handle *h, const void *host, size_t bytes)
{
    size_t need = 0;
    if (!h || !host) return fail(h, SHE_EINVAL, "NULL argument");
    she_state_bytes(h, &need);
    if (bytes < need) return fail(h, SHE_ESTATE, "checkpoint smaller than this handle's state");
    Blob b;
    std::memcpy(&b, host, sizeof b);
    Blob mine = header(h);
    if (b.magic != kMagic || b.version != 3 || b.batch_len != mine.batch_len || b.dim != mine.dim || b.prec != mine.prec ||
        b.n_inst != mine.n_inst || b.cells != mine.cells || b.x_elems != mine.x_elems ||
        b.c_elems != mine.c_elems || b.stat_cells != mine.stat_cells || b.hist_elems != mine.hist_elems ||
        b.tc_elems != mine.tc_elems)
        return fail(h, SHE_ESTATE, "checkpoint does not match this handle's layout");
    const char *p = static_cast<const char *>(host) + sizeof b;
    if (h->dim > 1) h->cur = static_cast<int>(b.steps & 1);  // the buffer a step from b.steps reads
    for (const Section &s : sections(h)) {
        SHE_HIP(h, hipMemcpyAsync(s.dev, p, s.bytes, hipMemcpyHostToDevice, h->stream));
        p += s.bytes;
    }
    SHE_HIP(h, hipStreamSynchronize(h->stream));
    h->steps = b.steps;
    h->samples = b.tc_samples;
    return SHE_OK;
}

// ------------------------------------------------------------------ verification

extern "C" she_status she_debug_philox(uint64_t seed, const uint32_t *ctr, int64_t count, uint32_t *out,
                                       void *stream)
{
    if (!ctr || !out || count < 0) return fail(nullptr, SHE_EINVAL, "bad argument");
    if (count == 0) return SHE_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t *dc = nullptr, *dout = nullptr;
    hipError_t e = hipMalloc(&dc, sizeof(uint32_t) * 4 * count);
    if (e == hipSuccess) e = hipMalloc(&dout, sizeof(uint32_t) * 4 * count);
    if (e == hipSuccess) e = hipMemcpyAsync(dc, ctr, sizeof(uint32_t) * 4 * count, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_debug_philox(s, seed, dc, count, dout);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dout, sizeof(uint32_t) * 4 * count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dc);
    (void)hipFree(dout);
    if (e != hipSuccess) return fail(nullptr, SHE_EDEVICE, std::string("debug_philox: ") + hipGetErrorString(e));
    return SHE_OK;
}

// Staging array of she_debug_normals_noalloc: one per GPU for the life of the
// process.  Host code never uses its name as an address; it takes the device
// address from hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) double scratch[SHE_NOALLOC_MAX_NORMALS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (nullptr with *err set).
void *scratch_address(hipError_t *err)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *err = e;
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" she_status she_debug_normals_noalloc(uint64_t seed, uint32_t realisation, uint32_t tag, uint64_t step,
                                                uint64_t face0, int64_t count, int32_t precision, double *out,
                                                void *stream)
{
    if (!out || count < 0 || (precision != SHE_F32 && precision != SHE_F64))
        return fail(nullptr, SHE_EINVAL, "bad argument");
    if (count > SHE_NOALLOC_MAX_NORMALS)
        return fail(nullptr, SHE_EINVAL, "she_debug_normals_noalloc: count above SHE_NOALLOC_MAX_NORMALS");
    if (count == 0) return SHE_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    double *dout = static_cast<double *>(scratch_address(&e));
    if (dout) e = launch_debug_normals(s, precision, seed, realisation, tag, step, face0, count, dout);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dout, sizeof(double) * count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail(nullptr, SHE_EDEVICE, std::string("debug_normals_noalloc: ") + hipGetErrorString(e));
    return SHE_OK;
}

extern "C" she_status she_debug_normals(uint64_t seed, uint32_t realisation, uint32_t tag, uint64_t step,
                                        uint64_t face0, int64_t count, int32_t precision, double *out, void *stream)
{
    if (!out || count < 0 || (precision != SHE_F32 && precision != SHE_F64))
        return fail(nullptr, SHE_EINVAL, "bad argument");
    if (count == 0) return SHE_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *dout = nullptr;
    hipError_t e = hipMalloc(&dout, sizeof(double) * count);
    if (e == hipSuccess) e = launch_debug_normals(s, precision, seed, realisation, tag, step, face0, count, dout);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dout, sizeof(double) * count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dout);
    if (e != hipSuccess) return fail(nullptr, SHE_EDEVICE, std::string("debug_normals: ") + hipGetErrorString(e));
    return SHE_OK;
}
