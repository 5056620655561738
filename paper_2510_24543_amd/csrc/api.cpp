// C ABI of the gfx950 library (declared in include/bec.h): context and
// workspace management, host tables, the 3D FFT driver, the energy /
// Hamiltonian / gradient / preconditioner / line-search entry points and the
// preconditioned nonlinear CG loop of arXiv:2510.24543 (Sec. III Algorithm 1,
// Sec. IV direction, Sec. V step).  Every per-point operation runs in the HIP
// kernels of fft.hip and pointwise.hip; the host only takes the scalar
// decisions (beta, alpha, accept / backtrack / restart) from reduced sums.
#include "bec.h"
#include "bec_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using bec::FftPassArgs;
using bec::PwParams;

namespace {

thread_local std::string g_err;

bec_status fail(bec_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return fail(BEC_EHIP, "%s: %s", #x, hipGetErrorString(e_));  \
    } while (0)

#define STCHK(x)                                 \
    do {                                         \
        bec_status s_ = (x);                     \
        if (s_ != BEC_OK) return s_;             \
    } while (0)

constexpr long double kPiL = 3.141592653589793238462643383279502884L;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Gauss-Legendre nodes/weights on [0,1] by the Golub-Welsch method: the nodes
// are the eigenvalues of the symmetric tridiagonal Jacobi matrix of the
// Legendre polynomials (off-diagonal k/sqrt(4k^2-1)); the weights are twice the
// squared first components of the normalised eigenvectors (halved on [0,1]).
// Implicit QL iteration with Wilkinson shifts, in long double, then one Newton
// polish of each node on the Legendre recurrence.
void gauss_legendre01(int n, std::vector<double>& u, std::vector<double>& w)
{
    std::vector<long double> d(n, 0.0L), e(n, 0.0L), z(n, 0.0L);
    for (int k = 1; k < n; ++k) e[k - 1] = (long double)k / sqrtl(4.0L * k * k - 1.0L);
    z[0] = 1.0L;
    for (int l = 0; l < n; ++l) {
        for (int iter = 0; iter < 200; ++iter) {
            int m = l;
            for (; m < n - 1; ++m) {
                long double dd = fabsl(d[m]) + fabsl(d[m + 1]);
                if (fabsl(e[m]) <= 1e-30L * dd || fabsl(e[m]) < 1e-300L) break;
            }
            if (m == l) break;
            long double g = (d[l + 1] - d[l]) / (2.0L * e[l]);
            long double r = hypotl(g, 1.0L);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? fabsl(r) : -fabsl(r)));
            long double s = 1.0L, c = 1.0L, p = 0.0L;
            int i = m - 1;
            bool early = false;
            for (; i >= l; --i) {
                long double f = s * e[i], b = c * e[i];
                r = hypotl(f, g);
                e[i + 1] = r;
                if (r == 0.0L) {
                    d[i + 1] -= p;
                    e[m] = 0.0L;
                    early = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0L * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                long double zf = z[i + 1];
                z[i + 1] = s * z[i] + c * zf;
                z[i] = c * z[i] - s * zf;
            }
            if (early) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0L;
        }
    }
    std::vector<std::pair<long double, long double>> nw(n);
    for (int i = 0; i < n; ++i) {
        long double x = d[i];
        // Newton polish on P_n(x) = 0
        for (int it = 0; it < 3; ++it) {
            long double p0 = 1.0L, p1 = x;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = x; p0 = 1.0L; }
            long double dp = n * (x * p1 - p0) / (x * x - 1.0L);
            x -= p1 / dp;
        }
        nw[i] = {0.5L * (1.0L + x), z[i] * z[i]};   // weight on [0,1] = (2 z^2)/2
    }
    std::sort(nw.begin(), nw.end());
    u.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        u[i] = (double)nw[i].first;
        w[i] = (double)nw[i].second;
    }
}

// Rule for the u integral of the LHY term (Sec. II, Eq. (3)).  lhy_quad 0:
// n_u Gauss-Legendre nodes on [0,1].  lhy_quad 1, root-split: with a = 3u^2 - 1
// the branch potentials satisfy V_+ V_- = 4 n1 n2 det(a), det quadratic in a, and
// (N_i eta_ij being symmetric, eta_12 eta_21 >= 0) change sign only at the zeros
// of det(a), or of eta_11(a), eta_22(a) when one density vanishes -- points fixed
// by the couplings alone.  n_u nodes go on each piece between consecutive such
// points in u, through u = p + (q - p)(1 - cos(pi t))/2, which turns the
// (u - u_b)^(k/2) ends of the clipped powers into smooth integrands.
void lhy_rule(const bec_params& p, std::vector<double>& u, std::vector<double>& w)
{
    std::vector<double> t, tw;
    gauss_legendre01(p.n_u, t, tw);
    if (p.lhy_quad != 1) {
        u = t;
        w = tw;
        return;
    }
    std::vector<long double> ub;
    auto add = [&](long double a) {
        if (std::isfinite((double)a) && a > -1.0L && a < 2.0L) ub.push_back(sqrtl((a + 1.0L) / 3.0L));
    };
    const long double g11 = p.G[0][0], g22 = p.G[1][1], g12 = p.G[0][1], g21 = p.G[1][0];
    const long double d11 = p.Gdd[0][0], d22 = p.Gdd[1][1], d12 = p.Gdd[0][1], d21 = p.Gdd[1][0];
    // det(a) = qa a^2 + qb a + qc
    const long double qa = d11 * d22 - d12 * d21;
    const long double qb = g11 * d22 + d11 * g22 - g12 * d21 - d12 * g21;
    const long double qc = g11 * g22 - g12 * g21;
    if (qa != 0.0L) {
        const long double disc = qb * qb - 4.0L * qa * qc;
        if (disc >= 0.0L) {
            const long double r = sqrtl(disc);
            add((-qb + r) / (2.0L * qa));
            add((-qb - r) / (2.0L * qa));
        }
    } else if (qb != 0.0L) {
        add(-qc / qb);
    }
    if (d11 != 0.0L) add(-g11 / d11);
    if (d22 != 0.0L) add(-g22 / d22);
    std::sort(ub.begin(), ub.end());
    std::vector<long double> ends{0.0L};
    for (long double b : ub)
        if (b > ends.back() + 1e-15L) ends.push_back(b);
    if (ends.back() < 1.0L) ends.push_back(1.0L);
    u.clear();
    w.clear();
    for (size_t k = 0; k + 1 < ends.size(); ++k) {
        const long double lo = ends[k], len = ends[k + 1] - ends[k];
        for (int j = 0; j < p.n_u; ++j) {
            const long double th = kPiL * (long double)t[j];
            u.push_back((double)(lo + len * 0.5L * (1.0L - cosl(th))));
            w.push_back((double)((long double)tw[j] * len * 0.5L * kPiL * sinl(th)));
        }
    }
}

// Spherical cutoff of the dipolar kernel (radius R in real space):
// c(q) = 1 + 3 cos q / q^2 - 3 sin q / q^3, q = |k| R; below q = 1 its series
// sum_{m>=1} (-1)^(m+1) 6 (m+1) q^(2m) / (2m+3)! = q^2/10 - q^4/280 + ...,
// in long double.
long double cutoff_factor(long double q)
{
    if (q >= 1.0L) return 1.0L + 3.0L * cosl(q) / (q * q) - 3.0L * sinl(q) / (q * q * q);
    long double q2 = q * q, term = q2, fact = 120.0L, s = 0.0L;   // (2m+3)! at m = 1 is 5! = 120
    for (int m = 1; m <= 14; ++m) {
        s += ((m % 2) ? 1.0L : -1.0L) * 6.0L * (m + 1) * term / fact;
        term *= q2;
        fact *= (2.0L * m + 4.0L) * (2.0L * m + 5.0L);
    }
    return s;
}

// Unit-amplitude dipolar kernel at wavevector k (dipoles along z), in long
// double.  dip_cut 0: (3 kz^2/k^2 - 1) c(|k| r_cut), 0 at k = 0 (spherical
// cutoff).  dip_cut 1, the slab cut of the periodic-xy setups: the interaction is
// kept for |z - z'| < Z = r_cut and not cut in x, y; inverting the uncut
// kernel in kz gives 2 delta(u) - (3/2) k_rho exp(-k_rho |u|) at height u, and
// its transform over |u| < Z is
//   (3 kz^2/k^2 - 1) + 3 exp(-k_rho Z)(k_rho^2 cos(kz Z) - k_rho kz sin(kz Z))/k^2,
// 2 at k = 0.  Even in each component, so the octant table serves all k.
long double dipolar_kernel(long double kx, long double ky, long double kz, const bec_params& p)
{
    const long double kr2 = kx * kx + ky * ky, k2 = kr2 + kz * kz;
    if (p.dip_cut == 1) {
        if (k2 == 0.0L) return 2.0L;
        const long double kr = sqrtl(kr2), Z = (long double)p.r_cut;
        return (3.0L * kz * kz / k2 - 1.0L) + 3.0L * expl(-kr * Z) * (kr2 * cosl(kz * Z) - kr * kz * sinl(kz * Z)) / k2;
    }
    if (k2 == 0.0L) return 0.0L;
    return (3.0L * kz * kz / k2 - 1.0L) * cutoff_factor(sqrtl(k2) * (long double)p.r_cut);
}

// Optional per-kernel timing: HIP events recorded on the context stream around
// every launch, resolved when the statistics are read.
struct Prof {
    bool on = false;
    struct Rec {
        int id;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<Rec> recs;
    std::vector<std::string> names;
    std::vector<long long> launches;
    std::vector<double> total_ms, total_bytes;
};

}  // namespace

struct bec_ctx {
    bec_grid g{};
    bec_params p{};
    hipStream_t st = nullptr;
    int n[3] = {0, 0, 0};
    long long N = 0;
    double h[3] = {0, 0, 0}, L[3] = {0, 0, 0}, dV = 0;
    double2 *psi[2] = {}, *hpsi[2] = {}, *aux[2] = {};
    // search directions and residuals in pairs: a direction write reads p_old
    // (pold) and r_old and writes p (pdir) and r (r_new); an accepted step swaps
    // each pair, so a write enqueued ahead of the acceptance test leaves the
    // state that a rejected step falls back to intact
    double2 *pdir = nullptr, *pold = nullptr, *r_old = nullptr, *r_new = nullptr;
    double2 *z = nullptr, *z_next = nullptr, *rho = nullptr, *W = nullptr;   // z_next: a pipelined lookahead
    double *udtab = nullptr, *kv[3] = {}, *vv[3] = {}, *nodes = nullptr;
    double *partials = nullptr, *fft_partials = nullptr, *ls_partials = nullptr;
    double* scal = nullptr;    // device address of `host` (reduced scalars), or device memory (scal_on_device)
    bool scal_on_device = false;   // scal is plain device memory: fetch() copies it into `host`
    double* dscal = nullptr;   // device copies of the scalars that later launches read (same offsets)
    double2* tw[3] = {};
    double* host = nullptr;   // pinned scalars
    double* lhytab = nullptr;  // class-A LHY Chebyshev series (device, 3 * kLhyTabMax)
    std::vector<double> lhy_host = std::vector<double>(3 * bec::kLhyTabMax, 0.0);
    int lhy_K_built = 0;       // terms per series of the built table (0: none met the bar)
    int lhy_table_on = 1;      // tuning: use the table when built
    int kin_axes_on = 1;       // tuning: kinetic term of the energy evaluation from one-axis transforms
    int fuse_z = 3;            // tuning: bit 0 fused direction write + z pass, bit 1 fused z pass + epilogue
    int nblk_pw = 0;
    // the last direction write: fused with the line search's z pass (its partials
    // then come from dir_nblk z-pass blocks and the model skips that pass)
    int dir_fused = 0, dir_nblk = 0;
    int nblk_x = 0;
    int fft_var[3][2] = {{0, 0}, {0, 0}, {0, 0}};   // plan variant per axis: [plain, fused k-space]
    // the iteration state a bec_solve stopped at its max_iter leaves for BEC_SOLVE_CONTINUE;
    // every other call that uses the context clears `valid`
    struct {
        bool valid = false;
        bec_opts o{};
        int cur = 0, n = 0, stall_it = 0;
        bool have_prev = false, spec_write = false;
        double E_prev = 0.0, alpha_prev = 0.0, rz_old = 0.0, stall_ref = 0.0;
        double R[bec::kDirReduceSums] = {};
        bec_terms t{};
        double sums[bec::kHevalSums] = {};
    } resume;
    PwParams P{};
    Prof prof;
};

namespace {

hipEvent_t prof_event(bec_ctx* c)
{
    Prof& P = c->prof;
    if (P.used == P.pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        P.pool.push_back(e);
    }
    return P.pool[P.used++];
}

int prof_id(bec_ctx* c, const char* name)
{
    Prof& P = c->prof;
    for (size_t i = 0; i < P.names.size(); ++i)
        if (P.names[i] == name) return (int)i;
    P.names.emplace_back(name);
    P.launches.push_back(0);
    P.total_ms.push_back(0.0);
    P.total_bytes.push_back(0.0);
    return (int)P.names.size() - 1;
}

// resolve recorded event pairs into the per-kernel totals (synchronises)
bec_status prof_flush(bec_ctx* c)
{
    Prof& P = c->prof;
    if (P.recs.empty()) return BEC_OK;
    HIPCHK(hipStreamSynchronize(c->st));
    for (const auto& r : P.recs) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
        P.launches[r.id] += 1;
        P.total_ms[r.id] += ms;
        P.total_bytes[r.id] += r.bytes;
    }
    P.recs.clear();
    P.used = 0;
    return BEC_OK;
}

// launch `call` (a hipError_t expression); when profiling, bracket it with events
#define LAUNCH(c, name, bytes, call)                                                   \
    do {                                                                               \
        hipEvent_t e0_ = nullptr;                                                      \
        if ((c)->prof.on) {                                                            \
            if ((c)->prof.used + 2 > 8192) STCHK(prof_flush(c));                       \
            e0_ = prof_event(c);                                                       \
            if (e0_) HIPCHK(hipEventRecord(e0_, (c)->st));                             \
        }                                                                              \
        HIPCHK(call);                                                                  \
        if ((c)->prof.on && e0_) {                                                     \
            hipEvent_t e1_ = prof_event(c);                                            \
            if (e1_) {                                                                 \
                HIPCHK(hipEventRecord(e1_, (c)->st));                                  \
                (c)->prof.recs.push_back({prof_id(c, name), e0_, e1_, (double)(bytes)}); \
            }                                                                          \
        }                                                                              \
    } while (0)

// Scalar slots (pinned host buffer and its device copy): each reduction of a
// pipelined iteration has its own range, so one synchronisation reads them all.
constexpr int kScalSlots = 128;
constexpr int kScalModel = 0;     // direction-write sums [0,18), line-search sums [18,25), Parseval [30,32)
constexpr int kScalHeval = 32;    // energy sums (kHevalSums)
constexpr int kScalDir = 56;      // direction-reduce sums (kDirReduceSums)
constexpr int kScalStep = 72;     // device step decision (kStepOut)
constexpr int kScalIte0 = 0;      // imaginary-time sums of even steps (kIteSums + 2 Parseval)
constexpr int kScalIte1 = 96;     // and of odd steps
static_assert(kScalHeval >= 32 && kScalHeval + bec::kHevalSums <= kScalDir, "scalar ranges overlap");
static_assert(kScalDir + bec::kDirReduceSums <= kScalStep && kScalStep + bec::kStepOut <= kScalSlots,
              "scalar ranges overlap");

// The host waits for the scalars of a pipelined iteration by watching the
// pinned slots themselves: before the launches that write them it stores a
// marker there, a signalling-NaN bit pattern, which no arithmetic result can
// be (IEEE operations return quiet NaNs), and it reads a slot once the marker
// is gone.  Each slot is one aligned 8-byte store, so no ordering between slots
// is needed and no stream event is placed between the kernels.
constexpr uint64_t kScalMarker = 0x7ff4dead5e7f11edull;
struct ScalRange {
    int lo, n;
};

void arm_scalars(double* host, const ScalRange* r, int nr)
{
    for (int k = 0; k < nr; ++k)
        for (int i = r[k].lo; i < r[k].lo + r[k].n; ++i)
            __atomic_store_n(reinterpret_cast<uint64_t*>(host + i), kScalMarker, __ATOMIC_RELAXED);
    __atomic_thread_fence(__ATOMIC_SEQ_CST);
}

bool await_scalars(const double* host, const ScalRange* r, int nr, double timeout_s)
{
    const auto t0 = std::chrono::steady_clock::now();
    for (int k = 0; k < nr; ++k)
        for (int i = r[k].lo; i < r[k].lo + r[k].n; ++i) {
            const uint64_t* q = reinterpret_cast<const uint64_t*>(host + i);
            for (unsigned spin = 1; __atomic_load_n(q, __ATOMIC_ACQUIRE) == kScalMarker; ++spin)
                if ((spin & 0xfffu) == 0 &&
                    std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > timeout_s)
                    return false;
        }
    return true;
}

size_t ws_layout(const int n[3], size_t* off /* nullable, 32 entries */)
{
    const long long N = (long long)n[0] * n[1] * n[2];
    const size_t c2 = sizeof(double2);
    const long long nb_pw = std::min<long long>((N + bec::kPwThreads - 1) / bec::kPwThreads, bec::kPwMaxBlocks);
    // x and y blocks over the line search's half-spectrum geometry (z extent n_z + 2), the larger
    const long long nb_x = bec::fft_max_blocks(n[0], (long long)n[1] * (n[2] + 2));
    const long long nb_z = bec::fft_max_blocks(n[2], (long long)n[0] * n[1]);
    const long long nb_y = bec::fft_max_blocks(n[1], (long long)n[0] * (n[2] + 2));
    size_t sizes[] = {
        2 * N * c2, 2 * N * c2,                    // psi[0], psi[1]
        2 * N * c2, 2 * N * c2,                    // hpsi[0], hpsi[1]
        2 * N * c2, 2 * N * c2,                    // aux[0], aux[1]
        2 * N * c2,                                // pdir
        2 * N * c2,                                // r_old
        2 * N * c2,                                // z
        (size_t)n[0] * n[1] * (n[2] + 2) * c2,     // rho (or the line search's half spectra, z extent n_z + 2)
        3 * N * c2,                                // W
        (size_t)(n[0] / 2 + 1) * (n[1] / 2 + 1) * (n[2] / 2 + 1) * sizeof(double),   // udtab
        n[0] * c2, n[1] * c2, n[2] * c2,           // twiddles
        n[0] * sizeof(double), n[1] * sizeof(double), n[2] * sizeof(double),        // k
        n[0] * sizeof(double), n[1] * sizeof(double), n[2] * sizeof(double),        // V per axis
        bec::kMaxNodes * bec::kNodeStride * sizeof(double),                         // nodes
        // partials: the pointwise grid's sums, or the fused direction write's per z-pass block
        (size_t)std::max<long long>(bec::kMaxSums * nb_pw, bec::kDirWriteSums * nb_z) * sizeof(double),
        (size_t)3 * (nb_x + nb_y + nb_z) * sizeof(double),                          // fft partials
        kScalSlots * sizeof(double),                                                // device scalar copies
        (size_t)bec::kLsEpiSums * std::max(nb_z, nb_x) * sizeof(double),           // line-search partials
        2 * N * c2,                                                                 // pold
        2 * N * c2,                                                                 // r_new
        2 * N * c2,                                                                 // z_next
        3 * bec::kLhyTabMax * sizeof(double),                                       // LHY table
    };
    size_t total = 0;
    for (size_t i = 0; i < sizeof(sizes) / sizeof(sizes[0]); ++i) {
        if (off) off[i] = total;
        total += align256(sizes[i]);
    }
    return total;
}

bec_status check_grid(const bec_grid* g)
{
    if (!g) return fail(BEC_EINVAL, "grid is null");
    for (int d = 0; d < 3; ++d) {
        if (!bec::fft_supported(g->n[d]))
            return fail(BEC_EUNSUPPORTED, "axis %d length %d not supported (8,16,32,48,64,96,128,256)", d,
                        g->n[d]);
        if (!(g->hi[d] > g->lo[d]) || !std::isfinite(g->lo[d]) || !std::isfinite(g->hi[d]))
            return fail(BEC_EINVAL, "axis %d: need finite lo < hi", d);
    }
    if ((long long)g->n[0] * g->n[1] * g->n[2] >= (1LL << 31))   // 32-bit point indices in the kernels
        return fail(BEC_EUNSUPPORTED, "more than 2^31 - 1 points per component");
    return BEC_OK;
}

// The slab cut is exact on the periodic grid only if the cut kernel fits in
// one period along z: 2 r_cut <= L_z.
bec_status check_params_grid(const bec_grid* g, const bec_params* p)
{
    if (p->dip_cut == 1 && !(2.0 * p->r_cut <= g->hi[2] - g->lo[2]))
        return fail(BEC_EINVAL, "slab cut (dip_cut 1) needs 2 r_cut <= hi[2] - lo[2]");
    return BEC_OK;
}

bec_status check_params(const bec_params* p)
{
    if (!p) return fail(BEC_EINVAL, "params is null");
    if (!(p->N[0] > 0) || !(p->N[1] > 0)) return fail(BEC_EINVAL, "atom numbers must be positive");
    if (p->n_u < 1 || p->n_u > bec::kMaxNodes) return fail(BEC_EINVAL, "n_u must be in 1..%d", bec::kMaxNodes);
    if (!(p->r_cut > 0)) return fail(BEC_EINVAL, "r_cut must be positive");
    if (p->dip_cut != 0 && p->dip_cut != 1) return fail(BEC_EINVAL, "dip_cut must be 0 or 1");
    if (p->lhy_quad != 0 && p->lhy_quad != 1) return fail(BEC_EINVAL, "lhy_quad must be 0 or 1");
    const double* all[] = {p->omega, &p->G[0][0], &p->Gdd[0][0]};
    const int cnt[] = {3, 4, 4};
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < cnt[a]; ++k)
            if (!std::isfinite(all[a][k])) return fail(BEC_EINVAL, "non-finite parameter");
    if (!std::isfinite(p->c_lhy) || !std::isfinite(p->r_cut)) return fail(BEC_EINVAL, "non-finite parameter");
    const double a = p->N[0] * p->G[0][1], b = p->N[1] * p->G[1][0];
    const double c = p->N[0] * p->Gdd[0][1], d = p->N[1] * p->Gdd[1][0];
    if (std::fabs(a - b) > 1e-12 * std::max(std::fabs(a), std::fabs(b)) ||
        std::fabs(c - d) > 1e-12 * std::max(std::fabs(c), std::fabs(d)))
        return fail(BEC_EINVAL, "N_i G_ij and N_i Gdd_ij must be symmetric");
    if (p->lhy_quad == 1) {
        std::vector<double> u, w;
        lhy_rule(*p, u, w);
        if ((int)u.size() > bec::kMaxNodes)
            return fail(BEC_EINVAL, "the root-split u rule needs %zu nodes (n_u on each piece), at most %d", u.size(),
                        bec::kMaxNodes);
    }
    return BEC_OK;
}

// Node table of the LHY loops (Sec. II Eq. (3) with Gauss-Legendre nodes u_q):
// eta_ij = G_ij + Gdd_ij (3 u_q^2 - 1); class-A nodes (det >= 0, eta_11 or
// eta_22 > 0; both branch potentials >= 0) first, then class-B nodes (det < 0;
// V_- clipped); nodes with both branches clipped everywhere are left out.
void hot_nodes(const bec_params& p, const std::vector<double>& u, const std::vector<double>& w,
               double node5[][5], int* n_a, int* n_b)
{
    std::vector<std::array<double, 5>> A, B;
    for (size_t q = 0; q < u.size(); ++q) {
        const double a = 3.0 * u[q] * u[q] - 1.0;
        const double e11 = p.G[0][0] + p.Gdd[0][0] * a, e22 = p.G[1][1] + p.Gdd[1][1] * a;
        const double p12 = (p.G[0][1] + p.Gdd[0][1] * a) * (p.G[1][0] + p.Gdd[1][0] * a);
        const double det = e11 * e22 - p12;
        if (det < 0.0)
            B.push_back({e11, e22, p12, w[q], 0.0});
        else if (e11 > 0.0 || e22 > 0.0)
            A.push_back({e11, e22, p12, w[q], std::sqrt(det)});
    }
    int k = 0;
    for (const auto& v : A) { for (int j = 0; j < 5; ++j) node5[k][j] = v[j]; ++k; }
    for (const auto& v : B) { for (int j = 0; j < 5; ++j) node5[k][j] = v[j]; ++k; }
    for (; k < bec::kMaxNodes; ++k) for (int j = 0; j < 5; ++j) node5[k][j] = 0.0;
    *n_a = (int)A.size();
    *n_b = (int)B.size();
}

// Class-A sums at (n1, n2) = (x, 1 - x) in long double: f = F, f' = dF/dx along
// (1, -1) = (5/2)(a1 - a2), f'' = 5 times the model sum along n' = (1, -1), from
// the node formulas of the device loops (pw_math.h), without their guards.
struct ClassAVals {
    long double f, f1, f2;
};
ClassAVals class_a_sums(const double node5[][5], int n_a, long double n1, long double n2)
{
    ClassAVals o{0.0L, 0.0L, 0.0L};
    long double A1 = 0.0L, A2 = 0.0L, S2 = 0.0L;
    const long double sq = 2.0L * sqrtl(n1 * n2);
    for (int q = 0; q < n_a; ++q) {
        const long double e11 = node5[q][0], e22 = node5[q][1], p12 = node5[q][2], w = node5[q][3], rq = node5[q][4];
        const long double a = e11 * n1, b = e22 * n2, delta = a - b, pi = sq * rq;
        const long double X = 2.0L * (a + b + pi);
        if (!(X > 1e-300L)) continue;   // the node vanishes there with its derivatives
        const long double r = 1.0L / sqrtl(X), sg = X * r;
        const long double t1 = 2.0L * (X - pi) * r, t3 = sg * (X - 3.0L * pi);
        o.f += w * sg * (X * (X - 5.0L * pi) + 5.0L * pi * pi);
        A1 += w * (e11 * t3 + (e11 * delta + 2.0L * p12 * n2) * t1);
        A2 += w * (e22 * t3 + (-e22 * delta + 2.0L * p12 * n1) * t1);
        const long double d1 = e11 + e22, lin = e11 - e22, cross = 2.0L * (n2 - n1);
        const long double A = delta * d1 + p12 * cross, B0 = d1 * d1 - 4.0L * p12;
        S2 += w * (B0 * (X - pi) * r - A * A * r * r * r + 0.75L * sg * lin * lin + 3.0L * lin * A * r);
    }
    o.f1 = 2.5L * (A1 - A2);
    o.f2 = 5.0L * S2;
    return o;
}

// Chebyshev series of f, f', f'' in y = (sqrt x - sqrt(1-x))/(sqrt x + sqrt(1-x))
// (x = (1+y)^2 / (2 (1+y^2))): the smallest K in 24, 28, ..., kLhyTabMax whose
// series, summed in double as on the device, stay within 2e-14 of the long-double
// sums (relative to each function's largest value) at 257 points of [-1, 1].
// Returns K, or 0 when no K meets that bar (the device keeps the node loop).
int build_lhy_table(const double node5[][5], int n_a, double* coef /* 3 * kLhyTabMax */)
{
    std::fill(coef, coef + 3 * bec::kLhyTabMax, 0.0);
    if (n_a == 0) return 0;
    auto x_of = [](long double y, long double* x1, long double* x2) {
        const long double d = 2.0L * (1.0L + y * y);
        *x1 = (1.0L + y) * (1.0L + y) / d;
        *x2 = (1.0L - y) * (1.0L - y) / d;
    };
    constexpr int M = 257;
    std::vector<ClassAVals> ref(M);
    long double fmax[3] = {0.0L, 0.0L, 0.0L};
    for (int m = 0; m < M; ++m) {
        long double x1, x2;
        x_of(cosl(kPiL * m / (M - 1)), &x1, &x2);
        ref[m] = class_a_sums(node5, n_a, x1, x2);
        fmax[0] = std::max(fmax[0], fabsl(ref[m].f));
        fmax[1] = std::max(fmax[1], fabsl(ref[m].f1));
        fmax[2] = std::max(fmax[2], fabsl(ref[m].f2));
    }
    for (int K = 24; K <= bec::kLhyTabMax; K += 4) {   // even: the device sums two terms per trip
        std::vector<ClassAVals> v(K);
        for (int k = 0; k < K; ++k) {
            long double x1, x2;
            x_of(cosl(kPiL * (k + 0.5L) / K), &x1, &x2);
            v[k] = class_a_sums(node5, n_a, x1, x2);
        }
        std::vector<double> c(3 * bec::kLhyTabMax, 0.0);
        for (int j = 0; j < K; ++j) {
            long double s0 = 0.0L, s1 = 0.0L, s2 = 0.0L;
            for (int k = 0; k < K; ++k) {
                const long double t = cosl(kPiL * j * (k + 0.5L) / K);
                s0 += v[k].f * t;
                s1 += v[k].f1 * t;
                s2 += v[k].f2 * t;
            }
            const long double sc = (j == 0 ? 1.0L : 2.0L) / K;
            c[j] = (double)(sc * s0);
            c[bec::kLhyTabMax + j] = (double)(sc * s1);
            c[2 * bec::kLhyTabMax + j] = (double)(sc * s2);
        }
        bool ok = true;
        for (int m = 0; m < M && ok; ++m) {
            const double y = (double)cosl(kPiL * m / (M - 1));
            const long double want[3] = {ref[m].f, ref[m].f1, ref[m].f2};
            for (int sidx = 0; sidx < 3 && ok; ++sidx) {
                const double* cs = c.data() + sidx * bec::kLhyTabMax;
                // the device's order (lhy_cheb in pw_math.h): ascending k, T_k by recurrence
                double got = std::fma(cs[1], y, cs[0]), tm = 1.0, tk = y;
                for (int k = 2; k < K; k += 2) {
                    const double ta = std::fma(y + y, tk, -tm), tb = std::fma(y + y, ta, -tk);
                    got = std::fma(cs[k], ta, got);
                    got = std::fma(cs[k + 1], tb, got);
                    tm = ta;
                    tk = tb;
                }
                if (!(fabsl((long double)got - want[sidx]) <= 2e-14L * fmax[sidx])) ok = false;
            }
        }
        if (ok) {
            std::copy(c.begin(), c.end(), coef);
            return K;
        }
    }
    return 0;
}

// Host tables that depend on the parameters: quadrature nodes, couplings,
// trap, dipolar kernel.  Uploads asynchronously, then synchronises.
bec_status upload_params(bec_ctx* c, bool dipolar_table)
{
    const bec_params& p = c->p;
    std::vector<double> u, w;
    lhy_rule(p, u, w);
    std::vector<double> nodes((size_t)bec::kMaxNodes * bec::kNodeStride, 0.0);
    for (size_t q = 0; q < u.size(); ++q) {
        const double a = 3.0 * u[q] * u[q] - 1.0;
        double* nd = &nodes[(size_t)q * bec::kNodeStride];
        const double e12 = p.G[0][1] + p.Gdd[0][1] * a, e21 = p.G[1][0] + p.Gdd[1][0] * a;
        nd[0] = p.G[0][0] + p.Gdd[0][0] * a;
        nd[1] = p.G[1][1] + p.Gdd[1][1] * a;
        nd[2] = e12 * e21;
        nd[3] = w[q];
        nd[4] = e12;
        nd[5] = e21;
        nd[6] = a;
    }
    hot_nodes(p, u, w, c->P.node5, &c->P.n_a, &c->P.n_b);
    HIPCHK(hipMemcpyAsync(c->nodes, nodes.data(), nodes.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
    // the host copy outlives the upload: the function synchronises below
    c->lhy_K_built = p.c_lhy != 0.0 ? build_lhy_table(c->P.node5, c->P.n_a, c->lhy_host.data()) : 0;
    HIPCHK(hipMemcpyAsync(c->lhytab, c->lhy_host.data(), c->lhy_host.size() * sizeof(double), hipMemcpyHostToDevice,
                          c->st));
    std::vector<double> vv[3];
    for (int d = 0; d < 3; ++d) {
        vv[d].resize(c->n[d]);
        for (int j = 0; j < c->n[d]; ++j) {
            const double x = c->g.lo[d] + j * c->h[d];
            vv[d][j] = 0.5 * p.omega[d] * p.omega[d] * x * x;
        }
        HIPCHK(hipMemcpyAsync(c->vv[d], vv[d].data(), c->n[d] * sizeof(double), hipMemcpyHostToDevice, c->st));
    }
    std::vector<double> ud;
    if (dipolar_table) {
        const int ax = c->n[0] / 2 + 1, ay = c->n[1] / 2 + 1, az = c->n[2] / 2 + 1;
        ud.resize((size_t)ax * ay * az);
        for (int i = 0; i < ax; ++i)
            for (int j = 0; j < ay; ++j)
                for (int k = 0; k < az; ++k) {
                    const long double kx = 2.0L * kPiL * i / c->L[0], ky = 2.0L * kPiL * j / c->L[1],
                                      kz = 2.0L * kPiL * k / c->L[2];
                    ud[((size_t)i * ay + j) * az + k] = (double)dipolar_kernel(kx, ky, kz, p);
                }
        HIPCHK(hipMemcpyAsync(c->udtab, ud.data(), ud.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
    }
    HIPCHK(hipStreamSynchronize(c->st));

    PwParams& P = c->P;
    P.nx = c->n[0];
    P.ny = c->n[1];
    P.nz = c->n[2];
    P.N = c->N;
    bec::div_magic((uint32_t)(c->n[1] * c->n[2]), &P.m_nyz, &P.s_nyz);
    bec::div_magic((uint32_t)c->n[2], &P.m_nz, &P.s_nz);
    for (int i = 0; i < 2; ++i) {
        P.Nat[i] = p.N[i];
        for (int j = 0; j < 2; ++j) {
            P.G[i][j] = p.G[i][j];
            P.Gdd[i][j] = p.Gdd[i][j];
        }
    }
    P.K5 = p.c_lhy * std::sqrt(2.0) / (15.0 * M_PI * M_PI);
    P.K3 = p.c_lhy / (3.0 * std::sqrt(2.0) * M_PI * M_PI);
    P.n_u = (int)u.size();
    P.lhy_on = p.c_lhy != 0.0;
    P.lhy_tab = c->lhytab;
    P.lhy_K = c->lhy_table_on ? c->lhy_K_built : 0;
    P.nodes = c->nodes;
    P.vx = c->vv[0];
    P.vy = c->vv[1];
    P.vz = c->vv[2];
    P.nblk_pw = c->nblk_pw;
    return BEC_OK;
}

// ------------------------------------------------------------------ FFT driver
FftPassArgs pass_args(bec_ctx* c, int axis)
{
    FftPassArgs A{};
    A.nx = c->n[0];
    A.ny = c->n[1];
    A.nz = c->n[2];
    A.kx = c->kv[0];
    A.ky = c->kv[1];
    A.kz = c->kv[2];
    A.udtab = c->udtab;
    A.inv_n = 1.0 / (double)c->N;
    A.tw = c->tw[axis];
    A.scale = 1.0;
    A.partials = c->fft_partials;
    A.nblk_x = c->nblk_x;
    A.kaxis = c->kv[axis];
    A.pscale = 1.0;
    A.inv_na = 1.0 / (double)c->n[axis];
    for (int f = 0; f < 3; ++f) A.acc[f] = nullptr;
    A.n_inst = 1;
    A.inst_ids = nullptr;
    for (int f = 0; f < 3; ++f) A.src_stride[f] = A.dst_stride[f] = A.src_sel_stride[f] = 0;
    A.src_sel = nullptr;
    A.active = nullptr;
    A.per_inst_tab = 0;
    if (axis == 2) {
        A.S = 1;
        A.npencil = (long long)c->n[0] * c->n[1];
    } else if (axis == 1) {
        A.S = c->n[2];
        A.npencil = (long long)c->n[0] * c->n[2];
    } else {
        A.S = (long long)c->n[1] * c->n[2];
        A.npencil = A.S;
    }
    for (int f = 0; f < 3; ++f) A.op[f] = bec::kOpPlain;
    return A;
}

// Where a pass with kOpParsevalAxis fields writes its block sums: `partials`
// with block stride `stride`, each sum times `pscale` (N / n_axis).
struct ParsevalOut {
    double* partials;
    int stride;
    double pscale;
};

bec_status run_pass(bec_ctx* c, int axis, const double2* const* src, double2* const* dst, int nf, int sign,
                    double scale, const int* ops, const double* prec_a, const double* prec_state = nullptr,
                    double prec_sigma = 0.0, const ParsevalOut* po = nullptr, const double2* const* acc = nullptr)
{
    FftPassArgs A = pass_args(c, axis);
    if (acc)
        for (int f = 0; f < nf; ++f) A.acc[f] = acc[f];
    if (po) {
        A.partials = po->partials;
        A.nblk_x = po->stride;
        A.pscale = po->pscale;
    }
    A.nfield = nf;
    A.sign = sign;
    A.scale = scale;
    A.prec_state = prec_state;
    A.prec_sigma = prec_sigma;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) A.prec_Gdd[i][j] = c->P.Gdd[i][j];
    for (int f = 0; f < nf; ++f) {
        A.src[f] = src[f];
        A.dst[f] = dst[f];
        if (ops) A.op[f] = ops[f];
        if (prec_a) A.prec_a[f] = prec_a[f];
    }
    // algorithmic bytes: every field read once and (unless a Parseval field) written once
    double bytes = 0.0;
    const char* name = "fft";
    bool kin = false, axis_sums = false;
    for (int f = 0; f < nf; ++f) {
        const int op = ops ? ops[f] : bec::kOpPlain;
        kin = kin || op == bec::kOpKinAxis;
        axis_sums = axis_sums || op == bec::kOpParsevalAxis;
        bytes += (double)c->N * ((op == bec::kOpParseval || op == bec::kOpParsevalAxis) ? 16.0
                                 : (op == bec::kOpKinAxis && acc && acc[f]) ? 48.0 : 32.0);
    }
    const bool kspace = ops && axis == 0;    // the x pass with per-field operators
    // one label per kind of launch: the energy evaluation's x pass (kinetic axis
    // term + dipolar multiply), the line search's (Parseval axis sums + dipolar
    // multiply), and the other k-space x passes (preconditioner, imaginary time)
    if (kspace) name = kin ? "fft_x_kin" : axis_sums ? "fft_x_ls" : "fft_x_kspace";
    else if (axis == 2) name = sign < 0 ? (ops ? "fft_z_fwd_ls" : "fft_z_fwd") : "fft_z_inv";
    else if (axis == 1) name = sign < 0 ? (kin ? "fft_y_kin" : ops ? "fft_y_fwd_ls" : "fft_y_fwd") : "fft_y_inv";
    else name = sign < 0 ? "fft_x_fwd" : "fft_x_inv";
    LAUNCH(c, name, bytes, bec::fft_pass(c->n[axis], c->fft_var[axis][kspace ? 1 : 0], axis == 2, A, c->st));
    return BEC_OK;
}

// Plain 3D transform of nf fields (sign -1 forward unnormalised, +1 inverse / N).
bec_status fft3d_plain(bec_ctx* c, const double2* const* src, double2* const* dst, int nf, int sign)
{
    if (sign < 0) {
        STCHK(run_pass(c, 2, src, dst, nf, -1, 1.0, nullptr, nullptr));
        STCHK(run_pass(c, 1, dst, dst, nf, -1, 1.0, nullptr, nullptr));
        STCHK(run_pass(c, 0, dst, dst, nf, -1, 1.0, nullptr, nullptr));
    } else {
        STCHK(run_pass(c, 0, src, dst, nf, +1, 1.0, nullptr, nullptr));
        STCHK(run_pass(c, 1, dst, dst, nf, +1, 1.0, nullptr, nullptr));
        STCHK(run_pass(c, 2, dst, dst, nf, +1, 1.0 / (double)c->N, nullptr, nullptr));
    }
    return BEC_OK;
}

// Diagonal k-space operators on nf fields: forward z, y, then the fused x pass
// (ops per field), then inverse y, z for the fields that are stored.
// Parseval fields come first in the list (they end at the x pass).
bec_status kspace_after_z(bec_ctx* c, double2* const* dst, int nf, const int* ops, const double* prec_a,
                          const double* prec_state = nullptr, double prec_sigma = 0.0);

// prec_state / prec_sigma: kOpMulPrec shifts decided on the device (see FftPassArgs)
bec_status kspace_apply(bec_ctx* c, const double2* const* src, double2* const* dst, int nf, const int* ops,
                        const double* prec_a, const double* prec_state = nullptr, double prec_sigma = 0.0)
{
    STCHK(run_pass(c, 2, src, dst, nf, -1, 1.0, nullptr, nullptr));
    return kspace_after_z(c, dst, nf, ops, prec_a, prec_state, prec_sigma);
}

// The same for the three fields (psi_1, psi_2, packed density) of the trial
// point psi_dst = a_i psi_src + b_i p: the trial update rides in the loads of
// the forward z pass, which also stores psi_dst.
//
// With the kinetic multiply on psi_1, psi_2 (ops MulKin, MulKin, MulDip) the
// kinetic term uses T = T_x + T_y + T_z: the trial pass stores T_z psi_i, the
// y and x passes that carry the density's forward transforms add T_y psi_i and
// T_x psi_i from one-dimensional transforms of the stored trial point, and the
// inverse y and z passes carry the density alone.
// z_left (optional): with the one-axis kinetic terms, leave the last inverse z
// pass of dst[2] to the caller (set to true when it is left)
bec_status kspace_apply_trial(bec_ctx* c, const bec::TrialZArgs& Z, double2* const* dst, const int* ops,
                              const double* prec_a, bool* z_left = nullptr)
{
    const bool kin_axes =
        c->kin_axes_on && ops[0] == bec::kOpMulKin && ops[1] == bec::kOpMulKin && ops[2] == bec::kOpMulDip;
    bec::FftPassArgs A = pass_args(c, 2);
    A.nfield = 3;
    A.sign = -1;
    for (int f = 0; f < 3; ++f) {
        A.src[f] = dst[f];
        A.dst[f] = dst[f];
    }
    bec::TrialZArgs Zk = Z;
    Zk.kin_z = kin_axes ? 1 : 0;
    const double bytes = (double)c->N * ((Z.p ? 64.0 : 32.0) + 32.0 + 48.0);
    LAUNCH(c, "fft_z_trial", bytes, bec::fft_trial_z_pass(c->n[2], c->fft_var[2][0], A, Zk, c->st));
    if (!kin_axes) return kspace_after_z(c, dst, 3, ops, prec_a);
    const long long N = c->N;
    const double2* src[3] = {Z.psi_dst, Z.psi_dst + N, dst[2]};
    const double2* acc[3] = {dst[0], dst[1], nullptr};
    const int ops_y[3] = {bec::kOpKinAxis, bec::kOpKinAxis, bec::kOpPlain};
    const int ops_x[3] = {bec::kOpKinAxis, bec::kOpKinAxis, bec::kOpMulDip};
    STCHK(run_pass(c, 1, src, dst, 3, -1, 1.0, ops_y, prec_a, nullptr, 0.0, nullptr, acc));
    STCHK(run_pass(c, 0, src, dst, 3, -1, 1.0, ops_x, prec_a, nullptr, 0.0, nullptr, acc));
    STCHK(run_pass(c, 1, dst + 2, dst + 2, 1, +1, 1.0, nullptr, nullptr));
    if (z_left) {
        *z_left = true;
        return BEC_OK;
    }
    STCHK(run_pass(c, 2, dst + 2, dst + 2, 1, +1, 1.0, nullptr, nullptr));
    return BEC_OK;
}

bec_status kspace_after_z(bec_ctx* c, double2* const* dst, int nf, const int* ops, const double* prec_a,
                          const double* prec_state, double prec_sigma)
{
    STCHK(run_pass(c, 1, dst, dst, nf, -1, 1.0, nullptr, nullptr));
    STCHK(run_pass(c, 0, dst, dst, nf, -1, 1.0, ops, prec_a, prec_state, prec_sigma));
    int first = 0;
    while (first < nf && ops[first] == bec::kOpParseval) ++first;
    if (first < nf) {
        STCHK(run_pass(c, 1, dst + first, dst + first, nf - first, +1, 1.0, nullptr, nullptr));
        STCHK(run_pass(c, 2, dst + first, dst + first, nf - first, +1, 1.0, nullptr, nullptr));
    }
    return BEC_OK;
}

// ------------------------------------------------------------------ reductions
constexpr int kParsevalOut = 30;    // scal slots of the two Parseval sums of an x pass

// c->scal is the device address of the pinned host buffer c->host (or, for a
// context without pinned memory, device memory that is copied back here)
bec_status fetch(bec_ctx* c, int M)
{
    (void)M;
    if (c->scal_on_device)
        HIPCHK(hipMemcpyAsync(c->host, c->scal, kScalSlots * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return BEC_OK;
}

bec_status reduce_pw(bec_ctx* c, int M, int out_off)
{
    LAUNCH(c, "reduce_final", 8.0 * M * c->nblk_pw, bec::launch_reduce_final(c->partials, c->nblk_pw, M, c->scal + out_off, c->st));
    return BEC_OK;
}

// the same, with a device copy of the results at the same offset of c->dscal
bec_status reduce_pw_copy(bec_ctx* c, int M, int out_off, int nblk = 0)
{
    if (nblk <= 0) nblk = c->nblk_pw;
    const bec::RedSeg a{c->partials, nblk, M, c->scal + out_off, c->dscal + out_off};
    const bec::RedSeg none{nullptr, 0, 0, nullptr, nullptr};
    LAUNCH(c, "reduce_final", 8.0 * M * c->nblk_pw, bec::launch_reduce_segs(a, none, none, c->st));
    return BEC_OK;
}

// ------------------------------------------------------------------ H evaluation
struct Eval {
    bec_terms t{};
    double sums[bec::kHevalSums]{};
};

// psi[set] = a_i src + b_i p (p may be null; a, b from the device step
// decision at `coef` when that is set), then H psi, Phi, muLHY and the energy
// sums for that state (scalar range kScalHeval, host and device copy).
bec_status heval_launch(bec_ctx* c, const double2* src, const double2* p, const double a[2], const double b[2],
                        const double* coef, int set)
{
    const long long N = c->N;
    bec::TrialZArgs z{};
    z.psi_src = src;
    z.p = p;
    for (int i = 0; i < 2; ++i) {
        z.a[i] = coef ? 0.0 : a[i];
        z.b[i] = coef ? 0.0 : b[i];
    }
    z.coef = coef;
    z.psi_dst = c->psi[set];
    z.N = N;
    // the dipolar potentials Phi_1 + i Phi_2 land directly in aux[set] (its first
    // half), where the later passes read them
    double2* fdst[3] = {c->W, c->W + N, c->aux[set]};
    const int ops[3] = {bec::kOpMulKin, bec::kOpMulKin, bec::kOpMulDip};
    bool z_left = false;
    STCHK(kspace_apply_trial(c, z, fdst, ops, nullptr, (c->fuse_z & 2) ? &z_left : nullptr));
    bec::HevalArgs ha{};
    ha.psi = c->psi[set];
    ha.Tpsi = c->W;
    ha.phi = c->aux[set];
    ha.hpsi = c->hpsi[set];
    ha.aux = c->aux[set];
    ha.partials = c->partials;
    if (z_left) {   // the inverse z pass of Phi fused with the epilogue
        bec::FftPassArgs Zp = pass_args(c, 2);
        Zp.nfield = 1;
        Zp.sign = +1;
        Zp.src[0] = Zp.dst[0] = c->aux[set];
        const int nblk = bec::fft_blocks(c->n[2], c->fft_var[2][0], Zp.npencil);
        LAUNCH(c, "heval_z", (double)c->N * 144.0,
               bec::fft_heval_z_pass(c->n[2], c->fft_var[2][0], Zp, c->P, ha, c->st));
        return reduce_pw_copy(c, bec::kHevalSums, kScalHeval, nblk);
    }
    LAUNCH(c, "heval_epilogue", (double)c->N * 128.0, bec::launch_heval_epi(c->P, ha, c->nblk_pw, c->st));
    return reduce_pw_copy(c, bec::kHevalSums, kScalHeval);
}

// energy terms, chemical potentials and shifts from the energy sums of the last
// heval_launch (after a synchronisation)
bec_status heval_read(bec_ctx* c, Eval* out)
{
    const double* S = c->host + kScalHeval;
    std::memcpy(out->sums, S, sizeof(out->sums));
    const double dV = c->dV;
    bec_terms& t = out->t;
    std::memset(&t, 0, sizeof(t));
    const double snn[2][2] = {{S[4], S[5]}, {S[5], S[6]}};
    // the rule that pipelined launches apply on the device to the same sums
    bec::rule_mu_shift(S, c->P.Gdd, t.mu, t.shift);
    for (int i = 0; i < 2; ++i) {
        t.norm2[i] = dV * S[14 + i];
        t.E_kin[i] = c->p.N[i] * dV * S[i];
        t.E_trap[i] = c->p.N[i] * dV * S[2 + i];
        for (int j = 0; j < 2; ++j) {
            t.E_c[i][j] = 0.5 * c->p.N[i] * c->p.G[i][j] * dV * snn[i][j];
            t.E_dd[i][j] = 0.5 * c->p.N[i] * c->p.Gdd[i][j] * dV * S[7 + 2 * i + j];
        }
        t.res[i] = NAN;
    }
    t.E_lhy = dV * S[11];
    t.E = t.E_lhy;
    for (int i = 0; i < 2; ++i) {
        t.E += t.E_kin[i] + t.E_trap[i];
        for (int j = 0; j < 2; ++j) t.E += t.E_c[i][j] + t.E_dd[i][j];
    }
    if (!std::isfinite(t.E) || !std::isfinite(t.mu[0]) || !std::isfinite(t.mu[1]))
        return fail(BEC_ENONFINITE, "non-finite energy");
    return BEC_OK;
}

bec_status heval(bec_ctx* c, const double2* src, const double2* p, const double a[2], const double b[2], int set,
                 Eval* out)
{
    STCHK(heval_launch(c, src, p, a, b, nullptr, set));
    STCHK(fetch(c, 0));
    return heval_read(c, out);
}

bec::DirArgs dir_args(bec_ctx* c, int set, const Eval& ev, int zmode, double sigma)
{
    bec::DirArgs A{};
    A.psi = c->psi[set];
    A.hpsi = c->hpsi[set];
    A.aux = c->aux[set];
    A.zbuf = c->z;
    A.r_old = c->r_old;
    A.p = c->pold;
    A.p_out = c->pdir;
    A.r_out = c->r_new;
    A.rho = c->rho;
    for (int i = 0; i < 2; ++i) {
        A.mu[i] = ev.t.mu[i];
        A.diag_shift[i] = ev.t.shift[i];
    }
    A.sigma = sigma;
    A.zmode = zmode;
    A.zsign = -1.0;
    A.beta = 0.0;
    A.partials = c->partials;
    return A;
}

// Direction reduce pass into the scalar range kScalDir (host and device copy).
bec_status dir_reduce_launch(bec_ctx* c, const bec::DirArgs& A)
{
    const double rb = 64.0 + (A.zmode == 1 ? 16.0 : 0.0) + (A.zmode == 2 ? 32.0 : 0.0) + (A.zmode >= 3 ? 48.0 : 0.0) +
                      (A.have_prev ? 64.0 : 0.0);
    LAUNCH(c, "dir_reduce", (double)c->N * rb, bec::launch_dir_reduce(c->P, A, c->nblk_pw, c->st));
    return reduce_pw_copy(c, bec::kDirReduceSums, kScalDir);
}

// Direction reduce pass: returns the 12 sums (see kDirReduceSums).
bec_status dir_reduce(bec_ctx* c, const bec::DirArgs& A, double* R)
{
    STCHK(dir_reduce_launch(c, A));
    STCHK(fetch(c, bec::kDirReduceSums));
    std::memcpy(R, c->host + kScalDir, bec::kDirReduceSums * sizeof(double));
    return BEC_OK;
}

// z = P^-1 r into out (default c->z) for the kinetic / composite preconditioners;
// with dev_state the chemical potentials and shifts come from those device
// energy sums (a pipelined launch) instead of ev.
bec_status compute_z(bec_ctx* c, int set, const Eval& ev, const double2* rin, int apply_pv, double sigma,
                     double2* out = nullptr, const double* dev_state = nullptr)
{
    if (!out) out = c->z;
    bec::MakeRArgs m{};
    m.psi = c->psi[set];
    m.hpsi = c->hpsi[set];
    m.aux = c->aux[set];
    m.rin = rin;
    for (int i = 0; i < 2; ++i) {
        m.mu[i] = ev.t.mu[i];
        m.diag_shift[i] = ev.t.shift[i];
    }
    m.sigma = sigma;
    m.apply_pv = apply_pv;
    m.out = out;
    m.dev_state = dev_state;
    const long long N = c->N;
    const double2* src[2] = {out, out + N};
    double2* dst[2] = {out, out + N};
    const int ops[2] = {bec::kOpMulPrec, bec::kOpMulPrec};
    const double pa[2] = {std::max(ev.t.shift[0], 0.0) + sigma, std::max(ev.t.shift[1], 0.0) + sigma};
    if (!rin && apply_pv <= 2 && (c->fuse_z & 1)) {   // make_r and the first z pass in one kernel
        bec::FftPassArgs Z = pass_args(c, 2);
        Z.tw = c->tw[2];
        LAUNCH(c, "make_r_z", (double)N * (apply_pv ? 112.0 : 96.0),
               bec::fft_maker_z_pass(c->n[2], c->fft_var[2][0], Z, c->P, m, c->st));
        return kspace_after_z(c, dst, 2, ops, pa, dev_state, sigma);
    }
    LAUNCH(c, "make_r", (double)N * 112.0, bec::launch_make_r(c->P, m, c->st));
    return kspace_apply(c, src, dst, 2, ops, pa, dev_state, sigma);
}

struct Model {
    double D[bec::kDirWriteSums];
    double LS[bec::kLsEpiSums];
    double pars[2];
    double pnorm[2], rp, E1, E2, psip[2];
    double alpha, a[2], b[2];     // the device step decision and its trial coefficients
};

static_assert(bec::kDirWriteSums + bec::kLsEpiSums <= kParsevalOut, "model scalars overlap the Parseval slots");
static_assert(bec::kIteSums <= kParsevalOut, "imaginary-time sums overlap the Parseval slots");
static_assert(bec::kDirWriteSums + bec::kLsEpiSums <= bec::kMaxSums, "model partials exceed the partials area");
static_assert(kParsevalOut + 2 <= kScalHeval, "Parseval slots overlap the energy sums");

// Blocks of the line search's z (fused direction write), y and x passes when the
// densities travel as half spectra (z extent n_z + 2 in the y and x passes).
void ls_half_blocks(bec_ctx* c, int* nbz, int* nby, int* nbx)
{
    const long long nzh = c->n[2] + 2;
    *nbz = bec::fft_blocks(c->n[2], c->fft_var[2][1], (long long)c->n[0] * c->n[1]);
    *nby = bec::fft_blocks(c->n[1], c->fft_var[1][0], (long long)c->n[0] * nzh);
    *nbx = bec::fft_blocks(c->n[0], c->fft_var[0][1], (long long)c->n[1] * nzh);
}

// Direction write pass (p, r, rho).  With P_V or the composite (zmode 1, 2) and
// fuse_z bit 0 it is fused with the line search's forward z pass (the z-axis
// Parseval sums of p, and the z transforms of rho_1, rho_2 as half spectra in
// the rho buffer instead of rho itself), which model_launch then continues.
bec_status dir_write_launch(bec_ctx* c, const bec::DirArgs& A)
{
    const double wb = 96.0 + (A.beta != 0.0 || A.dev_dir ? 32.0 : 0.0) + (A.zmode >= 2 ? 32.0 : 0.0) + 80.0;
    if ((A.zmode == 1 || A.zmode == 2) && (c->fuse_z & 1)) {
        const long long N = c->N;
        bec::FftPassArgs Z = pass_args(c, 2);
        Z.nfield = 3;
        Z.sign = -1;
        Z.dst[2] = c->rho;                            // half spectra, z extent n_z + 2
        // its own plan variant (the z axis has no k-space pass, so the second slot is free)
        const int var = c->fft_var[2][1];
        int nbz, nby, nbx;
        ls_half_blocks(c, &nbz, &nby, &nbx);
        Z.tw = c->tw[2];
        Z.partials = c->fft_partials;                 // the z slot of the model's Parseval sums
        Z.nblk_x = nbz + nby + nbx;
        Z.pscale = (double)c->n[0] * c->n[1];
        bec::DirArgs Af = A;
        Af.rho = nullptr;                             // rho itself is not needed on this path
        LAUNCH(c, "dir_write_z", (double)N * (wb - 16.0) + 16.0 * c->n[0] * c->n[1] * (c->n[2] + 2),
               bec::fft_dirwrite_z_pass(c->n[2], var, Z, c->P, Af, c->st));
        c->dir_fused = 1;
        c->dir_nblk = nbz;
        return BEC_OK;
    }
    LAUNCH(c, "dir_write", (double)c->N * wb, bec::launch_dir_write(c->P, A, c->nblk_pw, c->st));
    c->dir_fused = 0;
    c->dir_nblk = c->nblk_pw;
    return BEC_OK;
}

bec_status model_finish(bec_ctx* c, int nbp, int nls, const double norm2[2], double alpha_prev, double theta_max);

// The line-search passes once rho_1, rho_2 are half spectra along z in hs (left
// there by the fused direction write, or by the z pass of model_launch): one y pass (the y-axis Parseval sums of p and
// the forward y transform of the half spectra) and one x pass (the x-axis Parseval
// sums of p and, from the forward x transform of the half spectra, the model's
// density sums in k-space, kOpDipSums); no inverse transform, nothing stored but
// the y pass's spectra.  Field 2 has its own geometry (z extent n_z + 2).
bec_status ls_half_passes(bec_ctx* c, double2* hs, int nbz, int nby, int nbx)
{
    const long long N = c->N, nzh = c->n[2] + 2, half = (long long)c->n[0] * c->n[1] * nzh;
    const int nbp = nbz + nby + nbx;
    for (int axis = 1; axis >= 0; --axis) {
        bec::FftPassArgs A = pass_args(c, axis);
        A.nfield = 3;
        A.sign = -1;
        A.src[0] = c->pdir;
        A.src[1] = c->pdir + N;
        A.src[2] = hs;
        A.dst[0] = A.dst[1] = nullptr;                // Parseval fields: no store
        A.dst[2] = hs;
        A.op[0] = A.op[1] = bec::kOpParsevalAxis;
        A.op[2] = axis == 1 ? bec::kOpPlain : bec::kOpDipSums;
        A.S2 = axis == 1 ? nzh : (long long)c->n[1] * nzh;
        A.npencil2 = axis == 1 ? (long long)c->n[0] * nzh : A.S2;
        A.partials = c->fft_partials + (axis == 1 ? nbz : nbz + nby);
        A.nblk_x = nbp;
        A.pscale = axis == 1 ? (double)c->n[0] * c->n[2] : (double)c->n[1] * c->n[2];
        A.ls_partials = c->ls_partials;
        const int var = c->fft_var[axis][axis == 0 ? 1 : 0];
        const double bytes = 32.0 * N + (axis == 1 ? 32.0 : 16.0) * half;
        LAUNCH(c, axis == 1 ? "fft_y_fwd_ls" : "fft_x_ls", bytes,
               bec::fft_pass(c->n[axis], var, false, A, c->st));
    }
    return BEC_OK;
}

// The line-search model after a direction write: the one-axis Parseval sums of p
// and the densities' sums in k-space (half spectra from the fused direction
// write, or from a z pass here), one reduction of the direction-write, Parseval
// and density partials (host and device copies), then the step decision on the
// device (kScalStep) from the state's norms, the previous step and the angle cap.
bec_status model_launch(bec_ctx* c, const double norm2[2], double alpha_prev, double theta_max)
{
    const long long N = c->N;
    int nbz, nby, nbx;
    ls_half_blocks(c, &nbz, &nby, &nbx);
    if (c->dir_fused) {
        STCHK(ls_half_passes(c, c->rho, nbz, nby, nbx));
        return model_finish(c, nbz + nby + nbx, nbx, norm2, alpha_prev, theta_max);
    }
    // after the grid-stride direction write: a z pass with the z-axis Parseval sums of p
    // and the half spectra of rho (from the packed rho it stored) into W + N, then the same
    // y and x passes (no launch between them and the z pass writes W)
    nbz = bec::fft_blocks(c->n[2], c->fft_var[2][0], (long long)c->n[0] * c->n[1]);
    {
        const double2* src[3] = {c->pdir, c->pdir + N, c->rho};
        double2* dst[3] = {nullptr, nullptr, c->W + N};
        const int ops[3] = {bec::kOpParsevalAxis, bec::kOpParsevalAxis, bec::kOpHalfSpectra};
        const ParsevalOut pz{c->fft_partials, nbz + nby + nbx, (double)c->n[0] * c->n[1]};
        STCHK(run_pass(c, 2, src, dst, 3, -1, 1.0, ops, nullptr, nullptr, 0.0, &pz));
    }
    STCHK(ls_half_passes(c, c->W + N, nbz, nby, nbx));
    return model_finish(c, nbz + nby + nbx, nbx, norm2, alpha_prev, theta_max);
}

// One reduction of the direction-write, Parseval (nbp blocks per field) and
// line-search (nls blocks) partials, then the step decision on the device.
bec_status model_finish(bec_ctx* c, int nbp, int nls, const double norm2[2], double alpha_prev, double theta_max)
{
    const long long N = c->N;
    const int o = kScalModel;
    const bec::RedSeg s1{c->partials, c->dir_nblk, bec::kDirWriteSums, c->scal + o, c->dscal + o};
    const bec::RedSeg s2{c->fft_partials, nbp, 2, c->scal + o + kParsevalOut, c->dscal + o + kParsevalOut};
    const bec::RedSeg s3{c->ls_partials, nls, bec::kLsEpiSums, c->scal + o + bec::kDirWriteSums,
                         c->dscal + o + bec::kDirWriteSums};
    LAUNCH(c, "reduce_final", 8.0 * (bec::kDirWriteSums * c->dir_nblk + 2 * nbp + bec::kLsEpiSums * nls),
           bec::launch_reduce_segs(s1, s2, s3, c->st));
    bec::StepArgs st{};
    st.D = c->dscal + o;
    st.LS = c->dscal + o + bec::kDirWriteSums;
    st.pars = c->dscal + o + kParsevalOut;
    st.dV = c->dV;
    st.inv_n = 1.0 / (double)N;
    st.norm2[0] = norm2[0];
    st.norm2[1] = norm2[1];
    st.alpha_prev = alpha_prev;
    st.theta_max = theta_max;
    st.out = c->dscal + kScalStep;
    st.out_host = c->scal + kScalStep;
    LAUNCH(c, "ls_step", 8.0 * 32, bec::launch_ls_step(c->P, st, c->st));
    return BEC_OK;
}

// model sums and the step decision of the last model_launch (after a synchronisation)
void model_read(bec_ctx* c, Model* m)
{
    const double* S = c->host + kScalModel;
    std::memcpy(m->D, S, sizeof(m->D));
    std::memcpy(m->LS, S + bec::kDirWriteSums, sizeof(m->LS));
    m->pars[0] = S[kParsevalOut];
    m->pars[1] = S[kParsevalOut + 1];
    const double* T = c->host + kScalStep;
    for (int i = 0; i < 2; ++i) {
        m->a[i] = T[i];
        m->b[i] = T[2 + i];
        m->pnorm[i] = T[8 + i];
        m->psip[i] = T[10 + i];
    }
    m->alpha = T[4];
    m->rp = T[5];
    m->E1 = T[6];
    m->E2 = T[7];
}

// Direction write + model + step decision; one synchronisation.
bec_status direction_and_model(bec_ctx* c, const bec::DirArgs& A, const Eval& ev, double alpha_prev,
                               double theta_max, Model* m)
{
    STCHK(dir_write_launch(c, A));
    STCHK(model_launch(c, ev.t.norm2, alpha_prev, theta_max));
    STCHK(fetch(c, 0));
    model_read(c, m);
    return BEC_OK;
}

// trial coefficients along the geodesic: psi_i(alpha) = (cos th psi_i + sin th p_i/|p_i|)/norm
void geodesic_coeffs(const Eval& ev, const Model& m, double alpha, double a[2], double b[2])
{
    for (int i = 0; i < 2; ++i) {
        if (m.pnorm[i] > 0.0) {
            const double th = alpha * m.pnorm[i];
            const double ca = std::cos(th), sb = std::sin(th) / m.pnorm[i];
            const double nrm2 = ca * ca * ev.t.norm2[i] + sb * sb * m.pnorm[i] * m.pnorm[i] + 2.0 * ca * sb * m.psip[i];
            const double s = 1.0 / std::sqrt(nrm2);
            a[i] = ca * s;
            b[i] = sb * s;
        } else {
            a[i] = 1.0 / std::sqrt(ev.t.norm2[i]);
            b[i] = 0.0;
        }
    }
}

bec_status normalise_into(bec_ctx* c, const double2* src, int set)
{
    LAUNCH(c, "norm2", (double)c->N * 32.0, bec::launch_norm2(c->P, src, c->partials, c->nblk_pw, c->st));
    STCHK(reduce_pw(c, 2, 0));
    STCHK(fetch(c, 2));
    const double n0 = c->dV * c->host[0], n1 = c->dV * c->host[1];
    if (!(n0 > 0) || !(n1 > 0) || !std::isfinite(n0) || !std::isfinite(n1))
        return fail(BEC_ENONFINITE, "initial state has zero or non-finite norm");
    LAUNCH(c, "scale2", (double)c->N * 64.0,
           bec::launch_scale2(c->P, src, c->psi[set], 1.0 / std::sqrt(n0), 1.0 / std::sqrt(n1), c->st));
    return BEC_OK;
}

bec_status residual_norms(bec_ctx* c, int set, Eval* ev)
{
    bec::DirArgs A = dir_args(c, set, *ev, 0, 0.0);
    double R[bec::kDirReduceSums];
    STCHK(dir_reduce(c, A, R));
    ev->t.res[0] = std::sqrt(c->dV * R[0]);
    ev->t.res[1] = std::sqrt(c->dV * R[6]);
    return BEC_OK;
}

const double kOne[2] = {1.0, 1.0};
const double kZero[2] = {0.0, 0.0};

// Grid geometry and workspace pointers of a context (layout `off` of ws_layout
// inside `base`); no device work.
void ctx_attach(bec_ctx* c, const bec_grid* grid, const bec_params* params, void* hip_stream, char* base,
                const size_t* off)
{
    c->g = *grid;
    c->p = *params;
    c->st = reinterpret_cast<hipStream_t>(hip_stream);
    for (int d = 0; d < 3; ++d) {
        c->n[d] = grid->n[d];
        c->L[d] = grid->hi[d] - grid->lo[d];
        c->h[d] = c->L[d] / grid->n[d];
    }
    c->N = (long long)c->n[0] * c->n[1] * c->n[2];
    c->dV = c->h[0] * c->h[1] * c->h[2];
    c->fft_var[2][1] = bec::fft_fused_default_variant(c->n[2]);   // the fused direction write's plan
    auto at = [&](int i) { return base + off[i]; };
    c->psi[0] = (double2*)at(0);
    c->psi[1] = (double2*)at(1);
    c->hpsi[0] = (double2*)at(2);
    c->hpsi[1] = (double2*)at(3);
    c->aux[0] = (double2*)at(4);
    c->aux[1] = (double2*)at(5);
    c->pdir = (double2*)at(6);
    c->r_old = (double2*)at(7);
    c->pold = (double2*)at(26);
    c->r_new = (double2*)at(27);
    c->z_next = (double2*)at(28);
    c->lhytab = (double*)at(29);
    c->dscal = (double*)at(24);
    c->z = (double2*)at(8);
    c->rho = (double2*)at(9);
    c->W = (double2*)at(10);
    c->udtab = (double*)at(11);
    for (int d = 0; d < 3; ++d) {
        c->tw[d] = (double2*)at(12 + d);
        c->kv[d] = (double*)at(15 + d);
        c->vv[d] = (double*)at(18 + d);
    }
    c->nodes = (double*)at(21);
    c->partials = (double*)at(22);
    c->fft_partials = (double*)at(23);
    c->ls_partials = (double*)at(25);
    c->nblk_pw = (int)std::min<long long>((c->N + bec::kPwThreads - 1) / bec::kPwThreads, bec::kPwDefaultBlocks);
    c->nblk_x = bec::fft_blocks(c->n[0], c->fft_var[0][1], (long long)c->n[1] * c->n[2]);
}

// Twiddles W_L^m and wavenumbers per axis, then the parameter tables
// (synchronises the context stream).
bec_status ctx_tables(bec_ctx* c)
{
    for (int d = 0; d < 3; ++d) {
        const int L = c->n[d];
        std::vector<double2> tw(L);
        std::vector<double> kv(L);
        for (int m = 0; m < L; ++m) {
            const long double a = -2.0L * kPiL * (long double)m / (long double)L;
            tw[m] = make_double2((double)cosl(a), (double)sinl(a));
            const int jj = m < L / 2 ? m : m - L;
            kv[m] = (double)(2.0L * kPiL * jj / (long double)c->L[d]);
        }
        HIPCHK(hipMemcpyAsync(c->tw[d], tw.data(), L * sizeof(double2), hipMemcpyHostToDevice, c->st));
        HIPCHK(hipMemcpyAsync(c->kv[d], kv.data(), L * sizeof(double), hipMemcpyHostToDevice, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
    }
    return upload_params(c, true);
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* bec_last_error(void) { return g_err.c_str(); }

bec_status bec_gauss_legendre(int32_t n, double* u, double* w)
{
    if (n < 1 || n > bec::kMaxNodes || !u || !w) return fail(BEC_EINVAL, "need 1 <= n <= %d and output arrays", bec::kMaxNodes);
    std::vector<double> uu, ww;
    gauss_legendre01(n, uu, ww);
    std::memcpy(u, uu.data(), n * sizeof(double));
    std::memcpy(w, ww.data(), n * sizeof(double));
    return BEC_OK;
}

bec_status bec_params_from_physical(const bec_physical* in, bec_params* out, double* length_m)
{
    // CODATA 2018: hbar (exact h / 2 pi), mu_0, Bohr magneton, Bohr radius, atomic mass unit
    constexpr double kHbar = 1.054571817e-34, kMu0 = 1.25663706212e-6, kMuB = 9.2740100783e-24;
    constexpr double kA0 = 5.29177210903e-11, kAmu = 1.66053906660e-27, kPi = 3.14159265358979323846;
    if (!in || !out) return fail(BEC_EINVAL, "in and out must not be null");
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!pos(in->mass_amu) || !pos(in->f0_hz) || !pos(in->N[0]) || !pos(in->N[1]) || !pos(in->r_cut_um))
        return fail(BEC_EINVAL, "mass, unit frequency, atom numbers and cutoff must be finite and positive");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(in->trap_hz[d]) || in->trap_hz[d] < 0.0)
            return fail(BEC_EINVAL, "trap frequencies must be finite and >= 0");
    for (int i = 0; i < 2; ++i) {
        if (!std::isfinite(in->mu_bohr[i])) return fail(BEC_EINVAL, "non-finite magnetic moment");
        for (int j = 0; j < 2; ++j)
            if (!std::isfinite(in->a_bohr[i][j])) return fail(BEC_EINVAL, "non-finite scattering length");
    }
    if (in->a_bohr[0][1] != in->a_bohr[1][0]) return fail(BEC_EINVAL, "a_12 and a_21 must be equal");
    if (!std::isfinite(in->c_lhy)) return fail(BEC_EINVAL, "non-finite c_lhy");
    if (in->contact_2pi != 0 && in->contact_2pi != 1) return fail(BEC_EINVAL, "contact_2pi must be 0 or 1");
    if (in->dip_cut != 0 && in->dip_cut != 1) return fail(BEC_EINVAL, "dip_cut must be 0 or 1");

    const double m = in->mass_amu * kAmu, w0 = 2.0 * kPi * in->f0_hz;
    const double l = std::sqrt(kHbar / (m * w0));
    const double cg = (in->contact_2pi ? 2.0 : 4.0) * kPi;
    const double dd = kMu0 * kMuB * kMuB / (3.0 * l * l * l * kHbar * w0);
    bec_params p{};
    for (int i = 0; i < 2; ++i) {
        p.N[i] = in->N[i];
        for (int j = 0; j < 2; ++j) {
            p.G[i][j] = cg * (in->a_bohr[i][j] * kA0 / l) * in->N[j];
            p.Gdd[i][j] = dd * in->mu_bohr[i] * in->mu_bohr[j] * in->N[j];
        }
    }
    for (int d = 0; d < 3; ++d) p.omega[d] = in->trap_hz[d] / in->f0_hz;
    p.c_lhy = in->c_lhy;
    p.r_cut = in->r_cut_um * 1e-6 / l;
    p.dip_cut = in->dip_cut;
    p.n_u = in->n_u;
    STCHK(check_params(&p));
    *out = p;
    if (length_m) *length_m = l;
    return BEC_OK;
}

bec_status bec_workspace_size(const bec_grid* grid, const bec_params* params, size_t* bytes)
{
    STCHK(check_grid(grid));
    if (params) STCHK(check_params(params));
    if (params) STCHK(check_params_grid(grid, params));
    if (!bytes) return fail(BEC_EINVAL, "bytes is null");
    *bytes = ws_layout(grid->n, nullptr);
    return BEC_OK;
}

bec_status bec_create(const bec_grid* grid, const bec_params* params, void* hip_stream, void* workspace,
                      size_t workspace_bytes, bec_ctx** out)
{
    try {
        STCHK(check_grid(grid));
        STCHK(check_params(params));
        STCHK(check_params_grid(grid, params));
        if (!out) return fail(BEC_EINVAL, "out is null");
        if (!workspace) return fail(BEC_EINVAL, "workspace is null");
        if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(BEC_EINVAL, "workspace must be 256-byte aligned");
        size_t off[32];
        const size_t need = ws_layout(grid->n, off);
        if (workspace_bytes < need)
            return fail(BEC_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
        bec_ctx* c = new bec_ctx();
        ctx_attach(c, grid, params, hip_stream, static_cast<char*>(workspace), off);
        // reduced scalars: the final-reduction kernels write straight into pinned
        // host memory, so reading them back needs a stream synchronisation only
        if (hipHostMalloc((void**)&c->host, kScalSlots * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            delete c;
            return fail(BEC_EHIP, "hipHostMalloc of the scalar buffer failed");
        }
        if (hipHostGetDevicePointer((void**)&c->scal, c->host, 0) != hipSuccess) {
            (void)hipHostFree(c->host);
            delete c;
            return fail(BEC_EHIP, "hipHostGetDevicePointer of the scalar buffer failed");
        }
        bec_status st = ctx_tables(c);
        if (st != BEC_OK) {
            (void)hipHostFree(c->host);
            delete c;
            return st;
        }
        *out = c;
        return BEC_OK;
    } catch (...) {
        return fail(BEC_EINVAL, "unexpected host exception in bec_create");
    }
}

bec_status bec_get_tuning(bec_ctx* c, bec_tuning* t)
{
    if (!c || !t) return fail(BEC_EINVAL, "null argument");
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 2; ++k) t->fft_variant[a][k] = c->fft_var[a][k];
    t->pw_blocks = c->nblk_pw;
    t->lhy_table = c->lhy_table_on;
    t->lhy_terms = c->P.lhy_K;
    t->kin_axes = c->kin_axes_on;
    t->fuse_z = c->fuse_z;
    return BEC_OK;
}

bec_status bec_set_tuning(bec_ctx* c, const bec_tuning* t)
{
    if (c) c->resume.valid = false;   // the context's buffers change
    if (!c || !t) return fail(BEC_EINVAL, "null argument");
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 2; ++k)
            if (t->fft_variant[a][k] < 0 || t->fft_variant[a][k] >= bec::fft_num_variants(c->n[a]))
                return fail(BEC_EINVAL, "axis %d has no plan variant %d", a, t->fft_variant[a][k]);
    const long long cap = std::min<long long>((c->N + bec::kPwThreads - 1) / bec::kPwThreads, bec::kPwMaxBlocks);
    if (t->pw_blocks < 1 || t->pw_blocks > cap) return fail(BEC_EINVAL, "pw_blocks must be in 1..%lld", cap);
    if (t->fuse_z < 0 || t->fuse_z > 3) return fail(BEC_EINVAL, "fuse_z must be in 0..3");
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 2; ++k) c->fft_var[a][k] = t->fft_variant[a][k];
    c->nblk_pw = t->pw_blocks;
    c->P.nblk_pw = c->nblk_pw;
    c->lhy_table_on = t->lhy_table != 0;
    c->P.lhy_K = c->lhy_table_on ? c->lhy_K_built : 0;
    c->kin_axes_on = t->kin_axes != 0;
    c->fuse_z = t->fuse_z;
    c->nblk_x = bec::fft_blocks(c->n[0], c->fft_var[0][1], (long long)c->n[1] * c->n[2]);
    return BEC_OK;
}

bec_status bec_fft_variant_count(int32_t L, int32_t* count)
{
    if (!count) return fail(BEC_EINVAL, "null argument");
    *count = bec::fft_num_variants(L);
    return *count > 0 ? BEC_OK : fail(BEC_EUNSUPPORTED, "length %d not supported", L);
}

bec_status bec_time_fft_pass(bec_ctx* c, int32_t axis, int32_t kind, int32_t variant, int32_t reps, double* ms_out)
{
    if (c) c->resume.valid = false;   // the context's buffers change
    if (!c || !ms_out) return fail(BEC_EINVAL, "null argument");
    if (axis < 0 || axis > 2 || kind < 0 || kind > 2 || (kind == 2 && axis != 0) || reps < 1)
        return fail(BEC_EINVAL, "bad axis / kind / reps");
    if (variant < 0 || variant >= bec::fft_num_variants(c->n[axis]))
        return fail(BEC_EINVAL, "axis %d has no plan variant %d", axis, variant);
    const long long N = c->N;
    const double2* src[3] = {c->W, c->W + N, c->W + 2 * N};
    double2* dst[3] = {c->W, c->W + N, c->W + 2 * N};
    const int ops[3] = {bec::kOpMulKin, bec::kOpMulKin, bec::kOpMulDip};
    const int saved = c->fft_var[axis][kind == 2 ? 1 : 0];
    c->fft_var[axis][kind == 2 ? 1 : 0] = variant;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    bec_status st = BEC_OK;
    const int sign = kind == 1 ? +1 : -1;
    st = run_pass(c, axis, src, dst, 3, sign, 1.0, kind == 2 ? ops : nullptr, nullptr);   // warm-up
    if (st == BEC_OK && hipEventRecord(e0, c->st) != hipSuccess) st = fail(BEC_EHIP, "event record");
    for (int r = 0; r < reps && st == BEC_OK; ++r)
        st = run_pass(c, axis, src, dst, 3, sign, 1.0, kind == 2 ? ops : nullptr, nullptr);
    float ms = 0.f;
    if (st == BEC_OK && (hipEventRecord(e1, c->st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = fail(BEC_EHIP, "event timing");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->fft_var[axis][kind == 2 ? 1 : 0] = saved;
    if (st == BEC_OK) *ms_out = ms / reps;
    return st;
}

bec_status bec_profile_enable(bec_ctx* c, int32_t on)
{
    if (!c) return fail(BEC_EINVAL, "ctx is null");
    STCHK(prof_flush(c));
    if (on) {
        c->prof.names.clear();
        c->prof.launches.clear();
        c->prof.total_ms.clear();
        c->prof.total_bytes.clear();
    }
    c->prof.on = on != 0;
    return BEC_OK;
}

bec_status bec_profile_read(bec_ctx* c, bec_kernel_stat* out_h, int32_t cap, int32_t* n_out)
{
    if (!c || !n_out || (cap > 0 && !out_h)) return fail(BEC_EINVAL, "null argument");
    STCHK(prof_flush(c));
    const Prof& P = c->prof;
    const int n = (int)P.names.size();
    for (int i = 0; i < n && i < cap; ++i) {
        std::memset(out_h[i].name, 0, sizeof(out_h[i].name));
        std::strncpy(out_h[i].name, P.names[i].c_str(), sizeof(out_h[i].name) - 1);
        out_h[i].launches = P.launches[i];
        out_h[i].total_ms = P.total_ms[i];
        out_h[i].total_bytes = P.total_bytes[i];
    }
    *n_out = n;
    return BEC_OK;
}

bec_status bec_destroy(bec_ctx* ctx)
{
    if (!ctx) return BEC_OK;
    (void)prof_flush(ctx);
    for (hipEvent_t e : ctx->prof.pool) (void)hipEventDestroy(e);
    if (ctx->host) (void)hipHostFree(ctx->host);
    delete ctx;
    return BEC_OK;
}

bec_status bec_set_params(bec_ctx* c, const bec_params* params)
{
    if (c) c->resume.valid = false;   // the context's buffers change
    if (!c) return fail(BEC_EINVAL, "ctx is null");
    STCHK(check_params(params));
    STCHK(check_params_grid(&c->g, params));
    const bool dip = params->r_cut != c->p.r_cut || params->dip_cut != c->p.dip_cut;
    c->p = *params;
    return upload_params(c, dip);
}

bec_status bec_fft3d(bec_ctx* c, const double* in, double* out, int32_t nfield, int32_t sign)
{
    if (c) c->resume.valid = false;   // the context's buffers change
    if (!c || !in || !out) return fail(BEC_EINVAL, "null argument");
    if (nfield < 1 || nfield > 3) return fail(BEC_EINVAL, "nfield must be 1..3");
    if (sign != -1 && sign != 1) return fail(BEC_EINVAL, "sign must be -1 or +1");
    const double2* src[3];
    double2* dst[3];
    for (int f = 0; f < nfield; ++f) {
        src[f] = reinterpret_cast<const double2*>(in) + f * c->N;
        dst[f] = reinterpret_cast<double2*>(out) + f * c->N;
    }
    return fft3d_plain(c, src, dst, nfield, sign);
}

bec_status bec_energy(bec_ctx* c, const double* psi, bec_terms* out_h)
{
    if (c) c->resume.valid = false;   // the context's buffers change
    if (!c || !psi || !out_h) return fail(BEC_EINVAL, "null argument");
    Eval ev;
    STCHK(heval(c, reinterpret_cast<const double2*>(psi), nullptr, kOne, kZero, 0, &ev));
    STCHK(residual_norms(c, 0, &ev));
    *out_h = ev.t;
    return BEC_OK;
}

bec_status bec_hamiltonian(bec_ctx* c, const double* psi, double* hpsi, bec_terms* out_h)
{
    if (c) c->resume.valid = false;   // the context's buffers change
    if (!c || !psi || !hpsi) return fail(BEC_EINVAL, "null argument");
    Eval ev;
    STCHK(heval(c, reinterpret_cast<const double2*>(psi), nullptr, kOne, kZero, 0, &ev));
    STCHK(residual_norms(c, 0, &ev));
    HIPCHK(hipMemcpyAsync(hpsi, c->hpsi[0], 2 * c->N * sizeof(double2), hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (out_h) *out_h = ev.t;
    return BEC_OK;
}

bec_status bec_gradient(bec_ctx* c, const double* psi, double* grad, int32_t projected, bec_terms* out_h)
{
    if (c) c->resume.valid = false;   // the context's buffers change
    if (!c || !psi || !grad) return fail(BEC_EINVAL, "null argument");
    Eval ev;
    STCHK(heval(c, reinterpret_cast<const double2*>(psi), nullptr, kOne, kZero, 0, &ev));
    STCHK(residual_norms(c, 0, &ev));
    HIPCHK(bec::launch_grad(c->P, c->psi[0], c->hpsi[0], reinterpret_cast<double2*>(grad), ev.t.mu[0], ev.t.mu[1],
                            2.0 * c->p.N[0] * c->dV, 2.0 * c->p.N[1] * c->dV, projected ? 1 : 0, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (out_h) *out_h = ev.t;
    return BEC_OK;
}

bec_status bec_energy_gradient_async(bec_ctx* c, const double* psi, double* grad, double* E_dev)
{
    if (c) c->resume.valid = false;   // the context's buffers change
    if (!c || !psi || !grad || !E_dev) return fail(BEC_EINVAL, "null argument");
    STCHK(heval_launch(c, reinterpret_cast<const double2*>(psi), nullptr, kOne, kZero, nullptr, 0));
    HIPCHK(bec::launch_grad(c->P, c->psi[0], c->hpsi[0], reinterpret_cast<double2*>(grad), 0.0, 0.0,
                            2.0 * c->p.N[0] * c->dV, 2.0 * c->p.N[1] * c->dV, 0, c->st));
    HIPCHK(bec::launch_energy_from_sums(c->P, c->dscal + kScalHeval, c->dV, E_dev, c->st));
    return BEC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// bec_gradient_noalloc: the workspace of a context (fields, FFT work area,
// tables, partial sums) and the reduced scalars live in this array instead of
// caller or pinned host memory.  Every GPU the library runs on holds its own
// copy from module load until the process ends.  In host code `scratch` names a
// host-side stand-in: its device address on the current device comes from
// hipGetSymbolAddress and only that address is handed to kernels and copies.
static __device__ __align__(256) char scratch[BEC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
struct NoAllocDevice {
    std::mutex lock;          // calls on one device run one at a time
    char* ptr = nullptr;      // device address of `scratch` on this device
};
NoAllocDevice g_noalloc[kMaxDevices];

}  // namespace

extern "C" {

bec_status bec_gradient_noalloc(const bec_grid* grid, const bec_params* params, void* hip_stream, const double* psi,
                                double* grad, int32_t projected, bec_terms* out_h)
{
    try {
        STCHK(check_grid(grid));
        STCHK(check_params(params));
        STCHK(check_params_grid(grid, params));
        if (!psi || !grad) return fail(BEC_EINVAL, "null argument");
        size_t off[32];
        const size_t ws = ws_layout(grid->n, off);
        const size_t need = ws + align256(kScalSlots * sizeof(double));
        if (need > sizeof(scratch))
            return fail(BEC_ENOMEM, "grid %dx%dx%d needs %zu bytes, the static scratch of bec_gradient_noalloc has %zu",
                        grid->n[0], grid->n[1], grid->n[2], need, sizeof(scratch));
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        if (dev < 0 || dev >= kMaxDevices) return fail(BEC_EUNSUPPORTED, "device index %d beyond %d", dev, kMaxDevices);
        NoAllocDevice& D = g_noalloc[dev];
        std::lock_guard<std::mutex> guard(D.lock);
        if (!D.ptr) {   // once per device, with that device current
            void* p = nullptr;
            HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            D.ptr = static_cast<char*>(p);
        }
        // a context on the host stack whose workspace is the device's scratch;
        // every table it needs is rebuilt here, no buffer has to start at zero
        bec_ctx c;
        double host[kScalSlots];
        ctx_attach(&c, grid, params, hip_stream, D.ptr, off);
        c.scal = reinterpret_cast<double*>(D.ptr + ws);
        c.host = host;
        c.scal_on_device = true;
        STCHK(ctx_tables(&c));
        Eval ev;
        STCHK(heval(&c, reinterpret_cast<const double2*>(psi), nullptr, kOne, kZero, 0, &ev));
        STCHK(residual_norms(&c, 0, &ev));
        HIPCHK(bec::launch_grad(c.P, c.psi[0], c.hpsi[0], reinterpret_cast<double2*>(grad), ev.t.mu[0], ev.t.mu[1],
                                2.0 * c.p.N[0] * c.dV, 2.0 * c.p.N[1] * c.dV, projected ? 1 : 0, c.st));
        HIPCHK(hipStreamSynchronize(c.st));
        c.host = nullptr;   // not owned
        if (out_h) *out_h = ev.t;
        return BEC_OK;
    } catch (...) {
        return fail(BEC_EINVAL, "unexpected host exception in bec_gradient_noalloc");
    }
}

bec_status bec_precond_apply_blend(bec_ctx* c, double blend, double sigma, const double* psi, const double* r,
                                   double* z)
{
    if (c) c->resume.valid = false;   // the context's buffers change
    if (!c || !psi || !r || !z) return fail(BEC_EINVAL, "null argument");
    if (!(sigma >= 0)) return fail(BEC_EINVAL, "sigma must be >= 0");
    if (!(blend <= 1.0)) return fail(BEC_EINVAL, "blend must be <= 1 (negative: adaptive)");
    Eval ev;
    STCHK(heval(c, reinterpret_cast<const double2*>(psi), nullptr, kOne, kZero, 0, &ev));
    STCHK(compute_z(c, 0, ev, reinterpret_cast<const double2*>(r), 0, sigma));    // P_Delta^-1 r into c->z
    bec::MakeRArgs m{};
    m.psi = c->psi[0];
    m.aux = c->aux[0];
    m.rin = reinterpret_cast<const double2*>(r);
    for (int i = 0; i < 2; ++i) m.diag_shift[i] = ev.t.shift[i];
    m.sigma = sigma;
    m.apply_pv = 3;
    m.zk = c->z;
    bec::rule_blend(ev.sums, ev.t.shift, blend, m.blend_w);
    m.out = reinterpret_cast<double2*>(z);
    HIPCHK(bec::launch_make_r(c->P, m, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return BEC_OK;
}

bec_status bec_precond_apply(bec_ctx* c, int32_t pc, double sigma, const double* psi, const double* r, double* z)
{
    if (c) c->resume.valid = false;   // the context's buffers change
    if (!c || !psi || !r || !z) return fail(BEC_EINVAL, "null argument");
    if (pc < 0 || pc > 5) return fail(BEC_EINVAL, "unknown preconditioner %d", pc);
    if (!(sigma >= 0)) return fail(BEC_EINVAL, "sigma must be >= 0");
    if (pc == BEC_PC_BLEND) return bec_precond_apply_blend(c, -1.0, sigma, psi, r, z);
    Eval ev;
    STCHK(heval(c, reinterpret_cast<const double2*>(psi), nullptr, kOne, kZero, 0, &ev));
    const double2* rin = reinterpret_cast<const double2*>(r);
    double2* zout = reinterpret_cast<double2*>(z);
    if (pc == BEC_PC_NONE) {
        if (z != r) HIPCHK(hipMemcpyAsync(z, r, 2 * c->N * sizeof(double2), hipMemcpyDeviceToDevice, c->st));
    } else if (pc == BEC_PC_V) {
        bec::MakeRArgs m{};
        m.psi = c->psi[0];
        m.aux = c->aux[0];
        m.rin = rin;
        for (int i = 0; i < 2; ++i) m.diag_shift[i] = ev.t.shift[i];
        m.sigma = sigma;
        m.apply_pv = 1;
        m.out = zout;
        HIPCHK(bec::launch_make_r(c->P, m, c->st));
    } else {
        const int pv = pc == BEC_PC_COMPOSITE ? 1 : (pc == BEC_PC_SYMMETRIC ? 2 : 0);
        STCHK(compute_z(c, 0, ev, rin, pv, sigma));
        if (pc == BEC_PC_SYMMETRIC) {   // the outer D^-1/2
            bec::MakeRArgs m{};
            m.psi = c->psi[0];
            m.aux = c->aux[0];
            m.rin = c->z;
            for (int i = 0; i < 2; ++i) m.diag_shift[i] = ev.t.shift[i];
            m.sigma = sigma;
            m.apply_pv = 2;
            m.out = zout;
            HIPCHK(bec::launch_make_r(c->P, m, c->st));
        } else {
            HIPCHK(hipMemcpyAsync(z, c->z, 2 * c->N * sizeof(double2), hipMemcpyDeviceToDevice, c->st));
        }
    }
    HIPCHK(hipStreamSynchronize(c->st));
    return BEC_OK;
}

bec_status bec_linesearch(bec_ctx* c, const double* psi, const double* d, double* psi_out, const bec_opts* o,
                          bec_ls_report* out_h)
{
    if (c) c->resume.valid = false;   // the context's buffers change
    if (!c || !psi || !d || !psi_out || !o) return fail(BEC_EINVAL, "null argument");
    if (psi_out == psi) return fail(BEC_EINVAL, "psi_out may not alias psi");
    Eval ev;
    STCHK(heval(c, reinterpret_cast<const double2*>(psi), nullptr, kOne, kZero, 0, &ev));
    bec::DirArgs A = dir_args(c, 0, ev, 2, 0.0);
    A.zbuf = reinterpret_cast<const double2*>(d);
    double R[bec::kDirReduceSums];
    STCHK(dir_reduce(c, A, R));
    A.zsign = 1.0;
    A.c[0] = c->dV * R[3];
    A.c[1] = c->dV * R[9];
    Model m;
    // step of the model: -E'/E'' when it has a minimum, else 0.1 / max|p_i|, capped at theta_max
    STCHK(direction_and_model(c, A, ev, 0.0, o->theta_max, &m));
    const double pmax = std::max(m.pnorm[0], m.pnorm[1]);
    if (!(pmax > 0)) return fail(BEC_EINVAL, "direction has no tangent component");
    double alpha = m.alpha;
    const double tau = o->tau_rel * std::fabs(ev.t.E);
    double a[2], b[2];
    Eval tr;
    int trials = 0, path = 0;
    bool ok = false;
    STCHK(heval(c, c->psi[0], c->pdir, m.a, m.b, 1, &tr));
    ++trials;
    if (tr.t.E <= ev.t.E + tau) ok = true;
    for (int k = 0; !ok && k < o->max_backtrack; ++k) {
        alpha *= 0.5;
        geodesic_coeffs(ev, m, alpha, a, b);
        STCHK(heval(c, c->psi[0], c->pdir, a, b, 1, &tr));
        ++trials;
        path |= 1;
        if (tr.t.E <= ev.t.E + o->armijo_c1 * alpha * m.E1 + tau) ok = true;
    }
    HIPCHK(hipMemcpyAsync(psi_out, c->psi[1], 2 * c->N * sizeof(double2), hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (out_h) {
        out_h->E0 = ev.t.E;
        out_h->E1 = m.E1;
        out_h->E2 = m.E2;
        out_h->alpha = alpha;
        out_h->theta[0] = alpha * m.pnorm[0];
        out_h->theta[1] = alpha * m.pnorm[1];
        out_h->E_new = tr.t.E;
        out_h->pnorm[0] = m.pnorm[0];
        out_h->pnorm[1] = m.pnorm[1];
        out_h->n_trials = trials;
        out_h->path = path;
    }
    return ok ? BEC_OK : fail(BEC_ESTAGNATED, "no decrease along the geodesic");
}

bec_status bec_solve(bec_ctx* c, double* psi_inout, const bec_opts* o, bec_report* out_h, bec_iter* log_h,
                     int32_t log_cap)
{
    if (!c || !psi_inout || !o) return fail(BEC_EINVAL, "null argument");
    const bool resumable = c->resume.valid;
    c->resume.valid = false;
    if (o->pc < 0 || o->pc > 5 || o->beta < 0 || o->beta > 2) return fail(BEC_EINVAL, "bad options");
    if (!(o->blend <= 1.0)) return fail(BEC_EINVAL, "blend must be <= 1 (negative: adaptive)");
    if (o->flags & ~(BEC_SOLVE_SYNCHRONOUS | BEC_SOLVE_CONTINUE))
        return fail(BEC_EINVAL, "unknown bits in opts.flags: 0x%x", o->flags);
    if (o->stall_window < 0) return fail(BEC_EINVAL, "stall_window must be >= 0");
    const bool cont = (o->flags & BEC_SOLVE_CONTINUE) != 0;
    if (cont) {
        const bec_opts& q = c->resume.o;
        if (!resumable)
            return fail(BEC_EINVAL, "BEC_SOLVE_CONTINUE: the last call on this context was not a solve stopped at "
                                    "its max_iter");
        if (q.pc != o->pc || q.beta != o->beta || q.restart_period != o->restart_period || q.sigma != o->sigma ||
            q.blend != o->blend || ((q.flags ^ o->flags) & BEC_SOLVE_SYNCHRONOUS))
            return fail(BEC_EINVAL, "BEC_SOLVE_CONTINUE: pc, beta, restart_period, sigma, blend and the "
                                    "synchronous bit must be those of the solve it continues");
    }
    const auto t0 = std::chrono::steady_clock::now();
    const double dV = c->dV;
    const bec_params& p = c->p;
    const double Ntot = p.N[0] + p.N[1];
    const double wS[2] = {(p.N[0] / Ntot) * (p.N[0] / Ntot), (p.N[1] / Ntot) * (p.N[1] / Ntot)};
    bec_report rep{};
    int cur = 0;
    Eval ev;
    bool have_prev = false;
    int n = 0, stall_it = 0;
    bec_status status = BEC_ENOTCONV;
    double E_prev = NAN, alpha_prev = 0.0, rz_old = 0.0, stall_ref = INFINITY;
    const int zmode_pc = o->pc == BEC_PC_V ? 1
                         : o->pc == BEC_PC_NONE ? 0
                         : o->pc == BEC_PC_SYMMETRIC ? 3
                         : o->pc == BEC_PC_BLEND ? 4 : 2;
    // Pipelined iterations: the first trial of a step is enqueued at the step
    // the device decides from the model sums, followed by the preconditioned
    // residual (Fourier / composite preconditioners, into z_next) and the
    // direction reduce of the trial state and, from there, the next direction
    // write with the device's beta; the host waits once, for the part before
    // that write, and checks every decision afterwards.  A step that needs a
    // restart or a backtrack falls back to host-synchronised launches; the
    // speculative work then only touched buffers the fallback rewrites.
    const bool pipe = !(o->flags & BEC_SOLVE_SYNCHRONOUS);
    const int pv_mode = o->pc == BEC_PC_COMPOSITE ? 1 : (o->pc == BEC_PC_SYMMETRIC ? 2 : 0);
    auto beta_rule = [&](int iter, bool prev, double rz_prev) {
        bec::BetaRule br{};
        br.restart = !prev || o->beta == BEC_BETA_ZERO || (o->restart_period > 0 && iter % o->restart_period == 0);
        br.mode = o->beta == BEC_BETA_PR_PLUS ? 1 : 0;
        br.rz_old = rz_prev;
        br.w[0] = wS[0];
        br.w[1] = wS[1];
        br.dV = dV;
        return br;
    };
    double R[bec::kDirReduceSums];
    bool R_ready = false;      // R holds the direction-reduce sums of the current state
    bool spec_write = false;   // the current state's direction write (device beta) is already enqueued
    if (cont) {   // the state the last solve stopped at: its z and reduce sums are current
        const auto& s = c->resume;
        cur = s.cur;
        n = s.n;
        stall_it = s.stall_it;
        have_prev = s.have_prev;
        spec_write = s.spec_write;
        E_prev = s.E_prev;
        alpha_prev = s.alpha_prev;
        rz_old = s.rz_old;
        stall_ref = s.stall_ref;
        std::memcpy(R, s.R, sizeof(R));
        R_ready = true;
        ev.t = s.t;
        std::memcpy(ev.sums, s.sums, sizeof(ev.sums));
    } else {
        STCHK(normalise_into(c, reinterpret_cast<const double2*>(psi_inout), 0));
        STCHK(heval(c, c->psi[0], nullptr, kOne, kZero, 0, &ev));
    }
    const int n0 = n;   // steps before this call

    for (;;) {
        // 1. residual, preconditioned residual and the conjugacy sums
        if (zmode_pc >= 2 && !R_ready) STCHK(compute_z(c, cur, ev, nullptr, pv_mode, o->sigma));
        bec::DirArgs A = dir_args(c, cur, ev, zmode_pc, o->sigma);
        A.blend = o->blend;
        bec::rule_blend(ev.sums, ev.t.shift, o->blend, A.blend_w);
        A.have_prev = have_prev;
        if (!R_ready) STCHK(dir_reduce(c, A, R));
        R_ready = false;
        ev.t.res[0] = std::sqrt(dV * R[0]);
        ev.t.res[1] = std::sqrt(dV * R[6]);
        const double res_max = std::max(ev.t.res[0], ev.t.res[1]);
        if (!std::isfinite(res_max) || !std::isfinite(ev.t.E)) { status = BEC_ENONFINITE; break; }
        if (res_max < o->tol_grad) { status = BEC_OK; break; }
        if (o->tol_dE > 0 && n > 0 && std::fabs(ev.t.E - E_prev) < o->tol_dE) { status = BEC_OK; break; }
        if (res_max < 0.5 * stall_ref) {
            stall_ref = res_max;
            stall_it = n;
        } else if (o->stall_window > 0 && n - stall_it >= o->stall_window) {
            status = BEC_ESTALLED;
            break;
        }
        if (n - n0 >= o->max_iter) { status = BEC_ENOTCONV; break; }

        // 2. beta (HS+ or PR+), restarts (Sec. IV.C)
        const double beta = bec::rule_beta(R, beta_rule(n, have_prev, rz_old));
        double rz_now = wS[0] * dV * R[5] + wS[1] * dV * R[11];
        int level = beta > 0 ? 0 : 1, path = 0, trials = 0;
        bool accepted = false, stagnated = false, first = true, tried = false, next_ready = false;
        double alpha = 0.0;
        double Rn[bec::kDirReduceSums];
        Model m{};
        Eval tr;
        bec_status hs = BEC_OK;
        while (!accepted && !stagnated) {
            // 3. direction d = -z + beta p_old, projected; restart when <r,p> >= 0
            for (;;) {
                const double b = level == 0 ? beta : 0.0;
                if (level >= 2) {
                    A = dir_args(c, cur, ev, level == 2 ? 1 : 0, o->sigma);
                    A.have_prev = false;
                    STCHK(dir_reduce(c, A, R));
                }
                A.beta = b;
                A.zsign = -1.0;
                bec::rule_proj(R, b, dV, A.c);
                if (!(first && spec_write)) STCHK(dir_write_launch(c, A));
                // the scalar slots the pipelined part writes: model, Parseval, energy, reduce, step
                const ScalRange waits[] = {{kScalModel, bec::kDirWriteSums + bec::kLsEpiSums},
                                           {kScalModel + kParsevalOut, 2},
                                           {kScalHeval, bec::kHevalSums},
                                           {kScalDir, bec::kDirReduceSums},
                                           {kScalStep, bec::kStepOut}};
                if (first && pipe) arm_scalars(c->host, waits, 5);
                // 4. the closed-form step of the second-order model (Sec. V), decided on the device
                STCHK(model_launch(c, ev.t.norm2, alpha_prev, o->theta_max));
                if (first && pipe) {
                    // 5a. the trial at the device's step, the reduce of the state it
                    // reaches and the next direction write, then one wait
                    const int nxt = 1 - cur;
                    STCHK(heval_launch(c, c->psi[cur], c->pdir, nullptr, nullptr, c->dscal + kScalStep, nxt));
                    bec::DirArgs An = dir_args(c, nxt, ev, zmode_pc, o->sigma);
                    An.blend = o->blend;            // weights from the device sums (dev_state)
                    An.dev_state = c->dscal + kScalHeval;
                    An.have_prev = 1;
                    An.r_old = c->r_new;      // r and p of this step: the pair after the swap
                    An.p = c->pdir;
                    An.p_out = c->pold;
                    An.r_out = c->r_old;
                    if (zmode_pc >= 2) {   // z of the trial state into the spare buffer
                        STCHK(compute_z(c, nxt, ev, nullptr, pv_mode, o->sigma, c->z_next, c->dscal + kScalHeval));
                        An.zbuf = c->z_next;
                    }
                    STCHK(dir_reduce_launch(c, An));
                    An.rule = beta_rule(n + 1, true, rz_now);
                    An.dev_dir = c->dscal + kScalDir;
                    An.zsign = -1.0;
                    STCHK(dir_write_launch(c, An));
                    if (!await_scalars(c->host, waits, 5, 120.0)) {
                        HIPCHK(hipStreamSynchronize(c->st));   // reports a device error if there is one
                        if (!await_scalars(c->host, waits, 5, 0.0))
                            return fail(BEC_EHIP, "reduced scalars did not arrive");
                    }
                    model_read(c, &m);
                    hs = heval_read(c, &tr);
                    std::memcpy(Rn, c->host + kScalDir, sizeof(Rn));
                    tried = true;
                } else {
                    STCHK(fetch(c, 0));
                    model_read(c, &m);
                }
                first = false;
                if (m.rp < 0 && std::isfinite(m.rp)) break;
                tried = false;
                if (level == 0) { level = 1; rep.n_restarts++; continue; }
                if (level == 1 && o->pc >= BEC_PC_COMPOSITE) { level = 2; path |= 4; continue; }
                if (level == 2) { level = 3; continue; }
                stagnated = true;
                break;
            }
            if (stagnated) break;
            rz_now = wS[0] * dV * R[5] + wS[1] * dV * R[11];

            // 5. validate along the exact geodesic, Armijo halving
            alpha = m.alpha;
            const double tau = o->tau_rel * std::fabs(ev.t.E);
            if (!tried) {
                STCHK(heval_launch(c, c->psi[cur], c->pdir, nullptr, nullptr, c->dscal + kScalStep, 1 - cur));
                STCHK(fetch(c, 0));
                hs = heval_read(c, &tr);
            }
            if (hs != BEC_OK && hs != BEC_ENONFINITE) return hs;
            ++trials;
            if (hs == BEC_OK && tr.t.E <= ev.t.E + tau) {
                accepted = true;
                next_ready = tried;
            } else {
                double a[2], bb[2];
                for (int k = 0; k < o->max_backtrack; ++k) {
                    alpha *= 0.5;
                    geodesic_coeffs(ev, m, alpha, a, bb);
                    hs = heval(c, c->psi[cur], c->pdir, a, bb, 1 - cur, &tr);
                    if (hs != BEC_OK && hs != BEC_ENONFINITE) return hs;
                    ++trials;
                    rep.n_backtracks++;
                    if (hs == BEC_OK && tr.t.E <= ev.t.E + o->armijo_c1 * alpha * m.E1 + tau) {
                        accepted = true;
                        path |= 1;
                        break;
                    }
                }
            }
            tried = false;
            if (!accepted) {
                if (level == 0) { level = 1; rep.n_restarts++; path |= 2; continue; }
                stagnated = true;
            }
        }
        if (stagnated) { status = BEC_ESTAGNATED; break; }

        // 6. accept
        if (log_h && n - n0 < log_cap) {
            bec_iter& L = log_h[n - n0];
            L.iter = n;
            L.n_trials = trials;
            L.restarted = level >= 1;
            L.path = path;
            L.E = tr.t.E;
            L.res_max = res_max;
            L.E1 = m.E1;
            L.E2 = m.E2;
            L.alpha = alpha;
            L.beta = level == 0 ? beta : 0.0;
        }
        E_prev = ev.t.E;
        ev = tr;
        cur = 1 - cur;
        std::swap(c->pdir, c->pold);
        std::swap(c->r_old, c->r_new);
        rz_old = rz_now;
        alpha_prev = alpha;
        have_prev = true;
        ++n;
        // the speculative reduce and write were made for exactly this state
        R_ready = spec_write = next_ready;
        if (next_ready) {
            std::memcpy(R, Rn, sizeof(R));
            std::swap(c->z, c->z_next);
        }
    }
    HIPCHK(hipMemcpyAsync(psi_inout, c->psi[cur], 2 * c->N * sizeof(double2), hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (status == BEC_ENOTCONV) {   // stopped at max_iter: R (and z) belong to the current state
        auto& s = c->resume;
        s.o = *o;
        s.cur = cur;
        s.n = n;
        s.stall_it = stall_it;
        s.have_prev = have_prev;
        s.spec_write = spec_write;
        s.E_prev = E_prev;
        s.alpha_prev = alpha_prev;
        s.rz_old = rz_old;
        s.stall_ref = stall_ref;
        std::memcpy(s.R, R, sizeof(R));
        s.t = ev.t;
        std::memcpy(s.sums, ev.sums, sizeof(ev.sums));
        s.valid = true;
    }
    rep.iters = n - n0;
    rep.status = status;
    rep.final = ev.t;
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (out_h) *out_h = rep;
    if (status != BEC_OK && status != BEC_ENOTCONV)
        fail(status, status == BEC_ESTAGNATED ? "no descent after a beta = 0 restart"
                     : status == BEC_ESTALLED ? "the residual did not halve within stall_window steps"
                                              : "non-finite state");
    return status;
}

bec_status bec_ite_solve(bec_ctx* c, double* psi_inout, const bec_ite_opts* o, bec_report* out_h, double* log_E,
                         int32_t log_cap)
{
    if (c) c->resume.valid = false;   // the context's buffers change
    if (!c || !psi_inout || !o) return fail(BEC_EINVAL, "null argument");
    if (!(o->dt > 0.0) || !std::isfinite(o->dt) || o->max_iter < 0 || !(o->tol_dE >= 0.0))
        return fail(BEC_EINVAL, "need dt > 0, tol_dE >= 0, max_iter >= 0");
    const auto t0 = std::chrono::steady_clock::now();
    const long long N = c->N;
    const double dV = c->dV;
    const bec_params& p = c->p;
    bec_report rep{};
    if (o->flags & ~BEC_SOLVE_SYNCHRONOUS) return fail(BEC_EINVAL, "unknown bits in opts.flags: 0x%x", o->flags);
    const bool pipe = !(o->flags & BEC_SOLVE_SYNCHRONOUS);
    STCHK(normalise_into(c, reinterpret_cast<const double2*>(psi_inout), 0));
    // Step n reads the unnormalised output of step n - 1 (or the normalised
    // start), stores the normalised iterate psi^n in slot A(n) and
    // exp(-dt U) F^-1 exp(-dt T) F psi^n in slot B(n); the slots alternate
    // between (psi[0], psi[1]) and (hpsi[0], hpsi[1]), so a step enqueued ahead
    // of the host's convergence test never overwrites the iterate it returns.
    // Its sums go to scalar range R(n % 2) (host and device copies).
    auto slotA = [&](int k) { return (k & 1) ? c->hpsi[0] : c->psi[0]; };
    auto slotB = [&](int k) { return (k & 1) ? c->hpsi[1] : c->psi[1]; };
    auto region = [](int k) { return (k & 1) ? kScalIte1 : kScalIte0; };
    auto enqueue_step = [&](int k, const double a_host[2]) -> bec_status {
        bec::TrialZArgs z{};
        z.psi_src = k == 0 ? c->psi[0] : slotB(k - 1);
        z.p = nullptr;
        z.a[0] = a_host ? a_host[0] : 0.0;
        z.a[1] = a_host ? a_host[1] : 0.0;
        if (!a_host) {   // normalisation of step k - 1's output, decided on the device
            z.norm_sums = c->dscal + region(k - 1) + 12;
            z.norm_dV = dV;
        }
        z.psi_dst = slotA(k);
        z.N = N;
        double2* fdst[3] = {c->W, c->W + N, c->aux[0]};
        const int ops[3] = {bec::kOpExpKin, bec::kOpExpKin, bec::kOpMulDip};
        const double dts[3] = {o->dt, o->dt, 0.0};
        STCHK(kspace_apply_trial(c, z, fdst, ops, dts));
        bec::IteArgs ia{};
        ia.psi = slotA(k);
        ia.hat = c->W;
        ia.phi = c->aux[0];
        ia.out = slotB(k);
        ia.dt = o->dt;
        ia.partials = c->partials;
        LAUNCH(c, "ite_epilogue", (double)N * 112.0, bec::launch_ite_epi(c->P, ia, c->nblk_pw, c->st));
        const int rb = region(k);
        const bec::RedSeg s1{c->partials, c->nblk_pw, bec::kIteSums, c->scal + rb, c->dscal + rb};
        const bec::RedSeg s2{c->fft_partials, c->nblk_x, 2, c->scal + rb + bec::kIteSums,
                             c->dscal + rb + bec::kIteSums};
        const bec::RedSeg none{nullptr, 0, 0, nullptr, nullptr};
        LAUNCH(c, "reduce_final", 8.0 * (bec::kIteSums * c->nblk_pw + 2 * c->nblk_x),
               bec::launch_reduce_segs(s1, s2, none, c->st));
        return BEC_OK;
    };
    const double one[2] = {1.0, 1.0};
    int n = 0;
    bec_status status = BEC_ENOTCONV;
    double E_prev = NAN;
    double a[2] = {1.0, 1.0};
    {
        const ScalRange w0[] = {{region(0), bec::kIteSums + 2}};
        if (pipe) arm_scalars(c->host, w0, 1);
        STCHK(enqueue_step(0, one));
    }
    for (;;) {
        // step n + 1 goes ahead of the host's test of step n (unless step n is the last allowed)
        const bool ahead = pipe && n < o->max_iter;
        const ScalRange wn[] = {{region(n), bec::kIteSums + 2}};
        if (ahead) {
            const ScalRange wn1[] = {{region(n + 1), bec::kIteSums + 2}};
            arm_scalars(c->host, wn1, 1);
            STCHK(enqueue_step(n + 1, nullptr));
        }
        if (pipe) {
            if (!await_scalars(c->host, wn, 1, 120.0)) {
                HIPCHK(hipStreamSynchronize(c->st));
                if (!await_scalars(c->host, wn, 1, 0.0)) return fail(BEC_EHIP, "reduced scalars did not arrive");
            }
        } else {
            STCHK(fetch(c, 0));
        }
        const double* S = c->host + region(n);
        // energy of psi^n (Sec. II, Eq. (1)); kinetic part by Parseval of F psi^n
        double E = dV * S[9];
        for (int i = 0; i < 2; ++i) {
            E += p.N[i] * dV * (S[bec::kIteSums + i] / (double)N + S[i]);
            const double nn[2] = {i == 0 ? S[2] : S[3], i == 0 ? S[3] : S[4]};
            for (int j = 0; j < 2; ++j)
                E += 0.5 * p.N[i] * dV * (p.G[i][j] * nn[j] + p.Gdd[i][j] * S[5 + 2 * i + j]);
        }
        if (log_E && n < log_cap) log_E[n] = E;
        if (!std::isfinite(E)) { status = BEC_ENONFINITE; break; }
        if (n >= 1 && std::fabs(E - E_prev) < o->tol_dE) { status = BEC_OK; break; }
        if (n >= o->max_iter) { status = BEC_ENOTCONV; break; }
        E_prev = E;
        for (int i = 0; i < 2; ++i) {
            const double nrm2 = dV * S[12 + i];
            if (!(nrm2 > 0.0) || !std::isfinite(nrm2)) {
                (void)hipStreamSynchronize(c->st);
                return fail(BEC_ENONFINITE, "imaginary-time step lost the norm");
            }
            a[i] = 1.0 / std::sqrt(nrm2);   // the trial pass's own formula, for the synchronous schedule
        }
        ++n;
        if (!pipe) STCHK(enqueue_step(n, a));
    }
    double2* const result = slotA(n);
    Eval ev;
    if (status != BEC_ENONFINITE) {
        STCHK(heval(c, result, nullptr, kOne, kZero, 1, &ev));
        STCHK(residual_norms(c, 1, &ev));
        rep.final = ev.t;
    }
    HIPCHK(hipMemcpyAsync(psi_inout, result, 2 * N * sizeof(double2), hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    rep.iters = n;
    rep.status = status;
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (out_h) *out_h = rep;
    if (status == BEC_ENONFINITE) fail(status, "non-finite energy");
    return status;
}

bec_status bec_param_grad(bec_ctx* c, const double* psi, double dG[2][2], double dGdd[2][2], double* dc_lhy)
{
    if (c) c->resume.valid = false;   // the context's buffers change
    if (!c || !psi || !dG || !dGdd || !dc_lhy) return fail(BEC_EINVAL, "null argument");
    Eval ev;
    STCHK(heval(c, reinterpret_cast<const double2*>(psi), nullptr, kOne, kZero, 0, &ev));
    bec::ParamGradArgs pa{};
    pa.psi = c->psi[0];
    pa.partials = c->partials;
    HIPCHK(bec::launch_param_grad(c->P, pa, c->nblk_pw, c->st));
    STCHK(reduce_pw(c, bec::kParamSums, 0));
    STCHK(fetch(c, bec::kParamSums));
    const double* S = c->host;
    const double dV = c->dV;
    const double K = std::sqrt(2.0) / (15.0 * M_PI * M_PI);
    const double snn[2][2] = {{ev.sums[4], ev.sums[5]}, {ev.sums[5], ev.sums[6]}};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            dG[i][j] = 0.5 * c->p.N[i] * dV * snn[i][j] + c->p.c_lhy * K * dV * S[2 * i + j];
            dGdd[i][j] = 0.5 * c->p.N[i] * dV * ev.sums[7 + 2 * i + j] + c->p.c_lhy * K * dV * S[4 + 2 * i + j];
        }
    *dc_lhy = K * dV * S[8];
    return BEC_OK;
}

}  // extern "C"

// ====================================================================== batched scan
namespace {

struct BatchGroup {
    int n[3] = {0, 0, 0};
    long long N = 0;
    int first = 0, count = 0, nblk = 0, nblk_x = 0;
    int nblk_pz = 0, nblk_py = 0;  // blocks of the z and y passes (Parseval axis sums of the line search);
                                   // nblk_x, nblk_py over the half-spectrum geometry (z extent n_z + 2)
    int var[3] = {0, 0, 0};        // FFT plan variant per axis (the x pass is always the k-space pass)
    double2 *psi = nullptr, *hpsi = nullptr, *aux = nullptr, *p = nullptr, *r_old = nullptr, *rho = nullptr,
            *W = nullptr, *zbuf = nullptr;
    double *partials = nullptr, *fft_partials = nullptr, *udtab = nullptr, *kv[3] = {}, *vv[3] = {};
    double* ls_partials = nullptr;  // the line search's k-space sums, [instance][sum][x-pass block]
    double2* tw[3] = {};
    long long udsize = 0;
    int* ids_all = nullptr;        // device: 0..count-1
    int* ids_act = nullptr;        // device: running instances (compacted launches)
    std::vector<int> act;          // host copy of the running list
    bec::BGroup g{};
};

// host tables of one instance: wavenumbers, trap per axis, dipolar kernel on the k octant
void instance_tables(const bec_grid& gr, const bec_params& p, std::vector<double> kv[3], std::vector<double> vv[3],
                     std::vector<double>& ud)
{
    double L[3], h[3];
    for (int d = 0; d < 3; ++d) {
        L[d] = gr.hi[d] - gr.lo[d];
        h[d] = L[d] / gr.n[d];
        kv[d].resize(gr.n[d]);
        vv[d].resize(gr.n[d]);
        for (int j = 0; j < gr.n[d]; ++j) {
            const int jj = j < gr.n[d] / 2 ? j : j - gr.n[d];
            kv[d][j] = (double)(2.0L * kPiL * jj / (long double)L[d]);
            const double x = gr.lo[d] + j * h[d];
            vv[d][j] = 0.5 * p.omega[d] * p.omega[d] * x * x;
        }
    }
    const int ax = gr.n[0] / 2 + 1, ay = gr.n[1] / 2 + 1, az = gr.n[2] / 2 + 1;
    ud.assign((size_t)ax * ay * az, 0.0);
    for (int i = 0; i < ax; ++i)
        for (int j = 0; j < ay; ++j)
            for (int k = 0; k < az; ++k) {
                const long double kx = 2.0L * kPiL * i / L[0], ky = 2.0L * kPiL * j / L[1], kz = 2.0L * kPiL * k / L[2];
                ud[((size_t)i * ay + j) * az + k] = (double)dipolar_kernel(kx, ky, kz, p);
            }
}

void instance_params(const bec_grid& gr, const bec_params& p, bec::BInstParams& P)
{
    std::memset(&P, 0, sizeof(P));
    double dV = 1.0;
    long long npts = 1;
    for (int d = 0; d < 3; ++d) {
        dV *= (gr.hi[d] - gr.lo[d]) / gr.n[d];
        npts *= gr.n[d];
    }
    for (int i = 0; i < 2; ++i) {
        P.Nat[i] = p.N[i];
        for (int j = 0; j < 2; ++j) {
            P.G[i][j] = p.G[i][j];
            P.Gdd[i][j] = p.Gdd[i][j];
        }
    }
    const double Ntot = p.N[0] + p.N[1];
    P.Ntot_w[0] = (p.N[0] / Ntot) * (p.N[0] / Ntot);
    P.Ntot_w[1] = (p.N[1] / Ntot) * (p.N[1] / Ntot);
    P.K5 = p.c_lhy * std::sqrt(2.0) / (15.0 * M_PI * M_PI);
    P.K3 = p.c_lhy / (3.0 * std::sqrt(2.0) * M_PI * M_PI);
    P.dV = dV;
    P.inv_npts = 1.0 / (double)npts;
    P.lhy_on = p.c_lhy != 0.0;
    std::vector<double> u, w;
    lhy_rule(p, u, w);
    P.n_u = (int)u.size();
    hot_nodes(p, u, w, P.node5, &P.n_a, &P.n_b);
    P.lhy_K = P.lhy_on ? build_lhy_table(P.node5, P.n_a, P.lhytab) : 0;
}

bool same_shape(const bec_grid& a, const bec_grid& b) { return a.n[0] == b.n[0] && a.n[1] == b.n[1] && a.n[2] == b.n[2]; }

// instance order grouped by grid shape (stable), and the group boundaries
void plan_groups(int n_inst, const bec_grid* grids, std::vector<int>& perm, std::vector<std::pair<int, int>>& ranges)
{
    perm.clear();
    ranges.clear();
    std::vector<bool> used(n_inst, false);
    for (int i = 0; i < n_inst; ++i) {
        if (used[i]) continue;
        const int first = (int)perm.size();
        for (int j = i; j < n_inst; ++j)
            if (!used[j] && same_shape(grids[i], grids[j])) {
                used[j] = true;
                perm.push_back(j);
            }
        ranges.emplace_back(first, (int)perm.size() - first);
    }
}

int group_nblk(long long N)
{
    long long b = N / (bec::kPwThreads * 4);
    return (int)std::max<long long>(16, std::min<long long>(1024, b));
}

// sizes of the batch workspace in carve order; off receives the offsets
size_t batch_layout(int n_inst, const bec_grid* grids, std::vector<size_t>* off)
{
    std::vector<int> perm;
    std::vector<std::pair<int, int>> ranges;
    plan_groups(n_inst, grids, perm, ranges);
    std::vector<size_t> sizes;
    sizes.push_back(n_inst * sizeof(bec::BInstParams));
    sizes.push_back(n_inst * sizeof(bec::BInstState));
    sizes.push_back((size_t)n_inst * bec::kBSumStride * sizeof(double));
    sizes.push_back(4 * (size_t)n_inst * sizeof(int));          // act_dir, act_trial, tsel, act_pre
    sizes.push_back(n_inst * sizeof(double*));                  // user pointers
    const size_t c2 = sizeof(double2);
    for (auto& r : ranges) {
        const bec_grid& g = grids[perm[r.first]];
        const long long N = (long long)g.n[0] * g.n[1] * g.n[2];
        const long long cnt = r.second;
        const int nblk = group_nblk(N);
        // any plan variant; x and y over the line search's half spectra (z extent n_z + 2)
        const int nbx = bec::fft_max_blocks(g.n[0], (long long)g.n[1] * (g.n[2] + 2));
        const int nby = bec::fft_max_blocks(g.n[1], (long long)g.n[0] * (g.n[2] + 2));
        const int nbz = bec::fft_max_blocks(g.n[2], (long long)g.n[0] * g.n[1]);
        const size_t ud = (size_t)(g.n[0] / 2 + 1) * (g.n[1] / 2 + 1) * (g.n[2] / 2 + 1);
        size_t gs[] = {cnt * 4 * N * c2, cnt * 4 * N * c2, cnt * 4 * N * c2,  // psi, hpsi, aux (2 buffers)
                       cnt * 2 * N * c2, cnt * 2 * N * c2, cnt * N * c2,      // p, r_old, rho
                       cnt * 3 * N * c2,                                      // W
                       cnt * 2 * N * c2,                                      // zbuf
                       (size_t)cnt * bec::kMaxSums * nblk * sizeof(double),   // partials
                       (size_t)cnt * 3 * (nbx + nby + nbz) * sizeof(double),  // fft partials
                       (size_t)cnt * bec::kLsEpiSums * nbx * sizeof(double),  // line-search k-space sums
                       cnt * ud * sizeof(double),                             // dipolar tables
                       cnt * g.n[0] * sizeof(double), cnt * g.n[1] * sizeof(double), cnt * g.n[2] * sizeof(double),
                       cnt * g.n[0] * sizeof(double), cnt * g.n[1] * sizeof(double), cnt * g.n[2] * sizeof(double),
                       g.n[0] * c2, g.n[1] * c2, g.n[2] * c2,
                       2 * (size_t)cnt * sizeof(int)};                          // instance id lists
        for (size_t s : gs) sizes.push_back(s);
    }
    size_t total = 0;
    if (off) off->clear();
    for (size_t s : sizes) {
        if (off) off->push_back(total);
        total += align256(s);
    }
    return total;
}

}  // namespace

struct bec_batch {
    int n_inst = 0;
    hipStream_t st = nullptr;
    hipStream_t cap = nullptr;     // capture stream
    std::vector<bec_grid> grids;
    std::vector<bec_params> params;
    std::vector<int> perm;         // internal index -> caller index
    std::vector<BatchGroup> groups;
    bec::BInstParams* ip = nullptr;
    bec::BInstState* state = nullptr;
    double* sums = nullptr;
    int *act_dir = nullptr, *act_trial = nullptr, *tsel = nullptr, *act_pre = nullptr;
    double** psi_user = nullptr;
    bec::BInstState* host_state = nullptr;   // pinned
    double** host_ptrs = nullptr;            // pinned
    hipGraphExec_t exec = nullptr;
    int graph_rounds = 0;
    bec::BOpts graph_opts{};
};

namespace {

bec_status check_batch_args(int32_t n_inst, const bec_grid* grids, const bec_params* params)
{
    if (n_inst < 1 || !grids || !params) return fail(BEC_EINVAL, "need n_inst >= 1 and grid/param arrays");
    for (int i = 0; i < n_inst; ++i) {
        STCHK(check_grid(&grids[i]));
        STCHK(check_params(&params[i]));
        STCHK(check_params_grid(&grids[i], &params[i]));
    }
    return BEC_OK;
}

FftPassArgs batch_pass_args(const BatchGroup& G, int axis, const int* active)
{
    FftPassArgs A{};
    A.nx = G.n[0];
    A.ny = G.n[1];
    A.nz = G.n[2];
    A.kx = G.kv[0];
    A.ky = G.kv[1];
    A.kz = G.kv[2];
    A.udtab = G.udtab;
    A.udsize = G.udsize;
    A.per_inst_tab = 1;
    A.inv_n = 1.0 / (double)G.N;
    A.tw = G.tw[axis];
    A.scale = 1.0;
    A.partials = G.fft_partials;
    A.nblk_x = G.nblk_x;
    A.kaxis = G.kv[axis];
    A.inv_na = 1.0 / (double)G.n[axis];
    A.n_inst = G.g.n_ids;
    A.inst_ids = G.g.ids;
    A.active = active + G.first;
    A.src_sel = nullptr;
    if (axis == 2) {
        A.S = 1;
        A.npencil = (long long)G.n[0] * G.n[1];
    } else if (axis == 1) {
        A.S = G.n[2];
        A.npencil = (long long)G.n[0] * G.n[2];
    } else {
        A.S = (long long)G.n[1] * G.n[2];
        A.npencil = A.S;
    }
    for (int f = 0; f < 3; ++f) {
        A.op[f] = bec::kOpPlain;
        A.src_stride[f] = A.dst_stride[f] = 3 * G.N;
        A.src_sel_stride[f] = 0;
    }
    return A;
}

bec_status bpass(bec_batch* b, const BatchGroup& G, FftPassArgs A, int axis, int nf, int sign)
{
    A.nfield = nf;
    A.sign = sign;
    HIPCHK(bec::fft_pass(G.n[axis], G.var[axis], axis == 2, A, b->st));
    return BEC_OK;
}

// Trial points and Hamiltonian FFTs of every active instance of the group: the
// trial update rides in the loads of the first (z) pass
bec_status batch_heval_fft(bec_batch* b, const BatchGroup& G, hipStream_t s)
{
    (void)s;
    const long long N = G.N;
    FftPassArgs A = batch_pass_args(G, 2, b->act_trial);
    HIPCHK(bec::fft_btrial_z_pass(G.n[2], G.var[2], A, G.g, b->st));
    A = batch_pass_args(G, 1, b->act_trial);
    for (int f = 0; f < 3; ++f) A.src[f] = A.dst[f] = G.W + f * N;
    STCHK(bpass(b, G, A, 1, 3, -1));
    A = batch_pass_args(G, 0, b->act_trial);
    for (int f = 0; f < 3; ++f) A.src[f] = A.dst[f] = G.W + f * N;
    A.op[0] = A.op[1] = bec::kOpMulKin;
    A.op[2] = bec::kOpMulDip;
    STCHK(bpass(b, G, A, 0, 3, -1));
    A = batch_pass_args(G, 1, b->act_trial);
    for (int f = 0; f < 3; ++f) A.src[f] = A.dst[f] = G.W + f * N;
    STCHK(bpass(b, G, A, 1, 3, +1));
    A = batch_pass_args(G, 2, b->act_trial);
    for (int f = 0; f < 3; ++f) A.src[f] = A.dst[f] = G.W + f * N;
    return bpass(b, G, A, 2, 3, +1);
}

// Block stride of a group's Parseval partials: the z, y and x passes of the
// line search write theirs side by side.
int batch_parseval_stride(const BatchGroup& G) { return G.nblk_pz + G.nblk_py + G.nblk_x; }

// line-search FFTs: <p_i, T p_i> as the sum of its one-axis terms (kOpParsevalAxis:
// p_1, p_2 read by each forward pass, nothing stored) while the passes carry the
// densities: the z pass unpacks the transform of the packed rho_1 + i rho_2 into
// their half spectra (W + N of each instance, z extent n_z + 2), the y pass
// carries those, and the x pass forms the model's density sums in k-space
// (kOpDipSums, into ls_partials); no inverse transform
bec_status batch_ls_fft(bec_batch* b, const BatchGroup& G)
{
    const long long N = G.N, nzh = G.n[2] + 2;
    const int T = batch_parseval_stride(G);
    const long long off[3] = {G.nblk_pz + G.nblk_py, G.nblk_pz, 0};   // per axis x, y, z
    for (int axis = 2; axis >= 0; --axis) {
        FftPassArgs A = batch_pass_args(G, axis, b->act_dir);
        A.src[0] = G.p;
        A.src[1] = G.p + N;
        A.src_stride[0] = A.src_stride[1] = 2 * N;
        A.src[2] = axis == 2 ? G.rho : G.W + N;
        A.src_stride[2] = axis == 2 ? N : 3 * N;
        A.dst[0] = A.dst[1] = nullptr;               // Parseval fields: no store
        A.dst[2] = G.W + N;
        A.dst_stride[2] = 3 * N;
        A.op[0] = A.op[1] = bec::kOpParsevalAxis;
        A.op[2] = axis == 2 ? bec::kOpHalfSpectra : axis == 1 ? bec::kOpPlain : bec::kOpDipSums;
        if (axis < 2) {
            A.S2 = axis == 1 ? nzh : (long long)G.n[1] * nzh;
            A.npencil2 = axis == 1 ? (long long)G.n[0] * nzh : A.S2;
        }
        A.ls_partials = G.ls_partials;
        A.partials = G.fft_partials + off[axis];
        A.nblk_x = T;
        A.pscale = (double)(N / G.n[axis]);
        STCHK(bpass(b, G, A, axis, 3, -1));
    }
    return BEC_OK;
}

bec_status breduce(bec_batch* b, const BatchGroup& G, int M, int off)
{
    HIPCHK(bec::launch_b_reduce(G.partials, (long long)bec::kMaxSums * G.nblk, G.nblk, G.nblk, M, G.g.ids,
                                G.g.n_ids, b->sums + (long long)G.first * bec::kBSumStride, off, b->st));
    return BEC_OK;
}

bec_status batch_trial_and_accept(bec_batch* b, const bec::BOpts& o)
{
    for (auto& G : b->groups) {
        if (G.g.n_ids == 0) continue;
        STCHK(batch_heval_fft(b, G, b->st));
        HIPCHK(bec::launch_b_heval_epi(G.g, b->st));
        STCHK(breduce(b, G, bec::kHevalSums, bec::kSH));
    }
    HIPCHK(bec::launch_b_decide_accept(b->n_inst, o, b->ip, b->state, b->sums, b->act_trial, b->st));
    return BEC_OK;
}

// z of the k-space preconditioners (zmode >= 2) for the instances in act_pre:
// make_r writes r, P_V^-1 r or D^-1/2 r to zbuf, then the z, y, x (multiply by
// 1/([shift_i]_+ + sigma + |k|^2/2), each instance its own shift), y and z passes
// transform it in place
bec_status batch_precond_fft(bec_batch* b, const BatchGroup& G)
{
    HIPCHK(bec::launch_b_make_r(G.g, b->st));
    const long long N = G.N;
    const int axes[5] = {2, 1, 0, 1, 2};
    const int signs[5] = {-1, -1, -1, +1, +1};
    for (int k = 0; k < 5; ++k) {
        FftPassArgs A = batch_pass_args(G, axes[k], b->act_pre);
        for (int f = 0; f < 2; ++f) {
            A.src[f] = A.dst[f] = G.zbuf + f * N;
            A.src_stride[f] = A.dst_stride[f] = 2 * N;
        }
        if (axes[k] == 0) {
            A.op[0] = A.op[1] = bec::kOpMulPrec;
            A.prec_bst = b->state + G.first;
            A.prec_sigma = G.g.sigma;
        }
        STCHK(bpass(b, G, A, axes[k], 2, signs[k]));
    }
    return BEC_OK;
}

// one round of the iteration for every instance (no host synchronisation)
bec_status batch_round(bec_batch* b, const bec::BOpts& o)
{
    bool kspace = false;
    for (auto& G : b->groups) kspace = kspace || (G.g.n_ids > 0 && G.g.zmode >= 2);
    if (kspace) {
        HIPCHK(bec::launch_b_mark_pre(b->n_inst, b->state, b->act_pre, b->st));
        for (auto& G : b->groups)
            if (G.g.n_ids > 0) STCHK(batch_precond_fft(b, G));
    }
    for (auto& G : b->groups) {
        if (G.g.n_ids == 0) continue;
        HIPCHK(bec::launch_b_dir_reduce(G.g, b->st));
        STCHK(breduce(b, G, bec::kDirReduceSums, bec::kSR));
    }
    HIPCHK(bec::launch_b_decide_dir(b->n_inst, o, b->ip, b->state, b->sums, b->act_dir, b->st));
    for (auto& G : b->groups) {
        if (G.g.n_ids == 0) continue;
        HIPCHK(bec::launch_b_dir_write(G.g, b->st));
        STCHK(breduce(b, G, bec::kDirWriteSums, bec::kSW));
        STCHK(batch_ls_fft(b, G));
        HIPCHK(bec::launch_b_reduce(G.ls_partials, (long long)bec::kLsEpiSums * G.nblk_x, G.nblk_x, G.nblk_x,
                                    bec::kLsEpiSums, G.g.ids, G.g.n_ids,
                                    b->sums + (long long)G.first * bec::kBSumStride, bec::kSL, b->st));
        const int T = batch_parseval_stride(G);
        HIPCHK(bec::launch_b_reduce(G.fft_partials, 3LL * T, T, T, 2, G.g.ids, G.g.n_ids,
                                    b->sums + (long long)G.first * bec::kBSumStride, bec::kSP, b->st));
    }
    HIPCHK(bec::launch_b_decide_step(b->n_inst, o, b->ip, b->state, b->sums, b->act_dir, b->act_trial, b->tsel,
                                     b->st));
    return batch_trial_and_accept(b, o);
}

bec::BOpts to_bopts(const bec_opts* o)
{
    bec::BOpts b{};
    b.beta_mode = o->beta;
    b.max_iter = o->max_iter;
    b.restart_period = o->restart_period;
    b.max_backtrack = o->max_backtrack;
    b.stall_window = o->stall_window;
    b.tol_grad = o->tol_grad;
    b.tol_dE = o->tol_dE;
    b.sigma = o->sigma;
    b.armijo_c1 = o->armijo_c1;
    b.theta_max = o->theta_max;
    b.tau_rel = o->tau_rel;
    b.pc = o->pc;
    b.blend = o->blend;
    return b;
}

bool same_bopts(const bec::BOpts& a, const bec::BOpts& b) { return std::memcmp(&a, &b, sizeof(a)) == 0; }

}  // namespace

extern "C" {

bec_status bec_batch_workspace_size(int32_t n_inst, const bec_grid* grids, const bec_params* params, size_t* bytes)
{
    STCHK(check_batch_args(n_inst, grids, params));
    if (!bytes) return fail(BEC_EINVAL, "bytes is null");
    *bytes = batch_layout(n_inst, grids, nullptr);
    return BEC_OK;
}

bec_status bec_batch_create(int32_t n_inst, const bec_grid* grids, const bec_params* params, void* hip_stream,
                            void* workspace, size_t workspace_bytes, bec_batch** out)
{
    try {
        STCHK(check_batch_args(n_inst, grids, params));
        if (!out || !workspace) return fail(BEC_EINVAL, "null argument");
        if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(BEC_EINVAL, "workspace must be 256-byte aligned");
        std::vector<size_t> off;
        const size_t need = batch_layout(n_inst, grids, &off);
        if (workspace_bytes < need) return fail(BEC_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
        bec_batch* b = new bec_batch();
        b->n_inst = n_inst;
        b->st = reinterpret_cast<hipStream_t>(hip_stream);
        b->grids.assign(grids, grids + n_inst);
        b->params.assign(params, params + n_inst);
        std::vector<std::pair<int, int>> ranges;
        plan_groups(n_inst, grids, b->perm, ranges);
        char* base = static_cast<char*>(workspace);
        size_t k = 0;
        b->ip = (bec::BInstParams*)(base + off[k++]);
        b->state = (bec::BInstState*)(base + off[k++]);
        b->sums = (double*)(base + off[k++]);
        b->act_dir = (int*)(base + off[k++]);
        b->act_trial = b->act_dir + n_inst;
        b->tsel = b->act_dir + 2 * n_inst;
        b->act_pre = b->act_dir + 3 * n_inst;
        b->psi_user = (double**)(base + off[k++]);
        auto cleanup = [&](bec_status s) {
            if (b->host_state) (void)hipHostFree(b->host_state);
            if (b->host_ptrs) (void)hipHostFree(b->host_ptrs);
            if (b->cap) (void)hipStreamDestroy(b->cap);
            delete b;
            return s;
        };
        if (hipHostMalloc((void**)&b->host_state, n_inst * sizeof(bec::BInstState), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&b->host_ptrs, n_inst * sizeof(double*), hipHostMallocDefault) != hipSuccess ||
            hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
            return cleanup(fail(BEC_EHIP, "host buffers / capture stream"));
        std::vector<bec::BInstParams> hip_params(n_inst);
        for (int i = 0; i < n_inst; ++i) instance_params(grids[b->perm[i]], params[b->perm[i]], hip_params[i]);
        if (hipMemcpyAsync(b->ip, hip_params.data(), n_inst * sizeof(bec::BInstParams), hipMemcpyHostToDevice, b->st) !=
            hipSuccess)
            return cleanup(fail(BEC_EHIP, "upload of instance parameters"));
        for (auto& r : ranges) {
            BatchGroup G;
            const bec_grid& g0 = grids[b->perm[r.first]];
            for (int d = 0; d < 3; ++d) G.n[d] = g0.n[d];
            G.N = (long long)G.n[0] * G.n[1] * G.n[2];
            G.first = r.first;
            G.count = r.second;
            G.nblk = group_nblk(G.N);
            G.nblk_x = bec::fft_blocks(G.n[0], 0, (long long)G.n[1] * (G.n[2] + 2));
            G.nblk_py = bec::fft_blocks(G.n[1], 0, (long long)G.n[0] * (G.n[2] + 2));
            G.nblk_pz = bec::fft_blocks(G.n[2], 0, (long long)G.n[0] * G.n[1]);
            G.udsize = (long long)(G.n[0] / 2 + 1) * (G.n[1] / 2 + 1) * (G.n[2] / 2 + 1);
            G.psi = (double2*)(base + off[k++]);
            G.hpsi = (double2*)(base + off[k++]);
            G.aux = (double2*)(base + off[k++]);
            G.p = (double2*)(base + off[k++]);
            G.r_old = (double2*)(base + off[k++]);
            G.rho = (double2*)(base + off[k++]);
            G.W = (double2*)(base + off[k++]);
            G.zbuf = (double2*)(base + off[k++]);
            G.partials = (double*)(base + off[k++]);
            G.fft_partials = (double*)(base + off[k++]);
            G.ls_partials = (double*)(base + off[k++]);
            G.udtab = (double*)(base + off[k++]);
            for (int d = 0; d < 3; ++d) G.kv[d] = (double*)(base + off[k++]);
            for (int d = 0; d < 3; ++d) G.vv[d] = (double*)(base + off[k++]);
            for (int d = 0; d < 3; ++d) G.tw[d] = (double2*)(base + off[k++]);
            G.ids_all = (int*)(base + off[k++]);
            G.ids_act = G.ids_all + G.count;
            {
                std::vector<int> iota(G.count);
                for (int l = 0; l < G.count; ++l) iota[l] = l;
                if (hipMemcpyAsync(G.ids_all, iota.data(), G.count * sizeof(int), hipMemcpyHostToDevice, b->st) !=
                        hipSuccess ||
                    hipStreamSynchronize(b->st) != hipSuccess)
                    return cleanup(fail(BEC_EHIP, "upload of instance lists"));
            }
            // per-instance tables
            std::vector<double> ud_all, kv_all[3], vv_all[3];
            for (int l = 0; l < G.count; ++l) {
                std::vector<double> kv[3], vv[3], ud;
                instance_tables(grids[b->perm[G.first + l]], params[b->perm[G.first + l]], kv, vv, ud);
                ud_all.insert(ud_all.end(), ud.begin(), ud.end());
                for (int d = 0; d < 3; ++d) {
                    kv_all[d].insert(kv_all[d].end(), kv[d].begin(), kv[d].end());
                    vv_all[d].insert(vv_all[d].end(), vv[d].begin(), vv[d].end());
                }
            }
            bool ok = hipMemcpyAsync(G.udtab, ud_all.data(), ud_all.size() * sizeof(double), hipMemcpyHostToDevice,
                                     b->st) == hipSuccess;
            for (int d = 0; d < 3 && ok; ++d) {
                ok = hipMemcpyAsync(G.kv[d], kv_all[d].data(), kv_all[d].size() * sizeof(double),
                                    hipMemcpyHostToDevice, b->st) == hipSuccess &&
                     hipMemcpyAsync(G.vv[d], vv_all[d].data(), vv_all[d].size() * sizeof(double),
                                    hipMemcpyHostToDevice, b->st) == hipSuccess;
                std::vector<double2> tw(G.n[d]);
                for (int m = 0; m < G.n[d]; ++m) {
                    const long double a = -2.0L * kPiL * (long double)m / (long double)G.n[d];
                    tw[m] = make_double2((double)cosl(a), (double)sinl(a));
                }
                ok = ok && hipMemcpyAsync(G.tw[d], tw.data(), G.n[d] * sizeof(double2), hipMemcpyHostToDevice,
                                          b->st) == hipSuccess &&
                     hipStreamSynchronize(b->st) == hipSuccess;
            }
            if (!ok || hipStreamSynchronize(b->st) != hipSuccess) return cleanup(fail(BEC_EHIP, "upload of tables"));
            bec::BGroup& g = G.g;
            g.first = G.first;
            g.count = G.count;
            g.nx = G.n[0];
            g.ny = G.n[1];
            g.nz = G.n[2];
            bec::div_magic((uint32_t)(G.n[1] * G.n[2]), &g.m_nyz, &g.s_nyz);
            bec::div_magic((uint32_t)G.n[2], &g.m_nz, &g.s_nz);
            g.N = G.N;
            g.nblk = G.nblk;
            g.ip = b->ip;
            g.st = b->state;
            g.sums = b->sums;
            g.act_dir = b->act_dir;
            g.act_trial = b->act_trial;
            g.psi_user = b->psi_user;
            g.vx = G.vv[0];
            g.vy = G.vv[1];
            g.vz = G.vv[2];
            g.psi = G.psi;
            g.hpsi = G.hpsi;
            g.aux = G.aux;
            g.p = G.p;
            g.r_old = G.r_old;
            g.rho = G.rho;
            g.W = G.W;
            g.zbuf = G.zbuf;
            g.act_pre = b->act_pre;
            g.partials = G.partials;
            g.ids = G.ids_all;
            g.n_ids = G.count;
            b->groups.push_back(G);
        }
        if (hipStreamSynchronize(b->st) != hipSuccess) return cleanup(fail(BEC_EHIP, "synchronise"));
        *out = b;
        return BEC_OK;
    } catch (...) {
        return fail(BEC_EINVAL, "unexpected host exception in bec_batch_create");
    }
}

bec_status bec_batch_destroy(bec_batch* b)
{
    if (!b) return BEC_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->host_state) (void)hipHostFree(b->host_state);
    if (b->host_ptrs) (void)hipHostFree(b->host_ptrs);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return BEC_OK;
}

bec_status bec_batch_set_tuning(bec_batch* b, const bec_grid* grid, const bec_tuning* t)
{
    if (!b || !grid || !t) return fail(BEC_EINVAL, "null argument");
    const int v[3] = {t->fft_variant[0][1], t->fft_variant[1][0], t->fft_variant[2][0]};
    int matched = 0;
    for (auto& G : b->groups) {
        if (G.n[0] != grid->n[0] || G.n[1] != grid->n[1] || G.n[2] != grid->n[2]) continue;
        for (int d = 0; d < 3; ++d)
            if (v[d] < 0 || v[d] >= bec::fft_num_variants(G.n[d]))
                return fail(BEC_EINVAL, "axis %d: plan variant %d of length %d does not exist", d, v[d], G.n[d]);
        for (int d = 0; d < 3; ++d) G.var[d] = v[d];
        G.nblk_x = bec::fft_blocks(G.n[0], G.var[0], (long long)G.n[1] * (G.n[2] + 2));
        G.nblk_py = bec::fft_blocks(G.n[1], G.var[1], (long long)G.n[0] * (G.n[2] + 2));
        G.nblk_pz = bec::fft_blocks(G.n[2], G.var[2], (long long)G.n[0] * G.n[1]);
        ++matched;
    }
    if (!matched) return fail(BEC_EINVAL, "no instance has the grid %dx%dx%d", grid->n[0], grid->n[1], grid->n[2]);
    if (b->exec) {   // a captured round holds the old plans
        HIPCHK(hipGraphExecDestroy(b->exec));
        b->exec = nullptr;
    }
    return BEC_OK;
}

bec_status bec_batch_solve(bec_batch* b, double* const* psi_inout, const bec_opts* o, int32_t rounds_per_sync,
                           int32_t use_graph, bec_report* reports_h)
{
    if (!b || !psi_inout || !o || !reports_h) return fail(BEC_EINVAL, "null argument");
    if (o->pc < BEC_PC_NONE || o->pc > BEC_PC_BLEND) return fail(BEC_EINVAL, "bad preconditioner %d", o->pc);
    if (o->pc == BEC_PC_BLEND && !(o->blend <= 1.0)) return fail(BEC_EINVAL, "blend weight must be <= 1");
    if (o->beta < 0 || o->beta > 2) return fail(BEC_EINVAL, "bad beta mode");
    const auto t0 = std::chrono::steady_clock::now();
    const int K = rounds_per_sync > 0 ? rounds_per_sync : 16;
    const bec::BOpts bo = to_bopts(o);
    // z per preconditioner: P_Delta and the composite read P_Delta^-1 of the
    // make_r output (r, P_V^-1 r); the symmetrised composite scales it by D^-1/2;
    // the blend mixes P_V^-1 r into it
    static const int zmode_of[6] = {0, 1, 2, 2, 3, 4}, papply_of[6] = {0, 0, 0, 1, 2, 0};
    for (auto& G : b->groups) {
        G.g.zmode = zmode_of[o->pc];
        G.g.papply = papply_of[o->pc];
        G.g.sigma = o->sigma;
        G.g.blend = o->blend;
    }
    for (int i = 0; i < b->n_inst; ++i) {
        if (!psi_inout[b->perm[i]]) return fail(BEC_EINVAL, "psi_inout[%d] is null", b->perm[i]);
        b->host_ptrs[i] = psi_inout[b->perm[i]];
    }
    HIPCHK(hipMemcpyAsync(b->psi_user, b->host_ptrs, b->n_inst * sizeof(double*), hipMemcpyHostToDevice, b->st));
    for (auto& G : b->groups) {
        G.g.ids = G.ids_all;
        G.g.n_ids = G.count;
        G.act.assign(G.count, 0);
        for (int l = 0; l < G.count; ++l) G.act[l] = l;
    }
    // initial state: normalise and evaluate
    for (auto& G : b->groups) {
        HIPCHK(bec::launch_b_norm2(G.g, b->st));
        STCHK(breduce(b, G, 2, bec::kSR));
    }
    HIPCHK(bec::launch_b_decide_init(b->n_inst, b->ip, b->state, b->sums, b->act_dir, b->act_trial, b->tsel, b->st));
    STCHK(batch_trial_and_accept(b, bo));

    // Rounds are launched in chunks of K; between chunks the host reads the
    // instance states and compacts every launch to the instances still running
    // (the graph is re-captured when that set changes).
    bool dirty = true;
    const long long max_rounds = (long long)(o->max_iter + 1) * (o->max_backtrack + 3) + 8;
    long long rounds = 0;
    for (;;) {
        if (use_graph) {
            if (dirty || !b->exec || b->graph_rounds != K || !same_bopts(b->graph_opts, bo)) {
                if (b->exec) {
                    HIPCHK(hipGraphExecDestroy(b->exec));
                    b->exec = nullptr;
                }
                hipStream_t user = b->st;
                b->st = b->cap;
                HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
                bec_status cs = BEC_OK;
                for (int r = 0; r < K && cs == BEC_OK; ++r) cs = batch_round(b, bo);
                hipGraph_t graph = nullptr;
                const hipError_t ce = hipStreamEndCapture(b->cap, &graph);
                b->st = user;
                if (cs != BEC_OK) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return cs;
                }
                if (ce != hipSuccess) return fail(BEC_EHIP, "graph capture failed: %s", hipGetErrorString(ce));
                const hipError_t ie = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (ie != hipSuccess) return fail(BEC_EHIP, "graph instantiation failed: %s", hipGetErrorString(ie));
                b->graph_rounds = K;
                b->graph_opts = bo;
            }
            HIPCHK(hipGraphLaunch(b->exec, b->st));
        } else {
            for (int r = 0; r < K; ++r) STCHK(batch_round(b, bo));
        }
        rounds += K;
        HIPCHK(hipMemcpyAsync(b->host_state, b->state, b->n_inst * sizeof(bec::BInstState), hipMemcpyDeviceToHost,
                              b->st));
        HIPCHK(hipStreamSynchronize(b->st));
        bool running = false;
        dirty = false;
        for (auto& G : b->groups) {
            std::vector<int> act;
            for (int l = 0; l < G.count; ++l)
                if (b->host_state[G.first + l].status == bec::kBRunning) act.push_back(l);
            running = running || !act.empty();
            if (act != G.act) {
                G.act = act;
                dirty = true;
                if (!act.empty())
                    HIPCHK(hipMemcpyAsync(G.ids_act, G.act.data(), act.size() * sizeof(int), hipMemcpyHostToDevice,
                                          b->st));
                G.g.ids = G.ids_act;
                G.g.n_ids = (int)act.size();
            }
        }
        if (dirty) HIPCHK(hipStreamSynchronize(b->st));   // the host list is reused on the next change
        if (!running || rounds >= max_rounds) break;
    }
    for (auto& G : b->groups) {
        G.g.ids = G.ids_all;
        G.g.n_ids = G.count;
    }
    if (b->exec) {
        HIPCHK(hipGraphExecDestroy(b->exec));
        b->exec = nullptr;
    }
    for (auto& G : b->groups) HIPCHK(bec::launch_b_copy_out(G.g, b->st));
    HIPCHK(hipStreamSynchronize(b->st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < b->n_inst; ++i) {
        const bec::BInstState& S = b->host_state[i];
        const bec_params& p = b->params[b->perm[i]];
        bec_report& R = reports_h[b->perm[i]];
        std::memset(&R, 0, sizeof(R));
        R.iters = S.iter;
        R.n_restarts = S.n_restarts;
        R.n_backtracks = S.n_backtracks;
        R.status = S.status == bec::kBConverged ? BEC_OK
                   : S.status == bec::kBRunning || S.status == bec::kBNotConv ? BEC_ENOTCONV
                   : S.status == bec::kBStagnated ? BEC_ESTAGNATED
                   : S.status == bec::kBStalled ? BEC_ESTALLED : BEC_ENONFINITE;
        bec::BInstParams P;
        instance_params(b->grids[b->perm[i]], p, P);
        const double* H = S.hsum;
        const double dV = P.dV;
        bec_terms& t = R.final;
        const double snn[2][2] = {{H[4], H[5]}, {H[5], H[6]}};
        for (int c = 0; c < 2; ++c) {
            t.norm2[c] = dV * H[14 + c];
            t.E_kin[c] = p.N[c] * dV * H[c];
            t.E_trap[c] = p.N[c] * dV * H[2 + c];
            for (int j = 0; j < 2; ++j) {
                t.E_c[c][j] = 0.5 * p.N[c] * p.G[c][j] * dV * snn[c][j];
                t.E_dd[c][j] = 0.5 * p.N[c] * p.Gdd[c][j] * dV * H[7 + 2 * c + j];
            }
            t.mu[c] = S.mu[c];
            t.shift[c] = S.shift[c];
            t.res[c] = S.res[c];
        }
        t.E_lhy = dV * H[11];
        t.E = S.E;
        R.seconds = secs;
    }
    return BEC_OK;
}

}  // extern "C"
