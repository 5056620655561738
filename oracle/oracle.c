/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the ground-state problem of a
 * two-component dipolar Bose-Einstein condensate with Lee-Huang-Yang (LHY)
 * corrections, and for the preconditioned nonlinear conjugate-gradient
 * iteration on the product-of-spheres manifold that minimises it
 * (arXiv:2510.24543, Secs. II-V).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant generator with the GPU library: it has its own
 * recursive mixed-radix (2,3) FFT, its own Gauss-Legendre nodes, its own
 * kernel tables and its own reductions.  Everything is IEEE binary64.
 *
 * Discrete problem (Fourier pseudo-spectral, periodic box [lo,hi)):
 *   x_d[j] = lo_d + j h_d,  h_d = (hi_d - lo_d)/n_d,
 *   k_d[j] = (2 pi / L_d) (j < n_d/2 ? j : j - n_d),
 *   <f,g>  = dV sum conj(f) g,  dV = hx hy hz,
 *   F = unnormalised forward DFT (kernel exp(-i k.x)), F^-1 carries 1/N.
 *   Field layout: component-major, then C order (x, y, z), z fastest.
 *
 * Readings of the paper that this file implements (each is also listed in the
 * design notes of the repository):
 *   - the dipolar coefficient Gdd_ij is the amplitude of the k-space kernel,
 *     Ud(k) = Gdd_ij (3 kz^2/k^2 - 1) c(|k| Rc), with the spherical-cutoff
 *     factor c(q) = 1 + 3 cos q / q^2 - 3 sin q / q^3 and Ud(0) = 0; the LHY
 *     couplings are eta_ij = G_ij + Gdd_ij (3u^2 - 1) (Sec. II, Eq. (3));
 *   - c_lhy multiplies the whole LHY term of Eq. (1) (the paper is c_lhy = 1);
 *   - fractional powers act on [V]_+ = max(V, 0); ratio terms with s = 0 are 0;
 *   - the u integral is Gauss-Legendre with n_u nodes on [0,1];
 *   - the P_V shift is alpha_i = <psi_i,(T + V + sum_j G_ij n_j + muLHY_i) psi_i>
 *     and the P_V diagonal is [alpha_i + V + sum_j G_ij n_j + muLHY_i]_+ + sigma;
 *     the kinetic preconditioner multiplies by 1/([alpha_i]_+ + sigma + |k|^2/2);
 *     the composite applies P_V^-1 first, then P_Delta^-1 (Sec. IV.B, Eq. (18));
 *   - one shared step alpha, theta_i = alpha ||p_i|| (Sec. V);
 *   - w_ij multiplies psi_i (the printed psi_j is a typo: only psi_i gives the
 *     second derivative along the geodesic);
 *   - the model step is accepted if E(alpha) <= E + tau, tau = tau_rel |E|,
 *     else Armijo halving along the same geodesic, else a beta = 0 restart.
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;

/* ------------------------------------------------------------------------- */
/* Public structures (mirrored by the ctypes wrapper in oracle/__init__.py)   */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t n[3];
    double lo[3], hi[3];
} orc_grid;

typedef struct {
    double N[2];        /* atom numbers N_i (Eq. (1))                       */
    double omega[3];    /* trap ratios lambda_d = omega_d/omega_0 (Eq. (2)) */
    double G[2][2];     /* contact couplings G_ij                            */
    double Gdd[2][2];   /* dipolar k-space amplitudes                        */
    double c_lhy;       /* multiplier of the LHY term                        */
    double r_cut;       /* cutoff of the dipolar kernel (radius, or slab half-height) */
    int32_t n_u;        /* Gauss-Legendre nodes for the u integral           */
    int32_t dip_cut;    /* 0: spherical cutoff of radius r_cut; 1: slab cut,
                           the interaction kept for |z - z'| < r_cut and
                           unbounded in the periodic x, y directions          */
    int32_t lhy_quad;   /* u rule: 0 Gauss-Legendre with n_u nodes on [0,1];
                           1 root-split, n_u nodes on each piece of [0,1]
                           between the zeros of the branch potentials        */
} orc_params;

typedef struct {
    double E;
    double E_kin[2], E_trap[2], E_c[2][2], E_dd[2][2], E_lhy;
    double mu[2];      /* <psi_i,H_i psi_i>/<psi_i,psi_i>                     */
    double shift[2];   /* preconditioner shift alpha_i                        */
    double res[2];     /* ||H_i psi_i - mu_i psi_i||                          */
    double norm2[2];   /* ||psi_i||^2                                         */
} orc_terms;

typedef struct {
    int32_t pc;             /* 0 none, 1 P_V, 2 P_Delta, 3 P_Delta P_V        */
    int32_t beta;           /* 0 HS+, 1 PR+, 2 always zero                    */
    int32_t max_iter;
    int32_t restart_period; /* K_r: beta = 0 when n mod K_r == 0 (0: never)    */
    int32_t max_backtrack;
    int32_t stall_window;   /* > 0: stop (ORC_ESTALLED) when max_i ||r_i|| has not
                               fallen below half of its reference value within the
                               last stall_window accepted steps; the reference is
                               the last value that halved it (0: off)             */
    double tol_grad;        /* stop when max_i ||r_i|| < tol_grad              */
    double tol_dE;          /* stop when |E_n - E_{n-1}| < tol_dE (0: off)     */
    double sigma;           /* regularising shift of the preconditioners      */
    double armijo_c1;
    double theta_max;
    double tau_rel;         /* accept band tau = tau_rel |E|                   */
    double blend;           /* mode 5: weight w of P_V in [0, 1]; < 0 adaptive */
} orc_opts;

typedef struct {
    int32_t iter;       /* index of the accepted step                           */
    int32_t n_trials;   /* energy evaluations spent on this step               */
    int32_t restarted;  /* 1 if beta was forced to zero                        */
    int32_t path;       /* bits: 1 Armijo, 2 beta=0 retry, 4 fallback z       */
    double E;           /* energy after the step                               */
    double res_max;     /* max_i ||r_i|| before the step                       */
    double E1, E2, alpha, beta;
    int32_t level;      /* direction of the accepted step: 0 the computed beta,
                           1 beta = 0, 2 z = P_V^-1 r, 3 z = r                 */
    int32_t halvings;   /* Armijo halvings of the accepted trial               */
    double beta_num;    /* sum_i w_i Re<r_i - r_old_i, z_i> (0 on restarts)     */
    double beta_den;    /* HS+: sum_i w_i Re<r_i - r_old_i, p_old_i>;
                           PR+: sum_i w_i Re<r_old_i, z_old_i> (0 on restarts) */
    double rp;          /* sum_i 2 N_i Re<p_i, r_i> of the accepted direction   */
    double alpha_model; /* step before halving: -E1/E2 or the fallback, clamped */
    double pmax;        /* max_i ||p_i||                                        */
    double E0;          /* energy at the start of the step                      */
    double tau;         /* acceptance band tau_rel |E0|                          */
} orc_iter;

typedef struct {
    int32_t iters, n_restarts, n_backtracks, status;
    orc_terms final;
} orc_report;

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENOMEM = 2, ORC_ENOTCONV = 4,
       ORC_ESTAGNATED = 5, ORC_ENONFINITE = 6, ORC_ESTALLED = 8 };

/* ------------------------------------------------------------------------- */
/* Deterministic sums: fixed blocks summed in order (independent of threads)  */
/* ------------------------------------------------------------------------- */
#define ORC_BLK 4096

static double sum_array(const double *v, long n)
{
    long nb = (n + ORC_BLK - 1) / ORC_BLK;
    double *part = (double *)malloc(sizeof(double) * (size_t)(nb > 0 ? nb : 1));
    #pragma omp parallel for schedule(static)
    for (long b = 0; b < nb; ++b) {
        double s = 0.0;
        long e = (b + 1) * ORC_BLK < n ? (b + 1) * ORC_BLK : n;
        for (long i = b * ORC_BLK; i < e; ++i) s += v[i];
        part[b] = s;
    }
    double s = 0.0;
    for (long b = 0; b < nb; ++b) s += part[b];
    free(part);
    return s;
}

/* Re <a,b> / dV = sum Re(conj(a) b) */
static double re_dot(const cplx *a, const cplx *b, long n)
{
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) t[i] = creal(conj(a[i]) * b[i]);
    double s = sum_array(t, n);
    free(t);
    return s;
}

/* sum w(x) |a(x)|^2 (w may be NULL for 1) */
static double weighted_norm2(const double *w, const cplx *a, long n)
{
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double m = creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
        t[i] = w ? w[i] * m : m;
    }
    double s = sum_array(t, n);
    free(t);
    return s;
}

/* sum a(x) b(x) for real arrays */
static double dot_real(const double *a, const double *b, long n)
{
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) t[i] = a[i] * b[i];
    double s = sum_array(t, n);
    free(t);
    return s;
}

/* ------------------------------------------------------------------------- */
/* FFT: recursive decimation in time, radices 2 and 3 (plain DFT otherwise)   */
/* ------------------------------------------------------------------------- */
/* tw[t] = exp(-2 pi i t / ntop), t = 0..ntop-1.  A sub-transform of length m
 * uses exp(-2 pi i t / m) = tw[t * (ntop/m)].                               */
static void fft_rec(const cplx *in, long stride, int m, int ntop, const cplx *tw,
                    int sign, cplx *out, cplx *work)
{
    if (m == 1) { out[0] = in[0]; return; }
    int p = (m % 2 == 0) ? 2 : ((m % 3 == 0) ? 3 : m);
    int q = m / p;               /* length of each decimated sub-sequence */
    int tstep = ntop / m;
    cplx *Y = work;              /* p sub-transforms of length q           */
    for (int s = 0; s < p; ++s)
        fft_rec(in + (long)s * stride, stride * p, q, ntop, tw, sign,
                Y + (long)s * q, work + m);
    /* X[k + q l] = sum_s exp(sign 2 pi i s (k + q l)/m) Y_s[k] */
    for (int k = 0; k < q; ++k) {
        for (int l = 0; l < p; ++l) {
            int kk = k + q * l;
            cplx acc = 0.0;
            for (int s = 0; s < p; ++s) {
                long t = ((long)s * kk) % m;
                cplx w = tw[t * tstep];
                if (sign > 0) w = conj(w);
                acc += w * Y[(long)s * q + k];
            }
            out[kk] = acc;
        }
    }
}

static cplx *make_twiddles(int n)
{
    cplx *tw = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    for (int t = 0; t < n; ++t) {
        double a = -2.0 * M_PI * (double)t / (double)n;
        tw[t] = cos(a) + I * sin(a);
    }
    return tw;
}

/* In-place 3D transform of one field of shape n[0] x n[1] x n[2].
 * sign = -1: forward, unnormalised.  sign = +1: inverse, scaled by 1/N.    */
static void fft3d(const int n[3], cplx *a, int sign)
{
    long N = (long)n[0] * n[1] * n[2];
    long str[3] = { (long)n[1] * n[2], n[2], 1 };
    for (int ax = 2; ax >= 0; --ax) {
        int L = n[ax];
        cplx *tw = make_twiddles(L);
        /* pencils along axis ax: the other two indices enumerate them */
        int o1 = (ax == 0) ? 1 : 0, o2 = (ax == 2) ? 1 : 2;
        long npen = (long)n[o1] * n[o2];
        #pragma omp parallel
        {
            cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)L);
            cplx *res = (cplx *)malloc(sizeof(cplx) * (size_t)L);
            cplx *work = (cplx *)malloc(sizeof(cplx) * (size_t)(4 * L + 8));
            #pragma omp for schedule(static)
            for (long pidx = 0; pidx < npen; ++pidx) {
                long i1 = pidx / n[o2], i2 = pidx % n[o2];
                long base = i1 * str[o1] + i2 * str[o2];
                for (int j = 0; j < L; ++j) buf[j] = a[base + (long)j * str[ax]];
                fft_rec(buf, 1, L, L, tw, sign, res, work);
                for (int j = 0; j < L; ++j) a[base + (long)j * str[ax]] = res[j];
            }
            free(buf); free(res); free(work);
        }
        free(tw);
    }
    if (sign > 0) {
        double s = 1.0 / (double)N;
        #pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) a[i] *= s;
    }
}

int orc_fft3d(const int32_t n[3], double *data, int32_t nfield, int32_t sign)
{
    int nn[3] = { n[0], n[1], n[2] };
    long N = (long)n[0] * n[1] * n[2];
    for (int f = 0; f < nfield; ++f) fft3d(nn, (cplx *)data + f * N, sign);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Gauss-Legendre nodes on [0,1]: Newton on the three-term recurrence         */
/* ------------------------------------------------------------------------- */
int orc_gauss_legendre(int32_t n, double *u, double *w)
{
    if (n < 1) return ORC_EINVAL;
    for (int i = 0; i < n; ++i) {
        double x = cos(M_PI * (i + 0.75) / (n + 0.5));   /* initial guess */
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = x; p0 = 1.0; }
            /* P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1) */
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        {   /* final derivative at the converged root */
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        /* map [-1,1] -> [0,1] */
        u[i] = 0.5 * (1.0 - x);
        w[i] = 1.0 / ((1.0 - x * x) * dp * dp);   /* = (2/((1-x^2)P'^2)) / 2 */
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Geometry: coordinates, wavenumbers, trap, kinetic and dipolar multipliers  */
/* ------------------------------------------------------------------------- */
typedef struct {
    int n[3];
    long N;
    double h[3], L[3], dV;
    double *V;      /* trap potential, Sec. II Eq. (2)                       */
    double *K2h;    /* |k|^2 / 2                                             */
    double *Ud;     /* (3 kz^2/k^2 - 1) c(|k| Rc), Ud(0) = 0                  */
    int nu;
    double *uq, *wq;
} geom;

/* spherical-cutoff factor c(q) = 1 + 3 cos q / q^2 - 3 sin q / q^3; for small
 * q its Taylor series (the closed form cancels catastrophically there).     */
static double cutoff_factor(double q)
{
    if (q >= 0.5) return 1.0 + 3.0 * cos(q) / (q * q) - 3.0 * sin(q) / (q * q * q);
    /* sum_{m>=2} 3 (-1)^m (2m) q^(2m-2) / (2m+1)! */
    double s = 0.0, q2 = q * q, pw = q2;          /* q^(2m-2) at m = 2 */
    double fact = 120.0;                          /* 5! */
    for (int m = 2; m <= 10; ++m) {
        double sgn = (m % 2 == 0) ? 1.0 : -1.0;
        s += 3.0 * sgn * (2.0 * m) * pw / fact;
        pw *= q2;
        fact *= (2.0 * m + 2.0) * (2.0 * m + 3.0);
    }
    return s;
}

/* Dipolar kernel cut to the slab |z| < Z (dipoles along z; x and y periodic
 * and not cut).  With k_rho = sqrt(kx^2 + ky^2), the in-plane transform of the
 * unit-amplitude kernel at height u is -(3/2) k_rho exp(-k_rho |u|) (from the
 * plane transform of 1/r^3, 2 pi exp(-k_rho |u|) / |u|) plus the contact part
 * 2 delta(u) that makes the uncut kernel (3 kz^2/k^2 - 1); integrating over
 * |u| < Z gives
 *   Ud = (3 kz^2/k^2 - 1) + 3 exp(-k_rho Z) (k_rho^2 cos(kz Z) - k_rho kz sin(kz Z)) / k^2,
 * and Ud(0) = 2, the limit along every direction. */
static double slab_kernel(double kx, double ky, double kz, double Z)
{
    double kr2 = kx * kx + ky * ky, k2 = kr2 + kz * kz;
    if (k2 == 0.0) return 2.0;
    double kr = sqrt(kr2);
    return (3.0 * kz * kz / k2 - 1.0) +
           3.0 * exp(-kr * Z) * (kr2 * cos(kz * Z) - kr * kz * sin(kz * Z)) / k2;
}

static double kvec(int j, int n, double L)
{
    int jj = (j < n / 2) ? j : j - n;
    return 2.0 * M_PI * (double)jj / L;
}

static int lhy_nodes(const orc_params *P, double **u_out, double **w_out);

static int geom_init(geom *g, const orc_grid *gr, const orc_params *P)
{
    memset(g, 0, sizeof(*g));
    for (int d = 0; d < 3; ++d) {
        g->n[d] = gr->n[d];
        g->L[d] = gr->hi[d] - gr->lo[d];
        g->h[d] = g->L[d] / gr->n[d];
    }
    g->N = (long)g->n[0] * g->n[1] * g->n[2];
    g->dV = g->h[0] * g->h[1] * g->h[2];
    g->V = (double *)malloc(sizeof(double) * (size_t)g->N);
    g->K2h = (double *)malloc(sizeof(double) * (size_t)g->N);
    g->Ud = (double *)malloc(sizeof(double) * (size_t)g->N);
    if (!g->V || !g->K2h || !g->Ud) return ORC_ENOMEM;
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    #pragma omp parallel for schedule(static)
    for (int ix = 0; ix < nx; ++ix) {
        double x = gr->lo[0] + ix * g->h[0], kx = kvec(ix, nx, g->L[0]);
        for (int iy = 0; iy < ny; ++iy) {
            double y = gr->lo[1] + iy * g->h[1], ky = kvec(iy, ny, g->L[1]);
            for (int iz = 0; iz < nz; ++iz) {
                double z = gr->lo[2] + iz * g->h[2], kz = kvec(iz, nz, g->L[2]);
                long i = ((long)ix * ny + iy) * nz + iz;
                g->V[i] = 0.5 * (P->omega[0] * P->omega[0] * x * x +
                                 P->omega[1] * P->omega[1] * y * y +
                                 P->omega[2] * P->omega[2] * z * z);
                double k2 = kx * kx + ky * ky + kz * kz;
                g->K2h[i] = 0.5 * k2;
                if (P->dip_cut == 1) g->Ud[i] = slab_kernel(kx, ky, kz, P->r_cut);
                else if (k2 == 0.0) g->Ud[i] = 0.0;
                else g->Ud[i] = (3.0 * kz * kz / k2 - 1.0) * cutoff_factor(sqrt(k2) * P->r_cut);
            }
        }
    }
    g->nu = lhy_nodes(P, &g->uq, &g->wq);
    return ORC_OK;
}

static void geom_free(geom *g)
{
    free(g->V); free(g->K2h); free(g->Ud); free(g->uq); free(g->wq);
}

/* ------------------------------------------------------------------------- */
/* LHY energy density and its derivatives at one point (Sec. II, Eqs. (1),    */
/* (3), (5)).  out[0] = e, out[1] = de/dn1, out[2] = de/dn2.                  */
/* ------------------------------------------------------------------------- */
static void lhy_point(const orc_params *P, int nu, const double *uq, const double *wq,
                      double n1, double n2, double out[3])
{
    double e = 0.0, d1 = 0.0, d2 = 0.0;
    for (int q = 0; q < nu; ++q) {
        double a = 3.0 * uq[q] * uq[q] - 1.0;
        double e11 = P->G[0][0] + P->Gdd[0][0] * a;
        double e22 = P->G[1][1] + P->Gdd[1][1] * a;
        double e12 = P->G[0][1] + P->Gdd[0][1] * a;
        double e21 = P->G[1][0] + P->Gdd[1][0] * a;
        double delta = e11 * n1 - e22 * n2;
        double s = sqrt(delta * delta + 4.0 * e12 * e21 * n1 * n2);
        for (int br = 0; br < 2; ++br) {
            double sg = br == 0 ? 1.0 : -1.0;
            double V = e11 * n1 + e22 * n2 + sg * s;
            if (V <= 0.0) continue;
            double sq = sqrt(V);
            e += wq[q] * V * V * sq;
            double r1 = (s > 0.0) ? (e11 * delta + 2.0 * e12 * e21 * n2) / s : 0.0;
            double r2 = (s > 0.0) ? (-e22 * delta + 2.0 * e12 * e21 * n1) / s : 0.0;
            d1 += wq[q] * V * sq * (e11 + sg * r1);
            d2 += wq[q] * V * sq * (e22 + sg * r2);
        }
    }
    out[0] = P->c_lhy * sqrt(2.0) / (15.0 * M_PI * M_PI) * e;
    out[1] = P->c_lhy / (3.0 * sqrt(2.0) * M_PI * M_PI) * d1;
    out[2] = P->c_lhy / (3.0 * sqrt(2.0) * M_PI * M_PI) * d2;
}

/* ------------------------------------------------------------------------- */
/* Root-split rule for the u integral of Eq. (3) (lhy_quad 1).                */
/* With a = 3u^2 - 1, V_+ V_- = 4 n1 n2 det(a), det = eta_11 eta_22 - eta_12 eta_21 */
/* quadratic in a, and V_+ + V_- = 2 (eta_11 n1 + eta_22 n2).  Since            */
/* N_i eta_ij is symmetric, eta_12 eta_21 >= 0 and s >= |delta|, so for n1 n2 > 0 */
/* a branch changes sign only where det(a) = 0; for n1 n2 = 0 only where        */
/* eta_11(a) = 0 or eta_22(a) = 0.  None of these depends on the densities.    */
/* Between two such points every [V]_+^(k/2) is smooth except at the ends,     */
/* where it behaves as (u - u_b)^(k/2); the map u = p + (q - p)(1 - cos(pi t))/2 */
/* makes those ends smooth (u - p ~ t^2, du ~ t dt), and n Gauss-Legendre nodes */
/* in t then converge exponentially.                                           */
/* ------------------------------------------------------------------------- */
static int add_root(double a, double *roots, int n)
{
    if (isfinite(a) && a > -1.0 && a < 2.0) roots[n++] = sqrt((a + 1.0) / 3.0);
    return n;
}

/* u nodes and weights on [0,1] for P (allocated here; returns the count) */
static int lhy_nodes(const orc_params *P, double **u_out, double **w_out)
{
    int n = P->n_u;
    double br[8];
    int nb = 0;
    if (P->lhy_quad == 1) {
        const double (*G)[2] = P->G, (*D)[2] = P->Gdd;
        double A = D[0][0] * D[1][1] - D[0][1] * D[1][0];
        double B = G[0][0] * D[1][1] + D[0][0] * G[1][1] - G[0][1] * D[1][0] - D[0][1] * G[1][0];
        double C = G[0][0] * G[1][1] - G[0][1] * G[1][0];
        if (A != 0.0) {
            double disc = B * B - 4.0 * A * C;
            if (disc >= 0.0) {
                double q = -0.5 * (B + copysign(sqrt(disc), B));   /* the stable pair of roots */
                if (q != 0.0) { nb = add_root(q / A, br, nb); nb = add_root(C / q, br, nb); }
                else nb = add_root(0.0, br, nb);
            }
        } else if (B != 0.0) {
            nb = add_root(-C / B, br, nb);
        }
        for (int i = 0; i < 2; ++i)
            if (D[i][i] != 0.0) nb = add_root(-G[i][i] / D[i][i], br, nb);
        /* sort, drop duplicates */
        for (int i = 1; i < nb; ++i)
            for (int j = i; j > 0 && br[j] < br[j - 1]; --j) { double t = br[j]; br[j] = br[j - 1]; br[j - 1] = t; }
        int m = 0;
        for (int i = 0; i < nb; ++i)
            if (m == 0 || br[i] > br[m - 1] + 1e-15) br[m++] = br[i];
        nb = m;
    }
    int pieces = nb + 1;
    int total = (P->lhy_quad == 1) ? n * pieces : n;
    double *u = (double *)malloc(sizeof(double) * (size_t)total);
    double *w = (double *)malloc(sizeof(double) * (size_t)total);
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    double *tw = (double *)malloc(sizeof(double) * (size_t)n);
    orc_gauss_legendre(n, t, tw);
    if (P->lhy_quad != 1) {
        memcpy(u, t, sizeof(double) * (size_t)n);
        memcpy(w, tw, sizeof(double) * (size_t)n);
    } else {
        for (int k = 0; k < pieces; ++k) {
            double p = (k == 0) ? 0.0 : br[k - 1], q = (k == nb) ? 1.0 : br[k];
            for (int j = 0; j < n; ++j) {
                u[k * n + j] = p + (q - p) * 0.5 * (1.0 - cos(M_PI * t[j]));
                w[k * n + j] = tw[j] * (q - p) * 0.5 * M_PI * sin(M_PI * t[j]);
            }
        }
    }
    free(t); free(tw);
    *u_out = u; *w_out = w;
    return total;
}

/* the u rule of P into u, w (host arrays of cap entries); returns the node count or -1 */
int orc_lhy_nodes(const orc_params *P, double *u, double *w, int32_t cap)
{
    double *uu, *ww;
    int n = lhy_nodes(P, &uu, &ww);
    if (n > cap) { free(uu); free(ww); return -1; }
    memcpy(u, uu, sizeof(double) * (size_t)n);
    memcpy(w, ww, sizeof(double) * (size_t)n);
    free(uu); free(ww);
    return n;
}

void orc_lhy_point(const orc_params *P, double n1, double n2, double out[3])
{
    double *u, *w;
    int nu = lhy_nodes(P, &u, &w);
    lhy_point(P, nu, u, w, n1, n2, out);
    free(u); free(w);
}

/* ------------------------------------------------------------------------- */
/* Evaluation of E, H_i psi_i and the per-point potentials (Sec. II)          */
/* ------------------------------------------------------------------------- */
typedef struct {
    cplx *Hpsi;     /* 2N: H_i psi_i (Eq. (6))                                */
    cplx *Tpsi;     /* 2N: -1/2 Laplacian psi_i                               */
    double *n;      /* 2N: n_i = |psi_i|^2                                    */
    double *phi;    /* 2N: Phi_j = Re F^-1[Ud F n_j]                           */
    double *muL;    /* 2N: muLHY_i = (1/N_i) de/dn_i (Eq. (5))                 */
    double *e;      /* N : LHY energy density                                 */
    orc_terms t;
} hstate;

static int hstate_alloc(hstate *s, long N)
{
    memset(s, 0, sizeof(*s));
    s->Hpsi = (cplx *)malloc(sizeof(cplx) * 2 * (size_t)N);
    s->Tpsi = (cplx *)malloc(sizeof(cplx) * 2 * (size_t)N);
    s->n = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    s->phi = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    s->muL = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    s->e = (double *)malloc(sizeof(double) * (size_t)N);
    return (s->Hpsi && s->Tpsi && s->n && s->phi && s->muL && s->e) ? ORC_OK : ORC_ENOMEM;
}

static void hstate_free(hstate *s)
{
    free(s->Hpsi); free(s->Tpsi); free(s->n); free(s->phi); free(s->muL); free(s->e);
}

/* -1/2 Laplacian by the Fourier multiplier |k|^2/2 */
static void apply_kinetic(const geom *g, const cplx *f, cplx *out)
{
    long N = g->N;
    memcpy(out, f, sizeof(cplx) * (size_t)N);
    fft3d(g->n, out, -1);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) out[i] *= g->K2h[i];
    fft3d(g->n, out, +1);
}

/* Phi = Re F^-1 [Ud F f] for a real field f (the dipolar convolution) */
static void dipolar_potential(const geom *g, const double *f, double *phi)
{
    long N = g->N;
    cplx *t = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) t[i] = f[i];
    fft3d(g->n, t, -1);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) t[i] *= g->Ud[i];
    fft3d(g->n, t, +1);
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) phi[i] = creal(t[i]);
    free(t);
}

static void heval(const geom *g, const orc_params *P, const cplx *psi, hstate *s)
{
    long N = g->N;
    double dV = g->dV;
    orc_terms *t = &s->t;
    memset(t, 0, sizeof(*t));
    for (int i = 0; i < 2; ++i) {
        const cplx *pi = psi + i * N;
        #pragma omp parallel for schedule(static)
        for (long x = 0; x < N; ++x)
            s->n[i * N + x] = creal(pi[x]) * creal(pi[x]) + cimag(pi[x]) * cimag(pi[x]);
        apply_kinetic(g, pi, s->Tpsi + i * N);
        dipolar_potential(g, s->n + i * N, s->phi + i * N);
    }
    const double *n1 = s->n, *n2 = s->n + N;
    #pragma omp parallel for schedule(dynamic, 256)
    for (long x = 0; x < N; ++x) {
        double o[3];
        lhy_point(P, g->nu, g->uq, g->wq, n1[x], n2[x], o);
        s->e[x] = o[0];
        s->muL[x] = o[1] / P->N[0];
        s->muL[N + x] = o[2] / P->N[1];
    }
    double *tmp = (double *)malloc(sizeof(double) * (size_t)N);
    for (int i = 0; i < 2; ++i) {
        const cplx *pi = psi + i * N;
        cplx *Hi = s->Hpsi + i * N;
        const double *ni = s->n + i * N;
        /* H_i psi_i = T psi_i + [V + sum_j (G_ij n_j + Gdd_ij Phi_j) + muLHY_i] psi_i */
        #pragma omp parallel for schedule(static)
        for (long x = 0; x < N; ++x) {
            double U = g->V[x] + s->muL[i * N + x];
            for (int j = 0; j < 2; ++j)
                U += P->G[i][j] * s->n[j * N + x] + P->Gdd[i][j] * s->phi[j * N + x];
            Hi[x] = s->Tpsi[i * N + x] + U * pi[x];
        }
        t->norm2[i] = dV * sum_array(ni, N);
        t->E_kin[i] = P->N[i] * dV * re_dot(pi, s->Tpsi + i * N, N);
        t->E_trap[i] = P->N[i] * dV * dot_real(g->V, ni, N);
        for (int j = 0; j < 2; ++j) {
            t->E_c[i][j] = 0.5 * P->N[i] * P->G[i][j] * dV * dot_real(ni, s->n + j * N, N);
            t->E_dd[i][j] = 0.5 * P->N[i] * P->Gdd[i][j] * dV * dot_real(ni, s->phi + j * N, N);
        }
        t->mu[i] = dV * re_dot(pi, Hi, N) / t->norm2[i];
        /* shift alpha_i = <psi_i,(H_i - sum_j Gdd_ij Phi_j) psi_i>/<psi_i,psi_i> */
        #pragma omp parallel for schedule(static)
        for (long x = 0; x < N; ++x) {
            double Ud = P->Gdd[i][0] * s->phi[x] + P->Gdd[i][1] * s->phi[N + x];
            tmp[x] = Ud * ni[x];
        }
        t->shift[i] = (dV * re_dot(pi, Hi, N) - dV * sum_array(tmp, N)) / t->norm2[i];
        /* residual norm ||H_i psi_i - mu_i psi_i|| (Sec. III, Eqs. (7)-(8)) */
        #pragma omp parallel for schedule(static)
        for (long x = 0; x < N; ++x) {
            cplx r = Hi[x] - t->mu[i] * pi[x];
            tmp[x] = creal(r) * creal(r) + cimag(r) * cimag(r);
        }
        t->res[i] = sqrt(dV * sum_array(tmp, N));
    }
    t->E_lhy = dV * sum_array(s->e, N);
    t->E = t->E_lhy;
    for (int i = 0; i < 2; ++i) {
        t->E += t->E_kin[i] + t->E_trap[i];
        for (int j = 0; j < 2; ++j) t->E += t->E_c[i][j] + t->E_dd[i][j];
    }
    free(tmp);
}

static int check_inputs(const orc_grid *gr, const orc_params *P)
{
    for (int d = 0; d < 3; ++d) {
        if (gr->n[d] < 2 || gr->n[d] % 2) return ORC_EINVAL;
        if (!(gr->hi[d] > gr->lo[d])) return ORC_EINVAL;
    }
    if (P->n_u < 1 || P->N[0] <= 0 || P->N[1] <= 0) return ORC_EINVAL;
    if (P->dip_cut != 0 && P->dip_cut != 1) return ORC_EINVAL;
    if (P->lhy_quad != 0 && P->lhy_quad != 1) return ORC_EINVAL;
    /* the slab cut is exact on the periodic grid when the cut kernel fits in one period */
    if (P->dip_cut == 1 && !(P->r_cut > 0.0 && 2.0 * P->r_cut <= gr->hi[2] - gr->lo[2])) return ORC_EINVAL;
    return ORC_OK;
}

/* Energy terms; optional outputs H_i psi_i (2N complex), Phi (2N), muLHY (2N). */
int orc_heval(const orc_grid *gr, const orc_params *P, const double *psi_d,
              double *hpsi_d, double *phi, double *muL, orc_terms *out)
{
    int st = check_inputs(gr, P);
    if (st) return st;
    geom g;
    if ((st = geom_init(&g, gr, P))) { geom_free(&g); return st; }
    hstate s;
    if ((st = hstate_alloc(&s, g.N))) { hstate_free(&s); geom_free(&g); return st; }
    heval(&g, P, (const cplx *)psi_d, &s);
    if (hpsi_d) memcpy(hpsi_d, s.Hpsi, sizeof(cplx) * 2 * (size_t)g.N);
    if (phi) memcpy(phi, s.phi, sizeof(double) * 2 * (size_t)g.N);
    if (muL) memcpy(muL, s.muL, sizeof(double) * 2 * (size_t)g.N);
    if (out) *out = s.t;
    hstate_free(&s);
    geom_free(&g);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Preconditioners (Sec. IV.B)                                                */
/* ------------------------------------------------------------------------- */
static void precond_V(const geom *g, const orc_params *P, const hstate *s, double sigma,
                      const cplx *r, cplx *z)
{
    long N = g->N;
    for (int i = 0; i < 2; ++i) {
        #pragma omp parallel for schedule(static)
        for (long x = 0; x < N; ++x) {
            double diag = s->t.shift[i] + g->V[x] + s->muL[i * N + x];
            for (int j = 0; j < 2; ++j) diag += P->G[i][j] * s->n[j * N + x];
            if (diag < 0.0) diag = 0.0;
            z[i * N + x] = r[i * N + x] / (diag + sigma);
        }
    }
}

static void precond_K(const geom *g, const hstate *s, double sigma, const cplx *r, cplx *z)
{
    long N = g->N;
    for (int i = 0; i < 2; ++i) {
        double a = s->t.shift[i] > 0.0 ? s->t.shift[i] : 0.0;
        cplx *zi = z + i * N;
        if (zi != r + i * N) memcpy(zi, r + i * N, sizeof(cplx) * (size_t)N);
        fft3d(g->n, zi, -1);
        #pragma omp parallel for schedule(static)
        for (long x = 0; x < N; ++x) zi[x] /= (a + sigma + g->K2h[x]);
        fft3d(g->n, zi, +1);
    }
}

/* Symmetrised composite (an extension beyond Sec. IV.B, where the composite of
 * Eq. (18) is P_Delta^-1 P_V^-1, which is not symmetric): with D the P_V
 * diagonal, z = D^(-1/2) P_Delta^-1 D^(-1/2) r, symmetric and positive
 * definite because both factors are. */
static void precond_S(const geom *g, const orc_params *P, const hstate *s, double sigma,
                      const cplx *r, cplx *z)
{
    long N = g->N;
    double *dh = (double *)malloc(sizeof(double) * 2 * (size_t)N);   /* D^(-1/2) */
    for (int i = 0; i < 2; ++i) {
        #pragma omp parallel for schedule(static)
        for (long x = 0; x < N; ++x) {
            double diag = s->t.shift[i] + g->V[x] + s->muL[i * N + x];
            for (int j = 0; j < 2; ++j) diag += P->G[i][j] * s->n[j * N + x];
            if (diag < 0.0) diag = 0.0;
            dh[i * N + x] = 1.0 / sqrt(diag + sigma);
        }
    }
    for (long x = 0; x < 2 * N; ++x) z[x] = dh[x] * r[x];
    precond_K(g, s, sigma, z, z);
    for (long x = 0; x < 2 * N; ++x) z[x] *= dh[x];
    free(dh);
}

/* Weight of P_V in the blended preconditioner for component i: `blend` when
 * it is in [0, 1]; otherwise (blend < 0) the potential share of the shift,
 * w_i = P / (P + K) with K = <psi_i, T psi_i> / ||psi_i||^2 the kinetic part
 * and P = [shift_i - K]_+ the rest (trap, contact, LHY), 1/2 if both vanish. */
static double blend_weight(const orc_params *Pp, const hstate *s, double blend, int i)
{
    if (blend >= 0.0) return blend;
    double K = s->t.E_kin[i] / (Pp->N[i] * s->t.norm2[i]);
    double Pot = s->t.shift[i] - K;
    if (Pot < 0.0) Pot = 0.0;
    return (Pot + K > 0.0) ? Pot / (Pot + K) : 0.5;
}

/* Blended preconditioner (a weighted combination of the two preconditioners of
 * Sec. IV.B, which Sec. III allows; not the composite of Eq. (18)):
 * z_i = w_i P_V,i^-1 r_i + (1 - w_i) P_Delta,i^-1 r_i, symmetric and positive
 * definite as a convex combination of two such operators. */
static void precond_B(const geom *g, const orc_params *P, const hstate *s, double sigma, double blend,
                      const cplx *r, cplx *z)
{
    long N = g->N;
    cplx *zv = (cplx *)malloc(sizeof(cplx) * 2 * (size_t)N);
    precond_V(g, P, s, sigma, r, zv);
    precond_K(g, s, sigma, r, z);
    for (int i = 0; i < 2; ++i) {
        double w = blend_weight(P, s, blend, i);
        for (long x = 0; x < N; ++x) z[i * N + x] = w * zv[i * N + x] + (1.0 - w) * z[i * N + x];
    }
    free(zv);
}

/* z = P^-1 r for mode 0 (identity), 1 (P_V), 2 (P_Delta), 3 (P_Delta P_V),
 * 4 (symmetrised composite), 5 (blend of P_V and P_Delta, weight `blend`) */
static void precond_apply(const geom *g, const orc_params *P, const hstate *s, int mode,
                          double sigma, double blend, const cplx *r, cplx *z)
{
    long N = g->N;
    switch (mode) {
    case 1: precond_V(g, P, s, sigma, r, z); break;
    case 2: precond_K(g, s, sigma, r, z); break;
    case 3: precond_V(g, P, s, sigma, r, z); precond_K(g, s, sigma, z, z); break;
    case 4: precond_S(g, P, s, sigma, r, z); break;
    case 5: precond_B(g, P, s, sigma, blend, r, z); break;
    default: memcpy(z, r, sizeof(cplx) * 2 * (size_t)N); break;
    }
}

int orc_precond(const orc_grid *gr, const orc_params *P, int32_t mode, double sigma, double blend,
                const double *psi_d, const double *r_d, double *z_d)
{
    int st = check_inputs(gr, P);
    if (st) return st;
    geom g;
    if ((st = geom_init(&g, gr, P))) { geom_free(&g); return st; }
    hstate s;
    if ((st = hstate_alloc(&s, g.N))) { hstate_free(&s); geom_free(&g); return st; }
    heval(&g, P, (const cplx *)psi_d, &s);
    precond_apply(&g, P, &s, mode, sigma, blend, (const cplx *)r_d, (cplx *)z_d);
    hstate_free(&s);
    geom_free(&g);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Second-order energy model along the geodesic (Sec. V)                      */
/* ------------------------------------------------------------------------- */
typedef struct {
    double E1p[2];      /* E'_i = 2 N_i Re<p_i, H_MF,i psi_i>                  */
    double E1_lhy;      /* E'_LHY                                              */
    double E2ij[2][2];  /* E''_ij (E''_ii includes the one-body part)          */
    double E2_lhy;      /* E''_LHY                                             */
    double E1, E2;      /* totals                                              */
    double pnorm[2];    /* ||p_i||                                             */
    double rp;          /* sum_i 2 N_i Re<p_i, r_i> (needs r)                  */
} model_t;

static void model_coeffs(const geom *g, const orc_params *P, const cplx *psi,
                         const hstate *s, const cplx *p, model_t *m)
{
    long N = g->N;
    double dV = g->dV;
    memset(m, 0, sizeof(*m));
    double *rho = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    double *phr = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    cplx *Tp = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    cplx *tmpc = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)N);
    double gam2inv[2];
    for (int i = 0; i < 2; ++i) {
        const cplx *pi = p + i * N, *si = psi + i * N;
        m->pnorm[i] = sqrt(dV * weighted_norm2(NULL, pi, N));
        gam2inv[i] = m->pnorm[i] * m->pnorm[i];      /* 1/gamma_i^2 */
        /* rho_i = Re(psi_i conj(p_i)) */
        #pragma omp parallel for schedule(static)
        for (long x = 0; x < N; ++x) rho[i * N + x] = creal(si[x] * conj(pi[x]));
        dipolar_potential(g, rho + i * N, phr + i * N);
    }
    for (int i = 0; i < 2; ++i) {
        const cplx *pi = p + i * N, *si = psi + i * N;
        /* H_MF,i psi_i = H_i psi_i - muLHY_i psi_i */
        #pragma omp parallel for schedule(static)
        for (long x = 0; x < N; ++x) tmpc[x] = s->Hpsi[i * N + x] - s->muL[i * N + x] * si[x];
        m->E1p[i] = 2.0 * P->N[i] * dV * re_dot(pi, tmpc, N);
        double psiHpsi = dV * re_dot(si, tmpc, N);
        /* <p_i, H_MF,i p_i> = <p_i, T p_i> + dV sum U_MF,i |p_i|^2 */
        apply_kinetic(g, pi, Tp);
        double pTp = dV * re_dot(pi, Tp, N);
        #pragma omp parallel for schedule(static)
        for (long x = 0; x < N; ++x) {
            double U = g->V[x];
            for (int j = 0; j < 2; ++j)
                U += P->G[i][j] * s->n[j * N + x] + P->Gdd[i][j] * s->phi[j * N + x];
            tmp[x] = U;
        }
        double pUp = dV * weighted_norm2(tmp, pi, N);
        /* w_ij = 2 [G_ij rho_j + Gdd_ij Phi[rho_j]] psi_i; E''_ij = 2 N_i Re<w_ij, p_i> */
        for (int j = 0; j < 2; ++j) {
            #pragma omp parallel for schedule(static)
            for (long x = 0; x < N; ++x)
                tmpc[x] = 2.0 * (P->G[i][j] * rho[j * N + x] + P->Gdd[i][j] * phr[j * N + x]) * si[x];
            m->E2ij[i][j] = 2.0 * P->N[i] * dV * re_dot(tmpc, pi, N);
        }
        m->E2ij[i][i] += 2.0 * P->N[i] * (pTp + pUp - gam2inv[i] * psiHpsi);
    }
    /* LHY part: V^1, V^2 per node; E'_LHY, E''_LHY */
    if (P->c_lhy != 0.0) {
        double *t1 = (double *)malloc(sizeof(double) * (size_t)N);
        double *t2 = (double *)malloc(sizeof(double) * (size_t)N);
        #pragma omp parallel for schedule(dynamic, 256)
        for (long x = 0; x < N; ++x) {
            double n1 = s->n[x], n2 = s->n[N + x];
            double n1p = 2.0 * rho[x], n2p = 2.0 * rho[N + x];
            double p1 = creal(p[x]) * creal(p[x]) + cimag(p[x]) * cimag(p[x]);
            double p2 = creal(p[N + x]) * creal(p[N + x]) + cimag(p[N + x]) * cimag(p[N + x]);
            double n1pp = p1 - n1 * gam2inv[0], n2pp = p2 - n2 * gam2inv[1];
            double a1 = 0.0, a2 = 0.0;
            for (int q = 0; q < g->nu; ++q) {
                double a = 3.0 * g->uq[q] * g->uq[q] - 1.0;
                double e11 = P->G[0][0] + P->Gdd[0][0] * a;
                double e22 = P->G[1][1] + P->Gdd[1][1] * a;
                double e12 = P->G[0][1] + P->Gdd[0][1] * a;
                double e21 = P->G[1][0] + P->Gdd[1][0] * a;
                double delta = e11 * n1 - e22 * n2;
                double d1 = e11 * n1p - e22 * n2p;
                double d2 = e11 * n1pp - e22 * n2pp;
                double s2 = delta * delta + 4.0 * e12 * e21 * n1 * n2;
                double sq = sqrt(s2);
                double A = delta * d1 + 2.0 * e12 * e21 * (n1 * n2p + n1p * n2);
                double B = d1 * d1 + 2.0 * delta * d2 + 4.0 * e12 * e21 * (n1p * n2p + n1 * n2pp + n1pp * n2);
                double lin1 = e11 * n1p + e22 * n2p, lin2 = e11 * n1pp + e22 * n2pp;
                for (int br = 0; br < 2; ++br) {
                    double sg = br == 0 ? 1.0 : -1.0;
                    double V = e11 * n1 + e22 * n2 + sg * sq;
                    if (V <= 0.0) continue;
                    /* B/(2s) - A^2/(2s^3) written as (B - (A/s)^2)/(2s): s^3 underflows
                     * where the densities are ~1e-135 (box corners) */
                    double As = sq > 0.0 ? A / sq : 0.0;
                    double V1 = lin1 + sg * As;
                    double V2 = lin2 + (sq > 0.0 ? sg * (B - As * As) / (2.0 * sq) : 0.0);
                    double rv = sqrt(V);
                    a1 += g->wq[q] * V * rv * V1;
                    a2 += g->wq[q] * (V * rv * V2 + 0.75 * rv * V1 * V1);
                }
            }
            t1[x] = a1;
            t2[x] = a2;
        }
        double K1 = P->c_lhy / (3.0 * sqrt(2.0) * M_PI * M_PI);
        m->E1_lhy = K1 * dV * sum_array(t1, N);
        m->E2_lhy = 2.0 * K1 * dV * sum_array(t2, N);
        free(t1); free(t2);
    }
    m->E1 = m->E1p[0] + m->E1p[1] + m->E1_lhy;
    m->E2 = m->E2ij[0][0] + m->E2ij[0][1] + m->E2ij[1][0] + m->E2ij[1][1] + m->E2_lhy;
    free(rho); free(phr); free(Tp); free(tmpc); free(tmp);
}

int orc_model(const orc_grid *gr, const orc_params *P, const double *psi_d, const double *p_d,
              double *out /* 14 doubles */)
{
    int st = check_inputs(gr, P);
    if (st) return st;
    geom g;
    if ((st = geom_init(&g, gr, P))) { geom_free(&g); return st; }
    hstate s;
    if ((st = hstate_alloc(&s, g.N))) { hstate_free(&s); geom_free(&g); return st; }
    heval(&g, P, (const cplx *)psi_d, &s);
    model_t m;
    model_coeffs(&g, P, (const cplx *)psi_d, &s, (const cplx *)p_d, &m);
    double v[14] = { m.E1p[0], m.E1p[1], m.E1_lhy, m.E2ij[0][0], m.E2ij[0][1], m.E2ij[1][0],
                     m.E2ij[1][1], m.E2_lhy, m.E1, m.E2, m.pnorm[0], m.pnorm[1], 0.0, 0.0 };
    memcpy(out, v, sizeof(v));
    hstate_free(&s);
    geom_free(&g);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Geodesic on the product of spheres (Sec. III, Eq. (9); Sec. V)             */
/* psi_i(alpha) = cos(theta_i) psi_i + sin(theta_i) p_i/||p_i||, theta_i =     */
/* alpha ||p_i||, then divided by its norm.                                   */
/* ------------------------------------------------------------------------- */
static void geodesic(const geom *g, const cplx *psi, const cplx *p, const double pnorm[2],
                     double alpha, cplx *out)
{
    long N = g->N;
    for (int i = 0; i < 2; ++i) {
        const cplx *si = psi + i * N, *pi = p + i * N;
        cplx *oi = out + i * N;
        if (pnorm[i] > 0.0) {
            double th = alpha * pnorm[i];
            double c = cos(th), sn = sin(th) / pnorm[i];
            #pragma omp parallel for schedule(static)
            for (long x = 0; x < N; ++x) oi[x] = c * si[x] + sn * pi[x];
        } else {
            memcpy(oi, si, sizeof(cplx) * (size_t)N);
        }
        double nrm = sqrt(g->dV * weighted_norm2(NULL, oi, N));
        #pragma omp parallel for schedule(static)
        for (long x = 0; x < N; ++x) oi[x] /= nrm;
    }
}

int orc_geodesic(const orc_grid *gr, const double *psi_d, const double *p_d, double alpha,
                 double *out_d)
{
    orc_params P;
    memset(&P, 0, sizeof(P));
    P.N[0] = P.N[1] = 1.0; P.n_u = 1;
    geom g;
    int st = geom_init(&g, gr, &P);
    if (st) { geom_free(&g); return st; }
    double pn[2];
    for (int i = 0; i < 2; ++i)
        pn[i] = sqrt(g.dV * weighted_norm2(NULL, (const cplx *)p_d + i * g.N, g.N));
    geodesic(&g, (const cplx *)psi_d, (const cplx *)p_d, pn, alpha, (cplx *)out_d);
    geom_free(&g);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Derivatives of E with respect to the couplings at fixed psi                */
/* out: dE/dG[2][2] (4), dE/dGdd[2][2] (4), dE/dc_lhy (1)                      */
/* ------------------------------------------------------------------------- */
int orc_param_grad(const orc_grid *gr, const orc_params *P, const double *psi_d, double *out)
{
    int st = check_inputs(gr, P);
    if (st) return st;
    geom g;
    if ((st = geom_init(&g, gr, P))) { geom_free(&g); return st; }
    hstate s;
    if ((st = hstate_alloc(&s, g.N))) { hstate_free(&s); geom_free(&g); return st; }
    heval(&g, P, (const cplx *)psi_d, &s);
    long N = g.N;
    double dV = g.dV;
    double dG[2][2], dD[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            dG[i][j] = 0.5 * P->N[i] * dV * dot_real(s.n + i * N, s.n + j * N, N);
            dD[i][j] = 0.5 * P->N[i] * dV * dot_real(s.n + i * N, s.phi + j * N, N);
        }
    /* LHY: de/d eta_ij at each node, chained through eta_ij = G_ij + Gdd_ij (3u^2-1) */
    double *acc = (double *)calloc((size_t)N * 8, sizeof(double));
    const double K = sqrt(2.0) / (15.0 * M_PI * M_PI);
    #pragma omp parallel for schedule(dynamic, 256)
    for (long x = 0; x < N; ++x) {
        double n1 = s.n[x], n2 = s.n[N + x];
        double a8[8] = { 0 };
        for (int q = 0; q < g.nu; ++q) {
            double a = 3.0 * g.uq[q] * g.uq[q] - 1.0;
            double e11 = P->G[0][0] + P->Gdd[0][0] * a;
            double e22 = P->G[1][1] + P->Gdd[1][1] * a;
            double e12 = P->G[0][1] + P->Gdd[0][1] * a;
            double e21 = P->G[1][0] + P->Gdd[1][0] * a;
            double delta = e11 * n1 - e22 * n2;
            double sq = sqrt(delta * delta + 4.0 * e12 * e21 * n1 * n2);
            for (int br = 0; br < 2; ++br) {
                double sg = br == 0 ? 1.0 : -1.0;
                double V = e11 * n1 + e22 * n2 + sg * sq;
                if (V <= 0.0) continue;
                double f = 2.5 * V * sqrt(V) * g.wq[q];
                double dv[4];   /* dV/d eta_11, eta_12, eta_21, eta_22 */
                dv[0] = n1 + (sq > 0.0 ? sg * delta * n1 / sq : 0.0);
                dv[3] = n2 - (sq > 0.0 ? sg * delta * n2 / sq : 0.0);
                dv[1] = sq > 0.0 ? sg * 2.0 * e21 * n1 * n2 / sq : 0.0;
                dv[2] = sq > 0.0 ? sg * 2.0 * e12 * n1 * n2 / sq : 0.0;
                for (int c = 0; c < 4; ++c) {
                    a8[c] += f * dv[c];
                    a8[4 + c] += f * dv[c] * a;
                }
            }
        }
        for (int c = 0; c < 8; ++c) acc[(long)c * N + x] = a8[c];
    }
    for (int c = 0; c < 4; ++c) {
        int i = c / 2, j = c % 2;
        dG[i][j] += P->c_lhy * K * dV * sum_array(acc + (long)c * N, N);
        dD[i][j] += P->c_lhy * K * dV * sum_array(acc + (long)(4 + c) * N, N);
    }
    /* dE/dc_lhy = E_LHY / c_lhy, evaluated directly with c = 1 */
    double *ec = (double *)malloc(sizeof(double) * (size_t)N);
    orc_params P1 = *P;
    P1.c_lhy = 1.0;
    #pragma omp parallel for schedule(dynamic, 256)
    for (long x = 0; x < N; ++x) {
        double o[3];
        lhy_point(&P1, g.nu, g.uq, g.wq, s.n[x], s.n[N + x], o);
        ec[x] = o[0];
    }
    double dc = dV * sum_array(ec, N);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) { out[2 * i + j] = dG[i][j]; out[4 + 2 * i + j] = dD[i][j]; }
    out[8] = dc;
    free(ec); free(acc);
    hstate_free(&s);
    geom_free(&g);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* The preconditioned nonlinear CG iteration (Sec. III Algorithm 1, Secs. IV-V)*/
/* ------------------------------------------------------------------------- */
static int finite2(double a, double b) { return isfinite(a) && isfinite(b); }

/* Optional trace of the first trace_cap accepted steps (test instrumentation):
 * per step n, six fields of 2 N complex values in this order: psi^(n) at the
 * start of the step, r^(n), the preconditioned residual z that the accepted
 * direction used, p^(n-1) (zero at n = 0), the unprojected direction d and the
 * projected direction p^(n). */
enum { TR_PSI = 0, TR_R, TR_Z, TR_POLD, TR_D, TR_P, TR_FIELDS };

int orc_solve_trace(const orc_grid *gr, const orc_params *P, const orc_opts *o, double *psi_d,
                    orc_report *rep, orc_iter *log, int32_t log_cap, double *trace, int32_t trace_cap)
{
    int st = check_inputs(gr, P);
    if (st) return st;
    geom g;
    if ((st = geom_init(&g, gr, P))) { geom_free(&g); return st; }
    long N = g.N;
    double dV = g.dV;
    cplx *psi = (cplx *)psi_d;
    hstate cur, tri;
    hstate_alloc(&cur, N);
    hstate_alloc(&tri, N);
    size_t vb = sizeof(cplx) * 2 * (size_t)N;
    cplx *r = (cplx *)malloc(vb), *z = (cplx *)malloc(vb), *p = (cplx *)malloc(vb);
    cplx *r_old = (cplx *)malloc(vb), *p_old = (cplx *)malloc(vb), *ptr = (cplx *)malloc(vb);
    cplx *d_last = trace ? (cplx *)malloc(vb) : NULL;   /* unprojected d, for the trace */
    memset(rep, 0, sizeof(*rep));

    /* the iterate lives on the manifold: normalise each component */
    for (int i = 0; i < 2; ++i) {
        double nrm = sqrt(dV * weighted_norm2(NULL, psi + i * N, N));
        for (long x = 0; x < N; ++x) psi[i * N + x] /= nrm;
    }
    heval(&g, P, psi, &cur);

    const double w[2] = { (P->N[0] / (P->N[0] + P->N[1])) * (P->N[0] / (P->N[0] + P->N[1])),
                          (P->N[1] / (P->N[0] + P->N[1])) * (P->N[1] / (P->N[0] + P->N[1])) };
    int have_prev = 0, n = 0, status = ORC_ENOTCONV, stall_it = 0;
    double E_prev = NAN, alpha_prev = 0.0, rz_old = 0.0, stall_ref = INFINITY;

    for (;;) {
        /* 1. residual r_i = H_i psi_i - mu_i psi_i and convergence (Sec. III) */
        double res_max = 0.0;
        for (int i = 0; i < 2; ++i) {
            double mu = cur.t.mu[i];
            for (long x = 0; x < N; ++x) r[i * N + x] = cur.Hpsi[i * N + x] - mu * psi[i * N + x];
            if (cur.t.res[i] > res_max) res_max = cur.t.res[i];
        }
        if (!finite2(cur.t.E, res_max)) { status = ORC_ENONFINITE; break; }
        if (res_max < o->tol_grad) { status = ORC_OK; break; }
        if (o->tol_dE > 0.0 && n > 0 && fabs(cur.t.E - E_prev) < o->tol_dE) { status = ORC_OK; break; }
        /* stall rule (not in the paper): the residual must halve within
         * stall_window accepted steps of its last halving */
        if (res_max < 0.5 * stall_ref) {
            stall_ref = res_max;
            stall_it = n;
        } else if (o->stall_window > 0 && n - stall_it >= o->stall_window) {
            status = ORC_ESTALLED;
            break;
        }
        if (n >= o->max_iter) { status = ORC_ENOTCONV; break; }

        /* 2. preconditioned residual z = P^-1 r (Sec. IV.B) */
        precond_apply(&g, P, &cur, o->pc, o->sigma, o->blend, r, z);

        /* 3. conjugacy parameter: HS+ (default) or PR+ (Sec. IV.C) */
        int restart = !have_prev || o->beta == 2 ||
                      (o->restart_period > 0 && n % o->restart_period == 0);
        double beta = 0.0, beta_num = 0.0, beta_den = 0.0;
        if (!restart) {
            double num = 0.0, den = 0.0;
            for (int i = 0; i < 2; ++i) {
                double yz = 0.0, yp = 0.0;
                for (long x = 0; x < N; ++x) {
                    cplx y = r[i * N + x] - r_old[i * N + x];
                    yz += creal(conj(y) * z[i * N + x]);
                    yp += creal(conj(y) * p_old[i * N + x]);
                }
                num += w[i] * dV * yz;
                den += w[i] * dV * (o->beta == 1 ? 0.0 : yp);
            }
            if (o->beta == 1) den = rz_old;
            beta = (den > 0.0 && isfinite(den) && isfinite(num)) ? num / den : 0.0;
            if (beta < 0.0) beta = 0.0;
            beta_num = num;
            beta_den = den;
        }
        /* level 0: computed beta; 1: beta = 0; 2: z = P_V^-1 r; 3: z = r.
         * path bits: 1 Armijo backtracking, 2 beta = 0 retry after a failed
         * line search, 4 fallback preconditioner (composite only).         */
        int level = (beta > 0.0) ? 0 : 1;
        int path = 0, accepted = 0, trials = 0, stagnated = 0, halvings = 0;
        double rz_now = 0.0, alpha = 0.0, alpha_model = 0.0, pmax = 0.0, rp_acc = 0.0, Et = NAN;
        model_t m;
        memset(&m, 0, sizeof(m));
        while (!accepted && !stagnated) {
            /* 4. direction d = -z + beta p_old, projected onto the tangent
             *    space; restart (beta = 0) when <r,p> >= 0 (Sec. IV.C, V)  */
            double rp = 0.0;
            for (;;) {
                double b = (level == 0) ? beta : 0.0;
                if (level == 2) precond_apply(&g, P, &cur, 1, o->sigma, 0.0, r, z);
                if (level == 3) memcpy(z, r, vb);
                rp = 0.0;
                for (int i = 0; i < 2; ++i) {
                    for (long x = 0; x < N; ++x)
                        p[i * N + x] = -z[i * N + x] + (b > 0.0 ? b * p_old[i * N + x] : 0.0);
                    if (d_last) memcpy(d_last + i * N, p + i * N, sizeof(cplx) * (size_t)N);
                    double c = dV * re_dot(p + i * N, psi + i * N, N);   /* Re<d_i,psi_i> */
                    for (long x = 0; x < N; ++x) p[i * N + x] -= c * psi[i * N + x];
                    rp += 2.0 * P->N[i] * dV * re_dot(p + i * N, r + i * N, N);
                }
                if (rp < 0.0 && isfinite(rp)) break;
                if (level == 0) { level = 1; rep->n_restarts++; continue; }
                if (level == 1 && o->pc >= 3) { level = 2; path |= 4; continue; }
                if (level == 2) { level = 3; continue; }
                stagnated = 1;
                break;
            }
            if (stagnated) break;
            rz_now = 0.0;
            for (int i = 0; i < 2; ++i) rz_now += w[i] * dV * re_dot(r + i * N, z + i * N, N);

            /* 5. second-order model and closed-form step (Sec. V) */
            model_coeffs(&g, P, psi, &cur, p, &m);
            m.rp = rp;
            rp_acc = rp;
            pmax = m.pnorm[0] > m.pnorm[1] ? m.pnorm[0] : m.pnorm[1];
            if (m.E2 > 0.0 && isfinite(m.E2) && isfinite(m.E1) && -m.E1 / m.E2 > 0.0)
                alpha = -m.E1 / m.E2;
            else
                alpha = alpha_prev > 0.0 ? alpha_prev : 0.1 / pmax;
            if (alpha * pmax > o->theta_max) alpha = o->theta_max / pmax;
            alpha_model = alpha;
            halvings = 0;

            /* 6. validate along the exact geodesic; Armijo backtracking */
            double tau = o->tau_rel * fabs(cur.t.E);
            geodesic(&g, psi, p, m.pnorm, alpha, ptr);
            heval(&g, P, ptr, &tri);
            trials++;
            Et = tri.t.E;
            if (isfinite(Et) && Et <= cur.t.E + tau) {
                accepted = 1;
            } else {
                for (int k = 0; k < o->max_backtrack; ++k) {
                    alpha *= 0.5;
                    geodesic(&g, psi, p, m.pnorm, alpha, ptr);
                    heval(&g, P, ptr, &tri);
                    trials++;
                    halvings++;
                    rep->n_backtracks++;
                    Et = tri.t.E;
                    if (isfinite(Et) && Et <= cur.t.E + o->armijo_c1 * alpha * m.E1 + tau) {
                        accepted = 1;
                        path |= 1;
                        break;
                    }
                }
            }
            if (!accepted) {
                if (level == 0) { level = 1; rep->n_restarts++; path |= 2; continue; }
                stagnated = 1;
            }
        }
        if (stagnated) { status = ORC_ESTAGNATED; break; }

        /* 7. accept: keep r, p (and <r,z>) for the next conjugacy parameter */
        if (log && n < log_cap) {
            orc_iter *L = &log[n];
            L->iter = n; L->n_trials = trials; L->restarted = (level >= 1);
            L->path = path; L->E = Et; L->res_max = res_max;
            L->E1 = m.E1; L->E2 = m.E2; L->alpha = alpha; L->beta = (level == 0) ? beta : 0.0;
            L->level = level; L->halvings = halvings;
            L->beta_num = beta_num; L->beta_den = beta_den; L->rp = rp_acc;
            L->alpha_model = alpha_model; L->pmax = pmax; L->E0 = cur.t.E;
            L->tau = o->tau_rel * fabs(cur.t.E);
        }
        if (trace && n < trace_cap) {
            cplx *T = (cplx *)trace + (size_t)n * TR_FIELDS * 2 * (size_t)N;
            memcpy(T + TR_PSI * 2 * N, psi, vb);
            memcpy(T + TR_R * 2 * N, r, vb);
            memcpy(T + TR_Z * 2 * N, z, vb);
            if (have_prev) memcpy(T + TR_POLD * 2 * N, p_old, vb);
            else memset(T + TR_POLD * 2 * N, 0, vb);
            memcpy(T + TR_D * 2 * N, d_last, vb);
            memcpy(T + TR_P * 2 * N, p, vb);
        }
        E_prev = cur.t.E;
        memcpy(psi, ptr, vb);
        hstate tmp = cur; cur = tri; tri = tmp;
        memcpy(r_old, r, vb);
        memcpy(p_old, p, vb);
        rz_old = rz_now;
        alpha_prev = alpha;
        have_prev = 1;
        n++;
    }
    rep->iters = n;
    rep->status = status;
    rep->final = cur.t;
    free(r); free(z); free(p); free(r_old); free(p_old); free(ptr); free(d_last);
    hstate_free(&cur); hstate_free(&tri);
    geom_free(&g);
    return status;
}

int orc_solve(const orc_grid *gr, const orc_params *P, const orc_opts *o, double *psi_d,
              orc_report *rep, orc_iter *log, int32_t log_cap)
{
    return orc_solve_trace(gr, P, o, psi_d, rep, log, log_cap, NULL, 0);
}

/* ------------------------------------------------------------------------- */
/* Imaginary-time evolution, the comparison method of Sec. VI (8 FFTs per     */
/* step in the paper's count: forward and inverse transforms of psi_1, psi_2  */
/* and of the two densities).  The paper states only the scheme's class and   */
/* its stopping rule; the step used here (a reading, listed in the design     */
/* notes) is the normalised first-order time splitting of the gradient flow   */
/* d psi_i / d tau = -H_i psi_i:                                              */
/*   psi_i <- N[ exp(-dt U_i(psi)) F^-1 exp(-dt |k|^2/2) F psi_i ],           */
/*   U_i = V + sum_j (G_ij n_j + Gdd_ij Phi_j) + muLHY_i  at the current psi, */
/* N normalising each component.  E is evaluated at every iterate; the run    */
/* stops at the first n >= 1 with |E(psi^n) - E(psi^(n-1))| < tol_dE          */
/* (Sec. VI.B uses 1e-6) and returns psi^n.                                   */
/* ------------------------------------------------------------------------- */
typedef struct {
    double dt;
    double tol_dE;
    int32_t max_iter;
    int32_t pad;
} orc_ite_opts;

int orc_ite(const orc_grid *gr, const orc_params *P, const orc_ite_opts *o, double *psi_d,
            orc_report *rep, double *logE, int32_t log_cap)
{
    int st = check_inputs(gr, P);
    if (st) return st;
    if (!(o->dt > 0.0) || o->max_iter < 0) return ORC_EINVAL;
    geom g;
    if ((st = geom_init(&g, gr, P))) { geom_free(&g); return st; }
    long N = g.N;
    double dV = g.dV;
    cplx *psi = (cplx *)psi_d;
    hstate cur;
    hstate_alloc(&cur, N);
    cplx *hat = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    memset(rep, 0, sizeof(*rep));

    for (int i = 0; i < 2; ++i) {
        double nrm = sqrt(dV * weighted_norm2(NULL, psi + i * N, N));
        for (long x = 0; x < N; ++x) psi[i * N + x] /= nrm;
    }
    int n = 0, status = ORC_ENOTCONV;
    double E_prev = NAN;
    for (;;) {
        heval(&g, P, psi, &cur);
        double E = cur.t.E;
        if (logE && n < log_cap) logE[n] = E;
        if (!isfinite(E)) { status = ORC_ENONFINITE; break; }
        if (n >= 1 && fabs(E - E_prev) < o->tol_dE) { status = ORC_OK; break; }
        if (n >= o->max_iter) { status = ORC_ENOTCONV; break; }
        E_prev = E;
        for (int i = 0; i < 2; ++i) {
            cplx *pi = psi + i * N;
            /* kinetic factor in Fourier space */
            memcpy(hat, pi, sizeof(cplx) * (size_t)N);
            fft3d(g.n, hat, -1);
            for (long x = 0; x < N; ++x) hat[x] *= exp(-o->dt * g.K2h[x]);
            fft3d(g.n, hat, +1);
            /* potential factor with U_i at the current iterate */
            for (long x = 0; x < N; ++x) {
                double U = g.V[x] + cur.muL[i * N + x];
                for (int j = 0; j < 2; ++j)
                    U += P->G[i][j] * cur.n[j * N + x] + P->Gdd[i][j] * cur.phi[j * N + x];
                pi[x] = exp(-o->dt * U) * hat[x];
            }
            double nrm = sqrt(dV * weighted_norm2(NULL, pi, N));
            for (long x = 0; x < N; ++x) pi[x] /= nrm;
        }
        n++;
    }
    rep->iters = n;
    rep->status = status;
    rep->final = cur.t;
    free(hat);
    hstate_free(&cur);
    geom_free(&g);
    return status;
}
