/*
 * bec.h -- C ABI of the MI355X (gfx950) library for ground states of a
 * two-component dipolar Bose-Einstein condensate with Lee-Huang-Yang (LHY)
 * corrections, computed by the preconditioned nonlinear conjugate-gradient
 * method on the product-of-spheres manifold of arXiv:2510.24543.
 *
 * Problem (Sec. II, Eq. (1); Sec. III): minimise E[psi_1, psi_2] subject to
 * ||psi_1|| = ||psi_2|| = 1, where
 *   E = sum_i N_i [ <psi_i, T psi_i> + int V n_i + 1/2 sum_j G_ij int n_i n_j
 *                   + 1/2 sum_j Gdd_ij int n_i Phi_j ] + int e_LHY(n_1, n_2),
 *   T = -1/2 Laplacian, V = 1/2 sum_d omega_d^2 x_d^2 (Eq. (2)), n_i = |psi_i|^2,
 *   Phi_j = F^-1[ Ud F n_j ], Ud(k) = (3 kz^2/|k|^2 - 1) c(|k| r_cut), Ud(0) = 0,
 *   c(q) = 1 + 3 cos q / q^2 - 3 sin q / q^3 (dipolar kernel cut off at radius
 *   r_cut, field along z), and e_LHY = c_lhy sqrt(2)/(15 pi^2) int_0^1 du
 *   sum_+- [V_+-(u)]_+^(5/2) with V_+- of Eq. (3) and couplings
 *   eta_ij = G_ij + Gdd_ij (3u^2 - 1).  The u integral is Gauss-Legendre with
 *   n_u nodes.  Gdd_ij is the amplitude of the k-space dipolar kernel.
 *
 * Discretisation: Fourier pseudo-spectral on the periodic box [lo, hi) with
 * n[d] points per axis, x_d[j] = lo_d + j h_d, h_d = (hi_d - lo_d)/n_d,
 * <f,g> = dV sum conj(f) g, dV = h_x h_y h_z.
 *
 * Conventions shared by every entry point
 *  - Fields are DEVICE pointers to complex128 stored as interleaved (re, im)
 *    double pairs, layout C order [2][nx][ny][nz] (component, x, y, z; z
 *    fastest), 16-byte aligned.  The caller owns every field buffer and the
 *    workspace; the library never allocates device memory after bec_create
 *    and never frees caller memory.
 *  - All device work is enqueued on the HIP stream given to bec_create.
 *    Entry points that return host structs synchronise that stream before
 *    returning; bec_fft3d is asynchronous.
 *  - Supported axis lengths: 8, 16, 32, 48, 64, 96, 128, 256 (each axis
 *    independently).  Other lengths return BEC_EUNSUPPORTED.
 *  - Errors are reported by the status code; bec_last_error() gives a
 *    thread-local message.  No C++ exception crosses this boundary.
 *    A non-finite reduced scalar gives BEC_ENONFINITE.
 *  - One context serves one stream and one thread at a time.
 */
#ifndef BEC_H
#define BEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BEC_OK = 0,
    BEC_EINVAL = 1,        /* invalid argument                                   */
    BEC_ENOMEM = 2,        /* workspace too small                                */
    BEC_EHIP = 3,          /* a HIP runtime call failed                          */
    BEC_ENOTCONV = 4,      /* solve stopped at max_iter                          */
    BEC_ESTAGNATED = 5,    /* no descent even after the beta = 0 restart         */
    BEC_ENONFINITE = 6,    /* a reduced scalar was NaN or infinite               */
    BEC_EUNSUPPORTED = 7,  /* axis length not supported                          */
    BEC_ESTALLED = 8       /* the residual stopped falling (bec_opts.stall_window) */
} bec_status;

/* Periodic box [lo, hi) with n points per axis (x, y, z). */
typedef struct {
    int32_t n[3];
    double lo[3], hi[3];
} bec_grid;

/* Physical parameters in harmonic-oscillator units (Sec. II).  N_i G_ij and
 * N_i Gdd_ij must be symmetric (the energy form requires it).
 * Dipolar truncation (dip_cut):
 *  0  spherical cutoff of radius r_cut, Ud(k) = (3 kz^2/|k|^2 - 1) c(|k| r_cut),
 *     Ud(0) = 0, for a condensate isolated in all three directions;
 *  1  slab cut for a condensate periodic in x and y (the setups of Sec. VI.C):
 *     the interaction kept for |z - z'| < r_cut, not cut in x, y:
 *     Ud(k) = (3 kz^2/|k|^2 - 1) + 3 exp(-k_rho r_cut)(k_rho^2 cos(kz r_cut)
 *             - k_rho kz sin(kz r_cut))/|k|^2, Ud(0) = 2, k_rho^2 = kx^2 + ky^2;
 *     needs 2 r_cut <= hi[2] - lo[2] (BEC_EINVAL otherwise), where it is the
 *     exact convolution with the cut kernel on the periodic grid. */
typedef struct {
    double N[2];        /* atom numbers N_i > 0                                */
    double omega[3];    /* trap ratios lambda_d (Eq. (2))                      */
    double G[2][2];     /* contact couplings G_ij                              */
    double Gdd[2][2];   /* dipolar k-space amplitudes                          */
    double c_lhy;       /* multiplier of the LHY term (1 = the paper)          */
    double r_cut;       /* dipolar cutoff: radius (dip_cut 0) or slab half-height (1), > 0 */
    int32_t n_u;        /* Gauss-Legendre nodes for the u integral, 1..64 (per
                           piece of [0,1] when lhy_quad = 1)                    */
    int32_t dip_cut;    /* 0 spherical cutoff, 1 slab cut (periodic x, y)      */
    int32_t lhy_quad;   /* u rule: 0 Gauss-Legendre, n_u nodes on [0,1];
                           1 root-split, n_u nodes on each piece between the
                           points where a branch potential can change sign
                           (zeros of det eta(u) and of eta_11(u), eta_22(u));
                           at most 64 nodes in all (BEC_EINVAL otherwise)     */
} bec_params;

/* Preconditioners of Sec. IV.B: identity, real-space diagonal P_V, kinetic
 * P_Delta (Fourier diagonal), and the composite P_Delta^-1 P_V^-1 (Eq. (18));
 * and, beyond the paper, the symmetrised composite D^-1/2 P_Delta^-1 D^-1/2
 * with D the P_V diagonal (symmetric and positive definite, unlike Eq. (18)). */
typedef enum { BEC_PC_NONE = 0, BEC_PC_V = 1, BEC_PC_KIN = 2, BEC_PC_COMPOSITE = 3, BEC_PC_SYMMETRIC = 4,
               BEC_PC_BLEND = 5 } bec_precond;

/* BEC_PC_BLEND: the weighted combination z_i = w_i P_V,i^-1 r_i + (1 - w_i)
 * P_Delta,i^-1 r_i of the two preconditioners (Sec. III allows weighted
 * combinations; the conclusion names dynamic weighting as an extension),
 * symmetric and positive definite.  w_i = bec_opts.blend in [0, 1], or, for a
 * negative bec_opts.blend, the potential share of the preconditioner shift:
 * [shift_i - K_i]_+ / ([shift_i - K_i]_+ + K_i), K_i = <psi_i, T psi_i> / ||psi_i||^2,
 * recomputed at every iterate (1/2 if both parts vanish). */

/* Conjugacy parameter of Sec. IV.C: Hestenes-Stiefel+, Polak-Ribiere+, or 0. */
typedef enum { BEC_BETA_HS_PLUS = 0, BEC_BETA_PR_PLUS = 1, BEC_BETA_ZERO = 2 } bec_beta;

/* bec_opts.flags.  BEC_SOLVE_SYNCHRONOUS: the host reads every reduced scalar
 * before it enqueues the launches that depend on it.  By default bec_solve
 * pipelines each iteration: the device decides the step, the trial, the next
 * preconditioned residual, its reduce sums and the next direction write
 * from the reduced sums it has just produced, and the host waits once per
 * iteration and checks every decision against the same rules; restarts and
 * backtracking fall back to synchronous launches.  Both give the same iterates
 * bit for bit.  Bits other than these two are rejected (BEC_EINVAL). */
#define BEC_SOLVE_SYNCHRONOUS 1
/* BEC_SOLVE_CONTINUE: continue the iteration the last bec_solve call on this
 * context stopped at its max_iter (status BEC_ENOTCONV) instead of starting
 * one: no normalisation, first Hamiltonian or first reduce, and the work that
 * call had already enqueued for the next step is used.  That call must have had
 * the same pc, beta, restart_period, sigma, blend and BEC_SOLVE_SYNCHRONOUS bit,
 * and no call that computes on the context may have come in between (every
 * call but bec_get_tuning, bec_profile_enable and bec_profile_read ends the
 * continuable state; else BEC_EINVAL).
 * psi_inout is only written (the final iterate); max_iter counts this call's
 * steps, the log starts at its first step (bec_iter.iter keeps the running
 * index, which the restart period and the stall window use), and report.iters
 * counts this call's steps.  A solve split this way gives the iterates of one
 * uninterrupted solve bit for bit. */
#define BEC_SOLVE_CONTINUE 2

typedef struct {
    int32_t pc;             /* bec_precond                                     */
    int32_t beta;           /* bec_beta                                        */
    int32_t max_iter;       /* accepted steps before BEC_ENOTCONV              */
    int32_t restart_period; /* beta = 0 when iter mod restart_period == 0; 0 off */
    int32_t max_backtrack;  /* Armijo halvings per step                        */
    int32_t flags;          /* BEC_SOLVE_* bits; 0 = default                   */
    int32_t stall_window;   /* > 0: stop with BEC_ESTALLED when max_i ||r_i||
                               has not fallen below half of its reference value
                               within the last stall_window accepted steps (the
                               reference is reset each time it is halved); 0 off */
    int32_t reserved;       /* 0                                               */
    double tol_grad;        /* stop when max_i ||H_i psi_i - mu_i psi_i|| < tol */
    double tol_dE;          /* stop when |E_n - E_(n-1)| < tol_dE (0: off)     */
    double sigma;           /* regularising shift of P_V and P_Delta           */
    double armijo_c1;       /* sufficient-decrease constant                    */
    double theta_max;       /* largest geodesic angle per step                 */
    double tau_rel;         /* a step is accepted when E_new <= E + tau_rel|E| */
    double blend;           /* BEC_PC_BLEND: weight of P_V in [0, 1]; < 0 adaptive */
} bec_opts;

/* Energy decomposition at one state (Sec. II, Eq. (1); Sec. III, Eq. (7)). */
typedef struct {
    double E;
    double E_kin[2], E_trap[2], E_c[2][2], E_dd[2][2], E_lhy;
    double mu[2];       /* <psi_i, H_i psi_i> / <psi_i, psi_i>                  */
    double shift[2];    /* preconditioner shift alpha_i                         */
    double res[2];      /* ||H_i psi_i - mu_i psi_i||                           */
    double norm2[2];    /* ||psi_i||^2                                          */
} bec_terms;

/* One line search (Sec. V).  path bits: 1 Armijo backtracking was used. */
typedef struct {
    double E0, E1, E2, alpha, theta[2], E_new, pnorm[2];
    int32_t n_trials, path;
} bec_ls_report;

/* Per accepted step of bec_solve.  path bits: 1 Armijo, 2 beta = 0 retry after
 * a failed line search, 4 fallback preconditioner (composite only). */
typedef struct {
    int32_t iter, n_trials, restarted, path;
    double E, res_max, E1, E2, alpha, beta;
} bec_iter;

typedef struct {
    int32_t iters, n_restarts, n_backtracks, status;
    bec_terms final;
    double seconds;     /* wall time of the solve (host clock)                 */
} bec_report;

typedef struct bec_ctx bec_ctx;

/* Bytes of device workspace bec_create needs for this grid (about 450 bytes per
 * grid point).  Returns BEC_EINVAL / BEC_EUNSUPPORTED for a bad grid. */
bec_status bec_workspace_size(const bec_grid* grid, const bec_params* params, size_t* bytes);

/* Create a context.  hip_stream: a hipStream_t (NULL = the null stream).
 * workspace: device buffer of at least bec_workspace_size bytes, 256-byte
 * aligned, owned by the caller and kept alive until bec_destroy.  Builds the
 * FFT twiddle tables, the dipolar kernel table and the quadrature nodes. */
bec_status bec_create(const bec_grid* grid, const bec_params* params, void* hip_stream,
                      void* workspace, size_t workspace_bytes, bec_ctx** out);

bec_status bec_destroy(bec_ctx* ctx);

/* Change the physical parameters of an existing context (same grid).  Rebuilds
 * the dipolar table if r_cut changed and the quadrature nodes. */
bec_status bec_set_params(bec_ctx* ctx, const bec_params* params);

/* 3D DFT of nfield consecutive fields of shape [nx][ny][nz] (in, out device
 * pointers, may alias).  sign = -1: forward, unnormalised; sign = +1: inverse
 * including the factor 1/(nx ny nz).  Asynchronous.  nfield in 1..3. */
bec_status bec_fft3d(bec_ctx* ctx, const double* in, double* out, int32_t nfield, int32_t sign);

/* Energy terms of psi (Sec. II, Eq. (1)).  Synchronises. */
bec_status bec_energy(bec_ctx* ctx, const double* psi, bec_terms* out_h);

/* H_i psi_i of Eq. (6) for both components into hpsi (device, same layout),
 * plus the energy terms.  Synchronises. */
bec_status bec_hamiltonian(bec_ctx* ctx, const double* psi, double* hpsi, bec_terms* out_h);

/* Gradient of E with respect to the discrete field, written to grad (device):
 *   projected = 0: dE/dRe psi + i dE/dIm psi = 2 N_i dV H_i psi_i;
 *   projected = 1: 2 N_i dV (H_i psi_i - mu_i psi_i), the tangent residual of
 *   Sec. III, Eq. (8), scaled the same way.
 * Synchronises. */
bec_status bec_gradient(bec_ctx* ctx, const double* psi, double* grad, int32_t projected,
                        bec_terms* out_h);

/* E (Sec. II, Eq. (1)) and the Euclidean gradient 2 N_i dV H_i psi_i of
 * bec_gradient (projected = 0) without synchronising: every launch is enqueued
 * on the context stream and the call returns.  E is written to E_dev (device
 * memory, one double) by the stream, bit for bit the E of bec_energy; a state
 * with a non-finite energy leaves a non-finite value there (no status).  The
 * autograd energy uses it so that its forward needs no host round trip. */
bec_status bec_energy_gradient_async(bec_ctx* ctx, const double* psi, double* grad, double* E_dev);

/* The gradient of bec_gradient without a context and without allocating:
 * for callers that cannot allocate device or pinned host memory at call time
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and results as bec_gradient (grad must not be
 * null, out_h may be) plus the grid, the parameters and the HIP stream (NULL =
 * the null stream) that bec_create would take.  The workspace of a context
 * (bec_workspace_size bytes) and the reduced scalars live in a fixed device
 * array of BEC_NOALLOC_SCRATCH_BYTES that every GPU the library runs on holds
 * until the process ends; a grid whose workspace does not fit (above about
 * 147,000 points: 48^3 and 64 x 64 x 32 fit, 64 x 64 x 48 does not) returns
 * BEC_ENOMEM before any device work.  The call rebuilds its tables each time
 * (host work growing with the grid), runs on default launch plans, and
 * synchronises the stream before returning.  Calls on one device are
 * serialised by a lock inside the library; the array keeps the last call's
 * contents.  Calls no hipMalloc / hipFree / hipHostMalloc. */
#define BEC_NOALLOC_SCRATCH_BYTES (64u << 20)
bec_status bec_gradient_noalloc(const bec_grid* grid, const bec_params* params, void* hip_stream, const double* psi,
                                double* grad, int32_t projected, bec_terms* out_h);

/* z = P^-1 r for the preconditioner pc evaluated at psi (Sec. IV.B; shift
 * alpha_i = <psi_i,(T + V + sum_j G_ij n_j + muLHY_i) psi_i>, regularised by
 * sigma).  r and z are device fields (may alias).  Synchronises. */
bec_status bec_precond_apply(bec_ctx* ctx, int32_t pc, double sigma, const double* psi,
                             const double* r, double* z);

/* z = w P_V^-1 r + (1 - w) P_Delta^-1 r (BEC_PC_BLEND) at psi with the weight
 * blend in [0, 1], or the adaptive weight when blend < 0 (bec_precond_apply with
 * BEC_PC_BLEND uses the adaptive weight).  Same conventions as
 * bec_precond_apply; BEC_EINVAL for blend > 1.  Synchronises. */
bec_status bec_precond_apply_blend(bec_ctx* ctx, double blend, double sigma, const double* psi, const double* r,
                                   double* z);

/* One manifold line search (Sec. V): projects d onto the tangent space at psi,
 * builds the second-order energy model, proposes alpha = -E1/E2, validates it
 * along the exact geodesic and falls back to Armijo halving.  psi_out receives
 * the accepted point (device; may not alias psi).  opts supplies theta_max,
 * armijo_c1, max_backtrack and tau_rel.  Synchronises. */
bec_status bec_linesearch(bec_ctx* ctx, const double* psi, const double* d, double* psi_out,
                          const bec_opts* opts, bec_ls_report* out_h);

/* Full preconditioned nonlinear CG solve (Sec. III, Algorithm 1, with the
 * direction of Sec. IV and the step of Sec. V).  psi_inout (device) holds the
 * initial state (normalised on entry) and receives the final state.  log_h is
 * an optional host array of log_cap bec_iter records.  Returns the solve
 * status (also in out_h->status). */
bec_status bec_solve(bec_ctx* ctx, double* psi_inout, const bec_opts* opts, bec_report* out_h,
                     bec_iter* log_h, int32_t log_cap);

/* Options of the imaginary-time baseline. */
typedef struct {
    double dt;          /* imaginary-time step > 0                              */
    double tol_dE;      /* stop when |E(psi^n) - E(psi^(n-1))| < tol_dE        */
    int32_t max_iter;   /* steps before BEC_ENOTCONV                            */
    int32_t flags;      /* BEC_SOLVE_SYNCHRONOUS or 0 (default: pipelined steps) */
} bec_ite_opts;

/* Imaginary-time evolution, the method the paper compares against (Sec. VI;
 * its stopping rule |Delta E| < 1e-6 is Sec. VI.B).  One step is the
 * normalised first-order splitting of d psi_i/d tau = -H_i psi_i:
 *   psi_i <- N[ exp(-dt U_i(psi)) F^-1 exp(-dt |k|^2/2) F psi_i ],
 * U_i = V + sum_j (G_ij n_j + Gdd_ij Phi_j) + muLHY_i at the current iterate,
 * N normalising each component.  The energy of every iterate is evaluated (its
 * kinetic part by Parseval inside the same transforms); the run stops at the
 * first n >= 1 with |E(psi^n) - E(psi^(n-1))| < tol_dE and returns psi^n.
 * psi_inout (device) holds the initial state (normalised on entry) and
 * receives the final one; log_h optionally receives E(psi^0..) (host, log_cap
 * doubles); out_h->final holds the energy terms and residual norms of the
 * returned state, out_h->iters the steps taken.  Returns BEC_OK, BEC_ENOTCONV
 * (max_iter steps), BEC_EINVAL or BEC_ENONFINITE.  By default step n + 1 is
 * enqueued (its normalisation taken on the device from step n's sums) before
 * the host reads step n's energy, so the host waits once per step without
 * leaving the GPU idle; the iterates and energies are bit-identical to the
 * BEC_SOLVE_SYNCHRONOUS schedule. */
bec_status bec_ite_solve(bec_ctx* ctx, double* psi_inout, const bec_ite_opts* opts, bec_report* out_h,
                         double* log_h, int32_t log_cap);

/* Derivatives of E with respect to the couplings at fixed psi, each matrix
 * entry treated as independent: dG[i][j] = dE/dG_ij, dGdd[i][j] = dE/dGdd_ij,
 * dc_lhy = dE/dc_lhy.  At a converged state these are the derivatives of the
 * ground-state energy (the constraint set does not depend on the couplings).
 * Synchronises. */
bec_status bec_param_grad(bec_ctx* ctx, const double* psi, double dG[2][2], double dGdd[2][2],
                          double* dc_lhy);

/* ---------------------------------------------------------------------------
 * Batched scan: many independent instances (grids may differ; instances with
 * the same grid shape are processed together by every kernel launch) solved by
 * the same preconditioned CG as bec_solve, with the scalar decisions taken on
 * the device so that a round of the iteration needs no host synchronisation.
 * Every preconditioner of bec_opts.pc (Sec. IV.B, Eqs. (14)-(18)); the
 * k-space ones (BEC_PC_KIN, _COMPOSITE, _SYMMETRIC, _BLEND) transform the
 * residual of the instances that start a direction in one batched FFT pass
 * set per round, each instance with its own P_V shift, and the composite
 * family keeps the fallback z = P_V^-1 r, then z = r, of bec_solve.
 * ------------------------------------------------------------------------- */
typedef struct bec_batch bec_batch;

/* Device workspace for n_inst instances (grids[i], params[i]); about 360 bytes
 * per grid point summed over the instances, plus per-instance tables. */
bec_status bec_batch_workspace_size(int32_t n_inst, const bec_grid* grids, const bec_params* params,
                                    size_t* bytes);

/* Create a batch.  Same conventions as bec_create; the batch also owns one
 * internal stream (default priority) used only to capture graphs. */
bec_status bec_batch_create(int32_t n_inst, const bec_grid* grids, const bec_params* params, void* hip_stream,
                            void* workspace, size_t workspace_bytes, bec_batch** out);

bec_status bec_batch_destroy(bec_batch* b);


/* Solve every instance.  opts->pc outside 0..5, or a blend weight above 1 with
 * BEC_PC_BLEND, is BEC_EINVAL.  psi_inout: host array of n_inst device pointers, each
 * an initial state of its instance's grid (normalised on entry) that receives
 * the final state.  rounds_per_sync: iteration rounds enqueued between two
 * host checks of the instance states (0: 16).  use_graph: capture those rounds
 * once in a hipGraph and replay it.  reports_h: host array of n_inst reports
 * (seconds = wall time of the whole batch).  Returns BEC_OK when the call
 * completed; per-instance outcomes are in reports_h[i].status. */
bec_status bec_batch_solve(bec_batch* b, double* const* psi_inout, const bec_opts* opts, int32_t rounds_per_sync,
                           int32_t use_graph, bec_report* reports_h);

/* ---------------------------------------------------------------------------
 * Launch tuning.  Every 3D FFT axis pass has several plan variants (threads per
 * pencil, radix order, workgroup size); the pointwise kernels have a grid size.
 * The autotuner (paper_2510_24543_amd/autotune.py) times the choices with
 * bec_time_fft_pass / full iterations and sets the fastest with
 * bec_set_tuning.  Results are identical up to rounding order for every FFT
 * variant and grid size; the LHY table agrees with the node loop to about 1e-14
 * of the LHY terms.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t fft_variant[3][2];  /* per axis (x, y, z): [0] plain passes; [0][1] the x pass with the
                                   fused k-space operator; [2][1] the direction write (P_V, composite) fused
                                   with the line search's forward z pass; [1][1] unused;
                                   0 = default plan */
    int32_t pw_blocks;          /* workgroups of the pointwise kernels (64 .. 4096) */
    int32_t lhy_table;          /* 1 (default): the class-A part of the LHY node sum from Chebyshev
                                   series of its restriction to n1 + n2 = 1 (it is homogeneous of
                                   degree 5/2), when those series match the node sum to 2e-14 of
                                   its range at creation; 0: the node loop */
    int32_t lhy_terms;          /* out: terms per series in use (0: node loop); ignored on set */
    int32_t kin_axes;           /* 1 (default): the kinetic term of the energy evaluation as
                                   T_x + T_y + T_z from one-dimensional transforms inside the trial,
                                   y and x passes; 0: the 3D multiply in the x pass (fewer
                                   transforms per pencil: faster on small, launch-bound grids).
                                   Not used by bec_batch_set_tuning */
    int32_t fuse_z;             /* bit 0 (default on): the direction write with P_V or the composite
                                   P_Delta^-1 P_V^-1 fused with the line search's forward z pass,
                                   and the input of the k-space preconditioners formed in their
                                   first forward z pass; bit 1 (default on): the energy
                                   evaluation's last inverse z pass fused with the Hamiltonian
                                   epilogue (with kin_axes).  A fused pass owns whole z pencils per
                                   workgroup, so on small grids it launches fewer workgroups than the
                                   chip has compute units; off, the grid-stride kernels run instead.
                                   Same results up to rounding order.  Not used by
                                   bec_batch_set_tuning */
} bec_tuning;

bec_status bec_get_tuning(bec_ctx* ctx, bec_tuning* out_h);
bec_status bec_set_tuning(bec_ctx* ctx, const bec_tuning* t);

/* FFT plans for the instances of one grid shape (as chosen for that grid by
 * bec_get_tuning after tuning a single-instance context): per axis the
 * variant of bec_tuning.fft_variant (x: the k-space pass entry [0][1]; y, z:
 * the plain entries); pw_blocks is not used.  Returns BEC_EINVAL if no
 * instance has that grid or a variant does not exist.  Takes effect from the
 * next bec_batch_solve (a captured graph is rebuilt). */
bec_status bec_batch_set_tuning(bec_batch* b, const bec_grid* grid, const bec_tuning* t);

/* Number of plan variants for an axis of length L (host-only). */
bec_status bec_fft_variant_count(int32_t L, int32_t* count);

/* Average duration in milliseconds of `reps` launches of one axis pass over the
 * three fields of the context's work area, with plan `variant`: kind 0 forward,
 * 1 inverse, 2 the x pass with the fused kinetic / dipolar operators (axis 0
 * only).  HIP events on the context stream; overwrites the work area (not
 * the caller's fields).  Synchronises. */
bec_status bec_time_fft_pass(bec_ctx* ctx, int32_t axis, int32_t kind, int32_t variant, int32_t reps,
                             double* ms_out);

/* Per-kernel timing statistics (see bec_profile_enable). */
typedef struct {
    char name[40];          /* kernel class, e.g. "fft_y_fwd", "heval_epilogue"  */
    int64_t launches;
    double total_ms;        /* sum of event-measured launch durations          */
    double total_bytes;     /* algorithmic HBM bytes of those launches: every
                               operand read once, every result written once   */
} bec_kernel_stat;

/* Start (on = 1, clearing earlier statistics) or stop (on = 0) per-kernel
 * timing.  While on, every launch of the context is bracketed by HIP events
 * recorded on the context stream; this adds a few microseconds per launch,
 * so timed runs keep it off. */
bec_status bec_profile_enable(bec_ctx* ctx, int32_t on);

/* Copy up to cap kernel statistics into out_h (host) and their number into
 * n_out.  Synchronises the context stream. */
bec_status bec_profile_read(bec_ctx* ctx, bec_kernel_stat* out_h, int32_t cap, int32_t* n_out);

/* Gauss-Legendre nodes u[0..n) and weights w[0..n) on [0,1] used for the LHY
 * u integral (host memory, caller-owned, n in 1..64).  Host-only: needs no GPU. */
bec_status bec_gauss_legendre(int32_t n, double* u, double* w);

/* A two-component dipolar mixture in laboratory units.  The energy functional
 * of Sec. II has one kinetic term -1/2 nabla^2 for both components, so a single
 * atomic mass m fixes the oscillator length l = sqrt(hbar / (m omega_0)). */
typedef struct {
    double mass_amu;        /* atomic mass m in unified atomic mass units, > 0           */
    double a_bohr[2][2];    /* s-wave scattering lengths a_ij in Bohr radii, symmetric   */
    double mu_bohr[2];      /* magnetic moments along the field in Bohr magnetons;
                               opposite signs make counter-polarised components          */
    double N[2];            /* atom numbers N_i > 0                                      */
    double f0_hz;           /* unit frequency omega_0 / 2 pi in Hz, > 0                  */
    double trap_hz[3];      /* trap frequencies omega_d / 2 pi in Hz, >= 0               */
    double c_lhy;           /* multiplier of the LHY term (1 = the paper's model)        */
    double r_cut_um;        /* dipolar cutoff radius in micrometres, > 0                 */
    int32_t n_u;            /* Gauss-Legendre nodes for the u integral, 1..64            */
    int32_t contact_2pi;    /* 0: G_ij = 4 pi a_ij N_j / l, the contact coupling
                               4 pi hbar^2 a / m that the LHY prefactor of Eq. (1)
                               assumes; 1: the prefactor 2 pi as printed in Sec. II       */
    int32_t dip_cut;        /* copied to bec_params.dip_cut (0 or 1)                      */
} bec_physical;

/* Convert laboratory units into the oscillator units of Sec. II (host-only:
 * needs no GPU).  lambda_d = omega_d / omega_0; G_ij = 4 pi a_ij N_j / l;
 * Gdd_ij = mu_0 mu_i mu_j N_j / (3 l^3 hbar omega_0), the k-space amplitude,
 * which is (4 pi / 3) times the real-space coefficient D_ij of Sec. II because
 * the Fourier transform of (1 - 3 cos^2 theta) / r^3 is (4 pi / 3)(3 cos^2 alpha - 1);
 * r_cut = r_cut_um / l; c_lhy and n_u are copied.  Constants: CODATA 2018.
 * in_h and out_h are caller-owned host structs; length_m_h (host, may be null)
 * receives l in metres, by which lengths such as the box edges are divided.
 * BEC_EINVAL on a null in_h/out_h, a mass, unit frequency, atom number or
 * cutoff that is not finite and positive, a negative or non-finite trap
 * frequency, a non-finite or asymmetric a_ij, a non-finite mu_i or c_lhy,
 * n_u outside 1..64, or contact_2pi other than 0 and 1. */
bec_status bec_params_from_physical(const bec_physical* in_h, bec_params* out_h, double* length_m_h);

/* Thread-local message of the last failing call on this thread. */
const char* bec_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BEC_H */
