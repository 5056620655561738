// Internal declarations of the gfx950 library: kernel argument blocks and
// launchers shared by the FFT, pointwise and host translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "pcg_rules.h"

namespace bec {

constexpr int kMaxNodes = 64;        // Gauss-Legendre nodes for the LHY u integral
constexpr int kNodeStride = 8;       // doubles per node in the node table
constexpr int kPwThreads = 256;      // threads per block of the pointwise kernels
constexpr int kPwMaxBlocks = 4096;   // largest grid of the pointwise kernels
constexpr int kPwDefaultBlocks = 1024;
constexpr int kMaxSums = 32;         // reduced scalars per pass
constexpr int kLhyTabMax = 64;       // terms per Chebyshev series of the class-A LHY table

// multiplier and shift of the division by d of indices below 2^31 (see PwParams)
inline void div_magic(uint32_t d, uint32_t* m, int* s)
{
    int l = 0;
    while ((1ull << l) < d) ++l;
    *s = 31 + l;
    *m = (uint32_t)(((1ull << (31 + l)) + d - 1) / d);
}

// Butterfly sums over the 64 lanes of a wavefront for M values at once; lane 0
// ends with the wavefront totals (the per-value order of additions is that of
// M separate butterflies).  All M values step through the butterfly together,
// so the lane exchanges of different values are in flight at the same time
// instead of M dependent chains one after another.
template <int M>
__device__ __forceinline__ void wave_sum_down(double (&v)[M])
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] += __shfl_down(v[m], off, 64);
}

// Per-node table entry (kNodeStride doubles):
//   [0] eta_11  [1] eta_22  [2] eta_12 eta_21  [3] w_q  [4] eta_12  [5] eta_21
//   [6] 3u^2 - 1  [7] unused
// eta_ij = G_ij + Gdd_ij (3 u_q^2 - 1); w_q are the weights on [0,1].

// Physical and geometric constants used inside the pointwise kernels.
struct PwParams {
    int nx, ny, nz;
    long long N;               // points per component
    double G[2][2], Gdd[2][2];
    double Nat[2];             // atom numbers N_i
    double K5;                 // c_lhy sqrt(2)/(15 pi^2)   (energy density)
    double K3;                 // c_lhy /(3 sqrt(2) pi^2)   (derivatives)
    int n_u;
    int lhy_on;                // c_lhy != 0
    const double* lhy_tab;     // class-A Chebyshev series (see pw_math.h), lhy_K terms each; lhy_K = 0: node loop
    int lhy_K;
    const double* nodes;       // n_u * kNodeStride (device copy, used by the non-hot kernels)
    // hot-loop copy of (eta_11, eta_22, eta_12 eta_21, w_q, sqrt(det_q)) per
    // node, class-A nodes first (n_a), then class-B nodes (n_b) (see
    // pw_math.h), passed in the kernel-argument block so the u loop reads it
    // through scalar loads
    int n_a, n_b;
    double node5[kMaxNodes][5];
    // i / (ny nz) and r / nz for linear indices below 2^31 by multiply and shift:
    // q = (i * m) >> s with m = ceil(2^(31 + l) / d), s = 31 + l, 2^l >= d (exact
    // for every i < 2^31), set by div_magic on the host
    uint32_t m_nyz, m_nz;
    int s_nyz, s_nz;
    const double* vx;          // 1/2 omega_x^2 x^2 per x index
    const double* vy;
    const double* vz;
    int nblk_pw;               // grid of the pointwise kernels
};

// ---------------------------------------------------------------- FFT passes
enum FftOp : int {
    kOpPlain = 0,       // one direction, store (optionally scaled)
    kOpMulKin = 1,      // forward, times |k|^2/2 /N, inverse, store
    kOpMulDip = 2,      // forward, times Ud(k)/N, inverse, store
    kOpMulPrec = 3,     // forward, times 1/(a_f + |k|^2/2)/N, inverse, store
    kOpParseval = 4,    // forward, accumulate sum |k|^2/2 |v|^2, no store
    kOpExpKin = 5,      // forward, accumulate as kOpParseval, times exp(-a_f |k|^2/2)/N, inverse, store
    // forward along the pass axis only (any pass), accumulate pscale * sum k_a^2/2 |v|^2
    // (k_a the wavenumber of that axis), no store.  T is separable, so the three axis
    // terms of <p, T p>, each from a one-dimensional transform of p itself, add up to
    // the kOpParseval sum when pscale = N / n_a
    kOpParsevalAxis = 6,
    // forward along the pass axis, times k_a^2/2 / n_a, inverse, plus acc[f] (if set), store:
    // the axis term T_a of the separable kinetic operator, accumulated over the passes
    kOpKinAxis = 7,
    // x pass of the line search's densities held as half spectra (field 2 with its own
    // geometry, see S2): forward x, then the kLsEpiSums model sums in k-space, no store.
    // Pencil 2m holds rho^_1 and pencil 2m+1 rho^_2 at the same (k_y, k_z), k_z = 0..n_z/2;
    // with w = 1 at k_z = 0, n_z/2 and 2 between (Hermitian symmetry of real fields) and
    // Parseval, sum_n rho_a rho_b = 1/N sum_k w Re(conj(rho^_a) rho^_b) and
    // sum_n rho_a (U * rho_b) = 1/N sum_k w Ud(k) Re(conj(rho^_a) rho^_b)
    kOpDipSums = 8,
    // forward along the contiguous z axis of the packed rho_1 + i rho_2 (sign -1), then the
    // half spectra of the two real densities stored with z extent n_z + 2: dst[pencil (L + 2)
    // + 2 k + c] = rho^_(c+1)(k), k = 0..L/2 (the input of the y and x passes of kOpDipSums)
    kOpHalfSpectra = 9
};

struct BInstState;

struct FftPassArgs {
    const double2* src[3];
    double2* dst[3];
    int op[3];             // per field: any op in a fused (mode 2) pass; Plain or ParsevalAxis otherwise
    double prec_a[3];      // per field shift for kOpMulPrec
    int nfield;
    long long S;           // stride between successive pencil elements
    long long npencil;     // pencils per field
    const double2* tw;     // W_L^m = exp(-2 pi i m / L), m = 0..L-1
    int sign;              // -1 forward, +1 inverse (kOpPlain)
    double scale;          // applied at store (kOpPlain)
    // x-pass multipliers
    int nx, ny, nz;
    const double* kx;      // wavenumbers per axis
    const double* ky;
    const double* kz;
    const double* udtab;   // dipolar kernel on the k octant [nx/2+1][ny/2+1][nz/2+1]
    double inv_n;          // 1/(nx ny nz)
    double* partials;      // kOpParseval / kOpParsevalAxis: [instance][field][block]
    int nblk_x;            // block stride of `partials`
    const double* kaxis;   // kOpParsevalAxis, kOpKinAxis: wavenumbers of the pass axis
    double pscale;         // kOpParsevalAxis: factor of the block sums
    double inv_na;         // kOpKinAxis: 1 / (length of the pass axis)
    const double2* acc[3]; // kOpKinAxis: field added to the result (may be the destination itself)
    // batched passes: grid.z = instance; field f of instance i starts at
    // src[f] + i * src_stride[f] (+ src_sel[i] * src_sel_stride[f]) and
    // dst[f] + i * dst_stride[f]; per-instance k / dipolar tables when
    // per_inst_tab; instances with active[i] == 0 are skipped
    int n_inst;
    long long src_stride[3], dst_stride[3];   // per-field instance strides (elements)
    const int* inst_ids;                      // optional: instance of blockIdx.z (compacted launch)
    const int* src_sel;                       // optional: buffer index per instance
    long long src_sel_stride[3];              // src offset += src_sel[i] * src_sel_stride[f]
    const int* active;
    int per_inst_tab;
    long long udsize;      // doubles per instance in udtab
    // kOpMulPrec shift from device memory (pipelined launches): when
    // prec_state is set, field f < 2 uses [shift_f]_+ + prec_sigma with
    // shift_f = rule_mu_shift(prec_state, prec_Gdd) instead of prec_a[f]
    const double* prec_state;
    double prec_sigma;
    // batched passes: when prec_bst is set, field f < 2 of instance l uses
    // [prec_bst[l].shift_f]_+ + prec_sigma (the instance's P_V shift)
    const BInstState* prec_bst;
    double prec_Gdd[2][2];
    // field of blockIdx.y in a fused pass: fields with an inverse transform
    // first, so that the blocks dispatched last are the light ones (set by the
    // launcher; the results do not depend on it)
    int forder[3];
    // S2 > 0: field 2 has its own geometry, stride S2 and npencil2 pencils (the
    // line search's half spectra, z extent n_z + 2); grid.x covers the larger
    // count and blocks beyond a field's pencils contribute nothing
    long long S2, npencil2;
    double* ls_partials;   // kOpDipSums: the kLsEpiSums block sums, [instance][sum][block]
};

// Forward z pass fused with the geodesic trial update: psi_dst = a_i psi_src +
// b_i p (p may be null) is stored, and the forward z transforms of psi_dst_1,
// psi_dst_2 and of the packed density |psi_dst_1|^2 + i |psi_dst_2|^2 go to
// args.dst[0..2].  args is a z-axis pass (S = 1).
struct TrialZArgs {
    const double2* psi_src;       // 2N
    const double2* p;             // 2N or null
    double a[2], b[2];
    const double* coef;           // non-null: a and b from device memory (a_1, a_2, b_1, b_2) instead
    const double* norm_sums;      // non-null: a_i = 1 / sqrt(norm_dV norm_sums[i]), b = 0 (imaginary time)
    double norm_dV;
    double2* psi_dst;             // 2N (may equal psi_src)
    long long N;                  // points per component
    int kin_z;                    // 1: store T_z psi_i (forward, times k_z^2/2 / n_z, inverse) for
                                  // i = 1, 2 instead of their forward z transforms
};
hipError_t fft_trial_z_pass(int L, int variant, const FftPassArgs& args, const TrialZArgs& z, hipStream_t s);

// Launch one axis pass of length L over args.nfield fields with plan variant
// `variant` (0 = default); `contiguous` for the z axis.
hipError_t fft_pass(int L, int variant, bool contiguous, const FftPassArgs& args, hipStream_t s);
bool fft_supported(int L);
int fft_num_variants(int L);
int fft_blocks(int L, int variant, long long npencil);   // grid.x of a pass
int fft_max_blocks(int L, long long npencil);            // over all variants
int fft_fused_default_variant(int L);                     // default plan of the fused z kernels

// ---------------------------------------------------------------- pointwise kernels

// Imaginary-time step epilogue: out_i = exp(-dt U_i) hat_i with U_i the
// potential part of H_i at psi; sums see kIteSums.
struct IteArgs {
    const double2* psi;           // 2N: the current iterate
    const double2* hat;           // 2N: F^-1 exp(-dt |k|^2/2) F psi_i
    const double2* phi;           // N: Phi_1 + i Phi_2 of psi
    double2* out;                 // 2N
    double dt;
    double* partials;
};
constexpr int kIteSums = 14;
// sums: 0,1 V n_i; 2 n1n1; 3 n1n2; 4 n2n2; 5..8 n_i Phi_j (11,12,21,22); 9 e_LHY;
//       10,11 n_i; 12,13 |out_i|^2

struct HevalArgs {
    const double2* psi;
    const double2* Tpsi;          // 2N: -1/2 Lap psi_i
    const double2* phi;           // N: Phi_1 + i Phi_2
    double2* hpsi;                // 2N out
    double2* aux;                 // 2N out: [0,N) Phi packed (copied unless phi == aux), [N,2N) muLHY_1 + i muLHY_2
    double* partials;
};
constexpr int kHevalSums = 18;
// sums: 0,1 Re<psi_i,Tpsi_i>; 2,3 V n_i; 4 n1n1; 5 n1n2; 6 n2n2; 7..10 n_i Phi_j (11,12,21,22);
//       11 e_LHY; 12,13 Re<psi_i,Hpsi_i>; 14,15 n_i; 16,17 muLHY_i n_i

struct DirArgs {
    const double2* psi;
    const double2* hpsi;
    const double2* aux;           // Phi packed, muLHY packed
    const double2* zbuf;          // z (when zmode == 2), 2N
    const double2* r_old;         // 2N (read by the reduce pass)
    double2* p;                   // 2N: p_old
    double2* p_out;               // 2N: p (write pass; may equal p)
    double2* r_out;               // 2N (write pass)
    double2* rho;                 // N (write pass): rho_1 + i rho_2
    double mu[2];
    double diag_shift[2];         // shift_i for P_V
    double sigma;
    int zmode;                    // 0 identity, 1 P_V, 2 from zbuf, 3 D^-1/2 zbuf (symmetrised composite),
                                  // 4 w P_V^-1 r + (1 - w) zbuf (blend; zbuf = P_Delta^-1 r)
    double blend;                 // zmode 4: bec_opts.blend (the weights from it when dev_state is set)
    double blend_w[2];            // zmode 4: weight of P_V per component
    double zsign;                 // d = zsign z + beta p_old
    double beta;
    double c[2];                  // projection coefficients Re<d_i,psi_i>
    int have_prev;
    double* partials;
    // Pipelined launches, enqueued before the host has read the sums they
    // depend on: when dev_state is set, mu and diag_shift come from the energy
    // sums there (rule_mu_shift); when dev_dir is set (write pass), beta and c
    // come from the direction-reduce sums there (rule_beta with `rule`, then
    // rule_proj).  Both point to device memory written by an earlier launch.
    const double* dev_state;
    const double* dev_dir;
    BetaRule rule;
};
constexpr int kDirReduceSums = 12;
// sums (per component i, index 6*i + k): 0 |r|^2, 1 Re<r - r_old, z>, 2 Re<r - r_old, p_old>,
//   3 Re<z, psi>, 4 Re<p_old, psi>, 5 Re<r, z>
constexpr int kDirWriteSums = 18;
// sums: 0,1 |p_i|^2; 2,3 Re<p_i,r_i>; 4,5 Re<p_i,(H - muL)psi_i>; 6,7 Re<psi_i,(H - muL) psi_i>;
//       8,9 U_MF,i |p_i|^2; 10,11 muL_i |p_i|^2; 12,13 muL_i n_i; 14 LHY V^1 sum; 15 LHY V^2 (n''=0) sum;
//       16,17 Re<p_i, psi_i>

constexpr int kLsEpiSums = 7;    // line-search model epilogue (rho_1 + i rho_2 against K*rho)
// sums: 0 rho1 rho1; 1 rho1 rho2; 2 rho2 rho2; 3..6 rho_i Phi[rho_j] (11, 12, 21, 22)

struct MakeRArgs {                // out = r, P_V^-1 r (apply_pv 1), D^-1/2 r (apply_pv 2; D the P_V diagonal)
                                  // or w P_V^-1 r + (1 - w) zk (apply_pv 3, the blend)
    const double2* psi;
    const double2* hpsi;
    const double2* aux;
    const double2* rin;           // if non-null: r given directly (ignores psi/hpsi/mu)
    double mu[2];
    double diag_shift[2];
    double sigma;
    int apply_pv;
    const double2* zk;            // apply_pv 3: P_Delta^-1 r, 2N
    double blend_w[2];            // apply_pv 3: weight of P_V per component
    double2* out;                 // 2N
    const double* dev_state;      // non-null: mu and diag_shift from these energy sums (rule_mu_shift)
};

struct ParamGradArgs {
    const double2* psi;
    double* partials;
};
constexpr int kParamSums = 9;     // 0..3 de/deta_ij (11,12,21,22); 4..7 same times (3u^2-1); 8 e (c = 1)

hipError_t launch_heval_epi(const PwParams& P, const HevalArgs& a, int nblk, hipStream_t s);
hipError_t launch_ite_epi(const PwParams& P, const IteArgs& a, int nblk, hipStream_t s);
hipError_t launch_dir_reduce(const PwParams& P, const DirArgs& a, int nblk, hipStream_t s);
hipError_t launch_dir_write(const PwParams& P, const DirArgs& a, int nblk, hipStream_t s);
// The direction write (zmode 1 or 2) fused with the line search's forward z pass:
// p, r, rho and the kDirWriteSums sums as launch_dir_write (sums into
// a.partials [sum][block], grid = fft_blocks(L, variant, z.npencil) blocks),
// plus the z-axis Parseval sums of p_1, p_2 (z.partials[f * z.nblk_x + block]
// times z.pscale, f = 0, 1) and the z transforms of rho_1 and rho_2 as half
// spectra: z.dst[2][pencil (L + 2) + 2 k + c] = rho^_(c+1)(k), k = 0..L/2
// (unpacked from the transform of rho_1 + i rho_2).  z: a z-axis pass of the
// grid (tw, kaxis, npencil, S = 1).
hipError_t fft_dirwrite_z_pass(int L, int variant, const FftPassArgs& z, const PwParams& P, const DirArgs& a,
                               hipStream_t s);
// The make_r pass (rin = null, apply_pv 0..2) fused with the forward z pass of
// the k-space preconditioner that follows: a.out (2N) receives the residual
// input already transformed along z.  z: a z-axis pass of the grid (tw,
// npencil, S = 1).
hipError_t fft_maker_z_pass(int L, int variant, const FftPassArgs& z, const PwParams& P, const MakeRArgs& a,
                            hipStream_t s);
// its zmode 2 instantiations (fft_fused_composite.hip)
hipError_t fft_dirwrite_z_pass_composite(int L, int variant, const FftPassArgs& z, const PwParams& P,
                                         const DirArgs& a, hipStream_t s);
// The last inverse z pass of the energy evaluation fused with the Hamiltonian
// epilogue: z.src[0] (= h.aux, in place) holds the packed Phi spectrum after
// the y inverse pass; stores Phi and H psi, muLHY into h.hpsi, h.aux and the
// kHevalSums sums into h.partials [sum][block] (grid = fft_blocks(L, variant,
// z.npencil)).
hipError_t fft_heval_z_pass(int L, int variant, const FftPassArgs& z, const PwParams& P, const HevalArgs& h,
                            hipStream_t s);
hipError_t launch_make_r(const PwParams& P, const MakeRArgs& a, hipStream_t s);
hipError_t launch_param_grad(const PwParams& P, const ParamGradArgs& a, int nblk, hipStream_t s);
hipError_t launch_norm2(const PwParams& P, const double2* f, double* partials, int nblk, hipStream_t s);
hipError_t launch_scale2(const PwParams& P, const double2* in, double2* out, double s0, double s1,
                         hipStream_t s);
hipError_t launch_grad(const PwParams& P, const double2* psi, const double2* hpsi, double2* out,
                       double mu0, double mu1, double s0, double s1, int projected, hipStream_t s);
// E from the reduced energy sums (device) into out[0] (device), one thread
hipError_t launch_energy_from_sums(const PwParams& P, const double* sums, double dV, double* out, hipStream_t s);
// Closed-form step of the second-order model (Sec. V) from the reduced model
// sums, on the device, so the trial point can be enqueued before the host has
// read them.  One thread; writes kStepOut values to out (device) and out_host
// (host-mapped).
struct StepArgs {
    const double* D;              // kDirWriteSums direction-write sums (device)
    const double* LS;             // kLsEpiSums line-search epilogue sums
    const double* pars;           // 2 Parseval sums sum_k |k|^2/2 |FFT(p_i)|^2
    double dV, inv_n;             // cell volume, 1 / points
    double norm2[2];              // |psi_i|^2 of the current state
    double alpha_prev;            // previous accepted step (fallback when the model has no minimum)
    double theta_max;             // largest geodesic angle
    double* out;
    double* out_host;
};
constexpr int kStepOut = 12;
// out: 0,1 a_i; 2,3 b_i (trial psi_i = a_i psi_i + b_i p_i); 4 alpha; 5 <r,p> sum; 6 E';
//      7 E''; 8,9 |p_i|; 10,11 Re<p_i, psi_i> dV
hipError_t launch_ls_step(const PwParams& P, const StepArgs& a, hipStream_t s);

// out[m] = sum_b partials[m * nblk + b] for m < M (fixed order), one block
hipError_t launch_reduce_final(const double* partials, int nblk, int M, double* out, hipStream_t s);
// two or three partial arrays in one launch (M1 rows of nblk1, then M2 rows of
// nblk2, then M3 rows of nblk3)
hipError_t launch_reduce_final2(const double* partials1, int nblk1, int M1, double* out1, const double* partials2,
                                int nblk2, int M2, double* out2, hipStream_t s);
hipError_t launch_reduce_final3(const double* partials1, int nblk1, int M1, double* out1, const double* partials2,
                                int nblk2, int M2, double* out2, const double* partials3, int nblk3, int M3,
                                double* out3, hipStream_t s);
// Reduction segment with an optional second destination: out[m] and, when
// copy is non-null, copy[m] (a device copy of host-mapped results).
struct RedSeg {
    const double* partials;
    int nblk, M;
    double* out;
    double* copy;
};
hipError_t launch_reduce_segs(const RedSeg& s1, const RedSeg& s2, const RedSeg& s3, hipStream_t s);

// ---------------------------------------------------------------- batched scan
// Instances with the same grid shape form a group; every batched kernel covers
// one group (grid.y or grid.z = instance within the group).  The scalar
// decisions of the CG loop run on the device, one thread per instance, so a
// round needs no host synchronisation and can be captured in a graph.
constexpr int kBSumStride = 64;   // reduced scalars per instance
constexpr int kSH = 0;            // 18 Hamiltonian-epilogue sums
constexpr int kSR = 18;           // 12 direction-reduce sums
constexpr int kSW = 30;           // 18 direction-write sums
constexpr int kSL = 48;           // 7 line-search epilogue sums
constexpr int kSP = 55;           // 2 Parseval sums

struct BInstParams {
    double G[2][2], Gdd[2][2], Nat[2], K5, K3, dV;
    double Ntot_w[2];             // stacked inner-product weights (N_i/N)^2
    double inv_npts;              // 1 / (nx ny nz)
    int n_u, lhy_on;
    int n_a, n_b;                 // class-A / class-B node counts of node5
    double node5[kMaxNodes][5];
    int lhy_K;                    // class-A LHY table terms per series (0: node loop), see pw_math.h
    double lhytab[3 * kLhyTabMax];
};

enum : int { kBRunning = 0, kBConverged = 1, kBNotConv = 2, kBStagnated = 3, kBNonFinite = 4, kBStalled = 5 };
enum : int { kBInit = 0, kBNewDir = 1, kBBacktrack = 2, kBRedo = 3 };

struct BInstState {
    int status, phase, cur, iter, have_prev, level, path, nbt, n_restarts, n_backtracks, rounds, stall_it;
    int zlevel;                   // 0: the configured z; 2: z = P_V^-1 r, 3: z = r (fallbacks of the composite family)
    int pad;
    double E, E_prev, mu[2], shift[2], norm2[2], res[2];
    double stall_ref;             // reference residual of the stall rule (halved -> reset)
    double beta, c[2], zpsi[2], ppsi[2], rz[2], rz_old, rz_now, alpha, alpha_prev, E1, E2, rp;
    double pnorm[2], psip[2], a[2], b[2];
    double hsum[kHevalSums];      // Hamiltonian sums of the accepted state
};

struct BOpts {                    // the bec_opts fields the device decisions use
    int beta_mode, max_iter, restart_period, max_backtrack, stall_window, pc;
    double tol_grad, tol_dE, sigma, armijo_c1, theta_max, tau_rel, blend;
};

struct BGroup {
    int first, count;             // global index of the first instance, instances in the group
    const int* ids;               // [n_ids] local indices this launch covers (grid.y = n_ids)
    int n_ids;
    int nx, ny, nz;
    uint32_t m_nyz, m_nz;         // index division by multiply and shift (div_magic)
    int s_nyz, s_nz;
    long long N;
    int nblk;                     // pointwise blocks per instance
    int zmode;                    // z: 0 r, 1 P_V^-1 r, 2 zbuf, 3 D^-1/2 zbuf, 4 w P_V^-1 r + (1 - w) zbuf
    int papply;                   // make_r into zbuf: 0 r, 1 P_V^-1 r, 2 D^-1/2 r (D the P_V diagonal)
    double sigma;
    double blend;                 // the blended mode's weight (< 0: adaptive)
    const int* act_pre;           // [n_inst] instances whose z is computed this round
    const BInstParams* ip;        // [n_inst] (global index)
    BInstState* st;               // [n_inst]
    double* sums;                 // [n_inst][kBSumStride]
    const int* act_dir;           // [n_inst]
    const int* act_trial;         // [n_inst]
    double* const* psi_user;      // [n_inst] caller's device fields
    const double* vx;             // [count][nx], trap per axis
    const double* vy;
    const double* vz;
    double2* psi;                 // [count][2 buffers][2N]
    double2* hpsi;                // [count][2][2N]
    double2* aux;                 // [count][2][2N]
    double2* p;                   // [count][2N]
    double2* r_old;               // [count][2N]
    double2* rho;                 // [count][N]
    double2* W;                   // [count][3N]
    double2* zbuf;                // [count][2N] P_Delta^-1 of the make_r output (zmode 2..4)
    double* partials;             // [count][kMaxSums][nblk]
};

// Batched form of fft_trial_z_pass over the running instances of a group
// (args: a z-axis pass of the group's grid; grid.z = g.n_ids).
hipError_t fft_btrial_z_pass(int L, int variant, const FftPassArgs& args, const BGroup& g, hipStream_t s);

hipError_t launch_b_norm2(const BGroup& g, hipStream_t s);
hipError_t launch_b_heval_epi(const BGroup& g, hipStream_t s);
hipError_t launch_b_dir_reduce(const BGroup& g, hipStream_t s);
// act_pre[i] = 1 for the running instances that start a new direction with the configured z
hipError_t launch_b_mark_pre(int n_inst, const BInstState* st, int* act_pre, hipStream_t s);
// zbuf = the residual of the instances in act_pre, with the papply factor
hipError_t launch_b_make_r(const BGroup& g, hipStream_t s);
hipError_t launch_b_dir_write(const BGroup& g, hipStream_t s);
hipError_t launch_b_copy_out(const BGroup& g, hipStream_t s);
// for l = ids[y], y < n_ids: sums[first + l][off + m] = sum_b partials[l * inst_stride + m * row_stride + b]
hipError_t launch_b_reduce(const double* partials, long long inst_stride, long long row_stride, int nblk, int M,
                           const int* ids, int n_ids, double* sums_first, int off, hipStream_t s);
// decision kernels over all n_inst instances
hipError_t launch_b_decide_init(int n_inst, const BInstParams* ip, BInstState* st, const double* sums,
                                int* act_dir, int* act_trial, int* tsel, hipStream_t s);
hipError_t launch_b_decide_dir(int n_inst, BOpts o, const BInstParams* ip, BInstState* st, const double* sums,
                               int* act_dir, hipStream_t s);
hipError_t launch_b_decide_step(int n_inst, BOpts o, const BInstParams* ip, BInstState* st, const double* sums,
                                const int* act_dir, int* act_trial, int* tsel, hipStream_t s);
hipError_t launch_b_decide_accept(int n_inst, BOpts o, const BInstParams* ip, BInstState* st, const double* sums,
                                  int* act_trial, hipStream_t s);

}  // namespace bec
