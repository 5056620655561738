// The direction-write pass fused with the first forward transform of the line
// search, for gfx950 (arXiv:2510.24543, Sec. IV.C, Sec. V).  Included by the
// translation units that instantiate it for P_V (fft_fused.hip) and for the
// composite preconditioner (fft_fused_composite.hip).
//
// A workgroup owns whole z pencils.  Each thread computes, at the points of its
// pencil slots, what the grid-stride direction write computes there (the
// direction p = d - Re<d,psi> psi with d = -z + beta p_old, the residual r,
// rho_i = Re(conj(psi_i) p_i) and the model sums), stores p, r and rho as that
// pass does, and keeps p_1, p_2 and the packed rho_1 + i rho_2 in registers.
// It then transforms them along z: the one-axis Parseval sums of p_i
// (<p_i, T_z p_i> by |k_z|^2/2 |p^_i|^2, no store) and the forward z transform
// of the packed density, unpacked into the half spectra of rho_1 and rho_2,
// which the line search's y and x passes continue (the x pass takes the model's
// density sums in k-space, so no inverse transform follows).  The separate z
// pass of the line search -- a second read of p and rho -- is gone.
#pragma once

#include "pw_point.h"
#include "fft_core.h"

namespace bec {
namespace {

using namespace fftcore;
using namespace pwpt;

// With P_V, plans with at most 8 points per thread load the operands of the
// next point before the current one is computed (register budget of two waves
// per SIMD), so that a wave keeps loads in flight through the per-point
// arithmetic; larger plans, and the composite (whose z operand would push the
// kernel into spills), keep one point's operands at a time.
template <int L, int T, int ZM>
constexpr bool dirwrite_prefetch() { return L / T <= 8 && ZM == 1; }

template <int L, int T, int R0, int R1, int R2, int NTHR, int ZM, bool LHY>
__global__ __launch_bounds__(NTHR, (dirwrite_prefetch<L, T, ZM>() ? 2 : 1)) void fft_dirwrite_z_kernel(FftPassArgs Z,
                                                                                                PwParams P, DirArgs A)
{
    using PL = Plan<L, T, R0, R1, R2, true>;
    constexpr int E = L / T, PB = NTHR / T, RS = lds_row<L>(), RL = PL::RL, M = kDirWriteSums;
    constexpr int NW = NTHR / 64;
    static_assert((M + 2) * NW * sizeof(double) <= PB * RS * sizeof(double2), "reduction fits the LDS rows");
    __shared__ double2 lds[PB * RS];
    if (A.dev_state) rule_mu_shift(A.dev_state, P.Gdd, A.mu, A.diag_shift);
    if (A.dev_dir) {
        A.beta = rule_beta(A.dev_dir, A.rule);
        rule_proj(A.dev_dir, A.beta, A.rule.dV, A.c);
    }
    const bool with_p = A.beta != 0.0;
    const long long N = P.N;
    const int tid = threadIdx.x;
    const int pl = tid / T, t = tid % T;
    const long long pg = (long long)blockIdx.x * PB + pl;
    const bool valid = pg < Z.npencil;
    const long long base = valid ? pg * (long long)L : 0;
    double2* row = lds + pl * RS;

    double acc[M + 2];
#pragma unroll
    for (int m = 0; m < M + 2; ++m) acc[m] = 0.0;
    double2 v0[E], v1[E], v2[E];
    constexpr bool PF = dirwrite_prefetch<L, T, ZM>();
    auto pt_index = [&](int k) { return base + t + (k / R0) * T + (k % R0) * (L / R0); };
    DirIn<ZM> nxt{};
    if (PF && valid) nxt = dir_load<ZM>(P, A, N, pt_index(0), with_p);
#pragma unroll
    for (int k = 0; k < E; ++k) {
        v0[k] = v1[k] = v2[k] = make_double2(0.0, 0.0);
        DirIn<ZM> cur = nxt;
        if (PF && valid && k + 1 < E) nxt = dir_load<ZM>(P, A, N, pt_index(k + 1), with_p);
        if (!PF && valid) cur = dir_load<ZM>(P, A, N, pt_index(k), with_p);
        if (valid) {
            double2 pp[2];
            double rr[2];
            dir_point<ZM, LHY>(P, A, N, pt_index(k), cur, acc, pp, rr);
            v0[k] = pp[0];
            v1[k] = pp[1];
            v2[k] = make_double2(rr[0], rr[1]);
        }
    }

    // one-axis Parseval sums of p_1, p_2 along z, then the packed density's transform
    const double dk = Z.kaxis[1];
    double2* vs[2] = {v0, v1};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        PL::template fwd_like<-1>(vs[c], row, t, Z.tw);
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < E / RL; ++b)
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const double k = kwave<L>(dk, t + b * T + r * (L / RL));
                const double2 w = vs[c][b * RL + r];
                s += 0.5 * (k * k) * (w.x * w.x + w.y * w.y);
            }
        acc[M + c] = valid ? s : 0.0;
    }
    PL::template fwd_like<-1>(v2, row, t, Z.tw);
    // rho_1 and rho_2 are real: with F the transform of rho_1 + i rho_2,
    // rho^_1(k) = (F(k) + conj F(-k)) / 2 and rho^_2(k) = (F(k) - conj F(-k)) / (2i),
    // stored for k = 0..L/2 only (the rest is their conjugate mirror), interleaved
    // per k; F(-k) comes from the pencil's LDS row
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) row[lds_pad(t + b * T + r * (L / RL))] = v2[b * RL + r];
    pencil_sync<true>();
    if (valid) {
        double2* d = Z.dst[2] + pg * (long long)(L + 2);
        for (int k = t; k <= L / 2; k += T) {
            const double2 fk = row[lds_pad(k)], fm = row[lds_pad(k == 0 ? 0 : L - k)];
            d[2 * k] = make_double2(0.5 * (fk.x + fm.x), 0.5 * (fk.y - fm.y));
            d[2 * k + 1] = make_double2(0.5 * (fk.y + fm.y), -0.5 * (fk.x - fm.x));
        }
    }

    // fixed-order block reduction: the M direction sums into A.partials
    // [m][block], the two Parseval sums into Z.partials [field][block]
    double* sh = reinterpret_cast<double*>(lds);
    const int lane = tid & 63, w = tid >> 6;
    __syncthreads();
    wave_sum_down(acc);
    if (lane == 0)
#pragma unroll
        for (int m = 0; m < M + 2; ++m) sh[m * NW + w] = acc[m];
    __syncthreads();
    if (tid < M + 2) {
        double s = 0.0;
        for (int k = 0; k < NW; ++k) s += sh[tid * NW + k];
        if (tid < M) A.partials[(long long)tid * gridDim.x + blockIdx.x] = s;
        else Z.partials[(long long)(tid - M) * Z.nblk_x + blockIdx.x] = s * Z.pscale;
    }
}

// Launch of the direction write for preconditioner mode ZM (1 P_V, 2 the
// composite) with plan `variant` of the z length L; see fft_dirwrite_z_pass.
template <int ZM>
hipError_t dirwrite_z_launch(int L, int variant, const FftPassArgs& Z, const PwParams& P, const DirArgs& A,
                             hipStream_t st)
{
    if (Z.S != 1 || A.zmode != ZM || !Z.partials || !Z.kaxis) return hipErrorInvalidValue;
#define BEC_DCASE(LL, VV, T, R0, R1, R2, NT, W)                                                              \
    if (L == LL && variant == VV) {                                                                           \
        const dim3 grid((unsigned)((Z.npencil + NT / T - 1) / (NT / T)));                                     \
        if (P.lhy_on)                                                                                         \
            hipLaunchKernelGGL((fft_dirwrite_z_kernel<LL, T, R0, R1, R2, NT, ZM, true>), grid, dim3(NT), 0, st, Z, P, A); \
        else                                                                                                  \
            hipLaunchKernelGGL((fft_dirwrite_z_kernel<LL, T, R0, R1, R2, NT, ZM, false>), grid, dim3(NT), 0, st, Z, P, A); \
        return hipGetLastError();                                                                             \
    }
    BEC_FFT_VARIANTS(BEC_DCASE)
#undef BEC_DCASE
    return hipErrorInvalidValue;
}

}  // namespace
}  // namespace bec
