// Scalar rules of one PCG iteration (arXiv:2510.24543, Sec. III Eqs. (8)-(9),
// Sec. IV.C, Sec. V) that both the host loop and the kernels evaluate: the
// chemical potentials and P_V shifts from the energy sums, the conjugacy
// parameter beta and the projection coefficients of the new direction.  The
// kernels of a pipelined iteration read the reduced sums from device memory and
// apply these rules themselves, before the host has seen the sums; the host
// applies the same rules to its copy afterwards.  Floating-point contraction
// is off inside every rule, so both sides produce the same bits.
#pragma once

#include <hip/hip_runtime.h>

namespace bec {

// Energy sums S (kHevalSums, see HevalArgs) -> mu_i = <psi_i, H_i psi_i>/|psi_i|^2
// (Sec. III) and the P_V shift alpha_i = (<psi_i, H_i psi_i> - sum_j Gdd_ij
// <n_i, Phi_j>)/|psi_i|^2 (Sec. IV.B).
__host__ __device__ inline void rule_mu_shift(const double* S, const double Gdd[2][2], double mu[2], double shift[2])
{
#pragma clang fp contract(off)
    for (int i = 0; i < 2; ++i) {
        double gdd_phi = 0.0;
        for (int j = 0; j < 2; ++j) gdd_phi += Gdd[i][j] * S[7 + 2 * i + j];
        mu[i] = S[12 + i] / S[14 + i];
        shift[i] = (S[12 + i] - gdd_phi) / S[14 + i];
    }
}

// Weight of P_V in the blended preconditioner z = w P_V^-1 r + (1 - w) P_Delta^-1 r
// for both components: `blend` when it is >= 0, else the potential share of the
// shift, [shift_i - K_i]_+ / ([shift_i - K_i]_+ + K_i) with the kinetic part
// K_i = <psi_i, T psi_i> / |psi_i|^2 from the energy sums S (1/2 if both vanish).
__host__ __device__ inline void rule_blend(const double* S, const double shift[2], double blend, double w[2])
{
#pragma clang fp contract(off)
    for (int i = 0; i < 2; ++i) {
        if (blend >= 0.0) {
            w[i] = blend;
            continue;
        }
        const double K = S[i] / S[14 + i];
        double pot = shift[i] - K;
        if (pot < 0.0) pot = 0.0;
        w[i] = (pot + K > 0.0) ? pot / (pot + K) : 0.5;
    }
}

// Inputs of the conjugacy rule that the host knows before the reduce sums.
struct BetaRule {
    int restart;       // beta = 0 (first step, beta rule 0, or the restart period)
    int mode;          // 0 Hestenes-Stiefel+, 1 Polak-Ribiere+
    double rz_old;     // sum_i w_i dV Re<r_i, z_i> of the previous step (Polak-Ribiere+ denominator)
    double w[2];       // (N_i / (N_1 + N_2))^2
    double dV;
};

// Direction-reduce sums R (kDirReduceSums) -> beta >= 0 (Sec. IV.C, HS+ / PR+).
__host__ __device__ inline double rule_beta(const double* R, const BetaRule& b)
{
#pragma clang fp contract(off)
    if (b.restart) return 0.0;
    double num = 0.0, den = 0.0;
    for (int i = 0; i < 2; ++i) {
        num += b.w[i] * b.dV * R[6 * i + 1];
        den += b.w[i] * b.dV * R[6 * i + 2];
    }
    if (b.mode == 1) den = b.rz_old;
    double beta = (den > 0.0 && __builtin_isfinite(den) && __builtin_isfinite(num)) ? num / den : 0.0;
    return beta < 0.0 ? 0.0 : beta;
}

// Projection coefficients c_i = Re<d_i, psi_i> dV of d = -z + beta p_old (Sec. V).
__host__ __device__ inline void rule_proj(const double* R, double beta, double dV, double c[2])
{
#pragma clang fp contract(off)
    for (int i = 0; i < 2; ++i) c[i] = -dV * R[6 * i + 3] + beta * dV * R[6 * i + 4];
}

}  // namespace bec
