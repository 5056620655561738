// Pointwise passes fused with a z transform, for gfx950 (arXiv:2510.24543).
//
// 1. The direction-write pass fused with the first forward transform of the
//    line search (Sec. IV.C, Sec. V), kernel in fft_dirwrite.h: P_V (zmode 1),
//    the benchmark's and the paper's recommended preconditioner, instantiated
//    here; the composite P_Delta^-1 P_V^-1 (zmode 2: z read from the k-space
//    passes' output) in fft_fused_composite.hip; the other modes keep the
//    two-kernel form.
//
// 2. The Hamiltonian epilogue fused with the last inverse transform of the
//    energy evaluation (Sec. II, Eq. (6)): with the kinetic term taken from
//    one-axis transforms, that z pass carries only the packed dipolar
//    potentials Phi_1 + i Phi_2; the workgroup inverts their z pencils in
//    registers, stores Phi and evaluates H psi, muLHY and the energy sums at
//    the same points, so Phi is written once and never read back.
//
// 3. The input of the k-space preconditioners fused with their first forward
//    z transform (Sec. IV.B).
#include "fft_dirwrite.h"

namespace bec {
namespace {

template <int L, int T, int R0, int R1, int R2, int NTHR>
__global__ __launch_bounds__(NTHR) void fft_heval_z_kernel(FftPassArgs Z, PwParams P, HevalArgs H)
{
    using PL = Plan<L, T, R0, R1, R2, true>;
    constexpr int E = L / T, PB = NTHR / T, RS = lds_row<L>(), RL = PL::RL, M = kHevalSums;
    constexpr int NW = NTHR / 64;
    static_assert(M * NW * sizeof(double) <= PB * RS * sizeof(double2), "reduction fits the LDS rows");
    __shared__ double2 lds[PB * RS];
    const long long N = P.N;
    const int tid = threadIdx.x;
    const int pl = tid / T, t = tid % T;
    const long long pg = (long long)blockIdx.x * PB + pl;
    const bool valid = pg < Z.npencil;
    const long long base = valid ? pg * (long long)L : 0;
    double2* row = lds + pl * RS;
    const double2* __restrict__ src = Z.src[0];
    double2 v[E];
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r)
            v[b * R0 + r] = valid ? src[base + t + b * T + r * (L / R0)] : make_double2(0.0, 0.0);
    PL::template fwd_like<+1>(v, row, t, Z.tw);     // inverse z transform (the 1/N is applied on x)
    // Phi of the pencil through its LDS row, then one point per trip (lanes on
    // consecutive points): a single copy of the epilogue, not E unrolled ones
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) row[lds_pad(t + b * T + r * (L / RL))] = v[b * RL + r];
    pencil_sync<true>();
    double acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0;
    if (valid) {
#pragma unroll 1
        for (int k = 0; k < E; ++k) {
            const int j = t + k * T;
            const long long i = base + j;
            const double2 s1 = H.psi[i], s2 = H.psi[N + i], t1 = H.Tpsi[i], t2 = H.Tpsi[N + i];
            heval_point(P, H, N, i, s1, s2, t1, t2, row[lds_pad(j)], true, acc);
        }
    }
    // fixed-order block reduction of the M energy sums into H.partials [m][block]
    double* sh = reinterpret_cast<double*>(lds);
    const int lane = tid & 63, w = tid >> 6;
    __syncthreads();
    wave_sum_down(acc);
    if (lane == 0)
#pragma unroll
        for (int m = 0; m < M; ++m) sh[m * NW + w] = acc[m];
    __syncthreads();
    if (tid < M) {
        double s = 0.0;
        for (int k = 0; k < NW; ++k) s += sh[tid * NW + k];
        H.partials[(long long)tid * gridDim.x + blockIdx.x] = s;
    }
}

// 3. The input of the k-space preconditioners fused with their first forward
//    transform (Sec. IV.B): the residual, times P_V^-1 for the composite
//    (apply_pv 1) or D^-1/2 for the symmetrised form (apply_pv 2), computed at
//    the points of whole z pencils and transformed along z in registers; the
//    field is written once, already z-transformed, for the y pass that follows.
template <int L, int T, int R0, int R1, int R2, int NTHR>
__global__ __launch_bounds__(NTHR) void fft_maker_z_kernel(FftPassArgs Z, PwParams P, MakeRArgs A)
{
    using PL = Plan<L, T, R0, R1, R2, true>;
    constexpr int E = L / T, PB = NTHR / T, RS = lds_row<L>(), RL = PL::RL;
    __shared__ double2 lds[PB * RS];
    if (A.dev_state) rule_mu_shift(A.dev_state, P.Gdd, A.mu, A.diag_shift);
    const long long N = P.N;
    const int tid = threadIdx.x;
    const int pl = tid / T, t = tid % T;
    const long long pg = (long long)blockIdx.x * PB + pl;
    const bool valid = pg < Z.npencil;
    const long long base = valid ? pg * (long long)L : 0;
    double2* row = lds + pl * RS;
    double2 v0[E], v1[E];
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = b * R0 + r;
            v0[k] = v1[k] = make_double2(0.0, 0.0);
            if (valid) make_r_point(P, A, N, base + t + b * T + r * (L / R0), v0[k], v1[k]);
        }
    PL::template fwd_like<-1>(v0, row, t, Z.tw);
    PL::template fwd_like<-1>(v1, row, t, Z.tw);
    if (valid) {
#pragma unroll
        for (int b = 0; b < E / RL; ++b)
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const long long i = base + t + b * T + r * (L / RL);
                A.out[i] = v0[b * RL + r];
                A.out[N + i] = v1[b * RL + r];
            }
    }
}

}  // namespace

hipError_t fft_maker_z_pass(int L, int variant, const FftPassArgs& Z, const PwParams& P, const MakeRArgs& A,
                            hipStream_t st)
{
    if (Z.S != 1 || !A.out || A.rin || A.apply_pv < 0 || A.apply_pv > 2) return hipErrorInvalidValue;
#define BEC_MCASE(LL, VV, T, R0, R1, R2, NT, W)                                                              \
    if (L == LL && variant == VV) {                                                                           \
        const dim3 grid((unsigned)((Z.npencil + NT / T - 1) / (NT / T)));                                     \
        hipLaunchKernelGGL((fft_maker_z_kernel<LL, T, R0, R1, R2, NT>), grid, dim3(NT), 0, st, Z, P, A);       \
        return hipGetLastError();                                                                             \
    }
    BEC_FFT_VARIANTS(BEC_MCASE)
#undef BEC_MCASE
    return hipErrorInvalidValue;
}

hipError_t fft_heval_z_pass(int L, int variant, const FftPassArgs& Z, const PwParams& P, const HevalArgs& H,
                            hipStream_t st)
{
    if (Z.S != 1 || !Z.src[0] || H.aux != Z.src[0]) return hipErrorInvalidValue;
#define BEC_HCASE(LL, VV, T, R0, R1, R2, NT, W)                                                              \
    if (L == LL && variant == VV) {                                                                           \
        const dim3 grid((unsigned)((Z.npencil + NT / T - 1) / (NT / T)));                                     \
        hipLaunchKernelGGL((fft_heval_z_kernel<LL, T, R0, R1, R2, NT>), grid, dim3(NT), 0, st, Z, P, H);       \
        return hipGetLastError();                                                                             \
    }
    BEC_FFT_VARIANTS(BEC_HCASE)
#undef BEC_HCASE
    return hipErrorInvalidValue;
}

hipError_t fft_dirwrite_z_pass(int L, int variant, const FftPassArgs& Z, const PwParams& P, const DirArgs& A,
                               hipStream_t st)
{
    if (A.zmode == 1) return dirwrite_z_launch<1>(L, variant, Z, P, A, st);
    if (A.zmode == 2) return fft_dirwrite_z_pass_composite(L, variant, Z, P, A, st);
    return hipErrorInvalidValue;
}

}  // namespace bec
