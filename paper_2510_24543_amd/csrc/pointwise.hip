// Fused pointwise + reduction kernels for gfx950 (FP64 vector ALU, no MFMA:
// nothing here is a dense contraction).
//
// Every kernel streams its operands once with 16-byte loads, does all per-point
// algebra in registers, and reduces its scalars per thread, per wavefront
// (lane shuffles) and per workgroup into a fixed slot of a partials array.  A
// one-workgroup kernel then sums the partials in a fixed order, so every
// reduced scalar is bitwise reproducible for a given grid size.
//
// Physics (arXiv:2510.24543):
//   H_i psi_i = T psi_i + [V + sum_j (G_ij n_j + Gdd_ij Phi_j) + muLHY_i] psi_i   (Sec. II, Eq. (6))
//   e_LHY = c sqrt(2)/(15 pi^2) int du sum_+- [V_+-]_+^(5/2)                      (Eq. (1), (3))
//   muLHY_i = (1/N_i) de/dn_i                                                       (Eq. (5))
//   residual r_i = H_i psi_i - mu_i psi_i                                           (Sec. III, Eq. (8))
//   P_V diagonal [alpha_i + V + sum_j G_ij n_j + muLHY_i]_+ + sigma                  (Sec. IV.B)
//   d = -z + beta p_old, p = d - Re<d,psi> psi                                      (Sec. IV.C, Sec. V)
//   second-order energy model along the geodesic                                    (Sec. V)
#include "pw_point.h"

namespace bec {
namespace {

using namespace pwpt;

// Fixed-order workgroup reduction of M per-thread sums into partials[m * nblk + block].
template <int M>
__device__ __forceinline__ void block_reduce_store(const double (&acc)[M], double* partials, int nblk)
{
    __shared__ double sh[M][kPwThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = acc[m];
    wave_sum_down(v);
    if (lane == 0)
#pragma unroll
        for (int m = 0; m < M; ++m) sh[m][w] = v[m];
    __syncthreads();
    if (threadIdx.x < M) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kPwThreads / 64; ++k) s += sh[threadIdx.x][k];
        partials[(long long)threadIdx.x * nblk + blockIdx.x] = s;
    }
}

#define GRID_STRIDE(i, N)                                                                      \
    for (long long i = (long long)blockIdx.x * kPwThreads + threadIdx.x; i < (N);             \
         i += (long long)gridDim.x * kPwThreads)

struct HevalIn {
    double2 s1, s2, t1, t2, ph;
};

__device__ __forceinline__ HevalIn heval_load(const HevalArgs& A, long long N, long long i)
{
    HevalIn v;
    v.s1 = A.psi[i];
    v.s2 = A.psi[N + i];
    v.t1 = A.Tpsi[i];
    v.t2 = A.Tpsi[N + i];
    v.ph = A.phi[i];
    return v;
}

__global__ __launch_bounds__(kPwThreads) void heval_epi_kernel(PwParams P, HevalArgs A)
{
    const long long N = P.N;
    const long long stride = (long long)gridDim.x * kPwThreads;
    double acc[kHevalSums];
#pragma unroll
    for (int m = 0; m < kHevalSums; ++m) acc[m] = 0.0;
    const bool store_phi = A.phi != A.aux;      // uniform: Phi already in place otherwise
    for (long long i = (long long)blockIdx.x * kPwThreads + threadIdx.x; i < N; i += stride) {
        const HevalIn cur = heval_load(A, N, i);
        heval_point(P, A, N, i, cur.s1, cur.s2, cur.t1, cur.t2, cur.ph, store_phi, acc);
    }
    block_reduce_store<kHevalSums>(acc, A.partials, gridDim.x);
}

// One imaginary-time step at point i (the potential factor of the splitting)
// with the energy sums of the current iterate.
__global__ __launch_bounds__(kPwThreads) void ite_epi_kernel(PwParams P, IteArgs A)
{
    const long long N = P.N;
    double acc[kIteSums];
#pragma unroll
    for (int m = 0; m < kIteSums; ++m) acc[m] = 0.0;
    for (long long i = (long long)blockIdx.x * kPwThreads + threadIdx.x; i < N;
         i += (long long)gridDim.x * kPwThreads) {
        const double2 s1 = A.psi[i], s2 = A.psi[N + i];
        const double2 h1 = A.hat[i], h2 = A.hat[N + i];
        const double2 ph = A.phi[i];
        const double n1 = sq2(s1), n2 = sq2(s2);
        const double V = trap_at(P, i);
        double e = 0.0, d1 = 0.0, d2 = 0.0;
        if (P.lhy_on) lhy_point(KernargNodes{P}, LhyTab{P.lhy_tab, P.lhy_K}, P.n_a, P.n_b, P.K5, P.K3, n1, n2, e, d1, d2);
        const double U1 = V + P.G[0][0] * n1 + P.G[0][1] * n2 + P.Gdd[0][0] * ph.x + P.Gdd[0][1] * ph.y + d1 / P.Nat[0];
        const double U2 = V + P.G[1][0] * n1 + P.G[1][1] * n2 + P.Gdd[1][0] * ph.x + P.Gdd[1][1] * ph.y + d2 / P.Nat[1];
        const double f1 = exp(-A.dt * U1), f2 = exp(-A.dt * U2);
        const double2 o1 = make_double2(f1 * h1.x, f1 * h1.y), o2 = make_double2(f2 * h2.x, f2 * h2.y);
        A.out[i] = o1;
        A.out[N + i] = o2;
        acc[0] += V * n1;
        acc[1] += V * n2;
        acc[2] += n1 * n1;
        acc[3] += n1 * n2;
        acc[4] += n2 * n2;
        acc[5] += n1 * ph.x;
        acc[6] += n1 * ph.y;
        acc[7] += n2 * ph.x;
        acc[8] += n2 * ph.y;
        acc[9] += e;
        acc[10] += n1;
        acc[11] += n2;
        acc[12] += sq2(o1);
        acc[13] += sq2(o2);
    }
    block_reduce_store<kIteSums>(acc, A.partials, gridDim.x);
}

// residual and preconditioned residual at point i for both components
struct RZ {
    double2 r[2], z[2];
};

#ifndef BEC_DIR_WRITE_UNROLL
#define BEC_DIR_WRITE_UNROLL 1
#endif
constexpr int kDirWriteUnroll = BEC_DIR_WRITE_UNROLL;   // points per thread and trip of the direction-write pass

// Operands of the direction-reduce pass at one point.  ZM is the
// preconditioner mode (DirArgs::zmode), PREV whether the previous residual and
// direction enter (DirArgs::have_prev).
template <int ZM, bool PREV>
struct RedIn {
    double2 s[2], h[2], ml, zb[2], ro[2], po[2];
};

template <int ZM, bool PREV>
__device__ __forceinline__ RedIn<ZM, PREV> red_load(const DirArgs& A, long long N, long long i)
{
    RedIn<ZM, PREV> v;
    v.s[0] = A.psi[i];
    v.s[1] = A.psi[N + i];
    v.h[0] = A.hpsi[i];
    v.h[1] = A.hpsi[N + i];
    if constexpr (ZM == 1 || ZM == 3 || ZM == 4) v.ml = A.aux[N + i];
    if constexpr (ZM >= 2 && ZM <= 4) {
        v.zb[0] = A.zbuf[i];
        v.zb[1] = A.zbuf[N + i];
    }
    if constexpr (PREV) {
        v.ro[0] = A.r_old[i];
        v.ro[1] = A.r_old[N + i];
        v.po[0] = A.p[i];
        v.po[1] = A.p[N + i];
    }
    return v;
}

// residual r = H psi - mu psi and z = P^-1 r at one point (zmode ZM)
template <int ZM, bool PREV>
__device__ __forceinline__ RZ red_rz(const PwParams& P, const DirArgs& A, long long i, const RedIn<ZM, PREV>& v)
{
    RZ o;
#pragma unroll
    for (int c = 0; c < 2; ++c)
        o.r[c] = make_double2(v.h[c].x - A.mu[c] * v.s[c].x, v.h[c].y - A.mu[c] * v.s[c].y);
    if constexpr (ZM == 0) {
        o.z[0] = o.r[0];
        o.z[1] = o.r[1];
    } else if constexpr (ZM == 2) {
        o.z[0] = v.zb[0];
        o.z[1] = v.zb[1];
    } else {
        const double n1 = sq2(v.s[0]), n2 = sq2(v.s[1]);
        const double V = trap_at(P, i);
        const double mlc[2] = {v.ml.x, v.ml.y};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const double g = pv_inv(P, c, A.diag_shift[c], A.sigma, V, n1, n2, mlc[c]);
            if constexpr (ZM == 1) {
                o.z[c] = make_double2(g * o.r[c].x, g * o.r[c].y);
            } else if constexpr (ZM == 3) {
                const double q = sqrt(g);
                o.z[c] = make_double2(q * v.zb[c].x, q * v.zb[c].y);
            } else {
                const double a = A.blend_w[c] * g, b = 1.0 - A.blend_w[c];
                o.z[c] = make_double2(a * o.r[c].x + b * v.zb[c].x, a * o.r[c].y + b * v.zb[c].y);
            }
        }
    }
    return o;
}

// Direction-reduce pass: the sums of kDirReduceSums.  Two points per thread and
// trip, their operands loaded before either is used; each thread adds its points
// in grid-stride order.
template <int ZM, bool PREV>
__global__ __launch_bounds__(kPwThreads) void dir_reduce_kernel(PwParams P, DirArgs A)
{
    if (A.dev_state) {
        rule_mu_shift(A.dev_state, P.Gdd, A.mu, A.diag_shift);
        if (ZM == 4) rule_blend(A.dev_state, A.diag_shift, A.blend, A.blend_w);
    }
    const long long N = P.N;
    const long long stride = (long long)gridDim.x * kPwThreads;
    double acc[kDirReduceSums];
#pragma unroll
    for (int m = 0; m < kDirReduceSums; ++m) acc[m] = 0.0;
    for (long long i = (long long)blockIdx.x * kPwThreads + threadIdx.x; i < N; i += 2 * stride) {
        const long long i2 = i + stride < N ? i + stride : i;
        const RedIn<ZM, PREV> in[2] = {red_load<ZM, PREV>(A, N, i), red_load<ZM, PREV>(A, N, i2)};
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (u == 1 && i2 == i) break;
            const long long k = u ? i2 : i;
            const RZ q = red_rz<ZM, PREV>(P, A, k, in[u]);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double2 s = in[u].s[c];
                acc[6 * c + 0] += sq2(q.r[c]);
                acc[6 * c + 3] += redot(q.z[c], s);
                acc[6 * c + 5] += redot(q.r[c], q.z[c]);
                if constexpr (PREV) {
                    const double2 ro = in[u].ro[c], po = in[u].po[c];
                    const double2 y = make_double2(q.r[c].x - ro.x, q.r[c].y - ro.y);
                    acc[6 * c + 1] += redot(y, q.z[c]);
                    acc[6 * c + 2] += redot(y, po);
                    acc[6 * c + 4] += redot(po, s);
                }
            }
        }
    }
    block_reduce_store<kDirReduceSums>(acc, A.partials, gridDim.x);
}

// Direction write pass with the LHY part of the line-search model.  UNR points
// per thread and trip, their operands loaded before the first is used; each
// thread handles its points in grid-stride order.
template <int ZM, bool LHY, int UNR>
__global__ __launch_bounds__(kPwThreads) void dir_write_kernel(PwParams P, DirArgs A)
{
    if (A.dev_state) {
        rule_mu_shift(A.dev_state, P.Gdd, A.mu, A.diag_shift);
        if (ZM == 4) rule_blend(A.dev_state, A.diag_shift, A.blend, A.blend_w);
    }
    if (A.dev_dir) {
        A.beta = rule_beta(A.dev_dir, A.rule);
        rule_proj(A.dev_dir, A.beta, A.rule.dV, A.c);
    }
    const bool with_p = A.beta != 0.0;
    const long long N = P.N;
    const long long stride = (long long)gridDim.x * kPwThreads;
    double acc[kDirWriteSums];
#pragma unroll
    for (int m = 0; m < kDirWriteSums; ++m) acc[m] = 0.0;
    for (long long i = (long long)blockIdx.x * kPwThreads + threadIdx.x; i < N; i += UNR * stride) {
        long long k[UNR];
        DirIn<ZM> cur[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            k[u] = i + u * stride < N ? i + u * stride : i;
            cur[u] = dir_load<ZM>(P, A, N, k[u], with_p);
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            if (u > 0 && k[u] == i) break;
            dir_point<ZM, LHY>(P, A, N, k[u], cur[u], acc);
        }
    }
    block_reduce_store<kDirWriteSums>(acc, A.partials, gridDim.x);
}

__global__ __launch_bounds__(kPwThreads) void make_r_kernel(PwParams P, MakeRArgs A)
{
    if (A.dev_state) rule_mu_shift(A.dev_state, P.Gdd, A.mu, A.diag_shift);
    const long long N = P.N;
    GRID_STRIDE(i, N)
    {
        double2 r1, r2;
        make_r_point(P, A, N, i, r1, r2);
        A.out[i] = r1;
        A.out[N + i] = r2;
    }
}

__global__ __launch_bounds__(kPwThreads) void param_grad_kernel(PwParams P, ParamGradArgs A)
{
    const long long N = P.N;
    double acc[kParamSums];
#pragma unroll
    for (int m = 0; m < kParamSums; ++m) acc[m] = 0.0;
    GRID_STRIDE(i, N)
    {
        const double n1 = sq2(A.psi[i]), n2 = sq2(A.psi[N + i]);
        for (int q = 0; q < P.n_u; ++q) {
            const double* nd = P.nodes + q * kNodeStride;
            const double e11 = nd[0], e22 = nd[1], p12 = nd[2], w = nd[3];
            const double e12 = nd[4], e21 = nd[5], au = nd[6];
            const double delta = e11 * n1 - e22 * n2;
            const double s = sqrt(delta * delta + 4.0 * p12 * n1 * n2);
            const double inv = s > 0.0 ? 1.0 / s : 0.0;
            const double base = e11 * n1 + e22 * n2;
            // dV_+-/d eta_11, eta_12, eta_21, eta_22 = (n1, 0, 0, n2) +- g
            const double g0 = delta * n1 * inv, g1 = 2.0 * e21 * n1 * n2 * inv;
            const double g2 = 2.0 * e12 * n1 * n2 * inv, g3 = -delta * n2 * inv;
#pragma unroll
            for (int br = 0; br < 2; ++br) {
                const double sg = br == 0 ? 1.0 : -1.0;
                const double V = base + sg * s;
                if (V <= 0.0) continue;
                const double v32 = V * sqrt(V);
                const double f = 2.5 * w * v32;
                const double dv[4] = {n1 + sg * g0, sg * g1, sg * g2, n2 + sg * g3};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    acc[c] += f * dv[c];
                    acc[4 + c] += f * dv[c] * au;
                }
                acc[8] += w * V * v32;
            }
        }
    }
    block_reduce_store<kParamSums>(acc, A.partials, gridDim.x);
}

__global__ __launch_bounds__(kPwThreads) void norm2_kernel(PwParams P, const double2* f, double* partials)
{
    const long long N = P.N;
    double acc[2] = {0.0, 0.0};
    GRID_STRIDE(i, N)
    {
        acc[0] += sq2(f[i]);
        acc[1] += sq2(f[N + i]);
    }
    block_reduce_store<2>(acc, partials, gridDim.x);
}

__global__ __launch_bounds__(kPwThreads) void scale2_kernel(PwParams P, const double2* in, double2* out,
                                                            double s0, double s1)
{
    const long long N = P.N;
    GRID_STRIDE(i, N)
    {
        const double2 a = in[i], b = in[N + i];
        out[i] = make_double2(s0 * a.x, s0 * a.y);
        out[N + i] = make_double2(s1 * b.x, s1 * b.y);
    }
}

__global__ __launch_bounds__(kPwThreads) void grad_kernel(PwParams P, const double2* psi, const double2* hpsi,
                                                          double2* out, double mu0, double mu1, double s0,
                                                          double s1, int projected)
{
    const long long N = P.N;
    GRID_STRIDE(i, N)
    {
        const double2 a = psi[i], b = psi[N + i], ha = hpsi[i], hb = hpsi[N + i];
        const double m0 = projected ? mu0 : 0.0, m1 = projected ? mu1 : 0.0;
        out[i] = make_double2(s0 * (ha.x - m0 * a.x), s0 * (ha.y - m0 * a.y));
        out[N + i] = make_double2(s1 * (hb.x - m1 * b.x), s1 * (hb.y - m1 * b.y));
    }
}

// E of Sec. II, Eq. (1) from the reduced energy sums S (kHevalSums), with the
// products and the order of the host's reading of the same sums, so both give
// the same bits.  One thread.
__global__ void energy_from_sums_kernel(PwParams P, const double* __restrict__ S, double dV, double* __restrict__ out)
{
#pragma clang fp contract(off)
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double snn[2][2] = {{S[4], S[5]}, {S[5], S[6]}};
    double E = dV * S[11];
    for (int i = 0; i < 2; ++i) {
        const double e_kin = P.Nat[i] * dV * S[i], e_trap = P.Nat[i] * dV * S[2 + i];
        E += e_kin + e_trap;
        for (int j = 0; j < 2; ++j) {
            const double e_c = 0.5 * P.Nat[i] * P.G[i][j] * dV * snn[i][j];
            const double e_dd = 0.5 * P.Nat[i] * P.Gdd[i][j] * dV * S[7 + 2 * i + j];
            E += e_c + e_dd;
        }
    }
    out[0] = E;
}

// One block per scalar: blocks [0, M1) reduce rows of s1.partials (s1.nblk per
// row) into s1.out, the next M2 blocks rows of s2 into s2.out, the rest rows of
// s3 into s3.out (and each into its copy when that is set).
__global__ __launch_bounds__(256) void reduce_final_kernel(RedSeg s1, RedSeg s2, RedSeg s3)
{
    __shared__ double sh[4];
    int m = (int)blockIdx.x;
    RedSeg g = s1;
    if (m >= s1.M) {
        m -= s1.M;
        g = s2;
        if (m >= s2.M) {
            m -= s2.M;
            g = s3;
        }
    }
    const double* partials = g.partials;
    const int nblk = g.nblk;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += partials[(long long)m * nblk + b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double v = ((sh[0] + sh[1]) + sh[2]) + sh[3];
        g.out[m] = v;
        if (g.copy) g.copy[m] = v;
    }
}

// Closed-form step of the second-order model along the geodesic (Sec. V), one
// thread, from the reduced model sums: E'(0) and E''(0), alpha* = -E'/E'' when
// the model has a minimum (else the previous step, else 0.1 / max|p_i|), capped
// at theta_max, and the trial coefficients psi_i(alpha) = (cos th_i psi_i +
// sin th_i p_i/|p_i|) / norm with th_i = alpha |p_i|.
__global__ void ls_step_kernel(PwParams P, StepArgs A)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double dV = A.dV;
    const double* D = A.D;
    const double* pars = A.pars;
    const double* LS = A.LS;
    double o[kStepOut];
    double rp = 0.0, E1 = 0.0, E2 = 0.0, pnorm[2], psip[2];
    for (int i = 0; i < 2; ++i) {
        pnorm[i] = sqrt(dV * D[i]);
        psip[i] = dV * D[16 + i];
        rp += 2.0 * P.Nat[i] * dV * D[2 + i];
        E1 += 2.0 * P.Nat[i] * dV * D[4 + i];                                  // E'_i
        const double pTp = dV * pars[i] * A.inv_n;                             // <p_i, T p_i> (Parseval)
        const double pn2 = pnorm[i] * pnorm[i];
        E2 += 2.0 * P.Nat[i] * (pTp + dV * D[8 + i] - pn2 * dV * D[6 + i]);    // one-body part of E''_ii
        for (int j = 0; j < 2; ++j) {
            const double rr = (i == 0 && j == 0) ? LS[0] : (i == 1 && j == 1) ? LS[2] : LS[1];
            E2 += 4.0 * P.Nat[i] * dV * (P.G[i][j] * rr + P.Gdd[i][j] * LS[3 + 2 * i + j]);
        }
        if (P.lhy_on) E2 += 2.0 * P.Nat[i] * dV * (D[10 + i] - pn2 * D[12 + i]);   // n'' part of E''_LHY
    }
    if (P.lhy_on) {
        E1 += P.K3 * dV * D[14];
        E2 += 2.0 * P.K3 * dV * D[15];
    }
    const double pmax = fmax(pnorm[0], pnorm[1]);
    double alpha;
    if (E2 > 0.0 && isfinite(E2) && isfinite(E1) && -E1 / E2 > 0.0) alpha = -E1 / E2;
    else alpha = A.alpha_prev > 0.0 ? A.alpha_prev : 0.1 / pmax;
    if (alpha * pmax > A.theta_max) alpha = A.theta_max / pmax;
    for (int i = 0; i < 2; ++i) {
        if (pnorm[i] > 0.0) {
            double sn, cs;
            sincos(alpha * pnorm[i], &sn, &cs);
            const double sb = sn / pnorm[i];
            const double nrm2 = cs * cs * A.norm2[i] + sb * sb * pnorm[i] * pnorm[i] + 2.0 * cs * sb * psip[i];
            const double s = 1.0 / sqrt(nrm2);
            o[i] = cs * s;
            o[2 + i] = sb * s;
        } else {
            o[i] = 1.0 / sqrt(A.norm2[i]);
            o[2 + i] = 0.0;
        }
    }
    o[4] = alpha;
    o[5] = rp;
    o[6] = E1;
    o[7] = E2;
    o[8] = pnorm[0];
    o[9] = pnorm[1];
    o[10] = psip[0];
    o[11] = psip[1];
    for (int m = 0; m < kStepOut; ++m) {
        A.out[m] = o[m];
        A.out_host[m] = o[m];
    }
}

int pw_blocks(const PwParams& P) { return P.nblk_pw; }

}  // namespace

hipError_t launch_ite_epi(const PwParams& P, const IteArgs& a, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(ite_epi_kernel, dim3(nblk), dim3(kPwThreads), 0, s, P, a);
    return hipGetLastError();
}

hipError_t launch_heval_epi(const PwParams& P, const HevalArgs& a, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(heval_epi_kernel, dim3(nblk), dim3(kPwThreads), 0, s, P, a);
    return hipGetLastError();
}

hipError_t launch_dir_reduce(const PwParams& P, const DirArgs& a, int nblk, hipStream_t s)
{
#define BEC_RED(ZM)                                                                              \
    case ZM:                                                                                     \
        if (a.have_prev) hipLaunchKernelGGL((dir_reduce_kernel<ZM, true>), dim3(nblk), dim3(kPwThreads), 0, s, P, a); \
        else hipLaunchKernelGGL((dir_reduce_kernel<ZM, false>), dim3(nblk), dim3(kPwThreads), 0, s, P, a);    \
        break;
    switch (a.zmode) {
        BEC_RED(0) BEC_RED(1) BEC_RED(2) BEC_RED(3) BEC_RED(4)
        default: return hipErrorInvalidValue;
    }
#undef BEC_RED
    return hipGetLastError();
}

hipError_t launch_dir_write(const PwParams& P, const DirArgs& a, int nblk, hipStream_t s)
{
#define BEC_DW(ZM)                                                                                          \
    case ZM:                                                                                                \
        if (P.lhy_on) hipLaunchKernelGGL((dir_write_kernel<ZM, true, kDirWriteUnroll>), dim3(nblk), dim3(kPwThreads), 0, s, P, a); \
        else hipLaunchKernelGGL((dir_write_kernel<ZM, false, kDirWriteUnroll>), dim3(nblk), dim3(kPwThreads), 0, s, P, a);       \
        break;
    switch (a.zmode) {
        BEC_DW(0) BEC_DW(1) BEC_DW(2) BEC_DW(3) BEC_DW(4)
        default: return hipErrorInvalidValue;
    }
#undef BEC_DW
    return hipGetLastError();
}

hipError_t launch_make_r(const PwParams& P, const MakeRArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(make_r_kernel, dim3(pw_blocks(P)), dim3(kPwThreads), 0, s, P, a);
    return hipGetLastError();
}

hipError_t launch_param_grad(const PwParams& P, const ParamGradArgs& a, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(param_grad_kernel, dim3(nblk), dim3(kPwThreads), 0, s, P, a);
    return hipGetLastError();
}

hipError_t launch_norm2(const PwParams& P, const double2* f, double* partials, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(norm2_kernel, dim3(nblk), dim3(kPwThreads), 0, s, P, f, partials);
    return hipGetLastError();
}

hipError_t launch_scale2(const PwParams& P, const double2* in, double2* out, double s0, double s1,
                         hipStream_t s)
{
    hipLaunchKernelGGL(scale2_kernel, dim3(pw_blocks(P)), dim3(kPwThreads), 0, s, P, in, out, s0, s1);
    return hipGetLastError();
}

hipError_t launch_grad(const PwParams& P, const double2* psi, const double2* hpsi, double2* out,
                       double mu0, double mu1, double s0, double s1, int projected, hipStream_t s)
{
    hipLaunchKernelGGL(grad_kernel, dim3(pw_blocks(P)), dim3(kPwThreads), 0, s, P, psi, hpsi, out, mu0,
                       mu1, s0, s1, projected);
    return hipGetLastError();
}

hipError_t launch_energy_from_sums(const PwParams& P, const double* sums, double dV, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(energy_from_sums_kernel, dim3(1), dim3(64), 0, s, P, sums, dV, out);
    return hipGetLastError();
}

hipError_t launch_reduce_segs(const RedSeg& s1, const RedSeg& s2, const RedSeg& s3, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_final_kernel, dim3(s1.M + s2.M + s3.M), dim3(256), 0, s, s1, s2, s3);
    return hipGetLastError();
}

hipError_t launch_reduce_final3(const double* partials1, int nblk1, int M1, double* out1, const double* partials2,
                                int nblk2, int M2, double* out2, const double* partials3, int nblk3, int M3,
                                double* out3, hipStream_t s)
{
    const RedSeg a{partials1, nblk1, M1, out1, nullptr}, b{partials2, nblk2, M2, out2, nullptr},
        c{partials3, nblk3, M3, out3, nullptr};
    return launch_reduce_segs(a, b, c, s);
}

hipError_t launch_ls_step(const PwParams& P, const StepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(ls_step_kernel, dim3(1), dim3(64), 0, s, P, a);
    return hipGetLastError();
}

hipError_t launch_reduce_final(const double* partials, int nblk, int M, double* out, hipStream_t s)
{
    return launch_reduce_final3(partials, nblk, M, out, nullptr, 0, 0, nullptr, nullptr, 0, 0, nullptr, s);
}

hipError_t launch_reduce_final2(const double* partials1, int nblk1, int M1, double* out1, const double* partials2,
                                int nblk2, int M2, double* out2, hipStream_t s)
{
    return launch_reduce_final3(partials1, nblk1, M1, out1, partials2, nblk2, M2, out2, nullptr, 0, 0, nullptr, s);
}

}  // namespace bec
