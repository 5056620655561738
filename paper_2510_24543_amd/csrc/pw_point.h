// Per-point algebra of the Hamiltonian epilogue (Sec. II, Eqs. (1), (3), (5),
// (6)) and of the direction-write pass (Sec. IV.B-IV.C, Sec. V), shared by the
// grid-stride kernels (pointwise.hip) and the passes that fuse them with a z
// transform (fft_fused.hip): the trap at a point, the inverse P_V diagonal, the
// operand loads, H psi with muLHY and the energy sums, and the point's z,
// direction p, residual r, rho = Re(conj(psi) p) and model sums.
#pragma once

#include "bec_internal.h"
#include "pcg_rules.h"
#include "pw_math.h"

namespace bec {
namespace pwpt {

__device__ __forceinline__ double trap_at(const PwParams& P, long long i)
{
    const uint32_t ii = (uint32_t)i;   // N < 2^31 (checked at creation)
    const uint32_t ix = (uint32_t)(((uint64_t)ii * P.m_nyz) >> P.s_nyz);
    const uint32_t rem = ii - ix * (uint32_t)(P.ny * P.nz);
    const uint32_t iy = (uint32_t)(((uint64_t)rem * P.m_nz) >> P.s_nz);
    const uint32_t iz = rem - iy * (uint32_t)P.nz;
    return P.vx[ix] + P.vy[iy] + P.vz[iz];
}

// the three table values of trap_at, unsummed
__device__ __forceinline__ void trap_parts(const PwParams& P, long long i, double* v)
{
    const uint32_t ii = (uint32_t)i;
    const uint32_t ix = (uint32_t)(((uint64_t)ii * P.m_nyz) >> P.s_nyz);
    const uint32_t rem = ii - ix * (uint32_t)(P.ny * P.nz);
    const uint32_t iy = (uint32_t)(((uint64_t)rem * P.m_nz) >> P.s_nz);
    const uint32_t iz = rem - iy * (uint32_t)P.nz;
    v[0] = P.vx[ix];
    v[1] = P.vy[iy];
    v[2] = P.vz[iz];
}

// node constants read from the kernel-argument block (scalar loads)
struct KernargNodes {
    const PwParams& P;
    __device__ double operator()(int q, int k) const { return P.node5[q][k]; }
};

// H psi_i = T psi_i + [V + sum_j (G_ij n_j + Gdd_ij Phi_j) + muLHY_i] psi_i at
// point i from psi (s1, s2), T psi (t1, t2) and Phi_1 + i Phi_2 (ph); stores
// H psi and muLHY (and Phi when store_phi) and adds the kHevalSums energy sums.
__device__ __forceinline__ void heval_point(const PwParams& P, const HevalArgs& A, long long N, long long i,
                                            double2 s1, double2 s2, double2 t1, double2 t2, double2 ph,
                                            bool store_phi, double* acc)
{
    const double n1 = sq2(s1), n2 = sq2(s2);
    const double V = trap_at(P, i);
    double e = 0.0, d1 = 0.0, d2 = 0.0;
    if (P.lhy_on) lhy_point(KernargNodes{P}, LhyTab{P.lhy_tab, P.lhy_K}, P.n_a, P.n_b, P.K5, P.K3, n1, n2, e, d1, d2);
    const double m1 = d1 / P.Nat[0], m2 = d2 / P.Nat[1];
    const double U1 = V + P.G[0][0] * n1 + P.G[0][1] * n2 + P.Gdd[0][0] * ph.x + P.Gdd[0][1] * ph.y + m1;
    const double U2 = V + P.G[1][0] * n1 + P.G[1][1] * n2 + P.Gdd[1][0] * ph.x + P.Gdd[1][1] * ph.y + m2;
    const double2 h1 = make_double2(t1.x + U1 * s1.x, t1.y + U1 * s1.y);
    const double2 h2 = make_double2(t2.x + U2 * s2.x, t2.y + U2 * s2.y);
    A.hpsi[i] = h1;
    A.hpsi[N + i] = h2;
    if (store_phi) A.aux[i] = ph;
    A.aux[N + i] = make_double2(m1, m2);
    acc[0] += redot(s1, t1);
    acc[1] += redot(s2, t2);
    acc[2] += V * n1;
    acc[3] += V * n2;
    acc[4] += n1 * n1;
    acc[5] += n1 * n2;
    acc[6] += n2 * n2;
    acc[7] += n1 * ph.x;
    acc[8] += n1 * ph.y;
    acc[9] += n2 * ph.x;
    acc[10] += n2 * ph.y;
    acc[11] += e;
    acc[12] += redot(s1, h1);
    acc[13] += redot(s2, h2);
    acc[14] += n1;
    acc[15] += n2;
    acc[16] += m1 * n1;
    acc[17] += m2 * n2;
}

// 1 / ([shift + V + sum_j G_cj n_j + muLHY_c]_+ + sigma): the inverse P_V diagonal
__device__ __forceinline__ double pv_inv(const PwParams& P, int c, double shift, double sigma, double V, double n1,
                                         double n2, double ml)
{
    const double g = shift + V + P.G[c][0] * n1 + P.G[c][1] * n2 + ml;
    return 1.0 / ((g > 0.0 ? g : 0.0) + sigma);
}

// The input of the k-space preconditioners at point i (see MakeRArgs): the
// residual r = H psi - mu psi (or the given r) as is, times P_V^-1, times
// D^-1/2, or blended with the kinetic preconditioner's output.
__device__ __forceinline__ void make_r_point(const PwParams& P, const MakeRArgs& A, long long N, long long i,
                                             double2& r1, double2& r2)
{
    const double2 s1 = A.psi[i], s2 = A.psi[N + i];
    if (A.rin) {
        r1 = A.rin[i];
        r2 = A.rin[N + i];
    } else {
        const double2 h1 = A.hpsi[i], h2 = A.hpsi[N + i];
        r1 = make_double2(h1.x - A.mu[0] * s1.x, h1.y - A.mu[0] * s1.y);
        r2 = make_double2(h2.x - A.mu[1] * s2.x, h2.y - A.mu[1] * s2.y);
    }
    if (A.apply_pv) {
        const double n1 = sq2(s1), n2 = sq2(s2);
        const double V = trap_at(P, i);
        const double2 ml = A.aux[N + i];
        double g1 = pv_inv(P, 0, A.diag_shift[0], A.sigma, V, n1, n2, ml.x);
        double g2 = pv_inv(P, 1, A.diag_shift[1], A.sigma, V, n1, n2, ml.y);
        if (A.apply_pv == 2) {
            g1 = sqrt(g1);
            g2 = sqrt(g2);
        }
        if (A.apply_pv == 3) {   // blend with the kinetic preconditioner's output zk
            const double a1 = A.blend_w[0] * g1, b1 = 1.0 - A.blend_w[0];
            const double a2 = A.blend_w[1] * g2, b2 = 1.0 - A.blend_w[1];
            const double2 k1 = A.zk[i], k2 = A.zk[N + i];
            r1 = make_double2(a1 * r1.x + b1 * k1.x, a1 * r1.y + b1 * k1.y);
            r2 = make_double2(a2 * r2.x + b2 * k2.x, a2 * r2.y + b2 * k2.y);
        } else {
            r1 = make_double2(g1 * r1.x, g1 * r1.y);
            r2 = make_double2(g2 * r2.x, g2 * r2.y);
        }
    }
}

// Operands of the direction-write pass at one point (ZM = DirArgs::zmode).
template <int ZM>
struct DirIn {
    double2 s[2], h[2], ph, ml, po[2], zb[2];
    double vt[3];   // the trap potential's x, y and z table values (summed where used, so the
                    // loads of a prefetched point are not waited for early)
};

template <int ZM>
__device__ __forceinline__ DirIn<ZM> dir_load(const PwParams& P, const DirArgs& A, long long N, long long i,
                                              bool with_p)
{
    DirIn<ZM> v;
    trap_parts(P, i, v.vt);
    v.s[0] = A.psi[i];
    v.s[1] = A.psi[N + i];
    v.h[0] = A.hpsi[i];
    v.h[1] = A.hpsi[N + i];
    v.ph = A.aux[i];
    v.ml = A.aux[N + i];
    if (with_p) {
        v.po[0] = A.p[i];
        v.po[1] = A.p[N + i];
    } else {
        v.po[0] = v.po[1] = make_double2(0.0, 0.0);
    }
    if constexpr (ZM >= 2 && ZM <= 4) {
        v.zb[0] = A.zbuf[i];
        v.zb[1] = A.zbuf[N + i];
    }
    return v;
}

// One point of the direction-write pass: z, the new direction p (stored with r
// and rho = Re conj(psi) p) and the line-search model sums.
template <int ZM, bool LHY>
__device__ __forceinline__ void dir_point(const PwParams& P, const DirArgs& A, long long N, long long i,
                                         const DirIn<ZM>& cur, double* acc, double2* p_pt = nullptr,
                                         double* rho_pt = nullptr)
{
    const double2* s = cur.s;
    double2 r[2], z[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) r[c] = make_double2(cur.h[c].x - A.mu[c] * s[c].x, cur.h[c].y - A.mu[c] * s[c].y);
    const double n[2] = {sq2(s[0]), sq2(s[1])};
    const double V = cur.vt[0] + cur.vt[1] + cur.vt[2];
    const double mlc[2] = {cur.ml.x, cur.ml.y};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        if constexpr (ZM == 0) {
            z[c] = r[c];
        } else if constexpr (ZM == 2) {
            z[c] = cur.zb[c];
        } else {
            const double g = pv_inv(P, c, A.diag_shift[c], A.sigma, V, n[0], n[1], mlc[c]);
            if constexpr (ZM == 1) {
                z[c] = make_double2(g * r[c].x, g * r[c].y);
            } else if constexpr (ZM == 3) {
                const double q = sqrt(g);
                z[c] = make_double2(q * cur.zb[c].x, q * cur.zb[c].y);
            } else {
                const double a = A.blend_w[c] * g, b = 1.0 - A.blend_w[c];
                z[c] = make_double2(a * r[c].x + b * cur.zb[c].x, a * r[c].y + b * cur.zb[c].y);
            }
        }
    }
    const double2 ph = cur.ph;
    double2 p[2];
    double rho[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        double2 d = make_double2(A.zsign * z[c].x, A.zsign * z[c].y);
        if (A.beta != 0.0) {
            d.x += A.beta * cur.po[c].x;
            d.y += A.beta * cur.po[c].y;
        }
        p[c] = make_double2(d.x - A.c[c] * s[c].x, d.y - A.c[c] * s[c].y);
        A.p_out[c * N + i] = p[c];
        A.r_out[c * N + i] = r[c];
        rho[c] = redot(s[c], p[c]);
        const double2 hmf = make_double2(cur.h[c].x - mlc[c] * s[c].x, cur.h[c].y - mlc[c] * s[c].y);
        const double U = V + P.G[c][0] * n[0] + P.G[c][1] * n[1] + P.Gdd[c][0] * ph.x + P.Gdd[c][1] * ph.y;
        const double pp = sq2(p[c]);
        acc[0 + c] += pp;
        acc[2 + c] += redot(p[c], r[c]);
        acc[4 + c] += redot(p[c], hmf);
        acc[6 + c] += redot(s[c], hmf);
        acc[8 + c] += U * pp;
        acc[10 + c] += mlc[c] * pp;
        acc[12 + c] += mlc[c] * n[c];
        acc[16 + c] += rho[c];
    }
    if (A.rho) A.rho[i] = make_double2(rho[0], rho[1]);
    if (p_pt) {                      // the point's p and rho for a caller that transforms them
        p_pt[0] = p[0];
        p_pt[1] = p[1];
        rho_pt[0] = rho[0];
        rho_pt[1] = rho[1];
    }
    if constexpr (LHY) {
        double L1, L2;
        lhy_model(KernargNodes{P}, LhyTab{P.lhy_tab, P.lhy_K}, P.n_a, P.n_b, n[0], n[1], 2.0 * rho[0], 2.0 * rho[1], L1, L2);
        acc[14] += L1;
        acc[15] += L2;
    }
}

}  // namespace pwpt
}  // namespace bec
