// FP64 device math shared by the single-instance and batched pointwise
// kernels: complex helpers, the reciprocal square root, and the LHY
// quadrature loops (arXiv:2510.24543, Sec. II Eqs. (1), (3), (5); Sec. V).
#pragma once
#include <hip/hip_runtime.h>

namespace bec {

__device__ __forceinline__ double sq2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double redot(double2 a, double2 b) { return a.x * b.x + a.y * b.y; }  // Re(conj(a) b)

// Reciprocal square root to full FP64 accuracy for x > kTiny: the hardware
// estimate followed by two Newton steps r <- r (3 - x r^2) / 2.
constexpr double kTiny = 1e-290;
__device__ __forceinline__ double rsq_nr(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    r = r * fma(-h * r, r, 1.5);
    r = r * fma(-h * r, r, 1.5);
    return r;
}

// Per node q the tables hold (eta_11, eta_22, eta_12 eta_21, w_q, r_q) with
// r_q = sqrt(eta_11 eta_22 - eta_12 eta_21) when that is >= 0, else -1.
// Since V_+ V_- = 4 n1 n2 (eta_11 eta_22 - eta_12 eta_21), sqrt(V_-) follows from
// 1/sqrt(V_+) as 2 sqrt(n1 n2) r_q / sqrt(V_+): two reciprocal square roots per
// node (s and V_+) instead of three.  A negative product means V_- < 0, whose
// branch is clipped away ([V]_+).
constexpr int kNodeVals = 5;

// LHY energy density and derivatives at one point.  Branches with V <= 0
// contribute nothing ([V]_+ powers); ratio terms vanish when s = 0.  Values
// below kTiny are treated as 0: their contributions (V^(3/2) < 1e-435) are
// below FP64 resolution.  Branch-free: masks instead of divergent ifs.
// Nodes: any type with operator()(q, k) giving the k-th table value of node q.
template <class Nodes>
__device__ __forceinline__ void lhy_point(const Nodes& nodes, int n_u, double K5, double K3, double n1,
                                          double n2, double& e, double& d1, double& d2)
{
    double ae = 0.0, a1 = 0.0, a2 = 0.0;
    const double n12x4 = 4.0 * n1 * n2, n1x2 = 2.0 * n1, n2x2 = 2.0 * n2;
    const double nn = n1 * n2;
    const double sqnn2 = nn > kTiny ? 2.0 * nn * rsq_nr(nn) : 0.0;      // 2 sqrt(n1 n2)
    for (int q = 0; q < n_u; ++q) {
        const double e11 = nodes(q, 0), e22 = nodes(q, 1), p12 = nodes(q, 2), w = nodes(q, 3), rq = nodes(q, 4);
        const double a = e11 * n1, b = e22 * n2, delta = a - b, base = a + b;
        const double ss = fma(delta, delta, p12 * n12x4);
        const double inv = ss > kTiny ? rsq_nr(ss) : 0.0;              // 1/s
        const double s = ss * inv;
        const double r1 = fma(e11, delta, p12 * n2x2) * inv;
        const double r2 = fma(-e22, delta, p12 * n1x2) * inv;
        const double Vp = base + s;
        const bool pp = Vp > kTiny;
        const double xp = pp ? Vp : 1.0;
        const double rp = rsq_nr(xp);                                  // 1/sqrt(V_+)
        const double sqp = xp * rp;                                    // sqrt(V_+)
        const double sqm = rq >= 0.0 ? sqnn2 * rq * rp : 0.0;          // sqrt(V_-) (0 when clipped)
        const double Vm = sqm * sqm;
        const double cp = (pp ? w : 0.0) * xp * sqp;                   // w V_+^(3/2)
        const double cm = (pp ? w : 0.0) * Vm * sqm;                   // w V_-^(3/2)
        ae = fma(cp, xp, fma(cm, Vm, ae));
        a1 = fma(cp, e11 + r1, fma(cm, e11 - r1, a1));
        a2 = fma(cp, e22 + r2, fma(cm, e22 - r2, a2));
    }
    e = K5 * ae;
    d1 = K3 * a1;
    d2 = K3 * a2;
}

// LHY part of the geodesic model with n'' = 0: sums of [V]_+^(3/2) V^1 and of
// [V]_+^(3/2) V^2_0 + 3/4 [V]_+^(1/2) (V^1)^2.  The n'' part of V^2 is linear in
// n''_i with coefficient dV/dn_i and is added from muLHY on the host.
// B/(2s) - A^2/(2s^3) is evaluated as (B - (A/s)^2)/(2s): s^3 underflows at
// tiny densities.
template <class Nodes>
__device__ __forceinline__ void lhy_model(const Nodes& nodes, int n_u, double n1, double n2, double n1p,
                                          double n2p, double& L1, double& L2)
{
    double s1 = 0.0, s2acc = 0.0;
    const double n12x4 = 4.0 * n1 * n2, cross = 2.0 * (n1 * n2p + n1p * n2), pp4 = 4.0 * n1p * n2p;
    const double nn = n1 * n2;
    const double sqnn2 = nn > kTiny ? 2.0 * nn * rsq_nr(nn) : 0.0;
    for (int q = 0; q < n_u; ++q) {
        const double e11 = nodes(q, 0), e22 = nodes(q, 1), p12 = nodes(q, 2), w = nodes(q, 3), rq = nodes(q, 4);
        const double delta = e11 * n1 - e22 * n2;
        const double d1 = e11 * n1p - e22 * n2p;
        const double ss = fma(delta, delta, p12 * n12x4);
        const double inv = ss > kTiny ? rsq_nr(ss) : 0.0;
        const double s = ss * inv;
        const double A = fma(delta, d1, p12 * cross);
        const double B0 = fma(d1, d1, p12 * pp4);
        const double lin1 = e11 * n1p + e22 * n2p;
        const double ra = A * inv;
        const double rb = 0.5 * fma(-ra, ra, B0) * inv;
        const double Vp = e11 * n1 + e22 * n2 + s;
        const bool pp = Vp > kTiny;
        const double xp = pp ? Vp : 1.0;
        const double rp = rsq_nr(xp);
        const double rvp = xp * rp;                                    // sqrt(V_+)
        const double rvm = rq >= 0.0 ? sqnn2 * rq * rp : 0.0;          // sqrt(V_-)
        const double xm = rvm * rvm;
        const double wp = pp ? w : 0.0;
        const double V1p = lin1 + ra, V1m = lin1 - ra;
        s1 = fma(wp * xp * rvp, V1p, fma(wp * xm * rvm, V1m, s1));
        s2acc = fma(wp * rvp, fma(xp, rb, 0.75 * V1p * V1p), fma(wp * rvm, fma(-xm, rb, 0.75 * V1m * V1m), s2acc));
    }
    L1 = s1;
    L2 = s2acc;
}

}  // namespace bec
