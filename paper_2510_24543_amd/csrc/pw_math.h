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

// Node classes.  With det_q = eta_11 eta_22 - eta_12 eta_21 (eta_12 eta_21 >= 0
// because N_i G_ij and N_i Gdd_ij are symmetric) the two branch potentials
// satisfy V_+ + V_- = 2 (eta_11 n1 + eta_22 n2) and V_+ V_- = 4 n1 n2 det_q, so
// for n1 n2 > 0 the signs of V_+- are fixed per node, independent of the point:
//   class A: det_q >= 0 and eta_11, eta_22 >= 0 (not both 0): V_+, V_- >= 0;
//   class B: det_q < 0: V_+ > 0 > V_-, the V_- branch is clipped ([V]_+);
//   otherwise (det_q >= 0, eta_11, eta_22 <= 0) both branches are clipped and
//   the node contributes nothing.
// The host stores the class-A nodes first, then the class-B nodes; per node the
// table holds (eta_11, eta_22, eta_12 eta_21, w_q, sqrt(det_q) or 0).
//
// Class A uses a = sqrt(V_+), b = sqrt(V_-) through sigma = a + b and pi = a b:
// sigma^2 = 2 (eta_11 n1 + eta_22 n2) + 2 pi, pi = 2 sqrt(n1 n2 det_q), and
//   a^5 + b^5 = sigma (sigma^4 - 5 sigma^2 pi + 5 pi^2),
//   a^3 + b^3 = sigma (sigma^2 - 3 pi),
//   a^3 - b^3 = (2 s / sigma) (sigma^2 - pi),
// so every sum over the two branches needs one reciprocal square root (of
// sigma^2) and no square root of s^2.  Class B needs s and sqrt(V_+).
// As in the definition of the ratio terms, terms carrying 1/s are dropped
// where s^2 <= kTiny.
constexpr int kNodeVals = 5;

// The class-A part of the node sum, F(n1, n2) = sum_q w_q sum_+- V_+-^(5/2) over
// the class-A nodes, is homogeneous of degree 5/2 (V is linear in n), so
// F = R^(5/2) f(x) with R = n1 + n2 and x = n1 / R.  The host can tabulate f, f'
// and f'' as Chebyshev series in y = (sqrt n1 - sqrt n2)/(sqrt n1 + sqrt n2) =
// (n1 - n2)/(R + 2 sqrt(n1 n2)), in which they are analytic on [-1, 1] (the
// V_-^(5/2) endpoint terms become polynomial), and checks the series against the
// node sum; then the point evaluations below replace the class-A loop (3 series
// of K <= kLhyTabMax terms instead of n_a nodes).  The class-B loop is unchanged.
struct LhyTab {
    const double* c;   // series s at c[s * kLhyTabMax + k], s = 0 f, 1 f', 2 f''
    int K;             // terms per series; 0: no table (class-A loop)
};

// Sums of the first NS series at y, sum_k c_k T_k(y) in ascending k, with
// T_k(y) from the three-term recurrence T_(k+1) = 2y T_k - T_(k-1): one FMA per
// term for T_k and one per series (Clenshaw's backward form takes two
// operations per term and series).  K is even: two terms per trip.  The
// coefficients are uniform across the wavefront and read through the scalar
// cache (constant address space).
template <int NS>
__device__ __forceinline__ void lhy_cheb(const LhyTab& T, double y, double (&g)[NS])
{
    using cptr = const __attribute__((address_space(4))) double*;
    const cptr c = (cptr)T.c;
    const double y2 = y + y;
    double s[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) s[q] = fma(c[q * kLhyTabMax + 1], y, c[q * kLhyTabMax]);
    double tm = 1.0, tk = y;   // T_(k-2), T_(k-1)
    for (int k = 2; k < T.K; k += 2) {
        const double ta = fma(y2, tk, -tm);   // T_k
        const double tb = fma(y2, ta, -tk);   // T_(k+1)
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            s[q] = fma(c[q * kLhyTabMax + k], ta, s[q]);
            s[q] = fma(c[q * kLhyTabMax + k + 1], tb, s[q]);
        }
        tm = ta;
        tk = tb;
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) g[q] = s[q];
}

// LHY energy density e and de/dn_i at one point.  Values below kTiny are
// treated as 0: their contributions (V^(3/2) < 1e-435) are below FP64
// resolution.  Branch-free: masks instead of divergent ifs.
// Nodes: any type with operator()(q, k) giving the k-th table value of node q.
template <class Nodes>
__device__ __forceinline__ void lhy_point(const Nodes& nodes, const LhyTab& tab, int n_a, int n_b, double K5,
                                          double K3, double n1, double n2, double& e, double& d1, double& d2)
{
    double ae = 0.0, a1 = 0.0, a2 = 0.0;
    const double n12x4 = 4.0 * n1 * n2;
    const double nn = n1 * n2;
    const double sqnn2 = nn > kTiny ? 2.0 * nn * rsq_nr(nn) : 0.0;      // 2 sqrt(n1 n2)
    const double tn1 = 2.0 * n1, tn2 = 2.0 * n2;
    if (tab.K > 0) {   // class A from the table: F, and dF/dn_i = R^(3/2) (5/2 f + (1 - x) f', 5/2 f - x f')
        const double R = n1 + n2;
        if (R > kTiny) {
            const double rr = rsq_nr(R), sR = R * rr, iR = rr * rr, R32 = R * sR;
            const double y = (n1 - n2) / (R + sqnn2);
            const double x1 = n1 * iR, x2 = n2 * iR;
            double g[2];
            lhy_cheb<2>(tab, y, g);
            ae = R * R32 * g[0];
            a1 = 0.4 * R32 * fma(2.5, g[0], x2 * g[1]);      // the loop's sums are (2/5) dF/dn_i
            a2 = 0.4 * R32 * fma(2.5, g[0], -x1 * g[1]);
        }
    }
    // Class A without per-node guards: where sigma^2 <= kTiny every term of the
    // node is below 1e-140 (r is taken at kTiny, so nothing overflows), and where
    // s^2 <= kTiny the ratio term u t1 carries a factor u = s ds/dn of size
    // sqrt(kTiny); both are below FP64 resolution against the other terms.
    const int na_loop = tab.K > 0 ? 0 : n_a;
    for (int q = 0; q < na_loop; ++q) {
        const double e11 = nodes(q, 0), e22 = nodes(q, 1), p12 = nodes(q, 2), w = nodes(q, 3), rq = nodes(q, 4);
        const double a = e11 * n1, b = e22 * n2, delta = a - b;
        const double pi = sqnn2 * rq;
        const double x = 2.0 * (a + b + pi);                            // sigma^2
        const double r = rsq_nr(fmax(x, kTiny));                       // 1/sigma
        const double sg = x * r;
        const double t1 = (x - pi) * (r + r);                           // 2 (sigma^2 - pi)/sigma
        const double t3 = sg * fma(-3.0, pi, x);                        // a^3 + b^3
        const double e5 = sg * fma(x, fma(-5.0, pi, x), 5.0 * pi * pi); // a^5 + b^5
        const double u1 = fma(e11, delta, p12 * tn2);                   // s ds/dn1
        const double u2 = fma(-e22, delta, p12 * tn1);                  // s ds/dn2
        ae = fma(w, e5, ae);
        a1 = fma(w, fma(e11, t3, u1 * t1), a1);
        a2 = fma(w, fma(e22, t3, u2 * t1), a2);
    }
    for (int q = n_a; q < n_a + n_b; ++q) {
        const double e11 = nodes(q, 0), e22 = nodes(q, 1), p12 = nodes(q, 2), w = nodes(q, 3);
        const double a = e11 * n1, b = e22 * n2, delta = a - b;
        const double ss = fma(delta, delta, p12 * n12x4);
        const double inv = ss > kTiny ? rsq_nr(ss) : 0.0;              // 1/s
        const double Vp = fma(ss, inv, a + b);
        const bool pp = Vp > kTiny;
        const double xp = pp ? Vp : 1.0;
        const double cp = (pp ? w : 0.0) * xp * (xp * rsq_nr(xp));     // w V_+^(3/2)
        const double r1 = fma(e11, delta, 2.0 * p12 * n2) * inv;
        const double r2 = fma(-e22, delta, 2.0 * p12 * n1) * inv;
        ae = fma(cp, xp, ae);
        a1 = fma(cp, e11 + r1, a1);
        a2 = fma(cp, e22 + r2, a2);
    }
    e = K5 * ae;
    d1 = K3 * a1;
    d2 = K3 * a2;
}

// LHY part of the geodesic model with n'' = 0: sums over nodes and branches of
// [V]_+^(3/2) V^1 and of [V]_+^(3/2) V^2_0 + 3/4 [V]_+^(1/2) (V^1)^2, with
// V^1 = lin +- A/s and V^2_0 = +-(B - (A/s)^2)/(2s) along (n1', n2').  The n''
// part of V^2 is linear in n''_i with coefficient dV/dn_i and is added from
// muLHY on the host.  For class A the branch sums reduce to
//   sum a^3 V^1      = lin (a^3 + b^3) + 2 A (sigma^2 - pi)/sigma,
//   sum a^3 V^2_0    = (B - A^2/s^2) (sigma^2 - pi)/sigma,
//   sum a (V^1)^2    = sigma (lin^2 + A^2/s^2) + 4 lin A / sigma,
// and since s^2 = sigma^2 (a - b)^2 / 4 the A^2/s^2 parts combine to
//   sum [a^3 V^2_0 + 3/4 a (V^1)^2] = B (sigma^2 - pi)/sigma - A^2/sigma^3
//                                     + 3/4 sigma lin^2 + 3 lin A / sigma,
// free of 1/s (and of the cancellation it carries where s is small).
template <class Nodes>
__device__ __forceinline__ void lhy_model(const Nodes& nodes, const LhyTab& tab, int n_a, int n_b, double n1,
                                          double n2, double n1p, double n2p, double& L1, double& L2)
{
    double s1 = 0.0, s2acc = 0.0;
    const double n12x4 = 4.0 * n1 * n2, cross = 2.0 * (n1 * n2p + n1p * n2), pp4 = 4.0 * n1p * n2p;
    const double nn = n1 * n2;
    const double sqnn2 = nn > kTiny ? 2.0 * nn * rsq_nr(nn) : 0.0;
    if (tab.K > 0) {   // class A from the table: (2/5) dF/ds and (1/5) d^2F/ds^2 along (n1', n2')
        const double R = n1 + n2;
        if (R > kTiny) {
            const double rr = rsq_nr(R), sR = R * rr, iR = rr * rr, R32 = R * sR;
            const double y = (n1 - n2) / (R + sqnn2);
            const double x1 = n1 * iR, x2 = n2 * iR;
            double g[3];
            lhy_cheb<3>(tab, y, g);
            // F_1 = R^(3/2) h1, F_2 = R^(3/2) h2; Hessian R^(1/2) (H11, H12, H22)
            const double h1 = fma(2.5, g[0], x2 * g[1]), h2 = fma(2.5, g[0], -x1 * g[1]);
            const double q1 = fma(1.5, g[1], x2 * g[2]), q2 = fma(1.5, g[1], -x1 * g[2]);
            const double H11 = fma(1.5, h1, x2 * q1), H12 = fma(1.5, h1, -x1 * q1), H22 = fma(1.5, h2, -x1 * q2);
            s1 = 0.4 * R32 * fma(h1, n1p, h2 * n2p);
            s2acc = 0.2 * sR * fma(H11 * n1p, n1p, n2p * fma(2.0 * H12, n1p, H22 * n2p));
        }
    }
    const int na_loop = tab.K > 0 ? 0 : n_a;
    for (int q = 0; q < na_loop; ++q) {
        const double e11 = nodes(q, 0), e22 = nodes(q, 1), p12 = nodes(q, 2), w = nodes(q, 3), rq = nodes(q, 4);
        const double a = e11 * n1, b = e22 * n2, delta = a - b;
        const double d1 = e11 * n1p - e22 * n2p;
        const double lin = fma(e11, n1p, e22 * n2p);
        const double pi = sqnn2 * rq;
        const double x = 2.0 * (a + b + pi);
        // no guard on sigma^2 <= kTiny (see lhy_point); the s^2 <= kTiny rule
        // stays, since B t1 is not small there
        const double r = rsq_nr(fmax(x, kTiny));
        const double sg = x * r;
        const double ss = fma(delta, delta, p12 * n12x4);
        const bool sp = ss > kTiny;
        const double A = sp ? fma(delta, d1, p12 * cross) : 0.0;
        const double B0 = sp ? fma(d1, d1, p12 * pp4) : 0.0;
        const double t1 = (x - pi) * r;                                 // (sigma^2 - pi)/sigma
        const double t3 = sg * fma(-3.0, pi, x);
        const double Ar = A * r;
        s1 = fma(w, fma(lin, t3, (A + A) * t1), s1);
        const double v2 = fma(B0, t1, -Ar * Ar * r);
        s2acc = fma(w, v2 + lin * fma(0.75 * sg, lin, 3.0 * Ar), s2acc);
    }
    for (int q = n_a; q < n_a + n_b; ++q) {
        const double e11 = nodes(q, 0), e22 = nodes(q, 1), p12 = nodes(q, 2), w = nodes(q, 3);
        const double delta = e11 * n1 - e22 * n2;
        const double d1 = e11 * n1p - e22 * n2p;
        const double ss = fma(delta, delta, p12 * n12x4);
        const double inv = ss > kTiny ? rsq_nr(ss) : 0.0;
        const double A = fma(delta, d1, p12 * cross);
        const double B0 = fma(d1, d1, p12 * pp4);
        const double lin = fma(e11, n1p, e22 * n2p);
        const double ra = A * inv;
        const double rb = 0.5 * fma(-ra, ra, B0) * inv;
        const double Vp = fma(ss, inv, fma(e11, n1, e22 * n2));
        const bool pp = Vp > kTiny;
        const double xp = pp ? Vp : 1.0;
        const double rvp = xp * rsq_nr(xp);                              // sqrt(V_+)
        const double wp = pp ? w : 0.0;
        const double V1 = lin + ra;
        s1 = fma(wp * xp * rvp, V1, s1);
        s2acc = fma(wp * rvp, fma(xp, rb, 0.75 * V1 * V1), s2acc);
    }
    L1 = s1;
    L2 = s2acc;
}

}  // namespace bec
