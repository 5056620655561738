"""Pins of the oracle's root-split rule for the u integral of the LHY term
(Sec. II, Eqs. (1), (3), (5); lhy_quad = 1).

The branch potentials V_+-(u) are clipped where they turn negative (eps_dd > 1);
the plain Gauss-Legendre sum then has an error of a few 1e-6.  The root-split
rule integrates between the zeros of the branches, with a map that smooths the
(u - u_b)^(k/2) behaviour at each zero, and converges exponentially.

Single component: e = c (8/(15 pi^2)) (G n)^(5/2) Q(eps) with
Q(eps) = int_0^1 [1 + eps (3u^2 - 1)]_+^(5/2) du, in closed form from the
antiderivatives of (x^2 + c^2)^(5/2) and (x^2 - c^2)^(5/2) (checked by finite
differences below).  Two components: against adaptive quadrature of the
integrand of Eq. (3) on each piece of the rule separately.

What the rule cannot split at: with n1 n2 small, s = sqrt(delta^2 + 4 eta_12
eta_21 n1 n2) has a rounded corner where delta(u) = 0, at a place that depends on
the densities; there 16 nodes per piece leave up to ~2e-8 (the plain rule ~1e-5),
and 48 reach round-off.
"""
import math

import numpy as np
import pytest
from scipy import integrate


def F_plus(x, c):
    """an antiderivative of (x^2 + c^2)^(5/2)"""
    r = math.sqrt(x * x + c * c)
    return (x * r ** 5 / 6 + 5 * c * c * x * r ** 3 / 24 + 5 * c ** 4 * x * r / 16
            + 5 * c ** 6 / 16 * math.log(x + r))


def F_minus(x, c):
    """an antiderivative of (x^2 - c^2)^(5/2), x >= c"""
    r = math.sqrt(max(x * x - c * c, 0.0))
    return (x * r ** 5 / 6 - 5 * c * c * x * r ** 3 / 24 + 5 * c ** 4 * x * r / 16
            - 5 * c ** 6 / 16 * math.log(x + r))


def Q_closed(eps):
    """int_0^1 [1 - eps + 3 eps u^2]_+^(5/2) du, x = sqrt(3 eps) u"""
    k = math.sqrt(3 * eps)
    X = k
    if eps < 1:
        c = math.sqrt(1 - eps)
        return (F_plus(X, c) - F_plus(0.0, c)) / k
    c = math.sqrt(eps - 1)
    return (F_minus(X, c) - F_minus(c, c)) / k


def test_antiderivatives():
    for F, sgn in ((F_plus, 1.0), (F_minus, -1.0)):
        for x, c in ((1.3, 0.7), (2.0, 1.1), (3.5, 0.4)):
            h = 1e-5
            d = (F(x + h, c) - F(x - h, c)) / (2 * h)
            assert abs(d - (x * x + sgn * c * c) ** 2.5) < 1e-7 * (x * x + sgn * c * c) ** 2.5


def params(G=((4.0, 0.0), (0.0, 3.0)), Gdd=((5.2, 0.0), (0.0, 1.0)), n_u=16, quad=1, N=(1.0, 1.0)):
    return {"N": list(N), "omega": [0.0, 0.0, 0.0], "G": [list(r) for r in G], "Gdd": [list(r) for r in Gdd],
            "c_lhy": 1.0, "r_cut": 8.0, "n_u": n_u, "lhy_quad": quad}


@pytest.mark.parametrize("eps,n_u", [(0.3, 16), (0.9, 32), (1.3, 16), (1.875, 16), (3.0, 16), (10.0, 16)])
def test_single_component_matches_closed_form(orc, eps, n_u):
    """eps > 1: 16 nodes per piece give the clipped integral to 1e-13.  eps = 0.9
    is not clipped but nearly so (complex zeros of V close to u = 0): 32 nodes."""
    G, n1 = 4.0, 0.8
    exact = 8.0 / (15 * math.pi ** 2) * (G * n1) ** 2.5 * Q_closed(eps)
    P = params(G=((G, 0.0), (0.0, 3.0)), Gdd=((eps * G, 0.0), (0.0, 1.0)), n_u=n_u)
    e = orc.lhy_point(P, n1, 0.0)
    assert abs(e[0] - exact) <= 1e-13 * exact
    # the plain rule is off by ~1e-6 once the branch is clipped
    if eps > 1:
        plain = orc.lhy_point(dict(P, lhy_quad=0), n1, 0.0)[0]
        assert abs(plain - exact) > 1e-9 * exact


K5 = math.sqrt(2) / (15 * math.pi ** 2)
K3 = 1 / (3 * math.sqrt(2) * math.pi ** 2)


def integrand(P, n1, n2, u, which):
    a = 3 * u * u - 1
    e = [[P["G"][i][j] + P["Gdd"][i][j] * a for j in range(2)] for i in range(2)]
    d = e[0][0] * n1 - e[1][1] * n2
    s = math.sqrt(d * d + 4 * e[0][1] * e[1][0] * n1 * n2)
    tot = 0.0
    for sg in (1.0, -1.0):
        V = e[0][0] * n1 + e[1][1] * n2 + sg * s
        if V <= 0:
            continue
        if which == 0:
            tot += V ** 2.5
        elif which == 1:
            tot += V ** 1.5 * (e[0][0] + sg * (e[0][0] * d + 2 * e[0][1] * e[1][0] * n2) / s)
        else:
            tot += V ** 1.5 * (e[1][1] + sg * (-e[1][1] * d + 2 * e[0][1] * e[1][0] * n1) / s)
    return tot


@pytest.mark.parametrize("G,Gdd,N", [
    (((80.0, 40.0), (40.0, 80.0)), ((150.0, 105.0), (105.0, 75.0)), (1.0, 1.0)),      # the droplet couplings
    (((60.0, 70.0), (70.0, 60.0)), ((78.0, 91.0), (91.0, 78.0)), (1.0, 1.0)),         # the stripe couplings
    (((100.0, 50.0), (31.25, 90.0)), ((160.0, 45.0), (28.125, 50.0)), (1.0, 1.6)),   # N_1 != N_2
])
def test_two_components_match_adaptive_quadrature(orc, G, Gdd, N):
    n = 48
    P = params(G=G, Gdd=Gdd, N=N, n_u=n)
    u, w = orc.lhy_nodes(P)
    assert len(u) > n and abs(w.sum() - 1.0) < 1e-14
    # the zeros of the branches: where the rule's pieces meet
    pieces = len(u) // n
    ends = [0.0] + [0.5 * (u[n * k - 1] + u[n * k]) for k in range(1, pieces)] + [1.0]
    for n1, n2 in ((0.31, 0.17), (0.05, 0.4), (0.2, 1e-3)):
        got = orc.lhy_point(P, n1, n2)
        for which, pre in ((0, K5), (1, K3), (2, K3)):
            ref = sum(integrate.quad(lambda x: integrand(P, n1, n2, x, which), a, b,
                                     epsabs=1e-18, epsrel=1e-14, limit=1000)[0] for a, b in zip(ends[:-1], ends[1:]))
            assert abs(got[which] - pre * ref) <= 1e-13 * abs(pre * ref), (which, got[which], pre * ref)
        # 16 nodes per piece: within 1e-7 even at a density ratio of 200 (the rounded corner)
        got16 = orc.lhy_point(dict(P, n_u=16), n1, n2)
        assert np.max(np.abs(got16 - got) / np.abs(got)) < 1e-7


def test_rule_converges_exponentially(orc):
    P = params(G=((80.0, 40.0), (40.0, 80.0)), Gdd=((150.0, 105.0), (105.0, 75.0)))
    vals = [orc.lhy_point(dict(P, n_u=n), 0.3, 0.2) for n in (12, 16, 24, 32)]
    for v in vals[1:]:
        assert np.max(np.abs(v - vals[-1]) / np.abs(vals[-1])) < 1e-13
    plain = [orc.lhy_point(dict(P, n_u=n, lhy_quad=0), 0.3, 0.2) for n in (16, 64)]
    assert np.max(np.abs(plain[0] - vals[-1]) / np.abs(vals[-1])) > 1e-8       # the plain rule's error


def test_unclipped_parameters_need_no_split(orc):
    """eps_dd < 1 and det > 0 on [0,1]: one piece; with 32 nodes both rules give
    the integral to round-off (with 16, to about 1e-12: complex zeros of the
    branches lie near the interval)."""
    P = params(G=((100.0, 50.0), (50.0, 100.0)), Gdd=((60.0, 60.0), (60.0, 60.0)), n_u=32)
    u, _ = orc.lhy_nodes(P)
    assert len(u) == 32
    a = orc.lhy_point(P, 0.3, 0.2)
    b = orc.lhy_point(dict(P, lhy_quad=0), 0.3, 0.2)
    assert np.max(np.abs(a - b) / np.abs(b)) < 1e-14
