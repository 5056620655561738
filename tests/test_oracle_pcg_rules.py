"""Pins of the oracle's direction and step rules: the conjugacy parameter and
its restarts (Sec. IV.C, Eqs. (19)-(23)), the tangent direction (Sec. III,
Algorithm 1; Sec. V), the closed-form step of the second-order model and its
validation along the exact geodesic with Armijo halving, the beta = 0 retry and
stagnation (Sec. V, last paragraph), and the composite preconditioner's
fallback when its direction is not a descent direction.

The oracle traces, for each accepted step, psi (start of the step), r, the z
its direction used, p_old, the unprojected d and the projected p.  Every check
below is a property that the paper's rule defines, evaluated by numpy on those
vectors or through separate oracle entry points (geodesic, energy, model,
preconditioner), never by re-running the oracle's own beta or Armijo code:

* HS+: the new direction is conjugate to the change of the residual in the
  stacked inner product, <r^(n) - r^(n-1), d^(n)>_S = 0 whenever beta > 0;
* PR+: beta <r^(n-1), z^(n-1)>_S = <r^(n) - r^(n-1), z^(n)>_S;
* beta >= 0, and beta = 0 with d = -z where the ratio is negative, at n = 0,
  at every restart period and where the direction with beta is not descending;
* the model step minimises E0 + E1 a + E2 a^2 / 2 (clamped at theta_max);
* an accepted Armijo step is the model step halved h times, satisfies
  E(a) <= E0 + c1 a E1 + tau, and every earlier trial of that step did not.

<a, b>_S = sum_i w_i Re<a_i, b_i>, w_i = (N_i / (N_1 + N_2))^2 (the stacked
inner product of the product manifold, Sec. IV.C; reading 19).  Every case has
N_1 != N_2, so a dropped weight changes beta.
"""
import functools

import numpy as np
import pytest

from paper_2510_24543_amd import inputs

GRID = {"n": [16, 16, 16], "lo": [-6.0, -6.0, -6.0], "hi": [6.0, 6.0, 6.0]}


def _params(scale=1.0):
    s = float(scale)
    return {"N": [1.0, 1.6], "omega": [1.0, 1.2, 2.6],
            "G": [[100.0 * s, 50.0 * s], [31.25 * s, 90.0 * s]],
            "Gdd": [[60.0 * s, 45.0 * s], [28.125 * s, 50.0 * s]],
            "c_lhy": 5.0, "r_cut": 6.0, "n_u": 16}


P_MIX = _params(1.0)
P_STRONG = _params(10.0)     # compressed cloud: the quadratic model overshoots, Armijo engages
DV = float(np.prod([(GRID["hi"][d] - GRID["lo"][d]) / GRID["n"][d] for d in range(3)]))
NTOT = sum(P_MIX["N"])
W = [(P_MIX["N"][i] / NTOT) ** 2 for i in range(2)]
C1 = 0.3          # a sufficient-decrease constant large enough that its sign matters


def S(a, b, w=W):
    """Stacked inner product sum_i w_i dV Re<a_i, b_i>."""
    return sum(w[i] * DV * np.vdot(a[i], b[i]).real for i in range(2))


def E1_of(p, r, P):
    """sum_i 2 N_i dV Re<p_i, r_i> (the descent test of Sec. IV.C / V)."""
    return sum(2.0 * P["N"][i] * DV * np.vdot(p[i], r[i]).real for i in range(2))


def project(d, psi):
    out = d.copy()
    for i in range(2):
        out[i] -= (DV * np.vdot(psi[i], d[i]).real) * psi[i]
    return out


def relerr(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@functools.lru_cache(maxsize=None)
def run(scale=1.0, seed=71, phase=True, n_steps=40, **kw):
    import oracle
    P = _params(scale)
    psi0 = inputs.initial_state(GRID, P["omega"], seed, phase=phase)
    opts = dict({"tol_grad": 1e-10, "max_iter": n_steps}, **kw)
    psi, rep, log, tr = oracle.solve_traced(GRID, P, psi0, opts, n_steps=n_steps)
    return P, opts, psi, rep, log, tr


def energy(orc, P, psi):
    return orc.heval(GRID, P, psi)[0]["E"]


def raw_ratio(tr, k, mode):
    """The conjugacy ratio of step k from the traced vectors (mode 0 HS, 1 PR)."""
    y = tr[k]["r"] - tr[k - 1]["r"]
    num = S(y, tr[k]["z"])
    den = S(y, tr[k]["p_old"]) if mode == 0 else S(tr[k - 1]["r"], tr[k - 1]["z"])
    return num, den


RUNS = [dict(pc=1, beta=0), dict(pc=1, beta=1), dict(pc=0, beta=0), dict(pc=3, beta=0),
        dict(pc=3, beta=1), dict(pc=2, beta=1), dict(pc=4, beta=0)]


# ---------------------------------------------------------------- direction
@pytest.mark.parametrize("kw", RUNS, ids=lambda k: f"pc{k['pc']}-beta{k['beta']}")
def test_direction_is_projected_minus_z_plus_beta_p_old(orc, kw):
    P, opts, _, rep, log, tr = run(**kw)
    assert len(log) >= 30
    for k, (L, T) in enumerate(zip(log, tr)):
        psi, r, z = T["psi"], T["r"], T["z"]
        # r is the tangent residual H psi - mu psi of the iterate (Sec. III, Eq. (8))
        t, h, _, _ = orc.heval(GRID, P, psi)
        ref_r = np.stack([h[i] - t["mu"][i] * psi[i] for i in range(2)])
        assert relerr(r, ref_r) < 1e-12, k
        # z is P^-1 r of the chosen preconditioner (Sec. IV.B)
        if L["level"] <= 1:
            assert relerr(z, orc.precond(GRID, P, opts["pc"], opts.get("sigma", 1e-6), psi, r)) < 1e-13, k
        # d = -z + beta p_old, p its projection onto the tangent space (Algorithm 1; Sec. V)
        beta = L["beta"]
        assert beta >= 0.0
        assert relerr(T["d"], -z + beta * T["p_old"]) < 1e-15, k
        assert relerr(T["p"], project(T["d"], psi)) < 1e-13, k
        for i in range(2):
            assert abs(DV * np.vdot(psi[i], T["p"][i]).real) < 1e-13 * np.sqrt(DV * np.vdot(T["p"][i], T["p"][i]).real)
        if k == 0:
            assert L["level"] >= 1 and beta == 0.0 and not np.any(T["p_old"])
        else:
            assert np.array_equal(T["p_old"], tr[k - 1]["p"])          # the stored direction of the last step
            # the accepted point of the last step is where this step starts
            nxt = orc.geodesic(GRID, tr[k - 1]["psi"], tr[k - 1]["p"], log[k - 1]["alpha"])
            assert relerr(psi, nxt) < 1e-13, k
        # a descent direction, and E1 of the model is its slope sum_i 2 N_i Re<p_i, r_i>
        rp = E1_of(T["p"], r, P)
        assert rp < 0.0 and abs(L["rp"] - rp) <= 1e-12 * abs(rp), k
        assert abs(L["E1"] - rp) <= 1e-9 * abs(rp), k


# ---------------------------------------------------------------- conjugacy parameter
@pytest.mark.parametrize("pc", [0, 1, 3])
def test_hs_plus_direction_is_conjugate_to_the_residual_change(orc, pc):
    P, _, _, _, log, tr = run(pc=pc, beta=0)
    checked = 0
    for k in range(1, len(log)):
        if log[k]["level"] != 0:
            continue
        y = tr[k]["r"] - tr[k - 1]["r"]
        scale = abs(S(y, tr[k]["z"])) + log[k]["beta"] * abs(S(y, tr[k]["p_old"]))
        assert abs(S(y, tr[k]["d"])) <= 1e-11 * scale, k
        num, den = raw_ratio(tr, k, 0)
        assert abs(log[k]["beta_num"] - num) <= 1e-12 * abs(num) and abs(log[k]["beta_den"] - den) <= 1e-12 * abs(den)
        # the pin tells the rules apart at this step: the PR+ ratio and the
        # unweighted HS ratio are different numbers
        pn, pd = raw_ratio(tr, k, 1)
        yu = [1.0, 1.0]
        hu = S(y, tr[k]["z"], yu) / S(y, tr[k]["p_old"], yu)
        assert abs(pn / pd - log[k]["beta"]) > 1e-6 * log[k]["beta"]
        assert abs(hu - log[k]["beta"]) > 1e-6 * log[k]["beta"]
        checked += 1
    assert checked >= 20


@pytest.mark.parametrize("pc", [1, 3])
def test_pr_plus_ratio(orc, pc):
    P, _, _, _, log, tr = run(pc=pc, beta=1)
    checked = 0
    for k in range(1, len(log)):
        if log[k]["level"] != 0:
            continue
        y = tr[k]["r"] - tr[k - 1]["r"]
        lhs = log[k]["beta"] * S(tr[k - 1]["r"], tr[k - 1]["z"])
        rhs = S(y, tr[k]["z"])
        assert abs(lhs - rhs) <= 1e-12 * abs(rhs), k
        # PR+ is not the HS+ direction: conjugacy to y does not hold
        scale = abs(S(y, tr[k]["z"])) + log[k]["beta"] * abs(S(y, tr[k]["p_old"]))
        assert abs(S(y, tr[k]["d"])) > 1e-6 * scale, k
        checked += 1
    assert checked >= 20


def test_beta_is_clipped_at_zero(orc):
    """beta = max(ratio, 0): where the ratio is negative the step restarts with
    d = -z (level 1); where it is positive and the direction descends, beta is
    the ratio."""
    negatives = 0
    for kw in RUNS:
        _, opts, _, _, log, tr = run(**kw)
        for k in range(1, len(log)):      # no restart period falls inside these 40 steps
            num, den = raw_ratio(tr, k, kw["beta"])
            ratio = num / den if den > 0 else -np.inf
            if ratio < 0:
                negatives += 1
                assert log[k]["beta"] == 0.0 and log[k]["level"] == 1, (kw, k)
                assert np.array_equal(tr[k]["d"], -tr[k]["z"])
            elif log[k]["level"] == 0:
                assert abs(log[k]["beta"] - ratio) <= 1e-12 * ratio, (kw, k)
    assert negatives >= 5


def test_restart_period(orc):
    _, _, _, _, log, tr = run(pc=1, beta=0, restart_period=4, n_steps=25)
    for k, L in enumerate(log):
        if k % 4 == 0:
            assert L["beta"] == 0.0 and L["level"] >= 1 and np.array_equal(tr[k]["d"], -tr[k]["z"])
    assert sum(1 for L in log if L["beta"] > 0) >= 12
    _, _, _, _, log0, _ = run(pc=1, beta=2, n_steps=25)
    assert all(L["beta"] == 0.0 for L in log0)


def test_ascending_direction_restarts_with_beta_zero(orc):
    """Where the direction with a positive beta is not a descent direction
    (<r, p> >= 0), the step is taken with beta = 0 (Sec. IV.C; reading 20)."""
    found = 0
    for kw in RUNS:
        P, opts, _, _, log, tr = run(**kw)
        for k in range(1, len(log)):
            if log[k]["level"] != 1 or log[k]["path"] & 2 or k % 50 == 0:
                continue
            num, den = raw_ratio(tr, k, kw["beta"])
            if not (den > 0 and num / den > 0):
                continue
            pb = project(-tr[k]["z"] + (num / den) * tr[k]["p_old"], tr[k]["psi"])
            assert E1_of(pb, tr[k]["r"], P) >= 0.0, (kw, k)
            found += 1
    assert found >= 1


# ---------------------------------------------------------------- step
def test_model_step_minimises_the_quadratic_model(orc):
    checked = {"interior": 0, "clamped": 0, "fallback": 0}
    for kw in (dict(pc=1, beta=0), dict(pc=1, beta=0, theta_max=0.02),
               dict(scale=10.0, pc=1, beta=0, armijo_c1=C1)):
        P, opts, _, _, log, tr = run(**kw)
        theta_max = opts.get("theta_max", np.pi / 2)
        prev = None
        for k, L in enumerate(log):
            m = orc.model(GRID, P, tr[k]["psi"], tr[k]["p"])
            assert abs(m["E1"] - L["E1"]) <= 1e-12 * abs(m["E1"]) and abs(m["E2"] - L["E2"]) <= 1e-12 * abs(m["E2"])
            pmax = max(m["pnorm_1"], m["pnorm_2"])
            assert abs(L["pmax"] - pmax) <= 1e-14 * pmax
            a = L["alpha_model"]
            if L["E2"] > 0 and L["E1"] < 0:
                if a * pmax < theta_max * (1 - 1e-14):
                    # d/da (E0 + E1 a + E2 a^2 / 2) = 0
                    assert abs(L["E1"] + L["E2"] * a) <= 1e-13 * abs(L["E1"]), (kw, k)
                    checked["interior"] += 1
                else:
                    assert abs(a * pmax - theta_max) <= 1e-15 * theta_max and -L["E1"] / L["E2"] >= a
                    checked["clamped"] += 1
            else:
                want = (0.1 / pmax) if prev is None else prev
                assert a == min(want, theta_max / pmax), (kw, k)
                checked["fallback"] += 1
            prev = L["alpha"]
    assert all(v >= 1 for v in checked.values()), checked


@pytest.mark.parametrize("kw", [dict(pc=1, beta=0, max_backtrack=4), dict(pc=0, beta=0, max_backtrack=4),
                                dict(pc=1, beta=1, max_backtrack=4)], ids=["pc1-hs", "pc0-hs", "pc1-pr"])
def test_armijo_halving_along_the_exact_geodesic(orc, kw):
    P, opts, _, _, log, tr = run(scale=10.0, armijo_c1=C1, **kw)
    halved = 0
    for k, L in enumerate(log):
        psi, p, E0, E1, tau = tr[k]["psi"], tr[k]["p"], L["E0"], L["E1"], L["tau"]
        assert abs(E0 - energy(orc, P, psi)) <= 1e-13 * abs(E0)
        assert abs(tau - 1e-14 * abs(E0)) <= 1e-30
        h = L["halvings"]
        assert L["alpha"] == L["alpha_model"] * 0.5 ** h           # halving is exact in binary64
        # the accepted point is the geodesic point at alpha and carries the logged energy
        Ea = energy(orc, P, orc.geodesic(GRID, psi, p, L["alpha"]))
        assert abs(Ea - L["E"]) <= 1e-13 * abs(L["E"]), k
        Em = energy(orc, P, orc.geodesic(GRID, psi, p, L["alpha_model"]))
        if L["path"] & 1:
            assert h >= 1
            assert L["E"] <= E0 + C1 * L["alpha"] * E1 + tau, k       # sufficient decrease
            assert Em > E0 + tau, k                                   # the model step was rejected
            for j in range(1, h):
                a = L["alpha_model"] * 0.5 ** j
                Ej = energy(orc, P, orc.geodesic(GRID, psi, p, a))
                assert Ej > E0 + C1 * a * E1 + tau, (k, j)            # and so was every earlier halving
            halved += 1
        else:
            assert h == 0 and L["E"] <= E0 + tau, k
    assert halved >= 3


def _failed_line_search(orc, P, opts, psi, p, E0, alpha0):
    """True if the model step at alpha0 and every halving up to max_backtrack
    fail the acceptance tests along the geodesic of p."""
    m = orc.model(GRID, P, psi, p)
    tau = 1e-14 * abs(E0) if "tau_rel" not in opts else opts["tau_rel"] * abs(E0)
    c1 = opts.get("armijo_c1", 1e-4)
    if not energy(orc, P, orc.geodesic(GRID, psi, p, alpha0)) > E0 + tau:
        return False
    for j in range(1, opts["max_backtrack"] + 1):
        a = alpha0 * 0.5 ** j
        if not energy(orc, P, orc.geodesic(GRID, psi, p, a)) > E0 + c1 * a * m["E1"] + tau:
            return False
    return True


def _model_alpha(orc, P, opts, psi, p):
    m = orc.model(GRID, P, psi, p)
    pmax = max(m["pnorm_1"], m["pnorm_2"])
    assert m["E2"] > 0 and m["E1"] < 0
    return min(-m["E1"] / m["E2"], opts.get("theta_max", np.pi / 2) / pmax)


def test_beta_zero_retry_after_a_failed_line_search(orc):
    """A step whose line search fails with beta > 0 is retried with beta = 0
    (path bit 2); the direction with beta fails every trial."""
    P, opts, _, _, log, tr = run(scale=10.0, pc=1, beta=0, max_backtrack=1, armijo_c1=C1)
    found = 0
    for k, L in enumerate(log):
        if not L["path"] & 2:
            continue
        assert L["level"] == 1 and L["beta"] == 0.0 and L["restarted"] == 1
        num, den = raw_ratio(tr, k, 0)
        assert den > 0 and num / den > 0
        pb = project(-tr[k]["z"] + (num / den) * tr[k]["p_old"], tr[k]["psi"])
        assert E1_of(pb, tr[k]["r"], P) < 0          # it was a descent direction ...
        assert _failed_line_search(orc, P, opts, tr[k]["psi"], pb, L["E0"],
                                   _model_alpha(orc, P, opts, tr[k]["psi"], pb))   # ... whose search failed
        found += 1
    assert found >= 2


def test_stagnation(orc):
    """With a negative acceptance band the iteration stops (ESTAGNATED) at a
    state from which the beta = 0 direction fails every trial."""
    import oracle
    opts = {"tol_grad": 1e-10, "max_iter": 60, "pc": 1, "beta": 0, "max_backtrack": 2, "tau_rel": -1e-3}
    psi0 = inputs.initial_state(GRID, P_STRONG["omega"], 71, phase=True)
    psi, rep, log = oracle.solve(GRID, P_STRONG, psi0, opts, log_cap=60)
    assert rep["status"] == "ESTAGNATED" and 0 < rep["iters"] < 60
    # the returned state is the last accepted one; a fresh start there (beta = 0)
    # stagnates at once, and the steepest-descent search from it fails by hand
    _, rep1, _ = oracle.solve(GRID, P_STRONG, psi, dict(opts, max_iter=5))
    assert rep1["status"] == "ESTAGNATED" and rep1["iters"] == 0
    t, h, _, _ = orc.heval(GRID, P_STRONG, psi)
    r = np.stack([h[i] - t["mu"][i] * psi[i] for i in range(2)])
    p = project(-orc.precond(GRID, P_STRONG, 1, 1e-6, psi, r), psi)
    assert E1_of(p, r, P_STRONG) < 0
    assert _failed_line_search(orc, P_STRONG, opts, psi, p, t["E"], _model_alpha(orc, P_STRONG, opts, psi, p))


# ---------------------------------------------------------------- composite fallback
def test_composite_fallback_ladder(orc):
    """For the composite preconditioner (not symmetric, Eq. (18)), a direction
    that does not descend even with beta = 0 falls back to z = P_V^-1 r (level 2)
    and then to z = r (level 3), path bit 4.  A negative regularising shift makes
    the P_V diagonal indefinite near the centre, which reaches both levels."""
    P, opts, _, _, log, tr = run(phase=False, pc=3, beta=0, sigma=-60.0, n_steps=30)
    sig = opts["sigma"]
    levels = [L["level"] for L in log]
    assert 2 in levels and 3 in levels
    for k, L in enumerate(log):
        psi, r = tr[k]["psi"], tr[k]["r"]
        if L["level"] < 2:
            assert not L["path"] & 4
            continue
        assert L["path"] & 4 and L["beta"] == 0.0
        comp = project(-orc.precond(GRID, P, 3, sig, psi, r), psi)
        assert E1_of(comp, r, P) >= 0.0, k                 # the composite direction ascends
        zv = orc.precond(GRID, P, 1, sig, psi, r)
        if L["level"] == 2:
            assert relerr(tr[k]["z"], zv) < 1e-14
        else:
            assert E1_of(project(-zv, psi), r, P) >= 0.0   # so does P_V^-1 r
            assert np.array_equal(tr[k]["z"], r)
        assert np.array_equal(tr[k]["d"], -tr[k]["z"])


# ---------------------------------------------------------------- stall stop (not in the paper)
@pytest.mark.parametrize("scale,window", [(1.0, 3), (1.0, 6), (10.0, 4)])
def test_stall_stop_fires_at_the_first_step_its_definition_names(orc, scale, window):
    """stall_window W: the solve stops (ESTALLED) at the first step n where
    max_i ||r_i|| has not fallen below half of its reference value for W steps,
    the reference being the last value that halved the one before it (the
    first residual to start with).  Checked against the logged residuals."""
    import oracle
    P = _params(scale)
    psi0 = inputs.initial_state(GRID, P["omega"], 71, phase=True)
    _, rep, log = oracle.solve(GRID, P, psi0, {"tol_grad": 1e-10, "max_iter": 200, "stall_window": window},
                               log_cap=200)
    assert rep["status"] == "ESTALLED"
    res = [L["res_max"] for L in log] + [max(rep["final"]["res"])]   # residual at the start of steps 0..n
    ref, ref_it, stop = np.inf, 0, None
    for k, r in enumerate(res):
        if r < 0.5 * ref:
            ref, ref_it = r, k
        elif k - ref_it >= window:
            stop = k
            break
    assert stop == rep["iters"]
    # without the rule the same run goes on
    _, rep0, _ = oracle.solve(GRID, P, psi0, {"tol_grad": 1e-10, "max_iter": rep["iters"] + 5})
    assert rep0["status"] == "ENOTCONV" and rep0["iters"] == rep["iters"] + 5
