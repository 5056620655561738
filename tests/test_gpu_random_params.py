"""Parity of the HIP path with the oracle on seeded random parameter sets.

Random grids (supported axis lengths up to 48), boxes, atom numbers, traps,
contact and dipolar couplings of either sign (symmetric N_i G_ij), LHY on or off
and 1 to 24 quadrature nodes, so that the LHY nodes fall into every class and the
class-A Chebyshev table is built on some sets and refused or empty on others;
cutoff radii from 0.5 to 10, so that on some sets the lowest modes take the
dipolar cutoff factor c(q) from its series (q = |k| R_c < 1).
Bars as in test_gpu_parity: energy terms 1e-12 of the energy scale, H psi 1e-11
in max norm, line-search model 1e-10.
"""
import numpy as np
import pytest

from paper_2510_24543_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LENGTHS = [8, 16, 32, 48]


def random_case(seed):
    rng = np.random.default_rng(1000 + seed)
    n = [int(rng.choice(LENGTHS)) for _ in range(3)]
    half = rng.uniform(4.0, 9.0, 3)
    N = rng.uniform(0.5, 2.0, 2)
    G12 = rng.uniform(-30.0, 120.0)
    Gdd12 = rng.uniform(-50.0, 150.0)
    params = {
        "N": [float(N[0]), float(N[1])],
        "omega": [float(x) for x in rng.uniform(0.5, 3.0, 3)],
        "G": [[float(rng.uniform(-20.0, 150.0)), float(G12)], [float(N[0] * G12 / N[1]), float(rng.uniform(-20.0, 150.0))]],
        "Gdd": [[float(rng.uniform(-50.0, 200.0)), float(Gdd12)],
                [float(N[0] * Gdd12 / N[1]), float(rng.uniform(-50.0, 200.0))]],
        "c_lhy": 0.0 if rng.uniform() < 0.2 else float(rng.uniform(0.5, 10.0)),
        "r_cut": float(rng.uniform(0.5, 10.0)),
        "n_u": int(rng.choice([1, 5, 16, 24])),
    }
    grid = {"n": n, "lo": [float(-h) for h in half], "hi": [float(h) for h in half]}
    return grid, params


SEEDS = list(range(16))


@pytest.fixture(scope="module")
def solver():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2510_24543_amd import solver as s
    return s


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("seed", SEEDS)
def test_random_parameters_energy_hamiltonian_model(solver, orc, seed):
    grid, params = random_case(seed)
    print(f"seed {seed}: grid {grid['n']} n_u {params['n_u']} c_lhy {params['c_lhy']:.3g}", flush=True)
    psi = inputs.initial_state(grid, params["omega"], 500 + seed, phase=True)
    ctx = solver.Context(grid, params)
    print(f"  LHY table terms {ctx.get_tuning()['lhy_terms']}", flush=True)
    h, t = ctx.hamiltonian(torch.from_numpy(psi))
    to, ho, _, _ = orc.heval(grid, params, psi)
    scale = abs(to["E_kin"][0]) + abs(to["E_kin"][1]) + abs(to["E_trap"][0]) + abs(to["E_trap"][1]) + \
        sum(abs(to[k][i][j]) for k in ("E_c", "E_dd") for i in range(2) for j in range(2)) + abs(to["E_lhy"])
    for k in ("E", "E_lhy"):
        assert abs(t[k] - to[k]) <= 1e-12 * scale, k
    for k in ("mu", "shift"):
        for i in range(2):
            assert abs(t[k][i] - to[k][i]) <= 1e-11 * scale / params["N"][i], (k, i)
    assert _rel(h.cpu().numpy(), ho) < 1e-11
    # the state is normalised per component; a direction near minus the residual
    dV = float(np.prod([(grid["hi"][a] - grid["lo"][a]) / grid["n"][a] for a in range(3)]))
    r = np.stack([ho[i] - to["mu"][i] * psi[i] for i in range(2)])
    d = -r + 0.01 * inputs.random_field(grid, 600 + seed)
    _, rep = ctx.linesearch(torch.from_numpy(psi), torch.from_numpy(d), {"max_backtrack": 30})
    p = np.stack([d[i] - dV * np.sum(np.real(np.conj(d[i]) * psi[i])) * psi[i] for i in range(2)])
    m = orc.model(grid, params, psi, p)
    assert abs(rep["E1"] - m["E1"]) <= 1e-10 * abs(m["E1"])
    assert abs(rep["E2"] - m["E2"]) <= 1e-10 * max(abs(m["E2"]), 1e-10 * abs(m["E1"]))
