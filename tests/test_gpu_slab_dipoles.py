"""The slab-cut dipolar kernel (bec_params.dip_cut = 1: the interaction kept for
|z - z'| < r_cut, x and y periodic and not cut) on the GPU against the oracle:
energy terms, H psi, the line-search model, solver steps, the batched solver,
and the 2 r_cut <= L_z rule.  Bars as in test_gpu_parity."""
import numpy as np
import pytest

from paper_2510_24543_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def solver():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2510_24543_amd import solver as s
    return s


def params(r_cut, **kw):
    p = {"N": [1.0, 1.6], "omega": [0.0, 0.0, 2.0], "G": [[100.0, 50.0], [31.25, 90.0]],
         "Gdd": [[60.0, -45.0], [-28.125, 50.0]], "c_lhy": 5.0, "r_cut": r_cut, "n_u": 16, "dip_cut": 1}
    p.update(kw)
    return p


GRID = {"n": [32, 32, 48], "lo": [-8.0, -8.0, -6.0], "hi": [8.0, 8.0, 6.0]}


def state(grid, seed, phase=True):
    # an in-plane pattern (a periodic sheet, not a cloud) over a Gaussian in z
    x, y, z = inputs.coords(grid)
    X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
    L = [grid["hi"][d] - grid["lo"][d] for d in range(3)]
    base = inputs.initial_state(grid, [0.0, 0.0, 2.0], seed, phase=phase)
    mod = [1.0 + 0.5 * np.cos(2 * np.pi * X / L[0]) * np.cos(4 * np.pi * Y / L[1]),
           1.0 - 0.4 * np.sin(2 * np.pi * (X + Y) / L[0])]
    psi = np.stack([base[i] * mod[i] for i in range(2)])
    dV = np.prod([L[d] / grid["n"][d] for d in range(3)])
    for i in range(2):
        psi[i] /= np.sqrt(dV * np.sum(np.abs(psi[i]) ** 2))
    return psi


@pytest.mark.parametrize("r_cut", [6.0, 2.5, 0.75])
def test_slab_energy_hamiltonian_and_model(solver, orc, r_cut):
    p = params(r_cut)
    psi = state(GRID, 41)
    ctx = solver.Context(GRID, p)
    h, t = ctx.hamiltonian(torch.from_numpy(psi))
    to, ho, _, _ = orc.heval(GRID, p, psi)
    for k in ("E", "E_lhy"):
        assert abs(t[k] - to[k]) <= 1e-12 * abs(to["E"]), k
    for i in range(2):
        for j in range(2):
            assert abs(t["E_dd"][i][j] - to["E_dd"][i][j]) <= 1e-12 * abs(to["E"]), (i, j)
        for k in ("mu", "shift", "res"):
            assert abs(t[k][i] - to[k][i]) <= 1e-12 * abs(to[k][i]), (k, i)
    assert np.max(np.abs(h.cpu().numpy() - ho)) <= 1e-11 * np.max(np.abs(ho))
    dV = float(np.prod([(GRID["hi"][d] - GRID["lo"][d]) / GRID["n"][d] for d in range(3)]))
    r = np.stack([ho[i] - to["mu"][i] * psi[i] for i in range(2)])
    d = -r + 0.01 * np.max(np.abs(r)) * inputs.random_field(GRID, 43)
    _, rep = ctx.linesearch(torch.from_numpy(psi), torch.from_numpy(d), {"max_backtrack": 30})
    pr = np.stack([d[i] - dV * np.sum(np.real(np.conj(d[i]) * psi[i])) * psi[i] for i in range(2)])
    m = orc.model(GRID, p, psi, pr)
    assert abs(rep["E1"] - m["E1"]) <= 1e-10 * abs(m["E1"])
    assert abs(rep["E2"] - m["E2"]) <= 1e-10 * abs(m["E2"])


def test_slab_solver_steps(solver, orc):
    p = params(6.0)
    psi0 = state(GRID, 45, phase=False)
    opts = {"tol_grad": 1e-10, "pc": 1, "max_iter": 10}
    ctx = solver.Context(GRID, p)
    _, rep, log = ctx.solve(torch.from_numpy(psi0), opts, log_cap=10)
    _, repo, logo = orc.solve(GRID, p, psi0, opts, log_cap=10)
    assert rep["iters"] == repo["iters"] == 10
    for a, b in zip(log, logo):
        assert a["path"] == b["path"] and a["n_trials"] == b["n_trials"]
        assert abs(a["E"] - b["E"]) <= 1e-11 * abs(b["E"])
        assert abs(a["alpha"] - b["alpha"]) <= 1e-8 * abs(b["alpha"])


def test_slab_in_the_batched_solver(solver, orc):
    """A batch holding a slab-cut and a spherically cut instance of the same grid."""
    grid = {"n": [16, 16, 32], "lo": [-6.0, -6.0, -6.0], "hi": [6.0, 6.0, 6.0]}
    ps = [params(6.0), params(4.0, dip_cut=0, omega=[1.0, 1.0, 2.0])]
    psi0 = [state(grid, 47 + k, phase=False) for k in range(2)]
    opts = {"tol_grad": 1e-10, "pc": 1, "max_iter": 5}
    b = solver.Batch([grid, grid], ps)
    _, reps = b.solve(psi0, opts, rounds_per_sync=2)
    for p, p0, rb in zip(ps, psi0, reps):
        _, repo, _ = orc.solve(grid, p, p0, opts)
        assert rb["iters"] == repo["iters"] == 5
        assert abs(rb["final"]["E"] - repo["final"]["E"]) <= 1e-11 * abs(repo["final"]["E"])


def test_slab_cut_longer_than_half_the_box_is_refused(solver):
    with pytest.raises(solver.B.BecError, match="EINVAL"):
        solver.Context(GRID, params(6.5))
