"""bec_gradient_noalloc (the context-free gradient whose workspace is the
library's fixed device array) against bec_gradient of a context, through the
C ABI: two calls in a row on the same device, the second on a smaller grid,
both projected and not; and the size limit, refused on the host."""
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


def params(**kw):
    p = {"N": [1.0, 1.6], "omega": [1.0, 1.2, 2.6], "G": [[100.0, 50.0], [31.25, 90.0]],
         "Gdd": [[60.0, 45.0], [28.125, 50.0]], "c_lhy": 5.0, "r_cut": 6.0, "n_u": 16}
    p.update(kw)
    return p


CASES = [({"n": [48, 32, 32], "lo": [-8.0, -6.0, -6.0], "hi": [8.0, 6.0, 6.0]}, params()),
         ({"n": [16, 16, 32], "lo": [-6.0, -6.0, -6.0], "hi": [6.0, 6.0, 6.0]},
          params(N=[1.0, 1.0], G=[[80.0, 40.0], [40.0, 80.0]], Gdd=[[150.0, 105.0], [105.0, 75.0]], c_lhy=8.0))]


def test_noalloc_gradient_matches_context_gradient_twice(solver):
    for k, (grid, p) in enumerate(CASES):                   # the second call is on a smaller grid
        psi = torch.from_numpy(inputs.initial_state(grid, p["omega"], 31 + k, phase=True)).cuda()
        ctx = solver.Context(grid, p)
        for projected in (False, True):
            print(f"grid {grid['n']} projected {projected}", flush=True)
            g_ref, t_ref = ctx.gradient(psi, projected)
            g, t = solver.gradient_noalloc(grid, p, psi, projected)
            torch.cuda.synchronize()
            a, b = g.cpu().numpy(), g_ref.cpu().numpy()
            assert np.max(np.abs(a - b)) <= 1e-11 * np.max(np.abs(b))
            for key in ("E", "E_lhy"):
                assert abs(t[key] - t_ref[key]) <= 1e-12 * abs(t_ref["E"]), key
            for key in ("mu", "shift", "res", "norm2"):
                for i in range(2):
                    assert abs(t[key][i] - t_ref[key][i]) <= 1e-12 * abs(t_ref[key][i]), (key, i)
        ctx.close()


def test_noalloc_refuses_grids_beyond_its_array(solver):
    grid = {"n": [64, 64, 64], "lo": [-6.0] * 3, "hi": [6.0] * 3}
    psi = torch.zeros((2, 64, 64, 64), dtype=torch.complex128, device="cuda")
    with pytest.raises(solver.B.BecError, match="ENOMEM"):
        solver.gradient_noalloc(grid, params(), psi)
