"""Write the stored oracle results used by the GPU parity tests.

Calls only the CPU oracle (oracle/) on the seeded inputs of
paper_2510_24543_amd/inputs.py.  Each file records the command that made it.
Run from the repository root:  python tests/golden/make_golden.py [name ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2510_24543_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_SAMPLES = 4096


def sample_indices(grid, seed=2024):
    rng = np.random.default_rng(seed)
    return [rng.integers(0, n, N_SAMPLES).tolist() for n in grid["n"]]


def converged(name, pc=1, tol=1e-10):
    c = inputs.CONFIGS[name]
    grid, params = c["grid"], c["params"]
    psi0 = inputs.config_state(name)
    t0 = time.time()
    psi, rep, log = oracle.solve(grid, params, psi0, {"tol_grad": tol, "pc": pc, "max_iter": 5000},
                                 log_cap=5000)
    idx = sample_indices(grid)
    n = np.abs(psi) ** 2
    # the densities at the densest point and the seeded samples
    peak = [np.unravel_index(np.argmax(n[i]), n[i].shape) for i in range(2)]
    out = {
        "what": f"oracle solve of workload {name}, P_V, HS+, tol_grad {tol}",
        "command": f"python tests/golden/make_golden.py {name}",
        "oracle_seconds": time.time() - t0,
        "status": rep["status"], "iters": rep["iters"], "final": rep["final"],
        "E_first10": [l["E"] for l in log[:10]],
        "sample_idx": idx,
        "n_samples": [n[i][tuple(idx)].tolist() for i in range(2)],
        "peak_idx": [[int(v) for v in p] for p in peak],
        "n_peak": [float(n[i][peak[i]]) for i in range(2)],
        "n_sum": [float(np.sum(n[i])) for i in range(2)],
    }
    path = os.path.join(HERE, f"{name.lower()}_oracle_solve.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, rep["status"], rep["iters"], rep["final"]["E"], f"{out['oracle_seconds']:.0f}s")


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["C2"]):
        converged(name)
