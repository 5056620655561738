"""Seeded synthetic inputs shared by the GPU path and the CPU oracle.

This module holds no arithmetic of the method: it defines the workload
configurations (grids, boxes, couplings) and the seeded initial states.  It
imports nothing from the rest of the package, so the oracle-side tests can use
it without touching the GPU library.

Initial state (the paper's Gaussian starts with weak seeded noise, Sec. VI.A):
    psi_i^0(x) ~ exp(-1/2 sum_d omega_d (x_d - c_{i,d})^2) (1 + 0.1 U_i(x)),
    c_1 = (+1, 0, 0), c_2 = (-1, 0, 0), each component normalised to one.
U_i(x) in [-1, 1) comes from a counter-based SplitMix64 stream:
    U = 2 * (mix(seed + (i*Npts + idx + 1) * 0x9E3779B97F4A7C15) >> 11) * 2^-53 - 1,
with mix the SplitMix64 finaliser (xor-shift 30, *0xBF58476D1CE4E5B9, xor-shift
27, *0x94D049BB133111EB, xor-shift 31) and idx the C-order point index.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform_stream(seed: int, counters: np.ndarray) -> np.ndarray:
    """U(-1,1) values for integer counters (counter 0 is never used by init)."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + c * _GOLDEN
    v = splitmix64_mix(z) >> np.uint64(11)
    return 2.0 * v.astype(np.float64) * (2.0 ** -53) - 1.0


def unit_stream(seed: int, counters: np.ndarray) -> np.ndarray:
    """U[0,1) values for integer counters."""
    return 0.5 * (uniform_stream(seed, counters) + 1.0)


def coords(grid: dict):
    n, lo, hi = grid["n"], grid["lo"], grid["hi"]
    return [lo[d] + (hi[d] - lo[d]) / n[d] * np.arange(n[d]) for d in range(3)]


def initial_state(grid: dict, omega, seed: int, noise: float = 0.1,
                  centers=((1.0, 0.0, 0.0), (-1.0, 0.0, 0.0)), phase: bool = False) -> np.ndarray:
    """Seeded initial state, complex128 of shape (2, nx, ny, nz), unit norm per component.

    ``phase=True`` multiplies each component by a seeded random phase
    exp(i pi U'), giving a genuinely complex field for parity tests.
    """
    n = grid["n"]
    npts = int(n[0]) * int(n[1]) * int(n[2])
    x, y, z = coords(grid)
    X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
    dV = np.prod([(grid["hi"][d] - grid["lo"][d]) / n[d] for d in range(3)])
    out = np.empty((2, n[0], n[1], n[2]), dtype=np.complex128)
    idx = np.arange(npts, dtype=np.uint64)
    for i in range(2):
        c = centers[i]
        g = np.exp(-0.5 * (omega[0] * (X - c[0]) ** 2 + omega[1] * (Y - c[1]) ** 2
                           + omega[2] * (Z - c[2]) ** 2))
        u = uniform_stream(seed, np.uint64(i * npts) + idx + np.uint64(1)).reshape(n)
        f = g * (1.0 + noise * u)
        if phase:
            ph = uniform_stream(seed + 7919, np.uint64(i * npts) + idx + np.uint64(1)).reshape(n)
            f = f * np.exp(1j * np.pi * ph)
        f = f.astype(np.complex128)
        f /= np.sqrt(dV * np.sum(np.abs(f) ** 2))
        out[i] = f
    return out


def random_field(grid: dict, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded complex field with i.i.d. U(-1,1) real and imaginary parts."""
    n = grid["n"]
    npts = int(n[0]) * int(n[1]) * int(n[2])
    idx = np.arange(2 * 2 * npts, dtype=np.uint64) + np.uint64(1)
    u = uniform_stream(seed, idx)
    re = u[: 2 * npts].reshape(2, *n)
    im = u[2 * npts:].reshape(2, *n)
    return scale * (re + 1j * im)


def _params(N=(1.0, 1.0), omega=(1.0, 1.0, 1.0), G=(100.0, 100.0, 50.0), Gdd=(60.0, 60.0, 60.0),
            c_lhy=0.0, r_cut=8.0, n_u=16) -> dict:
    g11, g22, g12 = G
    d11, d22, d12 = Gdd
    return {"N": list(N), "omega": list(omega), "G": [[g11, g12], [g12, g22]],
            "Gdd": [[d11, d12], [d12, d22]], "c_lhy": c_lhy, "r_cut": r_cut, "n_u": n_u}


def _grid(n, lo, hi) -> dict:
    return {"n": list(n), "lo": list(lo), "hi": list(hi)}


# Workload configurations (paper-scale synthetic parameter sets, harmonic-oscillator units).
CONFIGS = {
    # 32^3, box [-8,8)^3, trap (1,1,2.6), g11=g22=100, g12=50, gdd=60 all pairs, Rc=8
    "C1a": {"grid": _grid((32, 32, 32), (-8, -8, -8), (8, 8, 8)),
            "params": _params(omega=(1, 1, 2.6), c_lhy=0.0), "seed": 1001},
    "C1b": {"grid": _grid((32, 32, 32), (-8, -8, -8), (8, 8, 8)),
            "params": _params(omega=(1, 1, 2.6), c_lhy=5.0), "seed": 1001},
    # droplet regime, 64^3 on [-12,12)^3
    "C2": {"grid": _grid((64, 64, 64), (-12, -12, -12), (12, 12, 12)),
           "params": _params(omega=(1, 1, 3), G=(80, 80, 40), Gdd=(150, 75, 105), c_lhy=8.0,
                             r_cut=12.0), "seed": 1002},
    # headline workload: 128^3 x 2 components, C1 physics with LHY 5
    "M": {"grid": _grid((128, 128, 128), (-8, -8, -8), (8, 8, 8)),
          "params": _params(omega=(1, 1, 2.6), c_lhy=5.0), "seed": 1006},
    # stripe / supersolid regime, 128 x 128 x 96, elongated trap
    "C3": {"grid": _grid((128, 128, 96), (-16, -8, -8), (16, 8, 8)),
           "params": _params(omega=(0.3, 1, 2), G=(60, 60, 70), Gdd=(78, 78, 91), c_lhy=6.0,
                             r_cut=8.0), "seed": 1003},
    # large supersolid lattice 256 x 256 x 128
    "C5": {"grid": _grid((256, 256, 128), (-24, -24, -12), (24, 24, 12)),
           "params": _params(omega=(0.5, 0.5, 1.5), G=(50, 50, 45), Gdd=(140, 140, 140),
                             c_lhy=7.0, r_cut=12.0), "seed": 1005},
}


def scan_instances(n_inst: int = 96, seed: int = 4242):
    """Parameter scan: grids cycle 48^3, 64^3, 96^3; g12 ~ U(20,90), gdd ~ U(50,160)
    (all pairs), c_lhy ~ U(2,10); box [-12,12)^3, trap (1,1,3), g11 = g22 = 80."""
    sizes = (48, 64, 96)
    out = []
    for k in range(n_inst):
        u = unit_stream(seed, np.arange(3 * k + 1, 3 * k + 4, dtype=np.uint64))
        g12 = 20.0 + 70.0 * u[0]
        gdd = 50.0 + 110.0 * u[1]
        c = 2.0 + 8.0 * u[2]
        n = sizes[k % 3]
        out.append({"grid": _grid((n, n, n), (-12, -12, -12), (12, 12, 12)),
                    "params": _params(omega=(1, 1, 3), G=(80, 80, g12), Gdd=(gdd, gdd, gdd),
                                      c_lhy=c, r_cut=12.0),
                    "seed": 4000 + k})
    return out


def config_state(name: str, phase: bool = False) -> np.ndarray:
    c = CONFIGS[name]
    return initial_state(c["grid"], c["params"]["omega"], c["seed"], phase=phase)
