"""ctypes wrapper of the FP64 CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  Nothing in the GPU library imports
this package, and this package imports nothing from the GPU library.

Arrays are numpy ``complex128`` of shape ``(2, nx, ny, nz)`` (component, x, y,
z; z fastest) unless stated otherwise.  Every function validates shapes and
raises ``RuntimeError`` on a non-zero status of the C library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB_PATH loads another build of oracle.c instead (the mutation test of
# tests/test_oracle_mutations.py builds copies with planted mistakes).
_LIB_PATH = os.environ.get("ORACLE_LIB_PATH") or os.path.join(_HERE, "liboracle.so")
_SRC_PATH = os.path.join(_HERE, "oracle.c")

STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 4: "ENOTCONV", 5: "ESTAGNATED", 6: "ENONFINITE", 8: "ESTALLED"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               _SRC_PATH, "-o", _LIB_PATH, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class Params(C.Structure):
    _fields_ = [("N", C.c_double * 2), ("omega", C.c_double * 3),
                ("G", (C.c_double * 2) * 2), ("Gdd", (C.c_double * 2) * 2),
                ("c_lhy", C.c_double), ("r_cut", C.c_double), ("n_u", C.c_int32), ("dip_cut", C.c_int32),
                ("lhy_quad", C.c_int32)]


class Terms(C.Structure):
    _fields_ = [("E", C.c_double), ("E_kin", C.c_double * 2), ("E_trap", C.c_double * 2),
                ("E_c", (C.c_double * 2) * 2), ("E_dd", (C.c_double * 2) * 2),
                ("E_lhy", C.c_double), ("mu", C.c_double * 2), ("shift", C.c_double * 2),
                ("res", C.c_double * 2), ("norm2", C.c_double * 2)]

    def to_dict(self) -> dict:
        return {
            "E": self.E, "E_kin": list(self.E_kin), "E_trap": list(self.E_trap),
            "E_c": [list(r) for r in self.E_c], "E_dd": [list(r) for r in self.E_dd],
            "E_lhy": self.E_lhy, "mu": list(self.mu), "shift": list(self.shift),
            "res": list(self.res), "norm2": list(self.norm2),
        }


class Opts(C.Structure):
    _fields_ = [("pc", C.c_int32), ("beta", C.c_int32), ("max_iter", C.c_int32),
                ("restart_period", C.c_int32), ("max_backtrack", C.c_int32), ("stall_window", C.c_int32),
                ("tol_grad", C.c_double), ("tol_dE", C.c_double), ("sigma", C.c_double),
                ("armijo_c1", C.c_double), ("theta_max", C.c_double), ("tau_rel", C.c_double),
                ("blend", C.c_double)]


class Iter(C.Structure):
    _fields_ = [("iter", C.c_int32), ("n_trials", C.c_int32), ("restarted", C.c_int32),
                ("path", C.c_int32), ("E", C.c_double), ("res_max", C.c_double),
                ("E1", C.c_double), ("E2", C.c_double), ("alpha", C.c_double),
                ("beta", C.c_double), ("level", C.c_int32), ("halvings", C.c_int32),
                ("beta_num", C.c_double), ("beta_den", C.c_double), ("rp", C.c_double),
                ("alpha_model", C.c_double), ("pmax", C.c_double), ("E0", C.c_double),
                ("tau", C.c_double)]


class IteOpts(C.Structure):
    _fields_ = [("dt", C.c_double), ("tol_dE", C.c_double), ("max_iter", C.c_int32), ("pad", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("n_restarts", C.c_int32), ("n_backtracks", C.c_int32),
                ("status", C.c_int32), ("final", Terms)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_fft3d.argtypes = [C.POINTER(C.c_int32), dp, C.c_int32, C.c_int32]
        L.orc_gauss_legendre.argtypes = [C.c_int32, dp, dp]
        L.orc_lhy_point.argtypes = [C.POINTER(Params), C.c_double, C.c_double, dp]
        L.orc_lhy_point.restype = None
        L.orc_lhy_nodes.argtypes = [C.POINTER(Params), dp, dp, C.c_int32]
        L.orc_heval.argtypes = [C.POINTER(Grid), C.POINTER(Params), dp, dp, dp, dp, C.POINTER(Terms)]
        L.orc_precond.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.c_int32, C.c_double, C.c_double, dp, dp, dp]
        L.orc_model.argtypes = [C.POINTER(Grid), C.POINTER(Params), dp, dp, dp]
        L.orc_geodesic.argtypes = [C.POINTER(Grid), dp, dp, C.c_double, dp]
        L.orc_param_grad.argtypes = [C.POINTER(Grid), C.POINTER(Params), dp, dp]
        L.orc_solve.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.POINTER(Opts), dp,
                                C.POINTER(Report), C.POINTER(Iter), C.c_int32]
        L.orc_solve_trace.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.POINTER(Opts), dp,
                                      C.POINTER(Report), C.POINTER(Iter), C.c_int32, dp, C.c_int32]
        L.orc_ite.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.POINTER(IteOpts), dp,
                              C.POINTER(Report), dp, C.c_int32]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(st: int, what: str):
    if st != 0:
        raise RuntimeError(f"oracle {what} failed: {STATUS.get(st, st)}")


def make_grid(n, lo, hi) -> Grid:
    g = Grid()
    for d in range(3):
        g.n[d] = int(n[d]); g.lo[d] = float(lo[d]); g.hi[d] = float(hi[d])
    return g


def make_params(p: dict) -> Params:
    P = Params()
    for i in range(2):
        P.N[i] = float(p["N"][i])
        for j in range(2):
            P.G[i][j] = float(p["G"][i][j])
            P.Gdd[i][j] = float(p["Gdd"][i][j])
    for d in range(3):
        P.omega[d] = float(p["omega"][d])
    P.c_lhy = float(p["c_lhy"]); P.r_cut = float(p["r_cut"]); P.n_u = int(p["n_u"])
    P.dip_cut = int(p.get("dip_cut", 0))
    P.lhy_quad = int(p.get("lhy_quad", 0))
    return P


def make_opts(o: dict) -> Opts:
    O = Opts()
    for k, _ in Opts._fields_:
        if k in o:
            setattr(O, k, o[k])
    return O


def _field(psi, n):
    a = np.ascontiguousarray(psi, dtype=np.complex128)
    if a.shape != (2, n[0], n[1], n[2]):
        raise ValueError(f"expected shape (2,{n[0]},{n[1]},{n[2]}), got {a.shape}")
    return a


def fft3d(a: np.ndarray, sign: int = -1) -> np.ndarray:
    """3D DFT over the last three axes (sign -1 forward unnormalised, +1 inverse /N)."""
    a = np.ascontiguousarray(a, dtype=np.complex128).copy()
    shp = a.shape[-3:]
    nf = int(np.prod(a.shape[:-3])) if a.ndim > 3 else 1
    n = (C.c_int32 * 3)(*shp)
    _check(lib().orc_fft3d(n, _dp(a), nf, sign), "fft3d")
    return a


def gauss_legendre(n: int):
    u = np.zeros(n); w = np.zeros(n)
    _check(lib().orc_gauss_legendre(n, _dp(u), _dp(w)), "gauss_legendre")
    return u, w


def lhy_nodes(params: dict):
    """(u, w): the oracle's rule for the u integral of the LHY term."""
    u = np.zeros(512); w = np.zeros(512)
    n = lib().orc_lhy_nodes(C.byref(make_params(params)), _dp(u), _dp(w), 512)
    if n < 0:
        raise RuntimeError("oracle lhy_nodes: more than 512 nodes")
    return u[:n], w[:n]


def lhy_point(params: dict, n1: float, n2: float):
    """(e, de/dn1, de/dn2) of the LHY energy density at one point."""
    out = np.zeros(3)
    lib().orc_lhy_point(C.byref(make_params(params)), n1, n2, _dp(out))
    return out


def heval(grid: dict, params: dict, psi: np.ndarray):
    """Energy terms and H_i psi_i, Phi_j, muLHY_i of Sec. II."""
    g = make_grid(grid["n"], grid["lo"], grid["hi"])
    psi = _field(psi, grid["n"])
    h = np.zeros_like(psi)
    phi = np.zeros(psi.shape, dtype=np.float64)
    mul = np.zeros(psi.shape, dtype=np.float64)
    t = Terms()
    _check(lib().orc_heval(C.byref(g), C.byref(make_params(params)), _dp(psi), _dp(h),
                           _dp(phi), _dp(mul), C.byref(t)), "heval")
    return t.to_dict(), h, phi, mul


def precond(grid: dict, params: dict, mode: int, sigma: float, psi: np.ndarray, r: np.ndarray,
            blend: float = -1.0):
    """z = P^-1 r (mode 0 none, 1 P_V, 2 P_Delta, 3 composite, 4 symmetrised,
    5 blend with weight `blend` of P_V, < 0 adaptive) at the state psi."""
    g = make_grid(grid["n"], grid["lo"], grid["hi"])
    psi = _field(psi, grid["n"]); r = _field(r, grid["n"])
    z = np.zeros_like(psi)
    _check(lib().orc_precond(C.byref(g), C.byref(make_params(params)), mode, sigma, blend, _dp(psi),
                             _dp(r), _dp(z)), "precond")
    return z


MODEL_KEYS = ["E1p_1", "E1p_2", "E1_lhy", "E2_11", "E2_12", "E2_21", "E2_22", "E2_lhy",
              "E1", "E2", "pnorm_1", "pnorm_2"]


def model(grid: dict, params: dict, psi: np.ndarray, p: np.ndarray) -> dict:
    """Coefficients of the second-order energy model along the geodesic (Sec. V)."""
    g = make_grid(grid["n"], grid["lo"], grid["hi"])
    psi = _field(psi, grid["n"]); p = _field(p, grid["n"])
    out = np.zeros(14)
    _check(lib().orc_model(C.byref(g), C.byref(make_params(params)), _dp(psi), _dp(p), _dp(out)),
           "model")
    return dict(zip(MODEL_KEYS, out[:12].tolist()))


def geodesic(grid: dict, psi: np.ndarray, p: np.ndarray, alpha: float) -> np.ndarray:
    g = make_grid(grid["n"], grid["lo"], grid["hi"])
    psi = _field(psi, grid["n"]); p = _field(p, grid["n"])
    out = np.zeros_like(psi)
    _check(lib().orc_geodesic(C.byref(g), _dp(psi), _dp(p), alpha, _dp(out)), "geodesic")
    return out


def param_grad(grid: dict, params: dict, psi: np.ndarray) -> dict:
    """dE/dG_ij, dE/dGdd_ij (entries independent) and dE/dc_lhy at fixed psi."""
    g = make_grid(grid["n"], grid["lo"], grid["hi"])
    psi = _field(psi, grid["n"])
    out = np.zeros(9)
    _check(lib().orc_param_grad(C.byref(g), C.byref(make_params(params)), _dp(psi), _dp(out)),
           "param_grad")
    return {"dG": out[0:4].reshape(2, 2), "dGdd": out[4:8].reshape(2, 2), "dc_lhy": out[8]}


DEFAULT_OPTS = dict(pc=1, beta=0, max_iter=2000, restart_period=50, max_backtrack=30,
                    tol_grad=1e-10, tol_dE=0.0, sigma=1e-6, armijo_c1=1e-4,
                    theta_max=np.pi / 2, tau_rel=1e-14, blend=-1.0)


def solve(grid: dict, params: dict, psi0: np.ndarray, opts: dict | None = None, log_cap: int = 0):
    """Run the preconditioned nonlinear CG iteration; returns (psi, report, log)."""
    o = dict(DEFAULT_OPTS)
    o.update(opts or {})
    g = make_grid(grid["n"], grid["lo"], grid["hi"])
    psi = _field(psi0, grid["n"]).copy()
    rep = Report()
    logs = (Iter * max(log_cap, 1))()
    lib().orc_solve(C.byref(g), C.byref(make_params(params)), C.byref(make_opts(o)), _dp(psi),
                    C.byref(rep), logs, log_cap)
    out = {"iters": rep.iters, "n_restarts": rep.n_restarts, "n_backtracks": rep.n_backtracks,
           "status": STATUS.get(rep.status, rep.status), "final": rep.final.to_dict()}
    n_log = min(rep.iters, log_cap)
    log = [{k: getattr(logs[i], k) for k, _ in Iter._fields_} for i in range(n_log)]
    return psi, out, log


TRACE_FIELDS = ("psi", "r", "z", "p_old", "d", "p")


def solve_traced(grid: dict, params: dict, psi0: np.ndarray, opts: dict | None = None,
                 n_steps: int = 20):
    """solve() that also returns, for each of the first n_steps accepted steps,
    the fields psi (start of the step), r, z (the preconditioned residual the
    accepted direction used), p_old, d (unprojected direction) and p (projected),
    each of shape (2, nx, ny, nz): trace[k][name]."""
    o = dict(DEFAULT_OPTS)
    o.update(opts or {})
    g = make_grid(grid["n"], grid["lo"], grid["hi"])
    psi = _field(psi0, grid["n"]).copy()
    n = grid["n"]
    tr = np.zeros((max(n_steps, 1), len(TRACE_FIELDS), 2, n[0], n[1], n[2]), dtype=np.complex128)
    rep = Report()
    logs = (Iter * max(n_steps, 1))()
    lib().orc_solve_trace(C.byref(g), C.byref(make_params(params)), C.byref(make_opts(o)), _dp(psi),
                          C.byref(rep), logs, n_steps, _dp(tr), n_steps)
    out = {"iters": rep.iters, "n_restarts": rep.n_restarts, "n_backtracks": rep.n_backtracks,
           "status": STATUS.get(rep.status, rep.status), "final": rep.final.to_dict()}
    n_log = min(rep.iters, n_steps)
    log = [{k: getattr(logs[i], k) for k, _ in Iter._fields_} for i in range(n_log)]
    trace = [{name: tr[k, f] for f, name in enumerate(TRACE_FIELDS)} for k in range(n_log)]
    return psi, out, log, trace


def ite(grid: dict, params: dict, psi0: np.ndarray, dt: float, tol_dE: float = 1e-6, max_iter: int = 100000,
        log_cap: int = 0):
    """Imaginary-time evolution (normalised first-order time splitting) from
    psi0; returns (psi, report, energies of the iterates psi^0, psi^1, ...)."""
    g = make_grid(grid["n"], grid["lo"], grid["hi"])
    psi = _field(psi0, grid["n"]).copy()
    rep = Report()
    logE = np.zeros(max(log_cap, 1))
    st = lib().orc_ite(C.byref(g), C.byref(make_params(params)),
                       C.byref(IteOpts(dt=dt, tol_dE=tol_dE, max_iter=max_iter, pad=0)), _dp(psi),
                       C.byref(rep), _dp(logE), log_cap)
    if st == 1:
        raise RuntimeError("oracle ite: invalid input")
    out = {"iters": rep.iters, "status": STATUS.get(rep.status, rep.status), "final": rep.final.to_dict()}
    return psi, out, logE[:min(rep.iters + 1, log_cap)]
