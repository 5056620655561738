"""ctypes declarations of the C ABI in include/bec.h (argument marshalling only).

The shared library must have been built in-tree (``__graft_entry__.build()``);
loading fails loudly otherwise -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libbecpcg.so")

STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "ENOTCONV", 5: "ESTAGNATED",
          6: "ENONFINITE", 7: "EUNSUPPORTED", 8: "ESTALLED"}


class BecError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class Params(C.Structure):
    _fields_ = [("N", C.c_double * 2), ("omega", C.c_double * 3),
                ("G", (C.c_double * 2) * 2), ("Gdd", (C.c_double * 2) * 2),
                ("c_lhy", C.c_double), ("r_cut", C.c_double), ("n_u", C.c_int32), ("dip_cut", C.c_int32),
                ("lhy_quad", C.c_int32)]

    def to_dict(self) -> dict:
        return {"N": list(self.N), "omega": list(self.omega), "G": [list(r) for r in self.G],
                "Gdd": [list(r) for r in self.Gdd], "c_lhy": self.c_lhy, "r_cut": self.r_cut, "n_u": self.n_u,
                "dip_cut": self.dip_cut, "lhy_quad": self.lhy_quad}


class Opts(C.Structure):
    _fields_ = [("pc", C.c_int32), ("beta", C.c_int32), ("max_iter", C.c_int32),
                ("restart_period", C.c_int32), ("max_backtrack", C.c_int32), ("flags", C.c_int32),
                ("stall_window", C.c_int32), ("reserved", C.c_int32), ("tol_grad", C.c_double), ("tol_dE", C.c_double), ("sigma", C.c_double),
                ("armijo_c1", C.c_double), ("theta_max", C.c_double), ("tau_rel", C.c_double),
                ("blend", C.c_double)]


class Terms(C.Structure):
    _fields_ = [("E", C.c_double), ("E_kin", C.c_double * 2), ("E_trap", C.c_double * 2),
                ("E_c", (C.c_double * 2) * 2), ("E_dd", (C.c_double * 2) * 2),
                ("E_lhy", C.c_double), ("mu", C.c_double * 2), ("shift", C.c_double * 2),
                ("res", C.c_double * 2), ("norm2", C.c_double * 2)]

    def to_dict(self) -> dict:
        return {"E": self.E, "E_kin": list(self.E_kin), "E_trap": list(self.E_trap),
                "E_c": [list(r) for r in self.E_c], "E_dd": [list(r) for r in self.E_dd],
                "E_lhy": self.E_lhy, "mu": list(self.mu), "shift": list(self.shift),
                "res": list(self.res), "norm2": list(self.norm2)}


class LsReport(C.Structure):
    _fields_ = [("E0", C.c_double), ("E1", C.c_double), ("E2", C.c_double), ("alpha", C.c_double),
                ("theta", C.c_double * 2), ("E_new", C.c_double), ("pnorm", C.c_double * 2),
                ("n_trials", C.c_int32), ("path", C.c_int32)]


class Iter(C.Structure):
    _fields_ = [("iter", C.c_int32), ("n_trials", C.c_int32), ("restarted", C.c_int32),
                ("path", C.c_int32), ("E", C.c_double), ("res_max", C.c_double),
                ("E1", C.c_double), ("E2", C.c_double), ("alpha", C.c_double), ("beta", C.c_double)]


class IteOpts(C.Structure):
    _fields_ = [("dt", C.c_double), ("tol_dE", C.c_double), ("max_iter", C.c_int32), ("flags", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("n_restarts", C.c_int32), ("n_backtracks", C.c_int32),
                ("status", C.c_int32), ("final", Terms), ("seconds", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("fft_variant", (C.c_int32 * 2) * 3), ("pw_blocks", C.c_int32), ("lhy_table", C.c_int32),
                ("lhy_terms", C.c_int32), ("kin_axes", C.c_int32),
                ("fuse_z", C.c_int32)]


class Physical(C.Structure):
    _fields_ = [("mass_amu", C.c_double), ("a_bohr", (C.c_double * 2) * 2), ("mu_bohr", C.c_double * 2),
                ("N", C.c_double * 2), ("f0_hz", C.c_double), ("trap_hz", C.c_double * 3),
                ("c_lhy", C.c_double), ("r_cut_um", C.c_double), ("n_u", C.c_int32), ("contact_2pi", C.c_int32),
                ("dip_cut", C.c_int32)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("total_bytes", C.c_double)]


# (name, restype, argtypes) of every entry point declared in include/bec.h
_VP, _DP, _I32, _DBL = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_double
_D22 = (C.c_double * 2) * 2
SIGNATURES = [
    ("bec_workspace_size", C.c_int, [C.POINTER(Grid), C.POINTER(Params), C.POINTER(C.c_size_t)]),
    ("bec_create", C.c_int, [C.POINTER(Grid), C.POINTER(Params), _VP, _VP, C.c_size_t, C.POINTER(_VP)]),
    ("bec_destroy", C.c_int, [_VP]),
    ("bec_set_params", C.c_int, [_VP, C.POINTER(Params)]),
    ("bec_fft3d", C.c_int, [_VP, _VP, _VP, _I32, _I32]),
    ("bec_energy", C.c_int, [_VP, _VP, C.POINTER(Terms)]),
    ("bec_hamiltonian", C.c_int, [_VP, _VP, _VP, C.POINTER(Terms)]),
    ("bec_gradient", C.c_int, [_VP, _VP, _VP, _I32, C.POINTER(Terms)]),
    ("bec_energy_gradient_async", C.c_int, [_VP, _VP, _VP, _VP]),
    ("bec_gradient_noalloc", C.c_int, [C.POINTER(Grid), C.POINTER(Params), _VP, _VP, _VP, _I32,
                                       C.POINTER(Terms)]),
    ("bec_precond_apply", C.c_int, [_VP, _I32, _DBL, _VP, _VP, _VP]),
    ("bec_precond_apply_blend", C.c_int, [_VP, _DBL, _DBL, _VP, _VP, _VP]),
    ("bec_linesearch", C.c_int, [_VP, _VP, _VP, _VP, C.POINTER(Opts), C.POINTER(LsReport)]),
    ("bec_solve", C.c_int, [_VP, _VP, C.POINTER(Opts), C.POINTER(Report), C.POINTER(Iter), _I32]),
    ("bec_param_grad", C.c_int, [_VP, _VP, C.POINTER(_D22), C.POINTER(_D22), _DP]),
    ("bec_ite_solve", C.c_int, [_VP, _VP, C.POINTER(IteOpts), C.POINTER(Report), _DP, _I32]),
    ("bec_batch_set_tuning", C.c_int, [_VP, C.POINTER(Grid), C.POINTER(Tuning)]),
    ("bec_batch_workspace_size", C.c_int, [_I32, C.POINTER(Grid), C.POINTER(Params), C.POINTER(C.c_size_t)]),
    ("bec_batch_create", C.c_int, [_I32, C.POINTER(Grid), C.POINTER(Params), _VP, _VP, C.c_size_t,
                                   C.POINTER(_VP)]),
    ("bec_batch_destroy", C.c_int, [_VP]),
    ("bec_batch_solve", C.c_int, [_VP, C.POINTER(_VP), C.POINTER(Opts), _I32, _I32, C.POINTER(Report)]),
    ("bec_get_tuning", C.c_int, [_VP, C.POINTER(Tuning)]),
    ("bec_set_tuning", C.c_int, [_VP, C.POINTER(Tuning)]),
    ("bec_fft_variant_count", C.c_int, [_I32, C.POINTER(_I32)]),
    ("bec_time_fft_pass", C.c_int, [_VP, _I32, _I32, _I32, _I32, _DP]),
    ("bec_profile_enable", C.c_int, [_VP, _I32]),
    ("bec_profile_read", C.c_int, [_VP, C.POINTER(KernelStat), _I32, C.POINTER(_I32)]),
    ("bec_gauss_legendre", C.c_int, [_I32, _DP, _DP]),
    ("bec_params_from_physical", C.c_int, [C.POINTER(Physical), C.POINTER(Params), _DP]),
    ("bec_last_error", C.c_char_p, []),
]

_lib = None


def lib():
    """Load libbecpcg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, where: str, ok=(0,)):
    if status not in ok:
        raise BecError(status, where, lib().bec_last_error().decode(errors="replace"))
    return status


def make_grid(grid: dict) -> Grid:
    g = Grid()
    for d in range(3):
        g.n[d] = int(grid["n"][d]); g.lo[d] = float(grid["lo"][d]); g.hi[d] = float(grid["hi"][d])
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


# bec_opts.flags bits (include/bec.h)
SOLVE_SYNCHRONOUS = 1
SOLVE_CONTINUE = 2

DEFAULT_OPTS = dict(pc=1, beta=0, max_iter=2000, restart_period=50, max_backtrack=30, flags=0,
                    tol_grad=1e-10, tol_dE=0.0, sigma=1e-6, armijo_c1=1e-4,
                    theta_max=1.5707963267948966, tau_rel=1e-14, blend=-1.0)


def make_opts(o: dict | None) -> Opts:
    d = dict(DEFAULT_OPTS)
    d.update(o or {})
    O = Opts()
    for k, _ in Opts._fields_:
        if k in d:
            setattr(O, k, d[k])
    return O
