"""Python front end of the gfx950 library (argument marshalling only).

Every step of the hot path runs in the HIP kernels behind include/bec.h; this
module checks shapes, allocates the caller-owned buffers with PyTorch (device
memory and the current stream) and converts the C structs to dicts.

Fields are ``torch.complex128`` tensors of shape ``(2, nx, ny, nz)`` on a HIP
device, contiguous (component, x, y, z; z fastest).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import binding as B

PC = {"none": 0, "V": 1, "kin": 2, "composite": 3, "symmetric": 4, "blend": 5}
BETA = {"HS+": 0, "PR+": 1, "zero": 2}


def _ptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def gradient_noalloc(grid: dict, params: dict, psi: torch.Tensor, projected: bool = False, stream=None):
    """bec_gradient_noalloc: the gradient of bec_gradient without a context, its
    workspace in the library's fixed device array (no allocation by the library;
    the output tensor is allocated here).  psi: complex128 (2, nx, ny, nz) on the
    current device; stream: a torch stream (default: the current one)."""
    if psi.dtype != torch.complex128 or not psi.is_cuda or tuple(psi.shape) != (2, *grid["n"]):
        raise ValueError(f"psi must be a complex128 CUDA tensor of shape (2, {grid['n']})")
    psi = psi.contiguous()
    st = stream if stream is not None else torch.cuda.current_stream(psi.device)
    g = torch.empty_like(psi)
    t = B.Terms()
    B.check(B.lib().bec_gradient_noalloc(C.byref(B.make_grid(grid)), C.byref(B.make_params(params)),
                                         C.c_void_p(st.cuda_stream), _ptr(psi), _ptr(g), int(projected),
                                         C.byref(t)), "bec_gradient_noalloc")
    return g, t.to_dict()


class Context:
    """One grid + parameter set on one device and stream (bec_create / bec_destroy)."""

    def __init__(self, grid: dict, params: dict, device: str | torch.device = "cuda:0", stream=None):
        self.grid = {k: list(v) for k, v in grid.items()}
        self.params = {k: (v if not isinstance(v, (list, tuple)) else [list(r) if isinstance(r, (list, tuple)) else r for r in v])
                       for k, v in params.items()}
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the library runs on a HIP device only")
        self.shape = (2, *[int(n) for n in grid["n"]])
        self.N = int(np.prod(self.shape[1:]))
        L = B.lib()
        self._g = B.make_grid(grid)
        self._p = B.make_params(params)
        nbytes = C.c_size_t()
        B.check(L.bec_workspace_size(C.byref(self._g), C.byref(self._p), C.byref(nbytes)), "bec_workspace_size")
        self.workspace_bytes = int(nbytes.value)
        with torch.cuda.device(self.device):
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ctx = C.c_void_p()
        B.check(L.bec_create(C.byref(self._g), C.byref(self._p), C.c_void_p(self.stream.cuda_stream),
                             C.c_void_p(self._ws_ptr), C.c_size_t(self.workspace_bytes), C.byref(self._ctx)),
                "bec_create")

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            B.lib().bec_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ helpers
    def field(self, x, name="psi") -> torch.Tensor:
        """Return x as a contiguous complex128 device tensor of the context's shape."""
        if not isinstance(x, torch.Tensor):
            x = torch.as_tensor(np.asarray(x))
        x = x.to(device=self.device, dtype=torch.complex128).contiguous()
        if tuple(x.shape) != self.shape:
            raise ValueError(f"{name}: expected shape {self.shape}, got {tuple(x.shape)}")
        return x

    def empty(self) -> torch.Tensor:
        return torch.empty(self.shape, dtype=torch.complex128, device=self.device)

    def set_params(self, params: dict):
        self._p = B.make_params(params)
        self.params = params
        B.check(B.lib().bec_set_params(self._ctx, C.byref(self._p)), "bec_set_params")

    # ------------------------------------------------------------------ entry points
    def fft3d(self, x: torch.Tensor, sign: int = -1) -> torch.Tensor:
        """3D DFT of 1..3 fields of the grid shape (forward unnormalised, inverse / N)."""
        x = x.to(device=self.device, dtype=torch.complex128).contiguous()
        if tuple(x.shape[-3:]) != self.shape[1:]:
            raise ValueError("trailing shape must be the grid")
        nf = int(np.prod(x.shape[:-3])) if x.dim() > 3 else 1
        out = torch.empty_like(x)
        B.check(B.lib().bec_fft3d(self._ctx, _ptr(x), _ptr(out), nf, sign), "bec_fft3d")
        return out

    def energy(self, psi) -> dict:
        psi = self.field(psi)
        t = B.Terms()
        B.check(B.lib().bec_energy(self._ctx, _ptr(psi), C.byref(t)), "bec_energy")
        return t.to_dict()

    def hamiltonian(self, psi):
        psi = self.field(psi)
        h = self.empty()
        t = B.Terms()
        B.check(B.lib().bec_hamiltonian(self._ctx, _ptr(psi), _ptr(h), C.byref(t)), "bec_hamiltonian")
        return h, t.to_dict()

    def gradient(self, psi, projected: bool = False):
        psi = self.field(psi)
        g = self.empty()
        t = B.Terms()
        B.check(B.lib().bec_gradient(self._ctx, _ptr(psi), _ptr(g), int(projected), C.byref(t)), "bec_gradient")
        return g, t.to_dict()

    def energy_gradient_async(self, psi):
        """(E, grad): E a 0-d float64 tensor on the device and the Euclidean
        gradient, both produced by the context stream without a host sync."""
        psi = self.field(psi)
        g = self.empty()
        E = torch.empty((), dtype=torch.float64, device=self.device)
        B.check(B.lib().bec_energy_gradient_async(self._ctx, _ptr(psi), _ptr(g), _ptr(E)),
                "bec_energy_gradient_async")
        if self.stream != torch.cuda.current_stream(self.device):
            for t in (psi, g, E):      # in use on the context stream after this returns
                t.record_stream(self.stream)
        return E, g

    def precond_blend(self, psi, r, blend: float = -1.0, sigma: float = 1e-6) -> torch.Tensor:
        """z = w P_V^-1 r + (1 - w) P_Delta^-1 r at psi (bec_precond_apply_blend;
        blend < 0: the adaptive weight)."""
        psi, r = self.field(psi), self.field(r, "r")
        z = self.empty()
        B.check(B.lib().bec_precond_apply_blend(self._ctx, float(blend), float(sigma), _ptr(psi), _ptr(r), _ptr(z)),
                "bec_precond_apply_blend")
        return z

    def precond(self, pc, psi, r, sigma: float = 1e-6) -> torch.Tensor:
        pc = PC[pc] if isinstance(pc, str) else int(pc)
        psi = self.field(psi)
        r = self.field(r, "r")
        z = self.empty()
        B.check(B.lib().bec_precond_apply(self._ctx, pc, float(sigma), _ptr(psi), _ptr(r), _ptr(z)),
                "bec_precond_apply")
        return z

    def linesearch(self, psi, d, opts: dict | None = None):
        psi = self.field(psi)
        d = self.field(d, "d")
        out = self.empty()
        rep = B.LsReport()
        st = B.lib().bec_linesearch(self._ctx, _ptr(psi), _ptr(d), _ptr(out), C.byref(B.make_opts(opts)),
                                    C.byref(rep))
        B.check(st, "bec_linesearch", ok=(0, 5))
        return out, {k: (list(getattr(rep, k)) if k in ("theta", "pnorm") else getattr(rep, k))
                     for k, _ in B.LsReport._fields_} | {"status": B.STATUS[st]}

    def solve(self, psi0, opts: dict | None = None, log_cap: int = 0):
        """Preconditioned nonlinear CG; returns (psi, report, log).  With
        opts["flags"] containing SOLVE_CONTINUE the call continues the last solve
        on this context, which stopped at its max_iter, and psi0 may be None."""
        o = B.make_opts(opts)
        if psi0 is None:
            if not o.flags & B.SOLVE_CONTINUE:
                raise ValueError("psi0 is needed unless opts['flags'] has SOLVE_CONTINUE")
            psi = self.empty()
        else:
            psi = self.field(psi0).clone()
        rep = B.Report()
        cap = max(int(log_cap), 0)
        logs = (B.Iter * max(cap, 1))()
        st = B.lib().bec_solve(self._ctx, _ptr(psi), C.byref(o), C.byref(rep), logs, cap)
        B.check(st, "bec_solve", ok=(0, 4, 5, 8))
        out = {"iters": rep.iters, "n_restarts": rep.n_restarts, "n_backtracks": rep.n_backtracks,
               "status": B.STATUS[rep.status], "final": rep.final.to_dict(), "seconds": rep.seconds}
        log = [{k: getattr(logs[i], k) for k, _ in B.Iter._fields_} for i in range(min(rep.iters, cap))]
        return psi, out, log

    def ite(self, psi0, dt: float, tol_dE: float = 1e-6, max_iter: int = 100000, log_cap: int = 0,
            flags: int = 0):
        """Imaginary-time evolution baseline (normalised first-order splitting);
        returns (psi, report, energies of the iterates psi^0, psi^1, ...)."""
        psi = self.field(psi0).clone()
        rep = B.Report()
        cap = max(int(log_cap), 0)
        logE = (C.c_double * max(cap, 1))()
        o = B.IteOpts(dt=float(dt), tol_dE=float(tol_dE), max_iter=int(max_iter), flags=int(flags))
        st = B.lib().bec_ite_solve(self._ctx, _ptr(psi), C.byref(o), C.byref(rep), logE, cap)
        B.check(st, "bec_ite_solve", ok=(0, 4))
        out = {"iters": rep.iters, "status": B.STATUS[rep.status], "final": rep.final.to_dict(),
               "seconds": rep.seconds}
        return psi, out, np.array(logE[:min(rep.iters + 1, cap)])

    # ------------------------------------------------------------------ tuning
    def get_tuning(self) -> dict:
        t = B.Tuning()
        B.check(B.lib().bec_get_tuning(self._ctx, C.byref(t)), "bec_get_tuning")
        return {"fft_variant": [[t.fft_variant[a][k] for k in range(2)] for a in range(3)],
                "pw_blocks": t.pw_blocks, "lhy_table": t.lhy_table, "lhy_terms": t.lhy_terms,
                "kin_axes": t.kin_axes, "fuse_z": t.fuse_z}

    def set_tuning(self, tuning: dict):
        t = B.Tuning()
        for a in range(3):
            for k in range(2):
                t.fft_variant[a][k] = int(tuning["fft_variant"][a][k])
        t.pw_blocks = int(tuning["pw_blocks"])
        t.lhy_table = int(tuning.get("lhy_table", 1))
        t.kin_axes = int(tuning.get("kin_axes", 1))
        t.fuse_z = int(tuning.get("fuse_z", 3))
        B.check(B.lib().bec_set_tuning(self._ctx, C.byref(t)), "bec_set_tuning")

    def time_fft_pass(self, axis: int, kind: int, variant: int, reps: int = 20) -> float:
        ms = C.c_double()
        B.check(B.lib().bec_time_fft_pass(self._ctx, axis, kind, variant, reps, C.byref(ms)), "bec_time_fft_pass")
        return ms.value

    def profile(self, on: bool):
        B.check(B.lib().bec_profile_enable(self._ctx, int(on)), "bec_profile_enable")

    def kernel_stats(self) -> list:
        cap = 64
        arr = (B.KernelStat * cap)()
        n = C.c_int32()
        B.check(B.lib().bec_profile_read(self._ctx, arr, cap, C.byref(n)), "bec_profile_read")
        return [{"name": arr[i].name.decode(), "launches": arr[i].launches, "total_ms": arr[i].total_ms,
                 "total_bytes": arr[i].total_bytes} for i in range(min(n.value, cap))]

    def param_grad(self, psi) -> dict:
        psi = self.field(psi)
        dG = ((C.c_double * 2) * 2)()
        dD = ((C.c_double * 2) * 2)()
        dc = C.c_double()
        B.check(B.lib().bec_param_grad(self._ctx, _ptr(psi), C.byref(dG), C.byref(dD), C.byref(dc)),
                "bec_param_grad")
        return {"dG": np.array([[dG[i][j] for j in range(2)] for i in range(2)]),
                "dGdd": np.array([[dD[i][j] for j in range(2)] for i in range(2)]),
                "dc_lhy": dc.value}


class Batch:
    """Many independent instances solved together (bec_batch_*).

    Instances with the same grid shape share every kernel launch; the CG
    decisions run on the device; ``use_graph`` replays a captured hipGraph of
    ``rounds_per_sync`` rounds between host checks."""

    def __init__(self, grids: list, params: list, device: str | torch.device = "cuda:0", stream=None):
        if len(grids) != len(params) or not grids:
            raise ValueError("need one params dict per grid")
        self.n = len(grids)
        self.device = torch.device(device)
        self.shapes = [(2, *[int(v) for v in g["n"]]) for g in grids]
        L = B.lib()
        self._g = (B.Grid * self.n)(*[B.make_grid(g) for g in grids])
        self._p = (B.Params * self.n)(*[B.make_params(p) for p in params])
        nbytes = C.c_size_t()
        B.check(L.bec_batch_workspace_size(self.n, self._g, self._p, C.byref(nbytes)), "bec_batch_workspace_size")
        self.workspace_bytes = int(nbytes.value)
        with torch.cuda.device(self.device):
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
            self._ws_ptr = (self._ws.data_ptr() + 255) // 256 * 256
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._b = C.c_void_p()
        B.check(L.bec_batch_create(self.n, self._g, self._p, C.c_void_p(self.stream.cuda_stream),
                                   C.c_void_p(self._ws_ptr), C.c_size_t(self.workspace_bytes), C.byref(self._b)),
                "bec_batch_create")

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            B.lib().bec_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, grid: dict, tuning: dict):
        """FFT plans (a Context.get_tuning() dict) for the instances on `grid`."""
        t = B.Tuning()
        for a in range(3):
            for k in range(2):
                t.fft_variant[a][k] = int(tuning["fft_variant"][a][k])
        t.pw_blocks = int(tuning.get("pw_blocks", 0))
        B.check(B.lib().bec_batch_set_tuning(self._b, C.byref(B.make_grid(grid)), C.byref(t)),
                "bec_batch_set_tuning")

    def solve(self, psi0: list, opts: dict | None = None, rounds_per_sync: int = 16, use_graph: bool = True):
        """Returns (list of final states, list of reports)."""
        if len(psi0) != self.n:
            raise ValueError(f"need {self.n} initial states")
        psi = []
        for k, x in enumerate(psi0):
            if not isinstance(x, torch.Tensor):
                x = torch.as_tensor(np.asarray(x))
            x = x.to(device=self.device, dtype=torch.complex128).contiguous().clone()
            if tuple(x.shape) != self.shapes[k]:
                raise ValueError(f"instance {k}: expected shape {self.shapes[k]}, got {tuple(x.shape)}")
            psi.append(x)
        ptrs = (C.c_void_p * self.n)(*[t.data_ptr() for t in psi])
        reps = (B.Report * self.n)()
        B.check(B.lib().bec_batch_solve(self._b, ptrs, C.byref(B.make_opts(opts)), int(rounds_per_sync),
                                        int(bool(use_graph)), reps), "bec_batch_solve")
        out = [{"iters": r.iters, "n_restarts": r.n_restarts, "n_backtracks": r.n_backtracks,
                "status": B.STATUS[r.status], "final": r.final.to_dict(), "seconds": r.seconds} for r in reps]
        return psi, out


def theta_of(params: dict) -> torch.Tensor:
    """Coupling vector (G11, G12, G21, G22, Gdd11, Gdd12, Gdd21, Gdd22, c_lhy) in float64."""
    G, D = params["G"], params["Gdd"]
    return torch.tensor([G[0][0], G[0][1], G[1][0], G[1][1], D[0][0], D[0][1], D[1][0], D[1][1],
                         params["c_lhy"]], dtype=torch.float64)


def params_with_theta(params: dict, theta) -> dict:
    t = [float(v) for v in theta]
    p = dict(params)
    p["G"] = [[t[0], t[1]], [t[2], t[3]]]
    p["Gdd"] = [[t[4], t[5]], [t[6], t[7]]]
    p["c_lhy"] = t[8]
    return p


class Energy(torch.autograd.Function):
    """E[psi; theta] of Sec. II, Eq. (1) as a differentiable function.

    forward: one H evaluation on the GPU (bec_energy_gradient_async) gives E as
    a device tensor and the Euclidean gradient 2 N_i dV H_i psi_i, kept for
    backward, with no host synchronisation.
    backward: grad_psi = dL/dE * 2 N_i dV H_i psi_i (PyTorch's convention for a
    real function of a complex tensor: dE/dRe + i dE/dIm); grad_theta =
    dL/dE * (dE/dG_ij, dE/dGdd_ij, dE/dc_lhy) from bec_param_grad.  At a
    converged ground state grad_theta is dE*/dtheta (envelope theorem).
    """

    @staticmethod
    def forward(ctx_, psi: torch.Tensor, theta: torch.Tensor, bctx: Context):
        p = params_with_theta(bctx.params, theta.detach().cpu().tolist())
        if theta_of(bctx.params).tolist() != theta_of(p).tolist():
            bctx.set_params(p)
        E, grad = bctx.energy_gradient_async(psi.detach())
        ctx_.bctx = bctx
        ctx_.save_for_backward(psi.detach(), grad)
        return E

    @staticmethod
    def backward(ctx_, gE: torch.Tensor):
        psi, grad = ctx_.saved_tensors
        g_psi = g_theta = None
        if ctx_.needs_input_grad[0]:
            g_psi = gE.to(grad.dtype) * grad
        if ctx_.needs_input_grad[1]:
            pg = ctx_.bctx.param_grad(psi)
            v = np.concatenate([pg["dG"].reshape(-1), pg["dGdd"].reshape(-1), [pg["dc_lhy"]]])
            g_theta = gE.detach().cpu() * torch.tensor(v, dtype=torch.float64)
        return g_psi, g_theta, None


def energy(psi: torch.Tensor, theta: torch.Tensor, bctx: Context) -> torch.Tensor:
    return Energy.apply(psi, theta, bctx)
