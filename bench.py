#!/usr/bin/env python3
"""Benchmark of the preconditioned nonlinear CG hot path on one MI355X.

Workload: 128^3 grid x 2 components (box [-8,8)^3, trap (1,1,2.6), g11 = g22 = 100,
g12 = 50, gdd = 60 for all pairs, LHY coefficient 5, dipolar cutoff 8), FP64 /
complex128, seeded Gaussian + noise start, P_V preconditioner, HS+ conjugacy.

A step is one accepted PCG iteration (Hamiltonian at the trial point, residual,
preconditioner, conjugacy, projected direction, line-search model with its
FFTs, geodesic trial).  The warm-up is one bec_solve of W steps from the
seeded start (with the solve's start-up: normalisation, first Hamiltonian and
reduce); the timed call continues that solve (BEC_SOLVE_CONTINUE) for exactly K
steps, timed with HIP events on the library's stream and bracketed by device
syncs, so the timed region holds K steps and none of the start-up work.  The
time-to-solution solves run before them, so the GPU has left its idle clocks
(20 steps after a 5-step warm-up from idle read about 4 % slow).

Launch plans: the autotuner's stored plan for the grid
(paper_2510_24543_amd/tuning/gfx950.json, which the committed rocprofv3
summaries also use); --tuning auto tunes afresh, as it does for a grid that has
no stored plan.

Also reported: time to max_i ||H_i psi_i - mu_i psi_i|| < 1e-8 from the seeded
start; PCG against imaginary-time evolution under the paper's |Delta E| < 1e-6
stop rule; per-kernel HIP-event timings over a second, profiled run of the same K
steps (events around every launch on the library's stream; the roofline entry
is the kernel with the largest total time); and the CPU oracle timed on the
host cores on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --copy-probe MIB       (plain device copy, for counter calibration)
       python bench.py --pmc-summary FETCH.csv WRITE.csv COPY_FETCH.csv COPY_WRITE.csv COPY_MIB
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("PCG iter/s and time-to-|∇E|<1e-8 at 128³×2; HBM GB/s vs peak; "
          "batched vs plain")
HBM_PEAK_GBS = 8000.0
WORKLOAD = "M"


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_128cubed.json")
# library profiler labels -> kernel function names as rocprofv3 reports them
# (the direction kernels as instantiated for P_V with LHY, the benchmark's configuration)
# (a name ending in "<" matches any instantiation: the fused direction write + z pass
# is instantiated per z plan variant)
LABEL_KERNEL = {"dir_write": "dir_write_kernel<1, true, 1>", "dir_write_z": "fft_dirwrite_z_kernel<",
                "heval_z": "fft_heval_z_kernel<",
                "heval_epilogue": "heval_epi_kernel",
                "dir_reduce": "dir_reduce_kernel<1, true>", "trial_pack": "trial_kernel",
                "ls_epilogue": "ls_epi_kernel", "reduce_final": "reduce_final_kernel",
                "scale2": "scale2_kernel", "norm2": "norm2_kernel"}
# sources whose change invalidates the stored counter figures of the pointwise kernels
KERNEL_SOURCES = ["paper_2510_24543_amd/csrc/pointwise.hip", "paper_2510_24543_amd/csrc/pw_math.h",
                  "paper_2510_24543_amd/csrc/bec_internal.h", "paper_2510_24543_amd/csrc/pw_point.h",
                  "paper_2510_24543_amd/csrc/fft_fused.hip", "paper_2510_24543_amd/csrc/fft_core.h",
                  "paper_2510_24543_amd/csrc/fft_dirwrite.h", "paper_2510_24543_amd/csrc/fft_fused_composite.hip"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(label: str):
    """HBM bytes per launch of the kernel behind `label` from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by the
    copy-kernel calibration); None when there is no summary for it or the
    kernel sources changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE) or label not in LABEL_KERNEL:
        return None
    try:
        data = json.load(open(TRAFFIC_FILE))
        if data.get("source_hash") != kernel_source_hash():
            return None
        want, kernels = LABEL_KERNEL[label], data["kernels"]
        if want.endswith("<"):
            hits = [k for k in kernels if k.startswith(want)]
            return kernels[hits[0]]["bytes_per_launch"] if len(hits) == 1 else None
        return kernels[want]["bytes_per_launch"]
    except (KeyError, ValueError):
        return None


def copy_probe(mib: int, reps: int = 5):
    """A plain device-to-device copy of `mib` MiB, `reps` times: under
    rocprofv3 --pmc its FETCH_SIZE / WRITE_SIZE per dispatch calibrate the
    counters against a known byte count."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.arange(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    print(json.dumps({"copy_mib": mib, "bytes_read": 8 * n, "bytes_written": 8 * n,
                      "ms": round(ms, 4), "GB_per_s": round(16 * n / (ms * 1e6), 1)}), flush=True)


def kernel_short_name(full: str) -> str:
    """'ns::(anonymous namespace)::name<args>(params)' -> 'name<args>'"""
    end = len(full)
    if full.endswith(")"):
        depth = 0
        for i in range(len(full) - 1, -1, -1):
            depth += {")": 1, "(": -1}.get(full[i], 0)
            if depth == 0:
                end = i
                break
    head, depth, cut = full[:end], 0, 0
    for i, ch in enumerate(head):            # last '::' outside <...> and (...)
        if ch in "<(":
            depth += 1
        elif ch in ">)":
            depth -= 1
        elif ch == ":" and depth == 0 and head[i:i + 2] == "::":
            cut = i + 2
    return head[cut:]


def _pmc_table(path: str, counter: str):
    """mean counter value per dispatch, by kernel name, from a rocprofv3
    counter_collection.csv"""
    import csv
    sums, counts = {}, {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            name = row["Kernel_Name"]
            sums[name] = sums.get(name, 0.0) + float(row["Counter_Value"])
            counts[name] = counts.get(name, 0) + 1
    return {k: (sums[k] / counts[k], counts[k]) for k in sums}


def pmc_summary(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_mib, out_path=None):
    """Write the HBM-traffic summary: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) of each kernel, scaled by known_bytes / counter_bytes of the
    plain copy kernel."""
    known = copy_mib * (1 << 20)

    def copy_factor(path, counter):
        t = _pmc_table(path, counter)
        name, (kib, _) = max(t.items(), key=lambda kv: kv[1][0])
        return known / (kib * 1024.0), name

    f_fac, copy_name = copy_factor(copy_fetch_csv, "FETCH_SIZE")
    w_fac, _ = copy_factor(copy_write_csv, "WRITE_SIZE")
    fetch, write = _pmc_table(fetch_csv, "FETCH_SIZE"), _pmc_table(write_csv, "WRITE_SIZE")
    kernels = {}
    for full in sorted(set(fetch) & set(write)):
        short = kernel_short_name(full).replace("bec::(anonymous namespace)::", "")
        fb = fetch[full][0] * 1024.0 * f_fac
        wb = write[full][0] * 1024.0 * w_fac
        kernels[short] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                          "dispatches": fetch[full][1]}
    out = {"workload": "128^3 x 2", "copy_kernel": copy_name, "copy_bytes_each_way": known,
           "fetch_factor": f_fac, "write_factor": w_fac, "source_hash": kernel_source_hash(),
           "kernels": kernels}
    with open(out_path or TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: round(v["bytes_per_launch"] / 2**20, 2) for k, v in kernels.items()}))
    return out


def cpu_leg(sample_iters: int, repeats: int):
    """Child-process part of the CPU baseline: the oracle on the 128^3 x 2
    workload at the OpenMP thread count of this process; per repeat the rate
    sample_iters / (t(1 + sample_iters) - t(1)) from a 1-step and a longer
    oracle solve of the same seeded start; prints the rates as JSON."""
    import oracle
    from paper_2510_24543_amd import inputs
    cfg = inputs.CONFIGS[WORKLOAD]
    psi0 = inputs.config_state(WORKLOAD)
    opts = {"tol_grad": 0.0}
    rates, t_all = [], time.perf_counter()
    for _ in range(repeats):
        t0 = time.perf_counter()
        oracle.solve(cfg["grid"], cfg["params"], psi0, dict(opts, max_iter=1))
        t1 = time.perf_counter()
        _, rep, _ = oracle.solve(cfg["grid"], cfg["params"], psi0, dict(opts, max_iter=1 + sample_iters))
        t2 = time.perf_counter()
        rates.append((rep["iters"] - 1) / ((t2 - t1) - (t1 - t0)))
    print(json.dumps({"rates": rates, "seconds": time.perf_counter() - t_all}), flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sample_iters: int, repeats: int = 3):
    """The oracle as it stands, on the host cores, in child processes (the
    OpenMP thread count is fixed per process): all host threads (the harness's
    OMP_NUM_THREADS, else every core) with the median of `repeats` rates, then
    one thread with a one-iteration sample."""
    import statistics
    import subprocess

    def leg(threads, sample, reps):
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        p = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", str(sample), str(reps)],
                           env=env, capture_output=True, text=True, check=True)
        return json.loads(p.stdout.strip().splitlines()[-1])

    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    multi = leg(cores, sample_iters, repeats)
    single = leg(1, 1, 1)          # one thread is ~10x slower: one repeat keeps the sample bounded
    what = ("PCG iterations of the same 128^3 x 2 workload from the seeded start; each rate from the "
            "difference of a 1-step and a (1 + s)-step oracle solve")
    return {"value": round(statistics.median(multi["rates"]), 4), "unit": "iter/s", "cores": cores,
            "kind": "oracle",
            "sample": f"s = {sample_iters} {what}, median of {repeats} ({multi['seconds']:.1f} s of CPU work)",
            "rates": [round(r, 4) for r in multi["rates"]],
            "single_thread": {"value": round(single["rates"][0], 4), "unit": "iter/s", "cores": 1,
                              "sample": f"s = 1 {what}, one repeat ({single['seconds']:.1f} s of CPU work)"},
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def pcg_vs_ite(ctx, psi0, base_opts: dict, dt: float, tol_dE: float = 1e-6, E_ref=None, progress=None):
    """The paper's comparison (Sec. VI.B): PCG and imaginary-time evolution from
    the same start, both stopped by |E_n - E_(n-1)| < tol_dE; HIP-event times.
    E_ref (the PCG energy at |grad E| < 1e-8) measures how far each stopped
    state is from the minimum."""
    import torch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {"stop_rule": f"|dE| < {tol_dE:g} between successive iterates", "ite_dt": dt}
    torch.cuda.synchronize()
    ev0.record(ctx.stream)
    _, rep, _ = ctx.solve(psi0, dict(base_opts, tol_grad=0.0, tol_dE=tol_dE, max_iter=20000))
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    out["pcg"] = {"iters": rep["iters"], "seconds": round(ev0.elapsed_time(ev1) / 1000.0, 4),
                  "E": rep["final"]["E"], "res_max": max(rep["final"]["res"]), "status": rep["status"]}
    if progress:
        print(f"{progress}: PCG under the dE rule done ({rep['iters']} iterations)", file=sys.stderr, flush=True)
    ev0.record(ctx.stream)
    _, rep, _ = ctx.ite(psi0, dt, tol_dE=tol_dE, max_iter=100000)
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    t = ev0.elapsed_time(ev1) / 1000.0
    out["ite"] = {"iters": rep["iters"], "seconds": round(t, 4), "ms_per_step": round(1000.0 * t / max(rep["iters"], 1), 4),
                  "E": rep["final"]["E"], "res_max": max(rep["final"]["res"]), "status": rep["status"]}
    out["iteration_ratio"] = round(out["ite"]["iters"] / max(out["pcg"]["iters"], 1), 2)
    out["time_ratio"] = round(out["ite"]["seconds"] / max(out["pcg"]["seconds"], 1e-9), 2)
    out["E_ite_minus_E_pcg"] = out["ite"]["E"] - out["pcg"]["E"]
    if E_ref is not None:
        out["E_ref"] = E_ref
        out["pcg"]["E_minus_E_ref"] = out["pcg"]["E"] - E_ref
        out["ite"]["E_minus_E_ref"] = out["ite"]["E"] - E_ref
    out["paper_context"] = ("Sec. VI.B, 256x256x32 52Cr mixtures on the authors' hardware: CG needs one to two "
                            "orders of magnitude fewer iterations than ITE at |dE| < 1e-6 and reaches slightly "
                            "lower energies; 34 FFTs per CG step vs 8 per ITE step in their count")
    return out


def ite_workload(name: str, dt: float):
    """PCG vs ITE on another workload: the reference energy from a PCG solve to
    |grad E| < 1e-8 (or its last iterate after 20000 steps), then both methods
    under the |dE| < 1e-6 rule from the same seeded start."""
    import torch
    from paper_2510_24543_amd import inputs, solver
    cfg = inputs.CONFIGS[name]
    ctx = solver.Context(cfg["grid"], cfg["params"])
    cached = None
    try:
        from paper_2510_24543_amd import autotune
        cached = autotune.load_cached(cfg["grid"])
    except Exception:
        cached = None
    if cached:
        ctx.set_tuning(cached)
    psi0 = torch.from_numpy(inputs.config_state(name)).cuda()
    opts = {"pc": 1, "beta": 0, "restart_period": 50, "sigma": 1e-6}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(ctx.stream)
    _, ref, _ = ctx.solve(psi0, dict(opts, tol_grad=1e-8, max_iter=20000))
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    print(f"{name}: reference PCG solve done ({ref['iters']} iterations, {ref['status']})", file=sys.stderr, flush=True)
    out = pcg_vs_ite(ctx, psi0, opts, dt, E_ref=ref["final"]["E"], progress=name)
    out["workload"] = name
    out["grid"] = cfg["grid"]["n"]
    out["pcg_to_1e-8"] = {"iters": ref["iters"], "status": ref["status"], "seconds": round(ev0.elapsed_time(ev1) / 1000, 4),
                          "res_max": max(ref["final"]["res"])}
    return out


def precond_study(name: str, tol: float = 1e-8, max_iter: int = 20000):
    """The paper's first comparison (Sec. VI.B): the four preconditioners, the
    symmetrised composite and the blend of P_V and P_Delta (adaptive and
    w = 0.5) with both conjugacy rules, each from the same seeded start to
    max_i ||r_i|| < tol; HIP-event times."""
    import torch
    from paper_2510_24543_amd import inputs, solver, autotune
    cfg = inputs.CONFIGS[name]
    ctx = solver.Context(cfg["grid"], cfg["params"])
    cached = autotune.load_cached(cfg["grid"])
    if cached:
        ctx.set_tuning(cached)
    psi0 = torch.from_numpy(inputs.config_state(name)).cuda()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rows = []
    for pc, pname, blend in ((0, "none", -1.0), (1, "P_V", -1.0), (2, "P_Delta", -1.0), (3, "P_Delta P_V", -1.0),
                             (4, "symmetrised", -1.0), (5, "blend (adaptive)", -1.0), (5, "blend 0.5", 0.5)):
        for beta, bname in ((0, "HS+"), (1, "PR+")):
            opts = {"pc": pc, "beta": beta, "restart_period": 50, "sigma": 1e-6, "tol_grad": tol, "max_iter": max_iter,
                    "blend": blend}
            torch.cuda.synchronize()
            ev0.record(ctx.stream)
            _, rep, _ = ctx.solve(psi0, opts)
            ev1.record(ctx.stream)
            torch.cuda.synchronize()
            rows.append({"precond": pname, "beta": bname, "iters": rep["iters"], "status": rep["status"],
                         "seconds": round(ev0.elapsed_time(ev1) / 1000.0, 4), "E": rep["final"]["E"],
                         "res_max": max(rep["final"]["res"]), "restarts": rep["n_restarts"],
                         "backtracks": rep["n_backtracks"]})
            print(f"{name}: {pname} {bname} {rep['iters']} iterations {rep['status']}", file=sys.stderr, flush=True)
    return {"workload": name, "grid": cfg["grid"]["n"], "tol_grad": tol, "runs": rows}


def scan_comparison(n_inst: int, use_graph: bool = True):
    """Parameter scan of n_inst instances (grids cycling 48^3, 64^3, 96^3; seeded
    g12, gdd, LHY): one batched solve against the same instances solved one after
    another with the plain solver, both to |grad E| < 1e-10 from the same seeded
    starts, with the same stall stop (the residual must halve within 1000 steps:
    past the miscibility edge, g12 > 80, the separated components can turn about
    the trap's symmetry axis at almost no cost, and the iteration creeps along that
    soft mode).  Times are HIP-event times of the solve calls only."""
    import torch
    from paper_2510_24543_amd import inputs, solver

    from paper_2510_24543_amd import autotune
    scan = inputs.scan_instances(n_inst)
    grids = [s["grid"] for s in scan]
    params = [s["params"] for s in scan]
    psi0 = [torch.from_numpy(inputs.initial_state(s["grid"], s["params"]["omega"], s["seed"])).cuda()
            for s in scan]
    opts = {"pc": 1, "beta": 0, "restart_period": 50, "tol_grad": 1e-10, "max_iter": 5000, "stall_window": 1000}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    # FFT plans tuned once per grid shape on a single-instance context; both
    # the batched and the one-after-another solves use them
    plans, t_tune = {}, time.perf_counter()
    for s in scan:
        key = tuple(s["grid"]["n"])
        if key not in plans:
            c = solver.Context(s["grid"], s["params"])
            plans[key] = autotune.tune(c, opts=opts)["tuning"]
            c.close()
            del c
    t_tune = time.perf_counter() - t_tune

    b = solver.Batch(grids, params)
    for s in scan:
        b.set_tuning(s["grid"], plans[tuple(s["grid"]["n"])])
    b.solve(psi0, dict(opts, max_iter=2), use_graph=use_graph)   # warm-up (graph build)
    torch.cuda.synchronize()
    ev0.record(b.stream)
    _, brep = b.solve(psi0, opts, use_graph=use_graph)
    ev1.record(b.stream)
    torch.cuda.synchronize()
    t_batch = ev0.elapsed_time(ev1) / 1000.0
    b.close()
    del b

    t_seq = 0.0
    max_rel = 0.0
    seq_iters, seq_s, seq_ok, seq_status = [], [], [], []
    for k, s in enumerate(scan):
        ctx = solver.Context(s["grid"], s["params"])
        ctx.set_tuning(plans[tuple(s["grid"]["n"])])
        torch.cuda.synchronize()
        ev0.record(ctx.stream)
        _, rep, _ = ctx.solve(psi0[k], opts)
        ev1.record(ctx.stream)
        torch.cuda.synchronize()
        seq_s.append(ev0.elapsed_time(ev1) / 1000.0)
        t_seq += seq_s[-1]
        seq_iters.append(rep["iters"])
        seq_ok.append(rep["status"] == "OK")
        seq_status.append(rep["status"])
        if rep["status"] == "OK" and brep[k]["status"] == "OK":
            max_rel = max(max_rel, abs(rep["final"]["E"] - brep[k]["final"]["E"]) / abs(rep["final"]["E"]))
        ctx.close()
        del ctx

    # the same comparison over the instances that reach the tolerance in both
    # solvers: a second batched solve of that subset
    both = [k for k in range(n_inst) if seq_ok[k] and brep[k]["status"] == "OK"]
    sub = None
    if both:
        bs = solver.Batch([grids[k] for k in both], [params[k] for k in both])
        for k in both:
            bs.set_tuning(grids[k], plans[tuple(grids[k]["n"])])
        sub_psi = [psi0[k] for k in both]
        bs.solve(sub_psi, dict(opts, max_iter=2), use_graph=use_graph)
        torch.cuda.synchronize()
        ev0.record(bs.stream)
        _, srep = bs.solve(sub_psi, opts, use_graph=use_graph)
        ev1.record(bs.stream)
        torch.cuda.synchronize()
        t_sub = ev0.elapsed_time(ev1) / 1000.0
        bs.close()
        del bs
        t_seq_sub = sum(seq_s[k] for k in both)
        sub = {"instances": len(both), "batched_s": round(t_sub, 4), "sequential_plain_s": round(t_seq_sub, 4),
               "speedup": round(t_seq_sub / t_sub, 3), "batched_converged": sum(r["status"] == "OK" for r in srep),
               "iters_batched_total": sum(r["iters"] for r in srep),
               "iters_plain_total": sum(seq_iters[k] for k in both)}
    # the whole scan once more in the batch with the composite preconditioner
    # P_Delta^-1 P_V^-1 of Eq. (18) (same plans, tolerance and stall stop)
    bc = solver.Batch(grids, params)
    for s in scan:
        bc.set_tuning(s["grid"], plans[tuple(s["grid"]["n"])])
    copts = dict(opts, pc=3)
    bc.solve(psi0, dict(copts, max_iter=2), use_graph=use_graph)
    torch.cuda.synchronize()
    ev0.record(bc.stream)
    _, crep = bc.solve(psi0, copts, use_graph=use_graph)
    ev1.record(bc.stream)
    torch.cuda.synchronize()
    t_comp = ev0.elapsed_time(ev1) / 1000.0
    bc.close()
    del bc
    dE = [abs(crep[k]["final"]["E"] - brep[k]["final"]["E"]) / abs(brep[k]["final"]["E"])
          for k in range(n_inst) if crep[k]["status"] == "OK" and brep[k]["status"] == "OK"]
    comp = {"precond": "P_Delta^-1 P_V^-1", "batched_s": round(t_comp, 4),
            "speedup_vs_batched_P_V": round(t_batch / t_comp, 3),
            "batched_converged": sum(r["status"] == "OK" for r in crep),
            "iters_total": sum(r["iters"] for r in crep),
            "status": {st: sum(r["status"] == st for r in crep) for st in sorted({r["status"] for r in crep})},
            "max_rel_dE_vs_P_V": max(dE) if dE else None}
    return {"instances": n_inst, "grids": "48^3/64^3/96^3 cycling", "tol_grad": 1e-10,
            "batched_composite": comp,
            "plans": {"x".join(map(str, k)): v for k, v in plans.items()}, "tuning_s": round(t_tune, 3),
            "batched_s": round(t_batch, 4), "sequential_plain_s": round(t_seq, 4),
            "speedup": round(t_seq / t_batch, 3), "graph": use_graph,
            "batched_converged": sum(r["status"] == "OK" for r in brep),
            "max_rel_dE_vs_plain": max_rel,
            "iters_batched_total": sum(r["iters"] for r in brep), "iters_plain_total": sum(seq_iters),
            "stall_window": opts["stall_window"],
            "status_batched": {st: sum(r["status"] == st for r in brep) for st in sorted({r["status"] for r in brep})},
            "status_plain": {st: seq_status.count(st) for st in sorted(set(seq_status))},
            "not_converged": [{"k": k, "g12": round(params[k]["G"][0][1], 2), "batched": brep[k]["status"],
                               "plain": seq_status[k], "iters": brep[k]["iters"]}
                              for k in range(n_inst) if brep[k]["status"] != "OK" or seq_status[k] != "OK"],
            "converged_in_both": sub}


def describe_workload(name: str) -> str:
    """One-line description of a workload of inputs.CONFIGS."""
    from paper_2510_24543_amd import inputs
    c = inputs.CONFIGS[name]
    g, p = c["grid"], c["params"]

    def num(x):
        return f"{x:g}"
    n = g["n"]
    shape = f"{n[0]}^3" if n[0] == n[1] == n[2] else "x".join(map(str, n))
    box = "x".join(f"[{num(lo)},{num(hi)})" for lo, hi in zip(g["lo"], g["hi"]))
    G, D = p["G"], p["Gdd"]
    return (f"{shape} grid x 2 components, box {box}, trap ({','.join(num(w) for w in p['omega'])}), "
            f"g11={num(G[0][0])} g22={num(G[1][1])} g12={num(G[0][1])}, "
            f"gdd11={num(D[0][0])} gdd22={num(D[1][1])} gdd12={num(D[0][1])}, LHY {num(p['c_lhy'])}, "
            f"cutoff {num(p['r_cut'])}, seeded Gaussian+noise start, P_V + HS+ (restart 50), FP64")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=3, help="oracle iterations per CPU-baseline sample (0: skip)")
    ap.add_argument("--no-tts", action="store_true", help="skip the time-to-solution solve")
    ap.add_argument("--scan", type=int, default=96, help="instances of the batched-vs-plain scan (0: skip)")
    ap.add_argument("--ite-dt", type=float, default=0.01,
                    help="imaginary-time step of the PCG-vs-ITE comparison (0: skip it)")
    ap.add_argument("--precond-study", default=None, metavar="WORKLOAD",
                    help="only run the preconditioner x conjugacy-rule study on this workload and print it")
    ap.add_argument("--ite-only", default=None, metavar="WORKLOAD",
                    help="only run the PCG-vs-ITE comparison on this workload (e.g. C2, C3, C5) and print it")
    ap.add_argument("--workload", default=WORKLOAD, choices=("C1a", "C1b", "C2", "M", "C3", "C5"),
                    help="workload of the timed PCG steps (default: the 128^3 headline workload M)")
    ap.add_argument("--tuning", choices=("auto", "cache", "default"), default="cache",
                    help="launch plans: the autotuner's stored plan for the grid (autotune now if there is "
                         "none), autotune now, or the defaults")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--cpu-leg", nargs=2, type=int, default=None, metavar=("SAMPLE", "REPEATS"),
                    help="only time the oracle at this process's OpenMP thread count (child of the CPU baseline)")
    ap.add_argument("--pmc-summary", nargs=5, default=None,
                    metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE", "COPY_MIB"),
                    help="only turn rocprofv3 counter CSVs into the committed traffic summary")
    args = ap.parse_args()
    if args.cpu_leg:
        cpu_leg(*args.cpu_leg)
        return
    if args.pmc_summary:
        a = args.pmc_summary
        pmc_summary(a[0], a[1], a[2], a[3], int(a[4]))
        return
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU decomposition is a design note, "
              "not code (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_24543_amd import inputs, solver

    if args.precond_study:
        print(json.dumps(precond_study(args.precond_study)), flush=True)
        return
    if args.ite_only:
        print(json.dumps(ite_workload(args.ite_only, args.ite_dt)), flush=True)
        return

    cfg = inputs.CONFIGS[args.workload]
    grid, params = cfg["grid"], cfg["params"]
    psi0_np = inputs.config_state(args.workload)
    dev = torch.device("cuda:0")
    ctx = solver.Context(grid, params, dev)
    psi0 = torch.from_numpy(psi0_np).to(dev)
    base_opts = {"pc": 1, "beta": 0, "restart_period": 50, "sigma": 1e-6}

    from paper_2510_24543_amd import autotune, binding as B
    tuning = {"mode": args.tuning, "plan": ctx.get_tuning()}
    cached = autotune.load_cached(grid) if args.tuning == "cache" else None
    if cached:
        # the plan the autotuner stored for this grid (the one the committed profiles measured)
        ctx.set_tuning(cached)
        tuning.update(plan=ctx.get_tuning(), source=os.path.relpath(autotune.cache_path(), ROOT))
    elif args.tuning in ("auto", "cache"):
        res = autotune.tune(ctx, psi0=psi0, opts=base_opts)
        tuning.update(mode="auto", plan=res["tuning"], seconds=res["seconds"], iter_ms=res["iter_ms"],
                      iter_ms_variants=res["iter_ms_variants"])

    # time to |grad E| < 1e-8 from the seeded start (a fresh solve each, start-up included);
    # run first, so that the GPU has left its idle clocks when the W + K steps below start
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tts = None
    if not args.no_tts:
        ctx.solve(psi0, dict(base_opts, max_iter=2, tol_grad=0.0))   # untimed: the kernels' first launches
        torch.cuda.synchronize()
        ev0.record(ctx.stream)
        _, trep, _ = ctx.solve(psi0, dict(base_opts, max_iter=5000, tol_grad=1e-8))
        ev1.record(ctx.stream)
        torch.cuda.synchronize()
        tts = {"seconds": ev0.elapsed_time(ev1) / 1000.0, "iters": trep["iters"], "status": trep["status"],
               "E_star": trep["final"]["E"], "res_max": max(trep["final"]["res"]),
               "backtracks": trep["n_backtracks"], "restarts": trep["n_restarts"]}

    # the same with the composite preconditioner P_Delta^-1 P_V^-1 (fewest iterations on this grid)
    tts_comp = None
    if not args.no_tts:
        ctx.solve(psi0, dict(base_opts, pc=3, max_iter=2, tol_grad=0.0))   # untimed: its kernels' first launches
        torch.cuda.synchronize()
        ev0.record(ctx.stream)
        _, crep, _ = ctx.solve(psi0, dict(base_opts, pc=3, max_iter=5000, tol_grad=1e-8))
        ev1.record(ctx.stream)
        torch.cuda.synchronize()
        tts_comp = {"precond": "P_Delta^-1 P_V^-1", "seconds": ev0.elapsed_time(ev1) / 1000.0,
                    "iters": crep["iters"], "status": crep["status"], "E_star": crep["final"]["E"],
                    "res_max": max(crep["final"]["res"])}

    # warm-up (untimed): the solve's start-up and W steps
    warm = dict(base_opts, max_iter=max(args.warmup, 0), tol_grad=0.0)
    cont = dict(base_opts, max_iter=args.steps, tol_grad=0.0, flags=B.SOLVE_CONTINUE)
    ctx.solve(psi0, warm)
    torch.cuda.synchronize()

    # timed: exactly K steps, continuing the warm-up's solve
    torch.cuda.synchronize()
    ev0.record(ctx.stream)
    _, rep, _ = ctx.solve(None, cont)
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    steps_done = rep["iters"]
    ms_per_step = ms / max(steps_done, 1)
    value = 1000.0 * steps_done / ms

    # per-kernel timings: HIP events around every launch on the library stream,
    # over a second run of the same K steps (after the same warm-up)
    ctx.solve(psi0, warm)
    ctx.profile(True)
    torch.cuda.synchronize()
    ev0.record(ctx.stream)
    _, prep, _ = ctx.solve(None, cont)
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    prof_ms = ev0.elapsed_time(ev1)
    stats = ctx.kernel_stats()
    ctx.profile(False)
    tot = sum(s["total_ms"] for s in stats)
    kernels = sorted(({"name": s["name"], "launches": s["launches"],
                       "avg_us": 1000.0 * s["total_ms"] / max(s["launches"], 1),
                       "share": s["total_ms"] / tot if tot else 0.0,
                       "GB_per_s": s["total_bytes"] / (s["total_ms"] * 1e6) if s["total_ms"] else 0.0,
                       "bytes_per_launch": s["total_bytes"] / max(s["launches"], 1)} for s in stats),
                     key=lambda k: -k["share"])
    dom = kernels[0]
    # the whole step: algorithmic bytes of all launches per step over the unprofiled step time
    step_bytes = sum(s["total_bytes"] for s in stats) / max(prep["iters"], 1)
    step_bw = {"bytes_per_step": step_bytes, "GB_per_s": round(step_bytes / (ms_per_step * 1e6), 1),
               "frac_of_peak": round(step_bytes / (ms_per_step * 1e6) / HBM_PEAK_GBS, 4)}
    traffic = traffic_from_profiles(dom["name"])
    roofline = {"bound": "hbm", "kernel": dom["name"], "achieved": round(dom["GB_per_s"], 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom["GB_per_s"] / HBM_PEAK_GBS, 4),
                "traffic": traffic, "avg_us": round(dom["avg_us"], 2),
                "bytes_per_launch": dom["bytes_per_launch"],
                "profiled_ms_per_step": round(prof_ms / max(prep["iters"], 1), 4)}

    ite_cmp = (pcg_vs_ite(ctx, psi0, base_opts, args.ite_dt, E_ref=tts["E_star"] if tts else None)
               if args.ite_dt > 0 else None)

    scan = scan_comparison(args.scan) if args.scan > 0 else None

    cpu = None
    if args.cpu_sample > 0:
        cpu = cpu_baseline(args.cpu_sample)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "iter/s", "n_gpus": 1,
        "steps": steps_done, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": describe_workload(args.workload), "name": args.workload,
                   "grid": grid["n"], "points": ctx.N, "components": 2},
        "time_to_solution": tts,
        "time_to_solution_composite_precond": tts_comp,
        "tuning": tuning,
        "pcg_vs_ite": ite_cmp,
        "batched_vs_plain": scan,
        "roofline": roofline,
        "step_bandwidth": step_bw,
        "cpu_baseline": cpu,
        "kernels": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in kk.items()} for kk in kernels],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
