"""CPU checks of the C ABI library: it loads, exports every entry point that
include/bec.h declares, and its host-only logic (argument validation, workspace
sizing, quadrature) works without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2510_24543_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bec.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(bec_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 14
    L = B.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert {n for n, _, _ in B.SIGNATURES} == set(names)


def test_struct_layouts_match_the_header(tmp_path):
    """Compile a C probe against include/bec.h and compare sizes and offsets."""
    import subprocess
    structs = {"bec_grid": B.Grid, "bec_params": B.Params, "bec_opts": B.Opts, "bec_terms": B.Terms,
               "bec_ls_report": B.LsReport, "bec_iter": B.Iter, "bec_report": B.Report,
               "bec_kernel_stat": B.KernelStat, "bec_tuning": B.Tuning, "bec_ite_opts": B.IteOpts,
               "bec_physical": B.Physical}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bec.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0; }"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.split("\n") if l)
    for cname, py in structs.items():
        assert int(out[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_solve_flag_values_match_the_header():
    src = open(os.path.join(ROOT, "include", "bec.h")).read()
    defs = dict(re.findall(r"^#define (BEC_SOLVE_\w+) (\d+)", src, flags=re.M))
    assert defs == {"BEC_SOLVE_SYNCHRONOUS": str(B.SOLVE_SYNCHRONOUS), "BEC_SOLVE_CONTINUE": str(B.SOLVE_CONTINUE)}


def grid(n=(32, 32, 32)):
    return B.make_grid({"n": list(n), "lo": [-8.0] * 3, "hi": [8.0] * 3})


PARAMS = {"N": [1.0, 1.0], "omega": [1, 1, 2.6], "G": [[100, 50], [50, 100]],
          "Gdd": [[60, 60], [60, 60]], "c_lhy": 5.0, "r_cut": 8.0, "n_u": 16}


def test_workspace_size_and_validation():
    L = B.lib()
    sz = C.c_size_t()
    p = B.make_params(PARAMS)
    assert L.bec_workspace_size(C.byref(grid()), C.byref(p), C.byref(sz)) == 0
    assert 448 * 32 ** 3 < sz.value < 480 * 32 ** 3     # 28 complex fields of N points + tables
    assert L.bec_workspace_size(C.byref(grid((30, 32, 32))), C.byref(p), C.byref(sz)) == 7
    assert b"not supported" in L.bec_last_error()
    bad = B.make_params(dict(PARAMS, n_u=0))
    assert L.bec_workspace_size(C.byref(grid()), C.byref(bad), C.byref(sz)) == 1
    asym = B.make_params(dict(PARAMS, G=[[100, 50], [40, 100]]))
    assert L.bec_workspace_size(C.byref(grid()), C.byref(asym), C.byref(sz)) == 1
    g = B.make_grid({"n": [32, 32, 32], "lo": [1.0] * 3, "hi": [-1.0] * 3})
    assert L.bec_workspace_size(C.byref(g), C.byref(p), C.byref(sz)) == 1
    for n in (8, 16, 32, 48, 64, 96, 128, 256):
        assert L.bec_workspace_size(C.byref(grid((n, 8, 16))), C.byref(p), C.byref(sz)) == 0


@pytest.mark.parametrize("n", [1, 2, 7, 16, 40, 64])
def test_library_quadrature_is_exact_for_polynomials(n):
    L = B.lib()
    u, w = np.zeros(n), np.zeros(n)
    dp = C.POINTER(C.c_double)
    assert L.bec_gauss_legendre(n, u.ctypes.data_as(dp), w.ctypes.data_as(dp)) == 0
    assert np.all(np.diff(u) > 0) and np.all(w > 0)
    for k in range(2 * n):
        assert abs(np.sum(w * u ** k) - 1.0 / (k + 1)) < 1e-15
    assert L.bec_gauss_legendre(65, u.ctypes.data_as(dp), w.ctypes.data_as(dp)) == 1


def test_fft_variant_counts():
    L = B.lib()
    n = C.c_int32()
    for length in (8, 16, 32, 48, 64, 96, 128, 256):
        assert L.bec_fft_variant_count(length, C.byref(n)) == 0 and n.value >= 3
    assert L.bec_fft_variant_count(30, C.byref(n)) == 7 and n.value == 0
