"""Host-side logic (no GPU): the ctypes mirrors of the C-ABI structs match the
layout a C compiler gives include/mspcg.h, the binding marshals solve
parameters, and bench.py's accounting helpers behave."""
import ctypes
import os
import subprocess
import sys

import pytest

from paper_1804_08593_amd import mspcg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

STRUCTS = {
    "mspcg_action": mspcg.Action,
    "mspcg_blocking": mspcg.Blocking,
    "mspcg_tuning": mspcg.Tuning,
    "mspcg_solve_params": mspcg.SolveParams,
    "mspcg_solve_stats": mspcg.SolveStats,
}


def _c_layout(tmp_path):
    """sizeof and field offsets of every ABI struct, as gcc lays them out."""
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mspcg.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines.append('  printf("kc_count n %d\\n", (int)MSPCG_KC_COUNT);')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    cmd = ["gcc", "-std=c99", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", str(src), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("cannot compile the header with gcc here: " + r.stderr[-300:])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out.splitlines()}


def test_ctypes_structs_match_the_header(tmp_path):
    lay = _c_layout(tmp_path)
    for cname, py in STRUCTS.items():
        assert lay[(cname, "size")] == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert lay[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def test_kernel_class_count_matches_the_header(tmp_path):
    lay = _c_layout(tmp_path)
    assert lay[("kc_count", "n")] == mspcg.KC_COUNT == len(mspcg.KC_NAMES)


def test_make_params_marshals_every_field():
    p = mspcg.make_params(tol=3e-9, maxiter=77, solver=mspcg.SOLVER_MSPCG, use_x0=True,
                          block=(4, 6, 8, 10), pad=1, inner_iters=5, inner_prec=mspcg.FP32,
                          check_every=3, delta=0.25, timing=True, rhs_normal=True)
    assert (p.tol, p.maxiter, p.solver, p.use_x0) == (3e-9, 77, mspcg.SOLVER_MSPCG, 1)
    assert list(p.blocking.block) == [4, 6, 8, 10] and p.blocking.pad == 1
    assert (p.inner_iters, p.inner_prec, p.check_every) == (5, mspcg.FP32, 3)
    assert (p.delta, p.timing, p.rhs_normal) == (0.25, 1, 1)


def test_hop_algorithmic_bytes():
    # input + output spinor (2 x 192 B) + 8 links of 144 B shared by Ls outputs
    assert bench.hop_bytes_per_site(16) == 456
    assert bench.hop_bytes_per_site(12) == 480
    assert bench.hop_bytes_per_site(16, 96, 72) == 228


def test_traffic_lookup_needs_matching_sources_and_workload(tmp_path, monkeypatch):
    assert bench.measured_traffic("no-such-class", bench.DEFAULT) is None
    assert bench.measured_traffic("hop64", "no-such-workload") is None
    # a summary taken on other kernel sources is not used
    import json
    f = tmp_path / "hop64_w_traffic.json"
    f.write_text(json.dumps({"workload": "w", "kernel_source_hash": "0" * 16,
                             "traffic_bytes_per_launch": 123}))
    monkeypatch.setattr(bench, "traffic_file", lambda cls, w: str(f))
    assert bench.measured_traffic("hop64", "w") is None
    f.write_text(json.dumps({"workload": "w", "kernel_source_hash": bench.kernel_source_hash("hop64"),
                             "traffic_bytes_per_launch": 123}))
    assert bench.measured_traffic("hop64", "w") == 123


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_field_pointer_checks_need_a_complex128_device_tensor():
    import torch
    with pytest.raises(TypeError):
        mspcg._ptr(torch.zeros(4, dtype=torch.complex128))  # host memory
    with pytest.raises(TypeError):
        mspcg._ptr(object())
