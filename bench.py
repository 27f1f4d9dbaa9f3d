"""Benchmark: DWF dslash HBM GB/s and MSPCG vs plain CG time to a 1e-10
residual on one MI355X.

A step is one pass of the whole hot path on the 24^3x48, Ls=16 Moebius
workload (b=1.5, c=0.5, M5=1.8, mf=0.005, links exp(0.2 i H)): the even-odd
RHS preparation, a plain FP64 CG solve to a true residual of 1e-10, a
mixed-precision CG solve (FP32 iterations, FP64 reliable updates), an MSPCG
solve (16 blocks of 12^3x24, 6 local iterations, FP16 storage / FP32 math)
to the same residual, the same MSPCG with the block shape picked by the
library's blocking autotuner, and the odd-site reconstruction.  Inputs are
seeded synthetic fields already resident in HBM when the timed region starts;
autotuning is untimed set-up and reported separately.

value = algorithmic HBM bytes of every FP64 whole-lattice dslash launch in the
timed steps / their summed kernel time (HIP events on the solve stream).  The
last hop of each CG step, which also carries the fused vector update, is
timed as its own class ("hopcg") and is not part of `value`.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: dims, Ls, M5, mf, b, c, eps, blocks, gauge seed, rhs seed
    "dwf_moebius_24c48_ls16": dict(dims=(24, 24, 24, 48), Ls=16, M5=1.8, mf=0.005, b=1.5, c=0.5,
                                   eps=0.2, block=(12, 12, 12, 24), gseed=1003, rseed=2003),
    "dwf_moebius_16c16_ls12": dict(dims=(16, 16, 16, 16), Ls=12, M5=1.8, mf=0.01, b=1.5, c=0.5,
                                   eps=0.2, block=(8, 8, 8, 8), gseed=1002, rseed=2002),
    "dwf_moebius_32c64_ls12": dict(dims=(32, 32, 32, 64), Ls=12, M5=1.8, mf=0.01, b=1.5, c=0.5,
                                   eps=0.2, block=(16, 16, 16, 32), gseed=1006, rseed=2006),
}
DEFAULT = "dwf_moebius_24c48_ls16"


# committed rocprofv3 counter summaries (HBM bytes per launch of a kernel
# class), valid only for the kernel sources they were taken on
KERNEL_SOURCES = {
    "hop64": ["hop_impl.h", "hop_f64.hip", "common.h", "fived.h", "api.hip"],
    "hopdom": ["hop_impl.h", "hop_f16.hip", "common.h", "fived.h", "precond.hip"],
}


def traffic_file(cls: str, workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"{cls}_{workload}_traffic.json")


def kernel_source_hash(cls: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[cls]:
        h.update(open(os.path.join(ROOT, "paper_1804_08593_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(cls: str, workload: str):
    """HBM bytes per launch of kernel class `cls` from the committed rocprofv3
    counter summary, or None when it is missing or was taken on other kernel
    sources."""
    if cls not in KERNEL_SOURCES:
        return None
    try:
        t = json.load(open(traffic_file(cls, workload)))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash(cls) or t.get("workload") != workload:
        return None
    return t.get("traffic_bytes_per_launch")


def hop_bytes_per_site(Ls: int, prec_bytes=192, link_bytes=144) -> float:
    """Algorithmic bytes of one hop output (x, s): input + output spinor + 8 links / Ls."""
    return 2 * prec_bytes + 8 * link_bytes / Ls


def cpu_baseline(w, U, b, seconds_target=12.0):
    """The oracle's hop, timed on the host cores on a bounded sample of output
    sites of the same lattice; reported in the metric's unit (GB/s)."""
    import oracle as O

    act = O.Action(w["dims"], w["Ls"], w["M5"], w["mf"], w["b"], w["c"])
    V4 = int(np.prod(w["dims"]))
    rng = np.random.default_rng(0)
    O.hop_sites(act, U, b, rng.choice(V4, size=64, replace=False))  # thread pool warm-up
    n_total, t_total, chunk = 0, 0.0, 2048
    while t_total < seconds_target:
        sites = np.sort(rng.choice(V4, size=min(chunk, V4), replace=False))
        t0 = time.perf_counter()
        O.hop_sites(act, U, b, sites)
        t_total += time.perf_counter() - t0
        n_total += len(sites)
        chunk = min(2 * chunk, V4)
    nbytes = n_total * w["Ls"] * hop_bytes_per_site(w["Ls"])
    return {"value": round(nbytes / t_total / 1e9, 3), "unit": "GB/s", "cores": O.get_threads(),
            "kind": "oracle",
            "sample": f"oracle Wilson hop on {n_total} random output sites x Ls={w['Ls']} of the "
                      f"{'x'.join(map(str, w['dims']))} lattice in {t_total:.1f} s; algorithmic "
                      f"bytes {hop_bytes_per_site(w['Ls']):.0f} B per (x,s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--no-mspcg", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--inner-iters", type=int, default=6)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-tuned-blocking", action="store_true")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--calibrate", action="store_true",
                    help="only run 5 plain 1 GiB device copies (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; sharding the MSPCG blocks "
                                   "over several GPUs is not implemented"}))
        sys.exit(2)

    import torch

    if args.calibrate:
        a = torch.zeros(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "5 copies of 1 GiB (read 1 GiB + write 1 GiB each)"}))
        return

    from paper_1804_08593_amd import mspcg, synth

    w = WORKLOADS[args.workload]
    dims, Ls = w["dims"], w["Ls"]
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    log(f"[bench] generating {args.workload}")
    U = synth.gauge_field(dims, w["eps"], w["gseed"])
    b = synth.fermion_field(dims, Ls, w["rseed"])
    ctx = mspcg.Context(dims, Ls, w["M5"], w["mf"], w["b"], w["c"])
    Ud = torch.from_numpy(U).cuda()
    ctx.load_gauge(Ud)
    bd = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bd)
    torch.cuda.synchronize()
    log("[bench] inputs resident")
    tuning = None
    if not args.no_autotune:
        # traversal tiles / XCD order chosen by the library's autotuner (untimed set-up)
        t0 = time.perf_counter()
        tuning = ctx.autotune(block=w["block"], pad=2)
        tuning["seconds"] = round(time.perf_counter() - t0, 2)
        log(f"[bench] autotune: {tuning}")

    p_cg = mspcg.make_params(tol=args.tol, maxiter=20000, solver=mspcg.SOLVER_CG, timing=True)
    p_ms = mspcg.make_params(tol=args.tol, maxiter=20000, solver=mspcg.SOLVER_MSPCG,
                             block=w["block"], pad=2, inner_iters=args.inner_iters,
                             inner_prec=mspcg.FP16, timing=True)
    p_mx = mspcg.make_params(tol=args.tol, maxiter=20000, solver=mspcg.SOLVER_MIXED_CG,
                             delta=0.1, timing=True)
    run_ms = not args.no_mspcg
    run_mx = not args.no_mixed
    run_mt = run_ms and not args.no_tuned_blocking
    tuned_block = None
    if run_mt:
        # MSPCG with the block shape chosen by the library's blocking autotuner, on a
        # second context so neither solve rebuilds its block domains (untimed set-up);
        # the tuned solve uses the context blocking (block[0] == 0)
        t0 = time.perf_counter()
        ctx_t = mspcg.Context(dims, Ls, w["M5"], w["mf"], w["b"], w["c"])
        ctx_t.load_gauge(Ud)
        blk, pad = ctx_t.tune_blocking(mspcg.make_params(tol=args.tol, solver=mspcg.SOLVER_MSPCG,
                                                         pad=2, inner_iters=args.inner_iters,
                                                         inner_prec=mspcg.FP16))
        if not args.no_autotune:
            ctx_t.autotune(block=blk, pad=pad)
        tuned_block = {"block": list(blk), "pad": pad, "seconds": round(time.perf_counter() - t0, 2)}
        log(f"[bench] tuned blocking: {tuned_block}")
        p_mt = mspcg.make_params(tol=args.tol, maxiter=20000, solver=mspcg.SOLVER_MSPCG,
                                 inner_iters=args.inner_iters, inner_prec=mspcg.FP16, timing=True)

    def step():
        out = {"cg": ctx.solve(bd, x, p_cg)}
        if run_mx:
            out["mixed"] = ctx.solve(bd, x, p_mx)
        if run_ms:
            out["mspcg"] = ctx.solve(bd, x, p_ms)
        if run_mt:
            out["mspcg_tuned"] = ctx_t.solve(bd, x, p_mt)
        return out

    def describe(r):
        return ", ".join(f"{k} {v['outer_iters']} it {v['seconds']:.3f} s" for k, v in r.items())

    for i in range(args.warmup):
        r = step()
        log(f"[bench] warmup {i}: {describe(r)}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        r = step()
        results.append(r)
        log(f"[bench] step {i}: {describe(r)}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # aggregate kernel-class timings over the timed steps
    agg_ms, agg_b, agg_n = {}, {}, {}
    for r in results:
        # the kernel classes cover the fixed workload's solves (CG, mixed CG and the
        # 16-block MSPCG); the tuned-blocking MSPCG is reported beside them
        for name, solver in r.items():
            if name == "mspcg_tuned":
                continue
            for k, v in solver["kernel_ms"].items():
                agg_ms[k] = agg_ms.get(k, 0.0) + v
                agg_b[k] = agg_b.get(k, 0.0) + solver["kernel_bytes"][k]
                agg_n[k] = agg_n.get(k, 0) + solver["kernel_launches"][k]
    hop_gbs = agg_b["hop64"] / (agg_ms["hop64"] * 1e-3) / 1e9 if agg_ms.get("hop64") else None
    dom = max(agg_ms, key=lambda k: agg_ms[k])
    dom_gbs = agg_b[dom] / (agg_ms[dom] * 1e-3) / 1e9 if agg_ms[dom] else None
    per_class = {k: {"ms_total": round(agg_ms[k], 3), "launches": agg_n[k],
                     "avg_us": round(1e3 * agg_ms[k] / agg_n[k], 2) if agg_n[k] else None,
                     "bytes_per_launch": round(agg_b[k] / agg_n[k]) if agg_n[k] else None,
                     "GBps": round(agg_b[k] / (agg_ms[k] * 1e-3) / 1e9, 1) if agg_ms[k] else None}
                 for k in agg_ms}
    last = results[-1]
    cg_s = float(np.median([r["cg"]["seconds"] for r in results]))
    line = {
        "metric": "DWF dslash HBM GB/s; MSPCG vs plain CG time-to-1e-10 residual, 1 GPU",
        "value": round(hop_gbs, 1) if hop_gbs else None,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded exp(i eps H) links, Gaussian RHS)",
        "config": {"workload": args.workload, "dims": list(dims), "Ls": Ls, "M5": w["M5"],
                   "mf": w["mf"], "b": w["b"], "c": w["c"], "block": list(w["block"]),
                   "inner_iters": args.inner_iters, "tol": args.tol},
        "cg": {"seconds": round(cg_s, 4), "outer_iters": last["cg"]["outer_iters"],
               "true_rel_resid": last["cg"]["true_rel_resid"]},
        "kernels": per_class,
        "tuning": tuning,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(dom_gbs, 1) if dom_gbs else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dom_gbs / HBM_PEAK_GBS, 4) if dom_gbs else None,
                     "traffic": measured_traffic(dom, args.workload)},
    }
    if run_mx:
        mx_s = float(np.median([r["mixed"]["seconds"] for r in results]))
        line["mixed_cg"] = {"seconds": round(mx_s, 4), "outer_iters": last["mixed"]["outer_iters"],
                            "reliable_updates": last["mixed"]["restarts"],
                            "true_rel_resid": last["mixed"]["true_rel_resid"],
                            "speedup_vs_cg": round(cg_s / mx_s, 3)}
    if run_ms:
        ms_s = float(np.median([r["mspcg"]["seconds"] for r in results]))
        line["mspcg"] = {"seconds": round(ms_s, 4), "outer_iters": last["mspcg"]["outer_iters"],
                         "inner_iters_total": last["mspcg"]["inner_iters_total"],
                         "true_rel_resid": last["mspcg"]["true_rel_resid"],
                         "speedup_vs_cg": round(cg_s / ms_s, 3),
                         "outer_iter_reduction_g": round(last["cg"]["outer_iters"]
                                                         / max(1, last["mspcg"]["outer_iters"]), 3)}
    if run_mt:
        mt_s = float(np.median([r["mspcg_tuned"]["seconds"] for r in results]))
        line["mspcg_tuned_blocking"] = {"seconds": round(mt_s, 4), "blocking": tuned_block,
                                        "outer_iters": last["mspcg_tuned"]["outer_iters"],
                                        "inner_iters_total": last["mspcg_tuned"]["inner_iters_total"],
                                        "true_rel_resid": last["mspcg_tuned"]["true_rel_resid"],
                                        "speedup_vs_cg": round(cg_s / mt_s, 3)}
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(w, U, b)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
