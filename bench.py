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
import math
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
    "dwf_moebius_16c32_ls12": dict(dims=(16, 16, 16, 32), Ls=12, M5=1.8, mf=0.01, b=1.5, c=0.5,
                                   eps=0.2, block=(8, 8, 8, 16), gseed=1005, rseed=2005),
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


def _cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _hop_sample(O, act, U, b, seconds, rng):
    """Oracle hop on random output sites until `seconds` of CPU work: GB/s."""
    V4 = int(np.prod(act.dims))
    O.hop_sites(act, U, b, rng.choice(V4, size=64, replace=False))  # thread pool warm-up
    n_total, t_total, chunk = 0, 0.0, 1024
    while t_total < seconds:
        sites = np.sort(rng.choice(V4, size=min(chunk, V4), replace=False))
        t0 = time.perf_counter()
        O.hop_sites(act, U, b, sites)
        t_total += time.perf_counter() - t0
        n_total += len(sites)
        chunk = min(2 * chunk, V4)
    return n_total * act.Ls * hop_bytes_per_site(act.Ls) / t_total / 1e9, n_total, t_total


def a_bytes_per_site(Ls: int) -> float:
    """Algorithmic bytes of A = Mhat^+ Mhat per even (x, s) in FP64: four hops
    and the two re-reads of the source for the M5op terms."""
    return 4 * hop_bytes_per_site(Ls) + 2 * 192


def cpu_baseline(w, U, b, gpu_iters=None, c2_iters=None, full=False):
    """The oracle, as it stands, timed on the host cores on bounded samples of
    the workload (reported beside the GPU figures, never a target):
      value: the oracle's hop on random output sites, all threads, GB/s;
      hop_1thread: the same with one thread;
      A: one application of A = Mhat^+ Mhat on the whole lattice, GB/s;
      cg: time to a 1e-10 true residual on the 4^4x8 Shamir workload
          (measured), and on the 16^4x12 and the bench workload
          extrapolated from a few timed oracle CG iterations times the
          iteration count (the GPU's for the bench workload), labelled;
          `full` times the 16^4x12 solve to the end instead (about a minute)."""
    import oracle as O
    from paper_1804_08593_amd import synth

    rng = np.random.default_rng(0)
    act = O.Action(w["dims"], w["Ls"], w["M5"], w["mf"], w["b"], w["c"])
    nthreads = O.get_threads()
    gbs, n_total, t_total = _hop_sample(O, act, U, b, 10.0, rng)
    O.set_threads(1)
    gbs1, n1, t1 = _hop_sample(O, act, U, b, 3.0, rng)
    O.set_threads(nthreads)
    out = {"value": round(gbs, 3), "unit": "GB/s", "cores": nthreads, "kind": "oracle",
           "sample": f"oracle Wilson hop on {n_total} random output sites x Ls={w['Ls']} of the "
                     f"{'x'.join(map(str, w['dims']))} lattice in {t_total:.1f} s with "
                     f"{nthreads} threads; algorithmic bytes {hop_bytes_per_site(w['Ls']):.0f} B "
                     f"per (x,s)",
           "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
           "hop_1thread": {"GBps": round(gbs1, 3), "sites": n1, "seconds": round(t1, 1)}}
    # A on the whole lattice
    be = O.parity_mask(act, b, 0)
    O.normal(act, U, be)  # workspace allocation
    t0 = time.perf_counter()
    O.normal(act, U, be)
    ta = time.perf_counter() - t0
    nh = act.V4 // 2 * act.Ls
    out["A"] = {"GBps": round(nh * a_bytes_per_site(act.Ls) / ta / 1e9, 3),
                "seconds": round(ta, 3),
                "bytes_per_even_site": a_bytes_per_site(act.Ls)}
    cg = {}
    # 4^4 x 8 Shamir, mf = 0.1, links exp(0.3 i H): full solve
    a1 = O.Action((4, 4, 4, 4), 8, 1.8, 0.1, 1.0, 0.0)
    U1 = synth.gauge_field(a1.dims, 0.3, 1001)
    b1 = synth.fermion_field(a1.dims, 8, 2001)
    t0 = time.perf_counter()
    _, i1 = O.solve(a1, U1, b1, tol=1e-10)
    cg["dwf_shamir_4c4_ls8"] = {"seconds": round(time.perf_counter() - t0, 3),
                                "iters": i1.iters, "measured": True}

    def per_iter(a, Ua, ba, k=4):
        _, bh = O.prepare(a, Ua, ba)
        O.cg(a, Ua, bh, tol=1e-30, maxiter=1)
        t0 = time.perf_counter()
        O.cg(a, Ua, bh, tol=1e-30, maxiter=k)
        return (time.perf_counter() - t0) / k, bh

    a2 = O.Action((16, 16, 16, 16), 12, 1.8, 0.01, 1.5, 0.5)
    U2 = synth.gauge_field(a2.dims, 0.2, 1002)
    b2 = synth.fermion_field(a2.dims, 12, 2002)
    if full:
        t0 = time.perf_counter()
        _, i2 = O.solve(a2, U2, b2, tol=1e-10)
        cg["dwf_moebius_16c16_ls12"] = {"seconds": round(time.perf_counter() - t0, 2),
                                        "iters": i2.iters, "measured": True}
    elif c2_iters:
        t_it, _ = per_iter(a2, U2, b2)
        cg["dwf_moebius_16c16_ls12"] = {"seconds_per_iter": round(t_it, 4),
                                        "extrapolated": f"per-iteration time x {c2_iters} "
                                                        f"iterations (the GPU CG's count at "
                                                        f"1e-10)",
                                        "seconds": round(c2_iters * t_it, 1), "measured": False}
    if gpu_iters:
        t_it, _ = per_iter(act, U, b, k=2)
        cg[w["name"]] = {"seconds_per_iter": round(t_it, 3), "measured": False,
                         "extrapolated": f"per-iteration time x {gpu_iters} iterations (the "
                                         f"GPU CG's count at 1e-10)",
                         "seconds": round(gpu_iters * t_it, 1)}
    out["cg_time_to_1e-10"] = cg
    return out


def c5b_dslash(args, log):
    """FP64 dslash on the 32^3x64, Ls=12 lattice (fields 2.4 GB per parity,
    far above the 256 MB Infinity Cache): HIP-event timing of the hop
    launches of a fixed number of CG iterations."""
    import torch

    from paper_1804_08593_amd import mspcg, synth

    w = WORKLOADS["dwf_moebius_32c64_ls12"]
    log("[bench] generating dwf_moebius_32c64_ls12 for the dslash leg")
    U = synth.gauge_field(w["dims"], w["eps"], w["gseed"])
    b = synth.fermion_field(w["dims"], w["Ls"], w["rseed"])
    ctx = mspcg.Context(w["dims"], w["Ls"], w["M5"], w["mf"], w["b"], w["c"])
    ctx.load_gauge(torch.from_numpy(U).cuda())
    del U
    bd = torch.from_numpy(b).cuda()
    del b
    x = torch.zeros_like(bd)
    tuning = None if args.no_autotune else ctx.autotune()
    p = mspcg.make_params(tol=1e-30, maxiter=40, solver=mspcg.SOLVER_CG, timing=True)
    ctx.solve(bd, x, p, allow_noconv=True)
    st = ctx.solve(bd, x, p, allow_noconv=True)
    res = {"workload": "dwf_moebius_32c64_ls12", "dims": list(w["dims"]), "Ls": w["Ls"],
           "cg_iterations_timed": st["outer_iters"], "tuning": tuning}
    for k in ("hop64", "hopcg"):
        n = st["kernel_launches"][k]
        if n:
            gbs = st["kernel_bytes"][k] / (st["kernel_ms"][k] * 1e-3) / 1e9
            res[k] = {"launches": n, "avg_us": round(1e3 * st["kernel_ms"][k] / n, 2),
                      "bytes_per_launch": round(st["kernel_bytes"][k] / n),
                      "GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    del bd, x, ctx
    torch.cuda.empty_cache()
    return res


def force_bytes(w, with_grad=True):
    """Algorithmic HBM bytes of the force kernel: the four FP64 half spinors
    a_e, a_o, b_e, b_o once, the forward links once, F (and the gradient)
    written once, 144 B per 3x3 complex matrix."""
    V4 = int(np.prod(w["dims"]))
    return 4 * (V4 // 2) * w["Ls"] * 192 + 4 * V4 * 144 * (3 if with_grad else 2)


def force_c5a(args, log, calls=10):
    """HMC force on 16^3x32, Ls=12 (mspcg_force: two packs, B X, two hops,
    the force kernel; F and the gradient both written): wall time per call
    (each call ends with a stream synchronisation)."""
    import torch

    from paper_1804_08593_amd import mspcg, synth

    w = WORKLOADS["dwf_moebius_16c32_ls12"]
    U = synth.gauge_field(w["dims"], w["eps"], w["gseed"])
    ctx = mspcg.Context(w["dims"], w["Ls"], w["M5"], w["mf"], w["b"], w["c"])
    ctx.load_gauge(torch.from_numpy(U).cuda())
    X = torch.from_numpy(synth.fermion_field(w["dims"], w["Ls"], w["rseed"])).cuda()
    Y = torch.from_numpy(synth.fermion_field(w["dims"], w["Ls"], w["rseed"] + 1)).cuda()
    F = torch.empty((4,) + tuple(reversed(w["dims"])) + (3, 3), dtype=torch.complex128,
                    device="cuda")
    G = torch.empty_like(F)
    ctx.force(X, Y, F, G)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        ctx.force(X, Y, F, G)
    ms = 1e3 * (time.perf_counter() - t0) / calls
    res = {"workload": "dwf_moebius_16c32_ls12", "dims": list(w["dims"]), "Ls": w["Ls"],
           "calls": calls, "ms_per_call": round(ms, 4),
           "force_kernel_bytes": force_bytes(w)}
    log(f"[bench] 16^3x32 force: {res['ms_per_call']} ms per call")
    del ctx, X, Y, F, G
    torch.cuda.empty_cache()
    return res


# six uneven lattices solved together: dims, Ls, mf (b=1.5, c=0.5, M5=1.8,
# links exp(0.25 i H)); gauge seed 1040 + i, source seed 2040 + i
BATCH = [((8, 8, 8, 8), 8, 0.05), ((12, 12, 12, 12), 12, 0.01), ((16, 16, 16, 16), 16, 0.05),
         ((12, 12, 12, 24), 8, 0.01), ((16, 16, 16, 32), 12, 0.05), ((20, 20, 20, 20), 16, 0.01)]


def batch_compare(args):
    """Batched MSPCG of the six lattices (blockings from the library's
    blocking autotuner) with the local solves' block hops as persistent
    multi-lattice launches (batch_kernels 0) and as one launch per lattice
    and stage (batch_kernels 1); median of 3 after one warm-up."""
    import torch

    from paper_1804_08593_amd import mspcg, synth

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    ctxs, bs = [], []
    base = mspcg.make_params(tol=args.tol, maxiter=3000, solver=mspcg.SOLVER_MSPCG,
                             inner_iters=args.inner_iters, inner_prec=mspcg.FP16)
    for i, (d, Ls, mf) in enumerate(BATCH):
        c = mspcg.Context(d, Ls, 1.8, mf, 1.5, 0.5)
        c.load_gauge(torch.from_numpy(synth.gauge_field(d, 0.25, 1040 + i)).cuda())
        blk = c.tune_blocking(base, probe_iters=6)
        log(f"[batch] {d} Ls={Ls}: blocking {blk}")
        ctxs.append(c)
        bs.append(torch.from_numpy(synth.fermion_field(d, Ls, 2040 + i)).cuda())
    for kern in (0, 1):
        p = mspcg.make_params(tol=args.tol, maxiter=3000, solver=mspcg.SOLVER_MSPCG,
                              inner_iters=args.inner_iters, inner_prec=mspcg.FP16,
                              batch_kernels=kern)
        times, sts = [], None
        for rep in range(4):
            xs = [torch.zeros_like(b) for b in bs]
            sts = mspcg.solve_batch(ctxs, bs, xs, p)
            if rep:
                times.append(sts[0]["seconds"])
        print(json.dumps({"batch_kernels": kern, "persistent": sts[0]["batch_persistent"],
                          "seconds": round(float(np.median(times)), 4),
                          "outer_iters": [st["outer_iters"] for st in sts],
                          "true_rel_resid": [st["true_rel_resid"] for st in sts]}), flush=True)
    # each lattice alone: eager mspcg_solve, and a one-system solve_batch
    # (graph-replayed iteration) with per-lattice and with persistent block
    # hops; median of 3 after one warm-up
    tot = 0.0
    for (d, Ls, mf), c, b in zip(BATCH, ctxs, bs):
        row = {"lattice": list(d), "Ls": Ls}
        for mode in ("eager", "graph_per_lattice", "graph_persistent"):
            times = []
            for rep in range(4):
                x = torch.zeros_like(b)
                if mode == "eager":
                    st = c.solve(b, x, base)
                else:
                    pb = mspcg.make_params(tol=args.tol, maxiter=3000, solver=mspcg.SOLVER_MSPCG,
                                           inner_iters=args.inner_iters, inner_prec=mspcg.FP16,
                                           batch_kernels=1 if mode == "graph_per_lattice" else 0)
                    st = mspcg.solve_batch([c], [b], [x], pb)[0]
                if rep:
                    times.append(st["seconds"])
            row[mode + "_seconds"] = round(float(np.median(times)), 4)
        tot += row["eager_seconds"]
        print(json.dumps(row), flush=True)
    print(json.dumps({"separate_solves_seconds": round(tot, 4)}), flush=True)


READINGS = [  # (name, pad, form): the block operator A_s of the preconditioner
    ("dirichlet", 0, 0),   # Mhat_s^+ Mhat_s, hops between blocks dropped
    ("pad1", 1, 0),        # P_s Mhat_W^+ Mhat_W P_s, W = block widened by one site
    ("split", 1, 1),       # (P_s Mhat P_s)^+ (P_s Mhat P_s)
    ("literal", 2, 0),     # P_s A P_s, the diagonal block of A (Sec. 2.3, Fig. 3)
]


def ritz_range(coef):
    """Extreme eigenvalues of the Lanczos tridiagonal of (P)CG coefficients
    (alpha_k, beta_k): T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
    T_j,j+1 = sqrt(beta_j)/alpha_j."""
    import scipy.linalg

    c = np.asarray(coef, dtype=float)
    a, b = c[:, 0], c[:, 1]
    d = 1.0 / a
    d[1:] += b[:-1] / a[:-1]
    e = np.sqrt(np.maximum(b[:-1], 0.0)) / a[:-1]
    ev = scipy.linalg.eigh_tridiagonal(d, e, eigvals_only=True)
    return float(ev[0]), float(ev[-1])


def sweep_readings(ctx, w, bd, x, args, log):
    """Outer iterations (the paper's global iterations, Sec. 3) and time of
    MSPCG for each block reading and l, beside plain CG, on one GPU."""
    from paper_1804_08593_amd import mspcg

    p_cg = mspcg.make_params(tol=args.tol, maxiter=20000, solver=mspcg.SOLVER_CG)
    ctx.solve(bd, x, p_cg)
    cg = ctx.solve(bd, x, p_cg, coef=20000)
    lo, hi = ritz_range(cg["cg_coef"])
    print(json.dumps({"workload": args.workload, "solver": "cg", "outer_iters": cg["outer_iters"],
                      "seconds": round(cg["seconds"], 4), "ritz": [lo, hi],
                      "kappa_eff": round(hi / lo, 1)}), flush=True)
    for name, pad, form in READINGS:
        for l in (2, 3, 4, 6, 8):
            p = mspcg.make_params(tol=args.tol, maxiter=20000, solver=mspcg.SOLVER_MSPCG,
                                  block=w["block"], pad=pad, form=form, inner_iters=l,
                                  inner_prec=mspcg.FP16)
            ctx.solve(bd, x, p)  # domain set-up, untimed
            st = ctx.solve(bd, x, p, coef=20000)
            lo, hi = ritz_range(st["cg_coef"])
            row = {"workload": args.workload, "solver": "mspcg", "reading": name,
                   "block": list(w["block"]), "l": l, "outer_iters": st["outer_iters"],
                   "ritz": [lo, hi], "kappa_eff": round(hi / lo, 2),
                   "g": round(cg["outer_iters"] / st["outer_iters"], 3),
                   "seconds": round(st["seconds"], 4),
                   "speedup_vs_cg": round(cg["seconds"] / st["seconds"], 3),
                   "true_rel_resid": st["true_rel_resid"]}
            print(json.dumps(row), flush=True)
            log(f"[sweep] {name} l={l}: {st['outer_iters']} it {st['seconds']:.3f} s")


def sweep_blocks(ctx, w, bd, x, args, log):
    """MSPCG (literal blocks, FP16 local solves) for several block shapes and
    l on the workload, beside plain CG; best of two solves without per-kernel
    timing."""
    from paper_1804_08593_amd import mspcg

    L = w["dims"]
    shapes = [tuple(w["block"]), (L[0], L[1], L[2] // 2, L[3] // 2), (L[0], L[1], L[2], L[3] // 2),
              (L[0] // 2, L[1], L[2], L[3])]
    p_cg = mspcg.make_params(tol=args.tol, maxiter=20000, solver=mspcg.SOLVER_CG)
    cg = min((ctx.solve(bd, x, p_cg) for _ in range(2)), key=lambda st: st["seconds"])
    print(json.dumps({"workload": args.workload, "solver": "cg", "outer_iters": cg["outer_iters"],
                      "seconds": round(cg["seconds"], 4)}), flush=True)
    for blk in shapes:
        for l in (2, 3, 4, 6, 8):
            p = mspcg.make_params(tol=args.tol, maxiter=20000, solver=mspcg.SOLVER_MSPCG,
                                  block=blk, pad=2, inner_iters=l, inner_prec=mspcg.FP16)
            ctx.solve(bd, x, p)  # domain set-up
            st = min((ctx.solve(bd, x, p) for _ in range(2)), key=lambda r: r["seconds"])
            row = {"workload": args.workload, "block": list(blk), "l": l,
                   "outer_iters": st["outer_iters"], "seconds": round(st["seconds"], 4),
                   "speedup_vs_cg": round(cg["seconds"] / st["seconds"], 3)}
            print(json.dumps(row), flush=True)
            log(f"[blocks] {blk} l={l}: {st['outer_iters']} it {st['seconds']:.3f} s")


def tuner_check(ctx, w, bd, x, args, log):
    """The block-shape tuner's candidates (every set of halved directions and
    one quartering) on the workload: the tuner's score (-log of the relative
    residual after 8 outer iterations per second), the slope over iterations
    8..24, and the true time to the tolerance; then the tuner's own pick."""
    from paper_1804_08593_amd import mspcg

    L = w["dims"]
    cands = [tuple(L[m] // 2 if (mask >> m) & 1 else L[m] for m in range(4)) for mask in range(1, 16)]
    cands.append(tuple(L[m] // 4 if L[m] >= 16 else L[m] // 2 for m in range(4)))
    rows = []
    for blk in cands:
        if any(L[m] % blk[m] or blk[m] % 2 or (L[m] != blk[m] and L[m] - blk[m] < 4)
               for m in range(4)):
            continue
        t, hist = {}, None
        for k in (8, 24):
            p = mspcg.make_params(tol=1e-300, maxiter=k, solver=mspcg.SOLVER_MSPCG, block=blk,
                                  pad=2, inner_iters=args.inner_iters, inner_prec=mspcg.FP16)
            if k == 8:
                ctx.solve(bd, x, p, allow_noconv=True)  # domain set-up
            st = ctx.solve(bd, x, p, allow_noconv=True, history=k)
            t[k] = st["seconds"]
            hist = st["history"]
        p = mspcg.make_params(tol=args.tol, maxiter=20000, solver=mspcg.SOLVER_MSPCG, block=blk,
                              pad=2, inner_iters=args.inner_iters, inner_prec=mspcg.FP16)
        st = min((ctx.solve(bd, x, p) for _ in range(2)), key=lambda r: r["seconds"])
        row = {"workload": args.workload, "block": list(blk),
               "score_8": round(-math.log(hist[7]) / t[8], 3),
               "slope_8_24": round((math.log(hist[7]) - math.log(hist[23])) / (t[24] - t[8]), 3),
               "outer_iters": st["outer_iters"], "seconds": round(st["seconds"], 4)}
        rows.append(row)
        print(json.dumps(row), flush=True)
        log(f"[tuner] {blk}: {st['outer_iters']} it {st['seconds']:.3f} s")
    base = mspcg.make_params(tol=args.tol, solver=mspcg.SOLVER_MSPCG, pad=2,
                             inner_iters=args.inner_iters, inner_prec=mspcg.FP16)
    blk, pad = ctx.tune_blocking(base)
    t0 = time.perf_counter()
    blk0, _ = ctx.tune_blocking(base, probe_iters=0)
    t_full = time.perf_counter() - t0
    ts = np.argsort(np.argsort([r["seconds"] for r in rows]))
    sc = np.argsort(np.argsort([-r["score_8"] for r in rows]))
    print(json.dumps({"workload": args.workload, "tuner_pick": list(blk),
                      "tuner_pick_full_solves": list(blk0), "full_solve_tuning_seconds": round(t_full, 1),
                      "fastest": min(rows, key=lambda r: r["seconds"])["block"],
                      "rank_correlation_score_8": round(float(np.corrcoef(ts, sc)[0, 1]), 3)}),
          flush=True)


def tile_sweep(ctx, w, bd, x, args, log):
    """FP64 dslash time for each traversal tile in --tiles (AxBxCxD,...):
    60 plain CG iterations with per-class HIP-event timing per tile."""
    from paper_1804_08593_amd import mspcg

    for t in args.tiles.split(","):
        tile = tuple(int(v) for v in t.split("x"))
        ctx.set_tuning(1, tile, (0, 0, 0, 0), (0, 0, 0, 0))
        p = mspcg.make_params(tol=1e-30, maxiter=60, solver=mspcg.SOLVER_CG, timing=True)
        ctx.solve(bd, x, p, allow_noconv=True)
        st = ctx.solve(bd, x, p, allow_noconv=True)
        row = {"workload": args.workload, "fp64_tile": list(tile)}
        for k in ("hop64", "hopcg"):
            n = st["kernel_launches"][k]
            if n:
                row[k + "_avg_us"] = round(1e3 * st["kernel_ms"][k] / n, 1)
        print(json.dumps(row), flush=True)
        log(f"[tiles] {tile}: {row}")


def multisplit_compare(ctx, w, bd, x, args, log, sweeps=400):
    """The multisplitting iteration itself (Sec. 2.1, eq. (2)) beside MSPCG
    with the same local solves (literal blocks, l = 6, FP16): residual after
    a number of sweeps and the contraction per sweep over the last 100."""
    from paper_1804_08593_amd import mspcg

    for blk in (tuple(w["block"]), tuple(w["dims"][:3]) + (w["dims"][3] // 2,)):
        kw = dict(tol=args.tol, block=blk, pad=2, inner_iters=args.inner_iters,
                  inner_prec=mspcg.FP16)
        ms = ctx.solve(bd, x, mspcg.make_params(maxiter=20000, solver=mspcg.SOLVER_MSPCG, **kw))
        st = ctx.solve(bd, x, mspcg.make_params(maxiter=sweeps, solver=mspcg.SOLVER_MULTISPLIT,
                                                 **kw), history=sweeps, allow_noconv=True)
        h = st["history"]
        row = {"workload": args.workload, "block": list(blk), "l": args.inner_iters,
               "mspcg_outer_iters": ms["outer_iters"], "mspcg_seconds": round(ms["seconds"], 4),
               "multisplit_sweeps": st["outer_iters"], "multisplit_seconds": round(st["seconds"], 4),
               "converged": st["converged"],
               "resid_at": {str(k): float(h[k - 1]) for k in (1, 10, 50, 100, 200, 400)
                            if k <= len(h)},
               "rate_per_sweep": float((h[-1] / h[-101]) ** 0.01) if len(h) > 101 else None}
        print(json.dumps(row), flush=True)
        log(f"[multisplit] {blk}: {row}")


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
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the oracle's 16^4x12 CG solve to the end (about a minute)")
    ap.add_argument("--no-c5b", action="store_true", help="skip the 32^3x64 dslash leg")
    ap.add_argument("--no-fp64-inner", action="store_true")
    ap.add_argument("--no-force", action="store_true", help="skip the 16^3x32 force leg")
    ap.add_argument("--force-only", action="store_true",
                    help="run only the 16^3x32 force leg and print its JSON line")
    ap.add_argument("--batch", action="store_true",
                    help="instead of the bench line: the six uneven lattices solved together "
                         "with persistent multi-lattice block hops and with one launch per "
                         "lattice, one JSON line per variant")
    ap.add_argument("--sweep-readings", action="store_true",
                    help="instead of the bench line: MSPCG with the workload's blocks for "
                         "every block reading (Dirichlet, pad 1, split Schur, literal) and "
                         "l = 2..8, one JSON line per solve")
    ap.add_argument("--tuner-check", action="store_true",
                    help="block-shape tuner's candidates: its score vs the true time to solve")
    ap.add_argument("--sweep-blocks", action="store_true",
                    help="MSPCG time per block shape and l on the workload, then exit")
    ap.add_argument("--tiles", default=None,
                    help="FP64 dslash time per traversal tile AxBxCxD,... on the workload, then exit")
    ap.add_argument("--multisplit", action="store_true",
                    help="multisplitting sweeps beside MSPCG on the workload, then exit")
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

    if args.batch:
        batch_compare(args)
        return
    if args.force_only:
        print(json.dumps(force_c5a(args, lambda *a: print(*a, file=sys.stderr, flush=True))),
              flush=True)
        return
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

    if args.sweep_readings:
        sweep_readings(ctx, w, bd, x, args, log)
        return
    if args.multisplit:
        multisplit_compare(ctx, w, bd, x, args, log)
        return
    if args.tiles:
        tile_sweep(ctx, w, bd, x, args, log)
        return
    if args.sweep_blocks:
        sweep_blocks(ctx, w, bd, x, args, log)
        return
    if args.tuner_check:
        tuner_check(ctx, w, bd, x, args, log)
        return

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
        # every candidate solved to the tolerance (the short-probe score misranks
        # blockings whose advantage shows only late in the solve)
        blk, pad = ctx_t.tune_blocking(mspcg.make_params(tol=args.tol, solver=mspcg.SOLVER_MSPCG,
                                                         pad=2, inner_iters=args.inner_iters,
                                                         inner_prec=mspcg.FP16), probe_iters=0)
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

    def class_split(st):
        """Per-class [launches, ms] of one solve and the share of its wall time
        the classes cover."""
        cl = {k: [st["kernel_launches"][k], round(v, 1)] for k, v in st["kernel_ms"].items()
              if st["kernel_launches"][k]}
        tot = sum(v for v in st["kernel_ms"].values())
        return {"classes": cl, "kernel_share_of_wall": round(1e-3 * tot / st["seconds"], 3)}

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
                                                         / max(1, last["mspcg"]["outer_iters"]), 3),
                         "kernel_time": class_split(last["mspcg"])}
    if run_mt:
        mt_s = float(np.median([r["mspcg_tuned"]["seconds"] for r in results]))
        line["mspcg_tuned_blocking"] = {"seconds": round(mt_s, 4), "blocking": tuned_block,
                                        "outer_iters": last["mspcg_tuned"]["outer_iters"],
                                        "inner_iters_total": last["mspcg_tuned"]["inner_iters_total"],
                                        "true_rel_resid": last["mspcg_tuned"]["true_rel_resid"],
                                        "speedup_vs_cg": round(cg_s / mt_s, 3),
                                        "kernel_time": class_split(last["mspcg_tuned"])}
    if run_ms and not args.no_fp64_inner:
        # the same MSPCG with FP64 local solves (untimed): its outer count is
        # the one the oracle's FP64 MSPCG reaches (within one iteration on the
        # lattices the oracle can solve)
        p64 = mspcg.make_params(tol=args.tol, maxiter=20000, solver=mspcg.SOLVER_MSPCG,
                                block=w["block"], pad=2, inner_iters=args.inner_iters,
                                inner_prec=mspcg.FP64)
        s64 = ctx.solve(bd, x, p64)
        line["mspcg_fp64_inner"] = {"outer_iters": s64["outer_iters"],
                                    "seconds": round(s64["seconds"], 4),
                                    "true_rel_resid": s64["true_rel_resid"]}
        log(f"[bench] FP64-inner MSPCG: {s64['outer_iters']} outer iterations")
    if not args.no_force:
        line["c5a_force"] = force_c5a(args, log)
    if not args.no_c5b:
        line["c5b_dslash"] = c5b_dslash(args, log)
        log(f"[bench] 32^3x64 dslash: {line['c5b_dslash'].get('hop64')}")
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        w = dict(w, name=args.workload)
        # the GPU CG's iteration count on 16^4x12 (scales the oracle's
        # per-iteration time there)
        w2 = WORKLOADS["dwf_moebius_16c16_ls12"]
        c2 = mspcg.Context(w2["dims"], w2["Ls"], w2["M5"], w2["mf"], w2["b"], w2["c"])
        c2.load_gauge(torch.from_numpy(synth.gauge_field(w2["dims"], w2["eps"],
                                                         w2["gseed"])).cuda())
        b2 = torch.from_numpy(synth.fermion_field(w2["dims"], w2["Ls"], w2["rseed"])).cuda()
        s2 = c2.solve(b2, torch.zeros_like(b2), mspcg.make_params(tol=args.tol, maxiter=20000))
        del c2, b2
        line["cpu_baseline"] = cpu_baseline(w, U, b, gpu_iters=last["cg"]["outer_iters"],
                                            c2_iters=s2["outer_iters"], full=args.cpu_full)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
