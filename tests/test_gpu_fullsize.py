"""Parity at the full workload sizes, in the launch configuration bench.py
times (production tuning: XCD remap and traversal tiles).

24^3x48, Ls=16: D and D^+ against the oracle on the whole lattice, A against
the oracle's normal operator, and the bench's MSPCG / CG solves with their
true residual re-measured by the oracle.  16^4x12: mixed-precision vs FP64 CG.
32^3x64, Ls=12: the hop on sampled sites, and MSPCG to 1e-10 with 16 and with 128
blocks."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1804_08593_amd import mspcg, synth
from tests._util import lanczos_kappa
from tests.gpu_util import dev, host, relerr, say, setup

pytestmark = pytest.mark.gpu

C3 = dict(dims=(24, 24, 24, 48), Ls=16, mf=0.005, eps=0.2, gseed=1003, rseed=2003,
          block=(12, 12, 12, 24))


@pytest.fixture(scope="module")
def c3():
    say("generating 24^3x48 x 16 inputs")
    act, U, ctx = setup(C3["dims"], C3["Ls"], 1.8, C3["mf"], 1.5, 0.5, eps=C3["eps"],
                        gseed=C3["gseed"])
    b = synth.fermion_field(C3["dims"], C3["Ls"], C3["rseed"])
    return act, U, ctx, b


def test_c3_operator_parity_full_lattice(c3):
    act, U, ctx, b = c3
    bd = dev(b)
    out = torch.zeros_like(bd)
    for op, ref in ((mspcg.OP_D, lambda: O.dwf(act, U, b)),
                    (mspcg.OP_DDAG, lambda: O.dwf(act, U, b, dagger=True))):
        ctx.apply(op, bd, out)
        err = relerr(host(out), ref())
        say(f"  full-size op {op}: relerr {err:.2e}")
        assert err <= 1e-13
    ctx.apply(mspcg.OP_A, bd, out)
    err = relerr(host(out), O.normal(act, U, O.parity_mask(act, b, 0)))
    say(f"  full-size A: relerr {err:.2e}")
    assert err <= 1e-13


def test_c3_mspcg_and_cg_solves(c3):
    act, U, ctx, b = c3
    bd = dev(b)
    xm = torch.zeros_like(bd)
    sm = ctx.solve(bd, xm, mspcg.make_params(tol=1e-10, solver=mspcg.SOLVER_MSPCG,
                                             block=C3["block"], pad=2, inner_iters=6,
                                             inner_prec=mspcg.FP16))
    xc = torch.zeros_like(bd)
    sc = ctx.solve(bd, xc, mspcg.make_params(tol=1e-12, solver=mspcg.SOLVER_CG), coef=5000)
    say(f"  MSPCG {sm['outer_iters']} it, CG(1e-12) {sc['outer_iters']} it")
    assert sm["converged"] and sc["converged"]
    assert sm["outer_iters"] < sc["outer_iters"]
    _, bhat = O.prepare(act, U, b)
    nb = np.sqrt(O.norm2(bhat))
    res, xev = [], []
    for x, tol in ((xm, 1e-10), (xc, 1e-12)):
        xe = O.parity_mask(act, host(x), 0)
        r = bhat - O.normal(act, U, xe)
        rel = np.sqrt(O.norm2(r)) / nb
        say(f"  oracle true residual {rel:.2e}")
        assert rel <= tol * 1.01
        res.append(rel)
        xev.append(xe)
    # solution error qualified by the condition number (kappa from the CG's
    # Lanczos coefficients): |x1 - x2| / |x| <= kappa (r1 + r2)
    kappa, lo, hi = lanczos_kappa(sc["cg_coef"])
    err_e = relerr(xev[0], xev[1])
    bound = kappa * (res[0] + res[1])
    err = relerr(host(xm), host(xc))
    say(f"  kappa(A) ~ {kappa:.4g} (spectrum [{lo:.3g}, {hi:.3g}]); even-site "
        f"|x_mspcg - x_cg| / |x| = {err_e:.2e} <= {bound:.2e}; full x {err:.2e}")
    assert err_e <= bound
    assert err <= 1e-7


def test_c2_mixed_precision_vs_fp64_cg():
    dims, Ls = (16, 16, 16, 16), 12
    act, U, ctx = setup(dims, Ls, 1.8, 0.01, 1.5, 0.5, eps=0.2, gseed=1002)
    b = synth.fermion_field(dims, Ls, 2002)
    bd = dev(b)
    x64 = torch.zeros_like(bd)
    s64 = ctx.solve(bd, x64, mspcg.make_params(tol=1e-10, solver=mspcg.SOLVER_CG))
    x32 = torch.zeros_like(bd)
    s32 = ctx.solve(bd, x32, mspcg.make_params(tol=1e-10, solver=mspcg.SOLVER_MIXED_CG))
    say(f"  CG {s64['outer_iters']} it {s64['seconds']:.3f} s; mixed {s32['outer_iters']} it "
        f"{s32['seconds']:.3f} s ({s32['restarts']} reliable updates)")
    assert s64["converged"] and s32["converged"]
    _, bhat = O.prepare(act, U, b)
    for x in (x64, x32):
        r = bhat - O.normal(act, U, O.parity_mask(act, host(x), 0))
        assert np.sqrt(O.norm2(r) / O.norm2(bhat)) <= 1e-10
    assert relerr(host(x32), host(x64)) <= 1e-7


@pytest.fixture(scope="module")
def c5b():
    dims, Ls = (32, 32, 32, 64), 12
    say("generating 32^3x64 x 12 inputs")
    act, U, ctx = setup(dims, Ls, 1.8, 0.01, 1.5, 0.5, eps=0.2, gseed=1006)
    b = synth.fermion_field(dims, Ls, 2006)
    return act, U, ctx, b


def test_c5b_hop_sampled_sites(c5b):
    act, U, ctx, b = c5b
    bd = dev(b)
    out = torch.zeros_like(bd)
    ctx.apply(mspcg.OP_HOP, bd, out)
    rng = np.random.default_rng(5)
    sites = np.sort(rng.choice(act.V4, size=2000, replace=False))
    ref = O.hop_sites(act, U, b, sites)
    got = host(out).reshape(act.Ls, act.V4, 4, 3)[:, sites]
    err = relerr(got, ref)
    say(f"  32^3x64 hop on 2000 sampled sites: relerr {err:.2e}")
    assert err <= 1e-13


# 16 blocks of 16^3x32, and 128 blocks of 8x8x16x16 (one per node of the
# 128-node run of Sec. 3)
@pytest.mark.parametrize("block", [(16, 16, 16, 32), (8, 8, 16, 16)])
def test_c5b_mspcg_32c64(c5b, block):
    act, U, ctx, b = c5b
    bd = dev(b)
    x = torch.zeros_like(bd)
    st = ctx.solve(bd, x, mspcg.make_params(tol=1e-10, solver=mspcg.SOLVER_MSPCG,
                                            block=block, pad=2, inner_iters=6,
                                            inner_prec=mspcg.FP16))
    say(f"  32^3x64 MSPCG blocks {block}: {st['outer_iters']} it, {st['seconds']:.2f} s, "
        f"resid {st['true_rel_resid']:.2e}")
    assert st["converged"] and st["true_rel_resid"] <= 1e-10
    dx = torch.zeros_like(bd)
    ctx.apply(mspcg.OP_D, x, dx)
    r = (torch.linalg.vector_norm(dx - bd) / torch.linalg.vector_norm(bd)).item()
    say(f"  |D x - b| / |b| = {r:.2e}")
    assert r <= 1e-8
    # the same residual measured by the oracle's D on 2000 sampled sites
    del dx
    rng = np.random.default_rng(7)
    sites = np.sort(rng.choice(act.V4, size=2000, replace=False))
    dxs = O.dwf_sites(act, U, host(x), sites)
    bs = b.reshape(act.Ls, act.V4, 4, 3)[:, sites]
    rs = relerr(dxs, bs)
    say(f"  oracle |D x - b| / |b| on 2000 sampled sites = {rs:.2e}")
    assert rs <= 1e-8
