"""Batched solves of several uneven lattices with one hipGraph-captured outer
iteration replayed for all of them, against individual eager solves (every
replay is checked through the per-iteration residual history) and against
the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1804_08593_amd import mspcg, synth
from tests._util import lanczos_kappa
from tests.gpu_util import dev, host, relerr, say

pytestmark = pytest.mark.gpu


def _make(dims, Ls, mf, eps, gseed, rseed, block=None):
    ctx = mspcg.Context(dims, Ls, 1.8, mf, 1.5, 0.5)
    U = synth.gauge_field(dims, eps, gseed)
    ctx.load_gauge(dev(U))
    if block is not None:
        ctx.set_blocking(block, 2)
    b = dev(synth.fermion_field(dims, Ls, rseed))
    return ctx, U, b


SMALL = [((8, 4, 4, 8), 8, 0.05, (4, 4, 4, 4)), ((4, 4, 4, 8), 12, 0.01, (4, 4, 4, 4)),
         ((8, 8, 4, 4), 4, 0.1, (4, 4, 4, 4))]


@pytest.mark.parametrize("solver", [mspcg.SOLVER_MSPCG, mspcg.SOLVER_CG])
def test_batch_equals_individual_solves(solver):
    sys = [_make(d, Ls, mf, 0.25, 60 + i, 70 + i, blk) for i, (d, Ls, mf, blk) in enumerate(SMALL)]
    prm = mspcg.make_params(tol=1e-10, maxiter=2000, solver=solver, inner_iters=4,
                            inner_prec=mspcg.FP16)
    # individual eager solves
    ref = []
    for ctx, U, b in sys:
        x = torch.zeros_like(b)
        st = ctx.solve(b, x, prm, history=2000)
        ref.append((x.clone(), st))
    # one batched, graph-replayed solve (run twice: replays of a fresh graph
    # after eager work in between must give the same answer)
    # the eager solutions against the oracle's solution at 1e-13
    for (ctx, U, b), (xr, sr), (d, Ls, mf, blk) in zip(sys, ref, SMALL):
        act = O.Action(d, Ls, 1.8, mf, 1.5, 0.5)
        x_or, _ = O.solve(act, U, host(b), tol=1e-13)
        err = relerr(host(xr), x_or)
        say(f"system {d} Ls={Ls}: |x - x_oracle| / |x_oracle| = {err:.2e}")
        assert err <= 1e-8
    for rep in range(2):
        xs = [torch.zeros_like(b) for _, _, b in sys]
        sts = mspcg.solve_batch([c for c, _, _ in sys], [b for _, _, b in sys], xs, prm,
                                history=2000)
        # Ls = 4 has no persistent multi-lattice kernel: per-lattice launches
        assert not any(st["batch_persistent"] for st in sts)
        for i, ((xr, sr), xb, sb) in enumerate(zip(ref, xs, sts)):
            say(f"rep {rep} system {i}: iters {sb['outer_iters']} (eager {sr['outer_iters']})")
            assert sb["converged"] and sb["true_rel_resid"] <= 1e-10
            assert sb["outer_iters"] == sr["outer_iters"]
            assert np.array_equal(sb["history"], sr["history"])  # every replay
            assert torch.equal(xb, xr)
        # eager work between the two batched runs
        ctx0, U0, b0 = sys[0]
        tmp = torch.zeros_like(b0)
        ctx0.apply(mspcg.OP_A, b0, tmp)
        torch.cuda.synchronize()


# Ls 8, 12 and 16: every block-hop stage of the three lattices' local solves
# runs as one persistent multi-lattice launch
MULTI = [((8, 4, 4, 8), 8, 0.05, (4, 4, 4, 4)), ((4, 4, 4, 8), 12, 0.01, (4, 4, 4, 4)),
         ((8, 8, 4, 8), 16, 0.1, (4, 4, 4, 4))]


@pytest.mark.parametrize("prec", [mspcg.FP16, mspcg.FP32, mspcg.FP64])
def test_persistent_multi_lattice_launch_matches_per_lattice_launches(prec):
    sys = [_make(d, Ls, mf, 0.25, 80 + i, 90 + i, blk) for i, (d, Ls, mf, blk) in enumerate(MULTI)]
    out = {}
    for kern in (0, 1):
        prm = mspcg.make_params(tol=1e-10, maxiter=2000, solver=mspcg.SOLVER_MSPCG,
                                inner_iters=4, inner_prec=prec, batch_kernels=kern)
        xs = [torch.zeros_like(b) for _, _, b in sys]
        sts = mspcg.solve_batch([c for c, _, _ in sys], [b for _, _, b in sys], xs, prm,
                                history=2000)
        out[kern] = (xs, sts)
        for st in sts:
            assert st["converged"] and st["true_rel_resid"] <= 1e-10
            assert st["batch_persistent"] == (kern == 0)
    bitwise = True
    for i, (d, Ls, mf, blk) in enumerate(MULTI):
        (xa, sa), (xb, sb) = (out[0][0][i], out[0][1][i]), (out[1][0][i], out[1][1][i])
        say(f"lattice {d} Ls={Ls}: persistent {sa['outer_iters']} it, per-lattice "
            f"{sb['outer_iters']} it")
        assert sa["outer_iters"] == sb["outer_iters"]
        assert np.allclose(sa["history"], sb["history"], rtol=1e-9, atol=0)
        assert relerr(host(xa), host(xb)) <= 1e-12
        bitwise = bitwise and torch.equal(xa, xb)
        # against the oracle
        act = O.Action(d, Ls, 1.8, mf, 1.5, 0.5)
        _, bhat = O.prepare(act, sys[i][1], host(sys[i][2]))
        r = bhat - O.normal(act, sys[i][1], O.parity_mask(act, host(xa), 0))
        assert np.sqrt(O.norm2(r) / O.norm2(bhat)) <= 1e-10 * 1.01
    say(f"persistent vs per-lattice launches bitwise identical: {bitwise}")


def test_persistent_batch_mixed_readings():
    """One persistent batch whose lattices use different readings of A_s
    (Dirichlet pad 0, the split form, pad 1): the same iterations and x as
    per-lattice launches, and oracle-checked residuals."""
    readings = [(0, mspcg.FORM_DOMAIN), (2, mspcg.FORM_SPLIT), (1, mspcg.FORM_DOMAIN)]
    sys = [_make(d, Ls, mf, 0.25, 80 + i, 90 + i) for i, (d, Ls, mf, _) in enumerate(MULTI)]
    for (ctx, _, _), (d, Ls, mf, blk), (pad, form) in zip(sys, MULTI, readings):
        ctx.set_blocking(blk, pad, form)
    out = {}
    for kern in (0, 1):
        prm = mspcg.make_params(tol=1e-10, maxiter=3000, solver=mspcg.SOLVER_MSPCG,
                                inner_iters=4, inner_prec=mspcg.FP16, batch_kernels=kern)
        xs = [torch.zeros_like(b) for _, _, b in sys]
        sts = mspcg.solve_batch([c for c, _, _ in sys], [b for _, _, b in sys], xs, prm)
        out[kern] = (xs, sts)
        for st in sts:
            assert st["converged"] and st["batch_persistent"] == (kern == 0)
    for i, (d, Ls, mf, blk) in enumerate(MULTI):
        (xa, sa), (xb, sb) = (out[0][0][i], out[0][1][i]), (out[1][0][i], out[1][1][i])
        say(f"lattice {d} Ls={Ls} pad/form {readings[i]}: persistent {sa['outer_iters']} it, "
            f"per-lattice {sb['outer_iters']} it")
        assert sa["outer_iters"] == sb["outer_iters"]
        assert relerr(host(xa), host(xb)) <= 1e-12
        act = O.Action(d, Ls, 1.8, mf, 1.5, 0.5)
        _, bhat = O.prepare(act, sys[i][1], host(sys[i][2]))
        r = bhat - O.normal(act, sys[i][1], O.parity_mask(act, host(xa), 0))
        assert np.sqrt(O.norm2(r) / O.norm2(bhat)) <= 1e-10 * 1.01


def test_persistent_batch_degenerate_members():
    """Degenerate batches on the persistent path: a member with a zero
    right-hand side (x = 0, no iterations, left out of the others' launches),
    a batch of zero right-hand sides only, and a batch of one lattice against
    its own eager solve and the oracle."""
    sys = [_make(d, Ls, mf, 0.25, 80 + i, 90 + i, blk) for i, (d, Ls, mf, blk) in enumerate(MULTI)]
    prm = mspcg.make_params(tol=1e-10, maxiter=2000, solver=mspcg.SOLVER_MSPCG, inner_iters=4,
                            inner_prec=mspcg.FP16)
    (c0, _, b0), (c1, _, b1), (c2, U2, b2) = sys
    say("reference: lattices 0 and 2 batched on their own")
    xr = [torch.zeros_like(b0), torch.zeros_like(b2)]
    sr = mspcg.solve_batch([c0, c2], [b0, b2], xr, prm, history=2000)
    say("lattice 1 with a zero right-hand side between them")
    xs = [torch.zeros_like(b0), torch.ones_like(b1), torch.zeros_like(b2)]
    sts = mspcg.solve_batch([c0, c1, c2], [b0, torch.zeros_like(b1), b2], xs, prm, history=2000)
    assert sts[1]["converged"] and sts[1]["outer_iters"] == 0
    assert torch.count_nonzero(xs[1]) == 0
    for j, i in ((0, 0), (1, 2)):
        say(f"  lattice {i}: {sts[i]['outer_iters']} it (without lattice 1: {sr[j]['outer_iters']})")
        assert sts[i]["batch_persistent"] and sr[j]["batch_persistent"]
        assert sts[i]["converged"] and sts[i]["true_rel_resid"] <= 1e-10
        assert sts[i]["outer_iters"] == sr[j]["outer_iters"]
        assert relerr(host(xs[i]), host(xr[j])) <= 1e-12
    say("zero right-hand sides only")
    xz = [torch.ones_like(b0), torch.ones_like(b1)]
    sz = mspcg.solve_batch([c0, c1], [torch.zeros_like(b0), torch.zeros_like(b1)], xz, prm)
    for st, x in zip(sz, xz):
        assert st["converged"] and st["outer_iters"] == 0
        assert torch.count_nonzero(x) == 0
    say("one lattice: batch against eager solve and oracle")
    xb = [torch.zeros_like(b2)]
    sb = mspcg.solve_batch([c2], [b2], xb, prm, history=2000)[0]
    xe = torch.zeros_like(b2)
    se = c2.solve(b2, xe, prm, history=2000)
    say(f"  batch {sb['outer_iters']} it, eager {se['outer_iters']} it")
    assert sb["batch_persistent"] and sb["converged"]
    assert sb["outer_iters"] == se["outer_iters"]
    assert relerr(host(xb[0]), host(xe)) <= 1e-12
    d, Ls, mf, _ = MULTI[2]
    act = O.Action(d, Ls, 1.8, mf, 1.5, 0.5)
    _, bhat = O.prepare(act, U2, host(b2))
    r = bhat - O.normal(act, U2, O.parity_mask(act, host(xb[0]), 0))
    assert np.sqrt(O.norm2(r) / O.norm2(bhat)) <= 1e-10 * 1.01


C4_SHAPES = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16), (12, 12, 12, 24),
             (16, 16, 16, 32), (20, 20, 20, 20)]
C4_LSMF = [(8, 0.05), (12, 0.01), (16, 0.05), (8, 0.01), (12, 0.05), (16, 0.01)]


@pytest.fixture(scope="module")
def c4():
    """8^4, 12^4, 16^4, 12^3x24, 16^3x32, 20^4 Moebius lattices with
    (Ls, mf) = (8,.05) (12,.01) (16,.05) (8,.01) (12,.05) (16,.01), links
    exp(0.25 i H), autotuned blocking, one batched MSPCG solve to 1e-10."""
    sys = []
    base = mspcg.make_params(tol=1e-10, maxiter=3000, solver=mspcg.SOLVER_MSPCG, inner_iters=6,
                             inner_prec=mspcg.FP16, block=(0, 0, 0, 0))
    for i, (d, (Ls, mf)) in enumerate(zip(C4_SHAPES, C4_LSMF)):
        ctx, U, b = _make(d, Ls, mf, 0.25, 1040 + i, 2040 + i)
        blk = ctx.tune_blocking(base, probe_iters=6)
        say(f"lattice {d} Ls={Ls}: tuned blocking {blk}")
        sys.append((ctx, U, b, mf))
    xs = [torch.zeros_like(b) for _, _, b, _ in sys]
    sts = mspcg.solve_batch([c for c, _, _, _ in sys], [b for _, _, b, _ in sys], xs, base)
    return sys, xs, sts


def test_config4_six_uneven_lattices(c4):
    sys, xs, sts = c4
    for (ctx, U, b, mf), x, st in zip(sys, xs, sts):
        say(f"  {ctx.dims} Ls={ctx.Ls}: outer {st['outer_iters']} resid {st['true_rel_resid']:.2e}")
        assert st["converged"] and st["true_rel_resid"] <= 1e-10
        assert st["batch_persistent"]  # one persistent launch per block-hop stage
    say(f"  batched solve {sts[0]['seconds']:.3f} s")


@pytest.mark.parametrize("i", range(len(C4_SHAPES)))
def test_config4_lattice_against_oracle(c4, i):
    """Every batched lattice: the Schur residual of its x re-measured by the
    oracle, the full-system residual |D x - b| on sampled sites by the
    oracle, and the distance to an FP64 CG solution at 1e-12 within the
    kappa-qualified bound kappa (r_1 + r_2) (kappa from that CG's Lanczos
    coefficients, r the oracle-measured relative residuals)."""
    sys, xs, sts = c4
    ctx, U, b, mf = sys[i]
    x = xs[i]
    act = O.Action(ctx.dims, ctx.Ls, 1.8, mf, 1.5, 0.5)
    bh = host(b)
    _, bhat = O.prepare(act, U, bh)
    nb = np.sqrt(O.norm2(bhat))
    xe = O.parity_mask(act, host(x), 0)
    r_b = np.sqrt(O.norm2(bhat - O.normal(act, U, xe))) / nb
    xc = torch.zeros_like(b)
    sc = ctx.solve(b, xc, mspcg.make_params(tol=1e-12, maxiter=5000, solver=mspcg.SOLVER_CG),
                   coef=5000)
    kappa, lo, hi = lanczos_kappa(sc["cg_coef"])
    xce = O.parity_mask(act, host(xc), 0)
    r_c = np.sqrt(O.norm2(bhat - O.normal(act, U, xce))) / nb
    err = relerr(xe, xce)
    rng = np.random.default_rng(100 + i)
    sites = np.sort(rng.choice(act.V4, size=min(500, act.V4), replace=False))
    dx = O.dwf_sites(act, U, host(x), sites)
    bs = bh.reshape(act.Ls, act.V4, 4, 3)[:, sites]
    r_full = relerr(dx, bs)
    say(f"  {ctx.dims} Ls={ctx.Ls}: oracle resid {r_b:.2e} (CG {r_c:.2e}), kappa {kappa:.3g}, "
        f"|x - x_cg|/|x| {err:.2e} <= {kappa * (r_b + r_c):.2e}, sampled |Dx-b|/|b| {r_full:.2e}")
    assert r_b <= 1e-10 * 1.01 and r_c <= 1e-12 * 1.01
    assert err <= kappa * (r_b + r_c)
    assert r_full <= 1e-8
