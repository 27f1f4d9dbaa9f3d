"""Batched solves of several uneven lattices with one hipGraph-captured outer
iteration replayed for all of them, against individual eager solves (every
replay is checked through the per-iteration residual history) and against
the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1804_08593_amd import mspcg, synth
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
    for rep in range(2):
        xs = [torch.zeros_like(b) for _, _, b in sys]
        sts = mspcg.solve_batch([c for c, _, _ in sys], [b for _, _, b in sys], xs, prm,
                                history=2000)
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


def test_config4_six_uneven_lattices():
    """8^4, 12^4, 16^4, 12^3x24, 16^3x32, 20^4 Moebius lattices with
    (Ls, mf) = (8,.05) (12,.01) (16,.05) (8,.01) (12,.05) (16,.01), links
    exp(0.25 i H), autotuned blocking, one batched MSPCG solve to 1e-10."""
    shapes = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16), (12, 12, 12, 24),
              (16, 16, 16, 32), (20, 20, 20, 20)]
    lsmf = [(8, 0.05), (12, 0.01), (16, 0.05), (8, 0.01), (12, 0.05), (16, 0.01)]
    sys = []
    base = mspcg.make_params(tol=1e-10, maxiter=3000, solver=mspcg.SOLVER_MSPCG, inner_iters=6,
                             inner_prec=mspcg.FP16, block=(0, 0, 0, 0))
    for i, (d, (Ls, mf)) in enumerate(zip(shapes, lsmf)):
        ctx, U, b = _make(d, Ls, mf, 0.25, 1040 + i, 2040 + i)
        blk = ctx.tune_blocking(base, probe_iters=6)
        say(f"lattice {d} Ls={Ls}: tuned blocking {blk}")
        sys.append((ctx, U, b))
    xs = [torch.zeros_like(b) for _, _, b in sys]
    sts = mspcg.solve_batch([c for c, _, _ in sys], [b for _, _, b in sys], xs, base)
    for (ctx, U, b), x, st in zip(sys, xs, sts):
        say(f"  {ctx.dims} Ls={ctx.Ls}: outer {st['outer_iters']} resid {st['true_rel_resid']:.2e}")
        assert st["converged"] and st["true_rel_resid"] <= 1e-10
        # re-measure the full-system residual |D x - b| / |b| with the GPU operator
        dx = torch.zeros_like(b)
        ctx.apply(mspcg.OP_D, x, dx)
        r = (torch.linalg.vector_norm(dx - b) / torch.linalg.vector_norm(b)).item()
        assert r <= 1e-8
    # the smallest lattice also against the oracle's operator
    ctx, U, b = sys[0]
    act = O.Action(ctx.dims, ctx.Ls, 1.8, 0.05, 1.5, 0.5)
    bh = host(b)
    _, bhat = O.prepare(act, U, bh)
    xe = O.parity_mask(act, host(xs[0]), 0)
    rr = np.sqrt(O.norm2(bhat - O.normal(act, U, xe)) / O.norm2(bhat))
    assert rr <= 1e-10
