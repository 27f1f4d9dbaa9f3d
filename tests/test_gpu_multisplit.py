"""GPU multisplitting iteration (Sec. 2.1, eq. (2)) against the oracle's
sweeps, and its slow convergence beside MSPCG (Sec. 2.2)."""
import functools

import numpy as np
import pytest
import torch

import oracle as O
from paper_1804_08593_amd import mspcg, synth
from tests.gpu_util import cg16_bars, dev, host, relerr, say, setup, site_err

pytestmark = pytest.mark.gpu

DIMS, LS = (8, 4, 4, 8), 4
BLK2 = (8, 4, 4, 4)  # two blocks, t cut


@functools.lru_cache(maxsize=None)
def _ref(sweeps, l):
    act = O.Action(DIMS, LS, 1.8, 0.05, 1.5, 0.5)
    U = synth.gauge_field(DIMS, 0.25, 71)
    bh = O.parity_mask(act, synth.fermion_field(DIMS, LS, 72), 0)
    x, hist = O.multisplitting(act, U, bh, BLK2, l, sweeps)
    return bh, x, np.array(hist)


@pytest.mark.parametrize("sweeps", [1, 3])
@pytest.mark.parametrize("prec", [mspcg.FP64, mspcg.FP32, mspcg.FP16])
def test_multisplitting_sweeps_match_oracle(sweeps, prec):
    act, U, ctx = setup(DIMS, LS, 1.8, 0.05, 1.5, 0.5, eps=0.25, gseed=71)
    bh, x_ref, h_ref = _ref(sweeps, 8)
    x = torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda")
    st = ctx.solve(dev(bh), x, mspcg.make_params(tol=1e-30, maxiter=sweeps,
                                                 solver=mspcg.SOLVER_MULTISPLIT, block=BLK2,
                                                 pad=2, inner_iters=8, inner_prec=prec,
                                                 rhs_normal=True), history=16,
                   allow_noconv=True)
    assert st["rc"] == mspcg.ENOCONV and st["outer_iters"] == sweeps
    got = host(x)
    err, serr = relerr(got, x_ref), site_err(got, x_ref)
    herr = np.max(np.abs(st["history"] - h_ref[1:]) / h_ref[1:])
    say(f"multisplitting {sweeps} sweeps prec={prec}: x relerr {err:.2e} (entry {serr:.2e}), "
        f"residual history relerr {herr:.2e}")
    if prec == mspcg.FP64:
        assert err <= 1e-11 and serr <= 1e-10 and herr <= 1e-10
    elif prec == mspcg.FP32:
        # the FP32 local-CG bar (1e-4, as for mspcg_precond) once per sweep
        bar = sweeps * 1e-4
        assert err <= bar and herr <= bar
    else:
        # every sweep repeats the l-step local solve's FP16 roundings
        bar = sweeps * cg16_bars(8)[0]
        assert err <= bar and herr <= bar


def test_multisplitting_converges_slowly_to_the_solution():
    """Two blocks: the sweeps converge (to the oracle's solution) but need
    many more global iterations than MSPCG with the same local solves."""
    act, U, ctx = setup(DIMS, LS, 1.8, 0.05, 1.5, 0.5, eps=0.25, gseed=71)
    bh = O.parity_mask(act, synth.fermion_field(DIMS, LS, 72), 0)
    x = torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda")
    kw = dict(tol=1e-10, maxiter=1000, block=BLK2, pad=2, inner_iters=8,
              inner_prec=mspcg.FP64, rhs_normal=True)
    st = ctx.solve(dev(bh), x, mspcg.make_params(solver=mspcg.SOLVER_MULTISPLIT, **kw))
    xm = torch.zeros_like(x)
    sm = ctx.solve(dev(bh), xm, mspcg.make_params(solver=mspcg.SOLVER_MSPCG, **kw))
    say(f"multisplitting {st['outer_iters']} sweeps vs MSPCG {sm['outer_iters']} iterations")
    assert st["converged"] and st["true_rel_resid"] <= 1e-10
    assert st["outer_iters"] > 2 * sm["outer_iters"]
    x_ref, _ = O.cg(act, U, bh, tol=1e-13)
    assert relerr(host(x), x_ref) <= 1e-8
    r = bh - O.normal(act, U, host(x))
    assert np.sqrt(O.norm2(r) / O.norm2(bh)) <= 1e-10 * 1.01


def test_multisplitting_rejected_in_batch():
    act, U, ctx = setup(DIMS, LS, 1.8, 0.05, 1.5, 0.5, eps=0.25, gseed=71)
    b = dev(synth.fermion_field(DIMS, LS, 73))
    with pytest.raises(mspcg.MspcgError) as e:
        mspcg.solve_batch([ctx], [b], [torch.zeros_like(b)],
                          mspcg.make_params(solver=mspcg.SOLVER_MULTISPLIT, block=BLK2))
    assert e.value.code == mspcg.EUNSUPPORTED
