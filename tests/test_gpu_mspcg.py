"""GPU parity of the multisplitting preconditioner (Sec. 2.3), its sloppy
local CG and the MSPCG / mixed-precision solves against the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1804_08593_amd import mspcg, synth
from oracle.spectral import ritz_from_coef
from tests.gpu_util import cg16_bars, dev, host, k16_bars, relerr, say, setup, site_err

pytestmark = pytest.mark.gpu

# dims, Ls, block: x and t are cut into two blocks, y and z span the lattice
GEOM = ((8, 4, 4, 8), 8, (4, 4, 4, 4))
KTOL = {mspcg.FP64: (1e-13, 1e-12), mspcg.FP32: (1e-5, 1e-4), mspcg.FP16: k16_bars()}


@pytest.mark.parametrize("prec", [mspcg.FP64, mspcg.FP32, mspcg.FP16])
@pytest.mark.parametrize("pad,mode", [(2, "literal"), (0, "dirichlet")])
def test_block_operator_parity(prec, pad, mode):
    dims, Ls, blk = GEOM
    say(f"block operator prec={prec} pad={pad}")
    act, U, ctx = setup(dims, Ls, 1.8, 0.05, 1.5, 0.5, gseed=11)
    ctx.set_blocking(blk, pad)
    psi = O.parity_mask(act, synth.fermion_field(dims, Ls, 12), 0)
    out = torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda")
    ctx.apply(mspcg.OP_KBLOCK, dev(psi), out, prec=prec)
    ref = O.block_precond_op(act, U, psi, blk, mode)
    got = host(out)
    err, serr = relerr(got, ref), site_err(got, ref)
    say(f"  relerr {err:.3e} max entry err {serr:.3e}")
    assert err <= KTOL[prec][0] and serr <= KTOL[prec][1]


def test_block_operator_pad1_between_cut_and_literal():
    """pad = 1 keeps the out-and-back paths through nearest neighbours only."""
    dims, Ls, blk = GEOM
    act, U, ctx = setup(dims, Ls, 1.8, 0.05, 1.5, 0.5, gseed=11)
    psi = O.parity_mask(act, synth.fermion_field(dims, Ls, 12), 0)
    outs = {}
    for pad in (0, 1, 2):
        ctx.set_blocking(blk, pad)
        out = torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda")
        ctx.apply(mspcg.OP_KBLOCK, dev(psi), out)
        outs[pad] = host(out)
    lit = O.block_precond_op(act, U, psi, blk, "literal")
    assert relerr(outs[1], lit) < relerr(outs[0], lit)
    assert relerr(outs[2], lit) < 1e-13


ITOL = {mspcg.FP64: lambda l: (1e-11, 1e-10), mspcg.FP32: lambda l: (1e-4, 1e-3),
        mspcg.FP16: cg16_bars}


@pytest.mark.parametrize("prec", [mspcg.FP64, mspcg.FP32, mspcg.FP16])
@pytest.mark.parametrize("l", [1, 6])
def test_inner_block_cg_parity(prec, l):
    dims, Ls, blk = GEOM
    act, U, ctx = setup(dims, Ls, 1.8, 0.05, 1.5, 0.5, gseed=13)
    ctx.set_blocking(blk, 2)
    r = O.parity_mask(act, synth.fermion_field(dims, Ls, 14), 0)
    z = torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda")
    ctx.precond(dev(r), z, l, prec=prec)
    ref = O.inner_block_cg(act, U, r, blk, l, "literal")
    got = host(z)
    err, serr = relerr(got, ref), site_err(got, ref)
    say(f"inner CG prec={prec} l={l} relerr {err:.3e} max entry err {serr:.3e}")
    tol, stol = ITOL[prec](l)
    assert err <= tol and serr <= stol


def test_inner_block_cg_zero_block_and_l0():
    dims, Ls, blk = GEOM
    act, U, ctx = setup(dims, Ls, 1.8, 0.05, 1.5, 0.5, gseed=13)
    ctx.set_blocking(blk, 2)
    r = O.parity_mask(act, synth.fermion_field(dims, Ls, 15), 0)
    ids = O.block_ids(act, blk)
    r[:, ids == 1] = 0  # one block with zero residual
    z = torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda")
    ctx.precond(dev(r), z, 4, prec=mspcg.FP16)
    zh = host(z)
    assert np.all(np.isfinite(zh)) and np.all(zh[:, ids == 1] == 0)
    ctx.precond(dev(r), z, 0, prec=mspcg.FP16)
    assert torch.count_nonzero(z) == 0


@pytest.mark.parametrize("prec", [mspcg.FP64, mspcg.FP16])
def test_mspcg_solve_matches_oracle(prec):
    dims, Ls, blk = GEOM
    act, U, ctx = setup(dims, Ls, 1.8, 0.05, 1.5, 0.5, eps=0.25, gseed=17)
    b = synth.fermion_field(dims, Ls, 18)
    x = torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda")
    prm = mspcg.make_params(tol=1e-10, maxiter=500, solver=mspcg.SOLVER_MSPCG, block=blk, pad=2,
                            inner_iters=4, inner_prec=prec)
    st = ctx.solve(dev(b), x, prm, history=500)
    say("mspcg", prec, {k: st[k] for k in ("outer_iters", "true_rel_resid", "restarts")})
    assert st["converged"] and st["true_rel_resid"] <= 1e-10
    xg = host(x)
    _, bhat = O.prepare(act, U, b)
    r = bhat - O.normal(act, U, O.parity_mask(act, xg, 0))
    assert np.sqrt(O.norm2(r) / O.norm2(bhat)) <= 1e-10
    x_ref, _ = O.solve(act, U, b, tol=1e-13)
    assert relerr(xg, x_ref) <= 1e-8
    _, info_cg = O.solve(act, U, b, tol=1e-10)
    assert st["outer_iters"] < info_cg.iters  # fewer global iterations than CG (Sec. 3)
    if prec == mspcg.FP64:
        _, info = O.solve(act, U, b, tol=1e-10, precond=(blk, 4, "literal"))
        assert abs(st["outer_iters"] - info.iters) <= 1
    assert st["inner_iters_total"] >= 4 * st["outer_iters"]


def test_mspcg_coefficients_match_oracle():
    """The outer flexible PCG's (alpha, beta) per iteration, which define the
    Lanczos estimate of the spectrum of K_l^-1 A, against the oracle's MSPCG
    with the same FP64 local solves (literal blocks, l = 4)."""
    dims, Ls, blk = GEOM
    act, U, ctx = setup(dims, Ls, 1.8, 0.05, 1.5, 0.5, gseed=23)
    bh = O.parity_mask(act, synth.fermion_field(dims, Ls, 24), 0)
    x = torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda")
    st = ctx.solve(dev(bh), x, mspcg.make_params(tol=1e-10, maxiter=500,
                                                 solver=mspcg.SOLVER_MSPCG, block=blk, pad=2,
                                                 inner_iters=4, inner_prec=mspcg.FP64,
                                                 rhs_normal=True), coef=500)
    _, info = O.mspcg(act, U, bh, blk, 4, tol=1e-10)
    got, ref = np.asarray(st["cg_coef"]), np.asarray(info.coef)
    n = min(len(got), len(ref))
    say(f"MSPCG coefficients: GPU {len(got)}, oracle {len(ref)} iterations")
    assert n >= 10 and abs(len(got) - len(ref)) <= 1
    early = np.abs(got[:10] - ref[:10]) / np.abs(ref[:10]).max(axis=0)
    assert early.max() <= 1e-9
    rg, rr = ritz_from_coef(got[:n]), ritz_from_coef(ref[:n])
    lg, hg, lr, hr = rg[0], rg[-1], rr[0], rr[-1]
    say(f"  Ritz range GPU [{lg:.4g}, {hg:.4g}], oracle [{lr:.4g}, {hr:.4g}]")
    assert abs(lg - lr) <= 1e-3 * lr and abs(hg - hr) <= 1e-3 * hr


def test_mixed_precision_cg():
    dims, Ls = (8, 4, 4, 8), 12
    act, U, ctx = setup(dims, Ls, 1.8, 0.01, 1.5, 0.5, eps=0.2, gseed=19)
    b = synth.fermion_field(dims, Ls, 20)
    x = torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda")
    st = ctx.solve(dev(b), x, mspcg.make_params(tol=1e-10, maxiter=2000,
                                                solver=mspcg.SOLVER_MIXED_CG, delta=0.1))
    say("mixed", {k: st[k] for k in ("outer_iters", "true_rel_resid", "restarts")})
    assert st["converged"] and st["true_rel_resid"] <= 1e-10
    assert st["restarts"] >= 2  # reliable updates happened
    x_ref, _ = O.solve(act, U, b, tol=1e-13)
    assert relerr(host(x), x_ref) <= 1e-8


def test_solver_parameter_validation():
    dims, Ls, blk = GEOM
    act, U, ctx = setup(dims, Ls, 1.8, 0.05, 1.5, 0.5)
    b = dev(synth.fermion_field(dims, Ls, 1))
    x = torch.zeros_like(b)
    for bad in [dict(block=(3, 4, 4, 4)), dict(block=(4, 4, 4, 4), pad=3),
                dict(block=(4, 4, 4, 4), inner_prec=7), dict(block=(8, 4, 4, 6))]:
        prm = mspcg.make_params(solver=mspcg.SOLVER_MSPCG, **bad)
        with pytest.raises(mspcg.MspcgError) as e:
            ctx.solve(b, x, prm)
        assert e.value.code == mspcg.EINVAL
    with pytest.raises(mspcg.MspcgError):
        ctx.set_blocking((4, 4, 4, 3), 2)
