"""Traversal tiling and the autotuner change only the order in which output
sites are visited: results must be bitwise identical."""
import pytest
import torch

import oracle as O
from paper_1804_08593_amd import mspcg, synth
from tests.gpu_util import dev, host, relerr, say, setup

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tile", [(0, 0, 0, 0), (4, 2, 2, 2), (8, 4, 4, 4), (2, 2, 2, 2)])
@pytest.mark.parametrize("remap", [0, 1])
def test_tiles_are_bitwise_identical(tile, remap):
    dims, Ls, blk = (8, 4, 4, 8), 8, (4, 4, 4, 4)
    act, U, ctx = setup(dims, Ls, 1.8, 0.05, 1.5, 0.5, gseed=31)
    psi = O.parity_mask(act, synth.fermion_field(dims, Ls, 32), 0)
    d = dev(psi)
    ref = torch.zeros_like(d)
    ctx.set_tuning(1, (0, 0, 0, 0), (0, 0, 0, 0), (0, 0, 0, 0))
    ctx.apply(mspcg.OP_A, d, ref)
    ctx.set_blocking(blk, 2)
    kref = torch.zeros_like(d)
    ctx.apply(mspcg.OP_KBLOCK, d, kref, prec=mspcg.FP16)
    ctx.set_tuning(remap, tile, tile, tile)
    out = torch.zeros_like(d)
    ctx.apply(mspcg.OP_A, d, out)
    assert torch.equal(out, ref)
    kout = torch.zeros_like(d)
    ctx.apply(mspcg.OP_KBLOCK, d, kout, prec=mspcg.FP16)
    assert torch.equal(kout, kref)
    assert relerr(host(out), O.normal(act, U, psi)) <= 1e-13


def test_autotune_and_cache(tmp_path):
    dims, Ls, blk = (8, 8, 8, 8), 8, (4, 4, 4, 4)
    act, U, ctx = setup(dims, Ls, 1.8, 0.05, 1.5, 0.5, gseed=33)
    cache = str(tmp_path / "tune.txt")
    t1 = ctx.autotune(blk, 2, cache)
    say("autotune", t1)
    for k in ("fp64", "fp32", "fp16"):
        assert all(v % 2 == 0 and v >= 0 for v in t1["tile"][k])
    assert open(cache).read().count("|") == 1
    # a second context finds the cached choice without re-tuning
    ctx2 = mspcg.Context(dims, Ls, 1.8, 0.05, 1.5, 0.5)
    ctx2.load_gauge(dev(U))
    assert ctx2.autotune(blk, 2, cache) == t1
    assert open(cache).read().count("|") == 1
    # a cached line that mspcg_set_tuning would reject (odd tile) is skipped
    # and the context tuned afresh
    bad = str(tmp_path / "bad.txt")
    with open(bad, "w") as f:
        f.write("dims=8x8x8x8 Ls=8 block=4x4x4x4 pad=2| remap=1 t64=3,8,8,8 t32=8,8,8,8 "
                "t16=4,4,4,4\n")
    t3 = ctx2.autotune(blk, 2, bad)
    for k in ("fp64", "fp32", "fp16"):
        assert all(v % 2 == 0 and v >= 0 for v in t3["tile"][k])
    assert open(bad).read().count("|") == 2
    # the tuned context still solves correctly
    b = synth.fermion_field(dims, Ls, 34)
    x = torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda")
    st = ctx.solve(dev(b), x, mspcg.make_params(tol=1e-10, solver=mspcg.SOLVER_MSPCG, block=blk))
    assert st["converged"]
    _, bhat = O.prepare(act, U, b)
    r = bhat - O.normal(act, U, O.parity_mask(act, host(x), 0))
    assert (O.norm2(r) / O.norm2(bhat)) ** 0.5 <= 1e-10


def test_set_tuning_rejects_odd_tiles():
    ctx = mspcg.Context((4, 4, 4, 4), 8, 1.8, 0.1)
    with pytest.raises(mspcg.MspcgError):
        ctx.set_tuning(1, (3, 4, 4, 4))


def test_tune_blocking_short_probe_and_full_solves():
    """Both block-shape tuner modes return one of its candidates (every set of
    halved directions) as the context's blocking, and MSPCG with that
    blocking (params' block left at zero) reaches the oracle-checked
    residual; a negative probe length is rejected."""
    dims, Ls = (8, 8, 8, 8), 8
    act, U, ctx = setup(dims, Ls, 1.8, 0.05, 1.5, 0.5, gseed=35)
    base = mspcg.make_params(tol=1e-10, maxiter=3000, solver=mspcg.SOLVER_MSPCG, inner_iters=4,
                             inner_prec=mspcg.FP16)
    b = synth.fermion_field(dims, Ls, 36)
    _, bhat = O.prepare(act, U, b)
    for k in (6, 0):
        blk, pad = ctx.tune_blocking(base, probe_iters=k)
        say(f"probe_iters={k}: blocking {blk} pad {pad}")
        assert pad == 2 and blk != tuple(dims)
        assert all(v in (L, L // 2) for v, L in zip(blk, dims))
        x = torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda")
        st = ctx.solve(dev(b), x, base)
        assert st["converged"]
        r = bhat - O.normal(act, U, O.parity_mask(act, host(x), 0))
        assert (O.norm2(r) / O.norm2(bhat)) ** 0.5 <= 1e-10 * 1.01
    with pytest.raises(mspcg.MspcgError) as e:
        ctx.tune_blocking(base, probe_iters=-1)
    assert e.value.code == mspcg.EINVAL
