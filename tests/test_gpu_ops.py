"""GPU parity of the operator kernels against the FP64 oracle (through the C ABI).

Bars: FP64 relative norm error <= 1e-13, FP32 <= 1e-5.  Lattices span several
workgroups with a ragged tail (e.g. 48 sites per parity at Ls=12: 21+21+6)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1804_08593_amd import mspcg, synth
from tests.gpu_util import dev, host, relerr, say, setup

pytestmark = pytest.mark.gpu

CASES = [
    # dims, Ls, b, c, mf
    ((4, 2, 2, 6), 12, 1.5, 0.5, 0.05),   # ragged last workgroup
    ((4, 4, 4, 4), 8, 1.0, 0.0, 0.1),     # Shamir, c1 shape
    ((8, 4, 4, 4), 16, 1.5, 0.5, 0.005),  # several full workgroups
    ((2, 2, 2, 2), 4, 1.5, 0.5, 0.1),     # minimal extents (x+mu == x-mu)
    ((2, 4, 2, 4), 2, 2.0, 1.0, 0.2),     # Ls = 2
]
TOL = {mspcg.FP64: 1e-13, mspcg.FP32: 1e-5}


def _ref(op, act, U, psi):
    if op == mspcg.OP_D:
        return O.dwf(act, U, psi)
    if op == mspcg.OP_DDAG:
        return O.dwf(act, U, psi, dagger=True)
    if op == mspcg.OP_HOP:
        return O.hop(act, U, psi)
    if op == mspcg.OP_HOPDAG:
        return O.hop(act, U, psi, dagger=True)
    if op == mspcg.OP_M5INV:
        return O.m5(act, psi, "M5inv")
    e = O.parity_mask(act, psi, 0)
    if op == mspcg.OP_MHAT:
        return O.schur(act, U, e)
    if op == mspcg.OP_MHATDAG:
        return O.schur(act, U, e, dagger=True)
    if op == mspcg.OP_A:
        return O.normal(act, U, e)
    if op == mspcg.OP_PREPARE:
        return O.prepare(act, U, psi)[1]
    raise ValueError(op)


OPS = [mspcg.OP_HOP, mspcg.OP_HOPDAG, mspcg.OP_D, mspcg.OP_DDAG, mspcg.OP_M5INV, mspcg.OP_MHAT,
       mspcg.OP_MHATDAG, mspcg.OP_A, mspcg.OP_PREPARE]


@pytest.mark.parametrize("prec", [mspcg.FP64, mspcg.FP32])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}")
def test_operator_parity(case, prec):
    dims, Ls, b, c, mf = case
    say(f"operator parity dims={dims} Ls={Ls} prec={prec}")
    act, U, ctx = setup(dims, Ls, 1.8, mf, b, c, gseed=7)
    psi = synth.fermion_field(dims, Ls, 8)
    d_in = dev(psi)
    for op in OPS:
        out = torch.zeros_like(d_in)
        ctx.apply(op, d_in, out, prec=prec)
        got = host(out)
        ref = _ref(op, act, U, psi)
        err = relerr(got, ref)
        say(f"  op={op} relerr={err:.3e}")
        assert err <= TOL[prec], (op, err)
        if op in (mspcg.OP_MHAT, mspcg.OP_MHATDAG, mspcg.OP_A, mspcg.OP_PREPARE):
            odd = O.parity_mask(act, got, 1)
            assert np.all(odd == 0)


def test_periodic_time_and_bitwise_reproducibility():
    dims, Ls = (4, 2, 4, 4), 8
    act, U, ctx = setup(dims, Ls, 1.8, 0.05, 1.5, 0.5, antiperiodic_t=False, gseed=3)
    psi = synth.fermion_field(dims, Ls, 4)
    d_in = dev(psi)
    out1 = torch.zeros_like(d_in)
    out2 = torch.zeros_like(d_in)
    ctx.apply(mspcg.OP_A, d_in, out1)
    ctx.apply(mspcg.OP_A, d_in, out2)
    assert torch.equal(out1, out2)
    ref = O.normal(act, U, O.parity_mask(act, psi, 0))
    assert relerr(host(out1), ref) <= 1e-13


def test_free_field_wall_mode_on_gpu():
    """U = 1, zero-momentum constant fields: the GPU D reproduces the chirality
    block determinant (1 + M5 c)^Ls (w^Ls + mf) pinned in the oracle tests."""
    dims, Ls = (2, 2, 2, 2), 6
    M5, mf, b, c = 1.8, 0.01, 1.5, 0.5
    ctx = mspcg.Context(dims, Ls, M5, mf, b, c, antiperiodic_t=False)
    ctx.load_gauge(dev(synth.unit_gauge(dims)))
    cols = []
    for s in range(Ls):
        for sp in range(2):
            f = np.zeros(ctx.fshape, complex)
            f[s, ..., sp, 0] = 1.0
            out = torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda")
            ctx.apply(mspcg.OP_D, dev(f), out)
            cols.append(host(out)[:, 0, 0, 0, 0, :2, 0].ravel())
    Dup = np.array(cols).T
    w = (1 - M5 * b) / (1 + M5 * c)
    expect = (1 + M5 * c) ** Ls * (w ** Ls + mf)
    assert np.isclose(np.linalg.det(Dup), expect ** 2, rtol=1e-12)


def test_apply_rejects_aliasing_and_unloaded_gauge():
    ctx = mspcg.Context((4, 4, 4, 4), 8, 1.8, 0.1)
    t = torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda")
    with pytest.raises(mspcg.MspcgError) as e:
        ctx.apply(mspcg.OP_D, t, torch.zeros_like(t))
    assert e.value.code == mspcg.ENOGAUGE
    ctx.load_gauge(dev(synth.unit_gauge((4, 4, 4, 4))))
    with pytest.raises(mspcg.MspcgError) as e:
        ctx.apply(mspcg.OP_D, t, t)
    assert e.value.code == mspcg.EINVAL


def test_binding_rejects_fields_of_the_wrong_size():
    """The C ABI takes bare pointers; the binding checks each field's element
    count and device against the context before any call, so a field of
    another lattice never reaches a kernel."""
    ctx = mspcg.Context((4, 4, 4, 4), 8, 1.8, 0.1)
    ctx.load_gauge(dev(synth.unit_gauge((4, 4, 4, 4))))
    t = torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda")
    short = torch.zeros(t.numel() - 12, dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):
        ctx.apply(mspcg.OP_D, t, short)
    with pytest.raises(ValueError):
        ctx.solve(short, torch.zeros_like(short), mspcg.make_params())
    with pytest.raises(ValueError):
        ctx.load_gauge(torch.zeros(ctx.fshape, dtype=torch.complex128, device="cuda"))
    with pytest.raises(ValueError):
        ctx.force(t, t, F=torch.zeros_like(t))
    with pytest.raises(TypeError):
        ctx.apply(mspcg.OP_D, t.to(torch.complex64), torch.zeros_like(t))
    with pytest.raises(ValueError):
        mspcg.solve_batch([ctx], [t, t], [torch.zeros_like(t)], mspcg.make_params())
    # a field of the right size still goes through (a flat view included)
    ctx.apply(mspcg.OP_D, t.reshape(-1), torch.zeros_like(t))
