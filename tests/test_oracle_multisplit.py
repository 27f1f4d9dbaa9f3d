"""Pins of the oracle's multisplitting iteration (Sec. 2.1, eq. (2); Sec. 2.2
says it converges slowly on its own) by dense linear algebra on tiny lattices."""
import numpy as np
import pytest

import oracle as O
from paper_1804_08593_amd import synth
from tests._util import dense, parity, relerr

P = dict(M5=1.8, mf=0.1, b=1.5, c=0.5)


def _setup(dims, Ls, blk, seed=1, eps=0.3):
    act = O.Action(dims, Ls, P["M5"], P["mf"], P["b"], P["c"])
    U = synth.gauge_field(dims, eps, seed)
    even = np.broadcast_to((parity(dims) == 0)[None, ..., None, None], act.fshape)
    blk_of = np.broadcast_to(O.block_ids(act, blk)[None, ..., None, None], act.fshape)
    A = dense(lambda v: O.normal(act, U, v), act.fshape, even)
    return act, U, even, blk_of[even], A


def _block_diag(A, ids):
    K = np.zeros_like(A)
    same = ids[:, None] == ids[None, :]
    K[same] = A[same]
    return K


def test_sweeps_follow_eq2_with_exact_local_solves():
    """x_{k+1} = K^-1 (b - (A - K) x_k) (eq. (2) for every block at once)
    computed with dense matrices, against the oracle's sweeps with local CG
    run to convergence; the first sweep from zero is eq. (4), x_1 = K^-1 b."""
    dims, Ls, blk = (4, 2, 2, 2), 2, (2, 2, 2, 2)
    act, U, even, ids, A = _setup(dims, Ls, blk)
    K = _block_diag(A, ids)
    _, bhat = O.prepare(act, U, synth.fermion_field(dims, Ls, 3))
    b = bhat[even]
    xs = [np.zeros_like(b)]
    for _ in range(3):
        xs.append(np.linalg.solve(K, b - (A - K) @ xs[-1]))
    assert relerr(xs[1], np.linalg.solve(K, b)) < 1e-13
    for k in (1, 3):
        x, hist = O.multisplitting(act, U, bhat, blk, 200, k)
        assert relerr(x[even], xs[k]) < 1e-10, k
        assert np.all(x[~even] == 0)
        assert abs(hist[-1] - np.linalg.norm(b - A @ xs[k]) / np.linalg.norm(b)) < 1e-10


def test_convergence_follows_the_spectral_radius():
    """The error contracts by rho(I - K^-1 A) per sweep: the iteration reaches
    the dense solution when rho < 1, and the residual grows at the rate rho
    when rho > 1 (multisplitting alone converges slowly or not at all,
    Sec. 2.2).  Small blocks give rho > 1 here."""
    dims, Ls = (4, 2, 2, 4), 2
    rhos = {}
    for blk in ((4, 2, 2, 2), (2, 2, 2, 2)):
        act, U, even, ids, A = _setup(dims, Ls, blk, seed=5)
        K = _block_diag(A, ids)
        rho = np.max(np.abs(np.linalg.eigvals(np.eye(len(A)) - np.linalg.solve(K, A))))
        rhos[blk] = rho
        _, bhat = O.prepare(act, U, synth.fermion_field(dims, Ls, 6))
        x, hist = O.multisplitting(act, U, bhat, blk, 200, 40)
        rate = (hist[40] / hist[30]) ** 0.1
        assert abs(rate - rho) < 0.03 * rho, (blk, rate, rho)
        if rho < 1:
            x_ref = np.linalg.solve(A, bhat[even])
            assert relerr(x[even], x_ref) < 10 * rho ** 40
    assert rhos[(4, 2, 2, 2)] < 1 < rhos[(2, 2, 2, 2)]
