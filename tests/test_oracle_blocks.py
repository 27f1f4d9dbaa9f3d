"""Pins of the oracle's multisplitting preconditioner (Sec. 2.3, eqs. (4)-(5),
Fig. 3), its sloppy inner solve ("local iterations") and the flexible outer
PCG, by brute-force dense linear algebra on tiny lattices (no GPU)."""
import numpy as np
import pytest

import oracle as O
from paper_1804_08593_amd import synth
from tests._util import dense, parity, relerr

P = dict(M5=1.8, mf=0.1, b=1.5, c=0.5)


def _setup(dims, Ls, blk, seed=1):
    act = O.Action(dims, Ls, P["M5"], P["mf"], P["b"], P["c"])
    U = synth.gauge_field(dims, 0.3, seed)
    even = np.broadcast_to((parity(dims) == 0)[None, ..., None, None], act.fshape)
    ids = O.block_ids(act, blk)
    blk_of = np.broadcast_to(ids[None, ..., None, None], act.fshape)
    return act, U, even, blk_of


def test_literal_preconditioner_is_block_diagonal_of_A():
    """K has A's entries inside every diagonal block and zero elsewhere (Fig. 3)."""
    dims, Ls, blk = (4, 4, 2, 2), 2, (2, 2, 2, 2)
    act, U, even, blk_of = _setup(dims, Ls, blk)
    A = dense(lambda v: O.normal(act, U, v), act.fshape, even)
    K = dense(lambda v: O.block_precond_op(act, U, v, blk), act.fshape, even)
    b = blk_of[even]
    same = b[:, None] == b[None, :]
    assert np.allclose(K[same], A[same], rtol=0, atol=1e-13)
    assert np.all(K[~same] == 0)
    assert np.abs(A[~same]).max() > 0.1  # the blocks do couple in A
    # Hermitian positive definite (the paper's requirement for an exact preconditioner)
    assert np.allclose(K, K.conj().T, atol=1e-13)
    assert np.linalg.eigvalsh(K).min() > 0


def test_dirichlet_variant_is_schur_of_principal_submatrix():
    """The cheaper Dirichlet-cut block: A_s = Mhat_s^+ Mhat_s with Mhat_s the Schur
    complement of the principal submatrix of D on block s."""
    dims, Ls, blk = (4, 2, 2, 2), 2, (2, 2, 2, 2)
    act, U, even, blk_of = _setup(dims, Ls, blk)
    D = dense(lambda v: O.dwf(act, U, v), act.fshape)
    Kd = dense(lambda v: O.block_precond_op(act, U, v, blk, "dirichlet"), act.fshape, even)
    ev_idx = np.flatnonzero(even.ravel())
    for k in range(2):
        inb = (blk_of == k).ravel()
        e = inb & even.ravel()
        o = inb & ~even.ravel()
        Mh = D[np.ix_(e, e)] - D[np.ix_(e, o)] @ np.linalg.solve(D[np.ix_(o, o)], D[np.ix_(o, e)])
        As = Mh.conj().T @ Mh
        sel = np.isin(ev_idx, np.flatnonzero(e))
        assert np.allclose(Kd[np.ix_(sel, sel)], As, rtol=0, atol=1e-13)
        assert np.all(Kd[np.ix_(sel, ~sel)] == 0)


def _krylov_galerkin(A, r, l):
    """z = V (V^+ A V)^-1 V^+ r, V an orthonormal basis of K_l(A, r)."""
    V = np.zeros((len(r), l), complex)
    v = r / np.linalg.norm(r)
    for j in range(l):
        for _ in range(2):
            v = v - V[:, :j] @ (V[:, :j].conj().T @ v)
        V[:, j] = v / np.linalg.norm(v)
        v = A @ V[:, j]
    return V @ np.linalg.solve(V.conj().T @ A @ V, V.conj().T @ r)


@pytest.mark.parametrize("mode", ["literal", "dirichlet"])
@pytest.mark.parametrize("l", [1, 3, 5])
def test_inner_cg_is_krylov_galerkin_projection(mode, l):
    """l CG steps from zero = the Galerkin solution on K_l(A_s, r_s), per block."""
    dims, Ls, blk = (4, 2, 2, 2), 2, (2, 2, 2, 2)
    act, U, even, blk_of = _setup(dims, Ls, blk)
    r = O.parity_mask(act, synth.fermion_field(dims, Ls, 7), 0)
    z = O.inner_block_cg(act, U, r, blk, l, mode)
    K = dense(lambda v: O.block_precond_op(act, U, v, blk, mode), act.fshape, even)
    ev_blk = blk_of[even]
    rv = r[even]
    zv = z[even]
    for k in range(2):
        sel = ev_blk == k
        zk = _krylov_galerkin(K[np.ix_(sel, sel)], rv[sel], l)
        assert relerr(zv[sel], zk) < 1e-10
    assert np.all(z[~even] == 0)


def test_inner_cg_zero_block_is_left_zero():
    """A block whose residual is zero is skipped (no division by zero)."""
    dims, Ls, blk = (4, 2, 2, 2), 2, (2, 2, 2, 2)
    act, U, even, blk_of = _setup(dims, Ls, blk)
    r = O.parity_mask(act, synth.fermion_field(dims, Ls, 8), 0)
    r[blk_of == 1] = 0
    z = O.inner_block_cg(act, U, r, blk, 4)
    assert np.all(z[blk_of == 1] == 0)
    assert np.all(np.isfinite(z))


def test_zero_guess_multisplitting_step_is_local_solve():
    """Eq. (2) with x_l = x_r = 0 is eq. (4): enough local iterations solve
    A_s x_s = b_s exactly, i.e. z = K^-1 r."""
    dims, Ls, blk = (4, 2, 2, 2), 2, (2, 2, 2, 2)
    act, U, even, blk_of = _setup(dims, Ls, blk)
    r = O.parity_mask(act, synth.fermion_field(dims, Ls, 9), 0)
    K = dense(lambda v: O.block_precond_op(act, U, v, blk), act.fshape, even)
    z_exact = np.linalg.solve(K, r[even])
    z = O.inner_block_cg(act, U, r, blk, 120)
    assert relerr(z[even], z_exact) < 1e-9


@pytest.mark.parametrize("mode", ["literal", "dirichlet"])
def test_mspcg_reaches_the_dense_solution(mode):
    dims, Ls, blk = (4, 2, 2, 2), 4, (2, 2, 2, 2)
    act, U, even, blk_of = _setup(dims, Ls, blk, seed=3)
    b = synth.fermion_field(dims, Ls, 4)
    D = dense(lambda v: O.dwf(act, U, v), act.fshape)
    x_ref = np.linalg.solve(D, b.ravel()).reshape(act.fshape)
    x, info = O.solve(act, U, b, tol=1e-12, precond=(blk, 3, mode))
    assert info.converged and info.true_rel_resid <= 1e-12
    assert relerr(x, x_ref) < 1e-9
    xc, infoc = O.solve(act, U, b, tol=1e-12)
    assert relerr(x, xc) < 1e-9


def _dense_domain_block(D, even, blk_of, omega_site, k):
    """Dense A_s of block k on the domain Omega: Schur complement of the
    principal submatrix of D on Omega (over its odd sites), its normal matrix,
    and the rows / columns of block k's even sites."""
    om = np.broadcast_to(omega_site[None, ..., None, None], even.shape).ravel()
    ev = even.ravel()
    e, o = om & ev, om & ~ev
    Mh = D[np.ix_(e, e)] - D[np.ix_(e, o)] @ np.linalg.solve(D[np.ix_(o, o)], D[np.ix_(o, e)])
    AO = Mh.conj().T @ Mh
    sel = (blk_of.ravel() == k)[np.flatnonzero(e)]
    return AO[np.ix_(sel, sel)]


@pytest.mark.parametrize("pad", [0, 1, 2])
def test_padded_domain_block_is_schur_of_widened_principal_submatrix(pad):
    """Block operator on the block widened by `pad` sites (Sec. 2.3 Fig. 3 read
    on a padded domain): dense Schur complement of D's principal submatrix on
    the widened block, normal matrix, restricted to the block."""
    dims, Ls, blk = (8, 2, 2, 2), 2, (2, 2, 2, 2)
    act, U, even, blk_of = _setup(dims, Ls, blk)
    D = dense(lambda v: O.dwf(act, U, v), act.fshape)
    Kp = dense(lambda v: O.block_precond_op(act, U, v, blk, "domain", pad), act.fshape, even)
    ev_blk = blk_of[even]
    for k in range(4):
        om = O.domain_mask(act, blk, k, pad)
        assert om.sum() == (2 + 2 * pad) * 8  # widened in x only
        As = _dense_domain_block(D, even, blk_of, om, k)
        sel = ev_blk == k
        assert np.allclose(Kp[np.ix_(sel, sel)], As, rtol=0, atol=1e-13)
        assert np.all(Kp[np.ix_(sel, ~sel)] == 0)
    # HPD whenever Mhat_Omega is nonsingular
    assert np.allclose(Kp, Kp.conj().T, atol=1e-13)
    assert np.linalg.eigvalsh(Kp).min() > 0


def test_padded_domain_limits():
    """pad 0 is the Dirichlet block and pad 2 the literal block P_s A P_s (A
    couples sites two hops apart, so a domain widened by two sites holds
    every path that returns into the block); pad 1 lies strictly between."""
    dims, Ls, blk = (8, 8, 4, 2), 4, (4, 2, 4, 2)
    act, U, even, blk_of = _setup(dims, Ls, blk, seed=5)
    p = O.parity_mask(act, synth.fermion_field(dims, Ls, 6), 0)
    lit = O.block_precond_op(act, U, p, blk, "literal")
    dir_ = O.block_precond_op(act, U, p, blk, "dirichlet")
    d0 = O.block_precond_op(act, U, p, blk, "domain", 0)
    d1 = O.block_precond_op(act, U, p, blk, "domain", 1)
    d2 = O.block_precond_op(act, U, p, blk, "domain", 2)
    assert relerr(d0, dir_) < 1e-14
    assert relerr(d2, lit) < 1e-14
    assert 1e-6 < relerr(d1, lit) < relerr(d0, lit)


def test_domain_mask_wraps_periodically():
    act = O.Action((8, 4, 4, 8), 2, 1.8, 0.1)
    om = O.domain_mask(act, (4, 4, 4, 4), 0, 2)  # block at x, t in [0, 4)
    x_in = om[0, 0, 0, :]
    assert list(np.flatnonzero(x_in)) == [0, 1, 2, 3, 4, 5, 6, 7]
    om1 = O.domain_mask(act, (4, 4, 4, 4), 1, 1)  # block at x in [4, 8), t in [0, 4)
    assert list(np.flatnonzero(om1[0, 0, 0, :])) == [0, 3, 4, 5, 6, 7]
    assert list(np.flatnonzero(om1[:, 0, 0, 4])) == [0, 1, 2, 3, 4, 7]
    with pytest.raises(ValueError):
        O.domain_mask(O.Action((4, 4, 4, 8), 2, 1.8, 0.1), (2, 4, 4, 4), 0, 2)


def test_split_block_is_normal_of_schur_block():
    """The alternative block of Sec. 2.3's preconditioner where the block is
    taken of Mhat before the normal equations: A_s = Mhat_ss^+ Mhat_ss with
    Mhat_ss the diagonal block of the dense Schur complement of D."""
    dims, Ls, blk = (4, 4, 2, 2), 2, (2, 2, 2, 2)
    act, U, even, blk_of = _setup(dims, Ls, blk)
    D = dense(lambda v: O.dwf(act, U, v), act.fshape)
    ev = even.ravel()
    Mh = D[np.ix_(ev, ev)] - D[np.ix_(ev, ~ev)] @ np.linalg.solve(D[np.ix_(~ev, ~ev)],
                                                                   D[np.ix_(~ev, ev)])
    Ks = dense(lambda v: O.block_precond_op(act, U, v, blk, "split"), act.fshape, even)
    A = dense(lambda v: O.normal(act, U, v), act.fshape, even)
    b = blk_of[even]
    for k in range(int(b.max()) + 1):
        sel = b == k
        Mss = Mh[np.ix_(sel, sel)]
        assert np.allclose(Ks[np.ix_(sel, sel)], Mss.conj().T @ Mss, rtol=0, atol=1e-13)
        assert np.all(Ks[np.ix_(sel, ~sel)] == 0)
    # it differs from the literal block P_s A P_s and is HPD
    same = b[:, None] == b[None, :]
    assert np.abs(Ks[same] - A[same]).max() > 1e-3
    assert np.linalg.eigvalsh(Ks).min() > 0
