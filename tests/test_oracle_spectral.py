"""Pins of the spectral-study helpers (Sec. 4.2) on tiny lattices."""
import numpy as np

import oracle as O
from oracle import spectral as SP
from paper_1804_08593_amd import synth


def _tiny():
    act = O.Action((4, 2, 2, 2), 2, 1.8, 0.1, 1.5, 0.5)
    U = synth.gauge_field(act.dims, 0.3, 9)
    return act, U


def test_precond_eigs_match_symmetric_transform():
    """Eigenvalues of K^-1 A equal those of K^-1/2 A K^-1/2 (Hermitian)."""
    act, U = _tiny()
    A = SP.dense_A(act, U)
    K = SP.dense_K(act, U, A, (2, 2, 2, 2), "literal")
    w, V = np.linalg.eigh(K)
    Kmh = (V / np.sqrt(w)) @ V.conj().T
    ref = np.linalg.eigvalsh(Kmh @ A @ Kmh)
    assert np.allclose(SP.precond_eigs(A, K), ref, rtol=1e-10, atol=0)
    # one block covering the lattice: K = A and K^-1 A = 1
    K1 = SP.dense_K(act, U, A, act.dims, "literal")
    assert np.allclose(SP.precond_eigs(A, K1), 1.0, atol=1e-10)
    lam, q = SP.rayleigh_ratios(A, K1)
    assert np.allclose(q, 1.0, atol=1e-10) and np.all(np.diff(lam) >= 0)


def test_dense_K_readings():
    """The literal K has A's diagonal blocks; the oracle's literal operator
    reproduces it (two constructions of eq. (5))."""
    act, U = _tiny()
    A = SP.dense_A(act, U)
    K = SP.dense_K(act, U, A, (2, 2, 2, 2), "literal")
    Kop = SP.dense_even(act, lambda v: O.block_precond_op(act, U, v, (2, 2, 2, 2), "literal"))
    assert np.allclose(K, Kop, atol=1e-13)


def test_ritz_values_from_oracle_cg():
    """Ritz values from the oracle CG's coefficients lie inside the dense
    spectrum of A and reach both ends once CG has converged."""
    act, U = _tiny()
    A = SP.dense_A(act, U)
    lam = np.linalg.eigvalsh(A)
    _, bhat = O.prepare(act, U, synth.fermion_field(act.dims, act.Ls, 10))
    _, info = O.cg(act, U, bhat, tol=1e-12)
    r = SP.ritz_from_coef(info.coef)
    assert r[0] >= lam[0] * (1 - 1e-9) and r[-1] <= lam[-1] * (1 + 1e-9)
    assert abs(r[-1] - lam[-1]) < 1e-6 * lam[-1] and abs(r[0] - lam[0]) < 2e-2 * lam[0]
    # MSPCG with exact-enough local solves: Ritz values of K^-1 A inside its spectrum
    K = SP.dense_K(act, U, A, (2, 2, 2, 2), "literal")
    ev = SP.precond_eigs(A, K)
    _, info2 = O.mspcg(act, U, bhat, (2, 2, 2, 2), 60, tol=1e-12)
    r2 = SP.ritz_from_coef(info2.coef)
    assert r2[0] >= ev[0] * (1 - 1e-6) and r2[-1] <= ev[-1] * (1 + 1e-6)


def test_dense_split_block_from_schur_matrix():
    """The split block built from the dense Schur matrix equals the oracle's
    split block operator (two constructions)."""
    act, U = _tiny()
    A = SP.dense_A(act, U)
    K = SP.dense_K(act, U, A, (2, 2, 2, 2), "split")
    Kop = SP.dense_even(act, lambda v: O.block_precond_op(act, U, v, (2, 2, 2, 2), "split"))
    assert np.allclose(K, Kop, atol=1e-13)


def test_dense_dirichlet_block_from_full_matrix():
    """The Dirichlet block built from the dense D equals the oracle's
    Dirichlet block operator (two constructions)."""
    act, U = _tiny()
    A = SP.dense_A(act, U)
    D = SP.dense_full(act, lambda v: O.dwf(act, U, v))
    K = SP.dense_K(act, U, A, (2, 2, 2, 2), "dirichlet", D=D)
    Kop = SP.dense_even(act, lambda v: O.block_precond_op(act, U, v, (2, 2, 2, 2), "dirichlet"))
    assert np.allclose(K, Kop, atol=1e-13)
