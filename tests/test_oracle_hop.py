"""Pins of the oracle's Wilson hop and gamma basis against invariants and
closed forms (no GPU).  The DWF operator is a Wilson operator tensored with a
fifth dimension (Sec. 2.2); these tests fix its 4D hopping part."""
import numpy as np
import pytest

import oracle as O
from paper_1804_08593_amd import synth
from tests._util import (chiral_gammas, colour_rotate, gauge_transform, random_gauge_transform,
                         relerr)


def test_gamma_basis_clifford_and_chirality():
    g = O.gamma_matrices()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2.0 * (mu == nu) * np.eye(4), atol=0)
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    assert np.allclose(g5, np.diag([1, 1, -1, -1]), atol=0)
    # the oracle's basis is the chiral basis written out independently here
    assert np.array_equal(g, chiral_gammas())


@pytest.mark.parametrize("dims,Ls", [((2, 2, 2, 2), 2), ((4, 2, 2, 4), 3)])
def test_hop_adjoint_and_gamma5_hermiticity(dims, Ls):
    act = O.Action(dims, Ls, 1.8, 0.1)
    U = synth.gauge_field(dims, 0.3, 11)
    x = synth.fermion_field(dims, Ls, 12)
    y = synth.fermion_field(dims, Ls, 13)
    lhs = O.dot(x, O.hop(act, U, y))
    rhs = O.dot(O.hop(act, U, x, dagger=True), y)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    g5 = np.array([1, 1, -1, -1])[:, None]
    d = O.hop(act, U, x, dagger=True)
    assert relerr(g5 * O.hop(act, U, g5 * x), d) < 1e-15


def test_hop_gauge_covariance():
    dims, Ls = (4, 2, 2, 4), 2
    act = O.Action(dims, Ls, 1.8, 0.1)
    U = synth.gauge_field(dims, 0.3, 21)
    psi = synth.fermion_field(dims, Ls, 22)
    g = random_gauge_transform(dims, 23)
    lhs = O.hop(act, gauge_transform(U, g), colour_rotate(psi, g))
    rhs = colour_rotate(O.hop(act, U, psi), g)
    assert relerr(lhs, rhs) < 1e-14


@pytest.mark.parametrize("antiperiodic", [True, False])
def test_hop_free_field_plane_waves(antiperiodic):
    """At U = 1, exp(ipx) chi is an eigenfunction with the momentum-space matrix
    h(p) = sum_mu 2 cos p_mu - 2 i gamma_mu sin p_mu, p_t = (2n+1) pi / Lt when
    the time direction is antiperiodic."""
    dims, Ls = (4, 2, 2, 6), 1
    act = O.Action(dims, Ls, 1.8, 0.1, antiperiodic_t=antiperiodic)
    U = synth.unit_gauge(dims)
    G = chiral_gammas()
    rng = np.random.Generator(np.random.PCG64(5))
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                             indexing="ij")
    for n in [(0, 0, 0, 0), (1, 1, 0, 2), (3, 0, 1, 5), (2, 1, 1, 1)]:
        p = [2 * np.pi * n[i] / dims[i] for i in range(3)]
        p.append((2 * n[3] + (1 if antiperiodic else 0)) * np.pi / Lt)
        phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = (phase[..., None, None] * chi)[None]
        h = sum(2 * np.cos(p[m]) * np.eye(4) - 2j * np.sin(p[m]) * G[m] for m in range(4))
        expect = (phase[..., None, None] * (h @ chi))[None]
        assert relerr(O.hop(act, U, psi), expect) < 1e-14


def test_hop_free_field_singular_values_basis_free():
    """|h(p)|^2 = (sum 2 cos p)^2 + 4 sum sin^2 p for any Clifford basis."""
    dims, Ls = (2, 2, 2, 4), 1
    act = O.Action(dims, Ls, 1.8, 0.1)
    U = synth.unit_gauge(dims)
    from tests._util import dense
    H = dense(lambda v: O.hop(act, U, v), act.fshape)
    sv2 = np.sort(np.linalg.svd(H, compute_uv=False) ** 2)
    expect = []
    for nx in range(2):
        for ny in range(2):
            for nz in range(2):
                for nt in range(4):
                    p = [np.pi * nx, np.pi * ny, np.pi * nz, (2 * nt + 1) * np.pi / 4]
                    v = sum(2 * np.cos(q) for q in p) ** 2 + 4 * sum(np.sin(q) ** 2 for q in p)
                    expect += [v] * 12
    assert np.allclose(sv2, np.sort(expect), rtol=1e-12, atol=1e-12)


def test_dirichlet_hop_equals_sum_of_principal_blocks():
    """Dropping the hops between blocks = sum_s P_s D_h P_s (brute force)."""
    dims, Ls, blk = (4, 4, 2, 4), 2, (2, 4, 2, 2)
    act = O.Action(dims, Ls, 1.8, 0.1)
    U = synth.gauge_field(dims, 0.3, 31)
    psi = synth.fermion_field(dims, Ls, 32)
    ids = O.block_ids(act, blk)
    ref = np.zeros_like(psi)
    for k in range(int(ids.max()) + 1):
        m = (ids == k)[None, ..., None, None]
        ref += m * O.hop(act, U, m * psi)
    for dag in (False, True):
        ref_d = np.zeros_like(psi)
        for k in range(int(ids.max()) + 1):
            m = (ids == k)[None, ..., None, None]
            ref_d += m * O.hop(act, U, m * psi, dagger=dag)
        assert relerr(O.hop(act, U, psi, dagger=dag, block=blk), ref_d) < 1e-15


def test_hop_sites_matches_full():
    dims, Ls = (4, 2, 4, 4), 3
    act = O.Action(dims, Ls, 1.8, 0.1)
    U = synth.gauge_field(dims, 0.3, 41)
    psi = synth.fermion_field(dims, Ls, 42)
    sites = np.array([0, 5, 17, 63, 127])
    full = O.hop(act, U, psi).reshape(Ls, act.V4, 4, 3)[:, sites]
    assert np.array_equal(O.hop_sites(act, U, psi, sites), full)
