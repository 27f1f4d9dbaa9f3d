"""Seeded synthetic inputs: SU(3) gauge links and Gaussian fermion sources.

This module only draws inputs.  It holds none of the solver's arithmetic and is
the one piece of code shared by the oracle-side tests and the HIP-side tests
and benchmark.

The paper measures on a physical-pion-mass 32^3x64 ensemble (Sec. 3) that is
not available here; these fields stand in for it.  Links are
U = exp(i eps H) with H a random traceless Hermitian 3x3 matrix with Gaussian
entries, which are much smoother than an equilibrated ensemble.

Layouts (complex128, C order):
  gauge    [4][Lt][Lz][Ly][Lx][3][3]        (mu = 0:x 1:y 2:z 3:t; row, col)
  fermion  [Ls][Lt][Lz][Ly][Lx][4][3]       (s, site, spin, colour)
Random numbers come from numpy.random.Generator(PCG64(seed)); gauge draws are
taken in the order mu, lexicographic site, row, column, (re, im).
"""
from __future__ import annotations

import numpy as np

__all__ = ["gauge_field", "fermion_field", "random_su3", "unit_gauge"]


def _expi_hermitian(H: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) for a batch of Hermitian 3x3 matrices, via eigh."""
    w, V = np.linalg.eigh(H)
    return (V * np.exp(1j * eps * w)[..., None, :]) @ np.conj(np.swapaxes(V, -1, -2))


def _reunitarise(U: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1): det U = 1."""
    r0 = U[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def random_su3(rng: np.random.Generator, n: int, eps: float) -> np.ndarray:
    """n matrices exp(i eps H), H = (G + G^+)/2 - tr/3, G_ij = N(0,1) + i N(0,1)."""
    g = rng.standard_normal((n, 3, 3, 2))
    G = g[..., 0] + 1j * g[..., 1]
    H = 0.5 * (G + np.conj(np.swapaxes(G, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    H = H - tr[:, None, None] * np.eye(3)
    return _reunitarise(_expi_hermitian(H, eps))


def gauge_field(dims, eps: float, seed: int, chunk: int = 1 << 18) -> np.ndarray:
    """Seeded SU(3) gauge field [4][Lt][Lz][Ly][Lx][3][3] complex128.

    dims = (Lx, Ly, Lz, Lt).  Drawn in chunks so that large lattices stay within
    a few GB of host memory; the draw order does not depend on the chunk size.
    """
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    V4 = Lx * Ly * Lz * Lt
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((4 * V4, 3, 3), dtype=np.complex128)
    for start in range(0, 4 * V4, chunk):
        n = min(chunk, 4 * V4 - start)
        out[start:start + n] = random_su3(rng, n, eps)
    return out.reshape(4, Lt, Lz, Ly, Lx, 3, 3)


def unit_gauge(dims) -> np.ndarray:
    """Free field U = 1."""
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    U = np.zeros((4, Lt, Lz, Ly, Lx, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def fermion_field(dims, Ls: int, seed: int) -> np.ndarray:
    """Gaussian source [Ls][Lt][Lz][Ly][Lx][4][3]: Re, Im iid N(0, 1/2)."""
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (int(Ls), Lt, Lz, Ly, Lx, 4, 3)
    g = rng.standard_normal(shape + (2,)) * np.sqrt(0.5)
    return g[..., 0] + 1j * g[..., 1]
