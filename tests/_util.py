"""Helpers shared by the tests: dense matrices of linear maps, random SU(3)."""
import numpy as np

from paper_1804_08593_amd import synth


def dense(apply, shape, support=None):
    """Dense matrix of a complex-linear map on arrays of the given shape.

    support: boolean mask (same shape) of the basis vectors to use (columns) and
    of the output entries kept (rows); None means all."""
    n = int(np.prod(shape))
    idx = np.arange(n) if support is None else np.flatnonzero(support.ravel())
    cols = []
    for i in idx:
        e = np.zeros(n, dtype=np.complex128)
        e[i] = 1.0
        cols.append(apply(e.reshape(shape)).ravel()[idx])
    return np.array(cols).T


def random_gauge_transform(dims, seed):
    Lx, Ly, Lz, Lt = dims
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.random_su3(rng, Lx * Ly * Lz * Lt, 1.0).reshape(Lt, Lz, Ly, Lx, 3, 3)


def shift(f, mu, axis_offset):
    """f(x + mu) for a field whose site axes are [t][z][y][x] starting at axis_offset."""
    ax = axis_offset + (3 - mu)
    return np.roll(f, -1, axis=ax)


def gauge_transform(U, g):
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^+ (periodic shift)."""
    out = np.empty_like(U)
    for mu in range(4):
        gs = shift(g, mu, 0)
        out[mu] = g @ U[mu] @ np.conj(np.swapaxes(gs, -1, -2))
    return out


def colour_rotate(psi, g):
    """psi(x) -> g(x) psi(x) for psi [Ls][t][z][y][x][4][3]."""
    return np.einsum("tzyxab,stzyxkb->stzyxka", g, psi)


def chiral_gammas():
    """Euclidean chiral basis: gamma_k = [[0, -i s_k], [i s_k, 0]], gamma_t = [[0, 1], [1, 0]]."""
    s = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]),
         np.array([[1, 0], [0, -1]], complex)]
    Z = np.zeros((2, 2))
    g = [np.block([[Z, -1j * sk], [1j * sk, Z]]) for sk in s]
    g.append(np.block([[Z, np.eye(2)], [np.eye(2), Z]]))
    return np.array(g)


def parity(dims):
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                             indexing="ij")
    return (x + y + z + t) % 2


def relerr(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def lanczos_kappa(coef):
    """Condition-number estimate from CG coefficients (alpha_k, beta_k): the
    extreme eigenvalues of the Lanczos tridiagonal T with
      T[j, j] = 1/alpha_j + beta_{j-1}/alpha_{j-1},  T[j, j+1] = sqrt(beta_j)/alpha_j
    (Ritz values of A on the Krylov space, so lmin(T) >= lmin(A) and
    lmax(T) <= lmax(A)).  Returns (kappa, lmin, lmax)."""
    coef = np.asarray(coef, dtype=float)
    a, b = coef[:, 0], coef[:, 1]
    n = len(a)
    T = np.zeros((n, n))
    for j in range(n):
        T[j, j] = 1.0 / a[j] + (b[j - 1] / a[j - 1] if j > 0 else 0.0)
        if j + 1 < n:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(b[j]) / a[j]
    ev = np.linalg.eigvalsh(T)
    return ev[-1] / ev[0], ev[0], ev[-1]
