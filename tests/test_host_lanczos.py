"""The Lanczos condition-number estimate used to qualify solution errors
(error <= kappa * relative residual) recovers the spectrum of a known SPD
matrix from plain CG coefficients."""
import numpy as np

from tests._util import lanczos_kappa


def test_lanczos_kappa_from_cg_coefficients():
    rng = np.random.default_rng(3)
    n = 60
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(0.5, 400.0, n)
    A = (Q * ev) @ Q.T
    b = rng.standard_normal(n)
    x = np.zeros(n)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    coef = []
    for _ in range(n):
        q = A @ p
        al = rr / (p @ q)
        x += al * p
        r -= al * q
        rr_new = r @ r
        be = rr_new / rr
        coef.append((al, be))
        if np.sqrt(rr_new) < 1e-13 * np.linalg.norm(b):
            break
        p = r + be * p
        rr = rr_new
    kappa, lo, hi = lanczos_kappa(coef)
    # the largest Ritz value converges first; the smallest approaches lmin from
    # above by the time the residual has dropped by 1e-13
    assert abs(hi - 400.0) / 400.0 < 1e-6 and 0.5 <= lo < 0.5 * 1.05
    assert 800.0 / 1.05 < kappa <= 800.0 * (1 + 1e-9)
    # a few iterations give Ritz values inside the spectrum
    k5, lo5, hi5 = lanczos_kappa(coef[:5])
    assert lo5 >= 0.5 * (1 - 1e-12) and hi5 <= 400.0 * (1 + 1e-12) and k5 <= kappa
