"""Cost arithmetic of Sec. 4.1, eqs. (6)-(7).

With local compute P and communication alpha*P per global iteration of plain
CG, l local iterations per global iteration and a reduction g of the global
iteration count, plain CG costs (1 + alpha) P and MSPCG ((1 + l) P + alpha P)/g.
On one GPU there is no communication; the same arithmetic with alpha = 0 and
the local-iteration cost measured relative to the outer one (rho) gives the
break-even reduction g = 1 + l*rho.
"""


def t_cg(P: float, alpha: float) -> float:
    return (1.0 + alpha) * P


def t_mspcg(P: float, alpha: float, l: float, g: float, rho: float = 1.0) -> float:
    """rho = cost of one local iteration / cost P of one global one (1 in the paper)."""
    return ((1.0 + l * rho) * P + alpha * P) / g


def speedup(alpha: float, l: float, g: float, rho: float = 1.0) -> float:
    return t_cg(1.0, alpha) / t_mspcg(1.0, alpha, l, g, rho)
