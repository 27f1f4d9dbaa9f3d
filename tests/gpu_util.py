"""Helpers of the GPU parity tests: seeded inputs on host and device."""
import numpy as np
import torch

import oracle as O
from paper_1804_08593_amd import mspcg, synth


def setup(dims, Ls, M5=1.8, mf=0.1, b=1.0, c=0.0, eps=0.3, gseed=1, antiperiodic_t=True):
    act = O.Action(tuple(dims), Ls, M5, mf, b, c, antiperiodic_t=antiperiodic_t)
    U = synth.gauge_field(dims, eps, gseed)
    ctx = mspcg.Context(dims, Ls, M5, mf, b, c, antiperiodic_t=antiperiodic_t)
    Ud = torch.from_numpy(U).cuda()
    ctx.load_gauge(Ud)
    return act, U, ctx


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b) -> float:
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def say(*args):
    print(*args, flush=True)
