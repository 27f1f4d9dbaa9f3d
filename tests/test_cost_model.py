"""The paper's worked cost example (Sec. 4.1, eqs. (6)-(7))."""
import json
import os

from paper_1804_08593_amd import costmodel

HERE = os.path.dirname(os.path.abspath(__file__))


def test_paper_cost_example():
    g = json.load(open(os.path.join(HERE, "golden", "cost_model.json")))
    s = costmodel.speedup(g["alpha"], g["l"], g["g"])
    assert abs(s - 21.0 / 9.0) < 1e-15
    assert 2.0 <= s < 2.5  # "a factor of 2"


def test_one_gpu_break_even():
    # no communication: MSPCG wins only if g exceeds 1 + l*rho
    assert abs(costmodel.speedup(0.0, 6, 1 + 6 * 0.27, 0.27) - 1.0) < 1e-15
