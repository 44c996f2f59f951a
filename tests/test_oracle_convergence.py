"""Manufactured-solution convergence of the oracle (Sec. 5.1) and the paper's
published errors (Table tab:cpu)."""
import json
import os

import numpy as np
import pytest

from oracle import solve
from tests.oracle_cases import make

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("p", [1, 2, 3])
def test_mms_rates_2d(p):
    """Smooth solution, diffusion-dominated (Pe = 1): both fields converge at
    O(h^{p+1}) in L2."""
    errs = []
    for n in (4, 8):
        dg = make("cfg1", n=(n, n), p=p)
        x, hist = solve.newton(dg, tol=1e-13)
        errs.append(solve.l2_errors(dg, x))
    rates = np.log2(np.array(errs[0]) / np.array(errs[1]))
    assert np.all(rates > p + 0.75), rates


def test_paper3d_rates_p1():
    """The paper's 3-D manufactured problem: rate close to p + 1 for the potential
    and between p + 1/2 and p + 1 for the concentration (Sec. 5.1)."""
    errs = []
    for n in (2, 4):
        dg = make("e1", n=(n, n, n), p=1)
        x, hist = solve.newton(dg, tol=1e-13)
        errs.append(solve.l2_errors(dg, x))
    rates = np.log2(np.array(errs[0]) / np.array(errs[1]))
    assert rates[0] > 1.7 and rates[1] > 1.4, rates


def test_published_total_errors():
    """Table tab:cpu: total L2 error 3.84e-4 (p=1, 16^3) and 1.92e-7 (p=3, 8^3).
    The oracle's errors (written by tests/golden/make_e1.py) agree within a
    factor of 1.5; the discretisations differ in unstated details (penalty h,
    quadrature, weak Dirichlet form)."""
    with open(os.path.join(GOLD, "paper_table_cpu.json")) as f:
        paper = {(r[1], r[2]): r[3] for r in json.load(f)["rows"]}
    with open(os.path.join(GOLD, "e1_errors.json")) as f:
        ours = {(r["p"], r["n"]): r for r in json.load(f)["results"]}
    for key in ((1, 16), (3, 8)):
        ratio = ours[key]["total"] / paper[key]
        assert 1 / 1.5 < ratio < 1.5, (key, ratio)
    # the stored values still come out of the current oracle (the 8^3 p=1 stored case)
    r = ours[(1, 8)]
    dg = make("e1", n=(8, 8, 8), p=1)
    x, hist = solve.newton(dg, tol=1e-12)
    e = solve.l2_errors(dg, x)
    assert abs(e[0] + e[1] - r["total"]) <= 1e-8 * r["total"]
