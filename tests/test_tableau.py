"""Pins for oracle/tableau.py: printed coefficients, structural definitions of
Section 3.1, and the order of accuracy measured on a partitioned test problem."""

import json
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import tableau as tb

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tableaux.json")))


@pytest.mark.parametrize("name", tb.PRESETS)
def test_coefficients_match_golden(name):
    t = tb.preset(name)
    g = GOLD[name]
    for key in ("At", "bt", "A", "b"):
        assert np.allclose(getattr(t, key), np.array(g[key], dtype=float), atol=1e-15, rtol=0)


@pytest.mark.parametrize("name", tb.PRESETS)
def test_structure(name):
    t = tb.preset(name)
    assert t.is_explicit_part_ok() and t.is_dirk()
    assert t.is_gsa()
    assert t.is_ars() and t.is_type_ck() and not t.is_type_a()
    # the sums of both weight vectors agree (used in the proof of Theorem 3.4)
    assert abs(t.b.sum() - t.bt.sum()) < 1e-15


def test_paper2_gamma():
    At, bt, A, b = tb.paper2_fractions()
    assert A[2][2] == tb.Fr(7, 5)


def _imex_integrate(t, fE, M, y0, dt, n):
    """Textbook additive IMEX RK with a linear implicit part y' = fE(y) + M y."""
    y = y0.copy()
    I = np.eye(len(y0))
    for _ in range(n):
        Y = []
        for i in range(t.s):
            rhs = y.copy()
            for j in range(i):
                rhs += dt * t.At[i, j] * fE(Y[j]) + dt * t.A[i, j] * (M @ Y[j])
            Y.append(np.linalg.solve(I - dt * t.A[i, i] * M, rhs))
        ynew = y + dt * sum(t.bt[i] * fE(Y[i]) + t.b[i] * (M @ Y[i]) for i in range(t.s))
        # GSA: the last stage is the new solution
        assert np.allclose(ynew, Y[-1], atol=1e-12)
        y = ynew
    return y


@pytest.mark.parametrize("name", tb.PRESETS)
def test_observed_order(name):
    t = tb.preset(name)
    M = np.array([[-1.0, 0.5], [-0.3, -2.0]])
    fE = lambda y: np.array([np.sin(y[1]) - 0.5 * y[0] * y[1], y[0] ** 2 - np.cos(y[0])])
    y0 = np.array([0.7, -0.4])
    T = 1.0
    ref = solve_ivp(lambda _t, y: fE(y) + M @ y, (0, T), y0, method="DOP853",
                    rtol=1e-13, atol=1e-14).y[:, -1]
    errs = []
    for n in (20, 40, 80, 160):
        errs.append(np.max(np.abs(_imex_integrate(t, fE, M, y0, T / n, n) - ref)))
    orders = [np.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    assert abs(orders[-1] - GOLD[name]["order"]) < 0.2, (errs, orders)


@pytest.mark.parametrize("name,order", [("typea1", 1), ("typea2", 2)])
def test_type_a_presets(name, order):
    """The constructed type-A tableaux: structure, the order conditions in exact
    arithmetic, and the observed order on the partitioned test problem."""
    t = tb.preset(name)
    assert t.is_explicit_part_ok() and t.is_dirk() and t.is_gsa()
    assert t.is_type_a() and not t.is_type_ck()
    At, bt, A, b = tb.preset_fractions(name)
    s = len(b)
    c = [sum(A[i]) for i in range(s)]
    ct = [sum(At[i]) for i in range(s)]
    assert sum(b) == 1 and sum(bt) == 1
    if order >= 2:
        half = tb.Fr(1, 2)
        for w, x in ((b, c), (bt, ct), (b, ct), (bt, c)):
            assert sum(wi * xi for wi, xi in zip(w, x)) == half
    M = np.array([[-1.0, 0.5], [-0.3, -2.0]])
    fE = lambda y: np.array([np.sin(y[1]) - 0.5 * y[0] * y[1], y[0] ** 2 - np.cos(y[0])])
    y0 = np.array([0.7, -0.4])
    ref = solve_ivp(lambda _t, y: fE(y) + M @ y, (0, 1.0), y0, method="DOP853",
                    rtol=1e-13, atol=1e-14).y[:, -1]
    errs = [np.max(np.abs(_imex_integrate(t, fE, M, y0, 1.0 / n, n) - ref))
            for n in (20, 40, 80, 160)]
    obs = np.log2(errs[-2] / errs[-1])
    assert abs(obs - order) < 0.2, (errs, obs)
