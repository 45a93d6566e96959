"""Pins for oracle/operators.py: polynomial exactness, orders of accuracy, Fourier
symbols, and the slot assignment of the operator bundle against exact derivatives."""

import numpy as np
import pytest

from oracle import operators as op

RNG = np.random.default_rng(3)


def _cell_averages(coef, centres, h):
    """Cell averages of the polynomial sum coef[k] x^k over [x - h/2, x + h/2]."""
    P = np.polynomial.polynomial.Polynomial(coef)
    I = P.integ()
    return (I(centres + h / 2) - I(centres - h / 2)) / h, P


@pytest.mark.parametrize("deg,eps_w", [(2, op.WENO_EPS), (4, 1e30)])
def test_weno5_polynomial_exactness(deg, eps_w):
    """Finite-difference WENO reconstructs the primitive flux at the face: exact for
    degree <= 2 with any weights, and for degree <= 4 with the linear weights."""
    h = 0.37
    centres = np.arange(-2, 3) * h
    for _ in range(5):
        coef = RNG.standard_normal(deg + 1)
        avg, P = _cell_averages(coef, centres, h)
        got = op.weno5_face(*avg, eps_w=eps_w)
        assert abs(got - P(h / 2)) < 1e-12 * max(1.0, np.max(np.abs(avg)))


def test_weno5_linear_limit_closed_form():
    a, b, c, d, e = RNG.standard_normal(5)
    got = op.weno5_face(a, b, c, d, e, eps_w=1e30)
    assert abs(got - (2 * a - 13 * b + 47 * c + 27 * d - 3 * e) / 60) < 1e-14


def test_weno5_picks_smooth_stencil_at_a_jump():
    # data constant on the left, jump right of cell d: only candidate 0 is smooth
    got = op.weno5_face(1.0, 1.0, 1.0, 5.0, 5.0)
    assert abs(got - 1.0) < 1e-4


@pytest.mark.parametrize("deg,eps_w", [(1, op.WENO_EPS), (2, 1e30)])
def test_weno3_polynomial_exactness(deg, eps_w):
    """WENO3 reconstructs the primitive flux at the face from cell averages: exact for
    degree <= 1 with any weights, and for degree <= 2 with the linear weights."""
    h = 0.29
    centres = np.arange(-1, 2) * h
    for _ in range(5):
        coef = RNG.standard_normal(deg + 1)
        avg, P = _cell_averages(coef, centres, h)
        got = op.weno3_face(*avg, eps_w=eps_w)
        assert abs(got - P(h / 2)) < 1e-12 * max(1.0, np.max(np.abs(avg)))


def test_weno3_linear_limit_closed_form():
    """Linear weights give the third-order upwind-biased face value (-a + 5b + 2c)/6."""
    a, b, c = RNG.standard_normal(3)
    got = op.weno3_face(a, b, c, eps_w=1e30)
    assert abs(got - (-a + 5 * b + 2 * c) / 6) < 1e-14


def test_weno3_picks_smooth_stencil_at_a_jump():
    # constant on the left, jump right of cell b: only the candidate on {a, b} is smooth
    assert abs(op.weno3_face(1.0, 1.0, 5.0) - 1.0) < 1e-6
    # jump left of cell b: only the candidate on {b, c} is smooth
    assert abs(op.weno3_face(1.0, 5.0, 5.0) - 5.0) < 1e-6


def _orders(errs):
    return [np.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]


@pytest.mark.parametrize("alpha", [0.0, 1.0])
def test_weno_derivative_fifth_order(alpha):
    errs = []
    for n in (32, 64, 128, 256):
        h = 2 * np.pi / n
        x = (np.arange(n) + 0.5) * h
        f = np.sin(x) + 0.3 * np.cos(2 * x + 0.4)
        w = np.cos(x - 0.2)
        d = op.weno_derivative(f[None, :], w[None, :], alpha, 1, h)[0]
        ex = np.cos(x) - 0.6 * np.sin(2 * x + 0.4)
        errs.append(np.mean(np.abs(d - ex)))
    assert min(_orders(errs)[1:]) > 4.6, errs


@pytest.mark.parametrize("alpha", [0.0, 1.0])
def test_weno3_derivative_orders(alpha):
    """Third order with the linear weights; with eps_w = 1e-6 Jiang-Shu WENO3 loses an
    order at the critical points of the data, so the mean error converges at about two."""
    for eps_w, lo in ((1e30, 2.9), (op.WENO_EPS, 1.8)):
        errs = []
        for n in (64, 128, 256, 512):
            h = 2 * np.pi / n
            x = (np.arange(n) + 0.5) * h
            f = np.sin(x) + 0.3 * np.cos(2 * x + 0.4)
            w = np.cos(x - 0.2)
            d = op.weno_derivative(f[None, :], w[None, :], alpha, 1, h, eps_w, order=3)[0]
            ex = np.cos(x) - 0.6 * np.sin(2 * x + 0.4)
            errs.append(np.mean(np.abs(d - ex)))
        assert min(_orders(errs)[1:]) > lo, (eps_w, errs)


def test_weno3_lf_dissipation_is_dissipative():
    n = 64
    w = np.where(np.arange(n) < n // 2, 1.0, 0.0)[None, :]
    tv = lambda a: np.sum(np.abs(a - np.roll(a, 1, axis=1)))
    tv0, l20 = tv(w), np.sum(w * w)
    for _ in range(20):
        w = w - 0.2 * op.weno_derivative(0.0 * w, w, 1.0, 1, 1.0, order=3)
    assert np.sum(w * w) < l20
    assert tv(w) <= tv0 + 1e-3


def test_weno_axis_y_matches_axis_x_transposed():
    f = RNG.standard_normal((12, 12))
    w = RNG.standard_normal((12, 12))
    a = op.weno_derivative(f, w, 1.0, 1, 0.3)
    b = op.weno_derivative(f.T, w.T, 1.0, 0, 0.3).T
    assert np.allclose(a, b, atol=1e-14)


def test_lf_dissipation_is_dissipative():
    """-(D_LF flux of f = 0 with dissipation on w) diffuses w: the L2 norm and total
    variation of a step fall under small explicit steps."""
    n = 64
    w = np.where(np.arange(n) < n // 2, 1.0, 0.0)[None, :]
    tv = lambda a: np.sum(np.abs(a - np.roll(a, 1, axis=1)))  # periodic total variation
    tv0, l20 = tv(w), np.sum(w * w)
    for _ in range(20):
        w = w - 0.2 * op.weno_derivative(0.0 * w, w, 1.0, 1, 1.0)
    assert np.sum(w * w) < l20
    # essentially non-oscillatory, not strictly TVD: overshoots stay tiny
    assert tv(w) <= tv0 + 1e-3


def test_lf_printed_first_order_flux():
    f = RNG.standard_normal((1, 9))
    w = RNG.standard_normal((1, 9))
    got = op.lf_flux_first_order(f, w, 1.0, 1)[0, 3]
    assert abs(got - 0.5 * (f[0, 3] + f[0, 4] - (w[0, 4] - w[0, 3]))) < 1e-15


@pytest.mark.parametrize("order", [2, 4])
def test_central_symbols(order):
    n, h = 24, 0.21
    x = np.arange(n) * h
    for k in (1, 3, 7, 12):
        kk = 2 * np.pi * k / (n * h)
        f = np.sin(kk * x)[None, :]
        d = op.central_d(f, 1, h, order)[0]
        assert np.allclose(d, op.central_d_symbol(k, n, h, order) * np.cos(kk * x), atol=1e-12)
        l = op.central_l(f, 1, h, order)[0]
        assert np.allclose(l, op.central_l_symbol(k, n, h, order) * np.sin(kk * x), atol=1e-11)


@pytest.mark.parametrize("order", [2, 4])
def test_central_orders(order):
    eD, eL, eM = [], [], []
    for n in (16, 32, 64, 128):
        h = 2 * np.pi / n
        x = (np.arange(n) + 0.5) * h
        X, Y = np.meshgrid(x, x)
        f = np.exp(np.sin(X)) * np.cos(Y)
        eD.append(np.max(np.abs(op.central_d(f, 1, h, order) - np.cos(X) * f)))
        eL.append(np.max(np.abs(op.central_l(f, 1, h, order)
                                - (np.cos(X) ** 2 - np.sin(X)) * f)))
        mix = op.central_d(op.central_d(f, 0, h, order), 1, h, order)
        eM.append(np.max(np.abs(mix + np.cos(X) * np.exp(np.sin(X)) * np.sin(Y))))
    for e in (eD, eL, eM):
        assert min(_orders(e)[1:]) > order - 0.2, e


def _fields(n):
    h = 2 * np.pi / n
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x)
    u1 = np.sin(X) * np.cos(2 * Y) + 0.2
    u2 = np.cos(X + Y) - 0.1
    q = np.sin(2 * X - Y)
    th = np.cos(X) * np.sin(Y)
    dx = lambda g, gx: gx
    return h, X, Y, u1, u2, q, th


@pytest.mark.parametrize("wo,co,lo,top", [(5, 4, 3.8, 1e-5), (3, 2, 1.2, 3e-2)])
def test_production_bundle_slots_converge_to_exact_derivatives(wo, co, lo, top):
    """Each bundle operator converges to its continuous counterpart, which fixes
    which component and sign sits in which slot (high-order bundle, and the WENO3 +
    second-order central bundle of the convergence tables; Jiang-Shu WENO3 converges
    more slowly in the maximum norm at the critical points of the data)."""
    errs = {k: [] for k in ("div0_B", "grad_lf", "div_lf_B", "div0", "div_c", "grad_c",
                            "lap", "divdivB")}
    for n in (64, 128, 256):
        h = 2 * np.pi / n
        x = (np.arange(n) + 0.5) * h
        X, Y = np.meshgrid(x, x)
        a1, a2 = np.sin(X) * np.cos(2 * Y), np.cos(X + Y)
        a1x, a1y = np.cos(X) * np.cos(2 * Y), -2 * np.sin(X) * np.sin(2 * Y)
        a2x, a2y = -np.sin(X + Y), -np.sin(X + Y)
        a1xx, a1yy = -np.sin(X) * np.cos(2 * Y), -4 * np.sin(X) * np.cos(2 * Y)
        a2xy = -np.cos(X + Y)
        w1, w2 = np.cos(2 * X), np.sin(Y)
        ops = op.Production(h, h, central_order=co, weno_order=wo)
        got = {
            "div0_B": ops.div0_B(a1, a2), "grad_lf": ops.grad_lf(a1, w1, w2),
            "div_lf_B": ops.div_lf_B(a1, a2, w1, w2), "div0": (ops.div0(a1, a2),),
            "div_c": (ops.div_c(a1, a2),), "grad_c": ops.grad_c(a1),
            "lap": (ops.lap(a1),), "divdivB": (ops.divdivB(a1, a2),),
        }
        want = {
            "div0_B": (-a1x + a2y, a2x + a1y), "grad_lf": (a1x, a1y),
            "div_lf_B": (-a1x + a2y, a2x + a1y), "div0": (a1x + a2y,),
            "div_c": (a1x + a2y,), "grad_c": (a1x, a1y), "lap": (a1xx + a1yy,),
            "divdivB": (-a1xx + 2 * a2xy + a1yy,),
        }
        for k in errs:
            errs[k].append(max(np.max(np.abs(g - w)) for g, w in zip(got[k], want[k])))
    for k, e in errs.items():
        assert e[-1] < top and _orders(e)[-1] > lo, (k, e)


def test_consistent_bundle_uses_compositions():
    n = 16
    h = 2 * np.pi / n
    f = RNG.standard_normal((n, n))
    ops = op.Consistent(h, h)
    lx, ly = ops.lap_symbol(n, n)
    fh = np.fft.fft2(f)
    lap_spec = np.real(np.fft.ifft2(fh * (lx[None, :] + ly[:, None])))
    assert np.allclose(ops.lap(f), lap_spec, atol=1e-11)
