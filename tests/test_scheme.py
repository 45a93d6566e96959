"""Pins for oracle/scheme.py: the stage algebra of Algorithm 1 and the properties the
paper proves or the mathematics fixes."""

import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import d2q6, scheme, tableau as tb
from oracle.operators import Production, Consistent, central_d
from paper_2512_19847_amd import workloads as wl

RNG = np.random.default_rng(21)


def _random_state(n, seed, amp=1.0, divfree_with=None):
    rng = np.random.default_rng(seed)
    x = (np.arange(n) + 0.5) * 2 * np.pi / n
    X, Y = np.meshgrid(x, x)

    def smooth():
        a = rng.standard_normal(5)
        return amp * (a[0] * np.sin(X + a[1]) * np.cos(Y - a[2]) + a[3] * np.cos(2 * X + Y + a[4]))

    st = [smooth() for _ in range(6)]
    if divfree_with is not None:
        psi = smooth()
        st[0] = divfree_with._dy(psi)
        st[1] = -divfree_with._dx(psi)
    return st


def _stage_list(state, trace):
    u1, u2, th, v1, v2, q = state
    return [dict(u1=u1, u2=u2, th=th)] + trace


@pytest.mark.parametrize("name", ["paper2", "ars443"])
@pytest.mark.parametrize("eps", [0.5, 1e-2])
def test_consistent_invariant_theta_stage_equation(name, eps):
    """With consistent operators the Helmholtz stage solve must reproduce the theta
    stage equation theta(i) = theta^n - dt/(2 eps^2) sum_{j<=i} a_ij D.u(j) exactly."""
    n = 16
    h = 2 * np.pi / n
    ops = Consistent(h, h)
    t = tb.preset(name)
    st = _random_state(n, 1)
    p = scheme.Params(eps, 0.3, 0.05)
    trace = []
    scheme.step(st, p, t, ops, trace=trace)
    stages = _stage_list(st, trace)
    for tr in trace:
        i = tr["i"]
        want = st[2].copy()
        for j in range(i + 1):
            if t.A[i, j] != 0.0:
                S = stages[j]
                want = want - p.dt / (2 * eps * eps) * t.A[i, j] * ops.div_c(S["u1"], S["u2"])
        scale = np.max(np.abs(want))
        assert np.max(np.abs(tr["th"] - want)) < 1e-11 * scale, (i, name)


def test_printed_sign_breaks_invariant():
    """Planted in the oracle: with the printed '+' on the last Helmholtz term, the
    invariant fails from the first stage where that term is active."""
    n, eps = 16, 0.5
    h = 2 * np.pi / n
    ops = Consistent(h, h)
    t = tb.preset("ars443")
    st = _random_state(n, 1)
    p = scheme.Params(eps, 0.3, 0.05)
    trace = []
    scheme.step(st, p, t, ops, trace=trace, _last_sign=+1.0)
    stages = _stage_list(st, trace)
    worst = 0.0
    for tr in trace:
        i = tr["i"]
        want = st[2].copy()
        for j in range(i + 1):
            if t.A[i, j] != 0.0:
                S = stages[j]
                want = want - p.dt / (2 * eps * eps) * t.A[i, j] * ops.div_c(S["u1"], S["u2"])
        worst = max(worst, np.max(np.abs(tr["th"] - want)) / np.max(np.abs(want)))
    assert worst > 1e-6


@pytest.mark.parametrize("name", tb.PRESETS)
def test_eps0_stages_stay_discretely_divergence_free(name):
    """Discrete Theorem 3.5: at eps = 0 with consistent operators and D.u^n = 0,
    every stage velocity is discretely divergence free."""
    n = 16
    h = 2 * np.pi / n
    ops = Consistent(h, h)
    t = tb.preset(name)
    st = _random_state(n, 2, divfree_with=ops)
    assert np.max(np.abs(ops.div_c(st[0], st[1]))) < 1e-12
    trace = []
    scheme.step(st, scheme.Params(0.0, 0.05, 0.1), t, ops, trace=trace)
    for tr in trace:
        assert np.max(np.abs(ops.div_c(tr["u1"], tr["u2"]))) < 1e-11


@pytest.mark.parametrize("name", tb.PRESETS)
def test_time_order_against_semidiscrete_reference(name):
    """With consistent operators the scheme is an IMEX RK method for the semi-discrete
    moment system; its observed order in dt must equal the tableau's order.  The
    reference integrates moment_rhs (pinned against the population model)."""
    n = 8
    h = 2 * np.pi / n
    ops = Consistent(h, h)
    ddx = lambda f: central_d(f, 1, h)
    ddy = lambda f: central_d(f, 0, h)
    eps, tau, T = 1.0, 1.0, 0.4
    st = _random_state(n, 3, amp=0.3)

    def rhs(_t, y):
        f = y.reshape(6, n, n)
        return np.concatenate([g.ravel() for g in d2q6.moment_rhs(*f, eps, tau, ddx, ddy)])

    ref = solve_ivp(rhs, (0, T), np.concatenate([f.ravel() for f in st]), method="DOP853",
                    rtol=1e-13, atol=1e-13).y[:, -1].reshape(6, n, n)
    t = tb.preset(name)
    errs = []
    for m in (8, 16, 32):
        out = scheme.run(st, scheme.Params(eps, tau, T / m), t, ops, m)
        errs.append(max(np.max(np.abs(a - b)) for a, b in zip(out, ref)))
    order = {"euler1": 1, "paper2": 2, "ars443": 3}[name]
    obs = math.log2(errs[-2] / errs[-1])
    assert abs(obs - order) < 0.25, (errs, obs)


@pytest.mark.parametrize("wo,co", [(5, 4), (3, 2)])
@pytest.mark.parametrize("name", tb.PRESETS)
def test_conservation_production(name, wo, co):
    n = 24
    h = 2 * np.pi / n
    ops = Production(h, h, central_order=co, weno_order=wo)
    st = _random_state(n, 4, amp=0.3)
    sums0 = [np.sum(st[k]) for k in (0, 1, 2)]
    out = scheme.run(st, scheme.Params(0.1, 0.2, 0.02), tb.preset(name), ops, 3)
    for k, s0 in zip((0, 1, 2), sums0):
        assert abs(np.sum(out[k]) - s0) < 1e-12 * np.sum(np.abs(out[k])) + 1e-13


def test_ap_limit_is_second_order_in_eps():
    n = 32
    st = wl.taylor_green(n)
    h = 2 * np.pi / n
    ops = Production(h, h)
    t = tb.preset("ars443")
    w0 = scheme.run(st, scheme.Params(0.0, 0.05, 0.05), t, ops, 3)
    diffs = []
    # the expansion parameter is eps^2 / dt^2 (it enters through sigma): start where
    # it is small
    for eps in (1e-4, 1e-5, 1e-6):
        w = scheme.run(st, scheme.Params(eps, 0.05, 0.05), t, ops, 3)
        diffs.append(max(np.max(np.abs(w[k] - w0[k])) for k in (0, 1)))
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert 70 < r1 < 140 and 70 < r2 < 140, diffs


@pytest.mark.parametrize("name,order", [("paper2", 2), ("ars443", 3)])
def test_taylor_green_converges_to_ins_closed_form(name, order):
    """eps -> 0, tau = 0.05: the limit is incompressible Navier-Stokes with viscosity
    tau / 4, whose Taylor-Green solution decays as exp(-2 nu t)."""
    amp, tau, T = 0.1, 0.05, 1.0
    nu = tau / 4
    errs = []
    for n in (16, 32, 64):
        h = 2 * np.pi / n
        m = int(round(T / (0.25 * h)))
        st = wl.taylor_green(n, amp=amp)
        out = scheme.run(st, scheme.Params(1e-6, tau, T / m), tb.preset(name),
                         Production(h, h), m)
        u1, u2, _ = wl.taylor_green_exact(n, n, amp, nu, T)
        errs.append(max(np.max(np.abs(out[0] - u1)), np.max(np.abs(out[1] - u2))))
    obs = math.log2(errs[-2] / errs[-1])
    assert errs[-1] < 1e-5 and obs > order - 0.3, (errs, obs)


@pytest.mark.parametrize("name", ["euler1", "paper2"])
def test_taylor_green_low_order_bundle(name):
    """WENO3 + second-order central differences (the operators of the convergence
    tables): same Navier-Stokes limit; the error is dominated by the space
    discretisation here (the flow decays slowly) and converges at more than second
    order in the maximum norm.  The paper's second-order tableau needs c dt <= 0.225 h
    with WENO3 (its explicit stage of length 2.25 dt meets the alpha = 1 dissipation)."""
    amp, tau, T = 0.1, 0.05, 1.0
    nu = tau / 4
    errs = []
    for n in (16, 32, 64):
        h = 2 * np.pi / n
        m = int(round(T / (0.1 * h)))
        st = wl.taylor_green(n, amp=amp)
        out = scheme.run(st, scheme.Params(1e-6, tau, T / m), tb.preset(name),
                         Production(h, h, central_order=2, weno_order=3), m)
        u1, u2, _ = wl.taylor_green_exact(n, n, amp, nu, T)
        errs.append(max(np.max(np.abs(out[0] - u1)), np.max(np.abs(out[1] - u2))))
    obs = math.log2(errs[-2] / errs[-1])
    assert errs[-1] < 1e-3 and obs > 2.2, (errs, obs)


def test_fixed_grid_time_order_of_the_printed_operators():
    """On a fixed grid in the stiff regime (eps = 1e-6) the fully discrete scheme has the
    tableau's order in time with the consistent bundle, but only first order with the
    printed operators: D_Delta and D0^2:B(v) are not the compositions of the first
    derivatives that substituting step 3 into the theta equation assumes, which leaves
    an O(dt h^4) term (fourth-order operators).  With dt proportional to h this is
    O(h^5), below the space error, as in the convergence tables of Section 4.1."""
    T, tau = 0.5, 0.05
    tab = tb.preset("ars443")

    def errs(ops, n):
        st = wl.taylor_green(n)
        ref = scheme.run(st, scheme.Params(1e-6, tau, T / 256), tab, ops, 256)
        out = []
        for m in (8, 16):
            o = scheme.run(st, scheme.Params(1e-6, tau, T / m), tab, ops, m)
            out.append(max(np.max(np.abs(o[k] - ref[k])) for k in (0, 1)))
        return out

    h16, h32 = 2 * np.pi / 16, 2 * np.pi / 32
    c = errs(Consistent(h32, h32), 32)
    assert math.log2(c[0] / c[1]) > 2.6 and c[1] < 1e-12, c
    p16, p32 = errs(Production(h16, h16), 16), errs(Production(h32, h32), 32)
    assert 0.8 < math.log2(p32[0] / p32[1]) < 1.3, p32
    assert 10.0 < p16[1] / p32[1] < 30.0, (p16, p32)  # about 2^4


def test_eps_zero_tau_zero_runs_finite():
    n = 32
    st = wl.shear_layer(n)
    h = 2 * np.pi / n
    out = scheme.run(st, scheme.Params(0.0, 0.0, 0.02), tb.preset("paper2"), Production(h, h), 5)
    assert all(np.all(np.isfinite(f)) for f in out)


@pytest.mark.parametrize("nx,ny,kmax", [(64, 64, 8), (96, 72, 4)])
def test_random_fields_are_discretely_divergence_free(nx, ny, kmax):
    """The random initial velocities are the discrete curl of the stream function with
    the scheme's fourth-order central difference, so the scheme's D0.u vanishes to
    rounding (well-prepared data, Theorem 3.5), at the requested rms speed."""
    st = wl.random_divfree(nx, ny, kmax=kmax, rms=0.1, seed=3)
    ops = Production(2 * np.pi / nx, 2 * np.pi / ny)
    assert np.max(np.abs(ops.div_c(st[0], st[1]))) < 1e-13
    assert abs(math.sqrt(np.mean(st[0] ** 2 + st[1] ** 2)) - 0.1) < 1e-14
