"""Pins for oracle/d2q6.py: what Section 2.1 fixes about the six-velocity model."""

import numpy as np
import pytest

from oracle import d2q6
from oracle.operators import central_d

RNG = np.random.default_rng(11)


def test_velocity_set_is_unit_hexagon():
    cx, cy = d2q6.velocity_set()
    assert np.allclose(cx * cx + cy * cy, 1.0, atol=1e-15)
    s = np.sqrt(3.0) / 2.0
    ref = np.array([[1, 0], [0.5, s], [-0.5, s], [-1, 0], [-0.5, -s], [0.5, -s]])
    assert np.allclose(np.stack([cx, cy], 1), ref, atol=1e-15)


def test_basis_is_orthogonal_with_known_norms():
    M = d2q6.moment_matrix()
    G = M @ M.T
    assert np.allclose(G, np.diag([6.0, 3.0, 3.0, 0.75, 0.75, 0.375]), atol=1e-14)


def test_equilibrium_moment_identities():
    rho = 1.0 + 0.3 * RNG.standard_normal(50)
    u1 = 0.4 * RNG.standard_normal(50)
    u2 = 0.4 * RNG.standard_normal(50)
    Feq = d2q6.equilibrium(rho, u1, u2)
    m = d2q6.raw_moments(Feq)
    assert np.allclose(m[0], rho, atol=1e-15, rtol=0)
    assert np.allclose(m[1], u1, atol=1e-15, rtol=0)
    assert np.allclose(m[2], u2, atol=1e-15, rtol=0)
    # equilibrium of the second-order moments is F(u); the third-order one vanishes
    assert np.allclose(m[3], 0.5 * (u2 * u2 - u1 * u1), atol=1e-15, rtol=0)
    assert np.allclose(m[4], u1 * u2, atol=1e-15, rtol=0)
    assert np.allclose(m[5], 0.0, atol=1e-15)


def test_equilibrium_sign_of_v1_reading():
    # the printed definition (c_x^2 - 1/2) would give the opposite sign of F1(u)
    u1, u2 = np.array([0.3]), np.array([-0.1])
    cx, _ = d2q6.velocity_set()
    Feq = d2q6.equilibrium(np.ones(1), u1, u2)
    printed = np.sum((cx * cx - 0.5)[:, None] * Feq, axis=0)
    assert np.allclose(printed, -0.5 * (u2 * u2 - u1 * u1))


def test_collision_conserves_mass_and_momentum():
    F = 1.0 / 6.0 + 0.05 * RNG.standard_normal((6, 40))
    C = d2q6.bgk_collision(F, tau=0.37)
    m = d2q6.raw_moments(C)
    assert np.max(np.abs(m[:3])) < 1e-15
    # and it relaxes: the non-conserved moments decay
    mF = d2q6.raw_moments(F)
    meq = d2q6.raw_moments(d2q6.equilibrium(mF[0], mF[1], mF[2]))
    assert np.allclose(m[3:], -(mF[3:] - meq[3:]) / 0.37, atol=1e-15)


def test_scaling_map_roundtrip():
    fields = [RNG.standard_normal((4, 5)) for _ in range(6)]
    for eps in (1.0, 0.1, 1e-3):
        F = d2q6.populations_from_scaled(*fields, eps)
        back = d2q6.scaled_from_populations(F, eps)
        # populations are O(1/6); the scaled moment of order k is recovered from a
        # raw moment of size eps^k, so its round-off grows like 1e-16 / eps^k
        for k, (a, b) in zip((1, 1, 2, 2, 2, 3), zip(fields, back)):
            assert np.max(np.abs(a - b)) < 50 * 2.2e-16 / eps ** k


def _smooth_fields(n, seed):
    rng = np.random.default_rng(seed)
    x = (np.arange(n) + 0.5) * 2 * np.pi / n
    X, Y = np.meshgrid(x, x)
    out = []
    for _ in range(6):
        a = rng.standard_normal(4)
        out.append(a[0] * np.sin(X + a[1]) * np.cos(2 * Y) + a[2] * np.cos(X - 2 * Y + a[3]))
    return out


@pytest.mark.parametrize("eps,tau", [(0.3, 0.7), (1.0, 2.0), (0.05, 0.1)])
def test_population_rhs_maps_onto_moment_system(eps, tau):
    """The moments of the scaled population equation are exactly the closed moment
    system (pins the v1 sign, the q-equation divergence, the relaxation sign and
    the rescaling)."""
    n = 16
    h = 2 * np.pi / n
    ddx = lambda f: central_d(f, 1, h)  # any linear derivative works for this identity
    ddy = lambda f: central_d(f, 0, h)
    mom = _smooth_fields(n, 5)
    F = d2q6.populations_from_scaled(*mom, eps)
    dF = d2q6.population_rhs(F, eps, tau, ddx, ddy)
    dR, dU1, dU2, dV1, dV2, dQ = d2q6.raw_moments(dF)
    got = (dU1 / eps, dU2 / eps, dR / (2 * eps * eps), dV1 / eps ** 2, dV2 / eps ** 2,
           dQ / eps ** 3)
    want = d2q6.moment_rhs(*mom, eps, tau, ddx, ddy)
    for g, w in zip(got, want):
        scale = max(1.0, np.max(np.abs(w)))
        assert np.max(np.abs(g - w)) / scale < 1e-10


def test_printed_q_divergence_would_fail():
    """Planted in the oracle's formula: with d_x v2 (as printed) instead of d_y v2 the
    population identity breaks."""
    n, eps, tau = 16, 0.3, 0.7
    h = 2 * np.pi / n
    ddx = lambda f: central_d(f, 1, h)
    ddy = lambda f: central_d(f, 0, h)
    mom = _smooth_fields(n, 6)
    F = d2q6.populations_from_scaled(*mom, eps)
    dQ = d2q6.raw_moments(d2q6.population_rhs(F, eps, tau, ddx, ddy))[5] / eps ** 3
    u1, u2, th, v1, v2, q = mom
    printed = -(ddx(v1) + ddx(v2)) / (2 * eps * eps) - q / (eps * eps * tau)
    assert np.max(np.abs(dQ - printed)) > 1e-3
