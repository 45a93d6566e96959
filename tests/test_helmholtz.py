"""Pins for oracle/helmholtz.py: the solution satisfies the stencil equation."""

import numpy as np
import pytest

from oracle import helmholtz
from oracle.operators import Production, Consistent

RNG = np.random.default_rng(8)


@pytest.mark.parametrize("nx,ny,sigma", [(32, 32, 3.7), (48, 24, 1e-9), (24, 36, 0.0),
                                         (16, 16, 1e6)])
def test_residual_and_mean_rule(nx, ny, sigma):
    hx, hy = 2 * np.pi / nx, 4 * np.pi / ny
    ops = Production(hx, hy)
    R = RNG.standard_normal((ny, nx))
    lx, ly = ops.lap_symbol(nx, ny)
    th = helmholtz.solve(R, sigma, 0.123, lx, ly)
    res = ops.lap(th) - sigma * th - R
    # only the (0,0) mode of the equation is replaced by the mean rule
    scale = max(1.0, np.max(np.abs(R)), sigma * np.max(np.abs(th)))
    assert np.max(np.abs(res - res.mean())) < 1e-12 * scale
    assert abs(th.mean() - 0.123) < 1e-14


def test_consistent_bundle_nyquist_nullspace_at_sigma_zero():
    n = 16
    ops = Consistent(2 * np.pi / n, 2 * np.pi / n)
    f = RNG.standard_normal((n, n))
    R = ops.div_c(f, f.T)  # a discrete divergence: no component in the null space
    lx, ly = ops.lap_symbol(n, n)
    th = helmholtz.solve(R, 0.0, 0.0, lx, ly)
    assert np.max(np.abs(ops.lap(th) - R)) < 1e-11
