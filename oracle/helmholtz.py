"""Periodic Helmholtz solve of Algorithm 1, step 2.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Solves (D_Delta - sigma) theta = R on the periodic grid.  The paper names no solver;
the reading used here is exact diagonalisation: D_Delta is a sum of circulant
operators in x and y, so the 2D DFT turns it into multiplication by
lambda_x(kx) + lambda_y(ky).  The (0,0) mode is not obtained by dividing by -sigma:
every discrete derivative in R has zero mean, so in exact arithmetic the mean of the
solution equals the mean of theta^n, and that value is imposed directly (this also
covers sigma = 0, the eps = 0 limit scheme).  Any other mode whose divisor is exactly
zero (possible only for the test-only consistent bundle at sigma = 0, whose wide
Laplacian vanishes at the Nyquist modes) has zero right-hand side and is set to 0.
Pins (tests/test_helmholtz.py): stencil residual of the solution, mean rule, sigma = 0.
"""

import numpy as np


def solve(R, sigma, theta_mean, lam_x, lam_y):
    """R: (ny, nx) right-hand side; lam_x: (nx,), lam_y: (ny,) symbols in numpy FFT
    index order; theta_mean: value imposed on the mean of the solution."""
    ny, nx = R.shape
    Rh = np.fft.fft2(R)
    den = lam_y[:, None] + lam_x[None, :] - sigma
    safe = np.where(den == 0.0, 1.0, den)
    Th = np.where(den == 0.0, 0.0, Rh / safe)
    Th[0, 0] = theta_mean * nx * ny
    return np.real(np.fft.ifft2(Th))
