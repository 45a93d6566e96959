"""Spatial operators of Section 3.2 and their high-order extension.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Grid: periodic, cell-centred, arrays of shape (ny, nx) with x the fast (last) axis.
Every shift is written with np.roll, which is the periodic index map itself.

Low-order template (Section 3.2): local Lax-Friedrichs fluxes D_LF (alpha = 1) for
grad q and div B(v), the same without numerical diffusion D0_LF (alpha_0 = 0) for
div B(u) and div v, and central differences D0.u, D0^2:B(v), D_Delta theta, D0 theta.
High-order extension (end of Section 3.2, details not printed): every Lax-Friedrichs
flux becomes a WENO flux and every central difference becomes fourth order.  The
reading used here:
  * WENO5 of Jiang and Shu, smoothness indicators with weight power 2, eps_w = 1e-6,
    linear weights (1, 6, 3)/10, applied to the Lax-Friedrichs split fluxes
    f+- = (f +- alpha w)/2: the numerical flux at i+1/2 is the left-biased
    reconstruction of f+ plus the right-biased reconstruction of f-.  With first-order
    reconstruction this is exactly the printed Lax-Friedrichs flux.
  * The dissipation variable w of a flux is the unknown of the equation the flux
    appears in: v1 (x) and v2 (y) for grad q in the v equations; u1 (first
    component) and u2 (second component) for div B(v) in the u equations.  Each slot
    is pinned against its Fourier symbol at tiny amplitude, and the whole step against
    the amplification matrix G(k) (tests/test_linear_mode.py); the swapped readings
    make G(k) unstable.
  * Fourth-order central first derivative D, second derivative L, mixed derivative
    D_x D_y.
Third-order variant (Section 4.1 convergence tables, "third order WENO"): WENO3 of
Jiang and Shu (two two-cell candidates, linear weights 1/3 and 2/3) on the same split
fluxes, used with the second-order central differences of the printed template.
Pins (tests/test_operators.py): polynomial exactness of the WENO candidates and of
the linear-weight reconstruction, order of accuracy, Fourier symbols of the central
operators, first-order limit equal to the printed Lax-Friedrichs flux.
"""

import numpy as np

WENO_EPS = 1e-6
WENO_LINEAR = (0.1, 0.6, 0.3)


# --------------------------------------------------------------------------- WENO5

def weno5_face(a, b, c, d, e, eps_w=WENO_EPS):
    """WENO5 value at the right face of cell c from the five cells a..e centred on c
    (left-biased).  Jiang-Shu candidates, smoothness indicators and weights."""
    q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0
    q1 = (-b + 5.0 * c + 2.0 * d) / 6.0
    q2 = (2.0 * c + 5.0 * d - e) / 6.0
    b0 = 13.0 / 12.0 * (a - 2.0 * b + c) ** 2 + 0.25 * (a - 4.0 * b + 3.0 * c) ** 2
    b1 = 13.0 / 12.0 * (b - 2.0 * c + d) ** 2 + 0.25 * (b - d) ** 2
    b2 = 13.0 / 12.0 * (c - 2.0 * d + e) ** 2 + 0.25 * (3.0 * c - 4.0 * d + e) ** 2
    g0, g1, g2 = WENO_LINEAR
    a0 = g0 / (eps_w + b0) ** 2
    a1 = g1 / (eps_w + b1) ** 2
    a2 = g2 / (eps_w + b2) ** 2
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2)


def weno3_face(a, b, c, eps_w=WENO_EPS):
    """WENO3 value at the right face of cell b from the three cells a, b, c centred on b
    (left-biased; Jiang and Shu with r = 2): candidates (3b - a)/2 on {a, b} and
    (b + c)/2 on {b, c}, smoothness indicators (b - a)^2 and (c - b)^2, linear weights
    1/3 and 2/3, weights proportional to d_k / (eps_w + beta_k)^2."""
    q0 = (3.0 * b - a) / 2.0
    q1 = (b + c) / 2.0
    a0 = (1.0 / 3.0) / (eps_w + (b - a) ** 2) ** 2
    a1 = (2.0 / 3.0) / (eps_w + (c - b) ** 2) ** 2
    return (a0 * q0 + a1 * q1) / (a0 + a1)


def _shift(f, k, axis):
    """g[i] = f[i + k] along axis (periodic)."""
    return np.roll(f, -k, axis=axis)


def weno_flux(f, w, alpha, axis, eps_w=WENO_EPS, order=5):
    """Numerical flux at faces i+1/2 along axis for flux values f with
    Lax-Friedrichs dissipation alpha on the variable w: left-biased WENO (order 5 or 3)
    of f+ plus its mirror image, right-biased, of f-."""
    fp = 0.5 * (f + alpha * w)
    fm = 0.5 * (f - alpha * w)
    if order == 3:
        plus = weno3_face(_shift(fp, -1, axis), fp, _shift(fp, 1, axis), eps_w)
        minus = weno3_face(_shift(fm, 2, axis), _shift(fm, 1, axis), fm, eps_w)
        return plus + minus
    plus = weno5_face(_shift(fp, -2, axis), _shift(fp, -1, axis), fp,
                      _shift(fp, 1, axis), _shift(fp, 2, axis), eps_w)
    minus = weno5_face(_shift(fm, 3, axis), _shift(fm, 2, axis), _shift(fm, 1, axis),
                       fm, _shift(fm, -1, axis), eps_w)
    return plus + minus


def weno_derivative(f, w, alpha, axis, h, eps_w=WENO_EPS, order=5):
    """(fhat_{i+1/2} - fhat_{i-1/2}) / h along axis."""
    fh = weno_flux(f, w, alpha, axis, eps_w, order)
    return (fh - _shift(fh, -1, axis)) / h


def lf_flux_first_order(f, w, alpha, axis):
    """The printed first-order local Lax-Friedrichs flux at i+1/2 (Section 3.2):
    (f_i + f_{i+1} - alpha (w_{i+1} - w_i)) / 2.  Used only to pin weno_flux."""
    f1 = _shift(f, 1, axis)
    w1 = _shift(w, 1, axis)
    return 0.5 * (f + f1 - alpha * (w1 - w))


# --------------------------------------------------------------- central differences

def central_d(f, axis, h, order=4):
    """First derivative; order 4: (f_{i-2} - 8 f_{i-1} + 8 f_{i+1} - f_{i+2})/(12h),
    order 2: (f_{i+1} - f_{i-1})/(2h) as printed in Section 3.2."""
    if order == 2:
        return (_shift(f, 1, axis) - _shift(f, -1, axis)) / (2.0 * h)
    return (_shift(f, -2, axis) - 8.0 * _shift(f, -1, axis)
            + 8.0 * _shift(f, 1, axis) - _shift(f, 2, axis)) / (12.0 * h)


def central_l(f, axis, h, order=4):
    """Second derivative; order 4: (-f_{i-2} + 16 f_{i-1} - 30 f_i + 16 f_{i+1}
    - f_{i+2})/(12 h^2), order 2: (f_{i+1} - 2 f_i + f_{i-1})/h^2."""
    if order == 2:
        return (_shift(f, 1, axis) - 2.0 * f + _shift(f, -1, axis)) / (h * h)
    return (-_shift(f, -2, axis) + 16.0 * _shift(f, -1, axis) - 30.0 * f
            + 16.0 * _shift(f, 1, axis) - _shift(f, 2, axis)) / (12.0 * h * h)


def central_d_symbol(k, n, h, order=4):
    """Imaginary part of the Fourier symbol of central_d for integer wavenumber k on
    an n-point periodic grid (the symbol is i times this)."""
    k = np.asarray(k, dtype=np.float64)
    th = 2.0 * np.pi * k / n
    if order == 2:
        val = np.sin(th) / h
    else:
        val = (8.0 * np.sin(th) - np.sin(2.0 * th)) / (6.0 * h)
    # the symbol vanishes exactly at k = 0 and at the Nyquist wavenumber k = n/2
    return np.where(np.mod(2.0 * k, n) == 0.0, 0.0, val)


def central_l_symbol(k, n, h, order=4):
    """Fourier symbol (real) of central_l."""
    th = 2.0 * np.pi * np.asarray(k, dtype=np.float64) / n
    if order == 2:
        return (2.0 * np.cos(th) - 2.0) / (h * h)
    return (-2.0 * np.cos(2.0 * th) + 32.0 * np.cos(th) - 30.0) / (12.0 * h * h)


# ------------------------------------------------------------------ operator bundles

AX_X, AX_Y = 1, 0


class Production:
    """Operators of the scheme: WENO5 + fourth-order central differences (the
    high-order extension), or the narrower WENO3 + second-order central differences the
    paper's convergence tables use (weno_order, central_order)."""

    def __init__(self, hx, hy, alpha=1.0, central_order=4, eps_w=WENO_EPS, weno_order=5):
        self.hx, self.hy, self.alpha = hx, hy, alpha
        self.co = central_order
        self.eps_w = eps_w
        self.wo = weno_order

    # W^0 / W^1 directional flux derivatives
    def _w0(self, f, axis):
        h = self.hx if axis == AX_X else self.hy
        return weno_derivative(f, 0.0 * f, 0.0, axis, h, self.eps_w, self.wo)

    def _w1(self, f, w, axis):
        h = self.hx if axis == AX_X else self.hy
        return weno_derivative(f, w, self.alpha, axis, h, self.eps_w, self.wo)

    def div0_B(self, u1, u2):
        """D0_LF . B(u) -> WENO without dissipation: rows of B(u) = [[-u1, u2],[u2, u1]]."""
        return (self._w0(-u1, AX_X) + self._w0(u2, AX_Y),
                self._w0(u2, AX_X) + self._w0(u1, AX_Y))

    def grad_lf(self, q, v1, v2):
        """D_LF q with dissipation on v1 (x) and v2 (y)."""
        return self._w1(q, v1, AX_X), self._w1(q, v2, AX_Y)

    def div_lf_B(self, v1, v2, w1, w2):
        """D_LF . B(v) with dissipation on w1 (first row) and w2 (second row)."""
        return (self._w1(-v1, w1, AX_X) + self._w1(v2, w1, AX_Y),
                self._w1(v2, w2, AX_X) + self._w1(v1, w2, AX_Y))

    def div0(self, v1, v2):
        """D0_LF . v -> WENO without dissipation."""
        return self._w0(v1, AX_X) + self._w0(v2, AX_Y)

    def div_c(self, u1, u2):
        """D0 . u (central)."""
        return (central_d(u1, AX_X, self.hx, self.co)
                + central_d(u2, AX_Y, self.hy, self.co))

    def grad_c(self, th):
        """D0 theta (central)."""
        return central_d(th, AX_X, self.hx, self.co), central_d(th, AX_Y, self.hy, self.co)

    def lap(self, th):
        """D_Delta theta."""
        return central_l(th, AX_X, self.hx, self.co) + central_l(th, AX_Y, self.hy, self.co)

    def divdivB(self, v1, v2):
        """D0^2 : B(v) = -D_xx v1 + 2 D_xy v2 + D_yy v1 with D_xy = D_x D_y."""
        dxy = central_d(central_d(v2, AX_Y, self.hy, self.co), AX_X, self.hx, self.co)
        return (-central_l(v1, AX_X, self.hx, self.co) + 2.0 * dxy
                + central_l(v1, AX_Y, self.hy, self.co))

    def lap_symbol(self, nx, ny):
        """(lambda_x[kx], lambda_y[ky]) for the full FFT index ranges."""
        kx = np.fft.fftfreq(nx, d=1.0 / nx)
        ky = np.fft.fftfreq(ny, d=1.0 / ny)
        return (central_l_symbol(kx, nx, self.hx, self.co),
                central_l_symbol(ky, ny, self.hy, self.co))


class Consistent:
    """Test-only bundle in which every first derivative is the same central D and
    every second-order operator is a composition of D (D_Delta = D.D, D0^2:B(v) =
    D.(D.B(v))), with no numerical dissipation.  With it the fully discrete scheme is
    exactly an IMEX Runge-Kutta method for the semi-discrete moment system, so the
    stage algebra can be checked on its own."""

    def __init__(self, hx, hy, central_order=4):
        self.hx, self.hy, self.co = hx, hy, central_order

    def _dx(self, f):
        return central_d(f, AX_X, self.hx, self.co)

    def _dy(self, f):
        return central_d(f, AX_Y, self.hy, self.co)

    def div0_B(self, u1, u2):
        return -self._dx(u1) + self._dy(u2), self._dx(u2) + self._dy(u1)

    def grad_lf(self, q, v1, v2):
        return self._dx(q), self._dy(q)

    def div_lf_B(self, v1, v2, w1, w2):
        return -self._dx(v1) + self._dy(v2), self._dx(v2) + self._dy(v1)

    def div0(self, v1, v2):
        return self._dx(v1) + self._dy(v2)

    def div_c(self, u1, u2):
        return self._dx(u1) + self._dy(u2)

    def grad_c(self, th):
        return self._dx(th), self._dy(th)

    def lap(self, th):
        return self._dx(self._dx(th)) + self._dy(self._dy(th))

    def divdivB(self, v1, v2):
        b1, b2 = self.div_lf_B(v1, v2, None, None)
        return self._dx(b1) + self._dy(b2)

    def lap_symbol(self, nx, ny):
        kx = np.fft.fftfreq(nx, d=1.0 / nx)
        ky = np.fft.fftfreq(ny, d=1.0 / ny)
        sx = central_d_symbol(kx, nx, self.hx, self.co)
        sy = central_d_symbol(ky, ny, self.hy, self.co)
        return -sx * sx, -sy * sy
