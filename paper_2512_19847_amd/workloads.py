"""Seeded synthetic inputs shared by the oracle checks, the GPU tests and the
benchmark.  This module holds input recipes only (initial fields, tau from eps and
Mach, a time-step rule); none of the scheme's arithmetic lives here.  All arrays are
float64, shape (ny, nx), x the fast axis, cell centres x_i = (i + 1/2) h on a periodic
box [0, lx) x [0, ly).

Recipes
  taylor_green     u = A (sin x cos y, -cos x sin y), p = -(A^2/4)(cos 2x + cos 2y).
  shear_layer      the doubly periodic shear layer of Section 4.1:
                   u1 = tanh((y - pi/2)/rho) for y <= pi, tanh((3pi/2 - y)/rho) else,
                   u2 = delta sin x; rho = pi/15 (thick), pi/50 (thin); delta = 0.05.
  kelvin_helmholtz u = (cos y, 0.03 sin(x/2)) on [0, 4pi)^2 (Section 4.3).
  random_divfree   stream function with complex Gaussian amplitudes on the modes
                   1 <= |k| <= kmax, u = (D_y psi, -D_x psi) with the fourth-order
                   central difference D (the discrete curl: the scheme's central
                   divergence of u is then zero to rounding, the well-prepared data of
                   Theorem 3.5), scaled to the requested root-mean-square speed
                   sqrt(mean(u1^2 + u2^2)).
The kinetic moments start at local equilibrium: v = F(u) = (1/2 (u2^2 - u1^2), u1 u2),
q = 0, theta = p + |u|^2 / 2 (the definition p = theta - |u|^2/2 of Section 2.1), where
p is the incompressible pressure: closed form for Taylor-Green, else the spectral
solution of Lap p = -d_i u_j d_j u_i.
"""

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def tau_from(eps, mach):
    """tau = 4 eps / Ma: eps = Ma / Re and the limit Reynolds number is Re = 4 / tau."""
    return 4.0 * eps / mach


def dt_rule(umax, eps, tau, h, cfl=0.4, c_visc=0.2, alpha=1.0):
    """Largest dt with  dt * max(umax, alpha, tau eps / (tau eps^2 + dt)) <= cfl h  and
    dt * (tau / 4) * dt / (tau eps^2 + dt) <= c_visc h^2  (bisection; both left sides
    grow with dt).  The paper states no time-step rule; this one bounds the explicit
    transport speeds (the flow speed, the Lax-Friedrichs dissipation speed alpha = 1
    whose jump term acts explicitly, and the kinetic speed 1/eps damped by
    relaxation) and the explicit viscous term of the limit scheme."""
    te2 = tau * eps * eps

    def ok(dt):
        kin = tau * eps / (te2 + dt) if (te2 + dt) > 0 else 0.0
        hyp = dt * max(umax, alpha, kin) <= cfl * h
        par = dt * 0.25 * tau * dt / (te2 + dt) <= c_visc * h * h
        return hyp and par

    lo, hi = 0.0, 100.0 * h
    if ok(hi):
        return hi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if ok(mid):
            lo = mid
        else:
            hi = mid
    return lo


def grid(nx, ny, lx=TWO_PI, ly=TWO_PI):
    hx, hy = lx / nx, ly / ny
    x = (np.arange(nx) + 0.5) * hx
    y = (np.arange(ny) + 0.5) * hy
    X, Y = np.meshgrid(x, y)  # shape (ny, nx)
    return X, Y, hx, hy


def _spectral_k(n, L):
    return np.fft.fftfreq(n, d=L / n) * TWO_PI


def _spectral_d(f, axis, L):
    n = f.shape[axis]
    k = _spectral_k(n, L)
    shape = [1, 1]
    shape[axis] = n
    return np.real(np.fft.ifft(1j * k.reshape(shape) * np.fft.fft(f, axis=axis), axis=axis))


def _discrete_d(f, axis, h):
    """Fourth-order central first difference (f_{i-2} - 8 f_{i-1} + 8 f_{i+1} - f_{i+2})
    / (12 h) along axis, periodic."""
    r = lambda k: np.roll(f, -k, axis=axis)  # noqa: E731  r(k)[i] = f[i + k]
    return (r(-2) - 8.0 * r(-1) + 8.0 * r(1) - r(2)) / (12.0 * h)


def pressure_poisson(u1, u2, lx=TWO_PI, ly=TWO_PI):
    """Zero-mean p with Lap p = -(d_i u_j)(d_j u_i), spectral."""
    ux = _spectral_d(u1, 1, lx)
    uy = _spectral_d(u1, 0, ly)
    vx = _spectral_d(u2, 1, lx)
    vy = _spectral_d(u2, 0, ly)
    rhs = -(ux * ux + 2.0 * uy * vx + vy * vy)
    ny, nx = u1.shape
    kx = _spectral_k(nx, lx)
    ky = _spectral_k(ny, ly)
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    rh = np.fft.fft2(rhs)
    ph = np.where(k2 > 0, -rh / np.where(k2 > 0, k2, 1.0), 0.0)
    return np.real(np.fft.ifft2(ph))


def equilibrium_state(u1, u2, p):
    """(u1, u2, theta, v1, v2, q) with the kinetic moments at local equilibrium."""
    th = p + 0.5 * (u1 * u1 + u2 * u2)
    v1 = 0.5 * (u2 * u2 - u1 * u1)
    v2 = u1 * u2
    return (u1.copy(), u2.copy(), th, v1, v2, np.zeros_like(u1))


def taylor_green(nx, ny=None, amp=0.1):
    ny = nx if ny is None else ny
    X, Y, _, _ = grid(nx, ny)
    u1 = amp * np.sin(X) * np.cos(Y)
    u2 = -amp * np.cos(X) * np.sin(Y)
    p = -(amp * amp / 4.0) * (np.cos(2 * X) + np.cos(2 * Y))
    return equilibrium_state(u1, u2, p)


def taylor_green_exact(nx, ny, amp, nu, t):
    """Closed-form incompressible Navier-Stokes Taylor-Green velocity and pressure."""
    X, Y, _, _ = grid(nx, ny)
    d = math.exp(-2.0 * nu * t)
    u1 = amp * d * np.sin(X) * np.cos(Y)
    u2 = -amp * d * np.cos(X) * np.sin(Y)
    p = -(amp * amp / 4.0) * d * d * (np.cos(2 * X) + np.cos(2 * Y))
    return u1, u2, p


def shear_layer(nx, ny=None, rho=math.pi / 15.0, delta=0.05):
    ny = nx if ny is None else ny
    X, Y, _, _ = grid(nx, ny)
    u1 = np.where(Y <= math.pi, np.tanh((Y - math.pi / 2) / rho),
                  np.tanh((1.5 * math.pi - Y) / rho))
    u2 = delta * np.sin(X)
    return equilibrium_state(u1, u2, pressure_poisson(u1, u2))


def ill_prepared(nx, ny=None, kmax=4, rms=0.1, grad_rms=0.05, seed=0):
    """A divergence-free random field plus the gradient of a random potential (rms
    speeds rms and grad_rms, modes 1 <= |k| <= kmax, default_rng(seed) and seed + 1):
    initial data that is not well prepared for the incompressible limit (div u = O(1),
    Theorem 3.4 against Theorem 3.5), with theta from the pressure equation of the
    whole field and the kinetic moments at local equilibrium."""
    ny = nx if ny is None else ny
    u1, u2 = random_divfree(nx, ny, kmax=kmax, rms=rms, seed=seed)[:2]
    rng = np.random.default_rng(seed + 1)
    kx = np.fft.fftfreq(nx, d=1.0 / nx)
    ky = np.fft.fftfreq(ny, d=1.0 / ny)
    KX, KY = np.meshgrid(kx, ky)
    kk = np.sqrt(KX ** 2 + KY ** 2)
    amp = np.where((kk >= 1) & (kk <= kmax),
                   rng.standard_normal(kk.shape) + 1j * rng.standard_normal(kk.shape), 0.0)
    phi_h = np.fft.fft2(np.real(np.fft.ifft2(amp)))
    g1 = np.real(np.fft.ifft2(1j * KX * phi_h))
    g2 = np.real(np.fft.ifft2(1j * KY * phi_h))
    scale = grad_rms / math.sqrt(np.mean(g1 * g1 + g2 * g2))
    w1, w2 = u1 + scale * g1, u2 + scale * g2
    return equilibrium_state(w1, w2, pressure_poisson(w1, w2))


def thin_shear_layer(nx, ny=None):
    """Thin shear layer of Section 4.1: the thick layer with rho = pi / 50."""
    return shear_layer(nx, ny, rho=math.pi / 50.0)


def kelvin_helmholtz(nx, ny=None):
    ny = nx if ny is None else ny
    L = 2.0 * TWO_PI
    X, Y, _, _ = grid(nx, ny, L, L)
    u1 = np.cos(Y)
    u2 = 0.03 * np.sin(0.5 * X)
    return equilibrium_state(u1, u2, pressure_poisson(u1, u2, L, L))


def random_divfree(nx, ny=None, kmax=8, rms=0.1, seed=0):
    ny = nx if ny is None else ny
    rng = np.random.default_rng(seed)
    kx = np.fft.fftfreq(nx, d=1.0 / nx)
    ky = np.fft.fftfreq(ny, d=1.0 / ny)
    kk = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    mask = (kk >= 1.0) & (kk <= kmax)
    g = rng.standard_normal((2, ny, nx))
    psih = np.where(mask, (g[0] + 1j * g[1]) / math.sqrt(2.0), 0.0)
    psi = np.real(np.fft.ifft2(psih)) * (nx * ny)
    u1 = _discrete_d(psi, 0, TWO_PI / ny)
    u2 = -_discrete_d(psi, 1, TWO_PI / nx)
    r = math.sqrt(float(np.mean(u1 * u1 + u2 * u2)))
    u1 *= rms / r
    u2 *= rms / r
    return equilibrium_state(u1, u2, pressure_poisson(u1, u2))


def umax(state):
    return float(np.max(np.sqrt(state[0] ** 2 + state[1] ** 2)))


# ----------------------------------------------------------------- named workloads

class Case:
    """One simulation instance: fields plus (eps, tau, dt, tableau name)."""

    def __init__(self, name, state, eps, tau, dt, tableau, lx=TWO_PI, ly=TWO_PI):
        self.name, self.state = name, state
        self.eps, self.tau, self.dt, self.tableau = eps, tau, dt, tableau
        self.ny, self.nx = state[0].shape
        self.lx, self.ly = lx, ly

    @property
    def cells(self):
        return self.nx * self.ny


# Largest explicit stage abscissa (max_i sum_j at_ij) of each preset tableau.  The
# explicit part of a stage advances c~_i dt, so the CFL bound is applied to
# c~_max dt: with c~_max = 9/4 the paper's second-order tableau is unstable in the
# kinetic regime at dt = 0.4 h (eps = 1, tau = 40) and stable at 0.4 h / c~_max.
STAGE_REACH = {"euler1": 1.0, "paper2": 2.25, "ars443": 1.0}


def make_case(name, state, eps, mach, tableau, cfl=0.4, tau=None, lx=TWO_PI, ly=TWO_PI):
    tau = tau_from(eps, mach) if tau is None else tau
    ny, nx = state[0].shape
    h = min(lx / nx, ly / ny)
    dt = dt_rule(umax(state), eps, tau, h, cfl / STAGE_REACH[tableau])
    return Case(name, state, eps, tau, dt, tableau, lx, ly)


def taylor_green_64(tableau="paper2"):
    """64^2 Taylor-Green vortex, amplitude 0.1, eps = 1, Ma = 0.1 (tau = 40), CFL 0.4,
    100 steps: the small plain-method case."""
    return make_case("taylor_green_64", taylor_green(64), 1.0, 0.1, tableau)


# CFL number of the third-order runs: with max|u| = 1 the thick shear layer at
# eps = 1e-6 is unstable at 0.35 and stable at 0.3 up to t = 6 (oracle, 128^2).
CFL_ARS = 0.25


def shear_layer_512(eps, n=512):
    """512^2 thick shear layer, Ma = 0.05, third-order IMEX (ARS(4,4,3)), 2000 steps."""
    return make_case(f"shear_layer_{n}_eps{eps:g}", shear_layer(n), eps, 0.05, "ars443",
                     cfl=CFL_ARS)


def random_2048(n=2048):
    """2048^2 random divergence-free field, |k| <= 8, rms 0.1, eps = 1e-6, Ma = 0.01."""
    return make_case(f"random_{n}", random_divfree(n, kmax=8, rms=0.1, seed=3),
                     1e-6, 0.01, "ars443", cfl=CFL_ARS)


BATCH_SIDES = (64, 96, 128, 192, 256, 384, 512)


def _batch_params(count, seed, sides):
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.array(sides), count)
    epss = 10.0 ** rng.uniform(-6.0, 0.0, count)
    machs = rng.uniform(0.01, 0.1, count)
    return ns, epss, machs


def batched_256_instance(k, count=256, seed=4, sides=BATCH_SIDES):
    """Instance k of batched_256 alone (the same draws)."""
    ns, epss, machs = _batch_params(count, seed, sides)
    st = random_divfree(int(ns[k]), kmax=4, rms=0.1, seed=1000 + k)
    return make_case(f"batch_{k}", st, float(epss[k]), float(machs[k]), "ars443", cfl=CFL_ARS)


def batched_256(count=256, seed=4, sides=BATCH_SIDES):
    """256 independent instances: side uniform over sides, eps log-uniform in
    [1e-6, 1], Ma uniform in [0.01, 0.1], random divergence-free fields with |k| <= 4
    (rms 0.1, seed 1000 + k)."""
    return [batched_256_instance(k, count, seed, sides) for k in range(count)]


# Long runs of Section 4.1 and the Kelvin-Helmholtz test: (generator, box side, final
# time).  eps = 1e-6; tau = 0 (incompressible Euler limit) or 0.05 (Navier-Stokes).
FLOWS = {
    "thick_shear_layer": (shear_layer, TWO_PI, {0.0: 6.0, 0.05: 9.5}),
    "thin_shear_layer": (thin_shear_layer, TWO_PI, {0.0: 6.0, 0.05: 9.5}),
    "kelvin_helmholtz": (kelvin_helmholtz, 2.0 * TWO_PI, {0.0: 45.0, 0.05: 45.0}),
}


def flow_case(kind, n, tau, eps=1e-6, tableau="ars443", cfl=CFL_ARS):
    """One of FLOWS on an n x n grid with the time step of the rule above."""
    gen, L, _ = FLOWS[kind]
    return make_case(f"{kind}_{n}_tau{tau:g}", gen(n), eps, 1.0, tableau, cfl=cfl, tau=tau,
                     lx=L, ly=L)


def shear_layer_8192(n=8192):
    """8192^2 shear layer, eps = 1e-4, Ma = 0.02, ARS(4,4,3), 200 steps."""
    return make_case(f"shear_layer_{n}", shear_layer(n), 1e-4, 0.02, "ars443", cfl=CFL_ARS)
