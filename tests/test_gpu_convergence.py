"""Convergence study of Section 4.1 (Tables 1 and 2) on the GPU path: thick double shear
layer (rho = pi/15, delta = 0.05) at eps = 1e-6, tau = 0, t = 1, the paper's first-order
(GSA Euler) and second-order IMEX tableaux with third-order WENO and second-order central
differences, vorticity u2_x - u1_y against a 1024^2 run of the same scheme, dt a fixed
multiple of h.  A second test shows on the GPU what the oracle pins on the CPU: on a
fixed grid the printed operators leave an O(dt h^4) term, so the fixed-grid order in
time is one whatever the tableau, with a constant that falls like h^4.

Readings (the paper does not state them): N = 33..513 grid points of a periodic grid are
read as 32..1024 cells (cell-centred, h = 2 pi / N); dt = 0.2 h (Euler) and 0.2 h / 2.25
(second-order tableau, whose explicit stage of length 2.25 dt must stay below 0.2 h with
WENO3); the vorticity is the derivative of the trigonometric interpolant on each grid,
and the reference is sampled at the coarse cell centres through its interpolant (the flow
is smooth at t = 1); L1 = h^2 sum |e|, L2 = (h^2 sum e^2)^(1/2), Linf = max |e|.  Under
these readings the space error dominates at every N (halving dt changes the errors by a
few per cent), so both tableaux converge at the WENO3 rate, at least second order on the
finer grids.  Against the printed tables (tests/golden/convergence_tables.json): the L1
and L2 orders of Table 2's finest pair are reproduced; the magnitudes (printed errors
90x to 650x smaller) and Table 1's orders near one are not, under these readings or the
others tried (the layer profile tanh(rho (y - pi/2)), alpha = 0, which is unstable): they
stay parity unpinned."""

import json
import math
import os
import sys

import numpy as np
import pytest

from paper_2512_19847_amd import workloads as wl

pytestmark = pytest.mark.gpu

CFL = {"euler1": 0.2, "paper2": 0.2 / 2.25}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _solve(n, tab, m, T=1.0):
    from paper_2512_19847_amd import apdvm
    st = wl.shear_layer(n)
    sim = apdvm.Simulation([dict(nx=n, ny=n, eps=1e-6, tau=0.0, dt=T / m)], tableau=tab,
                           weno_order=3, central_order=2)
    sim.set_fields(0, *st)
    sim.step(m)
    out = sim.get_fields(0)
    sim.close()
    assert all(np.all(np.isfinite(f)) for f in out)
    return out


def _steps(n, tab):
    return int(math.ceil(1.0 / (CFL[tab] * 2 * math.pi / n)))


def _vorticity(u1, u2):
    n = u1.shape[0]
    k = np.fft.fftfreq(n, d=1.0 / n)
    k[n // 2] = 0.0  # the Nyquist mode has no odd derivative on the grid
    w = 1j * k[None, :] * np.fft.fft2(u2) - 1j * k[:, None] * np.fft.fft2(u1)
    return np.real(np.fft.ifft2(w))


def _sample(f, nc):
    """Trigonometric interpolant of the cell-centred f (n x n) at the cell centres of
    the nc x nc grid."""
    nf = f.shape[0]
    r = nf // nc
    k = np.fft.fftfreq(nf, d=1.0 / nf)
    ph = np.exp(2j * np.pi * k * (r - 1) / 2.0 / nf)
    F = np.fft.fft2(f) * ph[None, :] * ph[:, None]
    kc = np.fft.fftfreq(nc, d=1.0 / nc).astype(int)
    idx = np.where(kc >= 0, kc, kc + nf)
    Fc = F[np.ix_(idx, idx)] * (nc * nc) / (nf * nf)
    Fc[nc // 2, :] = 0.0
    Fc[:, nc // 2] = 0.0
    return np.real(np.fft.ifft2(Fc))


def _norms(e, n):
    h = 2 * math.pi / n
    return h * h * np.sum(np.abs(e)), math.sqrt(h * h * np.sum(e * e)), np.max(np.abs(e))


def _orders(rows):
    return [None] * 3 if len(rows) < 2 else [math.log2(rows[-2][j] / rows[-1][j])
                                             for j in (1, 2, 3)]


def test_fixed_grid_time_order_of_the_printed_operators():
    """Taylor-Green at eps = 1e-6, tau = 0.05, ARS(4,4,3), WENO5 + fourth-order central:
    first order in dt on a fixed grid, with an error constant falling like h^4."""
    from paper_2512_19847_amd import apdvm

    def run(n, m, T=0.25):
        sim = apdvm.Simulation([dict(nx=n, ny=n, eps=1e-6, tau=0.05, dt=T / m)], tableau="ars443")
        sim.set_fields(0, *wl.taylor_green(n))
        sim.step(m)
        out = sim.get_fields(0)
        sim.close()
        return out

    res = {}
    for n in (64, 128):
        ref = run(n, 1024)
        res[n] = [max(np.max(np.abs(o[k] - ref[k])) for k in (0, 1))
                  for o in (run(n, 32), run(n, 64))]
        _say(f"fixed grid {n}^2: dt = T/32, T/64 max |u - u_ref| {res[n]}, order "
             f"{math.log2(res[n][0] / res[n][1]):.2f}")
    for n in (64, 128):
        assert 0.8 < math.log2(res[n][0] / res[n][1]) < 1.3, res
    assert 10.0 < res[64][1] / res[128][1] < 30.0, res


def _table(tab):
    ref = _solve(1024, tab, _steps(1024, tab))
    w_ref = _vorticity(ref[0], ref[1])
    rows = []
    for n in (32, 64, 128, 256, 512):
        u = _solve(n, tab, _steps(n, tab))
        rows.append((n,) + _norms(_vorticity(u[0], u[1]) - _sample(w_ref, n), n))
    return rows


@pytest.fixture(scope="module")
def tables():
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "convergence_tables.json")))
    out = {}
    fmt = lambda x: "   --" if x is None else f"{x:5.2f}"
    for tab in ("euler1", "paper2"):
        rows = _table(tab)
        out[tab] = rows
        _say(f"space-time {tab} (ref 1024^2): N, L1, L2, Linf, orders | printed N, L1, "
             f"orders | ours / printed L1")
        for i, r in enumerate(rows):
            o = _orders(rows[:i + 1])
            g = gold[tab][i] if i < len(gold[tab]) else None
            ptxt = "" if g is None else (f" | {g[0]:4d} {g[1]:.3e} {fmt(g[2])} {fmt(g[4])} "
                                         f"{fmt(g[6])} | {r[1] / g[1]:7.1f}")
            _say(f"  {r[0]:5d} {r[1]:.4e} {r[2]:.4e} {r[3]:.4e}  "
                 + " ".join(fmt(x) for x in o) + ptxt)
    return gold, out


def test_second_order_tableau_orders_match_the_printed_table(tables):
    """Table 2 (the second-order tableau): the L1 and L2 orders of the finest printed pair
    (129 -> 257 points, 2.02 and 1.95) are reproduced by the 128 -> 256 pair within 0.25.
    The printed L-infinity order (2.13) is not: the layer is resolved by a few cells at
    these N, and the maximum error sits where the WENO3 weights switch stencils."""
    gold, rows = tables
    g = gold["paper2"]
    ours = _orders(rows["paper2"][:4])
    assert abs(ours[0] - g[3][2]) <= 0.25, (ours, g[3])
    assert abs(ours[1] - g[3][4]) <= 0.25, (ours, g[3])


def test_space_error_dominates_under_these_readings(tables):
    """Under the readings of the module docstring the space error dominates: the GSA Euler
    and the second-order tableau give L1 and L2 errors within 15% of each other at every N,
    and both converge at the WENO3 rate (at least 1.8 on the finer pairs).  The printed
    tables differ here: there the first-order tableau's errors are 1.6x (N = 33) to 12.6x
    (N = 257) the second-order ones and its orders stay near one, a time-error-dominated
    study, at errors 90x to 650x smaller than these.  Which setting produces that is not
    stated; the magnitudes and the Table 1 orders stay parity unpinned."""
    gold, rows = tables
    for a, b in zip(rows["euler1"], rows["paper2"]):
        assert abs(a[1] / b[1] - 1.0) <= 0.15 and abs(a[2] / b[2] - 1.0) <= 0.15, (a, b)
    for tab in ("euler1", "paper2"):
        r = rows[tab]
        for r0, r1 in zip(r[2:-1], r[3:]):
            assert math.log2(r0[1] / r1[1]) >= 1.8, r
            assert math.log2(r0[2] / r1[2]) >= 1.8, r
    ratios = [gold["euler1"][i][1] / gold["paper2"][i][1] for i in range(4)]
    assert ratios[0] > 1.5 and ratios[-1] > 10.0, ratios  # the printed tables, as stored
