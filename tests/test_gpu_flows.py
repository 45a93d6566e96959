"""Long runs of Section 4.1 and the Kelvin-Helmholtz test on the GPU path, eps = 1e-6,
ARS(4,4,3) with WENO5 and fourth-order central differences (the high-order scheme), with
the time history of the maximum norm of the discrete divergence D0.u that the paper's
figures show: the thick (rho = pi/15) and thin (rho = pi/50) double shear layers on
512^2 to t = 6 (tau = 0, incompressible Euler) and t = 9.5 (tau = 0.05, Navier-Stokes),
and the Kelvin-Helmholtz instability on [0, 4 pi]^2, 256^2, to t = 45 for both tau (the
text names tau = 0, the figure caption tau = 0.05).  The grid of the shear layers is not
stated in the paper; 512^2 is used.

Checks: every field stays finite; sum u and sum theta stay at their initial values to
rounding (the scheme conserves them exactly: flux differences telescope and the
Helmholtz solve keeps the mean of theta); the kinetic energy does not grow.  The
divergence norm starts at zero (both velocity components of these initial data depend on
one coordinate only) and its history is printed beside the vorticity extrema and the
energy."""

import math
import sys

import numpy as np
import pytest

from paper_2512_19847_amd import workloads as wl

pytestmark = pytest.mark.gpu

RUNS = [("thick_shear_layer", 512, 0.0), ("thick_shear_layer", 512, 0.05),
        ("thin_shear_layer", 512, 0.0), ("thin_shear_layer", 512, 0.05),
        ("kelvin_helmholtz", 256, 0.0), ("kelvin_helmholtz", 256, 0.05)]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("kind,n,tau", RUNS)
def test_long_run_divergence_history(kind, n, tau):
    from paper_2512_19847_amd import apdvm
    case = wl.flow_case(kind, n, tau)
    T = wl.FLOWS[kind][2][tau]
    nsteps = int(math.ceil(T / case.dt))
    dt = T / nsteps
    sim = apdvm.Simulation([dict(nx=n, ny=n, eps=case.eps, tau=tau, dt=dt, lx=case.lx,
                                 ly=case.ly)], tableau="ars443")
    sim.set_fields(0, *case.state)
    d0 = sim.diagnostics(0)
    _say(f"{kind} {n}^2 tau={tau} dt={dt:.5f} steps={nsteps}: t, max|div u|, vorticity "
         f"min/max, kinetic energy, sum theta")
    hist = [(0.0, d0)]
    _say(f"  {0.0:6.2f} {d0[3]:.3e} {d0[4]:+.4f} {d0[5]:+.4f} {d0[6]:.8f} {d0[0]:+.6e}")
    chunks = 20
    done = 0
    for c in range(1, chunks + 1):
        target = (nsteps * c) // chunks
        sim.step(target - done)
        done = target
        d = sim.diagnostics(0)
        hist.append((done * dt, d))
        _say(f"  {done * dt:6.2f} {d[3]:.3e} {d[4]:+.4f} {d[5]:+.4f} {d[6]:.8f} {d[0]:+.6e}")
    sim.close()
    area = case.lx * case.ly
    for t, d in hist:
        assert d[7] == 1.0, (t, d)
        assert abs(d[0] - d0[0]) <= 1e-12 * area * max(1.0, abs(d0[0]) / area), (t, d[0], d0[0])
        assert abs(d[1] - d0[1]) <= 1e-11 * area and abs(d[2] - d0[2]) <= 1e-11 * area, (t, d)
    ke = [d[6] for _, d in hist]
    assert max(ke) <= ke[0] * (1 + 1e-6), ke
