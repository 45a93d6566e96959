"""Parity at the full sizes of the benchmark workloads, in the launch configuration the
benchmark times (autotuned launch shapes and stream structure, graph replay; at 8192^2 and
2048^2 the FFT kernels' register forms, every row and column filling its form).

The Helmholtz solve couples every cell, so the oracle cannot produce single cells of a
large grid one by one.  These tests use a property that holds at any size instead: every
operator of the scheme is translation invariant on the periodic grid and the Fourier
symbols depend on k h only, so a field made of m x m copies of a periodic n x n field
(domain m times larger, same h, same dt) stays m x m copies of the n x n solution.  The
oracle computes the n x n run; the HIP path runs the full grid (row and column FFT
kernels at their full lengths, the full tile grids) and must match every copy: relative
L-infinity <= 1e-11 per field in float64, relative L2 <= 1e-5 for velocity, theta and
density in the FP32-split form.  The batched workload is checked on one instance of every grid side."""

import sys

import numpy as np
import pytest

from oracle import scheme, tableau as otab
from oracle.operators import Production
from paper_2512_19847_amd import workloads as wl

pytestmark = pytest.mark.gpu

FIELDS = ("u1", "u2", "theta", "v1", "v2", "q")
TOL = 1e-11
TOL_L2 = 1e-5
BASE = 512


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _oracle(case, nsteps):
    ny, nx = case.state[0].shape
    return scheme.run(case.state, scheme.Params(case.eps, case.tau, case.dt),
                      otab.preset(case.tableau), Production(case.lx / nx, case.ly / ny), nsteps)


def _gpu(cases, nsteps, precision, tile=1):
    """Run the cases (each field tiled tile x tile on a domain tile times larger) as the
    benchmark does: autotuned shapes, graph replay."""
    import torch

    from paper_2512_19847_amd import apdvm
    sim = apdvm.Simulation([dict(nx=c.nx * tile, ny=c.ny * tile, eps=c.eps, tau=c.tau, dt=c.dt,
                                 lx=c.lx * tile, ly=c.ly * tile) for c in cases],
                           tableau=cases[0].tableau, precision=precision,
                           stream=torch.cuda.Stream())
    for k, c in enumerate(cases):
        sim.set_fields(k, *[np.tile(f, (tile, tile)) for f in c.state])
    sim.set_graph(True)
    _say(f"  tuned {sim.autotune(1)}")
    sim.step(nsteps)
    out = [sim.get_fields(k) for k in range(len(cases))]
    sim.close()
    return out


def _copies(g, tile):
    """View a (tile n) x (tile n) field as tile x n x tile x n."""
    ny, nx = g.shape
    return g.reshape(tile, ny // tile, tile, nx // tile)


def _linf(got, ref, tile):
    """Per field max |gpu - oracle| over every copy, over max |oracle| (fields that vanish
    identically against the largest field)."""
    scale = max(np.max(np.abs(r)) for r in ref)
    out = {}
    for name, g, r in zip(FIELDS, got, ref):
        m = np.max(np.abs(r))
        den = m if m > 1e-12 * scale else scale
        out[name] = float(np.max(np.abs(_copies(g, tile) - r[None, :, None, :])) / den)
    return out


def _l2(got, ref, eps, tile):
    """Relative L2 of velocity, of theta (the density fluctuation (rho - 1) / (2 eps^2))
    and of the density 1 + 2 eps^2 theta over every copy."""
    gu = [_copies(g, tile) for g in got[:2]]
    du = sum(np.sum((g - r[None, :, None, :]) ** 2) for g, r in zip(gu, ref[:2]))
    nu = tile * tile * sum(np.sum(r ** 2) for r in ref[:2])
    gth = _copies(got[2], tile)
    rho_r = 1 + 2 * eps * eps * ref[2]
    dr = np.sum((1 + 2 * eps * eps * gth - rho_r[None, :, None, :]) ** 2)
    nr = tile * tile * np.sum(rho_r ** 2)
    dth = np.sum((gth - ref[2][None, :, None, :]) ** 2)
    nth = tile * tile * np.sum(ref[2] ** 2)
    return dict(u=float(np.sqrt(du / nu)), theta=float(np.sqrt(dth / nth)),
                rho=float(np.sqrt(dr / nr)))


@pytest.fixture(scope="module")
def shear_8192():
    """The 8192^2 shear-layer workload's parameters (eps = 1e-4, Ma = 0.02, ARS(4,4,3)) on
    copies of a 512^2 shear layer, and the oracle's two steps of that layer."""
    case = wl.make_case("shear_base", wl.shear_layer(BASE), 1e-4, 0.02, "ars443", cfl=wl.CFL_ARS)
    return case, _oracle(case, 2)


@pytest.fixture(scope="module")
def random_2048():
    """The 2048^2 random-field workload's parameters (eps = 1e-6, Ma = 0.01, |k| <= 8) on
    copies of a 512^2 random divergence-free field."""
    case = wl.make_case("random_base", wl.random_divfree(BASE, kmax=8, rms=0.1, seed=3), 1e-6,
                        0.01, "ars443", cfl=wl.CFL_ARS)
    return case, _oracle(case, 2)


@pytest.mark.parametrize("precision", ["fp64", "fp32split"])
def test_shear_layer_8192(shear_8192, precision):
    from paper_2512_19847_amd import apdvm
    case, ref = shear_8192
    tile = 8192 // BASE
    _say(f"case shear 8192^2 as {tile}x{tile} copies, {precision}, 2 steps dt={case.dt}")
    got = _gpu([case], 2, apdvm.FP64 if precision == "fp64" else apdvm.FP32_SPLIT, tile)[0]
    if precision == "fp64":
        err = _linf(got, ref, tile)
        _say(f"  relerr {err}")
        assert max(err.values()) <= TOL, err
    else:
        err = _l2(got, ref, case.eps, tile)
        _say(f"  rel L2 {err}")
        assert max(err.values()) <= TOL_L2, err


@pytest.mark.parametrize("precision", ["fp64", "fp32split"])
def test_random_field_2048(random_2048, precision):
    from paper_2512_19847_amd import apdvm
    case, ref = random_2048
    tile = 2048 // BASE
    _say(f"case random 2048^2 as {tile}x{tile} copies, {precision}, 2 steps dt={case.dt}")
    got = _gpu([case], 2, apdvm.FP64 if precision == "fp64" else apdvm.FP32_SPLIT, tile)[0]
    if precision == "fp64":
        err = _linf(got, ref, tile)
        _say(f"  relerr {err}")
        assert max(err.values()) <= TOL, err
    else:
        err = _l2(got, ref, case.eps, tile)
        _say(f"  rel L2 {err}")
        assert max(err.values()) <= TOL_L2, err


@pytest.mark.parametrize("precision", ["fp64", "fp32split"])
def test_batched_256_sampled_instances(precision):
    """All 256 instances in one context; the first instance of every grid side is checked
    against the oracle after one step."""
    from paper_2512_19847_amd import apdvm
    cases = wl.batched_256()
    sample = {}
    for k, c in enumerate(cases):
        sample.setdefault(c.nx, k)
    _say(f"case batched 256, {precision}, 1 step, sampled instances {sorted(sample.values())}")
    got = _gpu(cases, 1, apdvm.FP64 if precision == "fp64" else apdvm.FP32_SPLIT)
    for n, k in sorted(sample.items()):
        ref = _oracle(cases[k], 1)
        if precision == "fp64":
            err = _linf(got[k], ref, 1)
            _say(f"  instance {k} ({n}^2, eps={cases[k].eps:.3g}) relerr {err}")
            assert max(err.values()) <= TOL, (k, err)
        else:
            err = _l2(got[k], ref, cases[k].eps, 1)
            _say(f"  instance {k} ({n}^2, eps={cases[k].eps:.3g}) rel L2 {err}")
            assert max(err.values()) <= TOL_L2, (k, err)
