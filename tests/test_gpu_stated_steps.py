"""Parity and precision at the step counts the workloads state.

* 512^2 shear layer at eps = 1, 1e-2, 1e-6 (the float64 workload, stated 2000 steps):
  the full grid against the oracle over 40 steps per eps (the oracle's cost bounds the
  length: 40 steps are ~35 s of one core per eps; the oracle runs in parallel worker
  processes), with the twin experiment: the oracle against itself from inputs perturbed by
  1e-16 relative gives the intrinsic amplification floor of the flow, and the GPU's error
  must stay within 30 times that floor or 1e-11 at every checkpoint.  The growth curves
  are printed.
* The 256-instance batch (stated 500 steps): every instance against the oracle after 3
  steps in float64; every instance of the FP32-split form against the float64 GPU run
  after the stated 500 steps (relative L2 of u, theta and rho <= 1e-5).
* The 8192^2 shear layer (stated 200 steps): FP32-split against float64 after 200 steps.
"""

import sys

import numpy as np
import pytest

import _oracle_pool
from paper_2512_19847_amd import workloads as wl

pytestmark = pytest.mark.gpu

FIELDS = ("u1", "u2", "theta", "v1", "v2", "q")
TOL = 1e-11
TOL_L2 = 1e-5
WORKERS = 8


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _relerr(got, ref):
    scale = max(np.max(np.abs(r)) for r in ref)
    out = {}
    for name, g, r in zip(FIELDS, got, ref):
        m = np.max(np.abs(r))
        out[name] = float(np.max(np.abs(g - r)) / (m if m > 1e-12 * scale else scale))
    return out


def _l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2)) / np.sqrt(np.sum(b ** 2)))


def _split_errors(f32, f64, eps):
    return dict(u=_l2(np.stack(f32[:2]), np.stack(f64[:2])), theta=_l2(f32[2], f64[2]),
                rho=_l2(1 + 2 * eps * eps * f32[2], 1 + 2 * eps * eps * f64[2]))


def test_shear_layer_512_long_runs_with_twin_floor():
    from paper_2512_19847_amd import apdvm
    epss = (1.0, 1e-2, 1e-6)
    checkpoints = [10, 20, 30, 40]
    _say(f"case shear512 eps {epss}: {checkpoints[-1]} steps, oracle and twin in workers")
    specs = []
    for e in epss:
        specs.append(dict(kind="shear512", eps=e, checkpoints=checkpoints, perturb=None))
        specs.append(dict(kind="shear512", eps=e, checkpoints=checkpoints, perturb=7))
    ref = _oracle_pool.pool_map(specs, WORKERS)
    for m, e in enumerate(epss):
        case = wl.shear_layer_512(e)
        sim = apdvm.Simulation([dict(nx=512, eps=case.eps, tau=case.tau, dt=case.dt)],
                               tableau="ars443")
        sim.set_fields(0, *case.state)
        done = 0
        for ck in checkpoints:
            sim.step(ck - done)
            done = ck
            got = sim.get_fields(0)
            e_gpu = _relerr(got, ref[2 * m][ck])
            e_twin = _relerr(ref[2 * m + 1][ck], ref[2 * m][ck])
            _say(f"  eps={e:g} step {ck}: gpu max {max(e_gpu.values()):.2e} "
                 f"twin max {max(e_twin.values()):.2e}  gpu {e_gpu}")
            for f in FIELDS:
                assert e_gpu[f] <= max(TOL, 30 * e_twin[f]), (e, ck, f, e_gpu[f], e_twin[f])
        sim.close()


def test_batched_256_every_instance():
    import torch

    from paper_2512_19847_amd import apdvm
    cases = wl.batched_256()
    nsteps = 3
    _say(f"case batched 256, every instance against the oracle after {nsteps} steps")
    ref = _oracle_pool.pool_map([dict(kind="batched256", index=k, checkpoints=[nsteps])
                                 for k in range(len(cases))], 16)
    sim = apdvm.Simulation([dict(nx=c.nx, ny=c.ny, eps=c.eps, tau=c.tau, dt=c.dt)
                            for c in cases], tableau="ars443", stream=torch.cuda.Stream())
    for k, c in enumerate(cases):
        sim.set_fields(k, *c.state)
    sim.set_graph(True)
    sim.autotune(1)
    sim.step(nsteps)
    worst = 0.0
    for k in range(len(cases)):
        err = _relerr(sim.get_fields(k), ref[k][nsteps])
        worst = max(worst, max(err.values()))
        assert max(err.values()) <= TOL, (k, cases[k].nx, cases[k].eps, err)
    sim.close()
    _say(f"  worst relative L-infinity over 256 instances and 6 fields: {worst:.2e}")


def test_batched_256_split_stated_steps():
    import torch

    from paper_2512_19847_amd import apdvm
    cases = wl.batched_256()
    nsteps = 500
    _say(f"case batched 256 FP32-split against float64, {nsteps} steps")
    out = []
    for prec in (apdvm.FP32_SPLIT, apdvm.FP64):
        sim = apdvm.Simulation([dict(nx=c.nx, ny=c.ny, eps=c.eps, tau=c.tau, dt=c.dt)
                                for c in cases], tableau="ars443", precision=prec,
                               stream=torch.cuda.Stream())
        for k, c in enumerate(cases):
            sim.set_fields(k, *c.state)
        sim.set_graph(True)
        sim.autotune(1)
        sim.step(nsteps)
        out.append([sim.get_fields(k) for k in range(len(cases))])
        sim.close()
    worst = {"u": 0.0, "theta": 0.0, "rho": 0.0}
    for k, c in enumerate(cases):
        err = _split_errors(out[0][k], out[1][k], c.eps)
        for key in worst:
            worst[key] = max(worst[key], err[key])
    _say(f"  worst relative L2 over 256 instances: {worst}")
    assert max(worst.values()) <= TOL_L2, worst


def test_shear_layer_8192_split_stated_steps():
    import torch

    from paper_2512_19847_amd import apdvm
    case = wl.shear_layer_8192()
    nsteps = 200
    _say(f"case shear8192 FP32-split against float64, {nsteps} steps dt={case.dt}")
    out = []
    for prec in (apdvm.FP32_SPLIT, apdvm.FP64):
        sim = apdvm.Simulation([dict(nx=case.nx, ny=case.ny, eps=case.eps, tau=case.tau,
                                     dt=case.dt)], tableau="ars443", precision=prec,
                               stream=torch.cuda.Stream())
        sim.set_fields(0, *case.state)
        sim.set_graph(True)
        sim.autotune(1)
        sim.step(nsteps)
        out.append(sim.get_fields(0))
        sim.close()
        _say(f"  precision {prec} done")
    err = _split_errors(out[0], out[1], case.eps)
    _say(f"  rel L2 {err}")
    assert max(err.values()) <= TOL_L2, err
