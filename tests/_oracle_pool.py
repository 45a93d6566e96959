"""Oracle runs for the long GPU parity tests, in worker processes (CPU only; started
with the spawn method, so they never touch the GPU).  Each job regenerates its inputs
from the seeded recipes instead of receiving large arrays."""

import numpy as np

from oracle import scheme, tableau as otab
from oracle.operators import Production
from paper_2512_19847_amd import workloads as wl


def _case(spec):
    kind = spec["kind"]
    if kind == "shear512":
        return wl.shear_layer_512(spec["eps"])
    if kind == "batched256":
        return wl.batched_256_instance(spec["index"])
    raise ValueError(kind)


def run(spec):
    """spec: kind, parameters, nsteps, checkpoints (sorted step numbers), perturb (1-ulp
    relative perturbation seed or None).  Returns the states at the checkpoints."""
    c = _case(spec)
    st = c.state
    if spec.get("perturb") is not None:
        rng = np.random.default_rng(spec["perturb"])
        st = tuple(x * (1 + 1e-16 * rng.standard_normal(x.shape)) for x in st)
    p = scheme.Params(c.eps, c.tau, c.dt)
    tab = otab.preset(c.tableau)
    ops = Production(c.lx / c.nx, c.ly / c.ny)
    out = {}
    done = 0
    for ck in spec["checkpoints"]:
        st = scheme.run(st, p, tab, ops, ck - done)
        done = ck
        out[ck] = tuple(np.array(x) for x in st)
    return out


def pool_map(specs, workers):
    import multiprocessing as mp

    with mp.get_context("spawn").Pool(min(workers, len(specs))) as pool:
        return pool.map(run, specs)
