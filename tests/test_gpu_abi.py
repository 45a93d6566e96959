"""GPU checks of the C ABI beyond parity: launch modes, determinism, checkpoint and
resume, input handling, diagnostics and the profiling hooks."""

import numpy as np
import pytest

from oracle import d2q6
from oracle.operators import central_d
from paper_2512_19847_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _sim(n=64, eps=0.05, tau=0.3, dt=0.01, tab="ars443", count=1, stream=None, co=4, **kw):
    from paper_2512_19847_amd import apdvm
    return apdvm.Simulation([dict(nx=n, eps=eps, tau=tau, dt=dt, **kw)] * count, tableau=tab,
                            stream=stream, weno_order=5 if co == 4 else 3, central_order=co)


def _state(n=64, seed=5):
    return wl.random_divfree(n, kmax=4, rms=0.1, seed=seed)


def test_graph_replay_matches_direct_launches_bitwise():
    import torch

    st = _state()
    outs = []
    for graph in (False, True):
        s = torch.cuda.Stream()
        sim = _sim(stream=s)
        sim.set_graph(graph)
        sim.set_fields(0, *st)
        for _ in range(3):  # several replays with host work in between
            sim.step(2)
            sim.get_fields(0)
        outs.append(sim.get_fields(0))
        sim.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("graph", [False, True])
def test_solve_beside_updates_matches_one_stream_bitwise(graph):
    """The Helmholtz solve on the second stream beside the theta-free updates gives the
    same bits as every launch on one stream (two instances of different sizes, a
    ragged tile width, direct launches and graph replay)."""
    import torch

    from paper_2512_19847_amd import apdvm

    outs = []
    for on in (0, 1):
        sim = apdvm.Simulation([dict(nx=96, ny=64, eps=0.05, tau=0.3, dt=0.01),
                                dict(nx=64, ny=72, eps=1.0, tau=0.3, dt=0.01)],
                               tableau="ars443", stream=torch.cuda.Stream())
        sim.set_overlap(on)
        assert sim.overlap() == bool(on)
        sim.set_graph(graph)
        sim.set_fields(0, *wl.random_divfree(96, 64, kmax=4, rms=0.1, seed=3))
        sim.set_fields(1, *wl.random_divfree(64, 72, kmax=4, rms=0.1, seed=4))
        for _ in range(3):
            sim.step(2)
            sim.get_fields(0)
        outs.append([sim.get_fields(k) for k in range(2)])
        sim.close()
    for fa, fb in zip(*outs):
        for a, b in zip(fa, fb):
            assert np.array_equal(a, b)


def test_sampled_timing_between_graph_replays():
    """With graphs on, the steps whose launches are timed run launch by launch and the
    others replay the graph: the events count only the sampled steps and the result is
    bitwise the untimed run."""
    import torch

    from paper_2512_19847_amd import apdvm

    st = _state()
    cls = apdvm.KERNEL_CLASSES.index("stage_terms_relax_v")
    outs = []
    for timed in (False, True):
        sim = _sim(stream=torch.cuda.Stream())
        sim.set_graph(True)
        sim.set_fields(0, *st)
        if timed:
            sim.timing_enable(cls)
            sim.timing_stride(3)
        sim.step(6)
        if timed:
            n, ms = sim.timing_read()
            assert n == 2 * sim.traffic(cls)[1] and ms > 0.0
            sim.timing_enable(-1)
        outs.append(sim.get_fields(0))
        sim.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_runs_are_deterministic():
    st = _state()
    outs = []
    for _ in range(2):
        sim = _sim()
        sim.set_fields(0, *st)
        sim.step(5)
        outs.append(sim.get_fields(0))
        sim.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_checkpoint_resume_is_bitwise():
    st = _state()
    sim = _sim()
    sim.set_fields(0, *st)
    sim.step(6)
    full = sim.get_fields(0)
    sim.close()
    sim = _sim()
    sim.set_fields(0, *st)
    sim.step(3)
    ck = sim.get_fields(0)
    _, _, step = sim.info(0)
    sim.close()
    sim = _sim()
    sim.set_fields(0, *ck)
    sim.set_step(step)
    sim.step(3)
    res = sim.get_fields(0)
    assert sim.info(0)[2] == 6
    sim.close()
    for a, b in zip(full, res):
        assert np.array_equal(a, b)


def test_null_kinetic_fields_mean_local_equilibrium():
    st = _state()
    sim = _sim()
    sim.set_fields(0, st[0], st[1], st[2])
    got = sim.get_fields(0)
    F1, F2 = d2q6.flux_F(st[0], st[1])
    assert np.array_equal(got[3], F1) and np.array_equal(got[4], F2)
    assert np.all(got[5] == 0.0)
    sim.close()


def test_population_roundtrip_and_moments():
    n, eps = 32, 0.2
    st = _state(n)
    F = d2q6.populations_from_scaled(*st, eps)  # oracle-side map, independent of the library
    sim = _sim(n=n, eps=eps)
    sim.set_populations(0, F)
    got = sim.get_fields(0)
    for k, (a, b) in enumerate(zip(got, st)):
        assert np.max(np.abs(a - b)) < 1e-12 / eps ** 3, k
    F2 = sim.get_populations(0)
    assert np.max(np.abs(F2 - F)) < 1e-15
    rho, u1, u2, p = sim.get_moments(0)
    assert np.allclose(rho, 1 + 2 * eps * eps * got[2], rtol=0, atol=1e-15)
    assert np.allclose(p, got[2] - 0.5 * (got[0] ** 2 + got[1] ** 2), rtol=0, atol=1e-15)
    sim.close()


def test_errors_non_finite_and_order():
    from paper_2512_19847_amd import apdvm

    st = list(_state())
    sim = _sim()
    with pytest.raises(apdvm.ApdvmError) as e:
        sim.step(1)
    assert e.value.code == 7  # step before set_fields
    bad = st[2].copy()
    bad[3, 4] = np.nan
    with pytest.raises(apdvm.ApdvmError) as e:
        sim.set_fields(0, st[0], st[1], bad)
    assert e.value.code == 6
    with pytest.raises(apdvm.ApdvmError) as e:
        sim.step(1)  # the rejected call changed nothing
    assert e.value.code == 7
    sim.close()


@pytest.mark.parametrize("co", [4, 2])
def test_diagnostics_match_host_values(co):
    """Divergence and vorticity with the central differences of the context."""
    n = 64
    st = _state(n)
    sim = _sim(n=n, co=co)
    sim.set_fields(0, *st)
    sim.step(2)
    f = sim.get_fields(0)
    d = sim.diagnostics(0)
    h = 2 * np.pi / n
    div = central_d(f[0], 1, h, co) + central_d(f[1], 0, h, co)
    vor = central_d(f[1], 1, h, co) - central_d(f[0], 0, h, co)
    assert abs(d[0] - f[2].sum() * h * h) < 1e-12 * max(1.0, np.abs(f[2]).sum() * h * h)
    assert abs(d[1] - f[0].sum() * h * h) < 1e-12
    assert abs(d[2] - f[1].sum() * h * h) < 1e-12
    assert abs(d[3] - np.max(np.abs(div))) < 1e-12
    assert abs(d[4] - vor.min()) < 1e-12 and abs(d[5] - vor.max()) < 1e-12
    assert abs(d[6] - 0.5 * np.sum(f[0] ** 2 + f[1] ** 2) * h * h) < 1e-12
    assert d[7] == 1.0
    sim.close()


def test_timing_hooks_and_traffic():
    import torch

    from paper_2512_19847_amd import apdvm

    sim = _sim(stream=torch.cuda.Stream())
    sim.set_fields(0, *_state())
    per = {}
    total = 0.0
    for cls in range(len(apdvm.KERNEL_CLASSES)):
        b, nl = sim.traffic(cls)
        total += b
        assert nl > 0
        sim.timing_enable(cls)
        sim.step(2)
        n, ms = sim.timing_read()
        assert n == 2 * nl and ms > 0.0
        per[cls] = ms
    # sampling: with stride 2 only the launches of every second step are bracketed
    cls2 = max(per, key=per.get)
    sim.timing_enable(cls2)
    sim.timing_stride(2)
    sim.step(4)
    n2, _ = sim.timing_read()
    assert n2 == 2 * sim.traffic(cls2)[1]
    sim.timing_stride(1)
    sim.timing_enable(-1)
    b_all, n_all = sim.traffic(-1)
    assert abs(b_all - total) < 1e-6 * b_all and n_all == sim.launches_per_step() == 7 * 4
    sim.close()


def test_autotune_restores_state():
    """After autotuning, stepping gives bitwise the run of a fresh context forced to the
    same launch shapes and stream structure (the tuner restored state, step counter and
    parity)."""
    import torch

    st = _state()
    sim = _sim(stream=torch.cuda.Stream())
    sim.set_fields(0, *st)
    choice = sim.autotune(2)
    structure = sim.overlap()
    assert sim.info(0)[2] == 0
    sim.step(3)
    a = sim.get_fields(0)
    sim.close()
    sim = _sim()
    sim.set_tuning(choice)
    sim.set_overlap(structure)
    sim.set_fields(0, *st)
    sim.step(3)
    b = sim.get_fields(0)
    sim.close()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_autotune_cache_round_trip(tmp_path, monkeypatch):
    """APDVM_TUNE_CACHE: the first autotune appends one line keyed by the context's shape;
    a second context of the same shape reads its choice back (no trials, the file keeps
    one line) and steps bitwise like the first."""
    import torch

    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("APDVM_TUNE_CACHE", str(cache))
    st = _state()
    runs = []
    for _ in range(2):
        sim = _sim(stream=torch.cuda.Stream())
        sim.set_graph(True)
        sim.set_fields(0, *st)
        choice = sim.autotune(1)
        overlap = sim.overlap()
        sim.step(3)
        runs.append((choice, overlap, sim.get_fields(0)))
        sim.close()
        lines = cache.read_text().splitlines()
        assert len(lines) == 1 and "|" in lines[0], lines
    assert runs[0][0] == runs[1][0] and runs[0][1] == runs[1][1]
    for x, y in zip(runs[0][2], runs[1][2]):
        assert np.array_equal(x, y)
