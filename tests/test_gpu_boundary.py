"""GPU checks of the boundary contract: device-array entry points on a stream other than
the caller's, their validation, the finite check inside apdvm_step (the last state that
passed is kept), and the batch names of the C ABI."""

import ctypes
import sys

import numpy as np
import pytest

from paper_2512_19847_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _sim(precision, stream=None, n=64, eps=0.05, tau=0.3, dt=0.01, count=1):
    from paper_2512_19847_amd import apdvm
    return apdvm.Simulation([dict(nx=n, eps=eps, tau=tau, dt=dt)] * count, tableau="ars443",
                            precision=precision, stream=stream)


@pytest.mark.parametrize("prec", ["fp64", "fp32split"])
def test_device_fields_round_trip_on_another_stream(prec):
    """Fields produced on the caller's stream, handed over on the library's own stream,
    stepped, and read back into tensors the caller's stream consumes: bitwise the run
    through the host entry points."""
    import torch

    from paper_2512_19847_amd import apdvm
    p = apdvm.FP64 if prec == "fp64" else apdvm.FP32_SPLIT
    _say(f"case device round trip {prec}")
    st = wl.random_divfree(64, kmax=4, rms=0.1, seed=21)
    ref_sim = _sim(p)
    ref_sim.set_fields(0, *st)
    ref_sim.step(3)
    ref = ref_sim.get_fields(0)
    ref_sim.close()

    side = torch.cuda.Stream()
    sim = _sim(p, stream=side)
    # produced by kernels queued on the caller's (current) stream
    dev = [torch.from_numpy(f).cuda() * 1.0 for f in st]
    sim.set_fields_device(0, dev)
    del dev
    sim.step(3)
    out = [torch.full((64, 64), -1.0, dtype=torch.float64, device="cuda") for _ in range(6)]
    sim.get_fields_device(0, out)
    got = [o.cpu().numpy() for o in out]
    sim.close()
    for k, (a, b) in enumerate(zip(got, ref)):
        assert np.array_equal(a, b), k


def test_device_fields_reject_non_finite_and_change_nothing():
    import torch

    from paper_2512_19847_amd import apdvm
    _say("case device fields with NaN")
    st = wl.random_divfree(64, kmax=4, rms=0.1, seed=22)
    sim = _sim(apdvm.FP64)
    sim.set_fields(0, *st)
    sim.step(2)
    before = sim.get_fields(0)
    bad = [torch.from_numpy(f).cuda() for f in wl.random_divfree(64, kmax=4, rms=0.1, seed=23)]
    bad[5][7, 9] = float("nan")
    with pytest.raises(apdvm.ApdvmError) as e:
        sim.set_fields_device(0, bad)
    assert e.value.code == 6
    bad[5][7, 9] = 0.0
    bad[2][1, 2] = float("inf")
    with pytest.raises(apdvm.ApdvmError) as e:
        sim.set_fields_device(0, bad)
    assert e.value.code == 6
    after = sim.get_fields(0)
    assert sim.info(0)[2] == 2
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    sim.close()


@pytest.mark.parametrize("graph,structure", [(False, 1), (True, 1), (True, 2)])
def test_step_returns_nonfinite_and_keeps_last_checked_state(graph, structure):
    """A run whose time step is far beyond the stability limit (dt = 0.1 on 32^2 at
    eps = 1: the values overflow after about twenty steps) with a check every 4 steps:
    the call returns APDVM_ERR_NONFINITE, the step counter is back at the last check that
    passed, the state is bitwise the state of an unchecked run at that step, and stepping
    goes on from there."""
    import torch

    from paper_2512_19847_amd import apdvm
    _say(f"case blow-up with finite check every 4 steps, graph={graph} structure={structure}")
    st = wl.random_divfree(32, kmax=4, rms=0.1, seed=21)
    kw = dict(n=32, eps=1.0, tau=0.3, dt=0.1)
    sim = _sim(apdvm.FP64, stream=torch.cuda.Stream(), **kw)
    sim.set_graph(graph)
    sim.set_overlap(structure)
    sim.set_finite_check(4)
    sim.set_fields(0, *st)
    with pytest.raises(apdvm.ApdvmError) as e:
        sim.step(60)
    assert e.value.code == 6
    s_ck = sim.info(0)[2]
    kept = sim.get_fields(0)
    assert s_ck % 4 == 0 and 8 <= s_ck < 60, s_ck
    assert all(np.all(np.isfinite(f)) for f in kept)
    assert sim.diagnostics(0)[7] == 1.0
    sim.step(1)  # goes on from the kept state (the next check is not in this call)
    cont = sim.get_fields(0)
    sim.close()

    plain = _sim(apdvm.FP64, **kw)
    plain.set_overlap(structure)
    plain.set_finite_check(0)
    plain.set_fields(0, *st)
    plain.step(s_ck)
    same = plain.get_fields(0)
    plain.step(1)
    nxt = plain.get_fields(0)
    plain.step(3)
    blown = plain.get_fields(0)
    plain.close()
    _say(f"  kept step {s_ck}; unchecked run finite 4 steps later: "
         f"{all(np.all(np.isfinite(f)) for f in blown)}")
    for a, b in zip(kept, same):
        assert np.array_equal(a, b)
    for a, b in zip(cont, nxt):  # may already hold NaN one step on
        assert np.array_equal(a, b, equal_nan=True)
    assert not all(np.all(np.isfinite(f)) for f in blown)


def test_finite_check_does_not_change_results():
    import torch

    from paper_2512_19847_amd import apdvm
    st = wl.random_divfree(64, kmax=4, rms=0.1, seed=24)
    outs = []
    for every in (0, 1, 3):
        sim = _sim(apdvm.FP32_SPLIT, stream=torch.cuda.Stream())
        sim.set_graph(True)
        sim.set_finite_check(every)
        sim.set_fields(0, *st)
        sim.step(7)
        outs.append(sim.get_fields(0))
        sim.close()
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_batch_entry_points_alias_the_context():
    """apdvm_batch_create / set_fields / step / get_fields / destroy, called through the C
    ABI with a library-allocated workspace on the default stream, give bitwise the
    results of the same instances in a Simulation."""
    from paper_2512_19847_amd import apdvm
    L = apdvm.lib()
    keep = []
    specs = [(96, 64, 0.05, 0.3), (64, 72, 1e-4, 0.05)]
    cfgs = [apdvm.make_config(nx, ny, eps=e, tau=t, dt=0.005, keep=keep) for nx, ny, e, t in specs]
    arr = (apdvm.Config * 2)(*cfgs)
    b = ctypes.c_void_p()
    assert L.apdvm_batch_create(2, arr, None, 0, None, ctypes.byref(b)) == 0
    states = [wl.random_divfree(nx, ny, kmax=4, rms=0.1, seed=30 + k)
              for k, (nx, ny, _, _) in enumerate(specs)]
    for k, s in enumerate(states):
        s = [np.ascontiguousarray(f) for f in s]
        assert L.apdvm_batch_set_fields(b, k, *[ctypes.c_void_p(f.ctypes.data) for f in s]) == 0
    assert L.apdvm_batch_step(b, 3) == 0
    got = []
    for k, (nx, ny, _, _) in enumerate(specs):
        out = [np.empty((ny, nx)) for _ in range(6)]
        assert L.apdvm_batch_get_fields(b, k, *[ctypes.c_void_p(o.ctypes.data) for o in out]) == 0
        got.append(out)
    L.apdvm_batch_destroy(b)
    sim = apdvm.Simulation([dict(nx=nx, ny=ny, eps=e, tau=t, dt=0.005) for nx, ny, e, t in specs],
                           tableau="ars443")
    for k, s in enumerate(states):
        sim.set_fields(k, *s)
    sim.step(3)
    for k in range(2):
        for a, c in zip(got[k], sim.get_fields(k)):
            assert np.array_equal(a, c)
    sim.close()
