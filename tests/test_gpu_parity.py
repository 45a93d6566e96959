"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by
element on the same seeded inputs.  Bar: relative L-infinity <= 1e-11 per field
(max |gpu - oracle| / max |oracle|)."""

import math
import sys

import numpy as np
import pytest

from oracle import scheme, tableau as otab
from oracle.operators import Production
from paper_2512_19847_amd import workloads as wl

pytestmark = pytest.mark.gpu

FIELDS = ("u1", "u2", "theta", "v1", "v2", "q")
TOL = 1e-11


def _apdvm():
    from paper_2512_19847_amd import apdvm
    return apdvm


def _oracle(state, eps, tau, dt, tab, nsteps, lx=2 * np.pi, ly=2 * np.pi, wo=5, co=4):
    ny, nx = state[0].shape
    return scheme.run(state, scheme.Params(eps, tau, dt), otab.preset(tab),
                      Production(lx / nx, ly / ny, central_order=co, weno_order=wo), nsteps)


def _relerr(got, ref, kinetic_floor=False):
    """kinetic_floor: compare v1, v2 and q at least against max |u|^2, the size of F(u)
    and of the stage terms they are computed from (for cases where they end as a
    cancellation of such terms); each such plane's error against its own maximum is
    printed beside it."""
    out = {}
    own = {}
    scale = max(np.max(np.abs(r)) for r in ref)
    usq = float(np.max(ref[0] ** 2 + ref[1] ** 2))
    for name, g, r in zip(FIELDS, got, ref):
        # fields that vanish identically are compared against the largest field
        m = np.max(np.abs(r))
        den = m if m > 1e-12 * scale else scale
        if kinetic_floor and name in ("v1", "v2", "q"):
            own[name] = float(np.max(np.abs(g - r)) / den)
            den = max(den, usq)
        out[name] = float(np.max(np.abs(g - r)) / den)
    if own:
        _say(f"    planes against their own maximum: {own}")
    return out


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _stream():
    import torch
    return torch.cuda.Stream()


def _run_gpu(cases, tab, nsteps, precision=0, shape=None, wo=5, co=4, structure=None,
             graph=False):
    apdvm = _apdvm()
    sim = apdvm.Simulation([dict(nx=c["state"][0].shape[1], ny=c["state"][0].shape[0],
                                 eps=c["eps"], tau=c["tau"], dt=c["dt"],
                                 lx=c.get("lx", 2 * np.pi), ly=c.get("ly", 2 * np.pi))
                            for c in cases], tableau=tab, precision=precision,
                           weno_order=wo, central_order=co,
                           stream=_stream() if graph else None)
    if shape is not None:
        sim.set_tuning(*shape)
    if structure is not None:
        sim.set_overlap(structure)
    sim.set_graph(graph)
    for k, c in enumerate(cases):
        sim.set_fields(k, *c["state"])
    sim.step(nsteps)
    out = [sim.get_fields(k) for k in range(len(cases))]
    sim.close()
    return out


@pytest.mark.parametrize("tab,nsteps", [("paper2", 100), ("ars443", 100), ("euler1", 100)])
def test_taylor_green_64(tab, nsteps):
    """64^2 Taylor-Green, eps = 1, Ma = 0.1 (tau = 40): the small plain-method case."""
    case = wl.taylor_green_64(tab)
    _say(f"case taylor_green_64 {tab} steps={nsteps} dt={case.dt}")
    c = dict(state=case.state, eps=case.eps, tau=case.tau, dt=case.dt)
    got = _run_gpu([c], tab, nsteps)[0]
    ref = _oracle(case.state, case.eps, case.tau, case.dt, tab, nsteps)
    err = _relerr(got, ref)
    _say(f"  relerr {err}")
    assert max(err.values()) <= TOL, err


@pytest.mark.parametrize("eps,tau", [(0.05, 0.3), (1e-6, 0.05), (0.0, 0.05), (0.3, 0.0),
                                     (0.0, 0.0)])
def test_ragged_nonsquare(eps, tau):
    """96 x 72 cells (ragged tiles in x and y, radix-3 FFT factors), Ly = 1.5 Lx."""
    nx, ny = 96, 72
    st = wl.random_divfree(nx, ny, kmax=4, rms=0.1, seed=11)
    # the generator builds a square-periodic box; stretch y to ly = 3 pi
    lx, ly = 2 * np.pi, 3 * np.pi
    dt = 0.01
    _say(f"case ragged {nx}x{ny} eps={eps} tau={tau}")
    c = dict(state=st, eps=eps, tau=tau, dt=dt, lx=lx, ly=ly)
    got = _run_gpu([c], "ars443", 4)[0]
    ref = _oracle(st, eps, tau, dt, "ars443", 4, lx, ly)
    err = _relerr(got, ref)
    _say(f"  relerr {err}")
    assert max(err.values()) <= TOL, err


@pytest.mark.parametrize("shape", [(8, 256), (16, 256), (16, 512), (8, 512)])
def test_every_launch_shape_matches_oracle(shape):
    """The shapes the autotuner can pick: 64 x 8 or 64 x 16 tiles on 256 or 512 threads;
    ragged non-square grid, two instances."""
    cases = [dict(state=wl.random_divfree(96, 72, kmax=4, rms=0.1, seed=31), eps=0.05, tau=0.3,
                  dt=0.01),
             dict(state=wl.random_divfree(48, 36, kmax=4, rms=0.1, seed=32), eps=1e-5, tau=0.05,
                  dt=0.02)]
    _say(f"case launch shape {shape}")
    got = _run_gpu(cases, "ars443", 4, shape=shape)
    for k, c in enumerate(cases):
        ref = _oracle(c["state"], c["eps"], c["tau"], c["dt"], "ars443", 4)
        err = _relerr(got[k], ref)
        _say(f"  instance {k} relerr {err}")
        assert max(err.values()) <= TOL, (k, err)


@pytest.mark.parametrize("n", [8, 16, 24])
def test_tiny_grids(n):
    """Grids smaller than one tile: the periodic halo wraps several times."""
    st = wl.taylor_green(n)
    _say(f"case tiny {n}")
    c = dict(state=st, eps=0.2, tau=0.5, dt=0.02)
    got = _run_gpu([c], "paper2", 3)[0]
    ref = _oracle(st, 0.2, 0.5, 0.02, "paper2", 3)
    err = _relerr(got, ref)
    _say(f"  relerr {err}")
    assert max(err.values()) <= TOL, err


def test_shear_layer_small_eps():
    n = 64
    case = wl.make_case("sl64", wl.shear_layer(n), 1e-6, 0.05, "ars443", cfl=wl.CFL_ARS)
    _say(f"case shear64 eps=1e-6 dt={case.dt}")
    c = dict(state=case.state, eps=case.eps, tau=case.tau, dt=case.dt)
    got = _run_gpu([c], "ars443", 20)[0]
    ref = _oracle(case.state, case.eps, case.tau, case.dt, "ars443", 20)
    err = _relerr(got, ref)
    _say(f"  relerr {err}")
    assert max(err.values()) <= TOL, err


def test_twin_floor_where_roundoff_grows():
    """64^2 shear layer at eps = 1e-6 and CFL 0.4, where this flow amplifies round-off
    by about 2 per step: the GPU must stay within a small factor of the oracle's own
    sensitivity (oracle against itself from inputs perturbed by 1e-16 relative)."""
    n, nsteps = 64, 15
    case = wl.make_case("sl64", wl.shear_layer(n), 1e-6, 0.05, "ars443", cfl=0.4)
    c = dict(state=case.state, eps=case.eps, tau=case.tau, dt=case.dt)
    _say(f"case twin shear64 dt={case.dt}")
    got = _run_gpu([c], "ars443", nsteps)[0]
    ref = _oracle(case.state, case.eps, case.tau, case.dt, "ars443", nsteps)
    rng = np.random.default_rng(0)
    pert = tuple(x * (1 + 1e-16 * rng.standard_normal(x.shape)) for x in case.state)
    twin = _oracle(pert, case.eps, case.tau, case.dt, "ars443", nsteps)
    e_gpu, e_twin = _relerr(got, ref), _relerr(twin, ref)
    _say(f"  gpu {e_gpu}\n  twin {e_twin}")
    for f in FIELDS:
        assert e_gpu[f] <= 30 * e_twin[f] + TOL, (f, e_gpu[f], e_twin[f])


def test_batched_heterogeneous_instances():
    """One context, instances of different sizes and parameters, one launch per phase."""
    specs = [(64, 1e-3, 0.04, 0.01), (96, 0.5, 0.2, 0.01), (48, 1e-6, 0.0, 0.02),
             (128, 0.05, 1.0, 0.005)]
    cases = []
    for k, (n, eps, tau, dt) in enumerate(specs):
        cases.append(dict(state=wl.random_divfree(n, kmax=4, rms=0.1, seed=100 + k),
                          eps=eps, tau=tau, dt=dt))
    _say("case batched 4 instances")
    got = _run_gpu(cases, "ars443", 3)
    for k, c in enumerate(cases):
        ref = _oracle(c["state"], c["eps"], c["tau"], c["dt"], "ars443", 3)
        err = _relerr(got[k], ref)
        _say(f"  instance {k} relerr {err}")
        assert max(err.values()) <= TOL, (k, err)


@pytest.mark.parametrize("sides", [((2048, 16), (16, 2048)), ((8192, 8), (8, 8192)),
                                   ((3072, 8), (12, 4096), (6144, 8)),
                                   ((4374, 8), (8, 8)), ((2048, 16), (2048, 8)),
                                   ((512, 16), (64, 32))])
def test_extreme_aspect_ratios_every_fft_form(sides):
    """Long thin instances in one context: rows and columns of up to 2048 (8192) values
    take the 2048-value (8192-value) FFT forms, while the short sides put many rows
    (columns) into one workgroup; two steps against the oracle.  Rows longer than 2048
    are inverted in the split form when every nx is a multiple of 4 (radix-3 halves of 1536
    and 6, and 682 row pairs of 12 values in one workgroup, in the third case) and in the
    whole-row form otherwise (nx = 4374 = 2 * 3^7 in the fourth); in the fifth every row of
    both instances fills the 2048-value form, so the row kernels run their register forms
    over two instances in one launch; in the sixth the rows of 512 and of 64 values fill
    the 1024-value form's workgroups two and sixteen at a time (the register form of several
    lines, with each instance's own line length).  q is ~1e-4 here, a
    cancellation of O(|u|^2) terms whose rounding the 1/h = 1300 of the long side
    amplifies, so v and q are held against max |u|^2 (kinetic floor)."""
    cases = []
    for k, (nx, ny) in enumerate(sides):
        c = wl.make_case(f"thin{k}", wl.random_divfree(nx, ny, kmax=3, rms=0.1, seed=50 + k),
                         0.05, 0.05, "ars443", cfl=wl.CFL_ARS)
        cases.append(dict(state=c.state, eps=c.eps, tau=c.tau, dt=c.dt))
    _say(f"case aspect ratios {sides}")
    got = _run_gpu(cases, "ars443", 2)
    for k, c in enumerate(cases):
        ref = _oracle(c["state"], c["eps"], c["tau"], c["dt"], "ars443", 2)
        err = _relerr(got[k], ref, kinetic_floor=True)
        _say(f"  instance {k} {sides[k]} relerr {err}")
        assert max(err.values()) <= TOL, (k, err)


@pytest.mark.parametrize("side", [(8192, 8), (8, 8192), (2048, 16), (16, 2048), (1024, 8),
                                  (8, 1024)])
def test_lines_filling_their_fft_form(side):
    """One long thin instance per context, so that every row (column) fills its FFT form
    (1024, 2048 or 8192 values, the 8192-value rows inverted and columns transformed in the
    split halves): the FFT kernels run their register forms, which take the first pass from
    the loaded values and keep the last in registers.  Two steps against the oracle, v and
    q held against max |u|^2 as for the other thin instances."""
    nx, ny = side
    c = wl.make_case("full", wl.random_divfree(nx, ny, kmax=3, rms=0.1, seed=70),
                     0.05, 0.05, "ars443", cfl=wl.CFL_ARS)
    _say(f"case lines filling their form {side}")
    got = _run_gpu([dict(state=c.state, eps=c.eps, tau=c.tau, dt=c.dt)], "ars443", 2)[0]
    ref = _oracle(c.state, c.eps, c.tau, c.dt, "ars443", 2)
    err = _relerr(got, ref, kinetic_floor=True)
    _say(f"  relerr {err}")
    assert max(err.values()) <= TOL, err


@pytest.mark.parametrize("eps", [1.0, 1e-2, 1e-6])
def test_shear_layer_512_one_step(eps):
    """Full 512^2 size of the third-order shear-layer runs, one step, every cell."""
    case = wl.shear_layer_512(eps)
    _say(f"case shear512 eps={eps} dt={case.dt}")
    c = dict(state=case.state, eps=case.eps, tau=case.tau, dt=case.dt)
    got = _run_gpu([c], "ars443", 1)[0]
    ref = _oracle(case.state, case.eps, case.tau, case.dt, "ars443", 1)
    err = _relerr(got, ref)
    _say(f"  relerr {err}")
    assert max(err.values()) <= TOL, err


@pytest.mark.parametrize("wo,co,tab,shape", [(3, 2, "euler1", (8, 256)),
                                             (3, 2, "paper2", (16, 256)),
                                             (3, 4, "paper2", (8, 512)),
                                             (5, 2, "ars443", (16, 512))])
def test_space_orders_match_oracle(wo, co, tab, shape):
    """WENO3 and second-order central differences (the convergence-table operators) and
    the mixed combinations, on two ragged non-square instances from kinetic to small eps."""
    cases = [dict(state=wl.random_divfree(96, 72, kmax=4, rms=0.1, seed=41), eps=0.05, tau=0.3,
                  dt=0.005, ly=3 * np.pi),
             dict(state=wl.random_divfree(48, 36, kmax=4, rms=0.1, seed=42), eps=1e-6, tau=0.05,
                  dt=0.01)]
    _say(f"case space orders weno={wo} central={co} {tab} shape={shape}")
    got = _run_gpu(cases, tab, 6, shape=shape, wo=wo, co=co)
    for k, c in enumerate(cases):
        ref = _oracle(c["state"], c["eps"], c["tau"], c["dt"], tab, 6, ly=c.get("ly", 2 * np.pi),
                      wo=wo, co=co)
        err = _relerr(got[k], ref)
        _say(f"  instance {k} relerr {err}")
        assert max(err.values()) <= TOL, (k, err)


@pytest.mark.parametrize("tab", ["euler1", "paper2"])
def test_shear_layer_convergence_table_setting(tab):
    """The setting of the convergence tables (Section 4.1): 64^2 thick shear layer,
    eps = 1e-6, tau = 0, WENO3 + second-order central, dt = 1 / (2N)."""
    n = 64
    st = wl.shear_layer(n)
    dt, nsteps = 1.0 / (2 * n), 16
    _say(f"case table setting shear64 {tab}")
    c = dict(state=st, eps=1e-6, tau=0.0, dt=dt)
    got = _run_gpu([c], tab, nsteps, wo=3, co=2)[0]
    ref = _oracle(st, 1e-6, 0.0, dt, tab, nsteps, wo=3, co=2)
    err = _relerr(got, ref)
    _say(f"  relerr {err}")
    assert max(err.values()) <= TOL, err


@pytest.mark.parametrize("kind,tau", [("thin_shear_layer", 0.0), ("kelvin_helmholtz", 0.05)])
def test_long_run_flows_match_oracle(kind, tau):
    """The flows of the long runs (thin shear layer; Kelvin-Helmholtz on [0, 4 pi]^2),
    eps = 1e-6, 64^2, ten steps of the production time step."""
    case = wl.flow_case(kind, 64, tau)
    _say(f"case {kind} tau={tau} dt={case.dt}")
    c = dict(state=case.state, eps=case.eps, tau=case.tau, dt=case.dt, lx=case.lx, ly=case.ly)
    got = _run_gpu([c], "ars443", 10)[0]
    ref = _oracle(case.state, case.eps, case.tau, case.dt, "ars443", 10, case.lx, case.ly)
    err = _relerr(got, ref)
    _say(f"  relerr {err}")
    assert max(err.values()) <= TOL, err


@pytest.mark.parametrize("tab", ["typea1", "typea2"])
def test_type_a_tableaux_match_oracle(tab):
    """Type-A tableaux (every stage implicit; run on the device behind a zero first
    stage) against the oracle, which solves their first stage directly.  At eps = 1e-6
    the first stage has no explicit terms, so v relaxes to about te2 v^n / kappa there,
    and typea2's last stage cancels its explicit history down to about -2 v(1): its v
    and q end near 1e-12 while the stage terms are of the size of F(u); they are compared
    against max |u|^2."""
    cases = [dict(state=wl.random_divfree(96, 72, kmax=4, rms=0.1, seed=51), eps=0.05, tau=0.3,
                  dt=0.005, ly=3 * np.pi),
             dict(state=wl.random_divfree(48, 36, kmax=4, rms=0.1, seed=52), eps=1e-6, tau=0.05,
                  dt=0.01)]
    _say(f"case type A {tab}")
    got = _run_gpu(cases, tab, 6)
    for k, c in enumerate(cases):
        ref = _oracle(c["state"], c["eps"], c["tau"], c["dt"], tab, 6, ly=c.get("ly", 2 * np.pi))
        err = _relerr(got[k], ref, kinetic_floor=True)
        _say(f"  instance {k} relerr {err}")
        assert max(err.values()) <= TOL, (k, err)


@pytest.mark.parametrize("tab", ["ars443", "typea2"])
def test_ill_prepared_data(tab):
    """Velocity with a gradient part (max |D0.u| about 0.3) at eps = 1e-6: the device
    matches the oracle over three steps, and the first step removes the divergence down
    to the level the printed operators leave (their D_Delta is not D0.D0), for the ARS
    tableau as well as the type-A one."""
    from oracle.operators import central_d
    n = 64
    st = wl.ill_prepared(n, seed=61)
    h = 2 * np.pi / n
    div = lambda f: np.max(np.abs(central_d(f[0], 1, h) + central_d(f[1], 0, h)))
    c = dict(state=st, eps=1e-6, tau=0.05, dt=0.01)
    _say(f"case ill-prepared {tab}: initial max|div u| {div(st):.3e}")
    got1 = _run_gpu([c], tab, 1)[0]
    got = _run_gpu([c], tab, 3)[0]
    ref = _oracle(st, 1e-6, 0.05, 0.01, tab, 3)
    err = _relerr(got, ref, kinetic_floor=True)  # see test_type_a_tableaux_match_oracle
    _say(f"  after one step max|div u| {div(got1):.3e}; relerr after three {err}")
    assert max(err.values()) <= TOL, err
    assert div(got1) < 1e-2 * div(st)


@pytest.mark.parametrize("tab,wo,co", [("ars443", 5, 4), ("paper2", 5, 4), ("euler1", 3, 2),
                                       ("typea2", 5, 4), ("ars443", 3, 4)])
@pytest.mark.parametrize("graph", [False, True])
def test_fused_schedule_matches_oracle(tab, wo, co, graph):
    """Stream structure 2: the update launch completes u, Hu and L theta from theta after
    the solve (one stream).  Ragged 96 x 72 and 64 x 48 instances in one context, kinetic
    and stiff, every stage kind of the tableau (stored Hu and L theta, the last stage),
    launched directly and replayed as graphs."""
    cases = []
    for k, (nx, ny, eps, tau) in enumerate([(96, 72, 0.05, 0.3), (64, 48, 1e-6, 0.05)]):
        st = wl.random_divfree(nx, ny, kmax=4, rms=0.1, seed=70 + k)
        cases.append(dict(state=st, eps=eps, tau=tau, dt=0.01))
    _say(f"case fused schedule {tab} weno{wo} central{co} graph={graph}")
    got = _run_gpu(cases, tab, 5, wo=wo, co=co, structure=2, graph=graph)
    for k, c in enumerate(cases):
        ref = _oracle(c["state"], c["eps"], c["tau"], c["dt"], tab, 5, wo=wo, co=co)
        err = _relerr(got[k], ref, kinetic_floor=tab == "typea2")
        _say(f"  instance {k} relerr {err}")
        assert max(err.values()) <= TOL, (k, err)
