"""C-ABI checks that need no GPU: the library loads, exports every declared entry
point, and rejects invalid configurations before touching the device."""

import ctypes

import numpy as np
import pytest

from paper_2512_19847_amd import apdvm


def test_library_exports_every_declared_symbol():
    L = apdvm.lib()
    names = apdvm.declared_symbols()
    assert len(names) >= 16
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    for code in range(8):
        assert apdvm.lib().apdvm_status_string(code)


def _ws(cfg):
    return apdvm.workspace_bytes([cfg])


def test_workspace_bytes_valid_configs():
    for tab in ("euler1", "paper2", "ars443"):
        for prec in (apdvm.FP64, apdvm.FP32_SPLIT):
            keep = []
            b = _ws(apdvm.make_config(64, eps=1.0, mach=0.1, tableau=tab, precision=prec, keep=keep))
            assert b > 6 * 64 * 64 * 4
    keep = []
    b64 = _ws(apdvm.make_config(512, eps=1e-2, mach=0.05, tableau="ars443", keep=keep))
    b32 = _ws(apdvm.make_config(512, eps=1e-2, mach=0.05, tableau="ars443",
                                precision=apdvm.FP32_SPLIT, keep=keep))
    assert b32 < b64


def _code(cfg):
    with pytest.raises(apdvm.ApdvmError) as e:
        _ws(cfg)
    return e.value.code


@pytest.mark.parametrize("nx,ny", [(7, 8), (10, 8), (8, 10), (6, 6), (16, 14), (9, 9),
                                   (16384, 8)])
def test_rejects_bad_grids(nx, ny):
    keep = []
    assert _code(apdvm.make_config(nx, ny, keep=keep)) == 1


def test_accepts_mixed_radix_grids():
    keep = []
    for nx, ny in ((96, 72), (8, 8), (24, 18), (8192, 8)):
        assert _ws(apdvm.make_config(nx, ny, keep=keep)) > 0


def test_rejects_bad_velocity_set():
    keep = []
    cfg = apdvm.make_config(16, keep=keep)
    cfg.q = 9
    assert _code(cfg) == 2
    cfg = apdvm.make_config(16, keep=keep)
    ang = np.pi * np.arange(6) / 3
    cx, cy = np.cos(ang), np.sin(ang)
    cy[2] += 1e-6
    keep += [cx, cy]
    cfg.cx = cx.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    cfg.cy = cy.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert _code(cfg) == 2
    cy[2] -= 1e-6
    assert _ws(cfg) > 0


def _with_tableau(At, bt, A, b, keep):
    cfg = apdvm.make_config(16, keep=keep)
    arrs = [np.ascontiguousarray(np.array(x, dtype=np.float64)) for x in (At, bt, A, b)]
    keep.extend(arrs)
    P = ctypes.POINTER(ctypes.c_double)
    cfg.s = arrs[0].shape[0]
    cfg.a_ex, cfg.b_ex, cfg.a_im, cfg.b_im = (a.ctypes.data_as(P) for a in arrs)
    return cfg


def test_rejects_bad_tableaux():
    keep = []
    At, bt, A, b = (x.copy() for x in apdvm.TABLEAUX["paper2"])
    # not globally stiffly accurate
    b2 = b.copy()
    b2[1] += 0.1
    assert _code(_with_tableau(At, bt, A, b2, keep)) == 3
    # type A (every stage implicit) is accepted; a first implicit stage followed by a
    # zero diagonal entry is neither type A nor ARS
    A2 = A.copy()
    A2[0, 0] = 0.5
    assert _ws(_with_tableau(At, bt, A2, b, keep)) > 0
    A4 = A2.copy()
    A4[1, 1] = 0.0
    assert _code(_with_tableau(At, bt, A4, b, keep)) == 3
    # explicit part not strictly lower triangular
    At2 = At.copy()
    At2[1, 1] = 0.2
    assert _code(_with_tableau(At2, bt, A, b, keep)) == 3
    # CK but not ARS (nonzero first column)
    A3 = A.copy()
    A3[1, 0] = 0.1
    assert _code(_with_tableau(At, bt, A3, b, keep)) == 3


def test_rejects_bad_physics():
    keep = []
    assert _code(apdvm.make_config(16, eps=-1.0, keep=keep)) == 1
    assert _code(apdvm.make_config(16, eps=0.1, mach=0.0, tau=-1.0, keep=keep)) == 1
    assert _code(apdvm.make_config(16, eps=0.1, tau=float("nan"), keep=keep)) == 1
    assert _code(apdvm.make_config(16, eps=0.1, dt=0.0, cfl=0.0, keep=keep)) == 1
    cfg = apdvm.make_config(16, keep=keep)
    cfg.precision = 7
    assert _code(cfg) == 1


def test_space_discretisation_orders():
    keep = []
    for wo, co in ((5, 4), (3, 2), (3, 4), (5, 2), (0, 0)):
        assert _ws(apdvm.make_config(16, keep=keep, weno_order=wo, central_order=co)) > 0
    assert _code(apdvm.make_config(16, keep=keep, weno_order=4)) == 1
    assert _code(apdvm.make_config(16, keep=keep, central_order=6)) == 1
    # every instance of a context must use the same operators
    a = apdvm.make_config(16, keep=keep, weno_order=3, central_order=2)
    b = apdvm.make_config(16, keep=keep)
    arr = (apdvm.Config * 2)(a, b)
    out = ctypes.c_size_t(0)
    assert apdvm.lib().apdvm_workspace_bytes(2, arr, ctypes.byref(out)) == 1
    c = apdvm.make_config(16, keep=keep, weno_order=0, central_order=0)
    arr = (apdvm.Config * 2)(b, c)
    assert apdvm.lib().apdvm_workspace_bytes(2, arr, ctypes.byref(out)) == 0


def test_binding_tableaux_match_golden():
    import json
    import os

    from oracle import tableau as otab

    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tableaux.json")))
    for name, (At, bt, A, b) in apdvm.TABLEAUX.items():
        # the paper's tableaux against the printed coefficients, the constructed type-A
        # ones against the oracle's exact fractions
        g = gold[name] if name in gold else dict(zip(("At", "bt", "A", "b"),
                                                     otab.preset_fractions(name)))
        for got, key in ((At, "At"), (bt, "bt"), (A, "A"), (b, "b")):
            want = np.array([[float(x) for x in r] for r in g[key]] if np.ndim(g[key]) == 2
                            else [float(x) for x in g[key]], dtype=float)
            assert np.allclose(got, want, atol=1e-15, rtol=0), (name, key)
