"""Python binding of the C ABI in include/apdvm.h (ctypes; argument marshalling only).

Every step of the method runs in the HIP library libapdvm.so; this module only
converts arguments.  PyTorch supplies device memory for the workspace and the stream.
Importing this module does not need a GPU; creating a Simulation does.  If the
library is not built, every entry point raises (there is no fallback path).

Tableau presets (Section 4.1 of the paper for the first- and second-order schemes;
ARS(4,4,3) of Ascher, Ruuth and Spiteri 1997 for third order, which the paper cites
but does not print):
  euler1  first-order GSA IMEX Euler
  paper2  second-order GSA IMEX RK with c = 9/4, gamma = (c - 1/2)/(c - 1) = 7/5
  ars443  third-order ARS(4,4,3)
"""

import ctypes
import os
import re
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapdvm.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "apdvm.h")

FP64, FP32_SPLIT = 0, 1
KERNEL_CLASSES = ("helmholtz_rhs", "fft_rows_forward", "fft_columns", "fft_rows_inverse",
                  "update_uq", "stage_terms_relax_v", "grad_q")
# Entries of the launch-shape choice array: one per kernel class, then the workgroup
# threads of the four stencil classes.
TUNED_STENCIL = ("helmholtz_rhs", "update_uq", "stage_terms_relax_v", "grad_q")
TUNING_KEYS = KERNEL_CLASSES + tuple("threads_" + k for k in TUNED_STENCIL)
STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_VELSET", 3: "ERR_TABLEAU", 4: "ERR_NOMEM",
          5: "ERR_HIP", 6: "ERR_NONFINITE", 7: "ERR_STATE"}


class ApdvmError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)} ({_status_string(code)})")


class Config(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("lx", c_double), ("ly", c_double),
                ("q", c_int32), ("cx", POINTER(c_double)), ("cy", POINTER(c_double)),
                ("eps", c_double), ("mach", c_double), ("tau", c_double),
                ("s", c_int32), ("a_ex", POINTER(c_double)), ("b_ex", POINTER(c_double)),
                ("a_im", POINTER(c_double)), ("b_im", POINTER(c_double)),
                ("dt", c_double), ("cfl", c_double), ("c_visc", c_double),
                ("precision", c_int32), ("weno_order", c_int32), ("central_order", c_int32)]


def _tableaux():
    c = 9.0 / 4.0
    g = (c - 0.5) / (c - 1.0)
    t = {
        "euler1": ([[0, 0], [1, 0]], [1, 0], [[0, 0], [0, 1]], [0, 1]),
        "paper2": ([[0, 0, 0], [c, 0, 0], [1 - 1 / (2 * c), 1 / (2 * c), 0]],
                   [1 - 1 / (2 * c), 1 / (2 * c), 0],
                   [[0, 0, 0], [0, c, 0], [0, 1 - g, g]], [0, 1 - g, g]),
        "ars443": ([[0, 0, 0, 0, 0], [1 / 2, 0, 0, 0, 0], [11 / 18, 1 / 18, 0, 0, 0],
                    [5 / 6, -5 / 6, 1 / 2, 0, 0], [1 / 4, 7 / 4, 3 / 4, -7 / 4, 0]],
                   [1 / 4, 7 / 4, 3 / 4, -7 / 4, 0],
                   [[0, 0, 0, 0, 0], [0, 1 / 2, 0, 0, 0], [0, 1 / 6, 1 / 2, 0, 0],
                    [0, -1 / 2, 1 / 2, 1 / 2, 0], [0, 3 / 2, -3 / 2, 1 / 2, 1 / 2]],
                   [0, 3 / 2, -3 / 2, 1 / 2, 1 / 2]),
        # type A (every stage implicit), first and second order
        "typea1": ([[0, 0], [1, 0]], [1, 0], [[1, 0], [0, 1]], [0, 1]),
        "typea2": ([[0, 0, 0, 0], [1, 0, 0, 0], [1 / 2, 1 / 2, 0, 0], [1 / 2, 1 / 2, 0, 0]],
                   [1 / 2, 1 / 2, 0, 0],
                   [[1 / 4, 0, 0, 0], [1 / 2, 1 / 4, 0, 0], [1 / 4, 0, 1 / 4, 0],
                    [1 / 2, 0, 1 / 4, 1 / 4]], [1 / 2, 0, 1 / 4, 1 / 4]),
    }
    return {k: tuple(np.array(x, dtype=np.float64) for x in v) for k, v in t.items()}


TABLEAUX = _tableaux()

_lib = None


def _declare(L):
    P = c_void_p
    L.apdvm_status_string.restype = ctypes.c_char_p
    L.apdvm_status_string.argtypes = [ctypes.c_int]
    L.apdvm_workspace_bytes.argtypes = [c_int32, POINTER(Config), POINTER(c_size_t)]
    L.apdvm_create.argtypes = [c_int32, POINTER(Config), P, c_size_t, P, POINTER(P)]
    L.apdvm_set_fields.argtypes = [P, c_int32] + [P] * 6
    L.apdvm_set_fields_device.argtypes = [P, c_int32, POINTER(P)]
    L.apdvm_set_populations.argtypes = [P, c_int32, P]
    L.apdvm_step.argtypes = [P, c_int64]
    L.apdvm_get_fields.argtypes = [P, c_int32] + [P] * 6
    L.apdvm_get_fields_device.argtypes = [P, c_int32, POINTER(P)]
    L.apdvm_get_moments.argtypes = [P, c_int32] + [P] * 4
    L.apdvm_get_populations.argtypes = [P, c_int32, P]
    L.apdvm_get_info.argtypes = [P, c_int32, POINTER(c_double), POINTER(c_double),
                                 POINTER(c_int64)]
    L.apdvm_set_step.argtypes = [P, c_int64]
    L.apdvm_diagnostics.argtypes = [P, c_int32, P]
    L.apdvm_launches_per_step.argtypes = [P, POINTER(c_int32)]
    L.apdvm_set_graph.argtypes = [P, c_int32]
    L.apdvm_set_overlap.argtypes = [P, c_int32]
    L.apdvm_get_overlap.argtypes = [P, POINTER(c_int32)]
    L.apdvm_timing_enable.argtypes = [P, c_int32]
    L.apdvm_timing_read.argtypes = [P, POINTER(c_int64), POINTER(c_double)]
    L.apdvm_timing_stride.argtypes = [P, c_int32]
    L.apdvm_traffic.argtypes = [P, c_int32, POINTER(c_double), POINTER(c_int32)]
    L.apdvm_autotune.argtypes = [P, c_int32, POINTER(c_int32)]
    L.apdvm_set_tuning.argtypes = [P, POINTER(c_int32)]
    L.apdvm_set_finite_check.argtypes = [P, c_int32]
    L.apdvm_diagnostics_device.argtypes = [P, c_int32, P]
    L.apdvm_batch_create.argtypes = [c_int32, POINTER(Config), P, c_size_t, P, POINTER(P)]
    L.apdvm_batch_set_fields.argtypes = [P, c_int32] + [P] * 6
    L.apdvm_batch_step.argtypes = [P, c_int64]
    L.apdvm_batch_get_fields.argtypes = [P, c_int32] + [P] * 6
    L.apdvm_batch_destroy.argtypes = [P]
    L.apdvm_batch_destroy.restype = None
    L.apdvm_destroy.argtypes = [P]
    L.apdvm_destroy.restype = None
    for name in ("apdvm_workspace_bytes", "apdvm_create", "apdvm_set_fields",
                 "apdvm_set_fields_device", "apdvm_set_populations", "apdvm_step",
                 "apdvm_get_fields", "apdvm_get_fields_device", "apdvm_get_moments",
                 "apdvm_get_populations", "apdvm_get_info", "apdvm_set_step",
                 "apdvm_diagnostics", "apdvm_launches_per_step", "apdvm_set_graph",
                 "apdvm_set_overlap", "apdvm_get_overlap",
                 "apdvm_timing_enable", "apdvm_timing_read", "apdvm_timing_stride", "apdvm_traffic",
                 "apdvm_autotune", "apdvm_set_tuning", "apdvm_set_finite_check",
                 "apdvm_diagnostics_device",
                 "apdvm_batch_create", "apdvm_batch_set_fields", "apdvm_batch_step",
                 "apdvm_batch_get_fields"):
        getattr(L, name).restype = ctypes.c_int


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2512_19847_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _status_string(code):
    try:
        return lib().apdvm_status_string(int(code)).decode()
    except Exception:  # pragma: no cover - only while reporting another failure
        return "?"


def _check(code, where):
    if code != 0:
        raise ApdvmError(code, where)


def declared_symbols():
    """Names of the entry points declared in include/apdvm.h."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"\b(apdvm_[a-z_]+)\s*\(", text)))


def _dptr(a):
    return a.ctypes.data_as(POINTER(c_double))


def make_config(nx, ny=None, eps=1.0, mach=0.1, tau=-1.0, tableau="ars443", dt=0.0,
                lx=2 * np.pi, ly=2 * np.pi, cfl=0.4, c_visc=0.2, precision=FP64, keep=None,
                weno_order=5, central_order=4):
    """A Config for one instance.  keep: list that receives the numpy arrays the
    Config points to (they must stay alive until the C call that reads them)."""
    ny = nx if ny is None else ny
    At, bt, A, b = (np.ascontiguousarray(x) for x in TABLEAUX[tableau])
    if keep is not None:
        keep.extend([At, bt, A, b])
    cfg = Config()
    cfg.nx, cfg.ny, cfg.lx, cfg.ly = int(nx), int(ny), float(lx), float(ly)
    cfg.q = 6
    cfg.cx = cfg.cy = None
    cfg.eps, cfg.mach, cfg.tau = float(eps), float(mach), float(tau)
    cfg.s = At.shape[0]
    cfg.a_ex, cfg.b_ex, cfg.a_im, cfg.b_im = _dptr(At), _dptr(bt), _dptr(A), _dptr(b)
    cfg.dt, cfg.cfl, cfg.c_visc = float(dt), float(cfl), float(c_visc)
    cfg.precision = int(precision)
    cfg.weno_order, cfg.central_order = int(weno_order), int(central_order)
    return cfg


def workspace_bytes(cfgs):
    arr = (Config * len(cfgs))(*cfgs)
    out = c_size_t(0)
    _check(lib().apdvm_workspace_bytes(len(cfgs), arr, ctypes.byref(out)), "workspace_bytes")
    return out.value


class Simulation:
    """A context of one or more instances stepped together.

    cases: list of dicts with keys nx, ny, eps, tau (or mach), dt, and optionally lx,
    ly, cfl, c_visc.  All instances share the tableau, the precision and the space
    discretisation (weno_order 5 or 3, central_order 4 or 2)."""

    def __init__(self, cases, tableau="ars443", precision=FP64, device=0, stream=None,
                 weno_order=5, central_order=4):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("apdvm needs a GPU")
        self.torch = torch
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        keep = []
        cfgs = []
        for c in cases:
            cfgs.append(make_config(c["nx"], c.get("ny"), eps=c["eps"], mach=c.get("mach", 1.0),
                                    tau=c.get("tau", -1.0), tableau=tableau, dt=c.get("dt", 0.0),
                                    lx=c.get("lx", 2 * np.pi), ly=c.get("ly", 2 * np.pi),
                                    cfl=c.get("cfl", 0.4), c_visc=c.get("c_visc", 0.2),
                                    precision=precision, keep=keep, weno_order=weno_order,
                                    central_order=central_order))
        self.n = len(cfgs)
        self.shapes = [(c.ny, c.nx) for c in cfgs]
        nbytes = workspace_bytes(cfgs)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # allocated on the stream the library uses it on, so the caching allocator
        # orders its reuse after that stream's work
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        arr = (Config * self.n)(*cfgs)
        ctx = c_void_p()
        _check(lib().apdvm_create(self.n, arr, c_void_p(self.workspace.data_ptr()), nbytes,
                                  c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)),
               "create")
        self.ctx = ctx
        self._keep = keep

    def close(self):
        if getattr(self, "ctx", None):
            lib().apdvm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def _host(self, a, k):
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.shape != self.shapes[k]:
            raise ValueError(f"instance {k} expects shape {self.shapes[k]}, got {a.shape}")
        return a

    def set_fields(self, k, u1, u2, theta, v1=None, v2=None, q=None):
        arrs = [self._host(a, k) if a is not None else None for a in (u1, u2, theta, v1, v2, q)]
        ptrs = [c_void_p(a.ctypes.data) if a is not None else None for a in arrs]
        _check(lib().apdvm_set_fields(self.ctx, k, *ptrs), "set_fields")

    def set_fields_device(self, k, tensors):
        """Six float64 device tensors (u1, u2, theta, v1, v2, q).  The library reads them
        on its stream, after the work already queued on the caller's current stream
        (which produced them); the call returns once they have been read."""
        t = [x.contiguous() for x in tensors]
        for x in t:
            if x.dtype != self.torch.float64 or tuple(x.shape) != self.shapes[k]:
                raise ValueError("device fields must be float64 with the instance shape")
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        arr = (c_void_p * 6)(*[x.data_ptr() for x in t])
        _check(lib().apdvm_set_fields_device(self.ctx, k, arr), "set_fields_device")

    def set_populations(self, k, F):
        F = np.ascontiguousarray(F, dtype=np.float64)
        if F.shape != (6,) + self.shapes[k]:
            raise ValueError("populations must have shape (6, ny, nx)")
        _check(lib().apdvm_set_populations(self.ctx, k, c_void_p(F.ctypes.data)),
               "set_populations")

    def step(self, nsteps=1):
        _check(lib().apdvm_step(self.ctx, int(nsteps)), "step")

    def get_fields(self, k=0):
        out = [np.empty(self.shapes[k]) for _ in range(6)]
        _check(lib().apdvm_get_fields(self.ctx, k, *[c_void_p(a.ctypes.data) for a in out]),
               "get_fields")
        return tuple(out)

    def get_fields_device(self, k, tensors):
        """Write the fields into six float64 device tensors (None skips one).  The copies
        run on the library's stream after earlier work of the caller's current stream, and
        the caller's current stream waits for them before its next work."""
        for x in tensors:
            if x is not None and (x.dtype != self.torch.float64 or tuple(x.shape) != self.shapes[k]
                                  or not x.is_contiguous()):
                raise ValueError("device fields must be contiguous float64 with the instance shape")
        cur = self.torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        arr = (c_void_p * 6)(*[x.data_ptr() if x is not None else None for x in tensors])
        _check(lib().apdvm_get_fields_device(self.ctx, k, arr), "get_fields_device")
        cur.wait_stream(self.stream)

    def get_moments(self, k=0):
        out = [np.empty(self.shapes[k]) for _ in range(4)]
        _check(lib().apdvm_get_moments(self.ctx, k, *[c_void_p(a.ctypes.data) for a in out]),
               "get_moments")
        return tuple(out)

    def get_populations(self, k=0):
        F = np.empty((6,) + self.shapes[k])
        _check(lib().apdvm_get_populations(self.ctx, k, c_void_p(F.ctypes.data)),
               "get_populations")
        return F

    def info(self, k=0):
        dt, tau, st = c_double(), c_double(), c_int64()
        _check(lib().apdvm_get_info(self.ctx, k, ctypes.byref(dt), ctypes.byref(tau),
                                    ctypes.byref(st)), "get_info")
        return dt.value, tau.value, st.value

    def set_step(self, step):
        _check(lib().apdvm_set_step(self.ctx, int(step)), "set_step")

    def set_finite_check(self, every):
        """Check the state for NaN / Inf every `every` steps inside step() (0: off)."""
        _check(lib().apdvm_set_finite_check(self.ctx, int(every)), "set_finite_check")

    def diagnostics(self, k=0):
        out = np.empty(8)
        _check(lib().apdvm_diagnostics(self.ctx, k, c_void_p(out.ctypes.data)), "diagnostics")
        return out

    def diagnostics_device(self, k, out):
        """apdvm_diagnostics into a float64 device tensor of 8 values (enqueued on the
        library's stream; the caller's current stream waits for it)."""
        if out.dtype != self.torch.float64 or out.numel() != 8 or not out.is_cuda:
            raise ValueError("out must be a float64 device tensor of 8 values")
        cur = self.torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        _check(lib().apdvm_diagnostics_device(self.ctx, k, c_void_p(out.data_ptr())),
               "diagnostics_device")
        cur.wait_stream(self.stream)

    def set_graph(self, on):
        _check(lib().apdvm_set_graph(self.ctx, 1 if on else 0), "set_graph")

    def set_overlap(self, on):
        """Stream structure: True / 1 the Helmholtz solve on a second stream beside the
        theta-free part of steps 3-4, False / 0 one stream, 2 one stream with the theta
        completion fused into the update launch."""
        _check(lib().apdvm_set_overlap(self.ctx, int(on)), "set_overlap")

    def overlap(self):
        """The stream structure (0, 1 or 2, as set_overlap takes it)."""
        on = c_int32()
        _check(lib().apdvm_get_overlap(self.ctx, ctypes.byref(on)), "get_overlap")
        return on.value

    def timing_enable(self, cls):
        _check(lib().apdvm_timing_enable(self.ctx, int(cls)), "timing_enable")

    def timing_stride(self, stride):
        _check(lib().apdvm_timing_stride(self.ctx, int(stride)), "timing_stride")

    def timing_read(self):
        n, ms = c_int64(), c_double()
        _check(lib().apdvm_timing_read(self.ctx, ctypes.byref(n), ctypes.byref(ms)),
               "timing_read")
        return n.value, ms.value

    def traffic(self, cls=-1):
        b, n = c_double(), c_int32()
        _check(lib().apdvm_traffic(self.ctx, int(cls), ctypes.byref(b), ctypes.byref(n)),
               "traffic")
        return b.value, n.value

    def autotune(self, steps_per_trial=3):
        """Pick the launch shapes by timing; returns a dict over TUNING_KEYS: tile rows of
        each stencil class (1 for the FFT classes) and the workgroup threads of each
        stencil class."""
        arr = (c_int32 * len(TUNING_KEYS))()
        _check(lib().apdvm_autotune(self.ctx, int(steps_per_trial), arr), "autotune")
        return dict(zip(TUNING_KEYS, list(arr)))

    def set_tuning(self, tile_rows=16, threads=256):
        """Force the launch shapes: tile_rows (8 or 16) and threads (256 or 512) for every
        stencil class, or a dict in the format autotune() returns (then threads is read
        from it too)."""
        arr = (c_int32 * len(TUNING_KEYS))()
        if isinstance(tile_rows, dict):
            for k, name in enumerate(TUNING_KEYS):
                arr[k] = int(tile_rows.get(name, 256 if name.startswith("threads_") else 1))
        else:
            for k in range(len(KERNEL_CLASSES)):
                arr[k] = int(tile_rows)
            for k in range(len(KERNEL_CLASSES), len(TUNING_KEYS)):
                arr[k] = int(threads)
        _check(lib().apdvm_set_tuning(self.ctx, arr), "set_tuning")

    def launches_per_step(self):
        n = c_int32()
        _check(lib().apdvm_launches_per_step(self.ctx, ctypes.byref(n)), "launches_per_step")
        return n.value
