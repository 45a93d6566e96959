"""The bounds-checked CPU build of the host runtime (paper_2512_19847_amd/csrc/hostcheck,
built by build.build_hostcheck): the host code of the library, under AddressSanitizer and
UndefinedBehaviorSanitizer, drives every C-ABI entry point while each kernel launch is
replaced by a walk over its index space with the kernels' own index maps (tiles on the
grid and covering it once, staged halo cells the periodic images of their cells, plane
slots inside their arenas, no launch writing a plane it reads, FFT blocks fitting their
LDS form and covering every line once).  Scenarios: both precisions, every tableau
family, WENO3 / second-order operators, ragged and batched instances, and the long thin
grids that take every FFT form (including the split 8192-value column and inverse-row
forms, and the whole-row form that rows of nx = 2 mod 4 keep), and grids whose rows or
columns fill their form (the FFT register forms)."""

import os
import subprocess

import pytest

from paper_2512_19847_amd import apdvm, build

# name, precision, tableau, instances (nx, ny, eps, mach, tau, dt, weno, central)
SCENARIOS = [
    ("ars443_fp64_64", 0, "ars443", [(64, 64, 0.05, 0.1, -1.0, 0.0, 5, 4)]),
    ("ars443_split_ragged", 1, "ars443", [(96, 72, 0.05, 0.1, -1.0, 0.0, 5, 4),
                                          (64, 48, 1e-6, 0.05, -1.0, 0.0, 5, 4)]),
    ("euler1_weno3_fp64", 0, "euler1", [(48, 48, 1e-6, 0.1, 0.0, 0.0, 3, 2)]),
    ("paper2_split_eps0", 1, "paper2", [(32, 24, 0.0, 0.1, 0.05, 0.01, 5, 4)]),
    ("typea2_fp64", 0, "typea2", [(36, 36, 0.1, 0.1, -1.0, 0.0, 5, 4)]),
    ("typea1_split_weno3", 1, "typea1", [(24, 16, 0.5, 0.1, -1.0, 0.0, 3, 2)]),
    ("thin_2048_fp64", 0, "ars443", [(2048, 16, 0.05, 0.05, -1.0, 0.0, 5, 4),
                                     (16, 2048, 0.05, 0.05, -1.0, 0.0, 5, 4)]),
    ("thin_8192_split", 1, "ars443", [(8192, 8, 0.05, 0.05, -1.0, 0.0, 5, 4),
                                      (8, 8192, 0.05, 0.05, -1.0, 0.0, 5, 4)]),
    ("split_rows_radix3_fp64", 0, "ars443", [(3072, 8, 0.05, 0.05, -1.0, 0.0, 5, 4),
                                             (12, 4096, 0.05, 0.05, -1.0, 0.0, 5, 4),
                                             (6144, 8, 0.05, 0.05, -1.0, 0.0, 5, 4)]),
    ("whole_rows_nx_2mod4", 1, "ars443", [(4374, 8, 0.05, 0.05, -1.0, 0.0, 5, 4),
                                          (8, 8, 0.05, 0.05, -1.0, 0.0, 5, 4)]),
    # every row (column) as long as its form holds: the FFT register forms
    ("full_rows_1024_fp64", 0, "ars443", [(1024, 8, 0.05, 0.05, -1.0, 0.0, 5, 4)]),
    ("full_cols_2048_split", 1, "ars443", [(8, 2048, 0.05, 0.05, -1.0, 0.0, 5, 4)]),
    ("full_rows_8192_split", 1, "ars443", [(8192, 8, 0.05, 0.05, -1.0, 0.0, 5, 4)]),
    ("full_cols_8192_fp64", 0, "ars443", [(8, 8192, 0.05, 0.05, -1.0, 0.0, 5, 4)]),
    ("full_rows_two_instances_split", 1, "ars443", [(2048, 16, 0.05, 0.05, -1.0, 0.0, 5, 4),
                                                     (2048, 8, 1e-6, 0.05, -1.0, 0.0, 5, 4)]),
    # rows (columns) of 8^m values filling the blocks of a larger form: several per workgroup
    ("lines_512_rows_fp64", 0, "ars443", [(512, 16, 0.05, 0.05, -1.0, 0.0, 5, 4),
                                          (512, 32, 0.05, 0.05, -1.0, 0.0, 5, 4)]),
    ("lines_64_cols_split", 1, "ars443", [(32, 64, 0.05, 0.05, -1.0, 0.0, 5, 4)]),
    ("lines_512_and_64_rows_split", 1, "ars443", [(512, 16, 0.05, 0.05, -1.0, 0.0, 5, 4),
                                                   (64, 32, 0.05, 0.05, -1.0, 0.0, 5, 4)]),
    ("batch_sizes_split", 1, "ars443",
     [(n, n, 10.0 ** -(k % 7), 0.01 + 0.01 * k, -1.0, 0.0, 5, 4)
      for k, n in enumerate((64, 96, 128, 192, 64, 96, 8, 16, 24, 48))]),
]


def _input():
    out = []
    for name, prec, tab, insts in SCENARIOS:
        at, bt, a, b = apdvm.TABLEAUX[tab]
        out.append(f"scenario {name} {prec} {len(bt)} {len(insts)}")
        out.append(" ".join(repr(float(x)) for x in list(at.ravel()) + list(bt) +
                            list(a.ravel()) + list(b)))
        for inst in insts:
            out.append(" ".join(str(x) for x in inst))
    return "\n".join(out) + "\n"


@pytest.fixture(scope="module")
def checker():
    if not os.path.exists(build.CHECK):
        build.build_hostcheck()
    return build.CHECK


def test_every_launch_in_bounds_under_asan(checker):
    env = dict(os.environ)
    env.pop("APDVM_TUNE_CACHE", None)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    r = subprocess.run([checker], input=_input(), capture_output=True, text=True, env=env,
                       timeout=600)
    print(r.stdout)
    print(r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "0 violations, 0 unexpected statuses" in r.stdout
    assert f"{len(SCENARIOS)} scenarios" in r.stdout


def test_checks_catch_planted_mistakes(checker):
    """The checks are not vacuous: launches with a duplicated tile, a tile off the grid, a
    slot beyond its arena, an output that is also an input, a float launch on a float64
    arena, an FFT row block beyond its LDS form, the FFT register form on rows shorter than
    that form and the register form of several lines on blocks they do not fill are each
    reported, and the correct launch is not."""
    r = subprocess.run([checker, "--self-test"], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert "9 of 9 planted cases judged correctly" in r.stdout
