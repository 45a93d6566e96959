"""Build the HIP library libapdvm.so in-tree for gfx950.

    python -m paper_2512_19847_amd.build

Every source under csrc/ is compiled and linked in one hipcc call.  Packed FP32
instructions are disabled for device code (-packed-fp32-ops); hipcc's host pass warns
that it does not know that feature, which is harmless.
"""

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libapdvm.so")


def hipcc_command(out=LIB, extra=()):
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    return (["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-shared", "-Wall", "-Wno-unused-function",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
            + list(extra) + srcs + ["-o", out])


def build(verbose=False):
    cmd = hipcc_command()
    tmp = LIB + ".tmp"
    cmd[-1] = tmp
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


CHECK = os.path.join(HERE, "apdvm_hostcheck")


def hostcheck_command(out=CHECK):
    """The bounds-checked CPU build: the host runtime (host.hip as C++) against a host-only
    stand-in of the HIP runtime and launch functions that check every launch's index space
    instead of running kernels (csrc/hostcheck/), with AddressSanitizer and
    UndefinedBehaviorSanitizer.  Host code only: no device code is built."""
    d = os.path.join(HERE, "csrc", "hostcheck")
    srcs = [os.path.join(d, f) for f in ("host_unit.cpp", "hip_host.cpp", "launch_check.cpp",
                                         "driver.cpp")]
    return (["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-DAPDVM_HOSTCHECK", "-Wall", "-Wno-attributes", "-Wno-unused-function",
             "-I", d, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
            + srcs + ["-o", out])


def build_hostcheck():
    cmd = hostcheck_command()
    tmp = CHECK + ".tmp"
    cmd[-1] = tmp
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hostcheck build failed:\n" + res.stderr)
    os.replace(tmp, CHECK)
    return CHECK


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_hostcheck())
