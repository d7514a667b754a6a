"""Build libkf.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2409_09228_amd.build            # build
    python -m paper_2409_09228_amd.build --resource  # also print VGPR/SGPR/LDS use per kernel
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkf.so")
SOURCES = ["kf_api.hip", "kf_step.hip", "kf_batched.hip", "kf_adjoint.hip", "kf_host.hip", "kf_smooth.hip", "kf_gate.hip"]
HEADERS = ["kf_device.h", "kf_internal.h", "kf_lanes.h", "kf_track.h", "kf_batched.h", "kf_dual.h", "kf_host.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    # fuse a*b+c into an FMA only inside one source expression, never across
    # statements: the rounding of every track is then fixed by the source and
    # identical in every kernel that runs the step (plain, persistent, adjoint)
    "-ffp-contract=on",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wl,--no-undefined",
    # never emit packed FP32 instructions (v_pk_fma_f32 and friends)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
    "-Wno-bitwise-instead-of-logical",
    f"-I{os.path.join(ROOT, 'include')}",
]


def _run(cmd, verbose: bool, show_stderr: bool):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libkf.so")
    if show_stderr:
        sys.stderr.write(r.stderr)


def build(resource_usage: bool = False, verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source to an object file (in parallel: the translation
    units share no device code, so no relocatable device code is needed),
    then link the shared library."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    compile_flags = [f for f in FLAGS if f not in ("-shared", "-Wl,--no-undefined")]
    if resource_usage:
        compile_flags = ["-Rpass-analysis=kernel-resource-usage", *compile_flags]
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="kf_build_") as tmp:
        objs = [os.path.join(tmp, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[HIPCC, *compile_flags, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
        with ThreadPoolExecutor(jobs) as ex:
            list(ex.map(lambda c: _run(c, verbose, resource_usage or verbose), cmds))
        _run([HIPCC, *FLAGS, *objs, "-o", LIB + ".tmp"], verbose, verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(resource_usage="--resource" in sys.argv, verbose="-v" in sys.argv)
    print(LIB)
