"""Build the gfx950 HIP libraries in-tree with hipcc: ``librecon.so`` (the
reconstruction) and ``libstream_probe.so`` (the streaming-bandwidth probes the
benchmark measures its ceilings with).  Each source is compiled to its own
object in parallel, then linked."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librecon.so")
PROBE_LIB = os.path.join(HERE, "libstream_probe.so")
PROBE_SOURCES = ["stream_probe.hip"]
OBJ_DIR = os.path.join(HERE, "_build")
SOURCES = ["recon_kernels.hip", "rbgs_fused.hip", "stencil25.hip", "transfer25.hip", "resrestrict25.hip", "pdcheck25.hip", "outer25.hip", "massupdate.hip", "fullop25.hip", "particles.hip", "recon_adjoint.hip", "recon_api.hip"]
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics",
    # no packed FP32 instructions: hipcc would otherwise form them from scalar
    # and float2 code, and the kernels are kept on plain FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".o")
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    cmd = [hipcc()] + flags + ["-c", "-I", INCLUDE, "-o", obj, os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def _link(objs, lib: str, verbose: bool) -> str:
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP source (always recompiles) and link librecon.so and
    libstream_probe.so."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES + PROBE_SOURCES))
    _link(objs[:len(SOURCES)], LIB, verbose)
    _link(objs[len(SOURCES):], PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
