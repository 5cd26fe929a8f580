"""Build libpencil.so (HIP kernels + host library) for gfx950 with hipcc.

Run as `python -m paper_2403_11166_amd.build`; the output lands next to this
file so it travels with the source tree.  Each translation unit compiles to
its own object in parallel (under _build/), then one link makes the library.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpencil.so")
SOURCES = [os.path.join(CSRC, f) for f in
           ("k_ntt.hip", "k_step.hip", "k_do.hip", "k_mac.hip", "k_misc.hip", "host.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # gfx950 packed-FP32 forms are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
    return res.returncode


def build(verbose=False, jobs=None):
    """Compile every source and link libpencil.so (always recompiles)."""
    os.makedirs(OBJDIR, exist_ok=True)
    tag = os.getpid()
    objs = [os.path.join(OBJDIR, os.path.basename(src) + f".{tag}.o") for src in SOURCES]
    cmds = [[HIPCC] + FLAGS + ["-c", "-o", o, src] for src, o in zip(SOURCES, objs)]
    jobs = jobs or min(len(cmds), max(1, os.cpu_count() or 1), 16)
    with ThreadPoolExecutor(jobs) as ex:
        rcs = list(ex.map(lambda c: _run(c, verbose), cmds))
    if any(rcs):
        raise RuntimeError("hipcc failed to compile libpencil.so")
    tmp = LIB + f".tmp{tag}"
    if _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, verbose):
        raise RuntimeError("hipcc failed to link libpencil.so")
    for o in objs:
        os.remove(o)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
