"""Builds ``paper_1710_08259_amd/libnauticle.so`` for gfx950 with hipcc.

Packed-FP32 instruction selection is switched off
(``-target-feature -packed-fp32-ops``); every FP32 operation whose rounding is
part of a bit-exact result is written with contraction disabled in the source.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["api.hip", "search.hip", "sort.hip", "tile.hip", "sph.hip", "adjoint.hip", "interact.hip", "ch.hip", "verlet.hip"]
OUT = os.path.join(HERE, "libnauticle.so")
ARCH = os.environ.get("NAUTICLE_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    """Compiles every source to an object (in parallel; no device code
    crosses a source file, so no relocatable device code is needed), then
    links the shared library."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        res = subprocess.run([hipcc()] + _flags() + ["-c", "-o", obj, os.path.join(CSRC, src)],
                             capture_output=True, text=True)
        return src, obj, res

    jobs = min(len(SOURCES), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as pool:
        results = list(pool.map(compile_one, SOURCES))
    failed = False
    for src, _, res in results:
        if res.returncode != 0:
            sys.stderr.write(f"--- {src}\n" + res.stdout + res.stderr)
            failed = True
        elif verbose:
            sys.stderr.write(res.stderr)
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = OUT + ".tmp"
    res = subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp]
                         + [obj for _, obj, _ in results], capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
