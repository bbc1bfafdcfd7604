"""Build libfk.so (hipcc, gfx950) in-tree, next to this file."""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfk.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # Packed FP32 (v_pk_*_f32) stays off: the compiler would otherwise form
    # packed adds/multiplies from float2 and scalar pairs.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every HIP source of the library into libfk.so (always
    recompiles): one object per source, compiled in parallel, then linked."""
    import concurrent.futures
    import tempfile
    incs = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    objdir = tempfile.mkdtemp(prefix="fk_build_")
    srcs = sources()
    objs = [os.path.join(objdir, os.path.basename(f) + ".o") for f in srcs]

    def compile_one(src, obj):
        cmd = ["hipcc"] + [f for f in HIPCC_FLAGS if f != "-shared"] + incs + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd, capture_output=True, text=True)

    jobs = jobs or min(len(srcs), max(1, os.cpu_count() or 1), 8)
    try:
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(compile_one, srcs, objs))
        for src, res in zip(srcs, results):
            if res.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n" + res.stdout + res.stderr)
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("hipcc link failed:\n" + res.stdout + res.stderr)
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
        os.rmdir(objdir)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
