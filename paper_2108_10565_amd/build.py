"""Build the HIP library ``libstp.so`` in-tree for gfx950.

Steps: (1) compile and run the host table generator (``csrc/gen_tables.cpp``
+ ``csrc/basis.cpp``), which writes ``csrc/generated/khat_tables.h``;
(2) compile every ``.hip`` / ``.cpp`` source with hipcc for gfx950, one
object per source (per quantity count and degree for the fused kernels, in
parallel);
(3) link ``paper_2108_10565_amd/libstp.so``.  The tile shape of each
degree's fused kernels comes from ``tiles.json`` (written by ``autotune.py``).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libstp.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
DEGREES = range(0, 8)

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC", "-Wall", "-Werror",
    "-Wno-unused-function", "-Wno-unused-command-line-argument",
    # no packed-FP32 instructions (compiler-generated v_pk_* f32 ops are disabled)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-ffp-contract=fast",
]


def _run(cmd, cwd=None):
    r = subprocess.run(cmd, cwd=cwd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def generate_tables():
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(os.path.join(CSRC, "generated"), exist_ok=True)
    gen = os.path.join(BUILD, "gen_tables")
    _run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", "-o", gen,
          os.path.join(CSRC, "basis.cpp"), os.path.join(CSRC, "gen_tables.cpp")])
    out = os.path.join(CSRC, "generated", "khat_tables.h")
    tmp = out + ".tmp"
    _run([gen, tmp])
    if os.path.exists(out) and open(out).read() == open(tmp).read():
        os.remove(tmp)
    else:
        os.replace(tmp, out)


TILES = os.path.join(PKG, "tiles.json")


def tile_table(path: str = TILES) -> dict:
    """{degree: (threads, chunk)} of the fused kernels, as the autotuner wrote it."""
    import json
    t = json.load(open(path))["tiles"]
    return {int(n): (int(v[0]), int(v[1])) for n, v in t.items()}


# quantity counts with compiled kernels: poroelastic, damped Maxwell
QUANTITY_COUNTS = (13, 6)


def fused_object_name(nq: int, n: int) -> str:
    return f"kernel_fused_q{nq}_n{n}.o"


def fused_object_cmd(n: int, threads: int, chunk: int, obj: str, nq: int = 13):
    """hipcc command compiling the fused kernels of degree n for nq quantities
    with one tile shape."""
    return [HIPCC] + HIP_FLAGS + ["-x", "hip", f"-DSTP_NQ={nq}", f"-DSTP_DEGREE={n}",
                                  f"-DSTP_TILE_THREADS={threads}", f"-DSTP_TILE_CHUNK={chunk}", "-c",
                                  os.path.join(CSRC, "kernel_fused.hip"), "-o", obj]


def _objects():
    jobs = []
    for src in ("stp_api.hip", "kernel_ref.hip", "kernel_corrector.hip", "peaks.hip", "basis.cpp", "ader_host.cpp"):
        obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
        extra = ["-x", "hip"] if src.endswith(".hip") else []
        jobs.append(([HIPCC] + HIP_FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj], obj))
    tiles = tile_table()
    for nq in QUANTITY_COUNTS:
        for n in DEGREES:
            obj = os.path.join(BUILD, fused_object_name(nq, n))
            jobs.append((fused_object_cmd(n, *tiles[n], obj, nq), obj))
    return jobs


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile everything and link ``libstp.so``; returns its path."""
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    generate_tables()
    work = _objects()
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_run, cmd) for cmd, _ in work]
        for f in futs:
            out = f.result()
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + [o for _, o in work])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
