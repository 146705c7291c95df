"""Build the HIP library ``libstp.so`` in-tree for gfx950.

Steps: (1) compile and run the host table generator (``csrc/gen_tables.cpp``
+ ``csrc/basis.cpp``), which writes ``csrc/generated/khat_tables.h``;
(2) compile every ``.hip`` / ``.cpp`` source with hipcc for gfx950, one
object per source (per degree for the fused kernel, in parallel);
(3) link ``paper_2108_10565_amd/libstp.so``.
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


def _objects():
    jobs = []
    for src in ("stp_api.hip", "kernel_ref.hip", "peaks.hip", "basis.cpp"):
        obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
        extra = ["-x", "hip"] if src.endswith(".hip") else []
        jobs.append(([HIPCC] + HIP_FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj], obj))
    for n in DEGREES:
        obj = os.path.join(BUILD, f"kernel_fused_n{n}.o")
        jobs.append(([HIPCC] + HIP_FLAGS + ["-x", "hip", f"-DSTP_DEGREE={n}", "-c",
                      os.path.join(CSRC, "kernel_fused.hip"), "-o", obj], obj))
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
