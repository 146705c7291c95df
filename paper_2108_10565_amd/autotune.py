"""Autotuner of the fused kernels' tile shape per polynomial degree.

The tile shape of degree N is (threads per workgroup, modes per chunk): how
many elements one workgroup predicts together and how many modes of a degree
block go through LDS at once.  Both trade occupancy and lane use against
LDS, registers and how widely the per-element operators and Khat coefficient
lines are shared, so the best shape is measured, not derived.

Two phases, because kernels are compiled on the host and timed on the GPU:

    python -m paper_2108_10565_amd.autotune build   [--degrees 3 4 5 6]
        compiles, for every degree and candidate shape, the fused kernels of
        that degree with that shape and links a variant library
        ``_tune/libstp_N{N}_t{T}_c{C}.so`` (the other degrees and the C ABI
        come from the regular build's objects);

    python -m paper_2108_10565_amd.autotune measure [--out DIR]
        loads each variant library, times the float64 predictor and the
        float32 chain (the two paths of the benchmark; the tile serves both)
        on a seeded synthetic workload of that degree (HIP events on one
        stream, median of several calls), checks that every variant computes
        the same outputs as the others, and writes ``tiles.json`` (per degree
        the shape with the smallest sum of the two times, with all
        measurements) for build.py to consume.

Candidates that do not compile (LDS or register limits) are skipped.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import ctypes
import json
import os
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
TUNE_DIR = os.path.join(PKG, "_tune")
CANDIDATES = [(256, 6), (256, 10), (512, 6), (512, 8), (512, 10)]
ELEMENTS = {0: 262144, 1: 262144, 2: 262144, 3: 262144, 4: 262144, 5: 262144, 6: 262144, 7: 65536}


def effective(N: int, threads: int, chunk: int):
    """(threads launched, elements per workgroup, modes per chunk) the kernel
    derives from a candidate, or None if no element fits."""
    cols = 13 * (N + 1)
    elems = min(threads // cols, 16)
    if elems < 1:
        return None
    return ((elems * cols + 63) // 64 * 64, elems, min(chunk, (N + 1) * (N + 2) // 2))


def candidates(N: int):
    """Candidate shapes of degree N, one per distinct effective tile."""
    seen, out = set(), []
    for t, c in CANDIDATES:
        e = effective(N, t, c)
        if e is not None and e not in seen:
            seen.add(e)
            out.append((t, c))
    return out


def variant_path(N: int, t: int, c: int) -> str:
    return os.path.join(TUNE_DIR, f"libstp_N{N}_t{t}_c{c}.so")


def build_variants(degrees, jobs: int | None = None, verbose: bool = True):
    from . import build as b
    objs = dict((o, cmd) for cmd, o in b._objects())
    if not all(os.path.exists(o) for o in objs):
        if verbose:
            print("[autotune] running the regular build first", flush=True)
        b.build()
    os.makedirs(TUNE_DIR, exist_ok=True)
    tune_obj = os.path.join(b.BUILD, "tune")
    os.makedirs(tune_obj, exist_ok=True)
    work = []
    for N in degrees:
        for t, c in candidates(N):
            work.append((N, t, c, os.path.join(tune_obj, f"kernel_fused_q13_n{N}_t{t}_c{c}.o")))

    def one(item):
        N, t, c, obj = item
        try:
            b._run(b.fused_object_cmd(N, t, c, obj, 13))
        except RuntimeError as exc:
            return item, str(exc).splitlines()[-1][:200]
        others = [o for o in objs if os.path.basename(o) != b.fused_object_name(13, N)]
        b._run([b.HIPCC, f"--offload-arch={b.ARCH}", "-shared", "-fPIC", "-o", variant_path(N, t, c)] + others + [obj])
        return item, None

    failed = {}
    with cf.ThreadPoolExecutor(max_workers=jobs or min(8, os.cpu_count() or 4)) as ex:
        for item, err in ex.map(one, work):
            N, t, c, _ = item
            if verbose:
                print(f"[autotune] N={N} threads={t} chunk={c}: {'built' if err is None else 'skipped: ' + err}",
                      flush=True)
            if err is not None:
                failed[f"{N}:{t}:{c}"] = err
    json.dump({"failed": failed}, open(os.path.join(TUNE_DIR, "build.json"), "w"), indent=1)
    return failed


def _load(path):
    lib = ctypes.CDLL(path)
    vp, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    lib.stp_create.argtypes = [ctypes.POINTER(vp)]
    lib.stp_predict.argtypes = [vp, vp, ctypes.c_int, i64, dbl, vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_int,
                                vp, sz, ctypes.c_uint]
    lib.stp_predict.restype = ctypes.c_int
    h = vp()
    if lib.stp_create(ctypes.byref(h)) != 0:
        raise RuntimeError(f"stp_create failed in {path}")
    return lib, h


def measure(degrees, out_dir: str, reps: int = 7, warmup: int = 2):
    import numpy as np
    import torch

    from . import workload as wl
    results = {}
    for N in degrees:
        n = ELEMENTS[N]
        w = wl.make_small(N, n, seed=900 + N)
        dev = {k: torch.from_numpy(getattr(w, k)).to("cuda") for k in ("Q0", "star", "E")}
        B, T = wl.n_modes(N), N + 1
        Q = torch.empty((n, 13, B, T), dtype=torch.float64, device="cuda")
        Qi = torch.empty((n, 13, B), dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream()
        ref = None
        per = {}
        for t, c in candidates(N):
            path = variant_path(N, t, c)
            if not os.path.exists(path):
                continue
            lib, h = _load(path)

            def call(prec):
                st = lib.stp_predict(h, ctypes.c_void_p(stream.cuda_stream), N, n, float(w.dt),
                                     ctypes.c_void_p(dev["star"].data_ptr()), ctypes.c_void_p(dev["E"].data_ptr()),
                                     ctypes.c_void_p(dev["Q0"].data_ptr()), ctypes.c_void_p(Q.data_ptr()),
                                     ctypes.c_void_p(Qi.data_ptr()), prec, 0, None, 0, 0)
                if st != 0:
                    raise RuntimeError(f"stp_predict returned {st} ({path})")

            def timed(prec):
                for _ in range(warmup):
                    call(prec)
                torch.cuda.synchronize()
                out = []
                for _ in range(reps):
                    a, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    call(prec)
                    b_.record()
                    torch.cuda.synchronize()
                    out.append(a.elapsed_time(b_))
                return out

            ms32 = timed(1)   # float32 chain, no refinement
            ms = timed(0)     # float64 last: its outputs are compared below
            sample = Q[:: max(1, n // 64)].cpu().numpy()
            if ref is None:
                ref = sample
            diff = float(np.linalg.norm(sample - ref) / np.linalg.norm(ref))
            eff = effective(N, t, c)
            per[f"{t}x{c}"] = dict(threads=t, chunk=c, threads_launched=eff[0], elements_per_workgroup=eff[1],
                                   chunk_modes=eff[2], ms_median=float(np.median(ms)), ms_min=float(min(ms)),
                                   el_per_s=n / (float(np.median(ms)) * 1e-3), rel_diff_vs_first=diff,
                                   fp32_chain_ms_median=float(np.median(ms32)),
                                   score_ms=float(np.median(ms)) + float(np.median(ms32)))
            print(f"[autotune] N={N} n={n} {t}x{c}: float64 {np.median(ms):.3f} ms "
                  f"({n / np.median(ms) / 1e3:.2f} M el/s), float32 chain {np.median(ms32):.3f} ms, "
                  f"outputs rel diff {diff:.1e}", flush=True)
            if diff > 1e-12:
                raise RuntimeError(f"variant {t}x{c} of degree {N} computes different outputs ({diff:.2e})")
        best = min(per.values(), key=lambda r: r["score_ms"])
        results[str(N)] = dict(elements=n, best=[best["threads"], best["chunk"]], candidates=per)
        del dev, Q, Qi
        torch.cuda.empty_cache()
    from . import build as b
    old = json.load(open(b.TILES))
    tiles = dict(old["tiles"])
    for N, r in results.items():
        tiles[N] = r["best"]
    doc = {"comment": old["comment"], "arch": old.get("arch", "gfx950"), "tiles": tiles,
           "measurements": {"device": torch.cuda.get_device_name(0), "date": time.strftime("%Y-%m-%d"),
                            "method": f"float64 stp_predict and the float32 chain (no refinement), median of {reps} "
                                      f"calls after {warmup} warm-ups each, HIP events on one stream; the best shape "
                                      "has the smallest sum of the two medians", "degrees": results}}
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, "tiles.json")
    json.dump(doc, open(path, "w"), indent=1)
    print(f"[autotune] wrote {path}: {tiles}", flush=True)
    return doc


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("phase", choices=["build", "measure"])
    ap.add_argument("--degrees", type=int, nargs="+", default=list(range(0, 8)))
    ap.add_argument("--out", default=os.path.join(ROOT, "gpurun_out"),
                    help="directory of the measured tiles.json (copy it over paper_2108_10565_amd/tiles.json)")
    ap.add_argument("--jobs", type=int, default=None)
    args = ap.parse_args(argv)
    if args.phase == "build":
        failed = build_variants(args.degrees, args.jobs)
        print(f"[autotune] built; {len(failed)} candidate(s) skipped", flush=True)
    else:
        measure(args.degrees, args.out)


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    main()
