"""Benchmark of the element-local space-time predictor on one MI355X.

One step = one predictor call over the whole batch of elements (all of
Algorithm 3 for every element: setup, dark-blue solves, G coupling, star x
stiffness x time updates, outputs).  Inputs are generated on the host from
seeds, uploaded once, and are resident in HBM when the timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.  `value` is element-updates/s of the float64 path on
the N=6 workload of 262,144 heterogeneous poroelastic elements; the float32
chain + refinement path is timed on the same inputs and reported beside it.

    python bench.py --workload lts_mixed_1048576

times instead one cycle of clustered local time stepping (16 batches: four
rate-2 clusters x degrees 3..6, 1,048,576 elements) replayed from a captured
HIP graph.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2108_10565_amd import workload as wl  # noqa: E402

PEAK_FP64_VALU_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz
PEAK_FP32_MFMA_TFLOPS = 157.3    # dense float32 matrix-core peak
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_flops(N: int, khat_nnz: int, star_nnz: int = 54, g_nnz: int = 3, nq: int = 13) -> int:
    """FLOP per element that Algorithm 3 cannot avoid: RHS initialisation,
    dark-blue T x T solves, G couplings, star products with the non-zeros of
    the star matrices (54 per direction for the poroelastic system) for every
    mode above degree 0, and the non-zero Khat entries (the sparsity-aware
    count)."""
    B, T = wl.n_modes(N), N + 1
    return (nq * B * T + 2 * nq * T * T * B + 2 * T * B * g_nnz + 2 * 3 * star_nnz * T * (B - 1)
            + 2 * nq * T * khat_nnz)


def dense_block_flops(N: int) -> int:
    """Same count with dense star matrices and dense Khat upper blocks."""
    B, T = wl.n_modes(N), N + 1
    up = sum(g * (g + 1) * (g + 2) // 6 * (g + 1) * (g + 2) // 2 for g in range(1, N + 1))
    return (13 * B * T + 2 * 13 * T * T * B + 2 * T * B * 3 + 2 * 3 * 169 * T * (B - 1)
            + 2 * 13 * T * 3 * up)


def hbm_bytes(N: int, nq: int = 13) -> int:
    """Compulsory HBM bytes per element of one float64 call: read Q0, star, E;
    write Q and Qint."""
    B, T = wl.n_modes(N), N + 1
    return 8 * (nq * B + 4 * nq * nq + nq * B * T + nq * B)


# ---------------------------------------------------------------------------
# CPU baseline: the oracle, one element per core, before the GPU is touched
# ---------------------------------------------------------------------------

def _oracle_one(args):
    N, star, E, Q0, dt = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        from oracle import stp as ostp
        t = time.perf_counter()
        X, Qi = ostp.solve_element(N, star, E, Q0, dt)
        return X, Qi, time.perf_counter() - t


def cpu_baseline(w, ids, procs):
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    jobs = [(w.N, w.star[i], w.E[i], w.Q0[i], w.dt) for i in ids]
    t = time.perf_counter()
    with ctx.Pool(procs) as pool:
        res = pool.map(_oracle_one, jobs)
    wall = time.perf_counter() - t
    return res, wall


# ---------------------------------------------------------------------------

def torch_copy_gbs(torch, nbytes=1 << 30, reps=5):
    """Rate of torch's own device-to-device copy kernel (bytes read + written
    per second) on 1 GiB, beside the library's copy stream: what another
    implementation reaches on the same device."""
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbs


def time_path(torch, api, dev, w, steps, warmup, **kw):
    """Warm up, then time `steps` calls with HIP events on torch's current
    stream (the stream the library launches on)."""
    nq = w.Q0.shape[1]
    Q = torch.empty((w.n, nq, wl.n_modes(w.N), w.N + 1), dtype=torch.float64, device="cuda")
    Qi = torch.empty((w.n, nq, wl.n_modes(w.N)), dtype=torch.float64, device="cuda")
    # the workspace is allocated once, outside the timed calls, which then
    # allocate nothing
    ws = api.workspace_size(w.N, w.n, kw.get("precision", "fp64"), kw.get("refine_steps", 1), nq)
    kw = dict(kw, workspace=torch.empty(ws, dtype=torch.uint8, device="cuda") if ws else None)
    for _ in range(warmup):
        api.predict(dev["Q0"], dev["star"], dev["E"], w.dt, w.N, Q=Q, Qint=Qi, **kw)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_start.record()
    for k in range(steps):
        ev[k][0].record()
        api.predict(dev["Q0"], dev["star"], dev["E"], w.dt, w.N, Q=Q, Qint=Qi, **kw)
        ev[k][1].record()
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_call = [a.elapsed_time(b) for a, b in ev]
    total_ms = t_start.elapsed_time(t_end)
    return dict(ms_per_step=total_ms / steps, call_ms_mean=float(np.mean(per_call)),
                call_ms_median=float(np.median(per_call)), call_ms_min=float(np.min(per_call)),
                wall_s=wall), Q, Qi


def measured_traffic(workload: str):
    """HBM bytes per launch of the float64 fused kernel from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE of one dispatch, each scaled by
    the ratio measured on a plain device copy), or None if the summary is
    missing or was taken on other kernel sources."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_fused_fp64_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2108_10565_amd", "csrc", "kernel_fused.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec.get("kernel_fused_sha256"):
        return None
    return rec["hbm_bytes_per_launch"]


def run_lts(args):
    """One cycle of clustered local time stepping (several degrees and time
    steps, each cluster predicted rate^(K-1-k) times) captured once as a HIP
    graph and replayed: element updates per second over the cycle."""
    log(f"[bench] generating LTS workload {args.workload}")
    t = time.perf_counter()
    batches = wl.make_lts_workload(args.workload)
    cyc = wl.lts_cycle(batches)
    log(f"[bench] {len(batches)} batches, {sum(b.n for b in batches)} elements, {len(cyc)} launches per cycle, "
        f"generated in {time.perf_counter() - t:.1f}s")
    # oracle on the first element of every batch (before the GPU is touched)
    oracle = {}
    if not args.no_cpu_baseline:
        procs = args.cpu_procs or max(1, min(8, len(os.sched_getaffinity(0))))
        import multiprocessing as mp
        jobs = [(b.N, b.star[0], b.E[0], b.Q0[0], b.dt) for b in batches]
        with mp.get_context("fork").Pool(procs) as pool:
            res = pool.map(_oracle_one, jobs)
        oracle = {i: r[0] for i, r in enumerate(res)}
    import torch
    from paper_2108_10565_amd import api
    dev = [dict(degree=b.N, dt=b.dt, Q0=torch.from_numpy(b.Q0).to("cuda"),
                star=torch.from_numpy(b.star).to("cuda"), E=torch.from_numpy(b.E).to("cuda")) for b in batches]
    for d in dev:
        n, N = d["Q0"].shape[0], d["degree"]
        d["Q"] = torch.empty((n, 13, wl.n_modes(N), N + 1), dtype=torch.float64, device="cuda")
        d["Qint"] = torch.empty((n, 13, wl.n_modes(N)), dtype=torch.float64, device="cuda")
    updates = sum(batches[i].n for i in cyc)
    flops = 0
    for i in cyc:
        N = batches[i].N
        _, _, Kh = api.reference_matrices(N)
        nnz = sum(int((Kh[:, :wl.n_modes(g - 1), wl.n_modes(g - 1):wl.n_modes(g)] != 0).sum())
                  for g in range(1, N + 1))
        flops += algorithmic_flops(N, nnz) * batches[i].n
    stages = wl.lts_stages(batches)
    paths = {}
    for name, kw, staged in (("fp64", dict(precision="fp64", refine_steps=0), True),
                             ("fp64_serial_graph", dict(precision="fp64", refine_steps=0), False),
                             ("fp32_refine", dict(precision="fp32_refine", refine_steps=args.refine_steps), True)):
        if name == "fp32_refine" and args.skip_fp32:
            continue
        if staged:
            # the batches of one sub-step on parallel graph branches
            g = api.Graph([dev[i] for st in stages for i in st], stages=[len(st) for st in stages], **kw)
        else:
            g = api.Graph([dev[i] for i in cyc], **kw)
        for _ in range(args.warmup):
            g.launch()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.steps):
            g.launch()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.steps
        err = None
        if oracle:
            err = max(float(rel_l2(dev[i]["Q"][:1].cpu().numpy(), oracle[i][None])[0]) for i in oracle)
        paths[name] = dict(ms_per_cycle=ms, el_per_s=updates / (ms * 1e-3), max_rel_l2=err,
                           graph="staged (parallel branches per sub-step)" if staged else "serial", **kw)
        log(f"[bench] LTS {name}: {ms:.3f} ms per cycle, {updates / ms / 1e3:.3f} M el/s, max rel L2 {err}")
        g.close()
    p = paths["fp64"]
    achieved = flops / (p["ms_per_cycle"] * 1e-3) / 1e12
    out = {
        "metric": "element predictor updates/s over one clustered-LTS cycle (graph replay), % roofline",
        "value": p["el_per_s"], "unit": "element updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": p["ms_per_cycle"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded heterogeneous poroelastic materials, random tetrahedra, Q0 ~ N(0,1))",
        "config": {"workload": args.workload, "batches": len(batches), "launches_per_cycle": len(cyc),
                   "stages_per_cycle": len(stages),
                   "elements": sum(b.n for b in batches), "updates_per_cycle": updates,
                   "clusters": {str(k): sum(b.n for b in batches if b.meta["cluster"] == k)
                                for k in sorted({b.meta["cluster"] for b in batches})},
                   "degrees": sorted({b.N for b in batches}), "dt0": batches[0].dt},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_VALU_TFLOPS, "traffic": None,
                     "flop_per_cycle": flops},
        "cpu_baseline": None,
        "paths": paths,
    }
    print(json.dumps(out), flush=True)


ADER_CONFIGS = {
    # full ADER-DG steps (predictor + corrector), N=4, periodic cube of 32^3 x 5 = 163,840 elements
    "ader_n4_m32": dict(N=4, m=32, seed=8),
}


def _ader_oracle_predictor(args_tuple):
    N, seed = args_tuple
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        from oracle import stp as ostp
        from paper_2108_10565_amd import mesh as pmesh
        M = pmesh.periodic_cube(4)
        ABC, E = _ader_material(1)
        star = wl.star_matrices(ABC[:, 0], ABC[:, 1], ABC[:, 2], M.vertices[:1])
        Q = np.random.default_rng(seed).standard_normal((13, wl.n_modes(N)))
        t = time.perf_counter()
        ostp.solve_element(N, star[0], E[0], Q, 1e-7)
        return time.perf_counter() - t


def _ader_oracle_corrector(args_tuple):
    N, seed = args_tuple
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        from oracle import ader as oader
        from paper_2108_10565_amd import mesh as pmesh
        M = pmesh.periodic_cube(4)
        ABC, E = _ader_material(M.n)
        star = wl.star_matrices(ABC[:, 0], ABC[:, 1], ABC[:, 2], M.vertices)
        rng = np.random.default_rng(seed)
        Q = rng.standard_normal((M.n, 13, wl.n_modes(N)))
        corr = oader.Corrector(N, M, ABC)
        t = time.perf_counter()
        corr.step(star, E, Q, 1e-7 * Q)
        return (time.perf_counter() - t) / M.n


def _ader_material(n):
    mat = {k: np.array([v]) for k, v in wl.MATERIAL_CONVERGENCE.items()}
    A, B, C, E = wl.jacobians(mat)
    return (np.broadcast_to(np.stack([A[0], B[0], C[0]]), (n, 3, 13, 13)).copy(),
            np.broadcast_to(E, (n, 13, 13)).copy())


def run_ader(args):
    """Full ADER-DG steps on a periodic cube: predictor (stp_predict) and
    corrector (stp_correct) per step, each timed with HIP events; element
    updates per second of the whole step, and the corrector's roofline."""
    cfg = ADER_CONFIGS[args.workload]
    N, m = cfg["N"], cfg["m"]
    from paper_2108_10565_amd import mesh as pmesh
    log(f"[bench] {args.workload}: periodic cube mesh m={m}")
    t = time.perf_counter()
    M = pmesh.periodic_cube(m)
    ABC, E = _ader_material(M.n)
    Q0 = np.random.default_rng(cfg["seed"]).standard_normal((M.n, 13, wl.n_modes(N)))
    log(f"[bench] {M.n} elements, N={N}, generated in {time.perf_counter() - t:.1f}s")
    cpu = None
    if not args.no_cpu_baseline:
        import multiprocessing as mp
        procs = args.cpu_procs or max(1, min(8, len(os.sched_getaffinity(0))))
        log(f"[bench] cpu baseline: oracle predictor on {procs} elements ({procs} processes), "
            f"oracle corrector step on the 4^3 mesh")
        t = time.perf_counter()
        with mp.get_context("fork").Pool(procs) as pool:
            tp = pool.map(_ader_oracle_predictor, [(N, cfg["seed"] + i) for i in range(procs)])
            tc = pool.map(_ader_oracle_corrector, [(N, cfg["seed"])])[0]
        wall = time.perf_counter() - t
        per_el = float(np.mean(tp)) / procs + tc
        cpu = {"value": 1.0 / per_el, "unit": "element updates/s", "cores": procs, "kind": "oracle",
               "sample": f"oracle predictor (dense LU) on {procs} elements, one per process, mean "
                         f"{np.mean(tp):.2f}s each; oracle corrector {tc * 1e3:.2f} ms per element on the "
                         f"320-element mesh (one process); rate = 1 / (predictor / {procs} + corrector); "
                         f"wall {wall:.1f}s", "blas_threads_per_process": 1, **host_info()}
        log(f"[bench] cpu baseline {cpu['value']:.2f} el/s")

    import torch
    from paper_2108_10565_amd import api
    from paper_2108_10565_amd.ader import AderSolver
    solver = AderSolver(N, M, ABC, E)
    A, _, _, _ = wl.jacobians({k: np.array([v]) for k, v in wl.MATERIAL_CONVERGENCE.items()})
    dt = solver.cfl_dt(float(wl.max_wave_speed(A)[0]))
    Q = torch.from_numpy(Q0).cuda()
    for _ in range(args.warmup):
        solver.step(Q, dt)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for k in range(args.steps):
        ev[k][0].record()
        solver.predict(Q, dt)
        ev[k][1].record()
        solver.correct(Q)
        ev[k][2].record()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    pred = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    corr = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    nq, B = 13, wl.n_modes(N)
    corr_flop = 11 * (2 * nq * nq * B + 2 * nq * B * B) + 2 * nq * nq * B
    corr_bytes = 8 * (nq * B + 4 * nq * nq + 8 * nq * nq + 2 * nq * B) + 4 * 8
    achieved = corr_flop * M.n / (corr * 1e-3) / 1e12
    out = {
        "metric": "ADER-DG element updates/s (predictor + corrector per step), % roofline of the corrector",
        "value": M.n / (ms * 1e-3), "unit": "element updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (periodic cube mesh, material of the convergence table, Q0 ~ N(0,1))",
        "config": {"workload": args.workload, "degree": N, "elements": M.n, "mesh_subcubes": m, "dt": dt},
        # the corrector's products run on the float64 matrix cores, whose
        # dense peak equals the float64 vector peak (78.6 TFLOP/s)
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_VALU_TFLOPS, "traffic": None, "kernel": "corrector_kernel",
                     "flop_per_element": corr_flop, "bytes_per_element": corr_bytes,
                     "hbm_gbs": corr_bytes * M.n / (corr * 1e-3) / 1e9},
        "cpu_baseline": cpu,
        "paths": {"predictor_ms": pred, "corrector_ms": corr,
                  "predictor_el_per_s": M.n / (pred * 1e-3), "corrector_el_per_s": M.n / (corr * 1e-3)},
    }
    log(f"[bench] ADER step {ms:.3f} ms ({pred:.3f} predictor + {corr:.3f} corrector), "
        f"{out['value'] / 1e6:.2f} M el/s, corrector {achieved:.2f} TFLOP/s")
    print(json.dumps(out), flush=True)


def rel_l2(X, Xo):
    ax = tuple(range(1, X.ndim))
    return np.sqrt(((X - Xo) ** 2).sum(ax)) / np.sqrt((Xo ** 2).sum(ax))


def parity_report(X, Xo):
    """Max relative L2 error per element and, per quantity, the max over the
    checked elements of that quantity's relative L2 error (the quantities
    differ in size by orders of magnitude; each is measured on its own norm)."""
    el = float(rel_l2(X, Xo).max())
    ax = tuple(range(2, X.ndim))
    pq = (np.sqrt(((X - Xo) ** 2).sum(ax)) / np.sqrt((Xo ** 2).sum(ax))).max(axis=0)
    names = wl.QUANTITIES if X.shape[1] == 13 else wl.MAXWELL_QUANTITIES
    return dict(max_rel_l2=el, max_rel_l2_per_quantity=dict(zip(names, map(float, pq))),
                max_rel_l2_worst_quantity=float(pq.max()))


def host_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(cpu_model=model, nproc=os.cpu_count(), affinity_cpus=len(os.sched_getaffinity(0)))


def residual_flops(N: int, khat_nnz: int, star_nnz: int = 54, g_nnz: int = 3) -> int:
    """FLOP per element of the float64 matrix-free residual of the element
    system: right-hand side, Z X (T x T per quantity and mode), E* X (diagonal
    and G couplings), star and Khat products (sparsity-aware, as the solve)."""
    B, T = wl.n_modes(N), N + 1
    return (13 * B * T + 2 * 13 * T * T * B + 2 * T * B * (13 + g_nnz) + 2 * 3 * star_nnz * T * (B - 1)
            + 2 * 13 * T * khat_nnz + 13 * B * T)


def refine_bytes(N: int) -> int:
    """Compulsory HBM bytes per element of one refinement step: read Q0, star,
    E and the current Q; write the new Q and Qint."""
    B, T = wl.n_modes(N), N + 1
    return 8 * (13 * B + 3 * 169 + 169 + 2 * 13 * B * T + 13 * B)


def mixed_roofline(N, khat_nnz, K, ms_per_call, n):
    """Composite bound of the float32 chain + K float64-residual refinement
    steps: t >= (K+1) F/P32 + K F_res/P64 + bytes/BW (compute and memory
    terms added, as the steps depend on each other), with F the
    sparsity-aware FLOP of one solve, P32 the float32 matrix-core peak and
    P64 the float64 peak.  `frac` = bound time / measured time; `achieved`
    and `peak` are the path's FLOP over the measured and the bound time."""
    F = algorithmic_flops(N, khat_nnz)
    Fr = residual_flops(N, khat_nnz)
    by = hbm_bytes(N) + K * refine_bytes(N)
    t_bound = (K + 1) * F / (PEAK_FP32_MFMA_TFLOPS * 1e12) + K * Fr / (PEAK_FP64_VALU_TFLOPS * 1e12) \
        + by / (PEAK_HBM_GBS * 1e9)
    t = ms_per_call * 1e-3 / n
    flops = (K + 1) * F + K * Fr
    return {"bound": "composite", "achieved": flops / t / 1e12, "peak": flops / t_bound / 1e12,
            "unit": "TFLOP/s", "frac": t_bound / t, "traffic": None,
            "bound_ns_per_element": t_bound * 1e9, "measured_ns_per_element": t * 1e9,
            "flop_per_element": {"fp32_chain": F, "fp64_residual": Fr, "total": flops},
            "bytes_per_element": by,
            "peaks_used": {"fp32_tflops": PEAK_FP32_MFMA_TFLOPS, "fp64_tflops": PEAK_FP64_VALU_TFLOPS,
                           "hbm_gbs": PEAK_HBM_GBS}}


def khat_nnz(api, N):
    _, _, Kh = api.reference_matrices(N)
    return sum(int((Kh[:, :wl.n_modes(g - 1), wl.n_modes(g - 1):wl.n_modes(g)] != 0).sum())
               for g in range(1, N + 1))


def mixed_leg(args, torch, api, name):
    """The mixed-precision path on its own workload: the float32 chain alone
    (K = 0), then K = 1..3 refinement steps, each timed and checked against
    the oracle on sampled elements (error before refinement and after every
    step), beside the float64 path on the same inputs."""
    from oracle import pool as opool
    log(f"[bench] mixed-precision leg: generating {name}")
    t = time.perf_counter()
    w = wl.make_workload(name)
    # --no-cpu-baseline runs no oracle at all (profiling runs); the errors
    # against the oracle are then not reported
    ids = [] if args.no_cpu_baseline else wl.oracle_sample(w.n)[::2]
    log(f"[bench] generated n={w.n} in {time.perf_counter() - t:.1f}s; oracle on {len(ids)} elements {ids}")
    Xo = None
    if ids:
        t = time.perf_counter()
        Xo, _ = opool.solve_many(w.N, w.star[ids], w.E[ids], w.Q0[ids], w.dt)
        log(f"[bench] oracle done in {time.perf_counter() - t:.1f}s")
    dev = {k: torch.from_numpy(getattr(w, k)).to("cuda") for k in ("Q0", "star", "E")}
    torch.cuda.synchronize()
    nnz = khat_nnz(api, w.N)
    out = {"workload": name, "elements": w.n, "degree": w.N, "oracle_elements": ids, "steps": {}}
    for K in range(0, 4):
        steps = args.steps if K == args.refine_steps else max(3, min(args.steps, 10))
        tk, Q, Qi = time_path(torch, api, dev, w, steps, min(args.warmup, 3), precision="fp32_refine",
                              refine_steps=K)
        rep = parity_report(Q[ids].cpu().numpy(), Xo) if ids else {}
        del Q, Qi
        torch.cuda.empty_cache()
        rec = dict(tk, timed_calls=steps, el_per_s=w.n / (tk["call_ms_mean"] * 1e-3), **rep,
                   roofline=mixed_roofline(w.N, nnz, K, tk["call_ms_mean"], w.n))
        out["steps"][str(K)] = rec
        log(f"[bench] {name} fp32+{K}: {rec['el_per_s'] / 1e6:.3f} M el/s, call {tk['call_ms_mean']:.2f} ms, "
            f"rel L2 element {rep.get('max_rel_l2', float('nan')):.2e} worst quantity "
            f"{rep.get('max_rel_l2_worst_quantity', float('nan')):.2e}, "
            f"frac of composite bound {rec['roofline']['frac']:.3f}")
    # the same chain with its green update on the matrix cores (kept for comparison)
    out["mfma_float_chain"] = {}
    for K in (0, args.refine_steps):
        steps = max(3, min(args.steps, 10))
        tk, Q, Qi = time_path(torch, api, dev, w, steps, min(args.warmup, 3), precision="fp32_refine",
                              refine_steps=K, mfma_float_chain=True)
        rep = parity_report(Q[ids].cpu().numpy(), Xo) if ids else {}
        del Q, Qi
        torch.cuda.empty_cache()
        out["mfma_float_chain"][str(K)] = dict(tk, timed_calls=steps, el_per_s=w.n / (tk["call_ms_mean"] * 1e-3),
                                               **rep)
        log(f"[bench] {name} fp32+{K} matrix-core chain: {w.n / tk['call_ms_mean'] / 1e3:.3f} M el/s, "
            f"call {tk['call_ms_mean']:.2f} ms, worst quantity {rep.get('max_rel_l2_worst_quantity', float('nan')):.2e}")
    t64, Q, Qi = time_path(torch, api, dev, w, max(3, min(args.steps, 10)), min(args.warmup, 3),
                           precision="fp64")
    rep = parity_report(Q[ids].cpu().numpy(), Xo) if ids else {}
    del Q, Qi
    out["fp64_same_inputs"] = dict(t64, el_per_s=w.n / (t64["call_ms_mean"] * 1e-3), **rep)
    log(f"[bench] {name} fp64: {out['fp64_same_inputs']['el_per_s'] / 1e6:.3f} M el/s, "
        f"worst quantity {rep.get('max_rel_l2_worst_quantity', float('nan')):.2e}")
    del dev
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="n6_heterogeneous_262144")
    ap.add_argument("--mixed-workload", default="n6_heterogeneous_1048576",
                    help="workload of the mixed-precision leg ('none' to skip it)")
    ap.add_argument("--refine-steps", type=int, default=1,
                    help="refinement steps of the headline mixed-precision figure")
    ap.add_argument("--cpu-procs", type=int, default=0, help="oracle processes (0: min(8, cores))")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-fp32", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES (reads and writes BYTES each), "
                         "to calibrate the FETCH_SIZE / WRITE_SIZE counters, and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8, "calls": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the predictor is element-local and runs on a single "
              f"MI355X; --gpus {args.gpus} is not supported (several GPUs would each predict their "
              f"own share of the elements, with no communication inside the predictor).",
              file=sys.stderr)
        sys.exit(2)

    if args.workload in wl.LTS_CONFIGS:
        run_lts(args)
        return
    if args.workload in ADER_CONFIGS:
        run_ader(args)
        return
    log(f"[bench] generating workload {args.workload}")
    t = time.perf_counter()
    maxwell = args.workload in wl.MAXWELL_CONFIGS
    w = wl.make_maxwell_workload(args.workload) if maxwell else wl.make_workload(args.workload)
    nq = w.Q0.shape[1]
    log(f"[bench] generated n={w.n} N={w.N} dt={w.dt:.4e} in {time.perf_counter() - t:.1f}s")
    sample = wl.oracle_sample(w.n)

    cpu = None
    oracle = {}
    if not args.no_cpu_baseline:
        ncores = len(os.sched_getaffinity(0))
        procs = args.cpu_procs or max(1, min(8, ncores))
        ids = sample[:procs] if len(sample) >= procs else sample
        log(f"[bench] cpu baseline: oracle on {len(ids)} elements, {procs} processes x 1 BLAS thread")
        res, wall = cpu_baseline(w, ids, procs)
        for i, (X, Qi, _) in zip(ids, res):
            oracle[i] = (X, Qi)
        cpu = {"value": len(ids) / wall, "unit": "element updates/s", "cores": min(procs, len(ids)),
               "kind": "oracle",
               "sample": f"{len(ids)} elements of {w.name} (ids {ids[:4]}...), dense LU + "
                         f"extended-precision refinement, one element per process, 1 BLAS thread "
                         f"each, wall {wall:.1f}s",
               "per_element_s_mean": float(np.mean([r[2] for r in res])),
               "blas_threads_per_process": 1, **host_info()}
        log(f"[bench] cpu baseline {cpu['value']:.3f} el/s over {wall:.1f}s on {cpu['cpu_model']}, "
            f"nproc {cpu['nproc']}")

    import torch
    from paper_2108_10565_amd import api
    log(f"[bench] device {torch.cuda.get_device_name(0)}")
    peaks = api.measure_peaks()
    peaks["torch_copy_gbs"] = torch_copy_gbs(torch)
    log(f"[bench] measured ceilings: {peaks}")
    dev = {k: torch.from_numpy(getattr(w, k)).to("cuda") for k in ("Q0", "star", "E")}
    torch.cuda.synchronize()

    nnz = khat_nnz(api, w.N)
    # non-zeros per direction of the star matrices (54 poroelastic, 12 Maxwell)
    star_nnz = int((np.abs(w.star[:64]) != 0).sum(axis=(2, 3)).max())
    g_nnz = int((np.triu(w.E[:64], 1) != 0).sum(axis=(1, 2)).max())
    F_alg = algorithmic_flops(w.N, nnz, star_nnz, g_nnz, nq)
    F_dense = dense_block_flops(w.N) if nq == 13 else None
    F_paper, F_exec = api.flops(w.N) if nq == 13 else (None, None)
    bytes_el = hbm_bytes(w.N, nq)

    paths = {}
    log("[bench] fp64 path")
    t64, Q, Qi = time_path(torch, api, dev, w, args.steps, args.warmup, precision="fp64")
    rep64 = {}
    if oracle:
        ids = list(oracle)
        rep64 = parity_report(Q[ids].cpu().numpy(), np.stack([oracle[i][0] for i in ids]))
    paths["fp64"] = dict(t64, el_per_s=w.n / (t64["ms_per_step"] * 1e-3), **rep64)
    log(f"[bench] fp64 {paths['fp64']['el_per_s'] / 1e6:.3f} M el/s, call {t64['call_ms_mean']:.3f} ms,"
        f" {rep64}")
    dev_keep = dev if maxwell else None
    del Q, Qi, dev
    torch.cuda.empty_cache()
    if maxwell:
        log("[bench] fp32 + 1 refinement step on the same inputs")
        t32, Q, Qi = time_path(torch, api, dev_keep, w, args.steps, args.warmup, precision="fp32_refine",
                               refine_steps=args.refine_steps)
        rep32 = {}
        if oracle:
            ids = list(oracle)
            rep32 = parity_report(Q[ids].cpu().numpy(), np.stack([oracle[i][0] for i in ids]))
        paths["fp32_refine"] = dict(t32, refine_steps=args.refine_steps,
                                    el_per_s=w.n / (t32["call_ms_mean"] * 1e-3), **rep32)
        del Q, Qi, dev_keep
        torch.cuda.empty_cache()
    elif not args.skip_fp32 and args.mixed_workload != "none":
        try:
            paths["fp32_refine"] = mixed_leg(args, torch, api, args.mixed_workload)
        except Exception as exc:  # reported, never silently replaced
            paths["fp32_refine"] = dict(error=str(exc))
            log(f"[bench] fp32+refine failed: {exc}")

    p = paths["fp64"]
    kernel_s = p["call_ms_mean"] * 1e-3
    achieved = F_alg * w.n / kernel_s / 1e12
    traffic = measured_traffic(w.name)
    out = {
        "metric": "element predictor updates/s at N=6 (FP64 vs FP32+refine @ rel L2<=1e-10), % roofline",
        "value": p["el_per_s"],
        "unit": "element updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": p["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded heterogeneous poroelastic materials, random tetrahedra, Q0 ~ N(0,1))",
        "config": {"workload": w.name, "degree": w.N, "elements": w.n, "quantities": int(nq),
                   "unknowns_per_element": int(nq) * wl.n_modes(w.N) * (w.N + 1), "dt": w.dt},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU_TFLOPS, "traffic": traffic,
                     "measured_peak": peaks["fp64_valu_tflops"],
                     "flop_per_element": F_alg,
                     "hbm_gbs": bytes_el * w.n / kernel_s / 1e9,
                     "hbm_frac": bytes_el * w.n / kernel_s / 1e9 / PEAK_HBM_GBS,
                     "bytes_per_element": bytes_el},
        "cpu_baseline": cpu,
        "paths": paths,
        "machine_peaks_measured": peaks,
        "flop_counts_per_element": {"algorithmic_sparse": F_alg, "dense_block": F_dense,
                                    "executed_fused_kernel": F_exec, "paper_upper_bound": F_paper},
    }
    fr = paths.get("fp32_refine", {}).get("steps", {}).get(str(args.refine_steps))
    if fr:
        out["fp32_refine_value"] = fr["el_per_s"]
        out["fp32_refine_roofline"] = fr["roofline"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
