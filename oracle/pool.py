"""Run ``oracle.stp.solve_element`` over many elements in worker processes.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  No arithmetic of the
method lives here: every element is solved by ``solve_element`` exactly as a
serial loop would, one element per task, with the BLAS of each worker held
to one thread.  Workers are started with the "spawn" method, so the pool can
be created from a process that has already initialised a GPU runtime.
"""
from __future__ import annotations

import atexit
import multiprocessing as mp
import os
import sys

import numpy as np

from . import basis


def _one(args):
    N, star, E, Q0, dt = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        from . import stp
        return stp.solve_element(N, star, E, Q0, dt)


def default_procs() -> int:
    """Worker count: the CPUs this process may run on, at most 16."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


# rough single-thread seconds per element by degree (dense LU of 13 B (N+1)
# unknowns); small batches are solved in this process
_COST = {0: 1e-3, 1: 1e-3, 2: 0.01, 3: 0.1, 4: 0.6, 5: 4.0, 6: 30.0, 7: 120.0}
_POOL = None


def _pool():
    """The worker pool, started once (spawn) and kept for later calls."""
    global _POOL
    if _POOL is None:
        _POOL = mp.get_context("spawn").Pool(default_procs())
        atexit.register(_POOL.terminate)
    return _POOL


def solve_jobs(jobs, procs: int | None = None, progress=None):
    """Solves every job (N, star, E, Q0, dt) of one element with
    ``stp.solve_element``; returns the list of (X, Qint).  ``progress(k, n)``
    is called as results come in (in any order).  procs=1 solves in this
    process; otherwise a persistent worker pool is used unless the batch is
    cheap."""
    jobs = [(int(N), np.asarray(s), np.asarray(e), np.asarray(q), float(dt)) for N, s, e, q, dt in jobs]
    if not jobs:
        return []
    cost = sum(_COST.get(j[0], 120.0) for j in jobs)
    if procs == 1 or len(jobs) == 1 or cost < 2.0:
        out = []
        for k, j in enumerate(jobs):
            out.append(_one(j))
            if progress:
                progress(k + 1, len(jobs))
        return out
    out = [None] * len(jobs)
    # highest degree first, so the pool drains evenly
    order = sorted(range(len(jobs)), key=lambda i: -jobs[i][0])
    for k, (i, res) in enumerate(_pool().imap_unordered(_indexed, [(i, jobs[i]) for i in order])):
        out[i] = res
        if progress:
            progress(k + 1, len(jobs))
    return out


def _indexed(arg):
    i, job = arg
    return i, _one(job)


def _print_progress(k, n):
    if k == n or k % 4 == 0:
        print(f"[oracle] {k}/{n} elements solved", file=sys.stderr, flush=True)


def solve_many(N: int, star, E, Q0, dt: float, procs: int | None = None, progress=_print_progress):
    """(X [n,13,B,T], Qint [n,13,B]) of every element, as ``stp.solve``."""
    star = np.asarray(star); E = np.asarray(E); Q0 = np.asarray(Q0)
    n = star.shape[0]
    B = basis.n_modes(N)
    nq = E.shape[-1]
    X = np.empty((n, nq, B, N + 1))
    Qi = np.empty((n, nq, B))
    res = solve_jobs([(N, star[e], E[e], Q0[e], dt) for e in range(n)], procs, progress)
    for e, (x, q) in enumerate(res):
        X[e], Qi[e] = x, q
    return X, Qi
