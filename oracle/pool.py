"""Run ``oracle.stp.solve_element`` over many elements in worker processes.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  No arithmetic of the
method lives here: every element is solved by ``solve_element`` exactly as a
serial loop would, one element per task, with the BLAS of each worker held
to one thread.  Workers are started with the "spawn" method, so the pool can
be created from a process that has already initialised a GPU runtime.
"""
from __future__ import annotations

import multiprocessing as mp
import os

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


def solve_many(N: int, star, E, Q0, dt: float, procs: int | None = None):
    """(X [n,13,B,T], Qint [n,13,B]) of every element, as ``stp.solve``."""
    star = np.asarray(star); E = np.asarray(E); Q0 = np.asarray(Q0)
    n = star.shape[0]
    B = basis.n_modes(N)
    X = np.empty((n, 13, B, N + 1))
    Qi = np.empty((n, 13, B))
    if n == 0:
        return X, Qi
    procs = min(procs or default_procs(), n)
    jobs = [(N, star[e], E[e], Q0[e], float(dt)) for e in range(n)]
    if procs == 1:
        res = [_one(j) for j in jobs]
    else:
        with mp.get_context("spawn").Pool(procs) as pool:
            res = pool.map(_one, jobs, chunksize=1)
    for e, (x, q) in enumerate(res):
        X[e], Qi[e] = x, q
    return X, Qi
