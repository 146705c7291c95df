"""Parity metrics of the GPU tests (imported by them; not a test module).

The bar is a relative L2 error per element AND per (element, quantity):
the quantities of the poroelastic system differ in size by many orders of
magnitude (stresses dominate the element norm; the fluid velocities, which
the stiff Darcy source produces, weigh ~1e-9..1e-7 of it), so a single norm
over the element would not see errors in the small ones.  Every quantity of
every checked element is gated on its own norm.
"""
from __future__ import annotations

import numpy as np

TOL = 1e-10
QUANTITIES = ("sxx", "syy", "szz", "sxy", "syz", "sxz", "u", "v", "w", "p", "uf", "vf", "wf")


def rel_l2(X, Xo):
    """Relative L2 error per element over all its DOFs (arrays [n, ...])."""
    axes = tuple(range(1, X.ndim))
    return np.sqrt(((X - Xo) ** 2).sum(axes)) / np.sqrt((Xo ** 2).sum(axes))


def rel_l2_per_quantity(X, Xo):
    """Relative L2 error per element and quantity, shape [n, nq] (arrays
    [n, nq, ...]).  A quantity whose oracle values are all zero is measured
    against the element norm instead (it must then be zero to that scale)."""
    X = np.asarray(X); Xo = np.asarray(Xo)
    axes = tuple(range(2, X.ndim))
    num = np.sqrt(((X - Xo) ** 2).sum(axes))
    den = np.sqrt((Xo ** 2).sum(axes))
    el = np.sqrt((Xo ** 2).sum(tuple(range(1, X.ndim))))[:, None]
    den = np.where(den > 0, den, np.maximum(el, np.finfo(float).tiny))
    return num / den


def summary(X, Xo):
    """(max element rel L2, max over elements of each quantity's rel L2)."""
    q = rel_l2_per_quantity(X, Xo)
    return float(rel_l2(X, Xo).max()), q.max(axis=0)


def fmt(per_q):
    return " ".join(f"{QUANTITIES[i] if len(per_q) == 13 else i}={v:.1e}" for i, v in enumerate(per_q))


def check(X, Xo, tol=TOL, label="Q", say=print):
    """Asserts every element's and every (element, quantity)'s relative L2
    error <= tol; prints the per-quantity maxima; returns the worst value."""
    assert np.isfinite(X).all(), f"{label}: non-finite values"
    el, per_q = summary(X, Xo)
    worst = float(max(el, per_q.max()))
    say(f"  {label}: max rel L2 element {el:.3e}, per quantity {fmt(per_q)}")
    assert el <= tol, f"{label}: element rel L2 {el:.3e} > {tol:.0e}"
    bad = [QUANTITIES[i] if len(per_q) == 13 else str(i) for i in np.where(per_q > tol)[0]]
    assert not bad, f"{label}: per-quantity rel L2 above {tol:.0e} for {bad}: {fmt(per_q)}"
    return worst
