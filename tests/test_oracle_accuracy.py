"""Accuracy of the oracle per quantity (CPU).

The GPU parity gate is a relative L2 error of 1e-10 per element AND per
(element, quantity).  The quantities differ in size by orders of magnitude
(stresses ~1e5, fluid velocities ~1e-2 in the parity workloads), so the gate
is only meaningful if the oracle itself is accurate per quantity, not just
in the element norm dominated by the stresses.  These tests bound the
oracle's forward error per quantity a posteriori:

    |x - x*| <= |Y^-1| ( |r - Y x| + c eps (|Y| |x| + |r|) ) + eps |x|

(first order; Y^-1 in float64).  The first term is the residual of the
returned solution, evaluated in extended precision; the second covers the
rounding of the assembled operands (every entry of Y and r is a short sum
of products of rounded factors, c = 16 is generous); the last is the
rounding of x itself.  Each quantity's bound, relative to that quantity's
norm, must lie far below the GPU gate.
"""
import numpy as np
import pytest

from oracle import stp
from paper_2108_10565_amd import workload as wl

EPS = np.finfo(float).eps
BOUND = 1e-12          # two decades below the GPU gate of 1e-10


def per_quantity_bound(N, star, E, Q0, dt):
    Y, r, D = stp.assemble(N, star, E, Q0, dt)
    X, _ = stp.solve_element(N, star, E, Q0, dt)
    nq = len(D)
    x = (X.reshape(nq, -1) / D[:, None]).reshape(-1)     # equilibrated unknowns
    res = (r.astype(np.longdouble) - Y.astype(np.longdouble) @ x.astype(np.longdouble)).astype(np.float64)
    pert = np.abs(res) + 16 * EPS * (np.abs(Y) @ np.abs(x) + np.abs(r))
    dx = np.abs(np.linalg.inv(Y)) @ pert + EPS * np.abs(x)
    # quantity-wise scaling by D does not change a quantity's relative error
    dq = np.linalg.norm(dx.reshape(nq, -1), axis=1)
    xq = np.linalg.norm(x.reshape(nq, -1), axis=1)
    return dq / xq, np.linalg.norm(X.reshape(nq, -1), axis=1)


def _assert_bound(b, norms, label):
    print(f"{label}: per-quantity relative bound max {b.max():.2e}; quantity norms "
          f"{np.array2string(norms, precision=1)}")
    assert np.all(b <= BOUND), b


def test_config1_element_per_quantity_accuracy():
    """Homogeneous N=3 element of the 64-element parity workload: the fluid
    velocities are ~1e-7 of the stresses, and still accurate to ~1e-14."""
    w = wl.make_workload("n3_homogeneous_64", elements=[0, 37])
    for e in range(2):
        b, norms = per_quantity_bound(3, w.star[e], w.E[e], w.Q0[e], w.dt)
        _assert_bound(b, norms, f"n3_homogeneous_64[{[0, 37][e]}]")
        assert norms[10:].max() < 1e-5 * norms[:6].min()   # the scale gap the gate must see through


def test_heterogeneous_n5_per_quantity_accuracy():
    w = wl.make_small(5, 1, seed=23)
    b, norms = per_quantity_bound(5, w.star[0], w.E[0], w.Q0[0], w.dt)
    _assert_bound(b, norms, "heterogeneous N=5")


@pytest.mark.parametrize("decade", [-2, 2, 5])
def test_stiffness_n5_per_quantity_accuracy(decade):
    """Elements of the stiffness workload with dt |E_uf,uf| of 1e-2, 1e2, 1e5."""
    w = wl.make_small(5, 48, seed=41, kind="stiffness")
    z = wl.stiffness(w)
    e = int(np.where(np.floor(np.log10(z)).astype(int) == decade)[0][0])
    b, norms = per_quantity_bound(5, w.star[e], w.E[e], w.Q0[e], w.dt)
    _assert_bound(b, norms, f"stiffness decade 1e{decade}")


@pytest.mark.slow
def test_heterogeneous_n6_per_quantity_accuracy():
    """An element of the full-size N=6 benchmark workload."""
    w = wl.make_workload("n6_heterogeneous_262144", elements=[wl.oracle_sample(262144)[5]])
    b, norms = per_quantity_bound(6, w.star[0], w.E[0], w.Q0[0], w.dt)
    _assert_bound(b, norms, "n6_heterogeneous_262144")
