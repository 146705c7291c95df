"""Dense reference solution of the space-time predictor system.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Plain definition (Wolf et al., arXiv 2108.10565, eq:stp-lineq and
eq:linear_system):

    ( delta_pq W_rs M_kl - delta_pq K^tau_rs M_kl - E*_pq S_rs M_kl
      + sum_j A^{j*}_pq S_rs K^j_kl ) Q_qls  =  delta_pq w_r M_kl Q0_ql

with A^{j*} = dt A^j and E* = dt E (the dt-scaled operators defined after
eq:stp).  Multi-indices are unrolled as row (p, k, r) -> (p*B + k)*T + r and
column (q, l, s) -> (q*B + l)*T + s, so the matrix is a sum of Kronecker
products.  It is solved by dense LU with partial pivoting (LAPACK dgetrf /
dgetrs) in float64.

Before the factorisation the system is equilibrated with a diagonal matrix
of powers of two over the quantity index (X = D x', rows scaled by D^-1).
This changes no rounding of the operands (exact scaling) and keeps the
quantities' very different physical scales from spoiling the pivoted LU; it
is not part of the method, only of solving its definition accurately.

The pivoted LU alone leaves a forward error up to ~2e-10 (relative L2) at
N=6, although the system is componentwise well conditioned (one-ulp
entrywise perturbations of Y move the solution by ~4e-16).  The solution is
therefore refined (classical iterative refinement: residual r - Y x
accumulated in x87 extended precision, correction from the same LU) until
the correction drops below 1e-17 relative; this too is only about solving
the definition accurately.

Time-integrated DOFs: the paper does not define them; reading used is the
physical-time integral over the step,
    Qint_pl = dt * sum_s Q_pls * int_0^1 chi_s(tau) dtau.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
import scipy.linalg as sla

from . import basis

NQ = 13   # quantities of the poroelastic system; other systems pass their own (shape of E)


@lru_cache(maxsize=None)
def reference_operators(N: int):
    """float64 (M, K[3], S, W, w, Ktau, chi_int) for degree N."""
    M, K, _ = basis.spatial_matrices_f64(N)
    S, W, w, Kt = basis.time_matrices_f64(N)
    # int_0^1 chi_s, from the exact polynomial of chi_s
    chi_int = np.array([float(basis._pint01(basis._legendre_shifted(s))) for s in range(N + 1)])
    return M, K, S, W, w, Kt, chi_int


def _balance(Astar, Estar):
    """Power-of-two diagonal D (one entry per quantity) balancing
    sum_j |A^{j*}| + |E*|."""
    Mabs = np.abs(Astar).sum(axis=0) + np.abs(Estar)
    _, (scale, _perm) = sla.matrix_balance(Mabs, permute=False, separate=True)
    return scale


def assemble(N: int, star: np.ndarray, E: np.ndarray, Q0: np.ndarray, dt: float,
             equilibrate: bool = True):
    """Dense (Y, r, D) for one element.  star: (3,nq,nq), E: (nq,nq), Q0: (nq,B);
    nq = 13 for the poroelastic system, any other for the systems of section
    "Other applications" (same definition, another quantity count).

    Y and r are of the equilibrated system when ``equilibrate``; the
    physical solution is X = D x with x = Y^-1 r (quantity-wise scaling).
    """
    M, K, S, W, w, Kt, _ = reference_operators(N)
    B, T = M.shape[0], N + 1
    Astar = dt * np.asarray(star, dtype=np.float64)
    Estar = dt * np.asarray(E, dtype=np.float64)
    nq = Estar.shape[0]
    D = _balance(Astar, Estar) if equilibrate else np.ones(nq)
    Dinv = 1.0 / D
    Ap = Dinv[None, :, None] * Astar * D[None, None, :]
    Ep = Dinv[:, None] * Estar * D[None, :]
    Q0p = Dinv[:, None] * np.asarray(Q0, dtype=np.float64)
    Y = np.kron(np.eye(nq), np.kron(M, W - Kt))
    Y -= np.kron(Ep, np.kron(M, S))
    for j in range(3):
        Y += np.kron(Ap[j], np.kron(K[j], S))
    # r_pkr = w_r M_kk Q0_pk   (M_kl Q0_ql summed over l)
    r = np.einsum("r,kl,pl->pkr", w, M, Q0p).reshape(-1)
    return Y, r, D


def solve_element(N: int, star, E, Q0, dt, equilibrate: bool = True, return_residual=False,
                  refine: bool = True):
    """Space-time DOFs X (nq, B, N+1) and time-integrated DOFs (nq, B)."""
    Y, r, D = assemble(N, star, E, Q0, dt, equilibrate)
    lu = sla.lu_factor(Y, overwrite_a=False, check_finite=True)
    x = sla.lu_solve(lu, r)
    if refine:
        Yl = Y.astype(np.longdouble)
        rl = r.astype(np.longdouble)
        for _ in range(4):
            res = (rl - Yl @ x.astype(np.longdouble)).astype(np.float64)
            dx = sla.lu_solve(lu, res)
            x = (x.astype(np.longdouble) + dx.astype(np.longdouble)).astype(np.float64)
            if np.linalg.norm(dx) <= 1e-17 * np.linalg.norm(x):
                break
    B, T = basis.n_modes(N), N + 1
    nq = len(D)
    X = (D[:, None] * x.reshape(nq, B * T)).reshape(nq, B, T)
    _, _, _, _, _, _, chi_int = reference_operators(N)
    Qint = dt * np.einsum("pls,s->pl", X, chi_int)
    if return_residual:
        res = float(np.linalg.norm((r.astype(np.longdouble) - Y.astype(np.longdouble)
                                    @ x.astype(np.longdouble)).astype(np.float64))
                    / np.linalg.norm(r))
        return X, Qint, res
    return X, Qint


def solve(N: int, star, E, Q0, dt, equilibrate: bool = True, refine: bool = True):
    """Batched convenience wrapper: arrays with a leading element axis."""
    star = np.asarray(star); E = np.asarray(E); Q0 = np.asarray(Q0)
    n = star.shape[0]
    B = basis.n_modes(N)
    nq = E.shape[-1]
    X = np.empty((n, nq, B, N + 1))
    Qi = np.empty((n, nq, B))
    for e in range(n):
        X[e], Qi[e] = solve_element(N, star[e], E[e], Q0[e], dt, equilibrate, refine=refine)
    return X, Qi
