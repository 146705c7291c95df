"""Brute-force space-time assembly for tiny degrees (pins ``oracle.stp``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Builds the system of eq:stp entry by entry from its space-time integrals

    Y[(p,k,r),(q,l,s)] =  delta_pq chi_r(1) chi_s(1) <phi_k, phi_l>
                        - delta_pq [chi_r' phi_k, chi_s phi_l]
                        + sum_j A^{j*}_pq [chi_r phi_k, chi_s d_j phi_l]
                        - E*_pq [chi_r phi_k, chi_s phi_l]
    r[(p,k,r)]         =  chi_r(0) <phi_k, phi_l> Q0_pl

with <.,.> the spatial and [.,.] the space-time inner product of the
section "Space-Time predictor".  Nothing is factorised: every bracket is a
4-D Gauss quadrature of the full integrand.  The spatial basis is evaluated
from its Jacobi-polynomial definition with ``scipy.special.eval_jacobi``
(not from the monomial expansion used by ``oracle.basis``), spatial
derivatives by the complex-step method, and the temporal basis with
``numpy.polynomial.Legendre`` on the domain [0, 1].
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp
from numpy.polynomial import Legendre


def _mode_list(N):
    out = []
    for n in range(N + 1):
        for k in range(n + 1):
            for j in range(n - k + 1):
                out.append((n - k - j, j, k))
    return out


def phi(i, j, k, x, y, z):
    """Dubiner function from its definition in collapsed coordinates."""
    h1 = 1.0 - y - z
    h2 = 1.0 - z
    a = 2.0 * x / h1 - 1.0
    b = 2.0 * y / h2 - 1.0
    c = 2.0 * z - 1.0
    return (sp.eval_jacobi(float(i), 0.0, 0.0, a) * h1 ** i
            * sp.eval_jacobi(float(j), 2.0 * i + 1.0, 0.0, b) * h2 ** j
            * sp.eval_jacobi(float(k), 2.0 * i + 2.0 * j + 2.0, 0.0, c))


def dphi(i, j, k, x, y, z, axis, h=1e-30):
    """Complex-step derivative d phi / d x_axis (exact to rounding)."""
    pts = [np.asarray(x, complex), np.asarray(y, complex), np.asarray(z, complex)]
    pts[axis] = pts[axis] + 1j * h
    return np.imag(phi(i, j, k, *pts)) / h


def tet_quadrature(n):
    """Collapsed Gauss-Legendre rule on {x,y,z>0, x+y+z<1}: n^3 points."""
    t, wt = np.polynomial.legendre.leggauss(n)
    t = 0.5 * (t + 1.0); wt = 0.5 * wt
    U, V, Wc = np.meshgrid(t, t, t, indexing="ij")
    WU, WV, WW = np.meshgrid(wt, wt, wt, indexing="ij")
    z = Wc
    y = V * (1 - Wc)
    x = U * (1 - V) * (1 - Wc)
    w = WU * WV * WW * (1 - V) * (1 - Wc) ** 2
    return x.ravel(), y.ravel(), z.ravel(), w.ravel()


def assemble_brute(N, star, E, Q0, dt, nq_space=None, nq_time=None):
    """Unequilibrated dense (Y, r) of eq:stp for one element, tiny N only."""
    modes = _mode_list(N)
    B, T, NQ = len(modes), N + 1, np.asarray(E).shape[0]
    nq_space = nq_space or (N + 3)
    nq_time = nq_time or (N + 2)
    x, y, z, ws = tet_quadrature(nq_space)
    tau, wt = np.polynomial.legendre.leggauss(nq_time)
    tau = 0.5 * (tau + 1.0); wt = 0.5 * wt
    chi = [Legendre.basis(s, domain=[0.0, 1.0]) for s in range(T)]
    # 4-D evaluation grids: space points (P) x time points (Tq)
    ph = np.array([phi(*m, x, y, z) for m in modes])                        # (B, P)
    dph = np.array([[dphi(*m, x, y, z, a) for m in modes] for a in range(3)])  # (3, B, P)
    ch = np.array([c(tau) for c in chi])                                    # (T, Tq)
    dch = np.array([c.deriv()(tau) for c in chi])                           # (T, Tq)
    w4 = ws[:, None] * wt[None, :]                                          # (P, Tq)

    def st(f_r, g_k, f_s, g_l):
        # [f_r(tau) g_k(x), f_s(tau) g_l(x)] as a full 4-D quadrature
        integrand = (g_k[:, None] * f_r[None, :]) * (g_l[:, None] * f_s[None, :])
        return float((integrand * w4).sum())

    c1 = np.array([c(1.0) for c in chi])
    c0 = np.array([c(0.0) for c in chi])
    mass_sp = np.array([[float((ph[k] * ph[l] * ws).sum()) for l in range(B)] for k in range(B)])
    I_time = np.empty((B, B, T, T))
    I_dtime = np.empty((B, B, T, T))
    I_grad = np.empty((3, B, B, T, T))
    for k in range(B):
        for l in range(B):
            for r in range(T):
                for s in range(T):
                    I_time[k, l, r, s] = st(ch[r], ph[k], ch[s], ph[l])
                    I_dtime[k, l, r, s] = st(dch[r], ph[k], ch[s], ph[l])
                    for a in range(3):
                        I_grad[a, k, l, r, s] = st(ch[r], ph[k], ch[s], dph[a, l])
    Astar = dt * np.asarray(star, float)
    Estar = dt * np.asarray(E, float)
    s_all = NQ * B * T
    Y = np.zeros((s_all, s_all))
    r_vec = np.zeros(s_all)
    idx = lambda p, k, r: (p * B + k) * T + r
    for p in range(NQ):
        for k in range(B):
            for r in range(T):
                i = idx(p, k, r)
                r_vec[i] = c0[r] * sum(mass_sp[k, l] * Q0[p, l] for l in range(B))
                for q in range(NQ):
                    for l in range(B):
                        for s in range(T):
                            v = 0.0
                            if p == q:
                                v += c1[r] * c1[s] * mass_sp[k, l] - I_dtime[k, l, r, s]
                            v += sum(Astar[a, p, q] * I_grad[a, k, l, r, s] for a in range(3))
                            v -= Estar[p, q] * I_time[k, l, r, s]
                            Y[i, idx(q, l, s)] = v
    return Y, r_vec
