"""Exact rational construction of the predictor's reference matrices.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): never imported by
the product path.

Everything here follows the definitions of section "ADER-DG
discretisation" of Wolf et al. (arXiv 2108.10565):

* temporal basis chi_s on the reference interval [0, 1]: the paper only
  says "Jacobi polynomials"; S must be diagonal (section "Structure of the
  system matrix"), which singles out the Legendre family.  Reading used:
  chi_s(tau) = P_s(2 tau - 1), unnormalised (chi_s(1) = 1).
* matrices W_rs = chi_r(1) chi_s(1), w_r = chi_r(0),
  S_rs = int_0^1 chi_r chi_s, K^tau_rs = int_0^1 chi_r' chi_s
  (definitions following eq:stp).
* spatial basis: Dubiner polynomials on the reference tetrahedron
  {x, y, z > 0, x + y + z < 1}, ordered by total degree (subsection
  "Spatial discretisation").  The paper gives neither formula, intra-degree
  order nor normalisation; reading used:
      phi_ijk = P_i(a) (1-y-z)^i * P_j^(2i+1,0)(b) (1-z)^j
                * P_k^(2i+2j+2,0)(c),
      a = 2x/(1-y-z) - 1,  b = 2y/(1-z) - 1,  c = 2z - 1,
  unnormalised, ordered by n = i+j+k, then k = 0..n, then j = 0..n-k.
* M_kl = int phi_k phi_l and K^alpha_kl = int phi_k d_alpha phi_l
  (definitions following eq:stp).

All integrals are exact: every basis function is expanded into monomials
x^a y^b z^c with integer coefficients and integrated with
    int_E x^a y^b z^c dV = a! b! c! / (a+b+c+3)!.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import comb, factorial

import numpy as np

NQ = 13  # quantities of the poroelastic system (section "Governing equations")


# ----------------------------------------------------------------------------
# sizes
# ----------------------------------------------------------------------------

def n_modes(N: int) -> int:
    """Number of spatial basis functions of degree <= N: C(N+3, 3)."""
    return (N + 1) * (N + 2) * (N + 3) // 6


def block_size(g: int) -> int:
    """Number of basis functions of exact degree g: C(g+2, 2)."""
    return (g + 1) * (g + 2) // 2


def block_start(g: int) -> int:
    """Index of the first basis function of degree g (0-based)."""
    return g * (g + 1) * (g + 2) // 6


def mode_indices(N: int):
    """(i, j, k) of each spatial basis function in the order described above."""
    out = []
    for n in range(N + 1):
        for k in range(n + 1):
            for j in range(n - k + 1):
                out.append((n - k - j, j, k))
    return out


# ----------------------------------------------------------------------------
# tiny exact polynomial algebra in (x, y, z); dict exponent-tuple -> int
# ----------------------------------------------------------------------------

def _padd(p, q, s=1):
    r = dict(p)
    for e, c in q.items():
        r[e] = r.get(e, 0) + s * c
        if r[e] == 0:
            del r[e]
    return r


def _pmul(p, q):
    r = {}
    for e1, c1 in p.items():
        for e2, c2 in q.items():
            e = (e1[0] + e2[0], e1[1] + e2[1], e1[2] + e2[2])
            r[e] = r.get(e, 0) + c1 * c2
    return {e: c for e, c in r.items() if c != 0}


def _ppow(p, n):
    r = {(0, 0, 0): 1}
    for _ in range(n):
        r = _pmul(r, p)
    return r


def _pscale(p, s):
    return {e: c * s for e, c in p.items() if c * s != 0}


def _homogenised_jacobi(n, alpha, U, V):
    """h^n P_n^(alpha,0)(t) written with U = h (t-1)/2 and V = h (t+1)/2.

    Uses the explicit sum
        P_n^(a,b)(t) = sum_s C(n+a, n-s) C(n+b, s) ((t-1)/2)^s ((t+1)/2)^(n-s)
    (b = 0 here), so the result has integer coefficients.
    """
    r = {}
    for s in range(n + 1):
        term = _pmul(_ppow(U, s), _ppow(V, n - s))
        r = _padd(r, _pscale(term, comb(n + alpha, n - s) * comb(n, s)))
    return r


_X = {(1, 0, 0): 1}
_Y = {(0, 1, 0): 1}
_Zv = {(0, 0, 1): 1}
_ONE = {(0, 0, 0): 1}


def dubiner(i: int, j: int, k: int):
    """Monomial expansion of phi_ijk (integer coefficients)."""
    # a-part: h = 1-y-z, h (a+1)/2 = x, h (a-1)/2 = x - (1-y-z)
    Ua = _padd(_padd(_X, _ONE, -1), _padd(_Y, _Zv))
    fa = _homogenised_jacobi(i, 0, Ua, _X)
    # b-part: h = 1-z, h (b+1)/2 = y, h (b-1)/2 = y - (1-z)
    Ub = _padd(_padd(_Y, _ONE, -1), _Zv)
    fb = _homogenised_jacobi(j, 2 * i + 1, Ub, _Y)
    # c-part: h = 1, (c+1)/2 = z, (c-1)/2 = z - 1
    Uc = _padd(_Zv, _ONE, -1)
    fc = _homogenised_jacobi(k, 2 * i + 2 * j + 2, Uc, _Zv)
    return _pmul(_pmul(fa, fb), fc)


def derivative(p, axis: int):
    r = {}
    for e, c in p.items():
        if e[axis] > 0:
            ee = list(e)
            ee[axis] -= 1
            r[tuple(ee)] = r.get(tuple(ee), 0) + c * e[axis]
    return {e: c for e, c in r.items() if c != 0}


def monomial_integral(a: int, b: int, c: int) -> Fraction:
    """int over the reference tetrahedron of x^a y^b z^c (Dirichlet integral)."""
    return Fraction(factorial(a) * factorial(b) * factorial(c), factorial(a + b + c + 3))


def integrate(p) -> Fraction:
    return sum((c * monomial_integral(*e) for e, c in p.items()), Fraction(0))


# ----------------------------------------------------------------------------
# spatial matrices, exact
# ----------------------------------------------------------------------------

def _monomials(D):
    return [(a, b, c) for s in range(D + 1) for c in range(s + 1)
            for b in range(s - c + 1) for a in [s - c - b]]


@lru_cache(maxsize=None)
def spatial_matrices(N: int):
    """Exact M (B x B) and K^alpha (3 x B x B) as nested lists of Fractions.

    M_kl = int phi_k phi_l,  K^alpha_kl = int phi_k d_alpha phi_l.
    Computed as C G C^T with C the integer monomial coefficients of the
    basis and G the (scaled, integer) Gram matrix of monomials.
    """
    modes = mode_indices(N)
    B = len(modes)
    mons = _monomials(N)
    midx = {m: t for t, m in enumerate(mons)}
    nm = len(mons)
    polys = [dubiner(*m) for m in modes]

    def coeff_matrix(plist):
        C = np.zeros((len(plist), nm), dtype=object)
        C[:] = 0
        for r, p in enumerate(plist):
            for e, c in p.items():
                C[r, midx[e]] = c
        return C

    L = factorial(2 * N + 3)  # common denominator of every Gram entry
    G = np.zeros((nm, nm), dtype=object)
    for u, m1 in enumerate(mons):
        for v, m2 in enumerate(mons):
            a, b, c = m1[0] + m2[0], m1[1] + m2[1], m1[2] + m2[2]
            G[u, v] = factorial(a) * factorial(b) * factorial(c) * (L // factorial(a + b + c + 3))
    C = coeff_matrix(polys)
    CG = C.dot(G)
    M_int = CG.dot(C.T)
    M = [[Fraction(int(M_int[k, l]), L) for l in range(B)] for k in range(B)]
    K = []
    for axis in range(3):
        D = coeff_matrix([derivative(p, axis) for p in polys])
        K_int = CG.dot(D.T)
        K.append([[Fraction(int(K_int[k, l]), L) for l in range(B)] for k in range(B)])
    return M, K


def spatial_matrices_f64(N: int):
    """(M, K, Khat) as float64 arrays; Khat^alpha = M^{-1} K^alpha (exact
    division, M being diagonal for an orthogonal basis), then rounded."""
    M, K = spatial_matrices(N)
    B = len(M)
    Mf = np.array([[float(v) for v in row] for row in M])
    Kf = np.array([[[float(v) for v in row] for row in Ka] for Ka in K])
    Kh = np.array([[[float(K[a][k][l] / M[k][k]) for l in range(B)] for k in range(B)]
                   for a in range(3)])
    return Mf, Kf, Kh


# ----------------------------------------------------------------------------
# temporal matrices, exact
# ----------------------------------------------------------------------------

def _legendre_shifted(s: int):
    """Coefficients (ascending powers of tau) of chi_s(tau) = P_s(2 tau - 1),
    from the same explicit Jacobi sum with (t-1)/2 = tau-1, (t+1)/2 = tau."""
    coeffs = [0] * (s + 1)
    for m in range(s + 1):
        # C(s, s-m) C(s, m) (tau-1)^m tau^(s-m)
        w = comb(s, s - m) * comb(s, m)
        for t in range(m + 1):  # (tau-1)^m = sum_t C(m,t) tau^t (-1)^(m-t)
            coeffs[t + s - m] += w * comb(m, t) * (-1) ** (m - t)
    return coeffs


def _pint01(c):
    return sum((Fraction(v, n + 1) for n, v in enumerate(c)), Fraction(0))


def _pmul1(a, b):
    r = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            r[i + j] += x * y
    return r


@lru_cache(maxsize=None)
def time_matrices(N: int):
    """Exact (S, W, w, Ktau) for T = N+1 temporal modes (nested Fractions)."""
    T = N + 1
    chi = [_legendre_shifted(s) for s in range(T)]
    dchi = [[n * c for n, c in enumerate(p)][1:] or [0] for p in chi]
    S = [[_pint01(_pmul1(chi[r], chi[s])) for s in range(T)] for r in range(T)]
    W = [[Fraction(sum(chi[r])) * Fraction(sum(chi[s])) for s in range(T)] for r in range(T)]
    w = [Fraction(chi[r][0]) for r in range(T)]
    Kt = [[_pint01(_pmul1(dchi[r], chi[s])) for s in range(T)] for r in range(T)]
    return S, W, w, Kt


def time_matrices_f64(N: int):
    S, W, w, Kt = time_matrices(N)
    f = lambda A: np.array([[float(v) for v in row] for row in A])
    return f(S), f(W), np.array([float(v) for v in w]), f(Kt)
