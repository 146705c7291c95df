"""One ADER-DG time step on a mesh: predictor + corrector (CPU oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section "ADER-DG discretisation" of Wolf et al. (arXiv 2108.10565): the weak
form eq:poroelastic-weak, after integration by parts, gives the semi-discrete
system eq:semi_discrete; integrating it over one time step with the
predictor's space-time solution (``oracle.stp``) in place of q gives, for the
DOFs Q_pk of element T (test function phi_k, |J| the volume ratio of the
element map),

  |J| M_kk (Q^{n+1} - Q^n)_pk
      =  |J| sum_j A^j_pq Qint_ql int phi_l d_j phi_k         (volume)
       + |J| M_kk E_pq Qint_qk                                (source)
       - sum_faces int_face phi_k (An^+ q^- + An^- q^+)_p dS  (Godunov flux)

with Qint = int Q dt over the step (physical time), q^- / q^+ the own and the
neighbour's time-integrated solution on the face, An = nu . (A, B, C) the
physical normal Jacobian and An^+- its upwind split (Godunov's flux for a
linear system: the exact Riemann solution, section "Spatial discretisation").

Every integral here is evaluated directly: volume terms with the exact
rational basis matrices of ``oracle.basis``; face terms by Gauss quadrature
on the physical face, the points mapped into both elements' reference
coordinates with the inverse of each element's affine map and the basis
evaluated from its exact monomial expansion; An^+- from the eigenspaces of
the balanced normal Jacobian (null spaces by SVD, spectral projectors).

Reference solution (section "Planar wave convergence analysis"): q(x, t) =
Re sum_n alpha_n r_n exp(i (omega_n t - k . x)) with (omega_n, r_n) the
eigenpairs of k_x A + k_y B + k_z C - i E.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
import scipy.linalg as sla

from . import basis, stp


# ----------------------------------------------------------------------------
# basis at points, quadrature
# ----------------------------------------------------------------------------

@lru_cache(maxsize=None)
def _expansions(N):
    return [basis.dubiner(*m) for m in basis.mode_indices(N)]


def basis_at(N: int, pts):
    """phi_l at reference points pts [P, 3] -> [P, B], from the exact monomial
    expansions of the Dubiner functions."""
    pts = np.asarray(pts, float)
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    out = np.zeros((len(pts), basis.n_modes(N)))
    for l, poly in enumerate(_expansions(N)):
        for (a, b, c), coef in poly.items():
            out[:, l] += float(coef) * x ** a * y ** b * z ** c
    return out


def triangle_quadrature(n):
    """Points (s, t) and weights of a collapsed Gauss rule on {s, t >= 0,
    s + t <= 1} (weights sum to 1/2)."""
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1.0); w = 0.5 * w
    S, T = np.meshgrid(g, g, indexing="ij")
    WS, WT = np.meshgrid(w, w, indexing="ij")
    return (S * (1 - T)).ravel(), T.ravel(), (WS * WT * (1 - T)).ravel()


def tet_quadrature(n):
    """Collapsed Gauss rule on the reference tetrahedron: points [n^3, 3], weights."""
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1.0); w = 0.5 * w
    U, V, W = np.meshgrid(g, g, g, indexing="ij")
    WU, WV, WW = np.meshgrid(w, w, w, indexing="ij")
    z = W
    y = V * (1 - W)
    x = U * (1 - V) * (1 - W)
    wt = WU * WV * WW * (1 - V) * (1 - W) ** 2
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1), wt.ravel()


# ----------------------------------------------------------------------------
# Godunov split
# ----------------------------------------------------------------------------

def upwind_split(An, D=None, tol=1e-7):
    """(An^+, An^-) of a real-spectrum, diagonalisable matrix: sum of lambda
    P_lambda over the positive / negative eigenvalues, P_lambda the spectral
    projector R (L^T R)^-1 L^T on bases R, L of the right and left
    eigenspaces (null spaces by SVD).  Computed on D^-1 An D with the
    diagonal scaling D (powers of two; default: balancing of |An|), which
    must equalise the rows and columns of An well: an axis-aligned normal
    leaves exact zero rows in An, so the element's D (balancing of
    |A| + |B| + |C|) is the robust choice."""
    An = np.asarray(An, float)
    n = An.shape[0]
    if D is None:
        _, (D, _) = sla.matrix_balance(np.abs(An), permute=False, separate=True)
    Ab = An / D[:, None] * D[None, :]
    lam = np.linalg.eigvals(Ab)
    lmax = np.abs(lam).max()
    if lmax == 0.0:
        return np.zeros_like(An), np.zeros_like(An)
    assert np.abs(lam.imag).max() <= 1e-8 * lmax, "normal Jacobian is not hyperbolic"
    groups = []
    for v in np.sort(lam.real):
        if groups and v - groups[-1][-1] <= tol * lmax:
            groups[-1].append(v)
        else:
            groups.append([v])
    plus = np.zeros_like(An)
    minus = np.zeros_like(An)
    for g in groups:
        l = float(np.mean(g))
        if abs(l) <= tol * lmax:
            continue
        R = sla.null_space(Ab - l * np.eye(n), rcond=1e-9)
        L = sla.null_space((Ab - l * np.eye(n)).T, rcond=1e-9)
        assert R.shape[1] == len(g) == L.shape[1], "not diagonalisable"
        P = R @ np.linalg.solve(L.T @ R, L.T)
        if l > 0:
            plus += l * P
        else:
            minus += l * P
    return plus * D[:, None] / D[None, :], minus * D[:, None] / D[None, :]


def jacobian_scaling(ABC):
    """Power-of-two balancing D of |A| + |B| + |C| (one element's Jacobians)."""
    _, (D, _) = sla.matrix_balance(np.abs(np.asarray(ABC)).sum(axis=0), permute=False, separate=True)
    return D


# ----------------------------------------------------------------------------
# corrector and step
# ----------------------------------------------------------------------------

FACES = ((0, 2, 1), (0, 1, 3), (0, 3, 2), (1, 2, 3))


def _affine(v):
    Jm = np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]], axis=1)
    return Jm, np.linalg.inv(Jm)


class Corrector:
    """The corrector of one mesh and degree: the geometry-dependent face data
    (basis at the face quadrature points in both elements, weights, upwind
    operators) evaluated once, then applied by ``step``."""

    def __init__(self, N, mesh, ABC):
        M, K, _ = basis.spatial_matrices_f64(N)
        self.N, self.mesh, self.K = N, mesh, K
        self.Md = np.diag(M)
        s, t, w = triangle_quadrature(N + 2)
        n = mesh.n
        aff = [_affine(mesh.vertices[e]) for e in range(n)]
        self.detJ = np.array([abs(np.linalg.det(a[0])) for a in aff])
        self.faces = []
        split_cache = {}
        scale_cache = {}
        for e in range(n):
            v = mesh.vertices[e]
            Ji = aff[e][1]
            akey = ABC[e].tobytes()
            if akey not in scale_cache:
                scale_cache[akey] = jacobian_scaling(ABC[e])
            D = scale_cache[akey]
            per = []
            for f, tri in enumerate(FACES):
                Pa, Pb, Pc = v[tri[0]], v[tri[1]], v[tri[2]]
                pts = Pa[None] + s[:, None] * (Pb - Pa)[None] + t[:, None] * (Pc - Pa)[None]
                cr = np.cross(Pb - Pa, Pc - Pa)
                area = 0.5 * np.linalg.norm(cr)
                nu = cr / np.linalg.norm(cr)
                if nu @ (Pa - v[6 - sum(tri)]) < 0:
                    nu = -nu
                An = nu[0] * ABC[e, 0] + nu[1] * ABC[e, 1] + nu[2] * ABC[e, 2]
                key = An.tobytes() + akey
                if key not in split_cache:
                    split_cache[key] = upwind_split(An, D)
                Ap, Am = split_cache[key]
                e2 = int(mesh.neighbor[e, f])
                v2 = mesh.vertices[e2]
                xi_own = (pts - v[0]) @ Ji.T
                xi_nb = (pts + mesh.shift[e, f][None] - v2[0]) @ aff[e2][1].T
                per.append((e2, basis_at(N, xi_own), basis_at(N, xi_nb), w * 2.0 * area, Ap, Am))
            self.faces.append(per)

    def step(self, star, E, Q, Qint):
        """Q^{n+1} [n, nq, B] from Q^n and Qint; star [n, 3, nq, nq], E [n, nq, nq]."""
        new = np.array(Q, float, copy=True)
        for e in range(Q.shape[0]):
            # volume: sum_j A^j Qint K^j_lk / M_kk  (K^j_lk = int phi_l d_j phi_k)
            vol = sum(star[e, j] @ Qint[e] @ self.K[j] for j in range(3)) / self.Md[None, :]
            src = E[e] @ Qint[e]
            flux = np.zeros_like(Q[e])
            for e2, phi_own, phi_nb, wq, Ap, Am in self.faces[e]:
                Fq = Ap @ (Qint[e] @ phi_own.T) + Am @ (Qint[e2] @ phi_nb.T)   # [nq, P]
                flux += (Fq * wq[None, :]) @ phi_own
            new[e] += vol + src - flux / (self.detJ[e] * self.Md[None, :])
        return new


def corrector(N, mesh, ABC, star, E, Q, Qint):
    """Q^{n+1} [n, nq, B] from Q^n and Qint (both [n, nq, B]); ABC [n, 3, nq, nq]
    physical Jacobians, star [n, 3, nq, nq], E [n, nq, nq]."""
    return Corrector(N, mesh, ABC).step(star, E, Q, Qint)


def ader_step(corr, star, E, Q, dt):
    """One ADER-DG step: oracle predictor on every element, then the
    corrector ``corr`` (a ``Corrector`` of the mesh)."""
    Qint = np.empty_like(Q)
    for e in range(Q.shape[0]):
        _, Qint[e] = stp.solve_element(corr.N, star[e], E[e], Q[e], dt)
    return corr.step(star, E, Q, Qint)


# ----------------------------------------------------------------------------
# plane-wave reference solution and projection
# ----------------------------------------------------------------------------

def plane_wave_modes(A, B, C, E, k):
    """(omega [nq], r [nq, nq]) eigenpairs of k_x A + k_y B + k_z C - i E,
    ordered by decreasing real part of omega (fast waves first)."""
    Mk = k[0] * A + k[1] * B + k[2] * C - 1j * E
    om, R = np.linalg.eig(Mk)
    order = np.argsort(-om.real, kind="stable")
    return om[order], R[:, order]


def plane_wave(A, B, C, E, k, alpha):
    """q(x, t) = Re sum_n alpha_n r_n exp(i (omega_n t - k . x)); alpha [nq]."""
    om, R = plane_wave_modes(A, B, C, E, k)
    k = np.asarray(k, float)
    alpha = np.asarray(alpha, complex)

    def q(x, t):
        ph = np.exp(1j * (om[None, :] * t - (x @ k)[:, None]))      # [P, nq]
        return ((ph * alpha[None, :]) @ R.T).real                   # [P, nq]
    return q


def project(N, mesh, f, t, nquad=None):
    """L2 projection of f(x, t) (x [P, 3] -> [P, nq]) on every element:
    Q_pl = int f_p phi_l / M_ll over the reference element."""
    M, _, _ = basis.spatial_matrices_f64(N)
    Md = np.diag(M)
    pts, wt = tet_quadrature(nquad or N + 4)
    phi = basis_at(N, pts)                                           # [P, B]
    v = mesh.vertices                                                # [n, 4, 3]
    Jm = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2)   # [n, 3, 3]
    x = v[:, None, 0, :] + np.einsum("nij,pj->npi", Jm, pts)         # [n, P, 3]
    fv = f(x.reshape(-1, 3), t).reshape(v.shape[0], len(wt), -1)      # [n, P, nq]
    return np.einsum("npq,p,pl->nql", fv, wt, phi) / Md[None, None, :]
