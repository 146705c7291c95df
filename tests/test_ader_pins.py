"""Corrector of one ADER-DG step (section "ADER-DG discretisation") and the
plane-wave reference solution (section "Planar wave convergence
analysis"): pins of the CPU oracle ``oracle.ader`` and of the library's host
tables against it (CPU)."""
import numpy as np
import pytest

from oracle import ader, basis
from paper_2108_10565_amd import api
from paper_2108_10565_amd import mesh as pmesh
from paper_2108_10565_amd import workload as wl

MAT = {k: np.array([v]) for k, v in wl.MATERIAL_CONVERGENCE.items()}
A, B, C, E = wl.jacobians(MAT)
ABC1 = np.stack([A[0], B[0], C[0]])
NORMALS = [np.array(v, float) / np.linalg.norm(v) for v in
           ([1, 0, 0], [0, 0, -1], [0, 1, 0], [-1, 1, 1], [1, 2, 3], [0.3, -0.2, 0.9])]


def _setup(m, N, hetero=False, seed=0):
    M = pmesh.periodic_cube(m)
    n = M.n
    if hetero:
        w = wl.make_small(N, n, seed=seed)
        mats = {k: v for k, v in w.meta["materials"].items()}
        Aa, Bb, Cc, Ee = wl.jacobians(mats)
    else:
        Aa, Bb, Cc, Ee = (np.broadcast_to(X, (n, 13, 13)).copy() for X in (A, B, C, E))
    ABC = np.stack([Aa, Bb, Cc], axis=1)
    star = wl.star_matrices(Aa, Bb, Cc, M.vertices)
    return M, ABC, star, Ee


def _balanced(X, D):
    return X / D[:, None] * D[None, :]


@pytest.mark.parametrize("nu", NORMALS, ids=lambda v: ",".join(f"{x:.2f}" for x in v))
def test_upwind_split_is_the_spectral_split(nu):
    """An^+ + An^- = An, An^+ An^- = 0, and An^+ has the eigenvalues
    max(lambda, 0) of An (in the element's balanced scaling)."""
    An = np.einsum("d,dij->ij", nu, ABC1)
    D = ader.jacobian_scaling(ABC1)
    Ap, Am = ader.upwind_split(An, D)
    Ab, Apb, Amb = (_balanced(X, D) for X in (An, Ap, Am))
    s = np.abs(Ab).max()
    assert np.abs(Apb + Amb - Ab).max() <= 1e-13 * s
    assert np.abs(Apb @ Amb).max() <= 1e-13 * s * s
    lam = np.sort(np.linalg.eigvals(Ab).real)
    lp = np.sort(np.linalg.eigvals(Apb).real)
    np.testing.assert_allclose(lp, np.sort(np.maximum(lam, 0)), atol=1e-10 * s)


@pytest.mark.parametrize("nu", NORMALS, ids=lambda v: ",".join(f"{x:.2f}" for x in v))
def test_library_upwind_split_matches_oracle(nu):
    """stp_upwind_split (balanced Hessenberg QR + Lagrange projectors) against
    the oracle's null-space projectors."""
    An = np.einsum("d,dij->ij", nu, ABC1)
    D = ader.jacobian_scaling(ABC1)
    Ap, _ = ader.upwind_split(An, D)
    lp, lm = api.upwind_split(An)
    s = np.abs(_balanced(An, D)).max()
    assert np.abs(_balanced(lp - Ap, D)).max() <= 1e-12 * s
    assert np.array_equal(lp + lm, An) or np.abs(_balanced(lp + lm - An, D)).max() <= 1e-13 * s


@pytest.mark.parametrize("N", [1, 3])
def test_library_corrector_tables_match_oracle_integrals(N):
    """V, Fl and Fn of stp_corrector_tables against the oracle's exact
    stiffness matrices and its own quadrature of the face integrals."""
    Bn = basis.n_modes(N)
    tab = api.corrector_tables(N)
    BB = Bn * Bn
    V = tab[:3 * BB].reshape(3, Bn, Bn)
    Fl = tab[3 * BB:7 * BB].reshape(4, Bn, Bn)
    Fn = tab[7 * BB:].reshape(4, 4, 6, Bn, Bn)
    M, K, _ = basis.spatial_matrices_f64(N)
    Md = np.diag(M)
    tol = 1e-12 * np.abs(tab).max()
    np.testing.assert_allclose(V, K / Md[None, None, :], rtol=0, atol=tol)
    s, t, w = ader.triangle_quadrature(N + 3)
    Vref = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]

    def face_pts(f, s_, t_):
        a, b, c = ader.FACES[f]
        return Vref[a] + s_[:, None] * (Vref[b] - Vref[a]) + t_[:, None] * (Vref[c] - Vref[a])

    for i in range(4):
        phi_i = ader.basis_at(N, face_pts(i, s, t))
        np.testing.assert_allclose(Fl[i], (phi_i * w[:, None]).T @ phi_i / Md[None, :], rtol=0, atol=tol)
        wts = np.stack([1 - s - t, s, t], axis=1)
        for j in range(4):
            for h, pm in enumerate(perms):
                wn = np.empty_like(wts)
                wn[:, list(pm)] = wts
                phi_j = ader.basis_at(N, face_pts(j, wn[:, 1], wn[:, 2]))
                ref = (phi_j * w[:, None]).T @ phi_i / Md[None, :]
                np.testing.assert_allclose(Fn[i, j, h], ref, rtol=0, atol=tol)


def test_constant_state_is_steady():
    """E = 0 and a constant state: the Godunov fluxes balance the volume term
    exactly (divergence theorem), Q does not change."""
    M, ABC, star, Ee = _setup(4, 2)
    corr = ader.Corrector(2, M, ABC)
    Q = np.zeros((M.n, 13, basis.n_modes(2)))
    Q[:, :, 0] = np.arange(1, 14)[None, :]
    Qint = 1e-5 * Q
    new = corr.step(star, 0 * Ee, Q, Qint)
    vol = max(np.abs(sum(star[e, j] @ Qint[e] @ corr.K[j] for j in range(3)) / corr.Md).max() for e in range(4))
    assert np.abs(new - Q).max() <= 1e-13 * vol


def test_each_quantity_is_conserved_without_source():
    """Periodic mesh of one material, E = 0: the fluxes of two elements
    across their shared face cancel, so sum_e |J_e| Q_e,p0 (the integral of
    each quantity) is unchanged by a step, for any Q and Qint.  (Across a
    material interface the flux of each side uses its own Jacobians, so only
    a single material telescopes.)"""
    M, ABC, star, Ee = _setup(4, 2)
    corr = ader.Corrector(2, M, ABC)
    rng = np.random.default_rng(1)
    Q = rng.standard_normal((M.n, 13, basis.n_modes(2)))
    Qint = 1e-5 * rng.standard_normal(Q.shape)
    new = corr.step(star, 0 * Ee, Q, Qint)
    total = lambda X: (corr.detJ[:, None] * X[:, :, 0]).sum(axis=0)
    change = np.abs(new - Q)[:, :, 0].max(axis=0)
    assert np.all(np.abs(total(new) - total(Q)) <= 1e-12 * change * M.n)


def test_plane_wave_solves_the_pde():
    """q = Re sum alpha r exp(i (omega t - k.x)) satisfies q_t + A q_x + B q_y
    + C q_z = E q (fourth-order central differences; the eigenpairs of
    k.A - i E)."""
    k = np.pi * np.ones(3)
    alpha = np.zeros(13, complex); alpha[:4] = 100.0
    om, R = ader.plane_wave_modes(A[0], B[0], C[0], E[0], k)
    q = ader.plane_wave(A[0], B[0], C[0], E[0], k, alpha)
    x0 = np.array([[0.1, -0.2, 0.35]])
    d4 = lambda f, h: (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)   # 4th-order central
    qt = d4(lambda s: q(x0, s), 1e-7)
    grad = [d4(lambda s: q(x0 + s * np.eye(3)[d], 0.0), 1e-4) for d in range(3)]
    res = qt[0] + A[0] @ grad[0][0] + B[0] @ grad[1][0] + C[0] @ grad[2][0] - E[0] @ q(x0, 0)[0]
    scale = np.abs(A[0]).max(axis=1) * np.abs(q(x0, 0)[0]).max() * np.linalg.norm(k) + np.abs(qt[0])
    assert np.all(np.abs(res) <= 1e-8 * scale)
    # modes 1..4: fast P, two S polarisations, slow P (diffusive in this regime)
    assert om[0].real > om[1].real > 0 and om[1].real == pytest.approx(om[2].real, rel=1e-12)


def test_semi_discrete_operator_converges():
    """For a vanishing step the corrector is Q + dt L(Q) with Qint = dt Q:
    L applied to the projected plane wave approaches the projection of q_t
    as the mesh is refined, at order N (N = 2, meshes of 6^3 and 8^3
    sub-cubes)."""
    k = np.pi * np.ones(3)
    alpha = np.zeros(13, complex); alpha[:4] = 100.0
    om, R = ader.plane_wave_modes(A[0], B[0], C[0], E[0], k)
    q = ader.plane_wave(A[0], B[0], C[0], E[0], k, alpha)

    def qt(x, t):
        ph = np.exp(1j * (om[None, :] * t - (x @ k)[:, None]))
        return ((ph * (1j * om * alpha)[None, :]) @ R.T).real

    errs = []
    for m in (6, 8):
        M, ABC, star, Ee = _setup(m, 2)
        corr = ader.Corrector(2, M, ABC)
        Q0 = ader.project(2, M, q, 0.0)
        dt = 1e-10
        rate = (corr.step(star, Ee, Q0, dt * Q0) - Q0) / dt
        ref = ader.project(2, M, qt, 0.0)
        w = corr.detJ[:, None, None] * corr.Md[None, None, :]
        errs.append(np.sqrt((w * (rate - ref) ** 2).sum(axis=(0, 2)) / (w * ref ** 2).sum(axis=(0, 2))))
    order = np.log(errs[0] / errs[1]) / np.log(8 / 6)
    print("errors", errs, "orders", order)
    assert np.all(order >= 1.7) and np.all(errs[1] < errs[0])
