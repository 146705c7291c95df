"""Seeded synthetic inputs for the element-local space-time predictor.

This module holds no arithmetic of the predictor itself.  It turns seeds
into the per-element inputs of the predictor call -- star matrices
A^1..A^3 (NOT scaled by dt), source matrix E, initial spatial DOFs Q0 --
and the global time step dt.  Both the oracle's tests and the HIP path's
tests and benchmark read their inputs from here.

Physics (Wolf et al., arXiv 2108.10565, section "Governing equations"):
* 13 quantities in the order (sxx, syy, szz, sxy, syz, sxz, u, v, w, p,
  uf, vf, wf); q_t + A q_x + B q_y + C q_z = E q.
* The paper does not print A, B, C, E.  They are derived here from the
  constitutive law and the Biot equations of motion of that section:
  rho = phi rho_F + (1-phi) rho_S, K_M = lambda_M + 2/3 mu_M,
  alpha = 1 - K_M/K_S, M = K_S / ((1 - K_M/K_S) - phi (1 - K_S/K_F)),
  m = rho_F T / phi, b = nu / kappa, D = rho m - rho_F^2.
  Reading: the Darcy equation's inertial term multiplies dv_i/dt with
  rho_F (the printed rho is read as a typo; the rho_F reading reproduces
  the fast P-wave speeds printed for the two-half-space materials, see
  tests/golden/wave_speeds.json).  Shear rows use sigma_xy = mu (v_x + u_y).
* Reference-element Jacobians ("star matrices", subsection "Spatial
  discretisation"): A^j = A dxi_j/dx + B dxi_j/dy + C dxi_j/dz for the
  affine map of the element onto {x, y, z > 0, x+y+z < 1}.
* CFL (subsection "Temporal discretisation with ADER"):
  dt <= C(N) d / v, C(N) = 0.5 / (2N+1), d = insphere diameter,
  v = largest wave speed; global time stepping takes the minimum.

Element i belongs to chunk i // CHUNK; every chunk draws from its own
numpy ``Generator(PCG64(SeedSequence([seed, chunk])))`` so any element can
be regenerated alone.
"""
from __future__ import annotations

import dataclasses
from functools import lru_cache

import numpy as np

NQ = 13
CHUNK = 4096
QUANTITIES = ("sxx", "syy", "szz", "sxy", "syz", "sxz",
              "u", "v", "w", "p", "uf", "vf", "wf")
SXX, SYY, SZZ, SXY, SYZ, SXZ, U, V, W, P, UF, VF, WF = range(13)

# homogeneous material of the N=3 parity workload (kg/m^3, Pa, m^2, Pa s)
MATERIAL_HOMOGENEOUS = dict(rho_S=2650.0, rho_F=1000.0, phi=0.2, kappa=1e-12,
                            nu=1e-3, K_S=40e9, K_F=2.2e9, lambda_M=10e9,
                            mu_M=8e9, T=2.0)


# material of the planar-wave convergence test (Table tab:material_convergence)
MATERIAL_CONVERGENCE = dict(rho_S=2.5e3, rho_F=1.04e3, phi=0.2, kappa=6e-13, nu=1e-3, K_S=4.0e10,
                            K_F=2.5e9, lambda_M=1.2e10, mu_M=1.0e10, T=3.0)


def n_modes(N: int) -> int:
    return (N + 1) * (N + 2) * (N + 3) // 6


# ----------------------------------------------------------------------------
# material -> A, B, C, E
# ----------------------------------------------------------------------------

def derived_moduli(mat):
    """Vectorised derived quantities of the constitutive law."""
    rho = mat["phi"] * mat["rho_F"] + (1 - mat["phi"]) * mat["rho_S"]
    K_M = mat["lambda_M"] + 2.0 / 3.0 * mat["mu_M"]
    alpha = 1 - K_M / mat["K_S"]
    M = mat["K_S"] / ((1 - K_M / mat["K_S"]) - mat["phi"] * (1 - mat["K_S"] / mat["K_F"]))
    m = mat["rho_F"] * mat["T"] / mat["phi"]
    D = rho * m - mat["rho_F"] ** 2
    with np.errstate(divide="ignore"):
        b = mat["nu"] / mat["kappa"]
    return dict(rho=rho, K_M=K_M, alpha=alpha, M=M, m=m, D=D, b=b)


def jacobians(mat):
    """A, B, C, E of q_t + A q_x + B q_y + C q_z = E q, shape (n, 13, 13)."""
    d = derived_moduli(mat)
    lam, mu = np.asarray(mat["lambda_M"], float), np.asarray(mat["mu_M"], float)
    n = np.broadcast(lam, d["M"]).size
    lam = np.broadcast_to(lam, (n,))
    mu = np.broadcast_to(mu, (n,))
    M, alpha, rho, m, D, b = (np.broadcast_to(d[k], (n,)) for k in
                              ("M", "alpha", "rho", "m", "D", "b"))
    rho_F = np.broadcast_to(np.asarray(mat["rho_F"], float), (n,))
    J = np.zeros((3, n, NQ, NQ))
    # cyclic relabelling x -> y -> z of the x-direction matrix
    normal = (SXX, SYY, SZZ)
    vel = (U, V, W)
    fvel = (UF, VF, WF)
    shear = {(0, 1): SXY, (1, 2): SYZ, (0, 2): SXZ}

    def sh(a, c):
        return shear[(min(a, c), max(a, c))]

    for k in range(3):
        A = J[k]
        for i in range(3):
            A[:, normal[i], vel[k]] = -(lam + (2 * mu if i == k else 0) + M * alpha ** 2)
            A[:, normal[i], fvel[k]] = -M * alpha
        for i in range(3):
            if i != k:
                A[:, sh(i, k), vel[i]] = -mu
        A[:, P, vel[k]] = M * alpha
        A[:, P, fvel[k]] = M
        # momentum: rho v_t + rho_F vf_t = div sigma ; rho_F v_t + m vf_t = -grad p - b vf
        for i in range(3):
            s_ik = normal[i] if i == k else sh(i, k)
            A[:, vel[i], s_ik] = -m / D
            A[:, fvel[i], s_ik] = rho_F / D
        A[:, vel[k], P] = -rho_F / D
        A[:, fvel[k], P] = rho / D
    E = np.zeros((n, NQ, NQ))
    for i in range(3):
        E[:, vel[i], fvel[i]] = rho_F * b / D
        E[:, fvel[i], fvel[i]] = -rho * b / D
    return J[0], J[1], J[2], E


def max_wave_speed(A):
    """Largest |eigenvalue| of the x-direction Jacobian (isotropic medium)."""
    ev = np.linalg.eigvals(np.asarray(A).reshape(-1, NQ, NQ))
    return np.abs(ev).max(axis=-1)


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

_REGULAR_TET = np.array([[1.0, 1.0, 1.0], [1.0, -1.0, -1.0],
                         [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]]) / np.sqrt(8.0)  # edge 1


def _random_rotations(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - z * w); R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w); R[:, 2, 1] = 2 * (y * z + x * w); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _edges(v):
    idx = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    return np.stack([np.linalg.norm(v[:, a] - v[:, b], axis=-1) for a, b in idx], axis=-1)


def random_tets(rng, n, edge=100.0, jitter=10.0, lo=80.0, hi=120.0):
    """Regular tetrahedra of edge ``edge``, randomly rotated, vertices jittered
    by U[-jitter, jitter]^3; redrawn until every edge lies in [lo, hi] and the
    orientation is positive."""
    out = np.empty((n, 4, 3))
    todo = np.arange(n)
    while todo.size:
        m = todo.size
        R = _random_rotations(rng, m)
        v = np.einsum("nij,kj->nki", R, _REGULAR_TET * edge)
        v = v + rng.uniform(-jitter, jitter, size=(m, 4, 3))
        e = _edges(v)
        J = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=-1)
        det = np.linalg.det(J)
        ok = (e.min(axis=1) >= lo) & (e.max(axis=1) <= hi)
        # keep positively oriented: swap two vertices otherwise (edges unchanged)
        neg = det < 0
        v[neg, 1], v[neg, 2] = v[neg, 2].copy(), v[neg, 1].copy()
        out[todo[ok]] = v[ok]
        todo = todo[~ok]
    return out


def insphere_diameter(v):
    J = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=-1)
    vol = np.abs(np.linalg.det(J)) / 6.0
    faces = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]
    area = sum(0.5 * np.linalg.norm(np.cross(v[:, b] - v[:, a], v[:, c] - v[:, a]), axis=-1)
               for a, b, c in faces)
    return 2.0 * 3.0 * vol / area


def star_matrices(A, B, C, v):
    """(n, 3, 13, 13): A^j = A dxi_j/dx + B dxi_j/dy + C dxi_j/dz, where
    xi = Jmap^{-1} (x - v0) and Jmap has columns v1-v0, v2-v0, v3-v0."""
    J = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=-1)
    G = np.linalg.inv(J)  # G[n, j, i] = dxi_j / dx_i
    return (G[:, :, 0, None, None] * A[:, None] + G[:, :, 1, None, None] * B[:, None]
            + G[:, :, 2, None, None] * C[:, None])


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    N: int
    n: int
    dt: float
    star: np.ndarray   # (n, 3, 13, 13) float64, not scaled by dt
    E: np.ndarray      # (n, 13, 13) float64, upper triangular, not scaled by dt
    Q0: np.ndarray     # (n, 13, B) float64
    meta: dict


def _materials(kind, rng, n):
    base = MATERIAL_HOMOGENEOUS
    mat = {k: np.full(n, v) for k, v in base.items()}
    if kind == "homogeneous":
        return mat
    # heterogeneous: kappa log-uniform [1e-14, 1e-11], phi U[0.1, 0.3],
    # K_S, K_F, lambda_M, mu_M each scaled by U[0.7, 1.3]; redraw invalid ones
    todo = np.arange(n)
    while todo.size:
        m = todo.size
        mat["kappa"][todo] = 10.0 ** rng.uniform(-14, -11, m)
        mat["phi"][todo] = rng.uniform(0.1, 0.3, m)
        for k in ("K_S", "K_F", "lambda_M", "mu_M"):
            mat[k][todo] = base[k] * rng.uniform(0.7, 1.3, m)
        sub = {k: v[todo] for k, v in mat.items()}
        d = derived_moduli(sub)
        bad = (d["M"] <= 0) | (d["K_M"] >= sub["K_S"]) | (d["D"] <= 0)
        todo = todo[bad]
    return mat


def _chunk(seed, c, kind, N, count, dt=None):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, c])))
    mat = _materials("homogeneous" if kind == "homogeneous" else "heterogeneous", rng, count)
    A, B, C, E = jacobians(mat)
    v = random_tets(rng, count)
    star = star_matrices(A, B, C, v)
    Q0 = rng.standard_normal((count, NQ, n_modes(N)))
    cfl = insphere_diameter(v) / max_wave_speed(A)
    if kind == "stiffness" and dt is not None:
        # stiffness sweep: target z = dt |E_uf,uf| log-uniform in [1e-2, 1e6]
        # and viscosity log-uniform in [1e-3, 1e-1]; the permeability follows
        # from |E_uf,uf| = rho nu / (kappa D).  Wave speeds (and so dt) do not
        # depend on kappa or nu.
        r2 = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, c, 1])))
        z = 10.0 ** r2.uniform(-2.0, 6.0, count)
        nu = 10.0 ** r2.uniform(-3.0, -1.0, count)
        d = derived_moduli(mat)
        mat["nu"] = nu
        mat["kappa"] = d["rho"] * nu * dt / (d["D"] * z)
        A, B, C, E = jacobians(mat)
        star = star_matrices(A, B, C, v)
        mat["target_z"] = z
    return dict(mat=mat, star=star, E=E, Q0=Q0, cfl=cfl)


def _generate(name, seed, kind, N, n, elements=None):
    """Generate the whole workload (needed for the global dt); if ``elements``
    is given, return only those elements' inputs."""
    nchunks = (n + CHUNK - 1) // CHUNK
    want = None if elements is None else np.asarray(elements)
    dt_pre = None
    if kind == "stiffness":
        # first pass: the global time step from the CFL condition
        cmin = min(float(_chunk(seed, c, kind, N, min(CHUNK, n - c * CHUNK))["cfl"].min())
                   for c in range(nchunks))
        dt_pre = 0.5 / (2 * N + 1) * cmin
    parts, cfl_min = [], np.inf
    for c in range(nchunks):
        count = min(CHUNK, n - c * CHUNK)
        ch = _chunk(seed, c, kind, N, count, dt=dt_pre)
        cfl_min = min(cfl_min, float(ch["cfl"].min()))
        if want is None:
            parts.append(ch)
        else:
            sel = want[(want >= c * CHUNK) & (want < c * CHUNK + count)] - c * CHUNK
            if sel.size:
                parts.append({k: (v[sel] if not isinstance(v, dict) else
                                  {kk: vv[sel] for kk, vv in v.items()})
                              for k, v in ch.items()})
    dt = 0.5 / (2 * N + 1) * cfl_min
    cat = lambda key: np.concatenate([p[key] for p in parts]) if parts else None
    mats = {k: np.concatenate([p["mat"][k] for p in parts]) for k in parts[0]["mat"]} if parts else {}
    return Workload(name=name, N=N, n=n if want is None else len(want), dt=dt,
                    star=np.ascontiguousarray(cat("star")), E=np.ascontiguousarray(cat("E")),
                    Q0=np.ascontiguousarray(cat("Q0")),
                    meta=dict(seed=seed, kind=kind, n_total=n, materials=mats,
                              elements=None if want is None else want.tolist()))


# Named workloads.  Sizes and distributions follow the parity / benchmark plan.
CONFIGS = {
    # FP64, N=3, 64 elements, homogeneous medium
    "n3_homogeneous_64": dict(seed=1, kind="homogeneous", N=3, n=64),
    # FP64, N=6, 262,144 elements, heterogeneous materials
    "n6_heterogeneous_262144": dict(seed=2, kind="heterogeneous", N=6, n=262144),
    # FP32 chain + refinement, N=6, 1,048,576 elements, heterogeneous
    "n6_heterogeneous_1048576": dict(seed=3, kind="heterogeneous", N=6, n=1048576),
    # stiffness sweep, N=5, 524,288 elements: dt |E_uf,uf| from 1e-2 to 1e6
    "n5_stiffness_524288": dict(seed=5, kind="stiffness", N=5, n=524288),
}


def make_workload(name, elements=None):
    cfg = CONFIGS[name]
    return _generate(name, cfg["seed"], cfg["kind"], cfg["N"], cfg["n"], elements)


# Clustered local time stepping: shares of the elements per cluster (cluster k
# steps with dt_k = rate^k dt_0) and the polynomial degrees mixed in each.
LTS_SHARES = (0.60, 0.25, 0.10, 0.05)
LTS_DEGREES = (3, 4, 5, 6)
LTS_CONFIGS = {
    # 1,048,576 elements in 4 rate-2 clusters x degrees 3..6 (16 batches)
    "lts_mixed_1048576": dict(seed=4, n=1048576, rate=2),
}


def make_lts(n_total, seed=4, rate=2, shares=LTS_SHARES, degrees=LTS_DEGREES, name="lts"):
    """Synthetic clustered-LTS workload: a list of batches (Workload objects
    with ``meta["cluster"]``), one per (cluster k, degree N).

    Cluster k holds ``shares[k]`` of the elements, split evenly over
    ``degrees``; each batch is a heterogeneous workload of its own seed whose
    elements are ``rate**k`` times larger (the star matrices, which carry
    the inverse element size, are scaled by ``rate**-k``).  The time step of
    cluster k is ``rate**k * dt_0``, with dt_0 the global (most restrictive)
    step of the CFL condition at the highest degree over all elements before
    scaling -- so every batch satisfies its CFL condition."""
    raw, cfl_min = [], np.inf
    sizes = [int(round(n_total * sh)) for sh in shares]
    sizes[0] = n_total - sum(sizes[1:])          # the smallest-step cluster takes the rounding
    for k, nk in enumerate(sizes):
        per = [nk // len(degrees) + (1 if i < nk % len(degrees) else 0) for i in range(len(degrees))]
        for i, N in enumerate(degrees):
            if per[i] == 0:
                continue
            w = _generate(f"{name}_k{k}_N{N}", seed * 1000 + 10 * k + i, "heterogeneous", N, per[i])
            cfl_min = min(cfl_min, w.dt * (2 * N + 1) / 0.5)
            raw.append((k, w))
    dt0 = 0.5 / (2 * max(degrees) + 1) * cfl_min
    out = []
    for k, w in raw:
        meta = dict(w.meta, cluster=k, rate=rate)
        out.append(Workload(name=w.name, N=w.N, n=w.n, dt=dt0 * rate ** k,
                            star=np.ascontiguousarray(w.star * float(rate) ** -k), E=w.E, Q0=w.Q0, meta=meta))
    return out


def make_lts_workload(name):
    cfg = LTS_CONFIGS[name]
    return make_lts(cfg["n"], seed=cfg["seed"], rate=cfg["rate"], name=name)


def lts_cycle(batches):
    """Indices of ``batches`` in the order of one cycle of the largest time
    step: sub-steps s = 0 .. rate^(K-1) - 1 of dt_0; cluster k is predicted
    at the start of each of its steps (s a multiple of rate^k), so
    rate^(K-1-k) times per cycle."""
    if not batches:
        return []
    rate = batches[0].meta["rate"]
    K = 1 + max(b.meta["cluster"] for b in batches)
    return [i for s in range(rate ** (K - 1)) for i, b in enumerate(batches)
            if s % rate ** b.meta["cluster"] == 0]


def lts_stages(batches):
    """The cycle of ``lts_cycle`` split by sub-step: a list of lists of batch
    indices; the batches of one sub-step are independent of each other."""
    if not batches:
        return []
    rate = batches[0].meta["rate"]
    K = 1 + max(b.meta["cluster"] for b in batches)
    return [[i for i, b in enumerate(batches) if s % rate ** b.meta["cluster"] == 0]
            for s in range(rate ** (K - 1))]


# ----------------------------------------------------------------------------
# a second system with a stiff source: damped Maxwell equations
# ----------------------------------------------------------------------------
#
# Section "Other applications": eps E_t = curl H - sigma E + j and
# mu H_t = -curl E (Faraday's law; the sign printed there in front of curl E
# is read as a typo, since with it the Jacobians have imaginary eigenvalues
# and the system is not hyperbolic).  Quantities (Ex, Ey, Ez, Hx, Hy, Hz);
# with curl expanded, q_t + A q_x + B q_y + C q_z = Es q with the diagonal
# (hence upper triangular) source Es = diag(-sigma/eps x 3, 0 x 3); the
# current density j is an external source and not part of the predictor.
# Non-dimensional units: edge length ~1, relative eps and mu.

MAXWELL_QUANTITIES = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")
EX, EY, EZ, HX, HY, HZ = range(6)


def maxwell_jacobians(eps, mu, sigma):
    """A, B, C, Es of the damped Maxwell system, shape (n, 6, 6)."""
    eps, mu, sigma = (np.atleast_1d(np.asarray(v, float)) for v in (eps, mu, sigma))
    n = np.broadcast(eps, mu, sigma).size
    eps, mu, sigma = (np.broadcast_to(v, (n,)) for v in (eps, mu, sigma))
    J = np.zeros((3, n, 6, 6))
    # E_t - (1/eps) curl H = -(sigma/eps) E, curl H = (dy Hz - dz Hy, dz Hx - dx Hz, dx Hy - dy Hx)
    # H_t + (1/mu) curl E = 0,             curl E = (dy Ez - dz Ey, dz Ex - dx Ez, dx Ey - dy Ex)
    for k in range(3):                       # direction x_k
        i1, i2 = (k + 1) % 3, (k + 2) % 3    # cyclic pair: curl_i1 has +d_k of component i2
        J[k][:, EX + i1, HX + i2] = 1.0 / eps
        J[k][:, EX + i2, HX + i1] = -1.0 / eps
        J[k][:, HX + i1, EX + i2] = -1.0 / mu
        J[k][:, HX + i2, EX + i1] = 1.0 / mu
    Es = np.zeros((n, 6, 6))
    for i in range(3):
        Es[:, EX + i, EX + i] = -sigma / eps
    return J[0], J[1], J[2], Es


def make_maxwell(N, n, seed=0, name=None, zmin=-2.0, zmax=6.0):
    """Seeded damped-Maxwell workload: tetrahedra of edge ~1 (regular,
    rotated, vertices jittered by U[-0.1, 0.1]^3, edges in [0.8, 1.2]),
    eps ~ U[1, 10], mu ~ U[1, 2], and sigma chosen per element so that the
    stiffness dt sigma / eps is log-uniform in [10^zmin, 10^zmax]; global
    time step from the CFL condition with the light speed 1/sqrt(eps mu).
    Q0 ~ N(0, 1).  Returns a Workload with six quantities."""
    nchunks = (n + CHUNK - 1) // CHUNK
    parts, cfl_min = [], np.inf
    for c in range(nchunks):
        count = min(CHUNK, n - c * CHUNK)
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, c, 77])))
        eps = rng.uniform(1.0, 10.0, count)
        mu = rng.uniform(1.0, 2.0, count)
        v = random_tets(rng, count, edge=1.0, jitter=0.1, lo=0.8, hi=1.2)
        cfl = insphere_diameter(v) * np.sqrt(eps * mu)
        z = 10.0 ** rng.uniform(zmin, zmax, count)
        Q0 = rng.standard_normal((count, 6, n_modes(N)))
        parts.append(dict(eps=eps, mu=mu, v=v, z=z, Q0=Q0))
        cfl_min = min(cfl_min, float(cfl.min()))
    dt = 0.5 / (2 * N + 1) * cfl_min
    stars, Es, Q0s, mats = [], [], [], {"eps": [], "mu": [], "sigma": []}
    for p in parts:
        sigma = p["z"] * p["eps"] / dt
        A, B, C, Esrc = maxwell_jacobians(p["eps"], p["mu"], sigma)
        stars.append(star_matrices(A, B, C, p["v"]))
        Es.append(Esrc)
        Q0s.append(p["Q0"])
        for k, val in (("eps", p["eps"]), ("mu", p["mu"]), ("sigma", sigma)):
            mats[k].append(val)
    mats = {k: np.concatenate(v) for k, v in mats.items()}
    return Workload(name=name or f"maxwell_N{N}_n{n}_s{seed}", N=N, n=n, dt=dt,
                    star=np.ascontiguousarray(np.concatenate(stars)), E=np.ascontiguousarray(np.concatenate(Es)),
                    Q0=np.ascontiguousarray(np.concatenate(Q0s)),
                    meta=dict(seed=seed, kind="maxwell", n_total=n, materials=mats, quantities=MAXWELL_QUANTITIES))


MAXWELL_CONFIGS = {
    # damped Maxwell, N=6, 262,144 elements, dt sigma / eps from 1e-2 to 1e6
    "maxwell_n6_262144": dict(seed=6, N=6, n=262144),
}


def make_maxwell_workload(name):
    cfg = MAXWELL_CONFIGS[name]
    return make_maxwell(cfg["N"], cfg["n"], seed=cfg["seed"], name=name)


def stiffness(w: "Workload") -> np.ndarray:
    """dt |E_uf,uf| of every element of a workload."""
    return w.dt * np.abs(w.E[:, UF, UF])


def make_small(N, n, seed=0, kind="heterogeneous"):
    """Small ad-hoc workload (tests): same distributions, own seed."""
    return _generate(f"small_N{N}_n{n}_s{seed}", seed, kind, N, n)


def oracle_sample(n_total, count=16):
    """Element ids checked against the oracle at full size: the first element
    of ``count`` evenly spaced chunks (or evenly spaced ids if few chunks)."""
    nchunks = (n_total + CHUNK - 1) // CHUNK
    if nchunks >= count:
        cs = np.linspace(0, nchunks - 1, count).round().astype(int)
        return (cs * CHUNK).tolist()
    return np.linspace(0, n_total - 1, min(count, n_total)).round().astype(int).tolist()
