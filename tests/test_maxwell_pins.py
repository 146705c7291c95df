"""Second system with a stiff source (section "Other applications"): the
damped Maxwell equations, six quantities, diagonal source -sigma/eps on the
electric field.  Pins of its input generator and of the oracle on it (CPU).
"""
import numpy as np
import pytest
from numpy.polynomial import Legendre

from oracle import basis, brute, stp
from paper_2108_10565_amd import workload as wl
from test_oracle_accuracy import BOUND, per_quantity_bound
from test_oracle_pins import _pade_endpoint


def test_jacobians_reproduce_the_curl_operator():
    """For a field linear in x, -(A q_x + B q_y + C q_z) must equal
    ((1/eps) curl H, -(1/mu) curl E), the curls taken with numpy's cross
    product of the gradient (independent of how the matrices are filled)."""
    eps, mu = 3.0, 1.7
    A, B, C, _ = wl.maxwell_jacobians(eps, mu, 0.0)
    rng = np.random.default_rng(1)
    G = rng.standard_normal((6, 3))            # G[q, k] = d q / d x_k
    rate = -(A[0] @ G[:, 0] + B[0] @ G[:, 1] + C[0] @ G[:, 2])

    def curl(Gf):                              # Gf[i, k] = d F_i / d x_k
        return np.array([Gf[2, 1] - Gf[1, 2], Gf[0, 2] - Gf[2, 0], Gf[1, 0] - Gf[0, 1]])

    np.testing.assert_allclose(rate[:3], curl(G[3:]) / eps, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(rate[3:], -curl(G[:3]) / mu, rtol=1e-14, atol=1e-15)


def test_jacobian_eigenvalues_are_the_light_speed():
    """n . (A, B, C) has eigenvalues +-1/sqrt(eps mu) (twice each) and 0
    (twice) for every unit n: two transverse polarisations.  With the sign
    printed in the paper in front of curl E the eigenvalues would be
    imaginary (not hyperbolic): that reading is excluded here."""
    rng = np.random.default_rng(2)
    for _ in range(5):
        eps, mu = rng.uniform(1, 10), rng.uniform(1, 2)
        A, B, C, _ = wl.maxwell_jacobians(eps, mu, 0.0)
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        J = n[0] * A[0] + n[1] * B[0] + n[2] * C[0]
        ev = np.linalg.eigvals(J)
        assert np.abs(ev.imag).max() <= 1e-12
        c = 1 / np.sqrt(eps * mu)
        np.testing.assert_allclose(np.sort(ev.real), [-c, -c, 0, 0, c, c], atol=1e-12)
        Jp = J.copy()
        Jp[3:] *= -1                           # mu H_t = +curl E
        assert np.abs(np.linalg.eigvals(Jp).imag).max() > 0.1 * c


def test_generator_patterns_and_stiffness_range():
    w = wl.make_maxwell(3, 200, seed=3)
    assert w.star.shape == (200, 3, 6, 6) and w.E.shape == (200, 6, 6) and w.Q0.shape == (200, 6, 20)
    assert np.all(np.tril(w.E, -1) == 0)                             # upper triangular (diagonal)
    assert np.all(w.E[:, 3:, 3:] == 0) and np.all(np.diagonal(w.E, axis1=1, axis2=2)[:, :3] < 0)
    z = w.dt * np.abs(w.E[:, 0, 0])
    assert z.min() < 0.1 and z.max() > 1e5                           # spans the stiffness decades
    # every star row couples an E component to two H components or vice versa
    nz = (np.abs(w.star).sum(axis=1) != 0)
    assert np.all(nz[:, :3, :3] == 0) and np.all(nz[:, 3:, 3:] == 0)


@pytest.mark.parametrize("N", [0, 1])
def test_assembly_matches_brute_force(N):
    w = wl.make_maxwell(N, 2, seed=4)
    Yk, rk, _ = stp.assemble(N, w.star[1], w.E[1], w.Q0[1], w.dt, equilibrate=False)
    Yb, rb = brute.assemble_brute(N, w.star[1], w.E[1], w.Q0[1], w.dt)
    assert Yk.shape == (6 * basis.n_modes(N) * (N + 1),) * 2
    assert np.abs(Yk - Yb).max() <= 1e-12 * np.abs(Yk).max()
    np.testing.assert_allclose(rk, rb, rtol=0, atol=1e-13 * np.abs(rk).max())


@pytest.mark.parametrize("N", [2, 4])
def test_source_only_is_pade_per_component(N):
    """No spatial coupling: each electric mode decays by the (N, N+1) Pade
    approximant of exp(-dt sigma/eps); the magnetic field stays constant."""
    w = wl.make_maxwell(N, 6, seed=5)
    for e in range(6):
        X, Qint = stp.solve_element(N, np.zeros((3, 6, 6)), w.E[e], w.Q0[e], w.dt)
        end = X.sum(axis=2)
        for p in range(6):
            R = _pade_endpoint(N, w.dt * w.E[e][p, p])
            np.testing.assert_allclose(end[p], R * w.Q0[e][p], rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(X[3:, :, 0], w.Q0[e][3:], rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("N", [2, 3])
def test_no_conductivity_reproduces_taylor_series(N):
    """sigma = 0: exp(-tau L) Q0 is a polynomial of degree N in tau; the
    predictor returns its Legendre coefficients exactly."""
    w = wl.make_maxwell(N, 1, seed=6)
    B, T = basis.n_modes(N), N + 1
    _, _, Kh = basis.spatial_matrices_f64(N)
    As = w.dt * w.star[0]
    L = lambda Q: sum(As[j] @ Q @ Kh[j].T for j in range(3))
    C = [w.Q0[0]]
    for k in range(1, N + 1):
        C.append(-L(C[-1]) / k)
    X, _ = stp.solve_element(N, w.star[0], np.zeros((6, 6)), w.Q0[0], w.dt)
    ref = np.zeros((6, B, T))
    for s in range(T):
        chi = Legendre.basis(s, domain=[0.0, 1.0])
        for k in range(N + 1):
            mono = np.polynomial.Polynomial([0] * k + [1])
            moment = (mono * chi.convert(kind=np.polynomial.Polynomial)).integ()
            ref[:, :, s] += (2 * s + 1) * (moment(1.0) - moment(0.0)) * C[k]
    for p in range(6):
        np.testing.assert_allclose(X[p], ref[p], rtol=0, atol=1e-11 * np.abs(ref[p]).max())


@pytest.mark.parametrize("decade", [-2, 1, 5])
def test_oracle_per_quantity_accuracy(decade):
    """A posteriori bound of the oracle's error per quantity on elements of
    stiffness dt sigma / eps near 10^decade."""
    w = wl.make_maxwell(4, 200, seed=7)
    z = w.dt * np.abs(w.E[:, 0, 0])
    e = int(np.argmin(np.abs(np.log10(z) - decade)))
    b, norms = per_quantity_bound(4, w.star[e], w.E[e], w.Q0[e], w.dt)
    print(f"maxwell z={z[e]:.1e}: per-quantity bound max {b.max():.2e}, norms {np.array2string(norms, precision=2)}")
    assert np.all(b <= BOUND), b
