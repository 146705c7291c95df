"""Second system through the same kernels (section "Other applications"):
the damped Maxwell equations, six quantities, stiff diagonal source on the
electric field.  GPU parity against the oracle through the C ABI
(stp_predict_nq), per element and per (element, quantity), at the bar of
the poroelastic tests."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import pool as opool  # noqa: E402
from paper_2108_10565_amd import StpError, api  # noqa: E402
from paper_2108_10565_amd import workload as wl  # noqa: E402

import parity  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-10
PATHS = {
    "fp64": dict(precision="fp64"),
    "fp32_refine2": dict(precision="fp32_refine", refine_steps=2),
    "mfma_fp32_refine2": dict(precision="fp32_refine", refine_steps=2, mfma_float_chain=True),
}
_ORACLE = {}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _oracle(w, ids=None):
    ids = list(range(w.n)) if ids is None else list(ids)
    key = (w.name, tuple(ids))
    if key not in _ORACLE:
        _ORACLE[key] = opool.solve_many(w.N, w.star[ids], w.E[ids], w.Q0[ids], w.dt)
    return _ORACLE[key]


def _check(Q, Qi, Xo, Io):
    parity.check(Q, Xo, TOL, "Q", say=_say)
    parity.check(Qi, Io, TOL, "Qint", say=_say)


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("N,n", [(0, 5), (1, 7), (2, 9), (3, 40), (4, 13), (5, 11), (6, 30), (7, 5)])
def test_every_element_every_degree(path, N, n):
    """Every element against the oracle; the counts leave partial workgroups
    (6 quantities: 12 elements per 512-lane workgroup at N=6)."""
    _say(f"[gpu] maxwell path={path} N={N} n={n}")
    w = wl.make_maxwell(N, n, seed=500 + N)
    Q, Qi = api.predict(_dev(w.Q0), _dev(w.star), _dev(w.E), w.dt, N, **PATHS[path])
    torch.cuda.synchronize()
    assert Q.shape == (n, 6, wl.n_modes(N), N + 1)
    Xo, Io = _oracle(w)
    _check(Q.cpu().numpy(), Qi.cpu().numpy(), Xo, Io)


def test_stiffness_decades():
    """dt sigma / eps from 1e-2 to 1e6 at N=5: both paths within the bar in
    every decade."""
    _say("[gpu] maxwell stiffness decades N=5")
    w = wl.make_maxwell(5, 64, seed=510)
    z = w.dt * np.abs(w.E[:, 0, 0])
    dec = np.floor(np.log10(z)).astype(int)
    pick = [int(i) for d in range(-2, 6) for i in np.where(dec == d)[0][:2]]
    Xo, Io = _oracle(w, pick)
    for name in ("fp64", "fp32_refine2"):
        Q, Qi = api.predict(_dev(w.Q0), _dev(w.star), _dev(w.E), w.dt, 5, **PATHS[name])
        torch.cuda.synchronize()
        Qs = Q.cpu().numpy()[pick]
        worst = np.maximum(parity.rel_l2(Qs, Xo), parity.rel_l2_per_quantity(Qs, Xo).max(axis=1))
        per = {int(d): float(worst[dec[pick] == d].max()) for d in sorted(set(dec[pick].tolist()))}
        _say(f"  {name}: worst rel L2 per decade {per}")
        _check(Qs, Qi.cpu().numpy()[pick], Xo, Io)


def test_full_size_maxwell_n6_262144_sampled():
    """The Maxwell benchmark workload in one call, 16 oracle-checked elements."""
    _say("[gpu] full size maxwell_n6_262144")
    w = wl.make_maxwell_workload("maxwell_n6_262144")
    ids = wl.oracle_sample(w.n)
    Q, Qi = api.predict(_dev(w.Q0), _dev(w.star), _dev(w.E), w.dt, w.N)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(Q).all()) and bool(torch.isfinite(Qi).all())
    Qs, Is = Q[ids].cpu().numpy(), Qi[ids].cpu().numpy()
    del Q, Qi
    torch.cuda.empty_cache()
    Xo, Io = _oracle(w, ids)
    _check(Qs, Is, Xo, Io)


def test_validate_and_unsupported_quantity_counts():
    _say("[gpu] maxwell validate")
    w = wl.make_maxwell(3, 4, seed=520)
    api.validate(_dev(w.Q0), _dev(w.star), _dev(w.E), w.dt, 3)
    E = w.E.copy()
    E[1, 4, 2] = 1.0
    with pytest.raises(StpError, match="ENOTUPPER"):
        api.validate(_dev(w.Q0), _dev(w.star), _dev(E), w.dt, 3)
    # no kernels for 7 quantities
    Q0 = torch.zeros((2, 7, 20), dtype=torch.float64, device="cuda")
    star = torch.zeros((2, 3, 7, 7), dtype=torch.float64, device="cuda")
    E7 = torch.zeros((2, 7, 7), dtype=torch.float64, device="cuda")
    with pytest.raises(StpError, match="EINVAL"):
        api.predict(Q0, star, E7, w.dt, 3)
    # the reference kernel is for the poroelastic system only
    with pytest.raises(StpError, match="EINVAL"):
        api.predict(_dev(w.Q0), _dev(w.star), _dev(w.E), w.dt, 3, reference_kernel=True)
