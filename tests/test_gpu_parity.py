"""Parity of the HIP path (through the C ABI) against the CPU oracle.

Bar: relative L2 error <= 1e-10 per element over all 13*B*T space-time DOFs
in physical units AND per (element, quantity) over that quantity's B*T DOFs
(float64 path, and the float32 chain after refinement); Qint likewise.  Inputs are seeded synthetic workloads from
``paper_2108_10565_amd.workload``; expected values come only from ``oracle``.
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import pool as opool  # noqa: E402
from oracle import stp as ostp  # noqa: E402
from paper_2108_10565_amd import api  # noqa: E402
from paper_2108_10565_amd import workload as wl  # noqa: E402

import parity  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-10

KERNELS = {
    "reference": dict(reference_kernel=True),
    "fused_fp64": dict(precision="fp64"),
    "fused_fp32_refine2": dict(precision="fp32_refine", refine_steps=2),
    "mfma_fp32_refine2": dict(precision="fp32_refine", refine_steps=2, mfma_float_chain=True),
}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(w, elements=None, **kw):
    sl = slice(None) if elements is None else elements
    Q, Qi = api.predict(_dev(w.Q0[sl]), _dev(w.star[sl]), _dev(w.E[sl]), w.dt, w.N, **kw)
    torch.cuda.synchronize()
    return Q.cpu().numpy(), Qi.cpu().numpy()


rel_l2 = parity.rel_l2


def _check(Q, Qi, Xo, Io, tol=TOL, label=""):
    parity.check(Q, Xo, tol, f"{label} Q".strip(), say=_say)
    if Qi is not None:
        parity.check(Qi, Io, tol, f"{label} Qint".strip(), say=_say)


_ORACLE_CACHE = {}


def _oracle(w, idx):
    key = (w.name, tuple(idx))
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = opool.solve_many(w.N, w.star[idx], w.E[idx], w.Q0[idx], w.dt)
    return _ORACLE_CACHE[key]


@pytest.fixture(scope="module")
def cfg1():
    return wl.make_workload("n3_homogeneous_64")


@pytest.mark.parametrize("kernel", list(KERNELS))
def test_n3_homogeneous_all_64(cfg1, kernel):
    _say(f"[gpu] n3_homogeneous_64 kernel={kernel}")
    Q, Qi = _run(cfg1, **KERNELS[kernel])
    idx = list(range(64))
    Xo, Io = _oracle(cfg1, idx)
    _check(Q, Qi, Xo, Io)


@pytest.mark.parametrize("kernel", list(KERNELS))
@pytest.mark.parametrize("N,n", [(0, 5), (1, 3), (2, 7), (4, 5), (5, 4), (6, 5), (7, 2)])
def test_degrees_ragged(kernel, N, n):
    """Every supported degree, element counts that leave ragged tails."""
    _say(f"[gpu] degrees_ragged kernel={kernel} N={N} n={n}")
    w = wl.make_small(N, n, seed=100 + N)
    Q, Qi = _run(w, **KERNELS[kernel])
    Xo, Io = _oracle(w, list(range(n)))
    _check(Q, Qi, Xo, Io)


@pytest.mark.parametrize("kernel", ["fused_fp64", "fused_fp32_refine2", "mfma_fp32_refine2"])
@pytest.mark.parametrize("N,n", [(3, 10), (4, 16), (6, 11)])
def test_several_groups_with_ragged_tail(kernel, N, n):
    """Every element against the oracle where the fused kernel's workgroups
    (4 elements at N=3, 7 at N=4, 5 at N=6) come out as two full groups and a
    partial one, so the tail group's spare slots and the group offsets are
    exercised together."""
    _say(f"[gpu] several_groups_with_ragged_tail kernel={kernel} N={N} n={n}")
    w = wl.make_small(N, n, seed=200 + N)
    Q, Qi = _run(w, **KERNELS[kernel])
    Xo, Io = _oracle(w, list(range(n)))
    _check(Q, Qi, Xo, Io)


@pytest.mark.parametrize("kernel", ["reference", "fused_fp64"])
def test_special_operators(kernel):
    """E = 0 (no source), A = 0 with a stiff source, and all operators zero,
    mixed in one batch with ordinary elements."""
    _say(f"[gpu] special_operators kernel={kernel}")
    N = 4
    w = wl.make_small(N, 6, seed=7)
    star, E = w.star.copy(), w.E.copy()
    E[1] = 0.0
    star[2] = 0.0
    E[2] *= 1e4                     # dt*E_pp ~ -1e6
    star[3] = 0.0; E[3] = 0.0
    Q, Qi = api.predict(_dev(w.Q0), _dev(star), _dev(E), w.dt, N, **KERNELS[kernel])
    torch.cuda.synchronize()
    Xo, Io = opool.solve_many(N, star, E, w.Q0, w.dt)
    _check(Q.cpu().numpy(), Qi.cpu().numpy(), Xo, Io)
    # all-zero operators: constant in time
    np.testing.assert_allclose(Q.cpu().numpy()[3][:, :, 0], w.Q0[3], rtol=0, atol=1e-15)


@pytest.mark.parametrize("kernel", ["reference", "fused_fp64"])
def test_empty_and_no_qint(kernel):
    _say(f"[gpu] empty_and_no_qint kernel={kernel}")
    w = wl.make_small(3, 2, seed=8)
    e = torch.empty((0, 13, 20), dtype=torch.float64, device="cuda")
    Q, Qi = api.predict(e, torch.empty((0, 3, 13, 13), dtype=torch.float64, device="cuda"),
                        torch.empty((0, 13, 13), dtype=torch.float64, device="cuda"), w.dt, 3,
                        **KERNELS[kernel])
    assert Q.shape == (0, 13, 20, 4)
    Q, Qi = api.predict(_dev(w.Q0), _dev(w.star), _dev(w.E), w.dt, 3, with_qint=False,
                        **KERNELS[kernel])
    torch.cuda.synchronize()
    assert Qi is None
    Xo, Io = _oracle(w, [0, 1])
    _check(Q.cpu().numpy(), None, Xo, Io)


@pytest.mark.parametrize("kernel", ["reference", "fused_fp64", "fused_fp32_refine2", "mfma_fp32_refine2"])
def test_deterministic(kernel):
    _say(f"[gpu] deterministic kernel={kernel}")
    w = wl.make_small(6, 9, seed=9)
    Q1, I1 = _run(w, **KERNELS[kernel])
    Q2, I2 = _run(w, **KERNELS[kernel])
    assert np.array_equal(Q1, Q2) and np.array_equal(I1, I2)


def test_validate_reports_bad_inputs():
    _say("[gpu] validate")
    from paper_2108_10565_amd import StpError
    w = wl.make_small(3, 4, seed=10)
    api.validate(_dev(w.Q0), _dev(w.star), _dev(w.E), w.dt, 3)
    E = w.E.copy(); E[2, 5, 1] = 1.0
    with pytest.raises(StpError, match="ENOTUPPER"):
        api.validate(_dev(w.Q0), _dev(w.star), _dev(E), w.dt, 3)
    Q0 = w.Q0.copy(); Q0[1, 3, 2] = np.nan
    with pytest.raises(StpError, match="ENONFINITE"):
        api.validate(_dev(Q0), _dev(w.star), _dev(w.E), w.dt, 3)
    E = w.E.copy(); E[0, 4, 4] = 10.0 / w.dt
    with pytest.raises(StpError, match="ESINGULAR"):
        api.validate(_dev(w.Q0), _dev(w.star), _dev(E), w.dt, 3)


@pytest.mark.parametrize("kernel", ["reference", "fused_fp64", "fused_fp32_refine2"])
def test_predict_reports_unfit_inputs(kernel):
    """The prediction kernels report what their elimination without pivoting
    cannot take (dt E_pp >= 0.5) and an E with a non-zero below its diagonal
    through stp_check_inputs; fit inputs report nothing, and taking the
    report clears it."""
    _say(f"[gpu] input report kernel={kernel}")
    from paper_2108_10565_amd import StpError
    w = wl.make_small(3, 4, seed=12)
    try:
        api.check_inputs()  # take whatever an earlier call left
    except StpError:
        pass
    _run(w, **KERNELS[kernel])
    api.check_inputs()
    E = w.E.copy(); E[1, 11, 11] = 0.6 / w.dt
    api.predict(_dev(w.Q0), _dev(w.star), _dev(E), w.dt, 3, **KERNELS[kernel])
    with pytest.raises(StpError, match="ESINGULAR"):
        api.check_inputs()
    api.check_inputs()
    E = w.E.copy(); E[2, 5, 1] = 1.0
    api.predict(_dev(w.Q0), _dev(w.star), _dev(E), w.dt, 3, **KERNELS[kernel])
    with pytest.raises(StpError, match="ENOTUPPER"):
        api.check_inputs()
    _run(w, **KERNELS[kernel])
    api.check_inputs()


def test_caller_workspace_is_used_as_is():
    """predict() with the caller's workspace gives bitwise the results of a
    call that allocates its own."""
    _say("[gpu] caller workspace")
    w = wl.make_small(6, 7, seed=13)
    Q1, I1 = _run(w, **KERNELS["fused_fp32_refine2"])
    ws = api.workspace_size(6, w.n, "fp32_refine", 2)
    work = torch.full((ws + 64,), 255, dtype=torch.uint8, device="cuda")
    Q, Qi = api.predict(_dev(w.Q0), _dev(w.star), _dev(w.E), w.dt, 6, workspace=work, **KERNELS["fused_fp32_refine2"])
    torch.cuda.synchronize()
    assert np.array_equal(Q.cpu().numpy(), Q1) and np.array_equal(Qi.cpu().numpy(), I1)
    from paper_2108_10565_amd import StpError
    with pytest.raises(StpError, match="EWORKSPACE"):
        api.predict(_dev(w.Q0), _dev(w.star), _dev(w.E), w.dt, 6, workspace=work[:ws - 8],
                    **KERNELS["fused_fp32_refine2"])


def test_kernels_agree_with_each_other():
    _say("[gpu] kernels agree")
    w = wl.make_small(5, 11, seed=21)
    Qa, Ia = _run(w, **KERNELS["reference"])
    Qb, Ib = _run(w, **KERNELS["fused_fp64"])
    _check(Qb, Ib, Qa, Ia, label="fused vs reference")


def test_fp32_refinement_progression():
    """Float32 chain alone, then each float64-residual refinement step,
    against the oracle on N=6 elements of the heterogeneous distribution."""
    _say("[gpu] fp32 refinement progression N=6")
    w = wl.make_small(6, 10, seed=31)
    Xo, Io = _oracle(w, list(range(w.n)))
    errs = []
    for k in range(0, 4):
        Q, Qi = _run(w, precision="fp32_refine", refine_steps=k)
        if k == 0:
            # float32 chain alone: every quantity to float32 accuracy
            el, per_q = parity.summary(Q, Xo)
            _say(f"  chain alone: element {el:.2e}, per quantity {parity.fmt(per_q)}")
            errs.append(float(max(el, per_q.max())))
            assert errs[0] <= 1e-4
        else:
            errs.append(parity.check(Q, Xo, TOL, f"after {k} step(s) Q", say=_say))
            parity.check(Qi, Io, TOL, f"after {k} step(s) Qint", say=_say)
    _say(f"  worst rel L2 after 0..3 refinement steps: {['%.2e' % e for e in errs]}")
    assert errs[1] < errs[0] * 1e-3


def test_stiffness_sweep_per_decade():
    """dt |E_uf,uf| from 1e-2 to 1e6 (N=5): float64 and float32 + refinement
    within the bar in every stiffness decade."""
    _say("[gpu] stiffness sweep N=5")
    w = wl.make_small(5, 48, seed=41, kind="stiffness")
    z = wl.stiffness(w)
    dec = np.floor(np.log10(z)).astype(int)
    pick = []
    for d in range(-2, 6):
        pick += list(np.where(dec == d)[0][:2])
    Xo, Io = opool.solve_many(5, w.star[pick], w.E[pick], w.Q0[pick], w.dt)
    for kw in (dict(precision="fp64"), dict(precision="fp32_refine", refine_steps=1),
               dict(precision="fp32_refine", refine_steps=2)):
        Q, Qi = _run(w, **kw)
        worst = np.maximum(rel_l2(Q[pick], Xo), parity.rel_l2_per_quantity(Q[pick], Xo).max(axis=1))
        per = {int(d): float(worst[np.array(dec[pick]) == d].max()) for d in sorted(set(dec[pick]))}
        _say(f"  {kw}: worst rel L2 (element or quantity) per decade {per}")
        _check(Q[pick], Qi[pick], Xo, Io, label=str(kw))


def _full_size(name, kw):
    w = wl.make_workload(name)
    ids = wl.oracle_sample(w.n)
    _say(f"  generated {name} n={w.n}; {len(ids)} sampled elements {ids}")
    Q, Qi = api.predict(_dev(w.Q0), _dev(w.star), _dev(w.E), w.dt, w.N, **kw)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(Q).all()) and bool(torch.isfinite(Qi).all())
    Qs, Is = Q[ids].cpu().numpy(), Qi[ids].cpu().numpy()
    del Q, Qi
    torch.cuda.empty_cache()
    Xo, Io = _oracle(w, ids)
    _check(Qs, Is, Xo, Io)


def test_full_size_n6_262144_fp64_sampled():
    """The benchmark's workload and launch: all 262,144 N=6 elements in one
    call, sampled elements checked against the oracle, all outputs finite."""
    _say("[gpu] full size n6_heterogeneous_262144 fp64")
    _full_size("n6_heterogeneous_262144", dict(precision="fp64"))


def test_full_size_n6_1048576_fp32_refine_sampled():
    """1,048,576 N=6 elements through the float32 chain + one refinement step."""
    _say("[gpu] full size n6_heterogeneous_1048576 fp32_refine")
    _full_size("n6_heterogeneous_1048576", dict(precision="fp32_refine", refine_steps=1))


def _general_operators(N, n, seed, chain_prob=0.35):
    """Operators outside the poroelastic structure: dense star matrices
    (every row couples to all 13 quantities, scaled so that dt A^j is of
    order one) and a random upper-triangular E whose diagonal spans
    dt E_pp in [-50, 0] and whose rows hold several couplings, forming
    dependency chains up to the full depth.  Exercises the dense-star and
    the level-by-level coupling paths of the fused kernel."""
    w = wl.make_small(N, n, seed=seed)
    rng = np.random.default_rng(1000 + seed)
    star = rng.standard_normal((n, 3, 13, 13)) * (0.3 / w.dt)
    E = np.zeros((n, 13, 13))
    iu = np.triu_indices(13, 1)
    for e in range(n):
        E[e][np.diag_indices(13)] = -rng.uniform(0.0, 50.0, 13) / w.dt
        mask = rng.random(len(iu[0])) < chain_prob
        E[e][iu[0][mask], iu[1][mask]] = rng.uniform(-1.0, 1.0, mask.sum()) / w.dt
        E[e][np.arange(12), np.arange(1, 13)] = rng.uniform(0.5, 1.0, 12) / w.dt  # full-depth chain
    return w, star, E


_GENERAL_CACHE = {}


@pytest.mark.parametrize("kernel", list(KERNELS))
@pytest.mark.parametrize("N,n", [(2, 7), (5, 4)])
def test_general_operators_dense_star_coupling_chains(kernel, N, n):
    _say(f"[gpu] general operators kernel={kernel} N={N} n={n}")
    if (N, n) not in _GENERAL_CACHE:
        w, star, E = _general_operators(N, n, seed=60 + N)
        _GENERAL_CACHE[(N, n)] = (w, star, E) + tuple(opool.solve_many(N, star, E, w.Q0, w.dt))
    w, star, E, Xo, Io = _GENERAL_CACHE[(N, n)]
    Q, Qi = api.predict(_dev(w.Q0), _dev(star), _dev(E), w.dt, N, **KERNELS[kernel])
    torch.cuda.synchronize()
    _check(Q.cpu().numpy(), Qi.cpu().numpy(), Xo, Io)


@pytest.mark.parametrize("kernel", ["fused_fp64", "fused_fp32_refine2", "mfma_fp32_refine2"])
def test_one_dense_star_row_in_a_group(kernel):
    """Poroelastic elements, one of which has a star row with more than six
    non-zero columns: its whole workgroup takes the dense-star path, the
    other groups keep the sparse one."""
    _say(f"[gpu] one dense star row kernel={kernel}")
    N = 4
    w = wl.make_small(N, 12, seed=70)
    star = w.star.copy()
    rng = np.random.default_rng(71)
    star[3, :, 0, :] += rng.standard_normal((3, 13)) * np.abs(star[3]).max() * 1e-3
    Q, Qi = api.predict(_dev(w.Q0), _dev(star), _dev(w.E), w.dt, N, **KERNELS[kernel])
    torch.cuda.synchronize()
    Xo, Io = opool.solve_many(N, star, w.E, w.Q0, w.dt)
    _check(Q.cpu().numpy(), Qi.cpu().numpy(), Xo, Io)


def test_full_size_n5_stiffness_524288_per_decade():
    """The stiffness workload at its full size (524,288 N=5 elements,
    dt |E_uf,uf| from 1e-2 to 1e6): two oracle elements from every decade,
    float64 and float32 + 1 and 2 refinement steps, all within the bar."""
    _say("[gpu] full size n5_stiffness_524288 per decade")
    w = wl.make_workload("n5_stiffness_524288")
    z = wl.stiffness(w)
    dec = np.floor(np.log10(z)).astype(int)
    ids = []
    for d in range(-2, 6):
        ids += [int(i) for i in np.where(dec == d)[0][:2]]
    _say(f"  decades {sorted(set(dec[ids].tolist()))}, elements {ids}")
    Xo, Io = opool.solve_many(w.N, w.star[ids], w.E[ids], w.Q0[ids], w.dt)
    dQ0, dstar, dE = _dev(w.Q0), _dev(w.star), _dev(w.E)
    for kw in (dict(precision="fp64"), dict(precision="fp32_refine", refine_steps=1),
               dict(precision="fp32_refine", refine_steps=2)):
        Q, Qi = api.predict(dQ0, dstar, dE, w.dt, w.N, **kw)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(Q).all())
        Qs, Is = Q[ids].cpu().numpy(), Qi[ids].cpu().numpy()
        worst = np.maximum(rel_l2(Qs, Xo), parity.rel_l2_per_quantity(Qs, Xo).max(axis=1))
        per = {int(d): float(worst[dec[ids] == d].max()) for d in sorted(set(dec[ids].tolist()))}
        _say(f"  {kw}: worst rel L2 (element or quantity) per decade {per}")
        _check(Qs, Is, Xo, Io, label=str(kw))
        del Q, Qi
        torch.cuda.empty_cache()


def test_full_size_n6_1048576_refinement_progression():
    """1,048,576 N=6 elements: the float32 chain alone, then 1, 2 and 3
    refinement steps, on oracle-checked sampled elements, beside float64."""
    _say("[gpu] full size n6_heterogeneous_1048576 refinement progression")
    w = wl.make_workload("n6_heterogeneous_1048576")
    ids = wl.oracle_sample(w.n)
    Xo, _ = _oracle(w, ids)
    dQ0, dstar, dE = _dev(w.Q0), _dev(w.star), _dev(w.E)
    errs = {}
    for name, kw in (("fp64", dict(precision="fp64")),) + tuple(
            (f"fp32+{k}", dict(precision="fp32_refine", refine_steps=k)) for k in range(4)):
        Q, _ = api.predict(dQ0, dstar, dE, w.dt, w.N, with_qint=False, **kw)
        torch.cuda.synchronize()
        Qs = Q[ids].cpu().numpy()
        del Q
        torch.cuda.empty_cache()
        if name == "fp32+0":
            el, per_q = parity.summary(Qs, Xo)
            _say(f"  {name}: element {el:.2e}, per quantity {parity.fmt(per_q)}")
            errs[name] = float(max(el, per_q.max()))
        else:
            errs[name] = parity.check(Qs, Xo, TOL, name, say=_say)
    _say(f"  worst rel L2 (element or quantity): {errs}")
    assert errs["fp32+0"] <= 1e-4
