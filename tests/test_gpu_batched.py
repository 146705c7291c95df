"""Batched predictions of several (degree, time step) groups in one call, and
their replay from a captured HIP graph (one cycle of clustered local time
stepping).  Through the C ABI; expected values from the oracle and from
single stp_predict calls."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import pool as opool  # noqa: E402
from paper_2108_10565_amd import api  # noqa: E402
from paper_2108_10565_amd import workload as wl  # noqa: E402

import parity  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _batches(ws):
    return [dict(degree=w.N, dt=w.dt, Q0=_dev(w.Q0), star=_dev(w.star), E=_dev(w.E)) for w in ws]


@pytest.fixture(scope="module")
def lts_small():
    """Four rate-2 clusters x degrees 3..6 (16 batches, 60 launches per
    cycle), 32 elements: 4, 2, 1, 1 per degree in clusters 0..3."""
    return wl.make_lts(32, seed=9, shares=(0.5, 0.25, 0.125, 0.125))


_ORACLE = {}


def _oracle_all(batches):
    """Oracle of every element of every batch, in one worker pool (cached)."""
    missing = [w for w in batches if w.name not in _ORACLE]
    if missing:
        jobs = [(w.N, w.star[e], w.E[e], w.Q0[e], w.dt) for w in missing for e in range(w.n)]
        _say(f"  oracle on all {len(jobs)} elements of {len(missing)} batches")
        res = opool.solve_jobs(jobs, progress=opool._print_progress)
        k = 0
        for w in missing:
            _ORACLE[w.name] = (np.stack([r[0] for r in res[k:k + w.n]]), np.stack([r[1] for r in res[k:k + w.n]]))
            k += w.n
    return [_ORACLE[w.name] for w in batches]


@pytest.mark.parametrize("precision,refine", [("fp64", 0), ("fp32_refine", 2)])
def test_batched_equals_single_calls_and_oracle(lts_small, precision, refine):
    _say(f"[gpu] batched LTS {len(lts_small)} batches precision={precision}")
    oracles = _oracle_all(lts_small)
    bs = api.predict_batched(_batches(lts_small), precision=precision, refine_steps=refine)
    torch.cuda.synchronize()
    for w, b, (Xo, Io) in zip(lts_small, bs, oracles):
        Q1, I1 = api.predict(b["Q0"], b["star"], b["E"], w.dt, w.N, precision=precision, refine_steps=refine)
        torch.cuda.synchronize()
        assert torch.equal(b["Q"], Q1) and torch.equal(b["Qint"], I1), w.name
        _say(f"  {w.name} n={w.n} dt={w.dt:.3e}: every element")
        parity.check(b["Q"].cpu().numpy(), Xo, TOL, "Q", say=_say)
        parity.check(b["Qint"].cpu().numpy(), Io, TOL, "Qint", say=_say)


@pytest.mark.parametrize("precision,refine", [("fp64", 0), ("fp32_refine", 1)])
def test_graph_of_one_lts_cycle_replays(lts_small, precision, refine):
    """Capture the cycle (60 launches), replay it several times with eager
    work and synchronisations in between, and compare every replay with an
    eager batched call; then double Q0 in place: the replay, reading the new
    inputs through the captured pointers, must give exactly twice Q."""
    _say(f"[gpu] graph LTS cycle precision={precision}")
    cyc = wl.lts_cycle(lts_small)
    base = _batches(lts_small)
    eager = api.predict_batched([dict(b) for b in base], precision=precision, refine_steps=refine)
    torch.cuda.synchronize()
    batches = [dict(base[i]) for i in cyc]
    # repeated predictions of a batch share its outputs
    for j, i in enumerate(cyc):
        if cyc.index(i) < j:
            batches[j] = batches[cyc.index(i)]
        else:
            batches[j]["Q"] = torch.full_like(eager[i]["Q"], float("nan"))
            batches[j]["Qint"] = torch.full_like(eager[i]["Qint"], float("nan"))
    g = api.Graph(batches, precision=precision, refine_steps=refine)
    scratch = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
    for rep in range(3):
        g.launch()
        torch.cuda.synchronize()
        for j, i in enumerate(cyc):
            assert torch.equal(batches[j]["Q"], eager[i]["Q"]), (rep, j)
            assert torch.equal(batches[j]["Qint"], eager[i]["Qint"]), (rep, j)
        scratch.mul_(1.0001).add_(1.0)           # eager work between replays
        torch.cuda.synchronize()
        _say(f"  replay {rep}: all {len(cyc)} launches equal the eager call")
    for b in base:
        b["Q0"].mul_(2.0)
    g.launch()
    torch.cuda.synchronize()
    for j, i in enumerate(cyc):
        assert torch.equal(batches[j]["Q"], 2.0 * eager[i]["Q"]), j
    g.close()


@pytest.mark.parametrize("precision,refine", [("fp64", 0), ("fp32_refine", 1)])
def test_staged_graph_parallel_branches_replays(lts_small, precision, refine):
    """The cycle captured with the batches of each sub-step on parallel
    branches (stp_graph_create_staged): every replay, with eager work in
    between, equals the eager batched call bitwise; after Q0 is doubled in
    place a replay gives exactly twice Q."""
    _say(f"[gpu] staged graph LTS cycle precision={precision}")
    stages = wl.lts_stages(lts_small)
    base = _batches(lts_small)
    eager = api.predict_batched([dict(b) for b in base], precision=precision, refine_steps=refine)
    torch.cuda.synchronize()
    order = [i for st in stages for i in st]
    batches, seen = [], {}
    for i in order:
        if i not in seen:
            b = dict(base[i])
            b["Q"] = torch.full_like(eager[i]["Q"], float("nan"))
            b["Qint"] = torch.full_like(eager[i]["Qint"], float("nan"))
            seen[i] = b
        batches.append(seen[i])
    g = api.Graph(batches, precision=precision, refine_steps=refine, stages=[len(s) for s in stages])
    scratch = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
    for rep in range(3):
        g.launch()
        torch.cuda.synchronize()
        for i, b in seen.items():
            assert torch.equal(b["Q"], eager[i]["Q"]) and torch.equal(b["Qint"], eager[i]["Qint"]), (rep, i)
        scratch.mul_(1.0001).add_(1.0)
        torch.cuda.synchronize()
        _say(f"  replay {rep}: {len(order)} launches in {len(stages)} stages equal the eager call")
    for b in base:
        b["Q0"].mul_(2.0)
    g.launch()
    torch.cuda.synchronize()
    for i, b in seen.items():
        assert torch.equal(b["Q"], 2.0 * eager[i]["Q"]), i
    g.close()


def test_measured_machine_ceilings_are_plausible():
    """stp_measure_peaks: positive, and below 1.2x the published MI355X
    figures (FP64 vector and matrix 78.6 TFLOP/s, HBM 8 TB/s), which catches
    a FLOP or byte count off by a factor."""
    pk = api.measure_peaks()
    _say(f"[gpu] measured ceilings {pk}")
    assert 0 < pk["fp64_valu_tflops"] < 1.2 * 78.6
    assert 0 < pk["fp32_valu_tflops"] < 1.2 * 157.3
    assert 0 < pk["fp64_mfma_tflops"] < 1.2 * 78.6
    assert 0 < pk["hbm_copy_gbs"] < 1.2 * 8000 and 0 < pk["hbm_write_gbs"] < 1.2 * 8000
