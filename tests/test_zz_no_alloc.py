"""stp_predict_static (the entry point that allocates nothing) against
stp_predict with a caller workspace, through the C ABI: same kernels, so the
outputs must be bitwise equal, on two calls in a row, the second smaller
(and of another degree), so that what the first call left in the library's
scratch cannot leak into the second."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2108_10565_amd import StpError, api  # noqa: E402
from paper_2108_10565_amd import workload as wl  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _both(w, **kw):
    Q0, star, E = _dev(w.Q0), _dev(w.star), _dev(w.E)
    Qa, Ia = api.predict(Q0, star, E, w.dt, w.N, **kw)
    Qb = torch.full_like(Qa, float("nan"))
    Ib = torch.full_like(Ia, float("nan"))
    api.predict_static(Q0, star, E, w.dt, w.N, Qb, Ib, **kw)
    torch.cuda.synchronize()
    return Qa, Ia, Qb, Ib


@pytest.mark.parametrize("kw", [dict(precision="fp32_refine", refine_steps=2),
                                dict(precision="fp32_refine", refine_steps=1),
                                dict(precision="fp64")])
def test_static_equals_workspace_call_twice_second_smaller(kw):
    big = wl.make_small(6, 2000, seed=301)
    small = wl.make_small(4, 7, seed=302)
    for w in (big, small):
        _say(f"[gpu] predict_static vs predict {kw} N={w.N} n={w.n}")
        Qa, Ia, Qb, Ib = _both(w, **kw)
        assert bool(torch.isfinite(Qa).all())
        assert torch.equal(Qa, Qb) and torch.equal(Ia, Ib)


def test_static_rejects_calls_beyond_its_scratch():
    _say("[gpu] predict_static size limit")
    cap = api.static_scratch_bytes()
    n = cap // (13 * 84 * 7 * 4) + 1
    w = wl.make_small(6, 1, seed=303)
    Q0 = _dev(np.repeat(w.Q0, n, axis=0))
    star = _dev(np.repeat(w.star, n, axis=0))
    E = _dev(np.repeat(w.E, n, axis=0))
    Q = torch.empty((n, 13, 84, 7), dtype=torch.float64, device="cuda")
    with pytest.raises(StpError, match="EWORKSPACE"):
        api.predict_static(Q0, star, E, w.dt, 6, Q, None, precision="fp32_refine", refine_steps=1)
    # the same call within the limit works and matches the workspace path
    m = n - 1
    api.predict_static(Q0[:m], star[:m], E[:m], w.dt, 6, Q[:m], None, precision="fp32_refine",
                       refine_steps=1)
    Qa, _ = api.predict(Q0[:m], star[:m], E[:m], w.dt, 6, precision="fp32_refine", refine_steps=1,
                        with_qint=False)
    torch.cuda.synchronize()
    assert torch.equal(Q[:m], Qa)
