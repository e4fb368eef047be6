"""GPU tests of the request loop with continuous batching.

Requests of mixed dynamics, precision, mode and size share the device: every
admitted request advances by one Bellman step per batched launch. A request's
rows run the single-system per-state code, so its value function and policy
equal a lone solve with the same mode and sweep variant bit for bit, and the
FP64 oracle within the precision's tolerance.
"""
import time

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import TOL_FP32, TOL_FP64, compare, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _wide_window():
    lo, h, cnt = W.tiling((-1.0, -1.0), (1.0, 1.0), (48, 48))
    return W.linear2d(precision="fp32", mode="otf").with_(lo=lo, h=h, count=cnt, var=(0.1 ** 2, 0.1 ** 2),
                                                          cutoff=1e-3, horizon=6, name="wide-window")


def _mix():
    ps = list(W.batch_systems(count=6, seed=5, cells_lo=120.0, cells_hi=1600.0))
    ps.append(W.linear2d(cells=30, precision="fp32", mode="stored", horizon=5).with_(name="lin-stored-f32"))
    ps.append(W.linear2d(cells=24, precision="fp64", mode="stored", horizon=4).with_(name="lin-stored-f64"))
    ps.append(W.room5d(cells=6, n=3, precision="fp64", mode="otf", horizon=5).with_(name="room3-f64"))
    ps.append(_wide_window())
    ps.append(W.linear2d(cells=20, precision="fp32", mode="otf", horizon=0).with_(name="lin-T0"))
    # large enough for its own launch per step (compiled-shape sweep)
    ps.append(W.scaled_family(W.unicycle3d(horizon=3), 7.0e4).with_(name="uni-solo"))
    # a family the batched kernel lacks: own launch per step as well
    ps.append(_affine5())
    return ps


def _affine5():
    lo, h, cnt = W.tiling((-1.0,) * 5, (1.0,) * 5, (4,) * 5)
    A5 = np.eye(5) * 0.6 + np.eye(5, k=1) * 0.1
    B5 = np.array([[0.0], [0.0], [0.0], [0.0], [1.0]])
    return W.linear2d(precision="fp32", mode="otf", horizon=4).with_(
        lo=lo, h=h, count=cnt, var=(0.09,) * 5, cutoff=1e-3, params=W.affine_params(A5, B5), name="affine5")


def _tol(p):
    return TOL_FP64 if p.precision == "fp64" else TOL_FP32


def _check_against_solo_and_oracle(orc, p, V, pol, info):
    import paper_2005_06191_amd as A
    ref = orc.solve(p, gap=True)
    compare(p, ref, V, pol, _tol(p), gap=ref["gap"])
    solo = A.solve(p, mode=info["mode"], variant=info["variant"], policy=pol is not None)
    assert np.array_equal(V, solo.V.cpu().numpy()), f"{p.name}: server != solo ({info['mode']}, {info['variant']})"
    if pol is not None:
        assert np.array_equal(pol, solo.policy.cpu().numpy()), f"{p.name}: policy differs from solo"
    if p.horizon > 0:
        assert abs(info["max_row_tail"] - ref["max_tail"]) <= 1e-13 + 1e-9 * ref["max_tail"], p.name


def test_server_mix_matches_solo_and_oracle(orc):
    import paper_2005_06191_amd as A
    ps = _mix()
    say(f"[server] {len(ps)} mixed requests submitted at once")
    with A.Server(hbm_budget_bytes=512 << 20, max_slots=16) as srv:
        tickets = [srv.submit(p, want_policy=True) for p in ps]
        outs = [srv.wait(t, timeout_ms=60000) for t in tickets]
        st = srv.stats()
    modes = set()
    for p, (V, pol, info) in zip(ps, outs):
        say(f"[server]   {p.name}: {info['mode']} {info['variant']}")
        modes.add(info["mode"])
        _check_against_solo_and_oracle(orc, p, V, pol if p.horizon > 0 else None, info)
    assert {"stored", "otf"} <= modes
    assert outs[[p.name for p in ps].index("uni-solo")][2]["variant"] in ("fixed", "factored")
    assert st["completed"] == len(ps) and st["failed"] == 0
    assert st["hbm_in_use"] == 0 and st["active"] == 0 and st["queued"] == 0
    assert st["max_active"] > 1
    assert 0 < st["p50_ms"] <= st["p99_ms"]


def test_server_continuous_admission(orc):
    """Requests submitted while others run join at a step boundary; a tight
    arena forces queueing by footprint; results stay bitwise equal to solo."""
    import paper_2005_06191_amd as A
    ps = list(W.batch_systems(count=12, seed=9, cells_lo=200.0, cells_hi=3000.0))
    budget = 4 << 20
    say(f"[server] continuous admission, {len(ps)} requests, arena {budget >> 20} MiB")
    with A.Server(hbm_budget_bytes=budget, max_slots=4) as srv:
        first = [srv.submit(p) for p in ps[:4]]
        time.sleep(0.002)
        rest = [srv.submit(p) for p in ps[4:]]
        outs = [srv.wait(t, timeout_ms=60000) for t in first + rest]
        st = srv.stats()
    for p, (V, _, info) in zip(ps, outs):
        _check_against_solo_and_oracle(orc, p, V, None, info)
    assert st["completed"] == len(ps)
    assert st["max_active"] <= 4
    assert st["hbm_peak"] <= budget


def test_server_errors():
    import paper_2005_06191_amd as A
    from paper_2005_06191_amd.binding import E_INVALID, E_NOMEM, AmyError
    small = W.linear2d(cells=20, precision="fp32", mode="otf", horizon=3)
    big = W.unicycle3d(nxy=100, ntheta=60, horizon=4)
    say("[server] errors: footprint over budget, invalid problem, bad config")
    with A.Server(hbm_budget_bytes=2 << 20, max_slots=2) as srv:
        t_big = srv.submit(big)
        t_ok = srv.submit(small)
        with pytest.raises(AmyError) as e:
            srv.wait(t_big, timeout_ms=60000)
        assert e.value.status == E_NOMEM
        V, _, _ = srv.wait(t_ok, timeout_ms=60000)
        assert V.shape == (small.n_x,)
        # invalid problems are refused at submission: cutoff above the peak density
        with pytest.raises(AmyError) as e:
            srv.submit(small.with_(cutoff=1e3))
        assert e.value.status == E_INVALID
        assert srv.stats()["failed"] == 1
    with pytest.raises(AmyError):
        A.Server(hbm_budget_bytes=1024, max_slots=2)


def test_server_cancellation(orc):
    """A queued request leaves the queue at once, a running one at the next
    step boundary; both answer E_CANCELLED and free their arena space, and
    the request behind them finishes with the solo result."""
    import paper_2005_06191_amd as A
    from paper_2005_06191_amd.binding import E_CANCELLED, E_INVALID, AmyError
    long = W.room5d(horizon=400)  # a few hundred ms on the device
    quick = W.linear2d(cells=30, precision="fp32", mode="otf", horizon=4)
    say("[server] cancellation: one queued, one running")
    with A.Server(hbm_budget_bytes=1 << 30, max_slots=1) as srv:
        t_long = srv.submit(long)
        t_q1 = srv.submit(quick)
        t_q2 = srv.submit(quick)
        srv.cancel(t_q1)  # queued behind the long request (one slot)
        t0 = time.time()
        while srv.stats()["active"] < 1 and time.time() - t0 < 10.0:
            time.sleep(0.001)
        srv.cancel(t_long)  # running
        for t in (t_q1, t_long):
            with pytest.raises(AmyError) as e:
                srv.wait(t, timeout_ms=60000)
            assert e.value.status == E_CANCELLED
        V, _, info = srv.wait(t_q2, timeout_ms=60000)
        st = srv.stats()
        # released tickets are unknown to the server
        with pytest.raises(AmyError) as e:
            srv.cancel(t_q2)
        assert e.value.status == E_INVALID
    _check_against_solo_and_oracle(orc, quick, V, None, info)
    assert st["cancelled"] == 2 and st["completed"] == 1 and st["failed"] == 0
    assert st["hbm_in_use"] == 0 and st["active"] == 0 and st["queued"] == 0
