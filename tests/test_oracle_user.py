"""The oracle with a right-hand side given as source text (Sec. 3: the
tool reads f as text), and the road-traffic model of Sec. 8.3.1 (CPU only).

The oracle compiles the text with the host C compiler and calls it for
every mean.  Pins: the text of a built-in family gives that family's
values; the traffic model's means keep the properties its printed
equations fix (vehicles flow one cell downstream around the ring, only the
exits lose vehicles, the lights add 6 and 8)."""
import numpy as np
import pytest

import workloads as W


def _small_traffic(text, q=2.0, horizon=3, **kw):
    return W.traffic5d(q=q, precision="fp64", horizon=horizon, text=text, **kw)


def test_robot_text_equals_the_builtin_family(orc):
    lo, h, cnt = W.grid_from_quantization((-4.0, -4.0), (4.0, 4.0), (0.5, 0.5))
    base = W.robot2d(spec="reach_avoid", horizon=3).with_(lo=lo, h=h, count=cnt, u_count=(3, 3), w_count=(3,),
                                                         params=(1.0,))
    a = orc.solve(base)["V"]
    b = orc.solve(base.with_(dyn="user", rhs=W.ROBOT_RHS))["V"]
    assert np.array_equal(a, b)


def test_traffic_text_equals_the_affine_form(orc):
    a = orc.solve(_small_traffic(False))["V"]
    b = orc.solve(_small_traffic(True))["V"]
    assert np.abs(a - b).max() <= 1e-12


def test_traffic_means_follow_the_printed_model(orc):
    p = _small_traffic(True)
    rng = np.random.default_rng(2)
    fl, ex = W.TRAFFIC_FLOW, W.TRAFFIC_EXIT
    for _ in range(50):
        x = rng.uniform(0.0, 10.0, 5)
        u = rng.integers(0, 2, 2).astype(float)
        mu = orc.mean(p, x, u)
        # vehicles are conserved around the ring except at the two exits
        assert abs(mu.sum() - (x.sum() - ex * (x[1] + x[3]) + 6.0 * u[0] + 8.0 * u[1])) <= 1e-12
    for i in range(5):
        x = np.zeros(5)
        x[i] = 4.0
        mu = orc.mean(p, x, np.zeros(2))
        # one occupied cell: a share flows to the next cell downstream only
        down = (i + 1) % 5
        assert abs(mu[down] - fl * 4.0) <= 1e-12
        others = [k for k in range(5) if k not in (i, down)]
        assert np.all(mu[others] == 0.0)
        assert abs(mu[i] - (1.0 - fl - (ex if i in (1, 3) else 0.0)) * 4.0) <= 1e-12
    # the lights feed cells 1 and 3 only
    assert np.allclose(orc.mean(p, np.zeros(5), np.array([1.0, 0.0])), [6.0, 0, 0, 0, 0])
    assert np.allclose(orc.mean(p, np.zeros(5), np.array([0.0, 1.0])), [0, 0, 8.0, 0, 0])


def test_traffic_full_size_counts():
    """Sec. 8.3.1 quantisation gives Table 4's 68,841,472 state-input pairs."""
    p = W.traffic5d()
    assert p.n_x * p.n_u == 68841472


def test_user_text_that_does_not_compile_is_refused(orc):
    p = _small_traffic(True).with_(rhs="mu[0] = no_such_name;")
    with pytest.raises(Exception):
        orc.solve(p)
