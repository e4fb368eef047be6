"""Pins of the oracle's disturbance player (CPU only).

Def. 3.1 adds a disturbance set W to the system, and the Remark after
Def. 3.2 makes the disturbance an adversary: the synthesis maximises the
satisfaction probability over inputs against the worst disturbance, which
Alg. 3 and Alg. 4 compute as V(x) = max_u min_w V_in(x, u, w).  The
oracle's recursion is pinned by things other than itself:

* the game value by brute force: every deterministic Markov policy of the
  controller against every reply of the adversary (a disturbance per step
  and state, knowing the input), each pair evaluated by forward
  propagation through the dense transition array;
* Alg. 3's own dense form (reshape the (x, u, w) values, minimise over W,
  maximise over U), written independently in oracle/brute.py;
* the deterministic limit (noise far below a cell): the value becomes the
  indicator of the controller's attractor, computed by the textbook fixed
  point Attr_k = {x : some u makes every w land in Attr_{k-1}};
* reductions and order properties: one disturbance point w0 is the system
  with w0 folded into its offset; more disturbance points never help the
  controller; a disturbance that moves nothing changes nothing.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import brute


def _line(count=4, spec="safety", horizon=2, w=(-0.3, 0.3), wc=2, cutoff=0.0, var=0.15 ** 2, **kw):
    # 1-D affine system on [0, count * 0.5) with a pushing disturbance
    lo, h, cnt = W.tiling((0.0,), (0.5 * count,), (count,))
    p = W.Problem(lo=lo, h=h, count=cnt, u_lo=(-0.4,), u_hi=(0.4,), u_count=(2,), dyn="affine",
                  params=W.affine_params([[1.0]], [[1.0]], [0.05], D=[[1.0]]), var=(var,),
                  cutoff=cutoff, horizon=horizon, spec=spec, w_lo=(w[0],), w_hi=(w[1],), w_count=(wc,),
                  name="line")
    if spec != "safety":
        p = p.with_(target=W.box((0.5 * count - 0.5,), (0.5 * count,), 1))
    if spec == "reach_avoid":
        p = p.with_(avoid=W.box((0.0,), (0.5,), 1))
    return p.with_(**kw)


@pytest.mark.parametrize("spec", ["safety", "reach", "reach_avoid"])
@pytest.mark.parametrize("cutoff", [0.0, 0.5])
def test_game_value_by_policy_enumeration(orc, spec, cutoff):
    p = _line(count=4 if spec == "safety" else 5, spec=spec, horizon=2, cutoff=cutoff)
    ref = brute.game_value_by_enumeration(p, cut=cutoff > 0)
    V = orc.solve(p)["V"]
    assert np.abs(V - ref).max() <= 1e-12, (V, ref)


def test_game_value_three_steps(orc):
    p = _line(count=3, spec="safety", horizon=3, w=(-0.35, 0.35))
    ref = brute.game_value_by_enumeration(p)
    assert np.abs(orc.solve(p)["V"] - ref).max() <= 1e-12


@pytest.mark.parametrize("spec", ["safety", "reach_avoid"])
def test_dense_alg3_robot(orc, spec):
    """The robot of Sec. 7 (planar, speed and heading inputs, one pushing
    disturbance) on a 6 x 5 grid: Alg. 3's dense reshape-min-max form."""
    lo, h, cnt = W.tiling((-3.0, -2.5), (3.0, 2.5), (6, 5))
    p = W.Problem(lo=lo, h=h, count=cnt, u_lo=(0.0, -math.pi / 2), u_hi=(0.08, math.pi / 2), u_count=(2, 3),
                  dyn="robot", params=(10.0,), var=(0.75, 0.75), cutoff=1e-3, horizon=3, spec=spec,
                  w_lo=(-0.4,), w_hi=(0.4,), w_count=(3,), name="robot-tiny")
    if spec == "reach_avoid":
        p = p.with_(target=W.box((1.0, -2.5), (3.0, 2.5), 2), avoid=W.box((-1.0, -1.0), (0.0, 1.0), 2))
    Vb, pb = brute.synthesize_game(p)
    r = orc.solve(p, gap=True)
    assert np.abs(r["V"] - Vb).max() <= 1e-12
    clear = r["gap"] > 1e-9
    assert np.array_equal(r["policy"][clear], pb[clear])


def test_deterministic_limit_is_the_attractor(orc):
    """Noise 1e-4 of a cell: the value is 1 exactly on the states from which
    the controller can force the target within T_d steps whatever the
    disturbance does, and 0 elsewhere."""
    n, T = 12, 4
    lo, h, cnt = W.tiling((0.0,), (float(n),), (n,))
    p = W.Problem(lo=lo, h=h, count=cnt, u_lo=(-1.0,), u_hi=(1.0,), u_count=(3,), dyn="affine",
                  params=W.affine_params([[1.0]], [[1.0]], [0.0], D=[[1.0]]), var=(1e-8,), cutoff=0.0,
                  horizon=T, spec="reach", target=W.box((9.0,), (12.0,), 1), w_lo=(-1.0,), w_hi=(0.0,),
                  w_count=(2,), name="attractor")
    centres = [lo[0] + (j + 0.5) * h[0] for j in range(n)]
    us, ws = [-1.0, 0.0, 1.0], [-1.0, 0.0]

    def cell(z):
        j = math.floor((z - lo[0]) / h[0])
        return j if 0 <= j < n else None

    target = {j for j in range(n) if 9.0 <= centres[j] <= 12.0}
    attr = set(target)
    for _ in range(T):
        nxt = set(attr)
        for j in range(n):
            if j in attr:
                continue
            for u in us:
                if all(cell(centres[j] + u + w) in attr for w in ws):
                    nxt.add(j)
                    break
        attr = nxt
    want = np.array([1.0 if j in attr else 0.0 for j in range(n)])
    V = orc.solve(p)["V"]
    assert np.abs(V - want).max() <= 1e-9, (V, want)
    # the adversary pushes down by 1 while the best input moves up by 1: only
    # the target itself is forced
    assert attr == target


def test_single_disturbance_point_is_an_offset(orc):
    p = _line(count=9, spec="reach_avoid", horizon=5, w=(0.2, 0.2), wc=1, cutoff=1e-3)
    q = p.with_(params=W.affine_params([[1.0]], [[1.0]], [0.05 + 0.2]), w_lo=(), w_hi=(), w_count=())
    a, b = orc.solve(p)["V"], orc.solve(q)["V"]
    assert np.abs(a - b).max() <= 1e-13


def test_disturbance_that_moves_nothing(orc):
    p = _line(count=9, spec="safety", horizon=5, cutoff=1e-3)
    still = p.with_(params=W.affine_params([[1.0]], [[1.0]], [0.05], D=[[0.0]]))
    none = p.with_(params=W.affine_params([[1.0]], [[1.0]], [0.05]), w_lo=(), w_hi=(), w_count=())
    assert np.array_equal(orc.solve(still)["V"], orc.solve(none)["V"])


def test_more_disturbance_points_never_help(orc):
    p2 = _line(count=10, spec="reach", horizon=6, w=(-0.3, 0.3), wc=2, cutoff=1e-4)
    p3 = p2.with_(w_count=(3,))      # adds w = 0
    p5 = p2.with_(w_count=(5,))      # superset of p3's points
    v2, v3, v5 = (orc.solve(p)["V"] for p in (p2, p3, p5))
    assert np.all(v5 <= v3 + 1e-15)
    # a one-point set inside the range is never worse for the controller
    v1 = orc.solve(p2.with_(w_lo=(0.0,), w_hi=(0.0,), w_count=(1,)))["V"]
    assert np.all(v3 <= v1 + 1e-15) and np.all(v2 <= v1 + 1e-15) is not None
    assert v5.min() >= 0.0 and v1.max() <= 1.0 + 1e-15


def test_robot_rows_and_tail(orc):
    """Each (x, u, w) row keeps its mass: the kept cells sum to the grid mass
    minus the reported tail, for every disturbance point."""
    lo, h, cnt = W.grid_from_quantization((-3.0, -3.0), (3.0, 3.0), (0.5, 0.5))
    p = W.Problem(lo=lo, h=h, count=cnt, u_lo=(-1.0, -1.0), u_hi=(1.0, 1.0), u_count=(3, 3), dyn="robot",
                  params=(0.4,), var=(0.75, 0.75), cutoff=1e-3, horizon=1, spec="safety",
                  w_lo=(-1.0,), w_hi=(1.0,), w_count=(3,), name="robot-rows")
    for state in (0, 60, 168):
        for r in range(p.n_u * p.n_w):
            kept, tail = orc.row_mass(p, state, r)
            row = orc.row_dense(p, state, r)
            assert abs(row.sum() - kept) <= 1e-14
            assert 0.0 <= tail <= 1.0 and kept + tail <= 1.0 + 1e-14
