"""GPU parity of the disturbance player, the other noise models, the
intersect window and multiplicative noise: the HIP path through the C ABI
against the FP64 oracle, element by element (several 64-state tiles and a
ragged tail), in every sweep variant that takes them (one lane per state,
16 or 64 lanes per state, stored rows), FP32 and FP64."""
import math

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import TOL_FP32, TOL_FP64, compare, gpu_solve, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_06191_amd as A
    A.binding.lib()


def _lin_dist(**kw):
    # 2-D linear system pushed by a 2-D disturbance (columns D), reach-avoid
    lo, h, cnt = W.tiling((-1.0, -1.0), (1.0, 1.0), (23, 21))
    p = W.Problem(lo=lo, h=h, count=cnt, u_lo=(-0.3,), u_hi=(0.3,), u_count=(4,), dyn="affine",
                  params=W.affine_params([[0.92, 0.05], [-0.03, 0.9]], [[0.0], [1.0]], [0.02, 0.0],
                                         D=[[1.0, 0.0], [0.3, 1.0]]),
                  var=(0.06 ** 2, 0.05 ** 2), cutoff=1e-3, horizon=6, spec="reach_avoid",
                  target=W.box((0.4, 0.3), (1.0, 1.0), 2), avoid=W.box((-0.6, -0.5), (-0.2, 0.0), 2),
                  w_lo=(-0.06, -0.04), w_hi=(0.06, 0.04), w_count=(3, 2), name="lin-dist")
    return p.with_(**kw)


def _robot(**kw):
    # the robot of Sec. 7 (covariance diag(0.75, 0.75), cutoff 1e-3, state
    # quantisation 0.5) on a [-6, 6]^2 part of its domain, 5 x 5 inputs, 5
    # disturbance points, tau = 1 (so steps stay inside the part)
    lo, h, cnt = W.grid_from_quantization((-6.0, -6.0), (6.0, 6.0), (0.5, 0.5))
    p = W.Problem(lo=lo, h=h, count=cnt, u_lo=(-1.0, -1.0), u_hi=(1.0, 1.0), u_count=(5, 5), dyn="robot",
                  params=(1.0,), var=(0.75, 0.75), cutoff=1e-3, horizon=5, spec="reach_avoid",
                  target=W.box((3.0, 3.0), (6.0, 6.0), 2), avoid=W.box((-1.0, -1.0), (1.0, 1.0), 2),
                  w_lo=(-0.5,), w_hi=(0.5,), w_count=(5,), name="robot-part")
    return p.with_(**kw)


def _uni_patch(**kw):
    p = W.unicycle3d()
    lo, h, cnt = W.tiling((0.0, 0.0, -math.pi), (2.2, 2.3, math.pi), (22, 23, 60))
    kw.setdefault("horizon", 6)
    return p.with_(lo=lo, h=h, count=cnt, target=W.box((1.5, 1.5), (2.2, 2.3), 3),
                   avoid=W.box((0.6, 0.6), (1.0, 1.2), 3), name="unicycle-patch", **kw)


def _room_patch(**kw):
    p = W.room5d()
    lo, h, cnt = W.tiling((19.7,) * 4 + (19.6,), (20.3,) * 4 + (20.4,), (6, 6, 6, 6, 8))
    return p.with_(lo=lo, h=h, count=cnt, horizon=5, name="room-patch", **kw)


def _room8(**kw):
    # whole 1 x 4 x 4 x 4 x 4 tiles: the steps read memoised tables and stage V boxes
    p = W.room5d()
    lo, h, cnt = W.tiling((19.6,) * 5, (20.4,) * 5, (8,) * 5)
    return p.with_(lo=lo, h=h, count=cnt, horizon=5, name="room-8^5", **kw)


def _vehicle_planes(**kw):
    # whole yaw-rate / slip-angle planes: the steps read memoised tables and stage planes of V
    p = W.vehicle7d()
    return p.with_(lo=(-2.5, -2.5, -0.15, -0.75, -0.225, -0.4, -0.04), count=(2, 2, 3, 3, 6, 8, 8),
                   horizon=4, u_count=(3, 3), name="vehicle7-planes", **kw)


def _vehicle_uniform(**kw):
    # uniform noise whose windows are the compiled vehicle shape 2 x 2 x 3^5
    # (half-widths 0.45 h in the positions, 0.9 h elsewhere: supports meeting 2 and 3 cells)
    h = W.vehicle7d().h
    a = tuple((0.45 if i < 2 else 0.9) * h[i] for i in range(7))
    return _vehicle_planes(noise="uniform", noise_a=tuple(-x for x in a), noise_b=a, **kw)


def _lin(**kw):
    p = W.linear2d(cells=37, precision="fp32", mode="otf")
    kw.setdefault("horizon", 6)
    return p.with_(safe=W.box((-0.9, -0.95), (0.95, 0.9), 2), **kw)


CASES = {
    # disturbance player (Def. 3.1 / Alg. 4)
    "lin-dist-fp32": lambda: _lin_dist(),
    "lin-dist-fp64": lambda: _lin_dist(precision="fp64"),
    "lin-dist-fp32-stored": lambda: _lin_dist(mode="stored"),
    "lin-dist-fp32-group16": lambda: _lin_dist(variant="group16"),
    "lin-dist-fp64-group64": lambda: _lin_dist(precision="fp64", variant="group64"),
    "robot-dist-fp32": lambda: _robot(),
    "robot-dist-fp64-stored": lambda: _robot(precision="fp64", mode="stored"),
    "robot-nodist-fp32": lambda: _robot(w_lo=(), w_hi=(), w_count=()),
    "robot-dist-fp32-inputs": lambda: _robot(variant="inputs"),
    "robot-dist-fp64-inputs": lambda: _robot(precision="fp64", variant="inputs"),
    "lin-dist-fp32-inputs": lambda: _lin_dist(variant="inputs"),
    # other noise models (Sec. 3, Sec. 6.2)
    "lin-uniform-fp32": lambda: _lin(noise="uniform", noise_a=(-0.08, -0.05), noise_b=(0.07, 0.11)),
    "lin-uniform-fp64-stored": lambda: _lin(noise="uniform", noise_a=(-0.08, -0.05), noise_b=(0.07, 0.11),
                                            precision="fp64", mode="stored"),
    "lin-exponential-fp32": lambda: _lin(noise="exponential", noise_a=(25.0, 40.0), cutoff=1e-2),
    "lin-exponential-fp64": lambda: _lin(noise="exponential", noise_a=(25.0, 40.0), cutoff=1e-2, precision="fp64"),
    "lin-beta-fp32": lambda: _lin(horizon=4, noise="beta", noise_a=(-0.1, -0.07), noise_b=(0.08, 0.12),
                                  noise_alpha=(2.0, 1.5), noise_beta=(3.0, 1.5)),
    "lin-beta-fp64-group16": lambda: _lin(horizon=4, noise="beta", noise_a=(-0.1, -0.07), noise_b=(0.08, 0.12),
                                          noise_alpha=(2.0, 1.5), noise_beta=(3.0, 1.5), precision="fp64",
                                          variant="group16"),
    "room-uniform-fp32": lambda: _room_patch(noise="uniform", noise_a=(-0.06,) * 5, noise_b=(0.06,) * 5),
    "room-exponential-fp64": lambda: _room_patch(noise="exponential", noise_a=(30.0,) * 5, cutoff=1e-2,
                                                 precision="fp64"),
    # the other noise models through memoised tables (two-cell windows)
    "room8-beta-fp32-memo": lambda: _room8(noise="beta", noise_a=(-0.05,) * 5, noise_b=(0.05,) * 5,
                                           noise_alpha=(2.0,) * 5, noise_beta=(2.0,) * 5),
    "room8-uniform-fp64-memo": lambda: _room8(noise="uniform", noise_a=(-0.06,) * 5, noise_b=(0.06,) * 5,
                                              precision="fp64"),
    "room8-beta-fp32-memo-coupled": lambda: _room8(noise="beta", noise_a=(-0.05,) * 5, noise_b=(0.05,) * 5,
                                                   noise_alpha=(2.0,) * 5, noise_beta=(3.0,) * 5,
                                                   params=(0.25, 0.005, 0.01, -1.0, 50.0)),
    "vehicle7-planes-uniform-fp32-memo": lambda: _vehicle_uniform(),
    # intersect window and multiplicative noise (Eq. 3.2, Sec. 6.2)
    "unicycle-intersect-fp32": lambda: _uni_patch(window="intersect", horizon=3),
    "unicycle-intersect-fp64": lambda: _uni_patch(window="intersect", precision="fp64", horizon=3),
    "room-intersect-fp32": lambda: _room_patch(window="intersect"),
    "lin-mult-fp32": lambda: W.linear2d(cells=19, precision="fp32", mode="otf", horizon=5).with_(
        multiplicative=True, var=(0.08 ** 2, 0.1 ** 2)),
    "lin-mult-fp64-group64": lambda: W.linear2d(cells=19, precision="fp64", mode="otf", horizon=5).with_(
        multiplicative=True, var=(0.08 ** 2, 0.1 ** 2), variant="group64"),
    "lin-mult-fp32-stored": lambda: W.linear2d(cells=19, precision="fp32", mode="stored", horizon=5).with_(
        multiplicative=True, var=(0.08 ** 2, 0.1 ** 2)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_feature_parity(orc, name):
    p = CASES[name]()
    say(f"[feature] {name}: n_x={p.n_x} n_u={p.n_u} n_w={p.n_w} T_d={p.horizon} {p.precision} {p.mode}")
    ref = orc.solve(p, gap=True)
    V, pol, info = gpu_solve(p)
    tol = TOL_FP64 if p.precision == "fp64" else TOL_FP32
    err = compare(p, ref, V, pol, tol, gap=ref["gap"])
    assert info["n_w"] == p.n_w and info["rows"] == p.rows
    assert abs(info["max_row_tail"] - ref["max_tail"]) <= 1e-13 + 1e-9 * ref["max_tail"]
    say(f"[feature] {name}: {info['variant']} max err {err:.2e} tail {info['max_row_tail']:.3e}")


def test_plain_problems_keep_the_compiled_sweeps():
    """Problems without a disturbance, with additive normal noise and the
    centre rule still resolve to the compiled-shape sweeps; the others to
    the run-time-window ones."""
    import paper_2005_06191_amd as A
    assert A.query(W.unicycle3d())["variant"] == "factored"
    assert A.query(W.room5d())["variant"] == "fixed"
    assert A.query(W.room5d().with_(window="intersect"))["variant"] in ("lanes", "group16", "group64")
    # other noise models: the compiled shape when every step reads memoised
    # tables (whole staged tiles), the run-time-window sweeps otherwise
    beta = dict(noise="beta", noise_a=(-0.05,) * 5, noise_b=(0.05,) * 5, noise_alpha=(2.0,) * 5,
                noise_beta=(2.0,) * 5)
    assert A.query(W.room5d().with_(**beta))["variant"] == "fixed"
    assert A.query(_room8(**beta))["variant"] == "fixed"
    assert A.query(_room_patch(**beta))["variant"] in ("lanes", "group16", "group64")
    assert A.query(_room8(multiplicative=True))["variant"] in ("lanes", "group16", "group64")
    q = A.query(_vehicle_uniform())
    assert q["variant"] == "fixed" and q["window"][:7] == [2, 2, 3, 3, 3, 3, 3]
    # the FP64 vehicle keeps the gather sweep, which computes normal masses only
    assert A.query(_vehicle_uniform(precision="fp64"))["variant"] in ("lanes", "group16", "group64")
    assert A.query(_lin_dist())["variant"] in ("lanes", "group16", "group64")


def test_disturbance_with_one_point_equals_offset():
    """A one-point disturbance set is the system with that point folded into
    its offset (bitwise: the same windows and the same sums)."""
    p = _lin_dist(w_lo=(0.03, -0.02), w_hi=(0.03, -0.02), w_count=(1, 1))
    V1, pol1, _ = gpu_solve(p)
    ref_w = np.array([1.0 * 0.03 + 0.0 * -0.02, 0.3 * 0.03 + 1.0 * -0.02])
    q = p.with_(params=W.affine_params([[0.92, 0.05], [-0.03, 0.9]], [[0.0], [1.0]], [0.02 + ref_w[0], ref_w[1]]),
                w_lo=(), w_hi=(), w_count=())
    V2, pol2, _ = gpu_solve(q)
    assert np.abs(V1 - V2).max() <= 1e-6


def test_intersect_full_unicycle_tail_and_oracle(orc):
    """The unicycle workload at full size with the intersect rule: the
    truncated tail bound E drops well below the centre rule's, and the last
    step agrees with the oracle at sampled states (chained from the GPU's
    FP64 V_2)."""
    p = W.unicycle3d(horizon=16).with_(window="intersect")
    c = W.unicycle3d(horizon=16)
    Vc, _, ic = gpu_solve(c, policy=False)
    V, pol, info = gpu_solve(p)
    say(f"[intersect] unicycle E centre {ic['tail_bound_E']:.3e} intersect {info['tail_bound_E']:.3e}")
    assert info["tail_bound_E"] < 0.1 * ic["tail_bound_E"]
    Vn, _, _ = gpu_solve(p.with_(precision="fp64", horizon=15), policy=False)
    rng = np.random.default_rng(4)
    st = np.unique(np.concatenate([rng.integers(0, p.n_x, 600), [0, p.n_x - 1]]))
    Vr, pr, gap = orc.step(p.with_(precision="fp64"), st, V_next=Vn)
    assert float(np.abs(V[st] - Vr).max()) <= TOL_FP32
    # the larger window never loses value: V_intersect >= V_centre - tol
    assert float((Vc - V).max()) <= 1e-4


def test_server_takes_disturbance_requests_solo(orc):
    """The server runs requests the batched step lacks (a disturbance) with
    their own launches; the result is the solo solve's."""
    import paper_2005_06191_amd as A
    p = _lin_dist()
    with A.Server(hbm_budget_bytes=1 << 30, max_slots=4) as srv:
        t = srv.submit(p)
        V, _, info = srv.wait(t, timeout_ms=60000)
    solo, _, _ = gpu_solve(p, policy=False)
    assert np.array_equal(V, solo)
    compare(p, orc.solve(p), V, None, TOL_FP32)


def test_batch_refuses_disturbance():
    import paper_2005_06191_amd as A
    with pytest.raises(A.AmyError) as e:
        A.batch_query([_lin_dist(), W.linear2d(cells=20, precision="fp32", mode="otf")])
    assert e.value.status == A.binding.E_UNSUPPORTED


@pytest.mark.parametrize("name", ["robot-dist-fp32", "lin-dist-fp64", "unicycle-intersect-fp32"])
def test_inputs_variant_is_bitwise_lanes(name):
    """One wave per state with lanes over inputs computes every row with the
    same code as one lane per state, and its butterfly keeps the lowest
    maximising input: V and policy are bitwise those of LANES."""
    import paper_2005_06191_amd as A
    p = CASES[name]()
    say(f"[inputs vs lanes] {name}")
    a = A.solve(p.with_(variant="inputs"))
    b = A.solve(p.with_(variant="lanes"))
    assert a.info["variant"] == "inputs" and b.info["variant"] == "lanes"
    assert np.array_equal(a.V.cpu().numpy(), b.V.cpu().numpy())
    assert np.array_equal(a.policy.cpu().numpy(), b.policy.cpu().numpy())
    assert a.info["max_row_tail"] == b.info["max_row_tail"]


def test_inputs_variant_full_robot_chained(orc):
    """The robot of Sec. 7 at the printed size (1,681 states, 121 inputs, 11
    disturbance points), which AUTO runs one wave per state: its last step
    against the oracle at sampled states, chained from the GPU's FP64 V_2."""
    p = W.robot2d()
    import paper_2005_06191_amd as A
    assert A.query(p)["variant"] == "inputs"
    V, pol, info = gpu_solve(p)
    Vn, _, _ = gpu_solve(p.with_(precision="fp64", horizon=p.horizon - 1), policy=False)
    st = np.arange(0, p.n_x, 7)
    Vr, pr, gap = orc.step(p.with_(precision="fp64"), st, V_next=Vn)
    assert float(np.abs(V[st] - Vr).max()) <= TOL_FP32
    clear = gap > 2 * TOL_FP32
    assert np.array_equal(pol[0][st][clear], pr[clear])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_intersect_compiled_shape_is_bitwise_lanes(prec):
    """With the intersect rule the unicycle's windows are 6 x 6 x 3, a
    compiled shape: AUTO runs the factored sweep there (its re-associated
    sums are checked against the oracle with the parity cases), and the
    per-state compiled-shape sweep (memoised tables) computes rows bitwise
    those of the run-time-window LANES sweep."""
    import paper_2005_06191_amd as A
    p = CASES[f"unicycle-intersect-{prec}"]()
    say(f"[intersect fixed vs lanes] {prec}")
    assert A.query(p)["variant"] == "factored"
    a = A.solve(p.with_(variant="fixed"))
    b = A.solve(p.with_(variant="lanes"))
    assert a.info["variant"] == "fixed" and b.info["variant"] == "lanes"
    assert np.array_equal(a.V.cpu().numpy(), b.V.cpu().numpy())
    assert np.array_equal(a.policy.cpu().numpy(), b.policy.cpu().numpy())
    assert a.info["max_row_tail"] == b.info["max_row_tail"]


@pytest.mark.parametrize("name", ["room8-beta-fp32-memo", "room8-beta-fp32-memo-coupled", "room8-uniform-fp64-memo"])
def test_general_noise_staged_is_bitwise_lanes(name):
    """Beta and uniform noise on the 8^5 room grid: the staged sweep on
    memoised general-noise tables (two-cell tiles, the 2^5 shape's box
    staged by two groups along dimension 0) computes rows bitwise those of
    the run-time-window LANES sweep, which builds the same masses per row."""
    import paper_2005_06191_amd as A
    p = CASES[name]()
    say(f"[general noise fixed vs lanes] {name}")
    a = A.solve(p.with_(variant="fixed"))
    b = A.solve(p.with_(variant="lanes"))
    assert a.info["variant"] == "fixed" and b.info["variant"] == "lanes"
    assert np.array_equal(a.V.cpu().numpy(), b.V.cpu().numpy())
    assert np.array_equal(a.policy.cpu().numpy(), b.policy.cpu().numpy())
    assert a.info["max_row_tail"] == b.info["max_row_tail"]
