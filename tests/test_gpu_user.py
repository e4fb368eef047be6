"""GPU tests of dynamics given as source text (Sec. 3): the right-hand side
compiled at run time by hipRTC into the one-lane-per-state sweep, against
the oracle (which compiles the same text with the host compiler), and
against the built-in families the text restates."""
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


def _robot_small(**kw):
    lo, h, cnt = W.grid_from_quantization((-5.0, -5.0), (5.0, 5.0), (0.5, 0.5))
    return W.robot2d(spec="reach_avoid", horizon=4).with_(lo=lo, h=h, count=cnt, u_count=(5, 5), params=(1.0,),
                                                          **kw)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_robot_text_matches_the_builtin_robot_and_the_oracle(orc, prec):
    import paper_2005_06191_amd as A
    p = _robot_small(precision=prec)
    say(f"[user] robot text {prec}: n_x={p.n_x} n_u={p.n_u} n_w={p.n_w}")
    with A.UserDynamics(W.ROBOT_RHS, 2, 2, 1) as f:
        r = f.solve(p.with_(dyn="user", rhs=W.ROBOT_RHS))
    b = A.solve(p)
    # same arithmetic in the same per-state code: the same bits
    assert np.array_equal(r.V.cpu().numpy(), b.V.cpu().numpy())
    assert np.array_equal(r.policy.cpu().numpy(), b.policy.cpu().numpy())
    assert r.info["variant"] == "lanes"
    ref = orc.solve(p.with_(dyn="user", rhs=W.ROBOT_RHS), gap=True)
    tol = TOL_FP64 if prec == "fp64" else TOL_FP32
    compare(p, ref, r.V.cpu().numpy(), r.policy.cpu().numpy(), tol, gap=ref["gap"])
    assert abs(r.info["max_row_tail"] - ref["max_tail"]) <= 1e-13 + 1e-9 * ref["max_tail"]


@pytest.mark.parametrize("prec,variant", [("fp32", "auto"), ("fp64", "auto"), ("fp32", "group16"),
                                          ("fp64", "group64")])
def test_traffic_text_against_the_oracle(orc, prec, variant):
    """The 5-cell traffic ring of Sec. 8.3.1 written as text, on a coarser
    quantisation (6 points per cell): every state against the oracle, and
    within tolerance of the same model as the affine family."""
    import paper_2005_06191_amd as A
    p = W.traffic5d(q=2.0, precision=prec, horizon=4, text=True).with_(variant=variant)
    say(f"[user] traffic text {prec} {variant}: n_x={p.n_x} n_u={p.n_u}")
    with A.UserDynamics(p.rhs, 5, 2, 0) as f:
        r = f.solve(p)
    if variant != "auto":
        assert r.info["variant"] == variant
    ref = orc.solve(p, gap=True)
    tol = TOL_FP64 if prec == "fp64" else TOL_FP32
    compare(p, ref, r.V.cpu().numpy(), r.policy.cpu().numpy(), tol, gap=ref["gap"])
    aff = A.solve(W.traffic5d(q=2.0, precision=prec, horizon=4).with_(variant=variant))
    assert float(np.abs(aff.V.cpu().numpy() - r.V.cpu().numpy()).max()) <= tol


def test_text_errors():
    import paper_2005_06191_amd as A
    with pytest.raises(A.AmyError) as e:
        A.UserDynamics("mu[0] = undefined_name;", 2, 2, 0)
    assert e.value.status == A.binding.E_INVALID and "undefined_name" in str(e.value)
    p = _robot_small().with_(dyn="user", rhs=W.ROBOT_RHS)
    with pytest.raises(A.AmyError) as e:
        A.solve(p)                       # text dynamics need their compiled handle
    assert e.value.status == A.binding.E_INVALID
    with A.UserDynamics(W.ROBOT_RHS, 2, 2, 0) as f:
        with pytest.raises(A.AmyError):   # compiled for p = 0, problem has a disturbance
            f.solve(p)
