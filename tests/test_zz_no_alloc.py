"""GPU test of amy_solve_static, the solve that allocates nothing: it runs
amy_solve's kernels on the library's own static workspace, so its results
are bitwise those of amy_solve (without info) on the same problem, call
after call, whatever the previous call left in that workspace."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import TOL_FP32, compare, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _pair(p):
    import torch

    import paper_2005_06191_amd as A
    a = A.solve_static(p, policy=True)
    torch.cuda.synchronize()
    b = A.solve(p, policy=True, info=False)
    torch.cuda.synchronize()
    return a, b


def test_static_solve_matches_solve_twice(orc):
    """Two calls in a row, the second on a smaller problem: each bitwise
    equal to amy_solve and within the FP32 tolerance of the oracle."""
    big = W.room5d(cells=12, horizon=6)             # compiled-shape sweep, memoised tables
    small = W.unicycle3d(nxy=20, ntheta=30, horizon=5)  # factored sweep, shared tables
    for p in (big, small):
        say(f"[static] {p.name}: n_x={p.n_x} T_d={p.horizon}")
        a, b = _pair(p)
        assert np.array_equal(a.V.cpu().numpy(), b.V.cpu().numpy()), p.name
        assert np.array_equal(a.policy.cpu().numpy(), b.policy.cpu().numpy()), p.name
        ref = orc.solve(p, gap=True)
        compare(p, ref, a.V.cpu().numpy(), a.policy.cpu().numpy(), TOL_FP32, gap=ref["gap"])


def test_static_solve_full_size_and_limit():
    """The room workload at full size fits the static workspace and matches
    amy_solve; a problem needing more than the limit is refused."""
    import paper_2005_06191_amd as A
    p = W.room5d(horizon=4)
    assert A.query(p)["workspace_bytes"] <= A.binding.STATIC_WORKSPACE_BYTES
    say(f"[static] {p.name} full size")
    a, b = _pair(p)
    assert np.array_equal(a.V.cpu().numpy(), b.V.cpu().numpy())
    big = W.room5d(cells=26, horizon=2, precision="fp64")
    assert A.query(big)["workspace_bytes"] > A.binding.STATIC_WORKSPACE_BYTES
    with pytest.raises(A.AmyError) as e:
        A.solve_static(big)
    assert e.value.status == A.binding.E_NOMEM
