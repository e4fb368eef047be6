"""GPU tests of the batched persistent launch and of the group sweeps.

A system's result must not depend on what it is batched with: the batched
kernel runs the single-system per-state code, so every result is bitwise
equal to the same system solved alone with the same sweep variant, and
within 1e-5 of the FP64 oracle.
"""
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


def _mini_batch(count=10, seed=7, hi=1600.0):
    return W.batch_systems(count=count, seed=seed, cells_lo=120.0, cells_hi=hi)


def test_batch_matches_oracle_and_solo(orc):
    import paper_2005_06191_amd as A
    ps = _mini_batch()
    say(f"[batch] {len(ps)} systems vs oracle and solo")
    res = A.batch_solve(ps, policy=True)
    for p, r in zip(ps, res):
        V = r.V.cpu().numpy()
        ref = orc.solve(p, gap=True)
        pol = r.policy.cpu().numpy() if r.policy is not None else None
        compare(p, ref, V, pol, TOL_FP32, gap=ref["gap"])
        solo = A.solve(p, variant=r.info["variant"])
        assert np.array_equal(V, solo.V.cpu().numpy()), p.name
        assert abs(r.info["max_row_tail"] - ref["max_tail"]) <= 1e-13 + 1e-9 * ref["max_tail"]


def test_batch_fp64_matches_oracle(orc):
    import paper_2005_06191_amd as A
    ps = [p.with_(precision="fp64") for p in _mini_batch(count=6, seed=11)]
    say("[batch] fp64")
    res = A.batch_solve(ps)
    for p, r in zip(ps, res):
        compare(p, orc.solve(p), r.V.cpu().numpy(), None, TOL_FP64)


def test_batch64_full_equals_solo():
    """The 64-system batch: each result bitwise equal to its solo solve."""
    import paper_2005_06191_amd as A
    ps = W.batch_systems()
    say("[batch] 64 systems vs solo, bitwise")
    bs = A.BatchSolver(ps)
    res = bs.solve()
    for p, r in zip(ps, res):
        solo = A.solve(p, variant=r.info["variant"], policy=False)
        assert np.array_equal(r.V.cpu().numpy(), solo.V.cpu().numpy()), p.name
        v = r.V.cpu().numpy()
        # FP32 masses may sum past 1 by a few ulps
        assert v.min() >= 0.0 and v.max() <= 1.0 + TOL_FP32
    # repeated launches are deterministic
    again = bs.solve()
    assert all(np.array_equal(a.V.cpu().numpy(), b.V.cpu().numpy()) for a, b in zip(res, again))


def _wide_window(**kw):
    # 2-D linear system whose windows span ~ 40 x 40 cells
    lo, h, cnt = W.tiling((-1.0, -1.0), (1.0, 1.0), (48, 48))
    return W.linear2d(precision="fp32", mode="otf").with_(lo=lo, h=h, count=cnt, var=(0.1 ** 2, 0.1 ** 2),
                                                          cutoff=1e-3, horizon=6, name="wide-window", **kw)


@pytest.mark.parametrize("variant", ["group16", "group64", "lanes"])
def test_group_variants_match_oracle(orc, variant):
    p = _wide_window()
    say(f"[group] {variant} vs oracle")
    ref = orc.solve(p, gap=True)
    V, pol, info = gpu_solve(p, variant=variant)
    assert info["variant"] == variant
    compare(p, ref, V, pol, TOL_FP32, gap=ref["gap"])
    assert abs(info["max_row_tail"] - ref["max_tail"]) <= 1e-13 + 1e-9 * ref["max_tail"]


@pytest.mark.parametrize("variant", ["group16", "group64"])
def test_group_variants_fp64(orc, variant):
    p = _wide_window(precision="fp64", spec="reach_avoid", target=W.box((0.3, 0.3), (0.9, 0.9), 2),
                     avoid=W.box((-0.6, -0.2), (-0.1, 0.2), 2))
    say(f"[group] {variant} fp64 reach-avoid")
    ref = orc.solve(p, gap=True)
    V, pol, _ = gpu_solve(p, variant=variant)
    compare(p, ref, V, pol, TOL_FP64, gap=ref["gap"])


def test_tuner_picks_a_variant_and_caches_it(tmp_path):
    import paper_2005_06191_amd as A
    A.tune_clear()
    p = _wide_window()
    say("[tune] solve variants")
    r = A.tune_solve(p)
    assert r["candidates"] >= 2 and r["best_ms"] <= r["worst_ms"]
    assert A.tune_entries() == 1
    assert A.query(p)["variant"] == {1: "lanes", 2: "fixed", 3: "group16", 4: "group64"}[r["variant"]]
    path = str(tmp_path / "tune.json")
    A.tune_save(path)
    A.tune_clear()
    A.tune_load(path)
    assert A.tune_entries() == 1
    A.tune_clear()


def test_batch_tuner():
    import paper_2005_06191_amd as A
    A.tune_clear()
    ps = _mini_batch(count=8, seed=3)
    say("[tune] batch launch parameters")
    bs = A.BatchSolver(ps)
    r = bs.tune()
    assert r["candidates"] == 24 and r["chunk"] in (1, 2, 4, 8)
    res = bs.solve()  # uses the tuned parameters; results unchanged
    for p, x in zip(ps, res):
        solo = A.solve(p, variant=x.info["variant"], policy=False)
        assert np.array_equal(x.V.cpu().numpy(), solo.V.cpu().numpy())
    A.tune_clear()
