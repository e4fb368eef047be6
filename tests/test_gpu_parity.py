"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Element-by-element at sizes the oracle finishes in seconds (several 64-state
tiles and a ragged tail); sampled states at the full workload sizes for one
Bellman step; the FP32 path against the FP64 path and invariants at full
size over the whole horizon.
"""
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


def _uni_small(**kw):
    # the unicycle workload's cell widths, noise and cutoff on a smaller domain
    p = W.unicycle3d(nxy=100, ntheta=60)
    lo, h, cnt = W.tiling((0.0, 0.0, -math.pi), (2.2, 2.3, math.pi), (22, 23, 60))
    return p.with_(lo=lo, h=h, count=cnt, target=W.box((1.5, 1.5), (2.2, 2.3), 3),
                   avoid=W.box((0.6, 0.6), (1.0, 1.2), 3), horizon=kw.pop("horizon", 8),
                   name="unicycle-patch", **kw)


def _uni_even(ny=24, **kw):
    # a number of y cells divisible by 4 (by 2 only, for ny=26): the
    # relative-table steps take four (two) cells per workgroup
    p = W.unicycle3d(nxy=100, ntheta=60)
    lo, h, cnt = W.tiling((0.0, 0.0, -math.pi), (2.2, 0.1 * ny, math.pi), (22, ny, 60))
    return p.with_(lo=lo, h=h, count=cnt, target=W.box((1.5, 1.5), (2.2, 0.1 * ny), 3),
                   avoid=W.box((0.6, 0.6), (1.0, 1.2), 3), horizon=kw.pop("horizon", 8),
                   name="unicycle-even", **kw)


def _room_small(**kw):
    # the room workload's cell width, noise and cutoff on a 5^5 patch around 20
    p = W.room5d()
    lo, h, cnt = W.tiling((19.75,) * 5, (20.25,) * 5, (5,) * 5)
    return p.with_(lo=lo, h=h, count=cnt, horizon=kw.pop("horizon", 6), name="room-patch", **kw)


def _room8(**kw):
    # the room workload's cell width, noise and cutoff on an 8^5 grid: whole
    # 1 x 4 x 4 x 4 x 4 tiles, so the memoised steps stage V boxes in LDS
    p = W.room5d()
    lo, h, cnt = W.tiling((19.6,) * 5, (20.4,) * 5, (8,) * 5)
    return p.with_(lo=lo, h=h, count=cnt, horizon=kw.pop("horizon", 6), name="room-8^5", **kw)


def _vehicle_planes(n4=6, **kw):
    # the vehicle workload's cell widths, noise and cutoff on a 2x2x3x3xn4 x 8x8
    # sub-box: whole yaw-rate / slip-angle planes, so the memoised steps stage
    # planes of V in LDS (with n4 = 8 heading cells, one workgroup takes all
    # eight planes of states that share the other cells)
    p = W.vehicle7d()
    return p.with_(lo=(-2.5, -2.5, -0.15, -0.75, -0.225, -0.4, -0.04), count=(2, 2, 3, 3, n4, 8, 8),
                   horizon=kw.pop("horizon", 4), u_count=(3, 3), name="vehicle7-planes", **kw)


CASES = {
    "linear2d-full-fp64-stored": lambda: W.linear2d(precision="fp64", mode="stored"),
    "linear2d-full-fp64-otf": lambda: W.linear2d(precision="fp64", mode="otf"),
    "linear2d-full-fp32-otf": lambda: W.linear2d(precision="fp32", mode="otf"),
    "linear2d-full-fp32-stored": lambda: W.linear2d(precision="fp32", mode="stored"),
    "unicycle-patch-fp32-otf": lambda: _uni_small(precision="fp32", mode="otf"),
    "unicycle-patch-fp64-otf": lambda: _uni_small(precision="fp64", mode="otf"),
    "unicycle-patch-fp32-stored": lambda: _uni_small(precision="fp32", mode="stored"),
    "unicycle-patch-reach-fp32": lambda: _uni_small(precision="fp32", spec="reach"),
    # speeds up to 3: the x / y windows of one cell's headings spread past
    # the staged 7 x 7 box, and those windows are gathered from V instead
    "unicycle-patch-fast-fp32": lambda: _uni_small(precision="fp32", u_hi=(3.0, 1.0)),
    "unicycle-even-fp32": lambda: _uni_even(precision="fp32"),
    "unicycle-even-fast-fp32": lambda: _uni_even(precision="fp32", u_hi=(3.0, 1.0)),
    "unicycle-y26-fp32": lambda: _uni_even(ny=26, precision="fp32"),
    # the intersect window rule: 6 x 6 x 3 windows, relative tables keeping
    # every cell that meets the cutting interval
    "unicycle-patch-intersect-fp64": lambda: _uni_small(precision="fp64", window="intersect"),
    "unicycle-even-intersect-fp32": lambda: _uni_even(precision="fp32", window="intersect"),
    "room-patch-fp32-otf": lambda: _room_small(precision="fp32"),
    "room-patch-fp64-otf": lambda: _room_small(precision="fp64"),
    "room-patch-fp64-stored": lambda: _room_small(precision="fp64", mode="stored"),
    "room-8^5-fp32-otf": lambda: _room8(precision="fp32"),
    "room-8^5-fp64-otf": lambda: _room8(precision="fp64"),
    # neighbour coupling 0.25: about 4% of the (state, input) windows of a
    # tile fall outside its staged box and are gathered from V instead
    "room-8^5-coupled-fp32": lambda: _room8(precision="fp32", params=(0.25, 0.005, 0.01, -1.0, 50.0)),
    # states outside the safe box are not free: in the staged sweep they
    # write their value and still take part in every staging pass
    "room-8^5-safebox-fp32": lambda: _room8(precision="fp32", safe=W.box((19.65,) * 5, (20.3,) * 5, 5)),
    "vehicle7-planes-fp32": lambda: _vehicle_planes(precision="fp32"),
    "vehicle7-planes8-fp32": lambda: _vehicle_planes(n4=8, precision="fp32"),
    "vehicle7-planes8-fp64": lambda: _vehicle_planes(n4=8, precision="fp64"),
    "vehicle7-planes8-tau0.3-fp32": lambda: _vehicle_planes(n4=8, precision="fp32",
                                                            params=(0.3,) + W.VEHICLE7_BMW320I[1:]),
    # time step 0.3: about 7% of the windows spread past the staged planes
    # in the heading and are gathered from V instead
    "vehicle7-planes-tau0.3-fp32": lambda: _vehicle_planes(precision="fp32",
                                                           params=(0.3,) + W.VEHICLE7_BMW320I[1:]),
    "vehicle7-small-fp32": lambda: W.vehicle7d(cells=4, horizon=4).with_(u_count=(3, 3)),
    "vehicle7-small-fp64": lambda: W.vehicle7d(cells=4, horizon=4, precision="fp64").with_(u_count=(3, 3)),
    "linear2d-safebox-fp32": lambda: W.linear2d(cells=37, precision="fp32", mode="otf").with_(
        safe=W.box((-0.8, -0.9), (0.95, 0.7), 2)),
    "linear2d-nocut-fp64": lambda: W.linear2d(cells=21, precision="fp64", mode="otf").with_(cutoff=0.0),
    "linear2d-nocut-fp32-stored": lambda: W.linear2d(cells=21, precision="fp32", mode="stored").with_(cutoff=0.0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_parity_small(orc, name):
    p = CASES[name]()
    say(f"[parity] {name}: n_x={p.n_x} n_u={p.n_u} T_d={p.horizon} {p.precision} {p.mode}")
    ref = orc.solve(p, gap=True)
    V, pol, info = gpu_solve(p)
    tol = TOL_FP64 if p.precision == "fp64" else TOL_FP32
    err = compare(p, ref, V, pol, tol, gap=ref["gap"])
    # the FP64 tail bound agrees with the oracle's
    assert abs(info["max_row_tail"] - ref["max_tail"]) <= 1e-13 + 1e-9 * ref["max_tail"]
    say(f"[parity] {name}: max err {err:.2e}  tail {info['max_row_tail']:.3e}")


EDGE = {
    "single-partial-tile": lambda: W.linear2d(cells=7, precision="fp64", mode="otf"),
    "horizon0": lambda: _uni_small(precision="fp32", horizon=0),
    "horizon1": lambda: _uni_small(precision="fp32", horizon=1),
    "one-input": lambda: W.linear2d(cells=30, precision="fp32", mode="otf").with_(
        u_lo=(0.0,), u_hi=(0.0,), u_count=(1,)),
    "n1": lambda: W.Problem(lo=(-1.0,), h=(2.0 / 301,), count=(301,), u_lo=(-0.3,), u_hi=(0.3,),
                            u_count=(7,), dyn="affine", params=W.affine_params([[1.01]], [[1.0]]),
                            var=(0.02 ** 2,), cutoff=1e-3, horizon=10, spec="reach",
                            target=W.box((0.5,), (0.7,), 1), precision="fp32", mode="otf", name="n1"),
    "wide-cut-L1": lambda: W.linear2d(cells=8, precision="fp32", mode="otf").with_(cutoff=2.0),
    "leaves-grid": lambda: W.linear2d(cells=24, precision="fp64", mode="otf").with_(
        params=W.affine_params([[1.3, 0.0], [0.0, 1.25]], [[0.0], [1.0]], [0.4, -0.3])),
    "room3-per-room-heaters": lambda: W.room5d(cells=9, n=3, horizon=5, precision="fp32").with_(
        u_lo=(0.0, 0.0, 0.0), u_hi=(1.0, 1.0, 1.0), u_count=(2, 3, 2)),
}


@pytest.mark.parametrize("name", list(EDGE))
def test_parity_edge_cases(orc, name):
    p = EDGE[name]()
    say(f"[edge] {name}: n_x={p.n_x} n_u={p.n_u} T_d={p.horizon}")
    ref = orc.solve(p, gap=True)
    V, pol, _ = gpu_solve(p)
    tol = TOL_FP64 if p.precision == "fp64" else TOL_FP32
    compare(p, ref, V, pol, tol, gap=ref["gap"])


def test_deterministic_repeat():
    p = _uni_small(precision="fp32")
    say("[determinism] two solves bitwise equal")
    a, pa, _ = gpu_solve(p)
    b, pb, _ = gpu_solve(p)
    assert np.array_equal(a, b) and np.array_equal(pa, pb)


def test_stored_matches_otf():
    p = _room_small(precision="fp32", horizon=8)
    say("[stored vs otf] room patch fp32")
    a, pa, _ = gpu_solve(p.with_(mode="otf"))
    b, pb, _ = gpu_solve(p.with_(mode="stored"))
    assert np.abs(a - b).max() <= 2e-6


# ------------------------------------------------------------ full sizes

FULL = {
    "unicycle-100x100x60": lambda: W.unicycle3d(),
    "room5-20^5": lambda: W.room5d(),
    "vehicle7-8^7": lambda: W.vehicle7d(),
}


@pytest.mark.parametrize("name", list(FULL))
def test_full_size_first_step_sampled(orc, name):
    """One Bellman step (k = T_d) at full size in the bench's launch shape,
    checked at sampled states, each computed by the oracle on its own."""
    p = FULL[name]().with_(horizon=1)
    say(f"[full-step] {name}: n_x={p.n_x} n_u={p.n_u}")
    V, pol, _ = gpu_solve(p)
    rng = np.random.default_rng(11)
    states = np.unique(np.concatenate([rng.integers(0, p.n_x, 300), [0, p.n_x - 1]]))
    Vr, pr, gap = orc.step(p, states)
    err = float(np.abs(V[states] - Vr).max())
    assert err <= TOL_FP32, f"{name}: {err}"
    clear = gap > 2 * TOL_FP32
    assert np.array_equal(pol[0][states][clear], pr[clear])
    say(f"[full-step] {name}: max err {err:.2e} over {len(states)} states")


@pytest.mark.parametrize("name", ["unicycle-100x100x60", "room5-20^5"])
def test_full_size_fp32_vs_fp64_and_invariants(name):
    """Whole horizon at full size: FP32 within 1e-5 of the plain FP64 path,
    values in [0, 1] and monotone in the horizon."""
    p = FULL[name]()
    say(f"[full] {name}: fp32 vs fp64, T_d={p.horizon}")
    v32, _, i32 = gpu_solve(p.with_(precision="fp32"), policy=False)
    v64, _, i64 = gpu_solve(p.with_(precision="fp64"), policy=False)
    err = float(np.abs(v32 - v64).max())
    say(f"[full] {name}: max |fp32 - fp64| = {err:.2e}; sweeps {i32['t_sweeps_ms']:.1f} ms vs "
        f"{i64['t_sweeps_ms']:.1f} ms")
    assert err <= TOL_FP32
    assert v64.min() >= 0.0 and v64.max() <= 1.0 + 1e-12
    shorter, _, _ = gpu_solve(p.with_(precision="fp64", horizon=p.horizon // 2), policy=False)
    sign = -1.0 if p.spec == "safety" else 1.0
    assert np.all(sign * (v64 - shorter) >= -1e-12)


def test_full_size_separable_5d(orc):
    """20^5 grid, diagonal linear dynamics, one input, safety: the 5-D GPU
    value is the product of five 1-D oracle values."""
    a = [0.95, 0.9, 1.0, 0.92, 0.97]
    c = [0.03, -0.02, 0.0, 0.05, -0.01]
    lo, h, cnt = W.tiling((-1.0,) * 5, (1.0,) * 5, (20,) * 5)
    var = (0.05 ** 2, 0.04 ** 2, 0.06 ** 2, 0.05 ** 2, 0.03 ** 2)
    p = W.Problem(lo=lo, h=h, count=cnt, u_lo=(0.0,), u_hi=(0.0,), u_count=(1,), dyn="affine",
                  params=W.affine_params(np.diag(a), np.zeros((5, 1)), c), var=var, cutoff=1e-5,
                  horizon=12, spec="safety", precision="fp64", mode="otf", name="separable5")
    say("[separable] 20^5 product identity")
    V, _, _ = gpu_solve(p, policy=False)
    prod = np.ones(1)
    for i in range(5):
        p1 = W.Problem(lo=(lo[i],), h=(h[i],), count=(20,), u_lo=(0.0,), u_hi=(0.0,), u_count=(1,),
                       dyn="affine", params=W.affine_params([[a[i]]], [[0.0]], [c[i]]), var=(var[i],),
                       cutoff=1e-5, horizon=12, spec="safety")
        prod = np.multiply.outer(prod, orc.solve(p1)["V"])
    err = float(np.abs(V - prod.ravel()).max())
    assert err <= TOL_FP64, err
    v32, _, _ = gpu_solve(p.with_(precision="fp32"), policy=False)
    assert float(np.abs(v32 - prod.ravel()).max()) <= TOL_FP32


@pytest.mark.parametrize("name", ["unicycle-patch-fp32-otf", "unicycle-patch-fp64-otf", "room-patch-fp32-otf",
                                  "linear2d-full-fp32-otf", "room-patch-fp64-otf", "room-8^5-fp32-otf",
                                  "room-8^5-fp64-otf", "room-8^5-coupled-fp32", "room-8^5-safebox-fp32",
                                  "vehicle7-planes-fp32",
                                  "vehicle7-planes-tau0.3-fp32", "vehicle7-planes8-fp32",
                                  "vehicle7-planes8-tau0.3-fp32", "vehicle7-planes8-fp64"])
def test_fixed_shape_kernel_matches_generic(name):
    """The compiled-window-shape sweep does the generic sweep's arithmetic in
    the same order: results are bitwise equal."""
    import paper_2005_06191_amd as A
    p = CASES[name]().with_(horizon=4)
    assert A.query(p)["variant"] in ("fixed", "factored")
    say(f"[fixed vs lanes] {name}")
    a = A.solve(p, variant="fixed")
    b = A.solve(p, variant="lanes")
    assert a.info["variant"] == "fixed" and b.info["variant"] == "lanes"
    assert np.array_equal(a.V.cpu().numpy(), b.V.cpu().numpy())
    assert np.array_equal(a.policy.cpu().numpy(), b.policy.cpu().numpy())
    assert a.info["max_row_tail"] == b.info["max_row_tail"]


@pytest.mark.parametrize("name", ["unicycle-patch-fp32-otf", "unicycle-patch-fp64-otf", "unicycle-patch-reach-fp32",
                                  "unicycle-patch-fast-fp32", "unicycle-even-fp32", "unicycle-even-fast-fp32",
                                  "unicycle-y26-fp32", "unicycle-patch-intersect-fp64",
                                  "unicycle-even-intersect-fp32"])
def test_factored_sweep_matches_oracle_and_fixed(orc, name):
    """The factored sweep shares the outer contraction between inputs that
    differ only in the last digit: the window sum is re-associated, so it is
    checked against the oracle at the precision's tolerance and against the
    compiled-shape sweep at the same tolerance; the FP64 tail is the same."""
    import paper_2005_06191_amd as A
    p = CASES[name]()
    tol = TOL_FP64 if p.precision == "fp64" else TOL_FP32
    say(f"[factored] {name}")
    a = A.solve(p, variant="factored")
    assert a.info["variant"] == "factored"
    V, pol = a.V.cpu().numpy(), a.policy.cpu().numpy()
    ref = orc.solve(p, gap=True)
    compare(p, ref, V, pol, tol, gap=ref["gap"])
    b = A.solve(p, variant="fixed")
    assert float(np.abs(V - b.V.cpu().numpy()).max()) <= tol
    assert a.info["max_row_tail"] == b.info["max_row_tail"]


def test_factored_shared_tables_edges(orc):
    """The steps after the first read shared relative tables: states whose
    windows are clipped at every grid edge (a patch on which x, y and the
    heading all reach both ends), with and without the tail step, match the
    oracle; T_d = 1 without info uses the shared tables on its only step."""
    import paper_2005_06191_amd as A
    p = _uni_small(precision="fp32").with_(horizon=5, spec="safety")
    say("[factored] shared tables at the grid edges")
    assert A.query(p)["variant"] == "factored"
    ref = orc.solve(p, gap=True)
    r = A.solve(p, variant="factored", info=True)
    compare(p, ref, r.V.cpu().numpy(), r.policy.cpu().numpy(), TOL_FP32, gap=ref["gap"])
    r2 = A.solve(p, variant="factored", info=False)
    compare(p, ref, r2.V.cpu().numpy(), None, TOL_FP32)
    q = p.with_(horizon=1)
    r1 = A.solve(q, variant="factored", info=False, policy=False)
    compare(q, orc.solve(q), r1.V.cpu().numpy(), None, TOL_FP32)
    q64 = p.with_(precision="fp64", horizon=3)
    r64 = A.solve(q64, variant="factored", info=False, policy=False)
    compare(q64, orc.solve(q64), r64.V.cpu().numpy(), None, TOL_FP64)


def test_factored_full_size_vs_fixed():
    import paper_2005_06191_amd as A
    p = W.unicycle3d().with_(horizon=6)
    say("[factored] unicycle 100x100x60, T_d = 6, vs fixed")
    a = A.solve(p, variant="factored", policy=False)
    b = A.solve(p, variant="fixed", policy=False)
    assert a.info["variant"] == "factored"
    assert float(np.abs(a.V.cpu().numpy() - b.V.cpu().numpy()).max()) <= TOL_FP32
    q = p.with_(precision="fp64")
    a = A.solve(q, variant="factored", policy=False)
    b = A.solve(q, variant="fixed", policy=False)
    assert float(np.abs(a.V.cpu().numpy() - b.V.cpu().numpy()).max()) <= TOL_FP64


def test_vehicle7_full_fixed_vs_generic_first_step():
    import paper_2005_06191_amd as A
    p = W.vehicle7d().with_(horizon=2)
    say("[fixed vs lanes] vehicle7 full, T_d=2")
    a = A.solve(p, variant="fixed", policy=False)
    b = A.solve(p, variant="lanes", policy=False)
    assert np.array_equal(a.V.cpu().numpy(), b.V.cpu().numpy())


# ------------------------------------- full sizes against the oracle itself

@pytest.fixture(scope="module")
def uni_oracle(orc):
    """The oracle's whole-horizon solve of the unicycle workload at full size
    (600,000 states x 45 inputs x 16 steps; about a minute on 16 threads)."""
    p = W.unicycle3d(precision="fp64")
    say(f"[oracle] full unicycle solve: {p.rows * p.horizon:.3g} row-updates ...")
    return p, orc.solve(p, gap=True)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,mode", [("fp32", "otf"), ("fp64", "otf"), ("fp32", "stored")])
def test_full_size_unicycle_whole_horizon_vs_oracle(uni_oracle, prec, mode):
    """Every state of the 100 x 100 x 60 unicycle workload after all 16 steps,
    in the bench's launch configuration (FP32 and FP64 on the fly, FP32 with
    the 5.4 GB of stored rows), against the oracle's own full solve."""
    p0, ref = uni_oracle
    p = p0.with_(precision=prec, mode=mode)
    tol = TOL_FP64 if prec == "fp64" else TOL_FP32
    say(f"[full-oracle] unicycle {prec} {mode}")
    V, pol, info = gpu_solve(p)
    err = compare(p, ref, V, pol, tol, gap=ref["gap"])
    assert abs(info["max_row_tail"] - ref["max_tail"]) <= 1e-13 + 1e-9 * ref["max_tail"]
    say(f"[full-oracle] unicycle {prec} {mode} ({info['variant']}): max |V - V_oracle| = {err:.2e}")


def _chained(orc, p, n_states=1000, seed=3):
    """The last Bellman step at full size against the oracle: the plain FP64
    GPU path solves the problem with one step fewer (its V at k = 1 is V_2 of
    the full horizon); the oracle takes step k = 1 from that vector at
    sampled states, each on its own, and the GPU's full-horizon V_1 and
    policy of step 1 (FP32 and FP64) are compared with it.  The FP32 solve
    runs every step in FP32, so its error includes that of all T_d steps."""
    Vn, _, _ = gpu_solve(p.with_(precision="fp64", horizon=p.horizon - 1), policy=False)
    rng = np.random.default_rng(seed)
    states = np.unique(np.concatenate([rng.integers(0, p.n_x, n_states), [0, p.n_x - 1]]))
    Vr, pr, gap = orc.step(p.with_(precision="fp64"), states, V_next=Vn)
    out = {}
    for prec, tol in (("fp32", TOL_FP32), ("fp64", TOL_FP64)):
        V, pol, info = gpu_solve(p.with_(precision=prec))
        err = float(np.abs(V[states] - Vr).max())
        assert err <= tol, f"{p.name} {prec}: {err:.3e} > {tol:.1e}"
        clear = gap > 2 * tol
        bad = int((pol[0][states][clear] != pr[clear]).sum())
        assert bad == 0, f"{p.name} {prec}: {bad} policy entries differ"
        out[prec] = (err, info["variant"])
    return out, len(states)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["room5-20^5", "vehicle7-8^7", "unicycle-100x100x60"])
def test_full_size_last_step_chained_vs_oracle(orc, name):
    p = FULL[name]()
    say(f"[chained] {name}: n_x={p.n_x} n_u={p.n_u} T_d={p.horizon}")
    out, n = _chained(orc, p)
    say(f"[chained] {name}: over {n} states max err fp32 {out['fp32'][0]:.2e} ({out['fp32'][1]}), "
        f"fp64 {out['fp64'][0]:.2e} ({out['fp64'][1]})")
