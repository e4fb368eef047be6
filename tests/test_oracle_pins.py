"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check uses printed
values from the paper, textbook values, closed forms evaluated with mpmath,
an independent dense re-implementation (oracle/brute.py), or invariants that
a dropped term, a wrong sign or index, or a transposed operand would break.
"""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

import workloads as W
from oracle import brute

GOLD = os.path.join(os.path.dirname(__file__), "golden")
mp.mp.dps = 50


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ----------------------------------------------------------------- 1-D masses

def test_mass1d_textbook(orc):
    for c in gold("normal_mass.json")["cases"]:
        assert abs(orc.mass1d(c["a"], c["b"]) - c["mass"]) < 5e-16


def test_mass1d_vs_mpmath_tails_and_centre(orc):
    # relative accuracy across the body and far tails (erfc differencing)
    zs = [-38, -20, -9.5, -6, -3.3, -1.7, -0.8, -0.25, -1e-3, 0.0, 2e-3, 0.3, 0.9, 1.8,
          3.1, 5.5, 8.0, 12.0, 25.0, 37.5]
    for a in zs:
        for w in (1e-6, 0.01, 0.4, 2.5, 7.0):
            b = a + w
            # reference from the lower tails (mpmath's 50 digits cannot hold
            # 1 - 1e-138, so the upper side is mirrored)
            ref = mp.ncdf(-a) - mp.ncdf(-b) if a >= 0 else mp.ncdf(b) - mp.ncdf(a)
            got = orc.mass1d(a, b)
            if ref < 1e-300:
                assert got >= 0.0 and got < 1e-290
                continue
            # a difference of two tail values is as accurate as the tails it
            # subtracts; a tail's relative error grows like z^2 * ulp because
            # the argument a/sqrt(2) is itself rounded (condition of erfc)
            tails = sum((4 + z * z) * mp.ncdf(-abs(z)) for z in (a, b))
            tol = 2e-13 * float(ref) + 4e-16 * float(tails) + 1e-300
            assert abs(got - float(ref)) <= tol, (a, b, got, ref)


def test_mass1d_zero_width_and_symmetry(orc):
    for a in (-4.0, -0.5, 0.0, 0.7, 6.0):
        assert orc.mass1d(a, a) == 0.0
        assert orc.mass1d(a, a + 1.3) == pytest.approx(orc.mass1d(-a - 1.3, -a), rel=1e-14)


# ----------------------------------------------------- cutoff and window rule

@pytest.mark.parametrize("var,gamma", [(0.75, 1e-3), (0.01, 1e-6), (0.0025, 1e-4),
                                       (0.0004, 1e-4), (0.0004, 1e-5), (2.0, 0.05)])
def test_xstar_solves_density_equation(orc, var, gamma):
    xs = orc.xstar(var, gamma)
    s = mp.sqrt(var)
    pdf = mp.exp(-mp.mpf(xs) ** 2 / (2 * var)) / (s * mp.sqrt(2 * mp.pi))
    assert abs(pdf - gamma) <= 1e-13 * gamma
    assert abs(xs - brute.xstar(var, gamma)) < 1e-12


def test_xstar_limits(orc):
    assert math.isinf(orc.xstar(0.3, 0.0))
    # cutoff at or above the density peak has no cutting point
    peak = 1.0 / math.sqrt(2 * math.pi * 0.3)
    assert orc.xstar(0.3, peak * 1.0001) < 0


def test_paper_grid_counts():
    """Grid convention pinned by the sizes printed in Sec. 7 and Table 4."""
    for c in gold("paper_sizes.json")["cases"]:
        _, _, cx = W.grid_from_quantization(c["x_lb"], c["x_ub"], c["x_q"])
        _, _, cu = W.inputs_from_quantization(c["u_lb"], c["u_ub"], c["u_q"])
        assert int(np.prod(cx)) * int(np.prod(cu)) == c["pairs"], c["name"]


def test_table4_robot_memory_pins_window_rule(orc):
    """Table 4: stored - OFA memory = pairs * W * 4 B with W = L^2 and
    L = floor(2 x*/h) + 1 from the 1-D density reading of the cutoff."""
    g = gold("table4_robot_memory.json")
    xs = orc.xstar(g["var"][0], g["cutoff"])
    L = int(math.floor(2 * xs / g["x_q"])) + 1
    assert L == 13
    mib = g["pairs"] * L * L * g["bytes_per_entry"] / 2 ** 20
    assert abs(mib + g["mem_ofa_MB"] - g["mem_stored_MB"]) < 0.02
    # the oracle's cell-by-cell window realises exactly L or L-1 cells
    p = W.robot2d_paper()
    counts = set()
    for off in np.linspace(0.0, 0.5, 23):
        mu = np.array([0.0 + off, 0.1 - off])
        ok, lo, hi = orc.window(p, mu)
        assert ok
        counts.update((hi - lo + 1).tolist())
    assert counts <= {L, L - 1} and L in counts


def test_window_is_centre_in_interval(orc):
    p = W.linear2d(cells=50)
    rng = np.random.default_rng(1)
    xs = orc.xstar(p.var[0], p.cutoff)
    for _ in range(50):
        mu = rng.uniform(-1.3, 1.3, size=2)
        ok, lo, hi = orc.window(p, mu)
        for i in range(2):
            c = p.lo[i] + (np.arange(p.count[i]) + 0.5) * p.h[i]
            kept = np.nonzero(np.abs(c - mu[i]) <= xs)[0]
            if len(kept) == 0:
                assert not ok
            else:
                assert lo[i] == kept[0] and hi[i] == kept[-1]


# ----------------------------------------------------------------- dynamics

@pytest.mark.parametrize("prob", [W.linear2d(cells=6), W.unicycle3d(nxy=5, ntheta=4),
                                  W.room5d(cells=3), W.room5d(cells=3, n=3),
                                  W.vehicle7d(cells=3)])
def test_mean_matches_independent_transcription(orc, prob):
    rng = np.random.default_rng(7)
    X = brute.states(prob)
    U = brute.inputs(prob)
    for _ in range(40):
        x = X[rng.integers(len(X))]
        u = U[rng.integers(len(U))]
        a = orc.mean(prob, x, u)
        b = brute.mean(prob, x, u)
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12), (prob.dyn, x, u, a, b)


# -------------------------------------------------------- row masses / tail

def test_row_mass_telescopes(orc):
    """sum over kept cells (cell by cell) + tail = grid mass, with the grid
    mass evaluated here in 50 digits."""
    for prob in (W.linear2d(cells=20), W.unicycle3d(nxy=12, ntheta=10), W.room5d(cells=6)):
        rng = np.random.default_rng(3)
        X = brute.states(prob)
        U = brute.inputs(prob)
        for _ in range(6):
            s = int(rng.integers(prob.n_x))
            u = int(rng.integers(prob.n_u))
            tot, tail = orc.row_mass(prob, s, u)
            mu = brute.mean(prob, X[s], U[u])
            grid = mp.mpf(1)
            for i in range(prob.n):
                sg = math.sqrt(prob.var[i])
                grid *= brute.cell_mass(prob.lo[i], prob.lo[i] + prob.count[i] * prob.h[i], mu[i], sg)
            assert abs(tot + tail - float(grid)) < 1e-14
            assert tail >= -1e-15


def test_dense_row_matches_brute(orc):
    prob = W.unicycle3d(nxy=7, ntheta=6).with_(var=(0.9, 0.9, 0.3), cutoff=0.02, u_count=(2, 3))
    T = brute.dense_T(prob)
    for s in (0, 17, 100, prob.n_x - 1):
        for u in (0, 4, prob.n_u - 1):
            row = orc.row_dense(prob, s, u)
            assert np.abs(row - T[s * prob.n_u + u]).max() < 1e-15


# ---------------------------------------------------------- value iteration

def _tiny_cases():
    lin = W.linear2d(cells=5, horizon=3).with_(u_count=(3,), var=(0.09, 0.05), cutoff=0.05)
    uni = W.unicycle3d(nxy=5, ntheta=4, horizon=3).with_(u_count=(2, 3), var=(2.0, 2.0, 0.5),
                                                           cutoff=0.01)
    uni_ra = uni.with_(target=W.box((1.0, 1.0), (5.0, 5.0), 3), avoid=W.box((-5, -5), (-2, -2), 3))
    room = W.room5d(cells=3, n=3, horizon=2).with_(u_count=(3,), var=(0.4 ** 2,) * 3, cutoff=0.05)
    reach = lin.with_(spec="reach", target=W.box((0.2, 0.2), (1, 1), 2), horizon=4)
    ra = lin.with_(spec="reach_avoid", target=W.box((0.2, 0.2), (1, 1), 2),
                   avoid=W.box((-1, -1), (-0.5, 0.1), 2), horizon=4)
    safe_box = lin.with_(safe=W.box((-0.7, -1), (1, 0.9), 2))
    return [lin, uni_ra, room, reach, ra, safe_box]


@pytest.mark.parametrize("idx", range(6))
def test_oracle_matches_dense_serial_algorithm(orc, idx):
    prob = _tiny_cases()[idx]
    Vb, pb = brute.synthesize(prob)
    r = orc.solve(prob, gap=True)
    assert np.abs(Vb - r["V"]).max() < 1e-14
    assert 0.0 < r["V"].max() <= 1.0
    # policies agree wherever the maximiser is unique
    clear = r["gap"] > 1e-12
    assert np.array_equal(pb[clear], r["policy"][clear])


def test_oracle_no_cut_matches_dense(orc):
    prob = _tiny_cases()[0].with_(cutoff=0.0)
    Vb, _ = brute.synthesize(prob, cut=False)
    assert np.abs(Vb - orc.solve(prob)["V"]).max() < 1e-14


@pytest.mark.parametrize("idx", [0, 3, 4])
def test_bellman_optimality_by_policy_enumeration(orc, idx):
    prob = _tiny_cases()[idx].with_(horizon=2)
    prob = prob.with_(count=(2, 2), lo=(-1.0, -1.0), h=(1.0, 1.0), u_count=(2,),
                      var=(0.6, 0.8))
    best = brute.best_over_policies(prob)
    V = orc.solve(prob)["V"]
    assert np.abs(best - V).max() < 1e-13


def test_single_step_closed_form(orc):
    """T_d = 1, gamma = 0, safety on the whole grid:
    V_1(x) = max_u prod_i [Phi((hi_i - mu_i)/s_i) - Phi((lo_i - mu_i)/s_i)]."""
    prob = W.room5d(cells=4, n=3, horizon=1).with_(cutoff=0.0, var=(0.3 ** 2,) * 3)
    V = orc.solve(prob)["V"]
    X, U = brute.states(prob), brute.inputs(prob)
    rng = np.random.default_rng(5)
    for s in rng.integers(0, prob.n_x, size=12):
        best = 0.0
        for u in U:
            mu = brute.mean(prob, X[s], u)
            v = mp.mpf(1)
            for i in range(prob.n):
                sg = math.sqrt(prob.var[i])
                v *= brute.cell_mass(prob.lo[i], prob.lo[i] + prob.count[i] * prob.h[i], mu[i], sg)
            best = max(best, float(v))
        assert abs(V[s] - best) < 1e-14


def test_separable_product_identity(orc):
    """Diagonal linear dynamics, one input, safety on the whole grid: the
    n-D value is the product of the 1-D values, for any horizon."""
    A = np.diag([0.93, 1.02, 0.88])
    c = np.array([0.02, -0.03, 0.05])
    lo, h, cnt = W.tiling((-1, -1, -1), (1, 1, 1), (9, 7, 8))
    var = (0.03, 0.05, 0.02)
    prob = W.Problem(lo=lo, h=h, count=cnt, u_lo=(0.0,), u_hi=(0.0,), u_count=(1,),
                     dyn="affine", params=W.affine_params(A, np.zeros((3, 1)), c), var=var,
                     cutoff=1e-3, horizon=5, spec="safety")
    V = orc.solve(prob)["V"].reshape(cnt)
    parts = []
    for i in range(3):
        p1 = W.Problem(lo=(lo[i],), h=(h[i],), count=(cnt[i],), u_lo=(0.0,), u_hi=(0.0,),
                       u_count=(1,), dyn="affine",
                       params=W.affine_params([[A[i, i]]], [[0.0]], [c[i]]), var=(var[i],),
                       cutoff=1e-3, horizon=5, spec="safety")
        parts.append(orc.solve(p1)["V"])
    prod = parts[0][:, None, None] * parts[1][None, :, None] * parts[2][None, None, :]
    assert np.abs(V - prod).max() < 1e-14


def test_deterministic_limit_is_graph_reachability(orc):
    """Noise far below the cell width: T is the indicator of the cell holding
    mu, and safety / reach values become 0/1 reachability on the successor
    graph, computed here by plain dynamic programming on integers."""
    lo, h, cnt = W.tiling((-1, -1), (1, 1), (12, 12))
    A = np.array([[1.0, 0.0], [0.0, 1.0]])
    B = np.array([[1.0 / 6.0 + 1e-3, 0.0], [0.0, 1.0 / 6.0 + 1e-3]])
    prob = W.Problem(lo=lo, h=h, count=cnt, u_lo=(-1.0, -1.0), u_hi=(1.0, 1.0), u_count=(3, 3),
                     dyn="affine", params=W.affine_params(A, B), var=((1e-4 * h[0]) ** 2,) * 2,
                     cutoff=0.0, horizon=6, spec="reach_avoid",
                     target=W.box((0.5, 0.5), (1, 1), 2), avoid=W.box((-0.2, -1), (0.1, 0.4), 2))
    X, U = brute.states(prob), brute.inputs(prob)
    lab = brute.labels(prob)
    succ = np.full((prob.n_x, prob.n_u), -1)
    for s, x in enumerate(X):
        for k, u in enumerate(U):
            mu = brute.mean(prob, x, u)
            j = np.floor((mu - np.array(lo)) / np.array(h)).astype(int)
            if np.all(j >= 0) and np.all(j < np.array(cnt)):
                succ[s, k] = j[0] * cnt[1] + j[1]
    win = (lab == 2).astype(int)
    for _ in range(prob.horizon):
        nxt = win.copy()
        for s in range(prob.n_x):
            if lab[s] == 0:
                nxt[s] = int(any(succ[s, k] >= 0 and win[succ[s, k]] for k in range(prob.n_u)))
        win = nxt
    V = orc.solve(prob)["V"]
    assert np.abs(V - win).max() < 1e-9
    assert 0 < win.sum() < prob.n_x


def test_values_in_range_and_monotone_in_horizon(orc):
    base = W.unicycle3d(nxy=10, ntheta=8).with_(u_count=(3, 3))
    for spec, sign in (("safety", -1), ("reach", +1), ("reach_avoid", +1)):
        prev = None
        for T in (0, 1, 2, 4, 6):
            V = orc.solve(base.with_(spec=spec, horizon=T))["V"]
            assert V.min() >= 0.0 and V.max() <= 1.0 + 1e-15
            if prev is not None:
                assert np.all(sign * (V - prev) >= -1e-15), spec
            prev = V


def test_cutoff_error_bound(orc):
    """V_gamma <= V_{gamma=0} <= V_gamma + E, E = T_d * max row tail."""
    for prob in (W.linear2d(cells=16).with_(cutoff=0.3, horizon=6),
                 _tiny_cases()[4].with_(cutoff=0.4, count=(9, 9), h=(2 / 9, 2 / 9))):
        r = orc.solve(prob)
        full = orc.solve(prob.with_(cutoff=0.0))["V"]
        assert r["E"] > 1e-6  # the cut actually removes mass here
        assert np.all(r["V"] <= full + 1e-14)
        assert np.all(full <= r["V"] + r["E"] + 1e-14)


def test_step_equals_solve_first_step(orc):
    prob = _tiny_cases()[4].with_(count=(11, 9), h=(2 / 11, 2 / 9), horizon=1)
    r = orc.solve(prob)
    V, pol, _ = orc.step(prob, np.arange(prob.n_x))
    assert np.array_equal(V, r["V"])
    assert np.array_equal(pol, r["policy"][0])


def test_labels_and_fixed_values(orc):
    prob = _tiny_cases()[4]
    assert np.array_equal(orc.labels(prob), brute.labels(prob))
    r = orc.solve(prob)
    lab = brute.labels(prob)
    assert np.all(r["V"][lab == 2] == 1.0) and np.all(r["V"][lab == 1] == 0.0)
    assert np.all(r["policy"][:, lab != 0] == -1)


def test_policy_ties_go_to_the_lowest_input(orc):
    """Reading of the argmax (Alg. 4's collect step names no tie rule): among
    inputs with exactly equal values the lowest index wins.  Inputs that do
    not enter the dynamics tie exactly everywhere."""
    p = W.linear2d(cells=12, precision="fp64", mode="otf").with_(
        params=W.affine_params([[0.9, 0.05], [0.0, 0.9]], [[0.0], [0.0]]), u_count=(4,), horizon=3)
    r = orc.solve(p)
    lab = orc.labels(p)
    free = lab == 0
    assert free.any()
    assert np.all(r["policy"][:, free] == 0)
