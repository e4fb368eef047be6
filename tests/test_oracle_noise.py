"""Pins of the oracle's other noise models and window rules (CPU only).

Sec. 3 (after Eq. 3.2) and Sec. 6.2: besides the normal density the method
takes uniform, exponential and beta noise, with the cut tuned to the
support of the density, and multiplicative noise Upsilon = varsigma x with
the cut disabled.  The oracle's 1-D masses are pinned against library
routines it does not use (scipy's distribution functions and regularised
incomplete beta) and against exact values; its window rules against their
definitions; its whole solve against the one-step closed form and Alg. 3's
dense form written independently with mpmath.
"""
import math

import numpy as np
import pytest
from scipy import special, stats

import workloads as W
from oracle import brute


def _p1(noise="uniform", a=-0.15, b=0.15, al=1.0, be=1.0, var=0.01, window="centre", mult=False, cells=20,
        lo=-1.0, hi=1.0, cutoff=0.0, horizon=1, spec="safety", A=0.9, c=0.0):
    lo_, h, cnt = W.tiling((lo,), (hi,), (cells,))
    return W.Problem(lo=lo_, h=h, count=cnt, u_lo=(-0.2,), u_hi=(0.2,), u_count=(3,), dyn="affine",
                     params=W.affine_params([[A]], [[1.0]], [c]), var=(var,), cutoff=cutoff, horizon=horizon,
                     spec=spec, noise=noise, window=window, multiplicative=mult, noise_a=(a,), noise_b=(b,),
                     noise_alpha=(al,), noise_beta=(be,), name=f"{noise}-1d")


def test_uniform_masses_are_exact_fractions(orc):
    """Uniform noise on [-0.15, 0.15] over cells of width 0.1 with the mean
    at a cell centre: the support covers exactly three cells, 1/3 each."""
    p = _p1(a=-0.15, b=0.15)
    # offsets of the cell edges from the mean at a centre: -0.25, -0.15, -0.05, 0.05, 0.15, 0.25
    e = [-0.25, -0.15, -0.05, 0.05, 0.15, 0.25]
    m = [orc.noise_mass(p, 0, 0.0, e[k], e[k + 1]) for k in range(5)]
    assert m[0] == 0.0 and m[4] == 0.0
    assert abs(m[1] - 1 / 3) < 1e-15 and abs(m[2] - 1 / 3) < 1e-15 and abs(m[3] - 1 / 3) < 1e-15
    # a support edge inside a cell splits it linearly
    assert abs(orc.noise_mass(p, 0, 0.0, -0.2, -0.1) - (0.05 / 0.3)) < 1e-15


def test_exponential_masses_match_scipy(orc):
    lam = 7.5
    p = _p1(noise="exponential", a=lam, cutoff=1e-4)
    rng = np.random.default_rng(3)
    for _ in range(200):
        ta, tb = np.sort(rng.uniform(-0.3, 1.5, 2))
        want = stats.expon.cdf(tb, scale=1 / lam) - stats.expon.cdf(ta, scale=1 / lam)
        got = orc.noise_mass(p, 0, 0.0, ta, tb)
        assert abs(got - want) <= 1e-15 + 1e-13 * want
    # far tail: relative accuracy kept
    far = orc.noise_mass(p, 0, 0.0, 3.0, 3.1)
    assert abs(far - (math.exp(-lam * 3.0) - math.exp(-lam * 3.1))) <= 1e-14 * far


@pytest.mark.parametrize("al,be", [(1.0, 1.0), (2.0, 5.0), (1.5, 1.5), (4.0, 1.2)])
def test_beta_masses_match_the_regularised_incomplete_beta(orc, al, be):
    a, b = -0.2, 0.3
    p = _p1(noise="beta", a=a, b=b, al=al, be=be)
    rng = np.random.default_rng(5)
    total = orc.noise_mass(p, 0, 0.0, a - 0.1, b + 0.1)
    assert abs(total - 1.0) <= 1e-13
    for _ in range(60):
        ta, tb = np.sort(rng.uniform(a - 0.05, b + 0.05, 2))
        ya, yb = [min(max((t - a) / (b - a), 0.0), 1.0) for t in (ta, tb)]
        want = special.betainc(al, be, yb) - special.betainc(al, be, ya)
        assert abs(orc.noise_mass(p, 0, 0.0, ta, tb) - want) <= 1e-13


def test_multiplicative_normal_scale_and_point_mass(orc):
    p = _p1(noise="normal", var=0.04, mult=True)
    for xi in (-1.3, 0.4, 2.0):
        s = 0.2 * abs(xi)
        for ta, tb in ((-0.1, 0.05), (0.3, 0.9), (-2.0, -0.5)):
            want = stats.norm.cdf(tb / s) - stats.norm.cdf(ta / s)
            assert abs(orc.noise_mass(p, 0, xi, ta, tb) - want) <= 1e-14
    # at a zero coordinate the noise vanishes: all the mass at the mean
    assert orc.noise_mass(p, 0, 0.0, -0.05, 0.05) == 1.0
    assert orc.noise_mass(p, 0, 0.0, 0.0, 0.1) == 1.0
    assert orc.noise_mass(p, 0, 0.0, -0.1, 0.0) == 0.0


def test_window_rules_by_definition(orc):
    """Centre rule: centres in [mu - x*, mu + x*]; intersect rule: cells
    whose open interval meets it; bounded supports always intersect."""
    rng = np.random.default_rng(9)
    for window in ("centre", "intersect"):
        p = _p1(noise="normal", var=0.03 ** 2, cutoff=1.0, window=window, cells=40)
        xs = orc.xstar(p.var[0], p.cutoff)
        for mu in rng.uniform(-1.2, 1.2, 40):
            ok, lo, hi = orc.window(p, [mu])
            edges = p.lo[0] + p.h[0] * np.arange(41)
            cen = 0.5 * (edges[:-1] + edges[1:])
            if window == "centre":
                keep = np.nonzero(np.abs(cen - mu) <= xs)[0]
            else:
                keep = np.nonzero((edges[1:] > mu - xs) & (edges[:-1] < mu + xs))[0]
            if len(keep) == 0:
                assert not ok
            else:
                assert ok and lo[0] == keep[0] and hi[0] == keep[-1]
    p = _p1(noise="uniform", a=-0.07, b=0.12, cells=40)
    for mu in rng.uniform(-0.9, 0.9, 40):
        ok, lo, hi = orc.window(p, [mu])
        edges = p.lo[0] + p.h[0] * np.arange(41)
        keep = np.nonzero((edges[1:] > mu - 0.07) & (edges[:-1] < mu + 0.12))[0]
        assert ok and lo[0] == keep[0] and hi[0] == keep[-1]


def test_intersect_keeps_more_and_cuts_less(orc):
    """The intersect window contains the centre window, so its truncated
    tail is never larger; both rows' kept masses telescope."""
    base = W.linear2d(cells=24, precision="fp64")
    for state in (0, 100, 287, 400):
        for u in range(base.n_u):
            kc, tc = orc.row_mass(base, state, u)
            ki, ti = orc.row_mass(base.with_(window="intersect"), state, u)
            assert ki >= kc - 1e-15 and ti <= tc + 1e-15


@pytest.mark.parametrize("noise,kw", [("uniform", dict(a=-0.12, b=0.2)),
                                      ("exponential", dict(a=6.0, cutoff=1e-3)),
                                      ("beta", dict(a=-0.15, b=0.1, al=2.0, be=3.0)),
                                      ("normal", dict(var=0.05 ** 2, mult=True)),
                                      ("normal", dict(var=0.05 ** 2, window="intersect", cutoff=0.5))])
def test_one_step_closed_form(orc, noise, kw):
    """T_d = 1 safety on the whole grid: V_1(x) = max_u of the mass of the
    grid around mu = f(x, u), by the library distribution functions, minus
    what the window drops (nothing for bounded supports)."""
    p = _p1(noise=noise, horizon=1, cells=25, **kw)
    V = orc.solve(p)["V"]
    lo, hi = p.lo[0], p.lo[0] + p.count[0] * p.h[0]
    us = np.linspace(-0.2, 0.2, 3)
    for j in range(p.count[0]):
        x = p.lo[0] + (j + 0.5) * p.h[0]
        best = 0.0
        for u in us:
            mu = 0.9 * x + u
            ta, tb = lo - mu, hi - mu
            if noise == "uniform":
                d = stats.uniform(loc=kw["a"], scale=kw["b"] - kw["a"])
                m = d.cdf(tb) - d.cdf(ta)
            elif noise == "exponential":
                tcut = math.log(kw["a"] / kw["cutoff"]) / kw["a"]
                # the window keeps the cells meeting [mu, mu + t*]
                jhi = math.ceil((mu + tcut - lo) / p.h[0]) - 1
                top = min(hi, lo + (jhi + 1) * p.h[0]) - mu
                m = stats.expon.cdf(min(tb, top), scale=1 / kw["a"]) - stats.expon.cdf(ta, scale=1 / kw["a"])
            elif noise == "beta":
                ya, yb = [min(max((t - kw["a"]) / (kw["b"] - kw["a"]), 0.0), 1.0) for t in (ta, tb)]
                m = special.betainc(kw["al"], kw["be"], yb) - special.betainc(kw["al"], kw["be"], ya)
            elif kw.get("mult"):
                s = 0.05 * abs(x)
                m = stats.norm.cdf(tb / s) - stats.norm.cdf(ta / s) if s > 0 else float(lo <= mu < hi)
            else:
                xs = 0.05 * math.sqrt(-2 * math.log(kw["cutoff"] * 0.05 * math.sqrt(2 * math.pi)))
                jl = max(0, math.floor((mu - xs - lo) / p.h[0]))
                jh = min(p.count[0] - 1, math.ceil((mu + xs - lo) / p.h[0]) - 1)
                a, b = lo + jl * p.h[0] - mu, lo + (jh + 1) * p.h[0] - mu
                m = stats.norm.cdf(b / 0.05) - stats.norm.cdf(a / 0.05) if jh >= jl else 0.0
            best = max(best, m)
        assert abs(V[j] - best) <= 1e-12, (noise, j, V[j], best)


@pytest.mark.parametrize("noise,kw", [("uniform", dict(noise_a=(-0.3, -0.2), noise_b=(0.25, 0.3))),
                                      ("exponential", dict(noise_a=(5.0, 8.0), cutoff=1e-2)),
                                      ("beta", dict(noise_a=(-0.3, -0.25), noise_b=(0.2, 0.3),
                                                    noise_alpha=(2.0, 1.5), noise_beta=(2.0, 3.0)))])
def test_dense_alg3_other_noise(orc, noise, kw):
    """Alg. 3 on a 5 x 4 grid, written independently (mpmath CDFs, dense
    matrices), against the oracle's recursion, reach-avoid over 3 steps."""
    lo, h, cnt = W.tiling((-1.0, -1.0), (1.0, 1.0), (5, 4))
    p = W.Problem(lo=lo, h=h, count=cnt, u_lo=(-0.3,), u_hi=(0.3,), u_count=(3,), dyn="affine",
                  params=W.affine_params([[0.9, 0.1], [0.0, 0.95]], [[0.0], [1.0]]), var=(0.01, 0.01),
                  cutoff=kw.pop("cutoff", 0.0), horizon=3, spec="reach_avoid",
                  target=W.box((0.2, 0.5), (1.0, 1.0), 2), avoid=W.box((-1.0, -1.0), (-0.5, -0.4), 2),
                  noise=noise, name=f"dense-{noise}", **kw)
    Vb, pb = brute.synthesize_noise(p)
    r = orc.solve(p, gap=True)
    assert np.abs(r["V"] - Vb).max() <= 1e-12
    clear = r["gap"] > 1e-9
    assert np.array_equal(r["policy"][clear], pb[clear])
