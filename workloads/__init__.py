"""Problem descriptions and seeded synthetic workload generators.

This module is shared by the HIP path's Python binding, the CPU oracle, the
tests and the benchmark.  It holds *descriptions* only (grids, input sets,
dynamics parameters, noise variances, cutoff, horizon, specification boxes)
and the seeded random draws that produce them.  None of the method's
arithmetic (cell masses, windows, Bellman updates) lives here.

Conventions (they follow the problem statement of the paper's Alg. 2 / Alg. 4:
state partition, input set, noise covariance, cutoff level, horizon, spec):

* State grid: dimension ``i`` has ``count[i]`` cells
  ``[lo[i] + j*h[i], lo[i] + (j+1)*h[i])``, ``j = 0..count[i]-1``; the
  representative point of a cell is its centre.  States are numbered
  row-major, the last dimension varying fastest.
* Inputs: dimension ``k`` is the inclusive linspace ``u_lo[k] .. u_hi[k]``
  with ``u_count[k]`` points (a single point is ``u_lo[k]``); the input set
  is their Cartesian product, numbered row-major (last dimension fastest).
* Noise: additive Gaussian with diagonal covariance; ``var[i]`` is the
  variance of dimension ``i`` (the paper writes the covariance as
  ``diag(0.75, 0.75)`` in its robot example, Sec. 7).
* ``cutoff`` is the cutting level gamma of Sec. 5.2 (0 means no cut).
* Boxes are closed hyper-rectangles ``(lo, hi)``; +-inf is allowed; a state
  belongs to a box when its cell centre does.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Sequence, Tuple

import numpy as np

INF = float("inf")

DYN_KINDS = ("affine", "unicycle", "room", "vehicle7", "robot", "user")
SPECS = ("safety", "reach", "reach_avoid")
MODES = ("auto", "stored", "otf")
PRECISIONS = ("fp64", "fp32")

Box = Tuple[Tuple[float, ...], Tuple[float, ...]]

# Parameter order of the 7-D single-track vehicle model (Sec. 8.4.1 of the
# paper): tau, wheelbase, mass, friction, l_f, l_r, h_cg, I_z, C_Sf, C_Sr, g.
VEHICLE7_BMW320I = (0.1, 2.5789, 1093.3, 1.0489, 1.156, 1.422, 0.6137,
                    1791.6, 20.89, 20.89, 9.81)


@dataclass
class Problem:
    lo: Tuple[float, ...]
    h: Tuple[float, ...]
    count: Tuple[int, ...]
    u_lo: Tuple[float, ...]
    u_hi: Tuple[float, ...]
    u_count: Tuple[int, ...]
    dyn: str
    params: Tuple[float, ...]
    var: Tuple[float, ...]
    cutoff: float
    horizon: int
    spec: str = "safety"
    target: Optional[Box] = None
    avoid: Optional[Box] = None
    safe: Optional[Box] = None
    mode: str = "auto"
    precision: str = "fp32"
    name: str = ""
    # disturbance set (Def. 3.1): dimension l is the inclusive linspace
    # w_lo[l] .. w_hi[l] with w_count[l] points; empty = no disturbance
    w_lo: Tuple[float, ...] = ()
    w_hi: Tuple[float, ...] = ()
    w_count: Tuple[int, ...] = ()
    # noise model (Sec. 3 and Sec. 6.2): "normal" (variances in var),
    # "uniform" on [noise_a, noise_b], "exponential" with rate noise_a,
    # "beta"(noise_alpha, noise_beta) on [noise_a, noise_b]; the window rule
    # ("centre" as in Sec. 5.2, or "intersect") and multiplicative normal
    # noise (Eq. 3.2: scale |x_i| times sqrt(var_i), no cut)
    noise: str = "normal"
    window: str = "centre"
    multiplicative: bool = False
    noise_a: Tuple[float, ...] = ()
    noise_b: Tuple[float, ...] = ()
    noise_alpha: Tuple[float, ...] = ()
    noise_beta: Tuple[float, ...] = ()
    # sweep variant the GPU library is asked for ("auto" lets it choose)
    variant: str = "auto"
    # dyn == "user": the right-hand side as source text, the body of
    # rhs(x, u, w, params, mu) (Sec. 3: f given as text)
    rhs: str = ""

    @property
    def n(self) -> int:
        return len(self.count)

    @property
    def m(self) -> int:
        return len(self.u_count)

    @property
    def n_x(self) -> int:
        return int(np.prod(self.count, dtype=np.int64))

    @property
    def n_u(self) -> int:
        return int(np.prod(self.u_count, dtype=np.int64))

    @property
    def p_dist(self) -> int:
        return len(self.w_count)

    @property
    def n_w(self) -> int:
        return int(np.prod(self.w_count, dtype=np.int64)) if self.w_count else 1

    @property
    def rows(self) -> int:
        """(state, input, disturbance) rows of Alg. 2."""
        return self.n_x * self.n_u * self.n_w

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def full_box(n: int) -> Box:
    return (tuple([-INF] * n), tuple([INF] * n))


def box(lo: Sequence[float], hi: Sequence[float], n: int) -> Box:
    """Box given on the leading ``len(lo)`` dimensions, unbounded after."""
    lo = list(lo) + [-INF] * (n - len(lo))
    hi = list(hi) + [INF] * (n - len(hi))
    return (tuple(float(v) for v in lo), tuple(float(v) for v in hi))


def grid_from_quantization(lb: Sequence[float], ub: Sequence[float],
                           q: Sequence[float]):
    """Cells for the paper's "quantization parameter" convention.

    The paper's representative points are the lattice ``lb + j*q`` including
    both ends of ``[lb, ub]`` (this reproduces the printed sizes of Sec. 7
    and Table 4).  As cells: ``lo = lb - q/2``, ``h = q`` and
    ``count = floor((ub - lb)/q + 1e-9) + 1``.  The small epsilon absorbs the
    binary rounding of ratios such as 0.6/0.1 = 5.999...
    """
    lo, h, cnt = [], [], []
    for a, b, s in zip(lb, ub, q):
        lo.append(float(a) - float(s) / 2.0)
        h.append(float(s))
        cnt.append(int(math.floor((float(b) - float(a)) / float(s) + 1e-9)) + 1)
    return tuple(lo), tuple(h), tuple(cnt)


def inputs_from_quantization(lb, ub, q):
    """Input lattice ``lb + j*q`` (both ends included) as inclusive linspaces."""
    _, _, cnt = grid_from_quantization(lb, ub, q)
    hi = tuple(float(a) + (c - 1) * float(s) for a, s, c in zip(lb, q, cnt))
    return tuple(float(a) for a in lb), hi, cnt


def tiling(lo: Sequence[float], hi: Sequence[float], cells: Sequence[int]):
    """``cells[i]`` equal cells tiling ``[lo[i], hi[i]]``."""
    h = tuple((float(b) - float(a)) / int(c) for a, b, c in zip(lo, hi, cells))
    return tuple(float(a) for a in lo), h, tuple(int(c) for c in cells)


def affine_params(A, B, c=None, D=None) -> Tuple[float, ...]:
    """Flatten ``x+ = A x + B u + c + D w`` (row-major A[n*n], B[n*m], c[n],
    then D[n*p] when there is a disturbance)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    n = A.shape[0]
    B = B.reshape(n, -1)
    c = np.zeros(n) if c is None else np.asarray(c, dtype=np.float64)
    out = A.ravel().tolist() + B.ravel().tolist() + c.ravel().tolist()
    if D is not None:
        out += np.asarray(D, dtype=np.float64).reshape(n, -1).ravel().tolist()
    return tuple(out)


# ---------------------------------------------------------------------------
# The five workloads.  Seeds are fixed: 20260 + workload number.
# ---------------------------------------------------------------------------

def linear2d(cells: int = 50, precision: str = "fp64", mode: str = "stored",
             horizon: int = 8) -> Problem:
    """2-D linear system on [-1,1]^2 (the small workload).

    x+ = A x + B u + w, A = [[0.9, 0.05], [0, 0.9]], B = [0, 1]^T,
    u in 5 values on [-0.5, 0.5], w ~ N(0, diag(0.1^2, 0.1^2)), cutoff 1e-6,
    safety on the whole domain, horizon 8.
    """
    lo, h, cnt = tiling((-1.0, -1.0), (1.0, 1.0), (cells, cells))
    return Problem(lo=lo, h=h, count=cnt, u_lo=(-0.5,), u_hi=(0.5,), u_count=(5,),
                   dyn="affine", params=affine_params([[0.9, 0.05], [0.0, 0.9]], [[0.0], [1.0]]),
                   var=(0.01, 0.01), cutoff=1e-6, horizon=horizon, spec="safety",
                   mode=mode, precision=precision, name=f"linear2d-{cells}x{cells}")


def unicycle3d(nxy: int = 100, ntheta: int = 60, precision: str = "fp32",
               mode: str = "otf", horizon: int = 16, nv: int = 5, nw: int = 9) -> Problem:
    """3-D unicycle, reach-avoid (the bench workload at full size).

    x+ = x + tau v cos(theta), y+ = y + tau v sin(theta),
    theta+ = theta + tau omega, tau = 0.1; v in 5 values on [0,1],
    omega in 9 values on [-1,1]; domain [-5,5]^2 x [-pi,pi] on
    100 x 100 x 60 cells; noise variances (0.05^2, 0.05^2, 0.02^2);
    cutoff 1e-4; target [3,5]^2, avoid [-1,1]^2; horizon 16.
    """
    lo, h, cnt = tiling((-5.0, -5.0, -math.pi), (5.0, 5.0, math.pi), (nxy, nxy, ntheta))
    return Problem(lo=lo, h=h, count=cnt, u_lo=(0.0, -1.0), u_hi=(1.0, 1.0), u_count=(nv, nw),
                   dyn="unicycle", params=(0.1,), var=(0.05 ** 2, 0.05 ** 2, 0.02 ** 2),
                   cutoff=1e-4, horizon=horizon, spec="reach_avoid",
                   target=box((3.0, 3.0), (5.0, 5.0), 3), avoid=box((-1.0, -1.0), (1.0, 1.0), 3),
                   mode=mode, precision=precision, name=f"unicycle3d-{nxy}x{nxy}x{ntheta}")


def room5d(cells: int = 20, n: int = 5, precision: str = "fp32", mode: str = "otf",
           horizon: int = 32, n_levels: int = 10) -> Problem:
    """Ring of ``n`` rooms with one shared heater, safety (5-D at full size).

    x_i+ = (1 - 2a - b - g u) x_i + a (x_{i-1} + x_{i+1}) + b T_e + g T_h u + w_i
    with a = 0.05, b = 0.005, g = 0.01, T_e = -1, T_h = 50; u in 10 levels on
    [0,1]; domain [19,21]^n with ``cells`` per dimension; noise 0.02^2 I;
    cutoff 1e-5; horizon 32.  Neighbours wrap around the ring.
    """
    lo, h, cnt = tiling((19.0,) * n, (21.0,) * n, (cells,) * n)
    return Problem(lo=lo, h=h, count=cnt, u_lo=(0.0,), u_hi=(1.0,), u_count=(n_levels,),
                   dyn="room", params=(0.05, 0.005, 0.01, -1.0, 50.0), var=(0.02 ** 2,) * n,
                   cutoff=1e-5, horizon=horizon, spec="safety",
                   mode=mode, precision=precision, name=f"room{n}d-{cells}^{n}")


def vehicle7d(cells: int = 8, precision: str = "fp32", mode: str = "otf",
              horizon: int = 32) -> Problem:
    """7-D single-track vehicle (parameters of the paper's BMW 320i study).

    Domain: the paper's box [-10,10]^2 x [-0.4,0.4] x [-2,2] x [-0.3,0.3] x
    [-0.4,0.4] x [-0.04,0.04] tiled by ``cells`` per dimension; inputs the
    paper's 5 x 5 lattice on [-0.4,0.4] x [-4,4]; noise sigma_i = 0.3 h_i;
    cutoff 1e-2; reach-avoid with target [-2.5,0] x [0,2.5] and avoid
    [-2.5,0] x [-2.5,0] on the position plane; horizon 32.
    """
    dom_lo = (-10.0, -10.0, -0.4, -2.0, -0.3, -0.4, -0.04)
    dom_hi = (10.0, 10.0, 0.4, 2.0, 0.3, 0.4, 0.04)
    lo, h, cnt = tiling(dom_lo, dom_hi, (cells,) * 7)
    var = tuple((0.3 * hh) ** 2 for hh in h)
    return Problem(lo=lo, h=h, count=cnt, u_lo=(-0.4, -4.0), u_hi=(0.4, 4.0), u_count=(5, 5),
                   dyn="vehicle7", params=VEHICLE7_BMW320I, var=var, cutoff=1e-2,
                   horizon=horizon, spec="reach_avoid",
                   target=box((-2.5, 0.0), (0.0, 2.5), 7), avoid=box((-2.5, -2.5), (0.0, 0.0), 7),
                   mode=mode, precision=precision, name=f"vehicle7d-{cells}^7")


def robot2d_paper(input_q: float = 0.2) -> Problem:
    """The paper's 2-D robot grid (Sec. 7), used only for size pins.

    X = [-10,10]^2 with quantization 0.5, U = [-1,1]^2 with quantization
    ``input_q``, covariance diag(0.75, 0.75), cutoff 1e-3.  The disturbance
    player is not modelled here; the dynamics are a stand-in.
    """
    lo, h, cnt = grid_from_quantization((-10, -10), (10, 10), (0.5, 0.5))
    ulo, uhi, ucnt = inputs_from_quantization((-1, -1), (1, 1), (input_q, input_q))
    return Problem(lo=lo, h=h, count=cnt, u_lo=ulo, u_hi=uhi, u_count=ucnt,
                   dyn="affine", params=affine_params(np.eye(2), np.eye(2)),
                   var=(0.75, 0.75), cutoff=1e-3, horizon=8, spec="safety", name="robot2d")


# ---------------------------------------------------------------------------
# Batch of 64 uneven systems and the serving stream.
# ---------------------------------------------------------------------------

def _loguniform(rng, a, b):
    return float(math.exp(rng.uniform(math.log(a), math.log(b))))


def batch_systems(count: int = 64, seed: int = 20264, cells_lo: float = 400.0,
                  cells_hi: float = 40000.0, cutoff: float = 1e-4) -> list:
    """Uneven 2-D linear / 3-D unicycle systems for one batched launch.

    Total cells ~ logU[cells_lo, cells_hi]; inputs ~ logU[3, 50]; position
    noise sigma ~ U[0.02, 0.2] (heading 0.4 sigma); horizons U{4..32}; spec
    uniform over safety / reach / reach-avoid with seeded target (0.3 x side)
    and disjoint avoid (0.2 x side) boxes.
    """
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        kind = "affine" if rng.uniform() < 0.5 else "unicycle"
        N = _loguniform(rng, cells_lo, cells_hi)
        n_u = int(round(_loguniform(rng, 3, 50)))
        sig = float(rng.uniform(0.02, 0.2))
        T = int(rng.integers(4, 33))
        spec = SPECS[int(rng.integers(0, 3))]
        if kind == "affine":
            side = max(2, int(round(math.sqrt(N))))
            lo, h, cnt = tiling((-1.0, -1.0), (1.0, 1.0), (side, side))
            a11, a22 = rng.uniform(0.8, 0.95, size=2)
            a12 = rng.uniform(-0.1, 0.1)
            params = affine_params([[a11, a12], [0.0, a22]], [[0.0], [1.0]])
            ulo, uhi, ucnt = (-0.5,), (0.5,), (max(1, n_u),)
            var = (sig * sig, sig * sig)
            dom_lo, dom_hi = (-1.0, -1.0), (1.0, 1.0)
            nd = 2
        else:
            nth = int(min(60, max(4, round(0.6 * N ** (1.0 / 3.0)))))
            nxy = max(2, int(round(math.sqrt(N / nth))))
            lo, h, cnt = tiling((-5.0, -5.0, -math.pi), (5.0, 5.0, math.pi), (nxy, nxy, nth))
            nv = max(1, int(round(math.sqrt(n_u / 1.8))))
            nw = max(1, int(round(n_u / nv)))
            ulo, uhi, ucnt = (0.0, -1.0), (1.0, 1.0), (nv, nw)
            params = (0.1,)
            var = (sig * sig, sig * sig, (0.4 * sig) ** 2)
            dom_lo, dom_hi = (-5.0, -5.0), (5.0, 5.0)
            nd = 3
        target = avoid = None
        if spec != "safety":
            side_x = dom_hi[0] - dom_lo[0]
            tw, aw = 0.3 * side_x, 0.2 * side_x
            tx, ty = rng.uniform(dom_lo[0], dom_hi[0] - tw, size=2)
            target = box((tx, ty), (tx + tw, ty + tw), nd)
            if spec == "reach_avoid":
                for _ in range(100):
                    ax, ay = rng.uniform(dom_lo[0], dom_hi[0] - aw, size=2)
                    if ax + aw < tx or ax > tx + tw or ay + aw < ty or ay > ty + tw:
                        break
                avoid = box((ax, ay), (ax + aw, ay + aw), nd)
        out.append(Problem(lo=lo, h=h, count=cnt, u_lo=ulo, u_hi=uhi, u_count=ucnt, dyn=kind,
                           params=params, var=var, cutoff=cutoff, horizon=T, spec=spec,
                           target=target, avoid=avoid, mode="otf", precision="fp32",
                           name=f"batch{s}-{kind}"))
    return out


def scaled_family(parent: Problem, n_x_target: float) -> Problem:
    """A member of a workload family with about ``n_x_target`` states.

    The domain is kept and the cell widths change; the noise is rescaled with
    the cells so that sigma/h (hence the window shape) and gamma*sigma (hence
    the cutoff's reach in sigma units) stay those of the parent.
    """
    n = parent.n
    scale = (n_x_target / parent.n_x) ** (1.0 / n)
    cnt = tuple(max(2, int(round(c * scale))) for c in parent.count)
    hi = tuple(a + c * hh for a, c, hh in zip(parent.lo, parent.count, parent.h))
    lo, h, cnt = tiling(parent.lo, hi, cnt)
    ratio = [hn / ho for hn, ho in zip(h, parent.h)]
    var = tuple(v * r * r for v, r in zip(parent.var, ratio))
    geo = float(np.prod(ratio)) ** (1.0 / n)
    return parent.with_(lo=lo, h=h, count=cnt, var=var, cutoff=parent.cutoff / geo,
                        name=f"{parent.name.split('-')[0]}-{'x'.join(map(str, cnt))}")


def serving_stream(count: int = 500, seed: int = 20265, qps: float = 10.0,
                   share_vehicle: float = 0.1, nx_lo: float = 1e3, nx_hi: float = 2e6):
    """Poisson arrivals of solve requests: (arrival_time_s, Problem) pairs.

    90% are drawn from the 2-D linear / 3-D unicycle / 5-D room families with
    state counts ~ logU[nx_lo, nx_hi]; the rest are the 7-D vehicle at 8 cells
    per dimension.  Every request is FP32; the mode is left to the server.
    """
    rng = np.random.default_rng(seed)
    parents = [linear2d(precision="fp32", mode="auto"), unicycle3d(mode="auto"),
               room5d(mode="auto")]
    t = 0.0
    out = []
    for r in range(count):
        t += float(rng.exponential(1.0 / qps))
        if rng.uniform() < share_vehicle:
            p = vehicle7d(mode="auto")
        else:
            parent = parents[int(rng.integers(0, len(parents)))]
            p = scaled_family(parent, _loguniform(rng, nx_lo, nx_hi))
        out.append((t, p.with_(name=f"req{r}-{p.name}")))
    return out


# ---------------------------------------------------------------------------
# Road traffic (Sec. 8.3.1) and the robot (Sec. 7), also as source text.
# ---------------------------------------------------------------------------

# Sec. 8.3.1: cells of 0.5 km, flow speed 100 km/h, sampling time 6.48 s,
# so a cell passes tau v / L = 0.36 of its vehicles on; a quarter of what
# leaves cells 1 and 3 takes the exit (q = 0.25); the lights admit 6 and 8
# vehicles.  Cell i receives from cell i - 1 (cell 1 from cell 5).
TRAFFIC_FLOW, TRAFFIC_EXIT = 0.36, 0.25

TRAFFIC5_RHS = """
const double a = params[0], q = params[1];
mu[0] = ((1.0 - a) * x[0] + a * x[4]) + 6.0 * u[0];
mu[1] = (1.0 - a - q) * x[1] + a * x[0];
mu[2] = ((1.0 - a) * x[2] + a * x[1]) + 8.0 * u[1];
mu[3] = (1.0 - a - q) * x[3] + a * x[2];
mu[4] = (1.0 - a) * x[4] + a * x[3];
"""

ROBOT_RHS = """
const double a = params[0] * u[0];
mu[0] = (x[0] + a * cos(u[1])) + w[0];
mu[1] = (x[1] + a * sin(u[1])) + w[0];
"""


def traffic5d(q: float = 0.37, precision: str = "fp32", horizon: int = 7, text: bool = False,
              var: float = 0.7, cutoff: float = 2e-2, lo=(0.0,) * 5, hi=(10.0,) * 5) -> Problem:
    """The 5-cell road traffic ring of Sec. 8.3.1: X = [0, 10]^5 quantised by
    0.37 (28 points per cell), the two lights in {0, 1}, noise covariance
    diag(0.7, ...), cutoff 2e-2, safety (density below 10 in every cell),
    horizon 7.  text=True gives the same model as source text (dyn "user")."""
    a, e = TRAFFIC_FLOW, TRAFFIC_EXIT
    A = np.zeros((5, 5))
    for i in range(5):
        A[i, i] = 1.0 - a - (e if i in (1, 3) else 0.0)
        A[i, (i - 1) % 5] = a
    B = np.zeros((5, 2))
    B[0, 0], B[2, 1] = 6.0, 8.0
    lo_, h, cnt = grid_from_quantization(lo, hi, (q,) * 5)
    p = Problem(lo=lo_, h=h, count=cnt, u_lo=(0.0, 0.0), u_hi=(1.0, 1.0), u_count=(2, 2), dyn="affine",
                params=affine_params(A, B), var=(var,) * 5, cutoff=cutoff, horizon=horizon, spec="safety",
                safe=box((0.0,) * 5, (10.0,) * 5, 5), mode="otf", precision=precision,
                name="traffic5d" + ("-text" if text else ""))
    if text:
        p = p.with_(dyn="user", params=(a, e), rhs=TRAFFIC5_RHS)
    return p


def robot2d(input_q: float = 0.2, precision: str = "fp32", horizon: int = 8, spec: str = "safety",
            text: bool = False) -> Problem:
    """The robot of Sec. 7 with its disturbance: X = [-10, 10]^2 quantised by
    0.5, U = [-1, 1]^2 quantised by ``input_q`` (0.2 gives the 203,401
    state-input pairs printed there), W = [-1, 1] quantised by 0.2,
    covariance diag(0.75, 0.75), cutoff 1e-3, tau = 10, safety over 8 steps
    (or reach-avoid with the seeded boxes below).  text=True gives the same
    model as source text."""
    lo, h, cnt = grid_from_quantization((-10, -10), (10, 10), (0.5, 0.5))
    ulo, uhi, ucnt = inputs_from_quantization((-1, -1), (1, 1), (input_q, input_q))
    wlo, whi, wcnt = inputs_from_quantization((-1,), (1,), (0.2,))
    p = Problem(lo=lo, h=h, count=cnt, u_lo=ulo, u_hi=uhi, u_count=ucnt, dyn="robot", params=(10.0,),
                var=(0.75, 0.75), cutoff=1e-3, horizon=horizon, spec=spec, w_lo=wlo, w_hi=whi, w_count=wcnt,
                mode="otf", precision=precision, name="robot2d" + ("-text" if text else ""))
    if spec == "reach_avoid":
        p = p.with_(target=box((5.0, 5.0), (10.0, 10.0), 2), avoid=box((-2.0, -2.0), (2.0, 2.0), 2))
    if text:
        p = p.with_(dyn="user", rhs=ROBOT_RHS)
    return p
