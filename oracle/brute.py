"""Dense brute-force checker for tiny grids -- TEST INFRASTRUCTURE ONLY.

An independent second implementation of the paper's serial algorithms, in
Python with mpmath (50 digits) for the normal CDF:

* Alg. 1: the dense transition matrix T of shape (n_x * n_u, n_x), each
  entry the Gaussian mass of a target cell around mu = f(x_bar, u_bar),
  optionally restricted to the cutting region of Sec. 5.2;
* Alg. 3: backward value iteration with dense matrix-vector products,
  ``V_in = T V`` (safety) or ``V_in = T0 + T V`` (reach / reach-avoid, with
  the columns of T at T u A zeroed), reshaped to (n_x, n_u) and maximised;
* exhaustive enumeration of deterministic Markov policies, each evaluated by
  forward propagation of the state distribution, for Bellman optimality;
* with a disturbance (Def. 3.1 and its Remark: the disturbance is an
  adversary that sees the input), Alg. 3's reshape-minimise-maximise steps
  on the dense (x, u, w) rows, and the game value itself: the best
  controller policy against the adversary's best reply, both enumerated.

It shares no code with ``amy_oracle.c``: the dynamics, window rule, set
membership and CDF are written out again here.
"""
from __future__ import annotations

import itertools
import math

import mpmath as mp
import numpy as np

mp.mp.dps = 50


def ncdf(z) -> mp.mpf:
    return mp.ncdf(mp.mpf(z))


def cell_mass(a_edge, b_edge, mu, sigma) -> float:
    """Normal mass of [a_edge, b_edge] around mu (50-digit arithmetic)."""
    a = (mp.mpf(a_edge) - mp.mpf(mu)) / mp.mpf(sigma)
    b = (mp.mpf(b_edge) - mp.mpf(mu)) / mp.mpf(sigma)
    return ncdf(b) - ncdf(a)


def states(p):
    axes = [[p.lo[i] + (j + 0.5) * p.h[i] for j in range(p.count[i])] for i in range(p.n)]
    return [np.array(c) for c in itertools.product(*axes)]


def inputs(p):
    axes = []
    for k in range(p.m):
        if p.u_count[k] == 1:
            axes.append([p.u_lo[k]])
        else:
            st = (p.u_hi[k] - p.u_lo[k]) / (p.u_count[k] - 1)
            axes.append([p.u_lo[k] + j * st for j in range(p.u_count[k])])
    return [np.array(c) for c in itertools.product(*axes)]


def disturbances(p):
    """Points of the disturbance set (one empty point when there is none)."""
    wc = tuple(getattr(p, "w_count", ()) or ())
    axes = []
    for l in range(len(wc)):
        if wc[l] == 1:
            axes.append([p.w_lo[l]])
        else:
            st = (p.w_hi[l] - p.w_lo[l]) / (wc[l] - 1)
            axes.append([p.w_lo[l] + j * st for j in range(wc[l])])
    return [np.array(c) for c in itertools.product(*axes)]


def mean(p, x, u, w=None):
    """mu = f(x, u, w) for the model families (the paper's equations, retyped)."""
    q = p.params
    n, m = p.n, p.m
    pd = len(getattr(p, "w_count", ()) or ())
    if p.dyn == "affine":
        A = np.array(q[:n * n]).reshape(n, n)
        B = np.array(q[n * n:n * n + n * m]).reshape(n, m)
        c = np.array(q[n * n + n * m:n * n + n * m + n])
        out = A @ x + B @ u + c
        if pd:
            D = np.array(q[n * n + n * m + n:]).reshape(n, pd)
            out = out + D @ np.asarray(w)
        return out
    if p.dyn == "robot":
        # Sec. 7: a planar robot moved by speed u[0] along heading u[1], pushed by w
        tau = q[0]
        d = w[0] if pd else 0.0
        return np.array([x[0] + tau * u[0] * math.cos(u[1]) + d,
                         x[1] + tau * u[0] * math.sin(u[1]) + d])
    if p.dyn == "unicycle":
        tau = q[0]
        return np.array([x[0] + tau * u[0] * math.cos(x[2]),
                         x[1] + tau * u[0] * math.sin(x[2]),
                         x[2] + tau * u[1]])
    if p.dyn == "room":
        a, b, g, Te, Th = q
        out = np.zeros(n)
        for i in range(n):
            ui = u[0] if m == 1 else u[i]
            out[i] = ((1 - 2 * a - b - g * ui) * x[i] + a * (x[i - 1] + x[(i + 1) % n])
                      + b * Te + g * Th * ui)
        return out
    if p.dyn == "vehicle7":
        tau, lwb, M, mub, lf, lr, hcg, Iz, CSf, CSr, g = q
        x1, x2, x3, x4, x5, x6, x7 = x
        v1 = min(max(u[0], p.u_lo[0]), p.u_hi[0])
        v2 = min(max(u[1], p.u_lo[1]), p.u_hi[1])
        if abs(x4) < 0.1:
            d = [x4 * math.cos(x5), x4 * math.sin(x5), v1, v2, x4 / lwb * math.tan(x3),
                 v2 / lwb * math.tan(x3) + x4 / (lwb * math.cos(x3) ** 2) * v1, 0.0]
        else:
            Ff, Fr = g * lr - v2 * hcg, g * lf + v2 * hcg
            d6 = mub * M / (Iz * (lr + lf)) * (lf * CSf * Ff * x3 + (lr * CSr * Fr - lf * CSf * Ff) * x7
                                                - (lf ** 2 * CSf * Ff + lr ** 2 * CSr * Fr) * x6 / x4)
            d7 = mub / (x4 * (lr + lf)) * (CSf * Ff * x3 + (CSr * Fr + CSf * Ff) * x7
                                            - (lf * CSf * Ff - lr * CSr * Fr) * x6 / x4) - x6
            d = [x4 * math.cos(x5 + x7), x4 * math.sin(x5 + x7), v1, v2, x6, d6, d7]
        return np.array(x) + tau * np.array(d)
    raise ValueError(p.dyn)


def in_box(x, bx):
    if bx is None:
        return False
    return all(bx[0][i] <= x[i] <= bx[1][i] for i in range(len(x)))


def labels(p):
    """0 free, 1 fixed at 0, 2 fixed at 1 (same meaning as the oracle's)."""
    out = []
    for x in states(p):
        if p.spec == "safety":
            out.append(0 if (p.safe is None or in_box(x, p.safe)) else 1)
        elif p.spec == "reach_avoid" and in_box(x, p.avoid):
            out.append(1)
        elif in_box(x, p.target):
            out.append(2)
        else:
            out.append(0)
    return np.array(out, np.uint8)


def xstar(var, cutoff):
    """Solve N(x*|0,var) = cutoff for x* > 0 by bisection (no closed form)."""
    if cutoff == 0:
        return math.inf
    s = mp.sqrt(mp.mpf(var))
    pdf = lambda x: mp.exp(-x * x / (2 * s * s)) / (s * mp.sqrt(2 * mp.pi))
    lo, hi = mp.mpf(0), 40 * s
    for _ in range(200):
        mid = (lo + hi) / 2
        if pdf(mid) > cutoff:
            lo = mid
        else:
            hi = mid
    return float(lo)


def dense_T(p, cut: bool = True):
    """Alg. 1 as a dense matrix; row index = x * n_u + u."""
    X, U = states(p), inputs(p)
    sig = [math.sqrt(v) for v in p.var]
    xs = [xstar(v, p.cutoff) if cut else math.inf for v in p.var]
    nx, nu = len(X), len(U)
    T = np.zeros((nx * nu, nx))
    axes = [[(p.lo[i] + j * p.h[i], p.lo[i] + (j + 1) * p.h[i], p.lo[i] + (j + 0.5) * p.h[i])
             for j in range(p.count[i])] for i in range(p.n)]
    for xi, x in enumerate(X):
        for ui, u in enumerate(U):
            mu = mean(p, x, u)
            per_dim = []
            for i in range(p.n):
                col = []
                for (a, b, c) in axes[i]:
                    keep = abs(c - mu[i]) <= xs[i]
                    col.append(float(cell_mass(a, b, mu[i], sig[i])) if keep else 0.0)
                per_dim.append(col)
            for ci, combo in enumerate(itertools.product(*per_dim)):
                T[xi * nu + ui, ci] = float(np.prod(combo))
    return T


def synthesize(p, T=None, cut: bool = True):
    """Alg. 3 (serial synthesis).  Returns (V_1 with the readout convention, policy[T_d, n_x])."""
    if T is None:
        T = dense_T(p, cut)
    nx, nu = p.n_x, p.n_u
    lab = labels(p)
    if p.spec == "safety":
        V = (lab == 0).astype(float)
        Tm = T
        T0 = np.zeros(nx * nu)
    else:
        goal = (lab == 2).astype(float)
        T0 = T @ goal                       # transition mass into T \ A
        Tm = T * (lab == 0)[None, :]        # zero the columns at T u A
        V = np.zeros(nx)
    pol = np.zeros((p.horizon, nx), np.int16)
    for k in range(p.horizon, 0, -1):
        Vin = (T0 + Tm @ V).reshape(nx, nu)
        Vmax = Vin.max(axis=1)
        arg = Vin.argmax(axis=1)             # lowest index among maxima
        Vmax[lab != 0] = 0.0
        arg[lab != 0] = -1
        V = Vmax
        pol[k - 1] = arg
    out = V.copy()
    out[lab == 2] = 1.0
    out[lab == 1] = 0.0
    return out, pol


def best_over_policies(p, T=None, cut: bool = True):
    """Max over all deterministic Markov policies of the satisfaction
    probability from every initial state, by forward propagation."""
    if T is None:
        T = dense_T(p, cut)
    nx, nu, Td = p.n_x, p.n_u, p.horizon
    lab = labels(p)
    free = [x for x in range(nx) if lab[x] == 0]
    best = np.where(lab == 2, 1.0, 0.0)
    if Td == 0:
        if p.spec == "safety":
            best = (lab == 0).astype(float)
        return best
    choices = list(itertools.product(range(nu), repeat=len(free) * Td))
    for x0 in free:
        top = 0.0
        for ch in choices:
            pol = np.array(ch).reshape(Td, len(free))
            d = np.zeros(nx)
            d[x0] = 1.0
            won = 0.0
            for t in range(Td):
                nd = np.zeros(nx)
                for fi, x in enumerate(free):
                    if d[x] != 0.0:
                        nd += d[x] * T[x * nu + pol[t, fi]]
                if p.spec == "safety":
                    nd[lab != 0] = 0.0
                else:
                    won += nd[lab == 2].sum()
                    nd[lab != 0] = 0.0
                d = nd
            val = d.sum() if p.spec == "safety" else won
            top = max(top, val)
        best[x0] = top
    return best


# ----------------------------------------------------------- disturbance

def dense_T_game(p, cut: bool = True):
    """Alg. 1 with the loop over W: T[x, u, w, x'] as a dense array."""
    X, U, Wd = states(p), inputs(p), disturbances(p)
    sig = [math.sqrt(v) for v in p.var]
    xs = [xstar(v, p.cutoff) if cut else math.inf for v in p.var]
    nx, nu, nw = len(X), len(U), len(Wd)
    T = np.zeros((nx, nu, nw, nx))
    axes = [[(p.lo[i] + j * p.h[i], p.lo[i] + (j + 1) * p.h[i], p.lo[i] + (j + 0.5) * p.h[i])
             for j in range(p.count[i])] for i in range(p.n)]
    for xi, x in enumerate(X):
        for ui, u in enumerate(U):
            for wi, w in enumerate(Wd):
                mu = mean(p, x, u, w)
                per_dim = []
                for i in range(p.n):
                    col = []
                    for (a, b, c) in axes[i]:
                        keep = abs(c - mu[i]) <= xs[i]
                        col.append(float(cell_mass(a, b, mu[i], sig[i])) if keep else 0.0)
                    per_dim.append(col)
                for ci, combo in enumerate(itertools.product(*per_dim)):
                    T[xi, ui, wi, ci] = float(np.prod(combo))
    return T


def synthesize_game(p, T=None, cut: bool = True):
    """Alg. 3 with a disturbance: V_in over the (x, u, w) rows, reshaped to
    (x u, w) and minimised over W, reshaped to (x, u) and maximised over U.
    Returns (V_1 with the readout convention, policy[T_d, n_x])."""
    if T is None:
        T = dense_T_game(p, cut)
    nx, nu, nw = T.shape[0], T.shape[1], T.shape[2]
    lab = labels(p)
    rows = T.reshape(nx * nu * nw, nx)
    if p.spec == "safety":
        V = (lab == 0).astype(float)
        Tm, T0 = rows, np.zeros(nx * nu * nw)
    else:
        T0 = rows @ (lab == 2).astype(float)
        Tm = rows * (lab == 0)[None, :]
        V = np.zeros(nx)
    pol = np.zeros((p.horizon, nx), np.int16)
    for k in range(p.horizon, 0, -1):
        Vin = (T0 + Tm @ V).reshape(nx * nu, nw)
        Vmin = Vin.min(axis=1).reshape(nx, nu)
        Vmax = Vmin.max(axis=1)
        arg = Vmin.argmax(axis=1)
        Vmax[lab != 0] = 0.0
        arg[lab != 0] = -1
        V = Vmax
        pol[k - 1] = arg
    out = V.copy()
    out[lab == 2] = 1.0
    out[lab == 1] = 0.0
    return out, pol


def game_value_by_enumeration(p, T=None, cut: bool = True):
    """max over the controller's deterministic Markov policies of the min over
    the adversary's replies (a disturbance for every step and state, chosen
    knowing the input), each pair evaluated by forward propagation of the
    state distribution.  Tiny problems only."""
    if T is None:
        T = dense_T_game(p, cut)
    nx, nu, nw = T.shape[0], T.shape[1], T.shape[2]
    Td = p.horizon
    lab = labels(p)
    free = [x for x in range(nx) if lab[x] == 0]
    best = np.where(lab == 2, 1.0, 0.0)
    if Td == 0:
        if p.spec == "safety":
            best = (lab == 0).astype(float)
        return best
    pols = list(itertools.product(range(nu), repeat=len(free) * Td))
    advs = np.array(list(itertools.product(range(nw), repeat=len(free) * Td))).reshape(-1, Td, len(free))

    def values(x0, pol):
        # all adversary replies at once: d[a] is the state distribution under reply a
        d = np.zeros((len(advs), nx))
        d[:, x0] = 1.0
        won = np.zeros(len(advs))
        for t in range(Td):
            nd = np.zeros_like(d)
            for fi, x in enumerate(free):
                nd += d[:, x:x + 1] * T[x, pol[t, fi]][advs[:, t, fi]]
            if p.spec != "safety":
                won += nd[:, lab == 2].sum(axis=1)
            nd[:, lab != 0] = 0.0
            d = nd
        return d.sum(axis=1) if p.spec == "safety" else won

    for x0 in free:
        top = 0.0
        for ch in pols:
            pol = np.array(ch).reshape(Td, len(free))
            top = max(top, float(values(x0, pol).min()))
        best[x0] = top
    return best


# ----------------------------------------------------------- other noise

def noise_cell_mass(p, i, a_edge, b_edge, mu):
    """Mass of [a_edge, b_edge] for dimension i's noise around mu (mpmath)."""
    ta, tb = mp.mpf(a_edge) - mp.mpf(mu), mp.mpf(b_edge) - mp.mpf(mu)
    if p.noise == "uniform":
        A, B = mp.mpf(p.noise_a[i]), mp.mpf(p.noise_b[i])
        F = lambda t: min(max((t - A) / (B - A), mp.mpf(0)), mp.mpf(1))
        return F(tb) - F(ta)
    if p.noise == "exponential":
        lam = mp.mpf(p.noise_a[i])
        F = lambda t: mp.mpf(0) if t <= 0 else 1 - mp.exp(-lam * t)
        return F(tb) - F(ta)
    if p.noise == "beta":
        A, B = mp.mpf(p.noise_a[i]), mp.mpf(p.noise_b[i])
        y = lambda t: min(max((t - A) / (B - A), mp.mpf(0)), mp.mpf(1))
        return mp.betainc(p.noise_alpha[i], p.noise_beta[i], y(ta), y(tb), regularized=True)
    return cell_mass(a_edge, b_edge, mu, math.sqrt(p.var[i]))


def noise_interval(p, i):
    """Offsets from the mean of the kept interval and whether cells must meet
    it (True) or have their centre in it (False); None: keep every cell."""
    if p.noise in ("uniform", "beta"):
        return (p.noise_a[i], p.noise_b[i]), True
    if p.noise == "exponential":
        lam = p.noise_a[i]
        top = math.log(lam / p.cutoff) / lam if p.cutoff > 0 else math.inf
        return (0.0, top), True
    if p.multiplicative or p.cutoff == 0:
        return None, False
    xs = xstar(p.var[i], p.cutoff)
    return (-xs, xs), p.window == "intersect"


def dense_T_noise(p):
    """Alg. 1 with additive noise of any of the models, as a dense matrix."""
    X, U = states(p), inputs(p)
    nx, nu = len(X), len(U)
    T = np.zeros((nx * nu, nx))
    axes = [[(p.lo[i] + j * p.h[i], p.lo[i] + (j + 1) * p.h[i], p.lo[i] + (j + 0.5) * p.h[i])
             for j in range(p.count[i])] for i in range(p.n)]
    for xi, x in enumerate(X):
        for ui, u in enumerate(U):
            mu = mean(p, x, u)
            per_dim = []
            for i in range(p.n):
                iv, meet = noise_interval(p, i)
                col = []
                for (a, b, c) in axes[i]:
                    if iv is None:
                        keep = True
                    elif meet:
                        keep = (b - mu[i] > iv[0]) and (a - mu[i] < iv[1])
                    else:
                        keep = iv[0] <= c - mu[i] <= iv[1]
                    col.append(float(noise_cell_mass(p, i, a, b, mu[i])) if keep else 0.0)
                per_dim.append(col)
            for ci, combo in enumerate(itertools.product(*per_dim)):
                T[xi * nu + ui, ci] = float(np.prod(combo))
    return T


def synthesize_noise(p):
    """Alg. 3 over dense_T_noise."""
    return synthesize(p, T=dense_T_noise(p))
