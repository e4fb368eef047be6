"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``libamy_oracle.so`` (plain C,
FP64, OpenMP; see ``amy_oracle.h``) with ctypes and shares nothing with the
HIP library except the problem descriptions of the ``workloads`` module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# AMY_ORACLE_LIB points the tests at another build of the same source (used to
# check that the pins fail on a copy with a deliberate mistake).
BUILT_LIB = os.path.join(HERE, "libamy_oracle.so")
LIB_PATH = os.environ.get("AMY_ORACLE_LIB") or BUILT_LIB

MAX_DIM, MAX_IN, MAX_PARAMS = 8, 4, 128
_DYN = {"affine": 0, "unicycle": 1, "room": 2, "vehicle7": 3, "robot": 4, "user": 5}
_SPEC = {"safety": 0, "reach": 1, "reach_avoid": 2}
_NOISE = {"normal": 0, "uniform": 1, "exponential": 2, "beta": 3}
_WINDOW = {"centre": 0, "intersect": 1}


class OrcProblem(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("count", C.c_int32 * MAX_DIM),
        ("lo", C.c_double * MAX_DIM), ("h", C.c_double * MAX_DIM),
        ("m", C.c_int32), ("ucount", C.c_int32 * MAX_IN),
        ("ulo", C.c_double * MAX_IN), ("uhi", C.c_double * MAX_IN),
        ("dyn", C.c_int32), ("n_params", C.c_int32), ("params", C.c_double * MAX_PARAMS),
        ("var", C.c_double * MAX_DIM), ("cutoff", C.c_double),
        ("horizon", C.c_int32), ("spec", C.c_int32),
        ("tlo", C.c_double * MAX_DIM), ("thi", C.c_double * MAX_DIM),
        ("alo", C.c_double * MAX_DIM), ("ahi", C.c_double * MAX_DIM),
        ("slo", C.c_double * MAX_DIM), ("shi", C.c_double * MAX_DIM),
        ("p", C.c_int32), ("wcount", C.c_int32 * MAX_IN),
        ("wlo", C.c_double * MAX_IN), ("whi", C.c_double * MAX_IN),
        ("noise", C.c_int32), ("window", C.c_int32), ("mult", C.c_int32),
        ("na", C.c_double * MAX_DIM), ("nb", C.c_double * MAX_DIM),
        ("nalpha", C.c_double * MAX_DIM), ("nbeta", C.c_double * MAX_DIM),
        ("user_f", C.c_void_p),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no FP contraction)."""
    if force or not os.path.exists(BUILT_LIB):
        src = os.path.join(HERE, "amy_oracle.c")
        tmp = BUILT_LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, BUILT_LIB)
    return BUILT_LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp, i16p, i64p, u8p, i32p = (C.POINTER(C.c_double), C.POINTER(C.c_int16),
                                     C.POINTER(C.c_int64), C.POINTER(C.c_uint8),
                                     C.POINTER(C.c_int32))
        pp = C.POINTER(OrcProblem)
        L.orc_solve.argtypes = [pp, C.c_int, dp, i16p, dp, dp]
        L.orc_step.argtypes = [pp, dp, i64p, C.c_int64, C.c_int, dp, i16p, dp]
        L.orc_mass1d.argtypes = [C.c_double, C.c_double]
        L.orc_mass1d.restype = C.c_double
        L.orc_xstar.argtypes = [C.c_double, C.c_double]
        L.orc_xstar.restype = C.c_double
        L.orc_mean.argtypes = [pp, dp, dp, dp, dp]
        L.orc_window.argtypes = [pp, dp, i32p, i32p]
        L.orc_row_mass.argtypes = [pp, C.c_int64, C.c_int64, dp, dp]
        L.orc_row_dense.argtypes = [pp, C.c_int64, C.c_int64, dp]
        L.orc_labels.argtypes = [pp, u8p]
        L.orc_noise_mass.argtypes = [pp, C.c_int, C.c_double, C.c_double, C.c_double]
        L.orc_noise_mass.restype = C.c_double
        _lib = L
    return _lib


def _box(b, n, default_empty):
    if b is None:
        if default_empty:
            return [1.0] * n, [-1.0] * n          # empty (lo > hi)
        return [-np.inf] * n, [np.inf] * n       # whole space
    return list(b[0]), list(b[1])


def to_struct(p) -> OrcProblem:
    s = OrcProblem()
    n, m = len(p.count), len(p.u_count)
    s.n, s.m = n, m
    for i in range(n):
        s.count[i], s.lo[i], s.h[i], s.var[i] = int(p.count[i]), p.lo[i], p.h[i], p.var[i]
    for k in range(m):
        s.ucount[k], s.ulo[k], s.uhi[k] = int(p.u_count[k]), p.u_lo[k], p.u_hi[k]
    s.dyn = _DYN[p.dyn]
    s.n_params = len(p.params)
    for i, v in enumerate(p.params):
        s.params[i] = float(v)
    s.cutoff = float(p.cutoff)
    s.horizon = int(p.horizon)
    s.spec = _SPEC[p.spec]
    tlo, thi = _box(p.target, n, True)
    alo, ahi = _box(p.avoid, n, True)
    slo, shi = _box(p.safe, n, False)
    for i in range(n):
        s.tlo[i], s.thi[i], s.alo[i], s.ahi[i], s.slo[i], s.shi[i] = (
            tlo[i], thi[i], alo[i], ahi[i], slo[i], shi[i])
    wc = tuple(getattr(p, "w_count", ()) or ())
    s.p = len(wc)
    for l in range(len(wc)):
        s.wcount[l], s.wlo[l], s.whi[l] = int(wc[l]), float(p.w_lo[l]), float(p.w_hi[l])
    s.noise = _NOISE[getattr(p, "noise", "normal")]
    s.window = _WINDOW[getattr(p, "window", "centre")]
    s.mult = int(bool(getattr(p, "multiplicative", False)))
    for src, dst in (("noise_a", s.na), ("noise_b", s.nb), ("noise_alpha", s.nalpha), ("noise_beta", s.nbeta)):
        for i, v in enumerate(tuple(getattr(p, src, ()) or ())):
            dst[i] = float(v)
    if p.dyn == "user":
        s.user_f = user_rhs(p.rhs)
    return s


_user_libs = {}


def user_rhs(text: str) -> int:
    """Address of the right-hand side `text` compiled by gcc as
    void f(const double* x, const double* u, const double* w,
           const double* params, double* mu) { text }
    (FP64, no contraction), built once per text into a cache directory."""
    import hashlib
    import tempfile
    key = hashlib.sha256(text.encode()).hexdigest()[:16]
    if key not in _user_libs:
        d = os.path.join(tempfile.gettempdir(), f"amy_oracle_user_{os.getuid()}")
        os.makedirs(d, exist_ok=True)
        so = os.path.join(d, f"rhs_{key}.so")
        if not os.path.exists(so):
            src = os.path.join(d, f"rhs_{key}.c")
            with open(src, "w") as fh:
                fh.write("#include <math.h>\nvoid amy_user_rhs(const double* x, const double* u, const double* w,"
                         " const double* params, double* mu) {\n" + text + "\n}\n")
            tmp = so + f".{os.getpid()}.tmp"
            subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                                   "-fno-fast-math", "-w", "-o", tmp, src, "-lm"])
            os.replace(tmp, so)
        lib_ = C.CDLL(so)
        _user_libs[key] = (lib_, C.cast(lib_.amy_user_rhs, C.c_void_p).value)
    return _user_libs[key][1]


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def solve(p, threads: int = 0, policy: bool = True, gap: bool = False, tail: bool = True):
    """Full solve.  Returns dict(V, policy[T_d, n_x], gap, max_tail, E)."""
    s = to_struct(p)
    nx, T = p.n_x, p.horizon
    V = np.zeros(nx, np.float64)
    pol = np.zeros((T, nx), np.int16) if policy else None
    gp = np.zeros((T, nx), np.float64) if gap else None
    mt = np.zeros(1, np.float64) if tail else None
    rc = lib().orc_solve(C.byref(s), int(threads), _ptr(V, C.c_double), _ptr(pol, C.c_int16),
                         _ptr(gp, C.c_double), _ptr(mt, C.c_double))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    out = {"V": V, "policy": pol, "gap": gp}
    if tail:
        out["max_tail"] = float(mt[0])
        out["E"] = float(mt[0]) * T
    return out


def step(p, states, V_next=None, threads: int = 0):
    """One Bellman step at ``states`` given V_{k+1} (None: terminal vector)."""
    s = to_struct(p)
    st = np.ascontiguousarray(states, dtype=np.int64)
    V = np.zeros(len(st), np.float64)
    pol = np.zeros(len(st), np.int16)
    gp = np.zeros(len(st), np.float64)
    vn = None if V_next is None else np.ascontiguousarray(V_next, dtype=np.float64)
    rc = lib().orc_step(C.byref(s), _ptr(vn, C.c_double), _ptr(st, C.c_int64), len(st),
                        int(threads), _ptr(V, C.c_double), _ptr(pol, C.c_int16),
                        _ptr(gp, C.c_double))
    if rc != 0:
        raise ValueError("oracle rejected the problem or a state index")
    return V, pol, gp


def mass1d(a, b):
    return lib().orc_mass1d(float(a), float(b))


def noise_mass(p, i, xi, ta, tb):
    """Mass of dimension i's noise between offsets ta < tb from the mean."""
    return lib().orc_noise_mass(C.byref(to_struct(p)), int(i), float(xi), float(ta), float(tb))


def xstar(var, cutoff):
    return lib().orc_xstar(float(var), float(cutoff))


def mean(p, x, u, w=None):
    s = to_struct(p)
    x = np.ascontiguousarray(x, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    w = np.ascontiguousarray(w if w is not None else np.zeros(MAX_IN), np.float64)
    mu = np.zeros(len(p.count), np.float64)
    lib().orc_mean(C.byref(s), _ptr(x, C.c_double), _ptr(u, C.c_double), _ptr(w, C.c_double),
                   _ptr(mu, C.c_double))
    return mu


def window(p, mu):
    s = to_struct(p)
    mu = np.ascontiguousarray(mu, np.float64)
    lo = np.zeros(len(p.count), np.int32)
    hi = np.zeros(len(p.count), np.int32)
    ok = lib().orc_window(C.byref(s), _ptr(mu, C.c_double), _ptr(lo, C.c_int32), _ptr(hi, C.c_int32))
    return bool(ok), lo, hi


def row_mass(p, state, inp):
    s = to_struct(p)
    a, b = C.c_double(), C.c_double()
    if lib().orc_row_mass(C.byref(s), int(state), int(inp), C.byref(a), C.byref(b)) != 0:
        raise ValueError("bad row")
    return a.value, b.value


def row_dense(p, state, inp):
    s = to_struct(p)
    row = np.zeros(p.n_x, np.float64)
    if lib().orc_row_dense(C.byref(s), int(state), int(inp), _ptr(row, C.c_double)) != 0:
        raise ValueError("bad row")
    return row


def labels(p):
    s = to_struct(p)
    out = np.zeros(p.n_x, np.uint8)
    if lib().orc_labels(C.byref(s), _ptr(out, C.c_uint8)) != 0:
        raise ValueError("oracle rejected the problem")
    return out
