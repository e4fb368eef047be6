"""ctypes binding of libamytiss_hip.so (argument marshalling only).

Every step of the path runs in the HIP library; this module only mirrors
the C structs of include/amytiss.h, allocates device buffers with PyTorch
and passes pointers and the current HIP stream.  Loading fails loudly when
the library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# AMYTISS_LIB: path of another build of the same library (e.g. for A/B timing)
LIB_PATH = os.environ.get("AMYTISS_LIB") or os.path.join(HERE, "libamytiss_hip.so")

MAX_DIM, MAX_IN, MAX_PARAMS = 8, 4, 128

OK, E_INVALID, E_NOMEM, E_DEVICE, E_UNSUPPORTED, E_BUSY, E_NOTREADY, E_CANCELLED = range(8)
STATUS = {0: "OK", 1: "INVALID", 2: "NOMEM", 3: "DEVICE", 4: "UNSUPPORTED", 5: "BUSY", 6: "NOTREADY",
          7: "CANCELLED"}
DYN = {"affine": 0, "unicycle": 1, "room": 2, "vehicle7": 3, "robot": 4, "user": 5}
NOISE = {"normal": 0, "uniform": 1, "exponential": 2, "beta": 3}
WINDOW = {"centre": 0, "intersect": 1}
SPEC = {"safety": 0, "reach": 1, "reach_avoid": 2}
MODE = {"auto": 0, "stored": 1, "otf": 2}
MODE_NAME = {v: k for k, v in MODE.items()}
PREC = {"fp64": 0, "fp32": 1}
VARIANT = {"auto": 0, "lanes": 1, "fixed": 2, "group16": 3, "group64": 4, "factored": 5, "inputs": 6}
VARIANT_NAME = {v: k for k, v in VARIANT.items()}


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32), ("count", C.c_int32 * MAX_DIM),
                ("lo", C.c_double * MAX_DIM), ("h", C.c_double * MAX_DIM)]


class Inputs(C.Structure):
    _fields_ = [("m", C.c_int32), ("count", C.c_int32 * MAX_IN),
                ("lo", C.c_double * MAX_IN), ("hi", C.c_double * MAX_IN)]


class Box(C.Structure):
    _fields_ = [("lo", C.c_double * MAX_DIM), ("hi", C.c_double * MAX_DIM)]


class Dynamics(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_params", C.c_int32), ("params", C.c_double * MAX_PARAMS)]


class Disturbance(C.Structure):
    _fields_ = [("p", C.c_int32), ("count", C.c_int32 * MAX_IN),
                ("lo", C.c_double * MAX_IN), ("hi", C.c_double * MAX_IN)]


class Noise(C.Structure):
    _fields_ = [("kind", C.c_int32), ("window", C.c_int32), ("multiplicative", C.c_int32),
                ("reserved", C.c_int32), ("a", C.c_double * MAX_DIM), ("b", C.c_double * MAX_DIM),
                ("alpha", C.c_double * MAX_DIM), ("beta", C.c_double * MAX_DIM)]


class ProblemC(C.Structure):
    _fields_ = [("grid", Grid), ("inputs", Inputs), ("dyn", Dynamics),
                ("noise_var", C.c_double * MAX_DIM), ("cutoff", C.c_double),
                ("horizon", C.c_int32), ("spec", C.c_int32),
                ("target", Box), ("avoid", Box), ("safe", Box),
                ("mode", C.c_int32), ("precision", C.c_int32), ("variant", C.c_int32),
                ("dist", Disturbance), ("noise", Noise)]


class Info(C.Structure):
    _fields_ = [("mode_used", C.c_int32), ("window", C.c_int32 * MAX_DIM), ("kernel", C.c_int32),
                ("table_cache_mask", C.c_int32), ("lds_bytes", C.c_int32),
                ("n_x", C.c_int64), ("n_u", C.c_int64), ("rows", C.c_int64), ("W", C.c_int64),
                ("workspace_bytes", C.c_uint64), ("stored_bytes", C.c_uint64),
                ("max_row_tail", C.c_double), ("tail_bound_E", C.c_double),
                ("t_build_ms", C.c_double), ("t_sweeps_ms", C.c_double),
                ("t_main_sweeps_ms", C.c_double), ("t_readout_ms", C.c_double),
                ("t_total_ms", C.c_double), ("n_w", C.c_int64)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            if name == "window":
                v = [int(x) for x in v]
            d[name] = v
        d["mode"] = MODE_NAME.get(self.mode_used, "?")
        d["variant"] = VARIANT_NAME.get(self.kernel, "?")
        return d


class TuneResult(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("blocks_per_cu", C.c_int32), ("xcd_order", C.c_int32),
                ("variant", C.c_int32), ("candidates", C.c_int32), ("best_ms", C.c_double),
                ("worst_ms", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerCfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("max_slots", C.c_int32), ("device", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("failed", C.c_uint64),
                ("queued", C.c_int32), ("active", C.c_int32), ("max_active", C.c_int32),
                ("hbm_in_use", C.c_uint64), ("hbm_peak", C.c_uint64), ("steps", C.c_uint64),
                ("row_updates", C.c_double), ("busy_s", C.c_double), ("p50_ms", C.c_double),
                ("p99_ms", C.c_double), ("mean_ms", C.c_double), ("cancelled", C.c_uint64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class AmyError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"amytiss {STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        pp, ip = C.POINTER(ProblemC), C.POINTER(Info)
        L.amy_query.argtypes = [pp, C.c_uint64, ip]
        L.amy_query.restype = C.c_int
        L.amy_solve.argtypes = [pp, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, ip]
        L.amy_solve.restype = C.c_int
        L.amy_batch_query.argtypes = [pp, C.c_int32, C.POINTER(C.c_uint64)]
        L.amy_batch_query.restype = C.c_int
        L.amy_batch_solve.argtypes = [pp, C.c_int32, C.c_void_p, C.c_void_p, C.c_uint64,
                                      C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), ip]
        L.amy_batch_solve.restype = C.c_int
        L.amy_tune_solve.argtypes = [pp, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p,
                                     C.POINTER(TuneResult)]
        L.amy_tune_solve.restype = C.c_int
        L.amy_tune_batch.argtypes = [pp, C.c_int32, C.c_void_p, C.c_void_p, C.c_uint64,
                                     C.POINTER(C.c_void_p), C.POINTER(TuneResult)]
        L.amy_tune_batch.restype = C.c_int
        for fn in ("amy_tune_save", "amy_tune_load"):
            getattr(L, fn).argtypes = [C.c_char_p]
            getattr(L, fn).restype = C.c_int
        L.amy_tune_clear.restype = C.c_int
        L.amy_tune_entries.restype = C.c_int32
        sp = C.c_void_p
        L.amy_server_create.argtypes = [C.POINTER(ServerCfg), C.POINTER(sp)]
        L.amy_server_submit.argtypes = [sp, pp, C.c_int32, C.POINTER(C.c_uint64)]
        L.amy_server_wait.argtypes = [sp, C.c_uint64, C.c_int32, C.c_void_p, C.c_void_p, ip]
        L.amy_server_poll.argtypes = [sp, C.c_uint64, C.c_void_p, C.c_void_p, ip]
        L.amy_server_get_stats.argtypes = [sp, C.POINTER(ServerStats)]
        L.amy_server_reset_stats.argtypes = [sp]
        L.amy_server_destroy.argtypes = [sp]
        L.amy_server_cancel.argtypes = [sp, C.c_uint64]
        for fn in ("amy_server_create", "amy_server_submit", "amy_server_wait", "amy_server_poll",
                   "amy_server_get_stats", "amy_server_reset_stats", "amy_server_destroy", "amy_server_cancel"):
            getattr(L, fn).restype = C.c_int
        L.amy_solve_static.argtypes = [pp, C.c_void_p, C.c_void_p, C.c_void_p]
        L.amy_solve_static.restype = C.c_int
        dp = C.POINTER(C.c_double)
        L.amy_grid_from_quantization.argtypes = [C.c_int32, dp, dp, dp, C.POINTER(Grid)]
        L.amy_grid_from_quantization.restype = C.c_int
        L.amy_inputs_from_quantization.argtypes = [C.c_int32, dp, dp, dp, C.POINTER(Inputs)]
        L.amy_inputs_from_quantization.restype = C.c_int
        L.amy_user_dynamics_create.argtypes = [C.c_char_p, C.c_int32, C.c_int32, C.c_int32,
                                               C.POINTER(C.c_void_p)]
        L.amy_user_dynamics_create.restype = C.c_int
        L.amy_user_dynamics_destroy.argtypes = [C.c_void_p]
        L.amy_user_dynamics_destroy.restype = C.c_int
        L.amy_solve_user.argtypes = [C.c_void_p, pp, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, ip]
        L.amy_solve_user.restype = C.c_int
        L.amy_last_error.restype = C.c_char_p
        L.amy_version.restype = C.c_char_p
        _lib = L
    return _lib


def check(status):
    if status != OK:
        raise AmyError(status, lib().amy_last_error().decode())


def _box(dst, b, n, empty_default):
    for i in range(MAX_DIM):
        if b is None:
            lo, hi = (1.0, -1.0) if empty_default else (-math.inf, math.inf)
        elif i < n:
            lo, hi = float(b[0][i]), float(b[1][i])
        else:
            lo, hi = -math.inf, math.inf
        dst.lo[i], dst.hi[i] = lo, hi


def to_struct(p, mode=None, precision=None, variant=None) -> ProblemC:
    """Marshal a problem description (any object with the fields of
    workloads.Problem) into the C struct."""
    s = ProblemC()
    n, m = len(p.count), len(p.u_count)
    s.grid.n, s.inputs.m = n, m
    for i in range(n):
        s.grid.count[i], s.grid.lo[i], s.grid.h[i] = int(p.count[i]), float(p.lo[i]), float(p.h[i])
        s.noise_var[i] = float(p.var[i])
    for k in range(m):
        s.inputs.count[k], s.inputs.lo[k], s.inputs.hi[k] = (int(p.u_count[k]), float(p.u_lo[k]),
                                                              float(p.u_hi[k]))
    s.dyn.kind = DYN[p.dyn]
    s.dyn.n_params = len(p.params)
    for k, v in enumerate(p.params):
        s.dyn.params[k] = float(v)
    s.cutoff = float(p.cutoff)
    s.horizon = int(p.horizon)
    s.spec = SPEC[p.spec]
    _box(s.target, p.target, n, True)
    _box(s.avoid, p.avoid, n, True)
    _box(s.safe, p.safe, n, False)
    s.mode = MODE[mode or p.mode]
    s.precision = PREC[precision or p.precision]
    s.variant = VARIANT[variant or getattr(p, "variant", "auto")]
    wc = tuple(getattr(p, "w_count", ()) or ())
    s.dist.p = len(wc)
    for l in range(len(wc)):
        s.dist.count[l], s.dist.lo[l], s.dist.hi[l] = int(wc[l]), float(p.w_lo[l]), float(p.w_hi[l])
    s.noise.kind = NOISE[getattr(p, "noise", "normal")]
    s.noise.window = WINDOW[getattr(p, "window", "centre")]
    s.noise.multiplicative = int(bool(getattr(p, "multiplicative", False)))
    for name in ("a", "b", "alpha", "beta"):
        vals = tuple(getattr(p, "noise_" + name, ()) or ())
        arr = getattr(s.noise, name)
        for i, v in enumerate(vals):
            arr[i] = float(v)
    return s


def query(p, budget: int = 0, **kw) -> dict:
    s = to_struct(p, **kw)
    info = Info()
    check(lib().amy_query(C.byref(s), int(budget), C.byref(info)))
    return info.as_dict()


class Result:
    def __init__(self, V, policy, info):
        self.V = V            # torch float64 [n_x] on the device
        self.policy = policy  # torch int16 [T_d, n_x] on the device, or None
        self.info = info      # dict or None


class Solver:
    """Holds a device workspace for repeated solves of problems of one size
    (user: the UserDynamics of a problem whose dynamics are source text)."""

    def __init__(self, p, budget: int = 0, device=None, user=None, **kw):
        import torch
        self.torch = torch
        self.p = p
        self.user = user
        self.s = to_struct(p, **kw)
        self.device = torch.device(device or "cuda")
        info = Info()
        check(lib().amy_query(C.byref(self.s), int(budget), C.byref(info)))
        self.plan = info.as_dict()
        self.ws_bytes = int(info.workspace_bytes)
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws.data_ptr()) % 256
        self.ws_ptr = self._ws.data_ptr() + off

    def solve(self, policy: bool = True, info: bool = True, stream=None, out=None) -> Result:
        torch = self.torch
        n_x, T = self.p.n_x, self.p.horizon
        V = out if out is not None else torch.empty(n_x, dtype=torch.float64, device=self.device)
        pol = torch.empty((T, n_x), dtype=torch.int16, device=self.device) if (policy and T > 0) else None
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        inf = Info() if info else None
        args = (C.byref(self.s), C.c_void_p(st.cuda_stream), C.c_void_p(self.ws_ptr), self.ws_bytes,
                C.c_void_p(V.data_ptr()), C.c_void_p(pol.data_ptr()) if pol is not None else None,
                C.byref(inf) if inf is not None else None)
        if self.user is not None:
            rc = lib().amy_solve_user(self.user._h, *args)
        else:
            rc = lib().amy_solve(*args)
        check(rc)
        return Result(V, pol, inf.as_dict() if inf is not None else None)


def solve(p, policy: bool = True, info: bool = True, budget: int = 0, **kw) -> Result:
    """One solve; keyword overrides: mode=, precision=, variant=."""
    return Solver(p, budget=budget, **kw).solve(policy=policy, info=info)


STATIC_WORKSPACE_BYTES = 96 << 20   # AMY_STATIC_WORKSPACE_BYTES


def solve_static(p, policy: bool = True, stream=None, out=None, **kw) -> Result:
    """amy_solve_static: the solve on the library's own static workspace (no
    device allocation inside the call; V and the policy are allocated here,
    by the caller's side, unless `out` is given).  Only enqueues the work."""
    import torch
    s = to_struct(p, **kw)
    dev = torch.device("cuda")
    n_x, T = p.n_x, p.horizon
    V = out if out is not None else torch.empty(n_x, dtype=torch.float64, device=dev)
    pol = torch.empty((T, n_x), dtype=torch.int16, device=dev) if (policy and T > 0) else None
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    check(lib().amy_solve_static(C.byref(s), C.c_void_p(st.cuda_stream), C.c_void_p(V.data_ptr()),
                                 C.c_void_p(pol.data_ptr()) if pol is not None else None))
    return Result(V, pol, None)


def _quant_args(lb, ub, q):
    n = len(lb)
    arr = C.c_double * n
    return n, arr(*map(float, lb)), arr(*map(float, ub)), arr(*map(float, q))


def grid_from_quantization(lb, ub, q):
    """amy_grid_from_quantization: (lo, h, count) tuples of the paper's
    quantisation convention."""
    n, a, b, c = _quant_args(lb, ub, q)
    g = Grid()
    check(lib().amy_grid_from_quantization(n, a, b, c, C.byref(g)))
    return tuple(g.lo[:n]), tuple(g.h[:n]), tuple(int(x) for x in g.count[:n])


def inputs_from_quantization(lb, ub, q):
    """amy_inputs_from_quantization: (lo, hi, count) tuples."""
    m, a, b, c = _quant_args(lb, ub, q)
    u = Inputs()
    check(lib().amy_inputs_from_quantization(m, a, b, c, C.byref(u)))
    return tuple(u.lo[:m]), tuple(u.hi[:m]), tuple(int(x) for x in u.count[:m])


class UserDynamics:
    """amy_user_dynamics_create: a right-hand side given as source text (the
    body of rhs(x, u, w, params, mu)), compiled on the current device."""

    def __init__(self, rhs: str, n: int, m: int, p: int = 0):
        self._h = C.c_void_p()
        check(lib().amy_user_dynamics_create(rhs.encode(), int(n), int(m), int(p), C.byref(self._h)))

    def solver(self, prob, budget: int = 0, **kw) -> "Solver":
        return Solver(prob, budget=budget, user=self, **kw)

    def solve(self, prob, policy: bool = True, info: bool = True, budget: int = 0, **kw) -> Result:
        return self.solver(prob, budget=budget, **kw).solve(policy=policy, info=info)

    def close(self):
        if self._h:
            check(lib().amy_user_dynamics_destroy(self._h))
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version() -> str:
    return lib().amy_version().decode()


# ------------------------------------------------------------------ batch

def _struct_array(problems, **kw):
    arr = (ProblemC * len(problems))()
    for i, p in enumerate(problems):
        arr[i] = to_struct(p, **kw)
    return arr


def batch_query(problems, **kw) -> int:
    arr = _struct_array(problems, **kw)
    n = C.c_uint64()
    check(lib().amy_batch_query(arr, len(problems), C.byref(n)))
    return int(n.value)


class BatchSolver:
    """Device workspace and outputs for repeated batched solves of one set of systems."""

    def __init__(self, problems, device=None, **kw):
        import torch
        self.torch = torch
        self.problems = list(problems)
        self.arr = _struct_array(self.problems, **kw)
        self.device = torch.device(device or "cuda")
        self.ws_bytes = batch_query(self.problems, **kw)
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self.ws_ptr = self._ws.data_ptr() + ((-self._ws.data_ptr()) % 256)
        self.V = [torch.empty(p.n_x, dtype=torch.float64, device=self.device) for p in self.problems]
        self.vptr = (C.c_void_p * len(self.problems))(*[v.data_ptr() for v in self.V])

    def solve(self, policy: bool = False, info: bool = True, stream=None):
        torch = self.torch
        n = len(self.problems)
        pols = None
        pptr = None
        if policy:
            pols = [torch.empty((p.horizon, p.n_x), dtype=torch.int16, device=self.device)
                    if p.horizon > 0 else None for p in self.problems]
            pptr = (C.c_void_p * n)(*[(t.data_ptr() if t is not None else None) for t in pols])
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        infos = (Info * n)() if info else None
        check(lib().amy_batch_solve(self.arr, n, C.c_void_p(st.cuda_stream), C.c_void_p(self.ws_ptr),
                                    self.ws_bytes, self.vptr, pptr, infos))
        return [Result(self.V[i], pols[i] if pols else None, infos[i].as_dict() if info else None)
                for i in range(n)]

    def tune(self, stream=None) -> dict:
        st = stream if stream is not None else self.torch.cuda.current_stream(self.device)
        r = TuneResult()
        check(lib().amy_tune_batch(self.arr, len(self.problems), C.c_void_p(st.cuda_stream),
                                   C.c_void_p(self.ws_ptr), self.ws_bytes, self.vptr, C.byref(r)))
        return r.as_dict()


def batch_solve(problems, policy: bool = False, info: bool = True, **kw):
    return BatchSolver(problems, **kw).solve(policy=policy, info=info)


# -------------------------------------------------------------- autotuner

def tune_solve(p, **kw) -> dict:
    s = Solver(p, **kw)
    V = s.torch.empty(p.n_x, dtype=s.torch.float64, device=s.device)
    st = s.torch.cuda.current_stream(s.device)
    r = TuneResult()
    check(lib().amy_tune_solve(C.byref(s.s), C.c_void_p(st.cuda_stream), C.c_void_p(s.ws_ptr), s.ws_bytes,
                               C.c_void_p(V.data_ptr()), C.byref(r)))
    return r.as_dict()


def tune_save(path: str):
    check(lib().amy_tune_save(os.fsencode(path)))


def tune_load(path: str):
    check(lib().amy_tune_load(os.fsencode(path)))


def tune_clear():
    check(lib().amy_tune_clear())


def tune_entries() -> int:
    return int(lib().amy_tune_entries())


# ----------------------------------------------------------------- server

class Server:
    """Request loop with continuous batching (amy_server_* of the C ABI).
    Results come back in host memory (numpy)."""

    def __init__(self, hbm_budget_bytes: int = 8 << 30, max_slots: int = 64, device: int = 0):
        cfg = ServerCfg(int(hbm_budget_bytes), int(max_slots), int(device))
        self._h = C.c_void_p()
        check(lib().amy_server_create(C.byref(cfg), C.byref(self._h)))
        self._meta = {}

    def submit(self, p, want_policy: bool = False, **kw) -> int:
        s = to_struct(p, **kw)
        t = C.c_uint64()
        check(lib().amy_server_submit(self._h, C.byref(s), int(want_policy), C.byref(t)))
        self._meta[t.value] = (p.n_x, p.horizon, want_policy)
        return int(t.value)

    def _collect(self, fn, ticket, *extra):
        import numpy as np
        n_x, T, want_pol = self._meta[ticket]
        V = np.empty(n_x, np.float64)
        pol = np.empty((T, n_x), np.int16) if (want_pol and T > 0) else None
        inf = Info()
        rc = fn(self._h, C.c_uint64(ticket), *extra, C.c_void_p(V.ctypes.data),
                C.c_void_p(pol.ctypes.data) if pol is not None else None, C.byref(inf))
        if rc == E_NOTREADY:
            return None
        del self._meta[ticket]
        check(rc)
        return V, pol, inf.as_dict()

    def poll(self, ticket: int):
        """(V, policy, info) when finished, else None."""
        return self._collect(lib().amy_server_poll, ticket)

    def wait(self, ticket: int, timeout_ms: int = -1):
        return self._collect(lib().amy_server_wait, ticket, C.c_int32(int(timeout_ms)))

    def cancel(self, ticket: int):
        """Cancel a queued or running request; its poll / wait then raise
        AmyError with status E_CANCELLED."""
        check(lib().amy_server_cancel(self._h, C.c_uint64(int(ticket))))

    def stats(self) -> dict:
        st = ServerStats()
        check(lib().amy_server_get_stats(self._h, C.byref(st)))
        return st.as_dict()

    def reset_stats(self):
        check(lib().amy_server_reset_stats(self._h))

    def close(self):
        if self._h:
            check(lib().amy_server_destroy(self._h))
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
