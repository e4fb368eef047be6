"""CPU checks of the C ABI: the library loads, exports every declared
symbol, and validates problems before any device work."""
import ctypes
import glob
import math
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(amy_\w+)\s*\(", txt):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def A():
    import paper_2005_06191_amd as A
    A.binding.lib()
    return A


def test_every_declared_symbol_is_exported(A):
    names = _declared()
    assert {"amy_query", "amy_solve", "amy_last_error"} <= names
    lib = ctypes.CDLL(A.binding.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_version(A):
    assert "gfx950" in A.version()


def test_query_sizes_match_the_window_rule(A, orc):
    # L_i = floor(2 x*_i / h_i) + 1, clamped to the grid
    for p in (W.linear2d(), W.unicycle3d(), W.room5d(), W.vehicle7d()):
        q = A.query(p)
        for i in range(p.n):
            L = min(p.count[i], int(math.floor(2 * orc.xstar(p.var[i], p.cutoff) / p.h[i])) + 1)
            assert q["window"][i] == L
        assert q["W"] == math.prod(q["window"][:p.n])
        assert q["rows"] == p.n_x * p.n_u


def test_query_workspace_and_modes(A):
    p = W.room5d()
    otf = A.query(p.with_(mode="otf"))
    st = A.query(p.with_(mode="stored"))
    assert otf["mode"] == "otf" and st["mode"] == "stored"
    assert otf["stored_bytes"] == 0
    # FP32 stored rows: 64-state tiles x n_u x W x 4 B (+ int32 origins)
    tiles = (p.n_x + 63) // 64
    assert st["stored_bytes"] >= tiles * 64 * p.n_u * st["W"] * 4
    assert A.query(p.with_(mode="auto"))["mode"] == "otf"
    with pytest.raises(A.AmyError) as e:
        A.query(p.with_(mode="stored"), budget=1 << 30)
    assert e.value.status == A.binding.E_NOMEM


BAD = [
    ("zero variance", dict(var=(0.0, 0.01))),
    ("negative h", dict(h=(-0.04, 0.04))),
    ("zero count", dict(count=(0, 50))),
    ("negative horizon", dict(horizon=-1)),
    ("negative cutoff", dict(cutoff=-1e-3)),
    ("cutoff above density peak", dict(cutoff=10.0)),
    ("wrong param count", dict(params=(1.0, 2.0))),
    ("unicycle wrong dims", dict(dyn="unicycle", params=(0.1,))),
]


@pytest.mark.parametrize("what,kw", BAD, ids=[b[0] for b in BAD])
def test_invalid_problems_are_rejected(A, what, kw):
    p = W.linear2d().with_(**kw)
    with pytest.raises(A.AmyError) as e:
        A.query(p)
    assert e.value.status == A.binding.E_INVALID
    assert len(str(e.value)) > 20


def test_too_many_states_unsupported(A):
    p = W.linear2d().with_(count=(50000, 50000))
    with pytest.raises(A.AmyError) as e:
        A.query(p)
    assert e.value.status == A.binding.E_UNSUPPORTED


def test_variant_choice_on_the_host(A):
    """Variant feasibility is decided on the host: the factored sweep only
    where the last input digit moves the innermost window alone within the
    compiled bound (the unicycle workload), the compiled shapes only for
    their windows; AUTO picks the factored sweep where it applies."""
    uni = W.unicycle3d()
    assert A.query(uni)["variant"] == "factored"
    assert A.query(uni, variant="fixed")["variant"] == "fixed"
    assert A.query(uni, variant="lanes")["variant"] == "lanes"
    # a faster turn rate widens the heading windows' union beyond the bound
    fast = uni.with_(u_lo=(0.0, -3.0), u_hi=(1.0, 3.0))
    assert A.query(fast)["variant"] != "factored"
    for p in (W.room5d(), W.linear2d(mode="otf"), W.vehicle7d(), uni.with_(mode="stored")):
        with pytest.raises(A.AmyError) as e:
            A.query(p, variant="factored")
        assert e.value.status == A.binding.E_UNSUPPORTED


def test_grid_from_quantization_matches_printed_pair_counts(A):
    """The C helper of the paper's quantisation convention reproduces the
    pair counts |X x U| printed in Sec. 7 and Table 4."""
    import json
    import numpy as np
    with open(os.path.join(ROOT, "tests", "golden", "paper_sizes.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        lo, h, cx = A.grid_from_quantization(c["x_lb"], c["x_ub"], c["x_q"])
        ulo, uhi, cu = A.inputs_from_quantization(c["u_lb"], c["u_ub"], c["u_q"])
        assert int(np.prod(cx)) * int(np.prod(cu)) == c["pairs"], c["name"]
        for i in range(len(cx)):
            assert lo[i] == c["x_lb"][i] - c["x_q"][i] / 2 and h[i] == c["x_q"][i]
        for k in range(len(cu)):
            assert ulo[k] == c["u_lb"][k]
            assert abs(uhi[k] - c["u_ub"][k]) <= 1e-9 * max(1.0, abs(c["u_ub"][k]))
        # the Python description helper agrees
        assert W.grid_from_quantization(c["x_lb"], c["x_ub"], c["x_q"])[2] == cx


def test_grid_from_quantization_errors(A):
    with pytest.raises(A.AmyError):
        A.grid_from_quantization([0.0], [1.0], [0.0])
    with pytest.raises(A.AmyError):
        A.grid_from_quantization([1.0], [0.0], [0.1])
    with pytest.raises(A.AmyError):
        A.inputs_from_quantization([0.0] * 5, [1.0] * 5, [0.5] * 5)
    with pytest.raises(A.AmyError):
        A.grid_from_quantization([0.0], [math.inf], [0.1])
