"""Helpers shared by the GPU tests: solve through the C ABI, compare with the oracle."""
from __future__ import annotations

import sys
import time

import numpy as np

TOL_FP64 = 1e-12   # plain FP64 GPU path vs FP64 oracle
TOL_FP32 = 1e-5    # FP32 path vs FP64 oracle (the stated accuracy of the FP32 path)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_solve(p, policy=True, **kw):
    import paper_2005_06191_amd as A
    r = A.solve(p, policy=policy, **kw)
    V = r.V.cpu().numpy()
    pol = r.policy.cpu().numpy() if r.policy is not None else None
    return V, pol, r.info


def compare(p, ref, V, pol, tol, gap=None):
    """Element-wise value parity and policy parity where the oracle's best
    input beats the runner-up by more than 2 tol."""
    err = float(np.abs(V - ref["V"]).max()) if len(V) else 0.0
    assert err <= tol, f"{p.name}: max |V - V_oracle| = {err:.3e} > {tol:.1e}"
    if pol is not None and ref.get("policy") is not None and gap is not None:
        clear = gap > 2 * tol
        bad = int((pol[clear] != ref["policy"][clear]).sum())
        assert bad == 0, f"{p.name}: {bad} policy entries differ where the oracle gap > 2 tol"
    return err


class Timer:
    def __enter__(self):
        self.t = time.time()
        return self

    def __exit__(self, *a):
        self.dt = time.time() - self.t
