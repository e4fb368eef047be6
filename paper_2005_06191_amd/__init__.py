"""MI355X-native AMYTISS hot path: finite-MDP abstraction of stochastic
control systems and finite-horizon Bellman synthesis (safety, reach,
reach-avoid), stored or on-the-fly, behind the C ABI of include/amytiss.h.

The compute runs in libamytiss_hip.so (hand-written HIP for gfx950);
``binding`` marshals arguments and allocates device memory with PyTorch.
"""
from .binding import (AmyError, Result, Solver, query, solve, version)  # noqa: F401

__all__ = ["AmyError", "Result", "Solver", "query", "solve", "version"]
