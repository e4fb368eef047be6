"""MI355X-native AMYTISS hot path: finite-MDP abstraction of stochastic
control systems and finite-horizon Bellman synthesis (safety, reach,
reach-avoid), stored or on-the-fly, behind the C ABI of include/amytiss.h.

The compute runs in libamytiss_hip.so (hand-written HIP for gfx950);
``binding`` marshals arguments and allocates device memory with PyTorch.
"""
from .binding import (AmyError, BatchSolver, Result, Server, Solver, batch_query, batch_solve,  # noqa: F401
                      grid_from_quantization, inputs_from_quantization, query, solve, solve_static,
                      tune_clear, tune_entries, tune_load, tune_save, tune_solve, version, UserDynamics)

__all__ = ["AmyError", "BatchSolver", "Result", "Server", "Solver", "batch_query", "batch_solve",
           "grid_from_quantization", "inputs_from_quantization", "query", "solve", "solve_static", "UserDynamics", "tune_clear", "tune_entries", "tune_load", "tune_save", "tune_solve", "version"]
