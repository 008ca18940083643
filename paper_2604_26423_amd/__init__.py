"""MI355X (gfx950) state-vector simulation of LR-QAOA circuits (arXiv:2604.26423).

The compute path is libqs.so (HIP kernels behind the C ABI of include/qs.h);
``qs`` is its thin binding and ``lrqaoa`` the schedule / simulator layer.
Nothing here falls back to a CPU implementation: without the built library
every call raises.
"""
from . import qs  # noqa: F401
from .lrqaoa import (Batch, Simulator, Trajectories, expect_c, gate_grad_to_schedule, linear_ramp,  # noqa: F401
                     mean_of_means, to_gate_angles)

__all__ = ["qs", "Batch", "Simulator", "Trajectories", "expect_c", "linear_ramp", "to_gate_angles",
           "gate_grad_to_schedule", "mean_of_means"]
