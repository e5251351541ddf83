"""Cross-entropy optimisation of physically grounded task-and-motion plans on MI355X.

The hot path - Philox sampling, the persistent rollout kernels, elite select
and FP64 refit - lives in libcemtamp.so (C ABI: include/cemtamp.h), built from
csrc/ by `python -m paper_2512_11571_amd.build`.  `binding` marshals Python
arguments into it; `workloads` reads the synthetic scene descriptions.
"""
from . import workloads
from .binding import CemError, Context, lib

__all__ = ["Context", "CemError", "lib", "workloads"]
