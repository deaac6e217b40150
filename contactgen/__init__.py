"""Seeded synthetic inputs for the mortar-contact saddle-point solver.

Builds the linear two-body contact systems (blocks K, G, B, C, right-hand
side, interface maps, rigid-body modes) that both the CPU oracle and the GPU
library consume.  Holds no part of the multigrid method itself.
"""
from .problem import (ContactProblem, WORKLOADS, make_contact_problem, make_workload, rotate_problem,
                      weak_scaling_problem)

__all__ = ["ContactProblem", "WORKLOADS", "make_contact_problem", "make_workload", "rotate_problem",
           "weak_scaling_problem"]
