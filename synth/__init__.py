"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This module holds no arithmetic of the method: it only states problems (lattice
bond lists, fillings, U), draws seeded random vectors with numpy's PCG64, and
lists the named workloads.  Both the oracle and the HIP path consume what it
produces; neither imports the other.
"""
from .lattices import Bond, ring, torus, torus_nnn, single_bond
from .workloads import Workload, WORKLOADS, workload, batched_workloads
from .vectors import random_vector

__all__ = ["Bond", "ring", "torus", "torus_nnn", "single_bond", "Workload",
           "WORKLOADS", "workload", "batched_workloads", "random_vector"]
