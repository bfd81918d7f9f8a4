"""Seeded synthetic inputs for the EQS explicit-RKC hot path.

This package builds input data only: tetrahedral meshes of the unit cube,
material tables and per-tet material ids, Dirichlet node sets with their drive
functions, and seeded random states. It holds none of the method's arithmetic
(no element matrices, no solves, no time stepping), so both the CPU oracle and
the HIP library can consume its output without sharing any method code.

The workloads mirror the paper's field-grading setting (Sec. V: a microvaristor
coating with field-dependent conductivity inside a polymer insulator) on cube
meshes, because the paper's insulator model is not available.
"""

from .mesh import kuhn_cube_mesh, kuhn_cube_mesh_p2, permute_nodes, shuffle_tets
from .config import CONFIG_DIR, cases_from_config, config_names, load_config
from .cases import (
    Case,
    make_case,
    layered_case,
    case_c0,
    case_c1,
    case_c2,
    case_batch,
    case_p2,
    case_c0_p2,
    random_state,
    mlp_init,
    CASE_NAMES,
)

__all__ = [
    "Case",
    "kuhn_cube_mesh",
    "kuhn_cube_mesh_p2",
    "case_p2",
    "case_c0_p2",
    "permute_nodes",
    "shuffle_tets",
    "make_case",
    "layered_case",
    "case_c0",
    "case_c1",
    "case_c2",
    "case_batch",
    "random_state",
    "mlp_init",
    "CASE_NAMES",
    "CONFIG_DIR",
    "config_names",
    "load_config",
    "cases_from_config",
]
