"""Seeded synthetic FETI problems (inputs only).

This package builds the torn finite-element problems that both the CPU oracle
and the GPU library consume: subdomain stiffness matrices K_i and their
regularised form K_reg,i, the signed gluing/Dirichlet rows B~_i with their
dual-index maps D_i, loads f_i, kernel bases R_i, and seeded dual vectors.
It holds none of the dual-operator arithmetic (no factorisation, no solve, no
F_i): everything here is problem *definition* (Sec. II, the FEM system, the
Total-FETI tearing and the generalised-inverse regularisation).
"""
from .problems import (Problem, Subdomain, make_problem, config_problem,
                       element_matrix, simplex_element_matrix, kuhn_simplices,
                       assemble_stiffness, workload_name, CONFIGS, CONFIGS_SIMPLEX)

__all__ = ["Problem", "Subdomain", "make_problem", "config_problem",
           "element_matrix", "simplex_element_matrix", "kuhn_simplices",
           "assemble_stiffness", "workload_name", "CONFIGS", "CONFIGS_SIMPLEX"]
