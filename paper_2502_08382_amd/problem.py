"""Marshalling of a subdomain description into the C-ABI record fields."""
from __future__ import annotations

import numpy as np


def subdomain_dict(sub, with_elements=False, with_kernel=True):
    """Fields of fetiF_subdomain from an object exposing Kreg (scipy CSR with
    the full symmetric pattern), dpn, coords, b_dof, b_sign, dual_map, R (the
    kernel basis, for the solver) and, for the adjoint, elem_dofs() and
    Ke_ref (dK_reg/dtheta_e)."""
    A = sub.Kreg
    d = dict(n=A.shape[0], dofs_per_node=sub.dpn, k_ptr=A.indptr, k_idx=A.indices,
             coords=np.asarray(sub.coords, dtype=np.float64), b_dof=sub.b_dof, b_sign=sub.b_sign,
             dual_map=sub.dual_map)
    if with_kernel and getattr(sub, "R", None) is not None:
        d["R"] = sub.R
    if with_elements:
        if np.ndim(sub.Ke_ref) != 2:
            raise ValueError("element data needs one dK_reg/dtheta_e shared by every element of the subdomain")
        d["elem_dofs"] = sub.elem_dofs()
        d["dK"] = sub.Ke_ref
    return d


def values_in_pattern(K, pattern):
    """The entries of the sparse matrix K at the positions of the CSR matrix
    `pattern` (zero where K has none), in pattern's value order: the layout
    fetiF_precond_values takes (K_i in the pattern of K_reg,i)."""
    P = pattern.tocsr()
    rows = np.repeat(np.arange(P.shape[0]), np.diff(P.indptr))
    return np.asarray(K.tocsr()[rows, P.indices]).ravel().astype(np.float64)
