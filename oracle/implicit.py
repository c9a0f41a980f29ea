"""Python front of the oracle's C implicit apply (test infrastructure).

The fill-reducing order comes from a library routine (SuperLU's multiple
minimum degree on A^T+A, via scipy), taken only as a permutation; the
factorisation and the solves are the oracle's own plain C code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "implicit_cpu.c")
_LIB = os.path.join(_HERE, "liboracle_implicit.so")


def build():
    """Compile the oracle's C implicit apply (plain gcc, baseline x86-64)."""
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", _LIB, _SRC,
                           "-lm", "-lpthread"])
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p
        L.orc_create.restype = vp
        L.orc_create.argtypes = [ip]
        L.orc_destroy.argtypes = [vp]
        L.orc_set_sub.restype = ip
        L.orc_set_sub.argtypes = [vp, ip, ip, dp, dp, dp, dp, ip, dp, dp, dp]
        L.orc_factor_all.restype = ip
        L.orc_factor_all.argtypes = [vp, ip]
        L.orc_apply.argtypes = [vp, dp, dp, ip, ip]
        L.orc_nnz.restype = ctypes.c_long
        L.orc_nnz.argtypes = [vp, ip]
        _lib = L
    return _lib


def mmd_order(A):
    """Fill-reducing permutation (new -> old) from SuperLU's MMD on A^T+A."""
    lu = spla.splu(sp.csc_matrix(A), permc_spec="MMD_AT_PLUS_A",
                   diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
    return np.argsort(lu.perm_c).astype(np.int32)  # perm_c maps old -> new


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class ImplicitCPU:
    """q = sum_i D_i^T B~_i K_reg,i^{-1} B~_i^T D_i lambda on host threads."""

    def __init__(self, subs, n_lambda, nthreads=None, perms=None):
        L = _load()
        self.L = L
        self.n_lambda = int(n_lambda)
        self.nthreads = int(nthreads or os.cpu_count() or 1)
        self.h = L.orc_create(len(subs))
        self._keep = []
        for i, s in enumerate(subs):
            A = sp.csr_matrix(s.Kreg)
            Ap = A.indptr.astype(np.int32)
            Ai = A.indices.astype(np.int32)
            Ax = A.data.astype(np.float64)
            perm = perms[i] if perms is not None else mmd_order(A)
            perm = np.ascontiguousarray(perm, dtype=np.int32)
            bd = np.ascontiguousarray(s.b_dof, dtype=np.int32)
            bs = np.ascontiguousarray(s.b_sign, dtype=np.int8)
            dm = np.ascontiguousarray(s.dual_map, dtype=np.int32)
            rc = L.orc_set_sub(self.h, i, A.shape[0], _p(Ap), _p(Ai), _p(Ax), _p(perm),
                               len(bd), _p(bd), _p(bs), _p(dm))
            if rc != 0:
                raise RuntimeError("orc_set_sub failed")
        self.nsub = len(subs)

    def factor(self):
        rc = self.L.orc_factor_all(self.h, self.nthreads)
        if rc != 0:
            raise RuntimeError(f"oracle Cholesky failed on subdomain {-rc - 1}")

    def nnz(self):
        return sum(self.L.orc_nnz(self.h, i) for i in range(self.nsub))

    def apply(self, lam, out=None):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        q = out if out is not None else np.empty(self.n_lambda)
        self.L.orc_apply(self.h, _p(lam), _p(q), self.n_lambda, self.nthreads)
        return q

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_destroy(self.h)
            self.h = None
