"""Python front of the oracle's C implicit apply (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library.

The fill-reducing order is only a permutation (the factor of the permuted
matrix represents the same K_reg^{-1}): by default a geometric nested
dissection of the subdomain's grid nodes written here (plane separators
through the median of the longest axis, the order the paper's CPU solvers
get from METIS in spirit), or a library routine (SuperLU's multiple minimum
degree on A^T+A, via scipy).  The factorisation, the solves and the explicit
assembly are the oracle's own plain C code.
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
        L.orc_opnorm_all.argtypes = [vp, ip, dp, ip]
        L.orc_kappa_all.argtypes = [vp, ip, dp, ip]
        L.orc_assemble_all.argtypes = [vp, ip]
        L.orc_get_F.restype = ip
        L.orc_get_F.argtypes = [vp, ip, dp]
        L.orc_apply_explicit.argtypes = [vp, dp, dp, ip, ip]
        L.orc_solve.restype = ip
        L.orc_solve.argtypes = [vp, ip, dp]
        _lib = L
    return _lib


def nd_order(coords, dpn, leaf=64):
    """Nested-dissection order (new -> old DOF) of a structured grid
    subdomain from its integer node coordinates (nnodes x dim): the nodes
    on the grid plane through the median of the longest axis separate the
    two halves (elements live inside grid cells, so no element couples the
    two sides), each half is ordered recursively, the separator last; sets
    of at most `leaf` nodes keep their natural order.  DOFs of a node stay
    together (dof = dpn * node + component)."""
    coords = np.asarray(coords)
    parts = []

    def rec(idx):
        c = coords[idx]
        ext = c.max(axis=0) - c.min(axis=0) if len(idx) else np.zeros(1)
        ax = int(np.argmax(ext))
        if len(idx) <= leaf or ext[ax] < 2:
            parts.append(idx)
            return
        lo, hi = c[:, ax].min(), c[:, ax].max()
        v = min(max(np.sort(c[:, ax])[len(idx) // 2], lo + 1), hi - 1)
        rec(idx[c[:, ax] < v])
        rec(idx[c[:, ax] > v])
        parts.append(idx[c[:, ax] == v])

    rec(np.arange(len(coords)))
    nodes = np.concatenate(parts)
    return (nodes[:, None] * dpn + np.arange(dpn)[None, :]).ravel().astype(np.int32)


def mmd_order(A):
    """Fill-reducing permutation (new -> old) from SuperLU's MMD on A^T+A."""
    lu = spla.splu(sp.csc_matrix(A), permc_spec="MMD_AT_PLUS_A",
                   diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
    return np.argsort(lu.perm_c).astype(np.int32)  # perm_c maps old -> new


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class ImplicitCPU:
    """q = sum_i D_i^T B~_i K_reg,i^{-1} B~_i^T D_i lambda on host threads."""

    def __init__(self, subs, n_lambda, nthreads=None, perms=None, order="nd"):
        """perms: per-subdomain permutations (new -> old) to use as given;
        else order "nd" (geometric nested dissection from the subdomain's
        node coordinates) or "mmd" (SuperLU's minimum degree)."""
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
            if perms is not None:
                perm = perms[i]
            elif order == "nd":
                perm = nd_order(s.coords, s.dpn)
            else:
                perm = mmd_order(A)
            perm = np.ascontiguousarray(perm, dtype=np.int32)
            bd = np.ascontiguousarray(s.b_dof, dtype=np.int32)
            bs = np.ascontiguousarray(s.b_sign, dtype=np.int8)
            dm = np.ascontiguousarray(s.dual_map, dtype=np.int32)
            rc = L.orc_set_sub(self.h, i, A.shape[0], _p(Ap), _p(Ai), _p(Ax), _p(perm),
                               len(bd), _p(bd), _p(bs), _p(dm))
            if rc != 0:
                raise RuntimeError("orc_set_sub failed")
        self.nsub = len(subs)
        self.m = [len(s.b_dof) for s in subs]

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

    def opnorms(self, iters=60):
        """||F~_i||_2 of every subdomain (power iteration with the factors;
        the Rayleigh quotient of the last iterate, a lower estimate)."""
        out = np.empty(self.nsub)
        self.L.orc_opnorm_all(self.h, int(iters), _p(out), self.nthreads)
        return out

    def kappas(self, iters=60):
        """Condition numbers of every K_reg,i (power iteration for the
        largest eigenvalue, inverse iteration for the smallest)."""
        out = np.empty(self.nsub)
        self.L.orc_kappa_all(self.h, int(iters), _p(out), self.nthreads)
        return out

    def assemble(self):
        """Explicit F~_i of every subdomain, one unit solve per column."""
        self.L.orc_assemble_all(self.h, self.nthreads)

    def dual_operator(self, i):
        """The assembled F~_i (m_i x m_i, local multiplier order)."""
        out = np.empty((self.m[i], self.m[i]))
        if self.L.orc_get_F(self.h, int(i), _p(out)) != 0:
            raise RuntimeError("assemble() first")
        return out

    def apply_explicit(self, lam, out=None):
        """q = sum_i D_i^T F~_i D_i lambda with the assembled dense F~_i."""
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        q = out if out is not None else np.empty(self.n_lambda)
        self.L.orc_apply_explicit(self.h, _p(lam), _p(q), self.n_lambda, self.nthreads)
        return q

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_destroy(self.h)
            self.h = None


class SparseRegInverse:
    """K_reg^{-1} of one matrix through the oracle's sparse Cholesky factor
    (nested-dissection order from the node coordinates), with one step of
    iterative refinement whose residual is formed in extended precision,
    like oracle.feti.RegInverse but without the dense factorisation."""

    def __init__(self, Kreg, coords, dpn):
        L = _load()
        self.L = L
        A = sp.csr_matrix(Kreg)
        self.K = A
        self.Kl = A.astype(np.longdouble)
        self.n = A.shape[0]
        self.h = L.orc_create(1)
        Ap = A.indptr.astype(np.int32)
        Ai = A.indices.astype(np.int32)
        Ax = A.data.astype(np.float64)
        perm = nd_order(coords, dpn)
        none = np.zeros(1, np.int32)
        rc = L.orc_set_sub(self.h, 0, self.n, _p(Ap), _p(Ai), _p(Ax), _p(perm), 0, _p(none),
                           _p(np.zeros(1, np.int8)), _p(none))
        if rc != 0 or L.orc_factor_all(self.h, 1) != 0:
            raise RuntimeError("oracle sparse Cholesky failed")

    def _solve(self, b):
        x = np.array(b, dtype=np.float64, copy=True, order="C")
        self.L.orc_solve(self.h, 0, _p(x))
        return x

    def solve(self, rhs, refine=True):
        rhs = np.asarray(rhs, dtype=np.float64)
        x = self._solve(rhs)
        if refine:
            r = rhs.astype(np.longdouble) - self.Kl @ x.astype(np.longdouble)
            x = x + self._solve(np.asarray(r, dtype=np.float64))
        return x

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_destroy(self.h)
            self.h = None
