"""CPU tests of the library's host side: the C-ABI exports, the nested
dissection + supernodal Cholesky that feed the device, argument validation."""
import ctypes
import re

import numpy as np
import pytest
import scipy.sparse as sp

from synth import make_problem, config_problem
from oracle import feti
from paper_2502_08382_amd import HostFactor, subdomain_dict, load_library, FetiContext, FetiError
from paper_2502_08382_amd.fetif import EXPORTS


HEADER = __import__("os").path.join(__import__("os").path.dirname(__file__), "..", "include", "fetiF.h")


def _gpu_present():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_every_binding_declares_its_argument_types():
    """Without argtypes ctypes passes Python ints as C int: a 64-bit stream
    handle or pointer would be cut to 32 bits."""
    from paper_2502_08382_amd.fetif import EXPORTS, load_library
    L = load_library()
    missing = [n for n in EXPORTS if getattr(L, n).argtypes is None]
    assert not missing, missing


def test_library_exports_every_declared_symbol():
    src = open(HEADER).read()
    names = set(re.findall(r"\b(fetiF_[A-Za-z_]+)\s*\(", src))
    names = {n for n in names if not n.endswith("_s")}
    assert names, "no declarations found"
    L = load_library()
    for n in sorted(names):
        assert hasattr(L, n), f"{n} declared in include/fetiF.h but not exported"
    assert set(EXPORTS) <= names


def _problems():
    return {
        "heat2d": make_problem(2, "heat", [[5, 7], [6, 4]], 0.5, dirichlet_axis=0, seed=2),
        "heat3d": make_problem(3, "heat", [[4, 5], [5, 4], [3, 4]], 1.0, dirichlet_axis=2, seed=3),
        "elast3d": make_problem(3, "elasticity", [[3, 4], [3, 3], [4, 3]], 0.0, dirichlet_axis=2, seed=4),
        "heat1d": make_problem(1, "heat", [[9, 6, 11]], 0.5, dirichlet_axis=0, seed=5),
    }


@pytest.mark.parametrize("kind", list(_problems().keys()))
@pytest.mark.parametrize("coords", [True, False])
def test_host_factor_reproduces_permuted_matrix(kind, coords):
    P = _problems()[kind]
    for s in P.subs[:3]:
        d = subdomain_dict(s)
        if not coords:
            d["coords"] = None
        h = HostFactor(d, s.Kreg.data)
        perm, cp, ri, vv = h.export()
        assert np.array_equal(np.sort(perm), np.arange(s.n))        # a permutation
        if s.dpn > 1:  # DOFs of a node stay together
            assert np.all(perm.reshape(-1, s.dpn) // s.dpn == (perm.reshape(-1, s.dpn) // s.dpn)[:, :1])
        Lm = sp.csc_matrix((vv, ri, cp), shape=(s.n, s.n))
        assert sp.tril(Lm).nnz == Lm.nnz                            # lower triangular
        A = s.Kreg[perm][:, perm]
        err = abs(Lm @ Lm.T - A).max() / abs(A).max()
        assert err <= 1e-14
        sn = h.supernodes()
        # supernodes partition the columns, children precede parents
        ends = sn["first"] + sn["ncols"]
        assert sn["first"][0] == 0 and ends[-1] == s.n and np.all(sn["first"][1:] == ends[:-1])
        par = sn["parent"]
        assert np.all((par == -1) | (par > np.arange(len(par))))
        assert np.all(sn["level"][par[par >= 0]] > sn["level"][par >= 0])


def test_host_factor_is_independent_of_ordering_in_F():
    """F~_i computed from the library's factor equals the oracle's F~_i."""
    P = _problems()["heat3d"]
    for s in P.subs[:2]:
        h = HostFactor(subdomain_dict(s), s.Kreg.data)
        perm, cp, ri, vv = h.export()
        Lm = sp.csc_matrix((vv, ri, cp), shape=(s.n, s.n)).toarray()
        pinv = np.empty_like(perm)
        pinv[perm] = np.arange(s.n)
        Bt = np.zeros((s.n, s.m))
        Bt[pinv[s.b_dof], np.arange(s.m)] = s.b_sign
        from scipy.linalg import solve_triangular
        X = solve_triangular(Lm, Bt, lower=True)
        F = X.T @ X
        Fo = feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign)
        assert np.linalg.norm(F - Fo) <= 1e-12 * np.linalg.norm(Fo)


def test_host_factor_reports_non_spd():
    P = _problems()["heat2d"]
    s = P.subs[0]
    vals = s.Kreg.data.copy()
    A = s.Kreg.tocoo()
    diag = np.nonzero(A.row == A.col)[0]
    vals[diag[5]] = -1.0
    with pytest.raises(FetiError) as e:
        HostFactor(subdomain_dict(s), vals)
    assert e.value.status == 5  # FETIF_ENOTSPD


def test_nested_dissection_quality_3d():
    """Geometric ND keeps the 13^3 heat factor near the separator bound."""
    P = config_problem(2, scale=(2, 12))
    s = P.subs[0]
    h = HostFactor(subdomain_dict(s), None)
    assert h.nnz < 260_000          # natural order would give ~ 2197*183 = 402k
    sn = h.supernodes()
    assert sn["ncols"].max() == 169  # the top separator plane is one supernode


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device path")
def test_create_without_device_reports_edevice():
    P = _problems()["heat2d"]
    with pytest.raises(FetiError) as e:
        FetiContext([subdomain_dict(s) for s in P.subs], P.n_lambda)
    assert e.value.status == 4


@pytest.mark.parametrize("bad", ["dual_map_order", "dual_map_range", "b_sign", "b_dof", "n_lambda", "no_multipliers"])
def test_create_validates_arguments(bad):
    P = _problems()["heat2d"]
    subs = [subdomain_dict(s) for s in P.subs]
    nl = P.n_lambda
    d = dict(subs[1])
    if bad == "dual_map_order":
        d["dual_map"] = d["dual_map"][::-1].copy()
    elif bad == "dual_map_range":
        d["dual_map"] = d["dual_map"] + nl
    elif bad == "b_sign":
        d["b_sign"] = np.zeros_like(d["b_sign"])
    elif bad == "b_dof":
        d["b_dof"] = d["b_dof"] + 10 ** 6
    elif bad == "n_lambda":
        nl = 0
    elif bad == "no_multipliers":
        d["b_dof"] = np.zeros(0, np.int32)
        d["b_sign"] = np.zeros(0, np.int8)
        d["dual_map"] = np.zeros(0, np.int32)
    subs[1] = d
    with pytest.raises(FetiError) as e:
        FetiContext(subs, nl)
    assert e.value.status == 1


def test_binding_refuses_wrong_device_vectors():
    """Device vectors are checked before the library is called: float64,
    contiguous, exactly the expected length, on the context's GPU (the
    library reads and writes 8 bytes per element through the pointer)."""
    import torch
    ctx = FetiContext.__new__(FetiContext)          # no library call is reached
    ctx.h, ctx.L, ctx.device = None, None, 0
    ctx.n_lambda, ctx.n_dofs, ctx.n_elems, ctx.n_coarse = 10, 40, 8, 2
    good = torch.zeros(10, dtype=torch.float64)
    cases = [
        (lambda: ctx.apply(torch.zeros(10, dtype=torch.float32), good), TypeError, "float64"),
        (lambda: ctx.apply(torch.zeros(20, dtype=torch.float64)[::2], good), ValueError, "contiguous"),
        (lambda: ctx.apply(torch.zeros(9, dtype=torch.float64), good), ValueError, "expected 10"),
        (lambda: ctx.apply(good, good.clone()), ValueError, "cuda:0"),          # host tensor
        (lambda: ctx.apply_implicit(good, torch.zeros(11, dtype=torch.float64)), ValueError, "expected 10"),
        (lambda: ctx.apply_backward(good, good, good, torch.zeros(7, dtype=torch.float64)), ValueError,
         "expected 8"),
        (lambda: ctx.dual_rhs(torch.zeros(39, dtype=torch.float64), good), ValueError, "expected 40"),
        (lambda: ctx.coarse_rhs(torch.zeros(40, dtype=torch.float64), torch.zeros(3, dtype=torch.float64)),
         ValueError, "expected 2"),
        (lambda: ctx.pcpg(good, torch.zeros(2, dtype=torch.int64), good), TypeError, "float64"),
        (lambda: ctx.primal(torch.zeros(40, dtype=torch.float64), good, good, torch.zeros(2, dtype=torch.float64),
                            torch.zeros(41, dtype=torch.float64)), ValueError, "expected 40"),
    ]
    for fn, exc, text in cases:
        with pytest.raises(exc, match=text):
            fn()
