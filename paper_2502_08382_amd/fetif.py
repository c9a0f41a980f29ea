"""ctypes binding of the fetiF C-ABI (argument marshalling only).

Every computation runs in libfetiF.so: host analysis/factorisation in its
C++ part, assembly and application in its HIP kernels.  Device buffers are
torch tensors (or raw device pointers); streams are torch CUDA streams.
If the shared library is missing this module raises at import of the
library, so nothing can silently run elsewhere.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfetiF.so")

F64, F32, BF16 = 0, 1, 2
_PREC = {"f64": F64, "fp64": F64, "float64": F64, "f32": F32, "fp32": F32, "float32": F32,
         "bf16": BF16, "bfloat16": BF16}

_STATUS = {0: "FETIF_OK", 1: "FETIF_EINVAL", 2: "FETIF_ENOMEM", 3: "FETIF_ESTATE",
           4: "FETIF_EDEVICE", 5: "FETIF_ENOTSPD", 6: "FETIF_ENOTSUP", 7: "FETIF_ENONFINITE"}


class FetiError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")


class _Sub(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("dofs_per_node", ctypes.c_int32),
                ("k_ptr", ctypes.c_void_p), ("k_idx", ctypes.c_void_p),
                ("dim", ctypes.c_int32), ("coords", ctypes.c_void_p),
                ("m", ctypes.c_int32), ("b_dof", ctypes.c_void_p), ("b_sign", ctypes.c_void_p),
                ("dual_map", ctypes.c_void_p), ("nelem", ctypes.c_int32), ("edofs", ctypes.c_int32),
                ("elem_dofs", ctypes.c_void_p), ("dK", ctypes.c_void_p),
                ("nkernel", ctypes.c_int32), ("R", ctypes.c_void_p)]


class _Opt(ctypes.Structure):
    _fields_ = [("f_storage", ctypes.c_int), ("leaf_nodes", ctypes.c_int32),
                ("nthreads", ctypes.c_int32), ("apply_band", ctypes.c_int32),
                ("trsm_chunk", ctypes.c_int32), ("apply_rows", ctypes.c_int32),
                ("apply_nontemporal", ctypes.c_int32), ("apply_split", ctypes.c_int32),
                ("trsm_panel", ctypes.c_int32), ("apply_seg", ctypes.c_int32),
                ("assembly_groups", ctypes.c_int32), ("schur_order", ctypes.c_int32),
                ("debug_checks", ctypes.c_int32)]


class _PcpgOpt(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iters", ctypes.c_int32), ("fixed_iters", ctypes.c_int32),
                ("implicit", ctypes.c_int32), ("check_every", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("use_graph", ctypes.c_int32), ("precond", ctypes.c_int32)]


class _PcpgRes(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("w0", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("nsub", ctypes.c_int32), ("n_lambda", ctypes.c_int64), ("sum_m", ctypes.c_int64),
                ("factor_values", ctypes.c_int64), ("x_values", ctypes.c_int64),
                ("f_elements", ctypes.c_int64), ("f_tri_elements", ctypes.c_int64),
                ("trsm_flops", ctypes.c_double), ("syrk_flops", ctypes.c_double),
                ("factor_flops", ctypes.c_double), ("trsm_levels", ctypes.c_int32),
                ("apply_groups", ctypes.c_int32), ("apply_elements", ctypes.c_int64),
                ("assembly_groups", ctypes.c_int32), ("trsm_bwd_flops", ctypes.c_double)]


EXPORTS = ["fetiF_create", "fetiF_factor_upload", "fetiF_assemble", "fetiF_apply",
           "fetiF_apply_backward", "fetiF_download_F", "fetiF_query", "fetiF_destroy",
           "fetiF_last_error", "fetiF_host_factor", "fetiF_hfactor_info", "fetiF_hfactor_export",
           "fetiF_hfactor_supernodes", "fetiF_hfactor_free", "fetiF_profile_enable",
           "fetiF_profile_read", "fetiF_set_apply", "fetiF_apply_implicit", "fetiF_dual_rhs",
           "fetiF_coarse_rhs", "fetiF_pcpg", "fetiF_primal", "fetiF_set_assembly", "fetiF_factor_assemble",
           "fetiF_apply_static", "fetiF_set_assembly_path", "fetiF_apply_host", "fetiF_precond_values",
           "fetiF_read_probe"]

PHASES = ["factor_copy", "rhs_init", "trsm", "syrk", "apply_band", "apply_gather", "solves", "trsm_bwd", "spmm"]

_lib = None


def load_library(path=None):
    """Load libfetiF.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"fetiF library not built: {p} is missing (run __graft_entry__.build())")
    L = ctypes.CDLL(p)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.fetiF_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i64, i32, ctypes.POINTER(_Sub),
                               ctypes.POINTER(_Opt)]
    L.fetiF_factor_upload.argtypes = [vp, i32, i32, ctypes.POINTER(vp), vp]
    L.fetiF_assemble.argtypes = [vp, vp]
    L.fetiF_factor_assemble.argtypes = [vp, ctypes.POINTER(vp), vp]
    L.fetiF_apply.argtypes = [vp, vp, vp, vp]
    L.fetiF_apply_static.argtypes = [vp, vp, vp, vp]
    L.fetiF_apply_host.argtypes = [vp, vp, vp, i32, vp]
    L.fetiF_precond_values.argtypes = [vp, i32, i32, ctypes.POINTER(vp)]
    L.fetiF_read_probe.argtypes = [vp, i64, i64, vp, vp]
    L.fetiF_apply_backward.argtypes = [vp, vp, vp, vp, vp, vp]
    L.fetiF_download_F.argtypes = [vp, i32, vp]
    L.fetiF_query.argtypes = [vp, ctypes.POINTER(_Info)]
    L.fetiF_destroy.argtypes = [vp]
    L.fetiF_last_error.argtypes = [vp]
    L.fetiF_last_error.restype = ctypes.c_char_p
    L.fetiF_host_factor.argtypes = [ctypes.POINTER(_Sub), vp, ctypes.POINTER(_Opt), ctypes.POINTER(vp)]
    L.fetiF_hfactor_info.argtypes = [vp, vp, vp, vp, vp]
    L.fetiF_hfactor_export.argtypes = [vp, vp, vp, vp, vp]
    L.fetiF_hfactor_supernodes.argtypes = [vp, vp, vp, vp, vp, vp]
    L.fetiF_hfactor_free.argtypes = [vp]
    L.fetiF_profile_enable.argtypes = [vp, ctypes.c_int]
    L.fetiF_profile_read.argtypes = [vp, ctypes.c_int, vp, vp, i32]
    L.fetiF_set_apply.argtypes = [vp, i32, i32, i32, i32, i32]
    L.fetiF_set_assembly.argtypes = [vp, i32, i32]
    L.fetiF_set_assembly_path.argtypes = [vp, i32]
    L.fetiF_apply_implicit.argtypes = [vp, vp, vp, vp]
    L.fetiF_dual_rhs.argtypes = [vp, vp, vp, vp, vp]
    L.fetiF_coarse_rhs.argtypes = [vp, vp, vp, vp]
    L.fetiF_pcpg.argtypes = [vp, vp, vp, vp, ctypes.POINTER(_PcpgOpt), ctypes.POINTER(_PcpgRes), vp]
    L.fetiF_primal.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    for name in EXPORTS:
        getattr(L, name).restype = getattr(L, name).restype if name == "fetiF_last_error" else ctypes.c_int
    _lib = L
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p).value


def _dptr(t):
    """Device pointer of a torch tensor or an int."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _check_vecs(named, device):
    """Device vector arguments, name -> (value, expected length): each a raw
    pointer (int, passed as is), None where optional, or a contiguous
    float64 torch tensor of exactly that many elements on the context's
    device.  The library reads or writes 8 bytes per element through the
    pointer, so a shorter, strided, differently typed or host tensor is
    refused here (types and lengths of all arguments first, then devices)."""
    import torch
    tensors = []
    for name, (t, n) in named.items():
        if t is None or isinstance(t, int):
            continue
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name}: expected a torch tensor or a device pointer, got {type(t).__name__}")
        if t.dtype != torch.float64:
            raise TypeError(f"{name}: dtype must be torch.float64, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: must be contiguous")
        if t.numel() != n:
            raise ValueError(f"{name}: expected {n} elements, got {t.numel()}")
        tensors.append((name, t))
    for name, t in tensors:
        if t.device.type != "cuda" or (t.device.index if t.device.index is not None
                                        else torch.cuda.current_device()) != device:
            raise ValueError(f"{name}: must live on cuda:{device}, got {t.device}")


def _stream(stream):
    if stream is None:
        try:
            import torch
            return torch.cuda.current_stream().cuda_stream
        except Exception:
            return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class _SubArrays:
    """Keeps the numpy arrays of one subdomain alive and builds its record."""

    def __init__(self, d):
        self.k_ptr = np.ascontiguousarray(d["k_ptr"], dtype=np.int32)
        self.k_idx = np.ascontiguousarray(d["k_idx"], dtype=np.int32)
        self.n = int(d["n"])
        self.dpn = int(d.get("dofs_per_node", 1))
        c = d.get("coords")
        self.coords = None if c is None else np.ascontiguousarray(c, dtype=np.float64)
        self.dim = 0 if c is None else int(self.coords.shape[1])
        self.b_dof = np.ascontiguousarray(d["b_dof"], dtype=np.int32)
        self.b_sign = np.ascontiguousarray(d["b_sign"], dtype=np.int8)
        self.dual_map = np.ascontiguousarray(d["dual_map"], dtype=np.int32)
        ed = d.get("elem_dofs")
        self.elem_dofs = None if ed is None else np.ascontiguousarray(ed, dtype=np.int32)
        dk = d.get("dK")
        self.dK = None if dk is None else np.ascontiguousarray(dk, dtype=np.float64)
        R = d.get("R")
        self.R = None if R is None else np.ascontiguousarray(R, dtype=np.float64)

    def record(self):
        ne = 0 if self.elem_dofs is None else self.elem_dofs.shape[0]
        ed = 0 if self.elem_dofs is None else self.elem_dofs.shape[1]
        return _Sub(self.n, self.dpn, _ptr(self.k_ptr), _ptr(self.k_idx), self.dim, _ptr(self.coords),
                    len(self.b_dof), _ptr(self.b_dof), _ptr(self.b_sign), _ptr(self.dual_map), ne, ed,
                    _ptr(self.elem_dofs), _ptr(self.dK), 0 if self.R is None else self.R.shape[1],
                    _ptr(self.R))


def _options(f_storage="f64", leaf_nodes=0, nthreads=0, apply_band=0, trsm_chunk=0, apply_rows=0,
             apply_nontemporal=-1, apply_split=-1, trsm_panel=0, apply_seg=-1, assembly_groups=0, schur_order=0,
             debug_checks=0):
    prec = _PREC[f_storage] if isinstance(f_storage, str) else int(f_storage)
    return _Opt(prec, leaf_nodes, nthreads, apply_band, trsm_chunk, apply_rows, apply_nontemporal, apply_split,
                trsm_panel, apply_seg, assembly_groups, int(schur_order), int(bool(debug_checks)))


def read_probe(buf, region_bytes, out, stream=None):
    """Streaming-read probe (measurement aid, fetiF_read_probe): every
    work-group sums one contiguous region of the device tensor buf into out
    (a float64 device tensor of ceil(bytes / region_bytes) entries)."""
    L = load_library()
    nbytes = buf.numel() * buf.element_size()
    ngroups = -(-nbytes // region_bytes)
    if out.numel() < ngroups or out.dtype.itemsize != 8:
        raise ValueError(f"out needs {ngroups} float64 entries")
    st = L.fetiF_read_probe(_dptr(buf), int(nbytes), int(region_bytes), _dptr(out), _stream(stream))
    if st != 0:
        raise FetiError(st, L.fetiF_last_error(None).decode())


class FetiContext:
    """One fetiF context: F~_i of every subdomain on one device."""

    def __init__(self, subdomains, n_lambda, device=0, f_storage="f64", **opts):
        L = load_library()
        self.L = L
        self._subs = [_SubArrays(d) for d in subdomains]
        recs = (_Sub * len(self._subs))(*[s.record() for s in self._subs])
        opt = _options(f_storage, **opts)
        h = ctypes.c_void_p()
        st = L.fetiF_create(ctypes.byref(h), int(device), int(n_lambda), len(self._subs), recs,
                            ctypes.byref(opt))
        if st != 0:
            raise FetiError(st, L.fetiF_last_error(None).decode())
        self.h = h
        self.n_lambda = int(n_lambda)
        self.device = int(device)
        self.f_storage = opt.f_storage
        self.nsub = len(self._subs)
        self.m = [len(s.b_dof) for s in self._subs]
        self.n_dofs = sum(s.n for s in self._subs)
        self.n_elems = sum(0 if s.elem_dofs is None else s.elem_dofs.shape[0] for s in self._subs)
        self.n_coarse = sum(0 if s.R is None else s.R.shape[1] for s in self._subs)

    def _vecs(self, **named):
        """Validate device vector arguments: name=(tensor, expected length)."""
        _check_vecs(named, self.device)

    def _check(self, st):
        if st != 0:
            raise FetiError(st, self.L.fetiF_last_error(self.h).decode())

    def factor_upload(self, k_vals, first=0, stream=None):
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in k_vals]
        ptrs = (ctypes.c_void_p * len(arrs))(*[_ptr(a) for a in arrs])
        self._check(self.L.fetiF_factor_upload(self.h, int(first), len(arrs), ptrs, _stream(stream)))

    def assemble(self, stream=None):
        self._check(self.L.fetiF_assemble(self.h, _stream(stream)))

    def precond_values(self, k_vals, first=0):
        """Stiffness values (in each subdomain's K_reg pattern) for the lumped
        preconditioners (the C call fetiF_precond_values)."""
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in k_vals]
        ptrs = (ctypes.c_void_p * len(arrs))(*[_ptr(a) for a in arrs])
        self._check(self.L.fetiF_precond_values(self.h, int(first), len(arrs), ptrs))

    def factor_assemble(self, k_vals, stream=None):
        """Factorisation, copy and assembly of every subdomain, pipelined by
        the context's assembly groups (the C call fetiF_factor_assemble)."""
        if len(k_vals) != self.nsub:
            raise ValueError("factor_assemble needs the K_reg values of every subdomain")
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in k_vals]
        ptrs = (ctypes.c_void_p * len(arrs))(*[_ptr(a) for a in arrs])
        self._check(self.L.fetiF_factor_assemble(self.h, ptrs, _stream(stream)))

    def apply(self, lam, q, stream=None):
        self._vecs(lam=(lam, self.n_lambda), q=(q, self.n_lambda))
        self._check(self.L.fetiF_apply(self.h, _dptr(lam), _dptr(q), _stream(stream)))

    def apply_static(self, lam, q, stream=None):
        """fetiF_apply with the band partials in the library's static
        device array (allocation-free; see include/fetiF.h)."""
        self._vecs(lam=(lam, self.n_lambda), q=(q, self.n_lambda))
        self._check(self.L.fetiF_apply_static(self.h, _dptr(lam), _dptr(q), _stream(stream)))

    def apply_host(self, lam, q=None, cpu_scatter_gather=0, stream=None):
        """q = F lam with host (numpy) vectors; scatter/gather on the GPU (0)
        or on host threads (1).  Returns q."""
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        if lam.shape != (self.n_lambda,):
            raise ValueError(f"lam: expected {self.n_lambda} values, got shape {lam.shape}")
        if q is None:
            q = np.empty(self.n_lambda)
        if q.dtype != np.float64 or q.shape != (self.n_lambda,) or not q.flags.c_contiguous:
            raise ValueError("q: a contiguous float64 array of n_lambda values")
        self._check(self.L.fetiF_apply_host(self.h, _ptr(lam), _ptr(q), int(cpu_scatter_gather), _stream(stream)))
        return q

    def apply_backward(self, g, lam, dlam, dtheta=None, stream=None):
        self._vecs(g=(g, self.n_lambda), lam=(lam, self.n_lambda), dlam=(dlam, self.n_lambda),
                   dtheta=(dtheta, self.n_elems))
        self._check(self.L.fetiF_apply_backward(self.h, _dptr(g), _dptr(lam), _dptr(dlam), _dptr(dtheta),
                                                _stream(stream)))

    def apply_implicit(self, lam, q, stream=None):
        self._vecs(lam=(lam, self.n_lambda), q=(q, self.n_lambda))
        self._check(self.L.fetiF_apply_implicit(self.h, _dptr(lam), _dptr(q), _stream(stream)))

    def dual_rhs(self, f, d, c=None, stream=None):
        self._vecs(f=(f, self.n_dofs), d=(d, self.n_lambda), c=(c, self.n_lambda))
        self._check(self.L.fetiF_dual_rhs(self.h, _dptr(f), _dptr(c), _dptr(d), _stream(stream)))

    def coarse_rhs(self, f, e, stream=None):
        self._vecs(f=(f, self.n_dofs), e=(e, self.n_coarse))
        self._check(self.L.fetiF_coarse_rhs(self.h, _dptr(f), _dptr(e), _stream(stream)))

    def pcpg(self, d, e, lam, tol=1e-9, max_iters=1000, fixed_iters=0, implicit=False, check_every=10,
             refine=False, inner_tol=1e-4, use_graph=True, precond=0, stream=None):
        """PCPG (Alg. 1) on the device (precond 0: M = I, 1: lumped, 2: lumped with the
        scaled jump operator);
        returns dict(iters, outer, rel_residual, w0)."""
        self._vecs(d=(d, self.n_lambda), e=(e, self.n_coarse), lam=(lam, self.n_lambda))
        o = _PcpgOpt(tol, max_iters, fixed_iters, int(implicit), check_every, int(refine), inner_tol,
                     int(use_graph), int(precond))
        r = _PcpgRes()
        self._check(self.L.fetiF_pcpg(self.h, _dptr(d), _dptr(e), _dptr(lam), ctypes.byref(o), ctypes.byref(r),
                                      _stream(stream)))
        return {k: getattr(r, k) for k, _ in _PcpgRes._fields_}

    def primal(self, f, d, lam, alpha, u, stream=None):
        self._vecs(f=(f, self.n_dofs), d=(d, self.n_lambda), lam=(lam, self.n_lambda),
                   alpha=(alpha, self.n_coarse), u=(u, self.n_dofs))
        self._check(self.L.fetiF_primal(self.h, _dptr(f), _dptr(d), _dptr(lam), _dptr(alpha), _dptr(u),
                                        _stream(stream)))

    def download_F(self, i):
        out = np.empty((self.m[i], self.m[i]))
        self._check(self.L.fetiF_download_F(self.h, int(i), _ptr(out)))
        return out

    def info(self):
        inf = _Info()
        self._check(self.L.fetiF_query(self.h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in _Info._fields_}

    def set_apply(self, band_elems=0, rows=0, nontemporal=-1, split=-1, seg=-1):
        """Re-plan the apply (band size in stored elements, rows per pass,
        load policy, work split: 0 bands per triangle, 1 equal shares,
        kernel: 0 whole rows, 4/8 column segments of that many chunks)."""
        self._check(self.L.fetiF_set_apply(self.h, int(band_elems), int(rows), int(nontemporal), int(split),
                                           int(seg)))

    def set_assembly_path(self, path):
        """0: SYRK path (default); 1: TRSM path (backward solve + SpMM)."""
        self._check(self.L.fetiF_set_assembly_path(self.h, int(path)))

    def set_assembly(self, trsm_panel=0, trsm_chunk=0):
        """Re-plan the assembly TRSM (supernode columns per panel, RHS columns per work-group)."""
        self._check(self.L.fetiF_set_assembly(self.h, int(trsm_panel), int(trsm_chunk)))

    def profile(self, on=True):
        """Record HIP events around every device phase (see PHASES)."""
        self._check(self.L.fetiF_profile_enable(self.h, 1 if on else 0))

    def profile_read(self, reset=True):
        """{phase: (total ms, launches)} of the recorded phases (waits for them)."""
        ms = np.zeros(len(PHASES))
        cnt = np.zeros(len(PHASES), np.int64)
        self._check(self.L.fetiF_profile_read(self.h, 1 if reset else 0, _ptr(ms), _ptr(cnt), len(PHASES)))
        return {p: (float(ms[i]), int(cnt[i])) for i, p in enumerate(PHASES)}

    def close(self):
        if getattr(self, "h", None):
            self.L.fetiF_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HostFactor:
    """Host-only ordering + symbolic + numeric factorisation of one K_reg."""

    def __init__(self, sub, k_vals=None, **opts):
        L = load_library()
        self.L = L
        self._s = _SubArrays(sub)
        rec = self._s.record()
        opt = _options(**opts)
        vals = None if k_vals is None else np.ascontiguousarray(k_vals, dtype=np.float64)
        h = ctypes.c_void_p()
        st = L.fetiF_host_factor(ctypes.byref(rec), _ptr(vals), ctypes.byref(opt), ctypes.byref(h))
        if st != 0:
            raise FetiError(st, "host factorisation failed")
        self.h = h
        n, nnz, ns, nl = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        L.fetiF_hfactor_info(h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(ns), ctypes.byref(nl))
        self.n, self.nnz, self.nsuper, self.nlevels = n.value, nnz.value, ns.value, nl.value

    def export(self):
        perm = np.empty(self.n, np.int32)
        cp = np.empty(self.n + 1, np.int64)
        ri = np.empty(self.nnz, np.int32)
        vv = np.empty(self.nnz)
        self.L.fetiF_hfactor_export(self.h, _ptr(perm), _ptr(cp), _ptr(ri), _ptr(vv))
        return perm, cp, ri, vv

    def supernodes(self):
        a = [np.empty(self.nsuper, np.int32) for _ in range(5)]
        self.L.fetiF_hfactor_supernodes(self.h, *[_ptr(x) for x in a])
        return dict(zip(["first", "ncols", "nrows", "parent", "level"], a))

    def __del__(self):
        if getattr(self, "h", None):
            self.L.fetiF_hfactor_free(self.h)
            self.h = None
