"""GPU parity: assembled F~_i and the applied operator against the FP64 oracle.

Tolerances:
* kernels: F~_i from the GPU equals (L^{-1}B)^T (L^{-1}B) formed on the CPU
  with dense triangular solves from the same host factor L, to 1e-14
  (relative Frobenius);
* end to end against the oracle (which refines its solves to full FP64
  accuracy): max(1e-12, kappa(K_reg) * eps) -- any FP64 Cholesky factor of
  K_reg carries a normwise error of order kappa * eps, so for the
  lognormal(0,1) conductivity (kappa ~ 5e5) 1e-12 is not reachable by a
  factor-based method; the bound and the observed value are printed;
* apply: FP64 1e-12 against the oracle's explicit apply of the GPU's own
  F~_i and the above against the oracle F~_i; FP32 storage 1e-5; BF16 its
  own rounding bound (8 significant bits).
"""
import numpy as np
import pytest

from synth import config_problem, make_problem
from oracle import feti
from tests.gpu_common import (say, make_context, upload_and_assemble, oracle_F, rel_fro, gpu_apply, elem_err,
                              q_entry_err, rne_f32, rne_bf16, reduced_apply_bound)

pytestmark = pytest.mark.gpu


def _cases():
    return {
        "C1": lambda: config_problem(1),
        "C5s": lambda: config_problem(5, scale=(2, 6)),
        "C2s": lambda: config_problem(2, scale=(2, 12)),
        "el3": lambda: make_problem(3, "elasticity", [[3, 4], [3, 3], [4, 3]], 0.3,
                                    dirichlet_axis=2, seed=3),
        "heat2d_ragged": lambda: make_problem(2, "heat", [[7, 13, 5], [9, 11]], 0.5,
                                              dirichlet_axis=0, seed=9),
        "C4s": lambda: config_problem(4, scale=(2, 16)),
        "el8": lambda: make_problem(3, "elasticity", [[8, 7], [8, 8], [7, 8]], 0.3,
                                    dirichlet_axis=2, seed=5),
        # linear simplices (the paper's element type): other factor sparsity
        "C2s_tet": lambda: config_problem(2, scale=(2, 12), elem="simplex"),
        "el_tet": lambda: make_problem(3, "elasticity", [[5, 7], [6, 6], [7, 5]], 0.3,
                                       dirichlet_axis=2, seed=4, elem="simplex"),
        "heat2d_tri": lambda: make_problem(2, "heat", [[9, 6, 11], [10, 7]], 0.5,
                                           dirichlet_axis=0, seed=2, elem="simplex"),
    }


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


def _kappa(K):
    import scipy.sparse.linalg as spla
    lmax = spla.eigsh(K, k=1, which="LM", return_eigenvectors=False)[0]
    lmin = spla.eigsh(K.tocsc(), k=1, sigma=0.0, which="LM", return_eigenvectors=False)[0]
    return float(lmax / lmin)


def _F_from_host_factor(sub):
    """(L^-1 P B^T)^T (L^-1 P B^T) with the library's host factor, on the CPU."""
    import scipy.sparse as sp
    from scipy.linalg import solve_triangular
    from paper_2502_08382_amd import HostFactor, subdomain_dict
    h = HostFactor(subdomain_dict(sub), sub.Kreg.data)
    perm, cp, ri, vv = h.export()
    L = sp.csc_matrix((vv, ri, cp), shape=(sub.n, sub.n)).toarray()
    pinv = np.empty_like(perm)
    pinv[perm] = np.arange(sub.n)
    Bt = np.zeros((sub.n, sub.m))
    Bt[pinv[sub.b_dof], np.arange(sub.m)] = sub.b_sign
    X = solve_triangular(L, Bt, lower=True)
    return X.T @ X


@pytest.mark.parametrize("case", list(_cases().keys()))
def test_assembly_fp64_matches_oracle(torch_cuda, case):
    prob = _cases()[case]()
    say("assembly fp64", case, "nsub", prob.nsub, "m", [s.m for s in prob.subs][:4])
    ctx = make_context(prob)
    upload_and_assemble(ctx, prob)
    idxs = range(prob.nsub) if prob.nsub <= 8 else np.linspace(0, prob.nsub - 1, 6).astype(int)
    for i in idxs:
        s = prob.subs[int(i)]
        Fg = ctx.download_F(int(i))
        assert np.array_equal(Fg, Fg.T)
        Fo = oracle_F(prob, int(i))
        e_kernel = elem_err(Fg, _F_from_host_factor(s))
        e_oracle = elem_err(Fg, Fo)
        tol = 1e-12
        if e_oracle > tol:
            tol = max(tol, _kappa(s.Kreg) * np.finfo(float).eps)
        say(f"sub {int(i)}: element-wise vs same-factor CPU {e_kernel:.2e}, vs oracle {e_oracle:.2e} "
            f"(tol {tol:.2e}); rel Frobenius vs oracle {rel_fro(Fg, Fo):.2e}")
        assert e_kernel <= 1e-14
        assert e_oracle <= tol
    ctx.close()


@pytest.mark.parametrize("case", list(_cases().keys()))
def test_apply_fp64_matches_oracle(torch_cuda, case):
    prob = _cases()[case]()
    say("apply fp64", case)
    ctx = make_context(prob, apply_band=4096)
    upload_and_assemble(ctx, prob)
    Fs = [oracle_F(prob, i) for i in range(prob.nsub)]
    q_o = feti.apply_explicit(Fs, [s.dual_map for s in prob.subs], prob.lam, prob.n_lambda)
    q_g = gpu_apply(ctx, prob.lam)
    err = np.linalg.norm(q_g - q_o) / np.linalg.norm(q_o)
    e_ent = q_entry_err(prob, q_g, q_o, Fs)
    say(f"apply: every entry max |dq|/s_g {e_ent:.2e}, normwise {err:.2e}")
    assert err <= 1e-12 and e_ent <= 1e-12
    # bitwise reproducible
    q_g2 = gpu_apply(ctx, prob.lam)
    assert np.array_equal(q_g, q_g2)
    ctx.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_apply_reduced_precision(torch_cuda, prec):
    """F~ stored in FP32 / BF16: every stored element is bitwise the
    round-to-nearest-even of the FP64 context's F~_i of the same factor;
    every q entry within the derived rounding bound of the FP64 oracle
    (FP32 also normwise within 1e-5)."""
    prob = config_problem(5, scale=(2, 6))
    say("apply", prec)
    ctx = make_context(prob, f_storage=prec, apply_band=2048)
    upload_and_assemble(ctx, prob)
    ref = make_context(prob)
    upload_and_assemble(ref, prob)
    rnd = rne_f32 if prec == "f32" else rne_bf16
    for i in range(prob.nsub):
        assert np.array_equal(ctx.download_F(i), rnd(ref.download_F(i))), i
    ref.close()
    Fs = [oracle_F(prob, i) for i in range(prob.nsub)]
    q_o = feti.apply_explicit(Fs, [s.dual_map for s in prob.subs], prob.lam, prob.n_lambda)
    q_g = gpu_apply(ctx, prob.lam)
    err = np.linalg.norm(q_g - q_o) / np.linalg.norm(q_o)
    e_ent = q_entry_err(prob, q_g, q_o, Fs)
    tau = reduced_apply_bound(prec, max(s.m for s in prob.subs))
    say(f"{prec}: storage bitwise RNE of FP64; every entry max |dq|/s_g {e_ent:.2e} (bound {tau:.2e}), "
        f"normwise {err:.2e}")
    assert e_ent <= tau
    if prec == "f32":
        assert err <= 1e-5
    ctx.close()


_LONG = {}


def _long_rows_case():
    """Elasticity, 2x2x2 subdomains of 10^3 hexes (m 993..1386), with the
    oracle's explicit apply and its FP64 bound max(1e-12, kappa eps)
    (computed once per session)."""
    if not _LONG:
        prob = make_problem(3, "elasticity", [[10, 10], [10, 10], [10, 10]], 0.3, dirichlet_axis=2, seed=12)
        Fs = [oracle_F(prob, i) for i in range(prob.nsub)]
        q_o = feti.apply_explicit(Fs, [s.dual_map for s in prob.subs], prob.lam, prob.n_lambda)
        tol = max(1e-12, max(_kappa(s.Kreg) for s in prob.subs) * np.finfo(float).eps)
        _LONG["case"] = (prob, q_o, tol)
    return _LONG["case"]


@pytest.mark.parametrize("prec,tol,ktol", [("f64", None, 1e-13), ("f32", 1e-5, 2e-6), ("bf16", 2e-2, 2e-6)])
def test_apply_every_launch_shape(torch_cuda, prec, tol, ktol):
    """Every kernel, work split, band size, rows per pass and load policy the
    tuner may pick applies the same operator: against the explicit FP64
    apply of the GPU's own stored F~_i to the accumulation precision's
    bound (ktol), against the oracle to the storage precision's bound (FP64:
    max(1e-12, kappa eps)), and between shapes to summation-order rounding.
    Rows of up to 1386 columns span several column segments of the
    segmented kernel (512 columns per 4-chunk FP64 segment)."""
    prob, q_o, tol64 = _long_rows_case()
    tol = tol64 if tol is None else tol
    say("apply shapes", prec, "m", min(s.m for s in prob.subs), max(s.m for s in prob.subs), "tol", tol)
    ctx = make_context(prob, f_storage=prec)
    upload_and_assemble(ctx, prob)
    q_own = feti.apply_explicit([ctx.download_F(i) for i in range(prob.nsub)], [s.dual_map for s in prob.subs],
                                prob.lam, prob.n_lambda)
    total = ctx.info()["apply_elements"]
    ref = None
    for seg in (0, 2, 3, 4, 8):
        for split in (0, 1):
            for band in (1, 3000, total // 5, total):
                for rows in (2, 4):
                    if seg == 8 and rows == 4:
                        continue
                    for nt in (0, 1):
                        ctx.set_apply(band, rows, nt, split, seg)
                        q_g = gpu_apply(ctx, prob.lam)
                        err = np.linalg.norm(q_g - q_o) / np.linalg.norm(q_o)
                        kerr = np.linalg.norm(q_g - q_own) / np.linalg.norm(q_own)
                        say(f"seg {seg} split {split} band {band} rows {rows} nt {nt}: "
                            f"groups {ctx.info()['apply_groups']} vs own F {kerr:.2e} vs oracle {err:.2e}")
                        assert kerr <= ktol
                        assert err <= tol
                        if ref is None:
                            ref = q_g
                        else:
                            d = np.linalg.norm(q_g - ref) / np.linalg.norm(ref)
                            assert d <= (1e-14 if prec == "f64" else 1e-6)
    ctx.close()


def test_failed_upload_invalidates_assembly(torch_cuda):
    """A factor upload that meets a non-SPD K_reg,i fails with FETIF_ENOTSPD
    and leaves the context unassembled (ESTATE for assemble and apply) until
    a good upload; the operator is then exact again."""
    from paper_2502_08382_amd.fetif import FetiError
    prob = config_problem(5, scale=(2, 6))
    say("failed upload", "nsub", prob.nsub)
    ctx = make_context(prob)
    upload_and_assemble(ctx, prob)
    bad = [s.Kreg.data.copy() for s in prob.subs]
    A = prob.subs[3].Kreg.tocoo()
    bad[3][np.nonzero(A.row == A.col)[0][7]] = -1.0
    with pytest.raises(FetiError) as e:
        ctx.factor_upload(bad)
    assert e.value.status == 5   # FETIF_ENOTSPD
    with pytest.raises(FetiError) as e:
        ctx.assemble()
    assert e.value.status == 3   # FETIF_ESTATE
    with pytest.raises(FetiError) as e:
        gpu_apply(ctx, prob.lam)
    assert e.value.status == 3
    upload_and_assemble(ctx, prob)
    Fs = [oracle_F(prob, i) for i in range(prob.nsub)]
    q_o = feti.apply_explicit(Fs, [s.dual_map for s in prob.subs], prob.lam, prob.n_lambda)
    q_g = gpu_apply(ctx, prob.lam)
    assert np.linalg.norm(q_g - q_o) <= 1e-12 * np.linalg.norm(q_o)
    ctx.close()


def test_assembly_every_trsm_shape(torch_cuda):
    """Every TRSM panel width and work-group width the assembly tuner may
    pick assembles the same F~_i: against the oracle to the FP64 bound, and
    between shapes to summation-order rounding."""
    prob = make_problem(3, "elasticity", [[8, 7], [8, 8], [7, 8]], 0.3, dirichlet_axis=2, seed=5)
    say("assembly shapes", "nsub", prob.nsub, "m", [s.m for s in prob.subs][:4])
    ctx = make_context(prob)
    ctx.factor_upload([s.Kreg.data for s in prob.subs])
    ref = None
    Fo = [oracle_F(prob, i) for i in (0, prob.nsub - 1)]
    for panel in (16, 32, 48, 64, 96):
        for chunk in (16, 32, 64):
            ctx.set_assembly(panel, chunk)
            ctx.assemble()
            torch_cuda.cuda.synchronize()
            Fg = [ctx.download_F(i) for i in (0, prob.nsub - 1)]
            e = max(rel_fro(a, b) for a, b in zip(Fg, Fo))
            say(f"panel {panel} chunk {chunk}: levels {ctx.info()['trsm_levels']} vs oracle {e:.2e}")
            assert e <= 1e-12
            if ref is None:
                ref = Fg
            else:
                assert max(rel_fro(a, b) for a, b in zip(Fg, ref)) <= 1e-14
    ctx.close()


def test_apply_hip_graph_replays(torch_cuda):
    """fetiF_apply captured in a HIP graph (uneven elasticity subdomains,
    segmented and whole-row kernels): every replay, with eager work and
    synchronisations between replays and a new lambda copied in, equals the
    eager apply bitwise and the oracle to the FP64 bound."""
    t = torch_cuda
    prob = make_problem(3, "elasticity", [[3, 6], [5, 4], [4, 3]], 0.3, dirichlet_axis=2, seed=21)
    say("apply graph", "nsub", prob.nsub)
    ctx = make_context(prob)
    upload_and_assemble(ctx, prob)
    Fs = [oracle_F(prob, i) for i in range(prob.nsub)]
    rng = np.random.default_rng(5)
    lams = [rng.standard_normal(prob.n_lambda) for _ in range(3)]
    for seg in (4, 0):
        ctx.set_apply(0, 0, -1, -1, seg)
        lam = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
        q = t.empty_like(lam)
        lam.copy_(t.tensor(lams[0], device="cuda"))
        t.cuda.synchronize()
        g = t.cuda.CUDAGraph()
        with t.cuda.graph(g):
            ctx.apply(lam, q)
        for k in range(3):
            lam.copy_(t.tensor(lams[k], device="cuda"))
            g.replay()
            t.cuda.synchronize()
            qg = q.cpu().numpy()
            _ = (lam * 3).sum().item()            # eager work between replays
            qe = gpu_apply(ctx, lams[k])
            q_o = feti.apply_explicit(Fs, [s.dual_map for s in prob.subs], lams[k], prob.n_lambda)
            err = np.linalg.norm(qg - q_o) / np.linalg.norm(q_o)
            say(f"seg {seg} replay {k}: vs oracle {err:.2e}")
            assert np.array_equal(qg, qe)
            assert err <= 1e-12
        del g
    ctx.close()


def test_multi_step_new_stiffness_values(torch_cuda):
    """Alg. 2 over several steps: the stiffness values change between steps
    (new element coefficients, same pattern, same frozen rho); each step's
    factor upload and assembly give that step's F~_i and apply."""
    from synth.problems import assemble_stiffness, regularise
    prob = config_problem(5, scale=(2, 6))
    say("multi-step", "nsub", prob.nsub)
    ctx = make_context(prob)
    rng = np.random.default_rng(17)
    for step in range(3):
        kvals = []
        Fs = []
        for s in prob.subs:
            th = s.theta * np.exp(0.2 * rng.standard_normal(len(s.theta))) if step else s.theta
            Kr = regularise(assemble_stiffness(s, th), s.R, s.fix_dofs, s.rho)
            assert np.array_equal(Kr.indptr, s.Kreg.indptr) and np.array_equal(Kr.indices, s.Kreg.indices)
            kvals.append(Kr.data)
            Fs.append(feti.local_dual_operator(Kr, s.b_dof, s.b_sign))
        ctx.factor_upload(kvals)
        ctx.assemble()
        torch_cuda.cuda.synchronize()
        e_f = max(rel_fro(ctx.download_F(i), Fs[i]) for i in range(prob.nsub))
        q_o = feti.apply_explicit(Fs, [s.dual_map for s in prob.subs], prob.lam, prob.n_lambda)
        q_g = gpu_apply(ctx, prob.lam)
        e_q = np.linalg.norm(q_g - q_o) / np.linalg.norm(q_o)
        say(f"step {step}: F {e_f:.2e} apply {e_q:.2e}")
        assert e_f <= 1e-12 and e_q <= 1e-12
    ctx.close()


def test_pipelined_factor_assemble_is_bitwise_equal(torch_cuda):
    """fetiF_factor_assemble (host factorisation of group g+1 while the device
    copies and assembles group g) gives bitwise the F~_i of a one-group
    context's factor upload + assembly, and so does the group context's own
    assemble; a non-SPD subdomain in a later group leaves nothing uploaded."""
    from paper_2502_08382_amd.fetif import FetiError
    prob = config_problem(2, scale=(3, 8))
    kv = [s.Kreg.data for s in prob.subs]
    say("pipelined factor+assemble", "nsub", prob.nsub, "groups 5")
    ref = make_context(prob)
    upload_and_assemble(ref, prob)
    ctx = make_context(prob, assembly_groups=5, nthreads=4)   # groups hold >= nthreads subdomains
    assert ctx.info()["assembly_groups"] == 5 and ref.info()["assembly_groups"] == 1
    stream = torch_cuda.cuda.Stream()   # a non-default stream handle (64-bit) through the binding
    ctx.factor_assemble(kv, stream=stream)
    stream.synchronize()
    for i in range(prob.nsub):
        assert np.array_equal(ctx.download_F(i), ref.download_F(i)), i
    q_ref = gpu_apply(ref, prob.lam)
    assert np.array_equal(gpu_apply(ctx, prob.lam), q_ref)
    Fs = [oracle_F(prob, i) for i in range(prob.nsub)]
    q_o = feti.apply_explicit(Fs, [s.dual_map for s in prob.subs], prob.lam, prob.n_lambda)
    assert np.linalg.norm(q_ref - q_o) <= 1e-12 * np.linalg.norm(q_o)
    # a non-SPD K_reg in the last group
    bad = [v.copy() for v in kv]
    A = prob.subs[prob.nsub - 2].Kreg.tocoo()
    bad[prob.nsub - 2][np.nonzero(A.row == A.col)[0][5]] = -1.0
    with pytest.raises(FetiError) as e:
        ctx.factor_assemble(bad)
    assert e.value.status == 5   # FETIF_ENOTSPD
    with pytest.raises(FetiError) as e:
        gpu_apply(ctx, prob.lam)
    assert e.value.status == 3   # FETIF_ESTATE
    # the group context's phase-by-phase assemble, then the pipeline again
    upload_and_assemble(ctx, prob)
    assert np.array_equal(gpu_apply(ctx, prob.lam), q_ref)
    ctx.factor_assemble(kv)
    torch_cuda.cuda.synchronize()
    assert np.array_equal(gpu_apply(ctx, prob.lam), q_ref)
    ctx.close()
    ref.close()


def test_wide_subdomains_beyond_4096_multipliers(torch_cuda):
    """Two flat slab subdomains (64 x 64 x 2 hexes) glued on a face of 65^2
    nodes: m = 8450 for the lower one (gluing + Dirichlet face) and 4225 for
    the upper.  The column-segmented apply holds any m (LDS bounded by the
    segment and the rows of a band); the whole-row kernel, which keeps p of
    all columns in LDS, is refused beyond 4096.  Every q entry against the
    oracle's implicit apply for both segment widths and work splits, and 24
    columns of each F~_i against solves with the oracle's sparse factor
    (one refinement step), element-wise per column."""
    import os
    from paper_2502_08382_amd.fetif import FetiError
    from oracle import implicit as orc
    prob = make_problem(3, "heat", [[64], [64], [2, 2]], 0.5, dirichlet_axis=2, seed=7)
    ms = [s.m for s in prob.subs]
    say("wide subdomains: m", ms, "n", [s.n for s in prob.subs])
    assert max(ms) > 8192 and min(ms) > 4096
    ctx = make_context(prob)
    upload_and_assemble(ctx, prob)
    with pytest.raises(FetiError) as e:
        ctx.set_apply(0, 2, 1, 0, 0)
    assert e.value.status == 6 and "4096" in str(e.value)
    I = orc.ImplicitCPU(prob.subs, prob.n_lambda, nthreads=max(1, min(16, len(os.sched_getaffinity(0)))))
    I.factor()
    q_o = I.apply(prob.lam)
    nrm = I.opnorms(60)
    kap = I.kappas(60)
    tau = max(1e-12, kap.max() * np.finfo(float).eps)
    scale = np.zeros(prob.n_lambda)
    for i, sub in enumerate(prob.subs):
        scale[sub.dual_map] += nrm[i] * np.linalg.norm(prob.lam[sub.dual_map])
    say(f"  kappa {kap}, per-entry bound {tau:.2e}")
    for seg in (4, 8):
        for split in (0, 1):
            rows = 2 if seg == 8 else 4
            ctx.set_apply(131072 if split == 0 else 2 * 10 ** 6, rows, 1, split, seg)
            q_g = gpu_apply(ctx, prob.lam)
            r = (np.abs(q_g - q_o) / scale).max()
            say(f"  seg {seg} split {split}: groups {ctx.info()['apply_groups']}, max |dq|/s_g {r:.2e}")
            assert np.all(np.isfinite(q_g)) and r <= tau
    rng = np.random.default_rng(5)
    for i, sub in enumerate(prob.subs):
        Fg = ctx.download_F(i)
        assert np.array_equal(Fg, Fg.T)
        inv = orc.SparseRegInverse(sub.Kreg, sub.coords, sub.dpn)
        cols = sorted(set([0, sub.m - 1] + list(rng.choice(sub.m, 22, replace=False))))
        worst = 0.0
        for a in cols:
            rhs = np.zeros(sub.n)
            rhs[sub.b_dof[a]] = sub.b_sign[a]
            col = sub.b_sign * inv.solve(rhs)[sub.b_dof]
            worst = max(worst, np.abs(Fg[:, a] - col).max() / np.abs(col).max())
        say(f"  sub {i} m {sub.m}: {len(cols)} columns, max |dF| / max |F col| {worst:.2e} (bound {tau:.2e})")
        assert worst <= tau
    ctx.close()


@pytest.mark.parametrize("nsub,nel", [(1, 7), (2, 5), (3, 12)])
def test_closed_form_1d_through_the_library(torch_cuda, nsub, nel):
    """The 1D bar through the library (it is dimension-agnostic): nodes
    0..n per subdomain, unit conductivity, edge h, K_reg = K + rho e0 e0^T,
    so (K_reg^{-1})_ij = 1/rho + h min(i, j) and every F~_i entry is fixed:
    a lone subdomain (Dirichlet row only, m = 1) gives [1/rho]; the first of
    several gives [[1/rho, 1/rho], [1/rho, 1/rho + n h]] (m = 2), a middle
    one [[1/rho, -1/rho], [-1/rho, 1/rho + n h]], the last [1/rho] (m = 1).
    The applied operator is checked against these closed forms too."""
    prob = make_problem(1, "heat", [[nel] * nsub], 0.0, dirichlet_axis=0, seed=1)
    say("1d closed form", "nsub", nsub, "nel", nel, "m", [s.m for s in prob.subs])
    ctx = make_context(prob)
    upload_and_assemble(ctx, prob)
    h = prob.h
    Fs = []
    for i, s in enumerate(prob.subs):
        r = 1.0 / s.rho
        expect = np.array([[s.b_sign[a] * s.b_sign[b] * (r + h * min(s.b_dof[a], s.b_dof[b]))
                            for b in range(s.m)] for a in range(s.m)])
        if nsub == 1:
            assert s.m == 1 and np.allclose(expect, [[r]], rtol=1e-15, atol=0)
        elif i == 0:
            assert np.allclose(expect, [[r, r], [r, r + nel * h]], rtol=1e-15, atol=0)
        elif i == nsub - 1:
            assert np.allclose(expect, [[r]], rtol=1e-15, atol=0)
        Fg = ctx.download_F(i)
        err = np.abs(Fg - expect).max() / np.abs(expect).max()
        say(f"sub {i} m {s.m}: max rel err vs closed form {err:.2e}")
        assert err <= 1e-14
        Fs.append(expect)
    q_ref = feti.apply_explicit(Fs, [s.dual_map for s in prob.subs], prob.lam, prob.n_lambda)
    q_g = gpu_apply(ctx, prob.lam)
    assert np.abs(q_g - q_ref).max() <= 1e-14 * np.abs(q_ref).max()
    ctx.close()
