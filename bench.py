#!/usr/bin/env python3
"""Benchmark of the explicit FETI dual operator on one MI355X.

Workload (default, the largest of the five): 3D linear elasticity
(E = 1, nu = 0.3), trilinear hexes, 729 subdomains whose per-axis slab
widths are drawn from U{6..14} elements (1029..10125 DOFs, 600..3438 local
multipliers), rigid-body modes removed by fixing three non-collinear corner
nodes, Dirichlet on z=0; seeded synthetic data.  `--config 2` selects the
512-subdomain 3D heat workload (12^3 hexes, lognormal(0, 0.5)
conductivity), `--config 4` the 216-subdomain one (16^3 hexes).  One step
follows the paper's multi-step skeleton (Alg. 2): numeric factorisation of
every K_reg,i on host threads + copy of the factor values, assembly of
every F~_i on the GPU (RHS init, supernodal TRSM, SYRK), the dual
right-hand sides d = B K^+ f - c and e = R^T f, then 200 iterations of the
projected conjugate gradient solver (Alg. 1), each applying
F = sum_i D_i^T F~_i D_i.  With --prec f32/bf16 the solver instead runs to
tol 1e-9 with FP64 iterative refinement (true residual through the
factors).

Printed: one JSON line with the apply bandwidth as `value`, the assembly
time per 1000 subdomains, the break-even iteration count against the CPU
oracle's implicit apply, the roofline of the dominant kernel and the CPU
oracle baseline (implicit apply on all host threads and on one, explicit
assembly and dense apply, the CPU model).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, vendor figure
COPY_CAL_BYTES = 1 << 30     # size of the counter-calibration copy
FP64_PEAK_TFS = 78.6         # MI355X dense FP64 (vector and matrix)
METRIC = "F assembly ms/1k subdomains; F·λ apply GB/s; break-even iters vs implicit"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def calibration_copies(torch, dev):
    """Three copies of a 1 GiB buffer: the reference the HBM byte counters
    of a profiling run are scaled by."""
    a = torch.empty(COPY_CAL_BYTES // 8, dtype=torch.float64, device=dev)
    a.fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("calibration copies done")


def even_sample(nsub, k):
    """k subdomain indices spread evenly over 0..nsub-1."""
    k = max(1, min(int(k), nsub))
    return sorted({int(round(x)) for x in np.linspace(0, nsub - 1, k)})


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def timed(fn, min_s, min_reps):
    """Mean seconds per call of fn over at least min_reps calls and min_s
    seconds (after one untimed call), and the call count."""
    fn()
    reps = 0
    t0 = time.perf_counter()
    while True:
        fn()
        reps += 1
        if time.perf_counter() - t0 >= min_s and reps >= min_reps:
            break
    return (time.perf_counter() - t0) / reps, reps


def cpu_oracle_leg(prob, sample_n):
    """The oracle as it stands, on the host cores: its implicit apply
    (sparse Cholesky forward + backward solves) on all threads and on one,
    and its explicit assembly (one unit solve per local multiplier) and
    dense apply on all threads, each on an evenly spaced sample of the
    subdomains scaled to the whole workload by the subdomain count."""
    from oracle import implicit as orc
    nthreads = len(os.sched_getaffinity(0))
    out = {"threads": nthreads, "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    N = prob.nsub
    # implicit apply, all threads
    idx = even_sample(N, sample_n)
    t0 = time.time()
    I = orc.ImplicitCPU([prob.subs[i] for i in idx], prob.n_lambda, nthreads=nthreads)
    I.factor()
    log(f"cpu oracle: ordering + factorisation of {len(idx)} subdomains {time.time() - t0:.1f}s")
    t, reps = timed(lambda: I.apply(prob.lam), 10.0, 3)
    out["implicit_ms"] = t * N / len(idx) * 1e3
    out["implicit_sample"] = (f"implicit apply (sparse Cholesky fwd+bwd solves, nested-dissection order) of "
                              f"{len(idx)} of {N} subdomains (evenly spaced) on {nthreads} threads, {reps} "
                              f"repetitions, scaled x{N / len(idx):.4g}")
    # implicit apply, one thread
    idx1 = even_sample(N, 16)
    I1 = orc.ImplicitCPU([prob.subs[i] for i in idx1], prob.n_lambda, nthreads=1)
    I1.factor()
    t, reps = timed(lambda: I1.apply(prob.lam), 3.0, 2)
    out["implicit_t1_ms"] = t * N / len(idx1) * 1e3
    out["implicit_t1_sample"] = (f"{len(idx1)} of {N} subdomains (evenly spaced), 1 thread, {reps} repetitions, "
                                 f"scaled x{N / len(idx1):.4g}")
    log(f"cpu oracle implicit apply: {out['implicit_ms']:.1f} ms on {nthreads} threads, "
        f"{out['implicit_t1_ms']:.1f} ms on 1 thread (whole workload)")
    del I1
    # explicit assembly and dense apply, all threads, one subdomain per thread
    idxe = even_sample(N, nthreads)
    Ie = orc.ImplicitCPU([prob.subs[i] for i in idxe], prob.n_lambda, nthreads=nthreads)
    Ie.factor()
    t0 = time.perf_counter()
    Ie.assemble()
    out["assembly_ms"] = (time.perf_counter() - t0) * N / len(idxe) * 1e3
    t, reps = timed(lambda: Ie.apply_explicit(prob.lam), 3.0, 3)
    out["explicit_apply_ms"] = t * N / len(idxe) * 1e3
    out["explicit_sample"] = (f"{len(idxe)} of {N} subdomains (evenly spaced) on {nthreads} threads, assembly "
                              f"once, dense apply {reps} repetitions, both scaled x{N / len(idxe):.4g}")
    log(f"cpu oracle explicit: assembly {out['assembly_ms']:.0f} ms, dense apply {out['explicit_apply_ms']:.1f} ms "
        f"(whole workload)")
    del Ie
    return out


def decision_table():
    """The paper's assembly parameters (Sec. IV-D, Table 1) measured here,
    per workload: assembly time of the SYRK and TRSM paths with the
    nested-dissection order and with the Schur-complement order (multiplier
    nodes last), each from HIP-event phase timers over 3 assemblies after one
    warm-up (the assembly tuner's TRSM shape of each context), and the
    host-vector apply with the scatter/gather on the GPU or on host threads
    (wall clock, 20 applies after 3 warm-ups, the stored apply shape)."""
    import torch
    from synth import config_problem, make_problem
    from paper_2502_08382_amd import FetiContext, subdomain_dict
    from paper_2502_08382_amd.fetif import FetiError
    from paper_2502_08382_amd.autotune import tune_assembly, install_stored_apply_shape
    workloads = [("3D heat, 64 subdomains of 10^3 hexes", lambda: config_problem(5)),
                 ("3D heat, 512 subdomains of 12^3 hexes", lambda: config_problem(2)),
                 ("3D heat, 216 subdomains of 16^3 hexes", lambda: config_problem(4)),
                 ("2D heat, 256 subdomains of 64^2 quads",
                  lambda: make_problem(2, "heat", [[64] * 16] * 2, 0.5, dirichlet_axis=0, seed=7))]
    stream = torch.cuda.Stream()
    for name, make in workloads:
        prob = make()
        kvals = [s.Kreg.data for s in prob.subs]
        subs = [subdomain_dict(s) for s in prob.subs]
        out = {"decision_table": name, "subdomains": prob.nsub, "dofs_per_subdomain": int(prob.subs[0].n),
               "m_max": int(max(s.m for s in prob.subs)), "assembly": {}, "apply_host_ms": {}}
        for order in (0, 1):
            t0 = time.time()
            ctx = FetiContext(subs, prob.n_lambda, device=0, schur_order=order)
            info = ctx.info()
            with torch.cuda.stream(stream):
                th = time.time()
                ctx.factor_upload(kvals, stream=stream)
                host_s = time.time() - th
                tune = tune_assembly(ctx, stream=stream)
            for path in (0, 1):
                key = ("schur_order" if order else "nested_dissection") + ("/trsm_path" if path else "/syrk_path")
                try:
                    ctx.set_assembly_path(path)
                except FetiError as e:
                    out["assembly"][key] = {"skipped": str(e)}
                    continue
                with torch.cuda.stream(stream):
                    ctx.assemble(stream=stream)
                    torch.cuda.synchronize()
                    ctx.profile(True)
                    ctx.profile_read(reset=True)
                    for _ in range(3):
                        ctx.assemble(stream=stream)
                    torch.cuda.synchronize()
                    ctx.profile(False)
                    prof = ctx.profile_read(reset=True)
                ph = {k: round(prof[k][0] / 3, 4) for k in ("rhs_init", "trsm", "syrk", "trsm_bwd", "spmm")
                      if prof[k][1]}
                ms = sum(ph.values())
                inf = ctx.info()
                flops = inf["trsm_flops"] + (inf["trsm_bwd_flops"] if path else inf["syrk_flops"])
                out["assembly"][key] = {"ms": round(ms, 3), "ms_per_1k_subdomains": round(1000 * ms / prob.nsub, 3),
                                        "phases_ms": ph, "algorithmic_flops": flops,
                                        "tflops": round(flops / (ms * 1e-3) / 1e12, 2),
                                        "trsm_shape": [tune["panel"], tune["chunk"]],
                                        "factor_values": info["factor_values"],
                                        "host_factor_s": round(host_s, 3)}
                log(f"{name}: {key}: {ms:.3f} ms ({ph})")
            ctx.set_assembly_path(0)
            if order == 0:
                with torch.cuda.stream(stream):
                    ctx.assemble(stream=stream)
                torch.cuda.synchronize()
                install_stored_apply_shape(ctx)
                for sg in (0, 1):
                    for _ in range(3):
                        ctx.apply_host(prob.lam, cpu_scatter_gather=sg, stream=stream)
                    tc = time.perf_counter()
                    for _ in range(20):
                        ctx.apply_host(prob.lam, cpu_scatter_gather=sg, stream=stream)
                    t = (time.perf_counter() - tc) / 20 * 1e3
                    out["apply_host_ms"]["cpu" if sg else "gpu"] = round(t, 4)
                    log(f"{name}: host-vector apply, scatter/gather on the {'CPU' if sg else 'GPU'}: {t:.3f} ms")
            ctx.close()
            log(f"{name}: order {order} done in {time.time() - t0:.1f}s")
        print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3, help="workload 1..5 (default 3, the largest)")
    ap.add_argument("--elem", default="box", choices=["box", "simplex"],
                    help="the workload's box elements, or the same grid cut into linear simplices")
    ap.add_argument("--iters", type=int, default=200,
                    help="solver iterations per step (FP64); 0: run to --tol")
    ap.add_argument("--tol", type=float, default=1e-9, help="solver tolerance with --prec f32/bf16")
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16"])
    ap.add_argument("--precond", default="none", choices=["none", "lumped", "scaled"],
                    help="M of the PCPG (Alg. 1): identity, the lumped preconditioner, or the lumped one on the "
                         "scaled jump operator (stiffness scaling, unregularised K)")
    ap.add_argument("--cpu-sample", type=int, default=128,
                    help="subdomains (evenly spaced) of the CPU oracle's implicit apply on all host threads")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--apply-band", type=int, default=0)
    ap.add_argument("--no-tune", action="store_true", help="skip the apply autotuner")
    ap.add_argument("--retune", action="store_true",
                    help="tune the apply shape even if the stored tuning has this workload")
    ap.add_argument("--groups", type=int, default=8,
                    help="assembly groups of the pipelined factorisation + copy + assembly measured after the "
                         "timed steps (0: skip that measurement)")
    ap.add_argument("--backward", action="store_true",
                    help="also time fetiF_apply_backward (dlambda and the element adjoint dtheta)")
    ap.add_argument("--pmc-assemble", type=int, default=0, metavar="N",
                    help="profiling mode: upload the factors, install the TRSM shape 96/32 (the tuned one on "
                         "the 3D heat workloads), run N assemblies and exit")
    ap.add_argument("--decision-table", action="store_true",
                    help="measure the paper's assembly parameters instead (Sec. IV-D): SYRK vs TRSM path, "
                         "nested-dissection vs Schur-complement order, scatter/gather on the GPU vs on host "
                         "threads, on the 64- and 512-subdomain heat workloads, the 216-subdomain one and a 2D "
                         "heat problem (256 subdomains of 64^2 quads); one JSON line per workload")
    ap.add_argument("--pmc-apply", type=int, default=0, metavar="N",
                    help="profiling mode: assemble, run N applies in the tuned shape, then copy a 1 GiB "
                         "buffer three times (the counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the subdomains would shard "
              "over GPUs with one process each, and that path is not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from synth import config_problem, workload_name
    from paper_2502_08382_amd import FetiContext, subdomain_dict

    assert torch.cuda.is_available(), "needs a GPU"
    if args.decision_table:
        decision_table()
        return
    dev = torch.device("cuda:0")
    t0 = time.time()
    prob = config_problem(args.config, elem=args.elem)
    wname = workload_name(args.config, args.elem)
    log(f"problem C{args.config}: {prob.nsub} subdomains, n_lambda={prob.n_lambda}, "
        f"gen {time.time() - t0:.1f}s")
    t0 = time.time()
    ctx = FetiContext([subdomain_dict(s, with_elements=args.backward) for s in prob.subs], prob.n_lambda,
                      device=0, f_storage=args.prec, apply_band=args.apply_band)
    info = ctx.info()
    log(f"create (ordering + symbolic + plan + device structures) {time.time() - t0:.1f}s; "
        f"L values {info['factor_values']:.3g}, X values {info['x_values']:.3g}, "
        f"trsm flops {info['trsm_flops']:.3g}, syrk flops {info['syrk_flops']:.3g}, "
        f"levels {info['trsm_levels']}, apply groups {info['apply_groups']}")
    kvals = [s.Kreg.data for s in prob.subs]
    lam = torch.tensor(prob.lam, dtype=torch.float64, device=dev)
    q = torch.empty_like(lam)
    f = torch.tensor(np.concatenate([s.f for s in prob.subs]), dtype=torch.float64, device=dev)
    e = torch.empty(sum(s.R.shape[1] for s in prob.subs), dtype=torch.float64, device=dev)
    d = torch.empty_like(lam)
    sol = torch.empty_like(lam)
    stream = torch.cuda.Stream()
    refine = args.prec != "f64"
    pc = {"none": 0, "lumped": 1, "scaled": 2}[args.precond]
    if pc:
        from paper_2502_08382_amd import values_in_pattern
        ctx.precond_values([values_in_pattern(s.K, s.Kreg) for s in prob.subs])
    tune_cache = os.path.join(ROOT, "paper_2502_08382_amd", "tuned_apply.json")

    def shape_key(t):
        return (f"{wname}|{args.prec}|seg{t.get('seg', 0)}-split{t['split']}-band{t['band']}"
                f"-rows{t['rows']}-nt{t['nontemporal']}")

    if args.pmc_assemble:
        with torch.cuda.stream(stream):
            ctx.factor_upload(kvals, stream=stream)
            ctx.set_assembly(96, 32)
            for _ in range(args.pmc_assemble):
                ctx.assemble(stream=stream)
            torch.cuda.synchronize()
        log(f"{args.pmc_assemble} assemblies done; trsm flops {info['trsm_flops']:.6g}, "
            f"syrk flops {info['syrk_flops']:.6g}")
        calibration_copies(torch, dev)
        ctx.close()
        return

    if args.pmc_apply:
        from paper_2502_08382_amd.autotune import tune_apply
        with torch.cuda.stream(stream):
            ctx.factor_upload(kvals, stream=stream)
            ctx.assemble(stream=stream)
            tune = tune_apply(ctx, lam, q, stream=stream, cache=tune_cache, reps=5)
            for _ in range(args.pmc_apply):
                ctx.apply(lam, q, stream=stream)
            torch.cuda.synchronize()
        log(f"{args.pmc_apply} applies done; key {shape_key(tune)}")
        calibration_copies(torch, dev)
        ctx.close()
        return

    host_factor_s = []
    solver = []
    pcpg_events = []
    tune = None
    atune = None

    def step():
        th = time.time()
        ctx.factor_upload(kvals, stream=stream)
        host_factor_s.append(time.time() - th)
        ctx.assemble(stream=stream)
        ctx.coarse_rhs(f, e, stream=stream)
        ctx.dual_rhs(f, d, stream=stream)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        if refine:
            r = ctx.pcpg(d, e, sol, tol=args.tol, refine=True, inner_tol=1e-4 if args.prec == "f32" else 1e-2,
                         max_iters=20000, use_graph=False, precond=pc, stream=stream)
        else:
            if args.iters > 0:
                r = ctx.pcpg(d, e, sol, fixed_iters=args.iters, use_graph=False, precond=pc, stream=stream)
            else:
                r = ctx.pcpg(d, e, sol, tol=args.tol, max_iters=20000, use_graph=False, precond=pc, stream=stream)
        ev1.record(stream)
        pcpg_events.append((ev0, ev1))
        solver.append(r)

    with torch.cuda.stream(stream):
        for w in range(args.warmup):
            step()
            torch.cuda.synchronize()
            log(f"warmup step {w} done: solver {solver[-1]}")
            if w == 0 and not args.no_tune:
                from paper_2502_08382_amd.autotune import tune_apply, tune_assembly
                tt = time.time()
                atune = tune_assembly(ctx, stream=stream)
                log(f"assembly autotune {time.time() - tt:.1f}s: TRSM panel={atune['panel']} "
                    f"chunk={atune['chunk']} ({atune['trsm_ms']:.3f} ms)")
                tt = time.time()
                tune = tune_apply(ctx, lam, q, stream=stream, cache=None if args.retune else tune_cache)
                log(f"apply autotune {time.time() - tt:.1f}s{' (stored)' if tune.get('cached') else ''}: "
                    f"seg={tune.get('seg', 0)} split={tune['split']} band={tune['band']} rows={tune['rows']} "
                    f"nontemporal={tune['nontemporal']} ({tune['ms'] * 1e3:.1f} us)")
        host_factor_s.clear()
        solver.clear()
        pcpg_events.clear()
        ctx.profile(True)
        ctx.profile_read(reset=True)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(args.steps):
            step()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        ctx.profile(False)
        prof = ctx.profile_read(reset=True)
    log(f"timed {args.steps} steps in {elapsed:.3f}s; phases {prof}; solver {solver[-1]}")

    # ---- the apply alone, eager and replayed from a captured HIP graph
    # (HIP events on the launching stream; outside the timed steps)
    def event_time(fn, n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            fn()
            e0.record(stream)
            for _ in range(n):
                fn()
            e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / n

    with torch.cuda.stream(stream):
        ctx.apply(lam, q, stream=stream)
    torch.cuda.synchronize()
    q_eager = q.clone()
    t_apply_eager = event_time(lambda: ctx.apply(lam, q, stream=stream), 50)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ctx.apply(lam, q)
    t_apply_graph = event_time(graph.replay, 50)
    torch.cuda.synchronize()
    graph_same = bool(torch.equal(q, q_eager))
    log(f"apply alone: eager {t_apply_eager * 1e3:.1f} us, graph replay {t_apply_graph * 1e3:.1f} us, "
        f"graph result bitwise equal to eager: {graph_same}")
    del graph
    # the same PCPG solve with its iterations captured in HIP graphs and replayed
    t_pcpg_graph = None
    if not refine and args.iters > 0:
        ctx.profile(False)
        t_pcpg_graph = event_time(lambda: ctx.pcpg(d, e, sol, fixed_iters=args.iters, use_graph=True, precond=pc,
                                                   stream=stream), 2)
        log(f"PCPG with graph-replayed iterations: {t_pcpg_graph:.3f} ms for {args.iters} iterations")
    t_backward = None
    if args.backward:
        g_d = torch.tensor(prob.mu, dtype=torch.float64, device=dev)
        dl = torch.empty_like(lam)
        dth = torch.empty(sum(len(s.theta) for s in prob.subs), dtype=torch.float64, device=dev)
        t_backward = event_time(lambda: ctx.apply_backward(g_d, lam, dl, dth, stream=stream), 10)
        log(f"apply_backward (dlambda + dtheta) {t_backward:.3f} ms")

    # a plain streaming read of the same byte count (torch's sum over a
    # resident buffer), the practical read ceiling the band kernel is set
    # against beside the nominal 8 TB/s
    nread = max(1, int(info["f_tri_elements"]) * {"f64": 8, "f32": 4, "bf16": 2}[args.prec] // 8)
    rbuf = torch.ones(nread, dtype=torch.float64, device=dev)
    rsum = torch.empty((), dtype=torch.float64, device=dev)
    t_read = event_time(lambda: torch.sum(rbuf, dim=0, out=rsum), 20)
    read_gbs = nread * 8 / (t_read * 1e-3) / 1e9
    log(f"plain read of {nread * 8 / 1e9:.3f} GB (torch sum): {t_read * 1e3:.1f} us, {read_gbs:.0f} GB/s")
    # the same bytes read by the library's streaming probe, each work-group
    # one contiguous region (the access pattern of the apply's bands)
    from paper_2502_08382_amd.fetif import read_probe
    nprobe = nread - nread % 2
    probe = {}
    for region in (256 << 10, 1 << 20, 4 << 20):
        pout = torch.empty(-(-nprobe * 8 // region), dtype=torch.float64, device=dev)
        t_p = event_time(lambda: read_probe(rbuf[:nprobe], region, pout, stream=stream), 20)
        probe[f"{region >> 10} KiB"] = round(nprobe * 8 / (t_p * 1e-3) / 1e9, 1)
        del pout
    probe_best = max(probe.values())
    del rbuf
    log(f"contiguous-region read probe (GB/s by region size): {probe}")

    K = args.steps
    ms = {p: v[0] for p, v in prof.items()}
    cnt = {p: max(1, v[1]) for p, v in prof.items()}
    t_upload = ms["factor_copy"] / K     # all chunks of one step's copy
    t_asm = (ms["rhs_init"] + ms["trsm"] + ms["syrk"]) / K
    t_band = ms["apply_band"] / cnt["apply_band"]
    t_gather = ms["apply_gather"] / cnt["apply_gather"]
    t_apply = t_band + t_gather
    bytes_el = {"f64": 8, "f32": 4, "bf16": 2}[args.prec]
    sum_m = info["sum_m"]
    tri_bytes = bytes_el * info["f_tri_elements"]
    # algorithmic bytes of one apply: each stored element of every triangle
    # once, plus per local multiplier the lambda value (8), its index (4) and
    # the partial q~ write (8); all of them move in the band kernel
    apply_bytes = tri_bytes + 20 * sum_m
    band_bytes = apply_bytes
    apply_gbs = apply_bytes / (t_apply * 1e-3) / 1e9
    band_gbs = band_bytes / (t_band * 1e-3) / 1e9
    asm_flops = info["trsm_flops"] + info["syrk_flops"]
    # the band kernel the stored or tuned shape selects (phase 4 times it)
    apply_kernel = "apply_seg_kernel" if (tune or {}).get("seg", 0) else "apply_band_kernel"

    result = {
        "metric": METRIC,
        "value": round(apply_gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / K * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32 (F storage; f64 assembly)", "bf16": "bf16 (F storage; f64 assembly)"}[args.prec],
        "data": "synthetic (seeded structured-grid FETI problem)",
        "config": {"workload": wname, "subdomains": prob.nsub,
                   "dofs_per_subdomain": int(prob.subs[0].n), "n_lambda": int(prob.n_lambda),
                   "sum_m": int(sum_m), "applies_per_step": int(solver[-1]["iters"]), "f_storage": args.prec},
        "assembly_ms_per_1k_subdomains": round(1000.0 * t_asm / prob.nsub, 3),
        "assembly_ms": round(t_asm, 3),
        "assembly_phase_ms": {"rhs_init": round(ms["rhs_init"] / K, 4), "trsm": round(ms["trsm"] / K, 4),
                              "syrk": round(ms["syrk"] / K, 4)},
        "assembly_tflops": round(asm_flops / (t_asm * 1e-3) / 1e12, 3),
        "assembly_mfma_frac": round(asm_flops / (t_asm * 1e-3) / 1e12 / FP64_PEAK_TFS, 4),
        "solver": {"kind": "PCPG (Alg. 1), M = " + ("I", "lumped", "lumped on the scaled jump operator")[pc] +
                           (", FP64 refinement" if refine else ""),
                   "iters": solver[-1]["iters"], "outer": solver[-1]["outer"],
                   "rel_residual": solver[-1]["rel_residual"],
                   "ms_per_iter": None},
        "apply_ms": round(t_apply, 4),
        "apply_alone_us": {"eager": round(t_apply_eager * 1e3, 2), "hip_graph": round(t_apply_graph * 1e3, 2),
                           "graph_bitwise_equal": graph_same},
        "backward_ms": None if t_backward is None else round(t_backward, 4),
        "apply_band_ms": round(t_band, 4),
        "apply_gather_ms": round(t_gather, 4),
        "factor_copy_ms": round(t_upload, 3),
        "apply_shape": None if tune is None else {k: tune.get(k, 0) for k in ("seg", "split", "band", "rows",
                                                                                "nontemporal")},
        "trsm_shape": None if atune is None else {k: atune[k] for k in ("panel", "chunk")},
        "host_factor_s": round(float(np.mean(host_factor_s)), 3) if host_factor_s else None,
        "roofline": {"bound": "hbm", "kernel": apply_kernel, "achieved": round(band_gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(band_gbs / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_launch": int(band_bytes)},
        "plain_read_reference": {"kernel": "torch.sum over a resident buffer of the operator's bytes",
                                 "bytes": int(nread * 8), "us": round(t_read * 1e3, 1),
                                 "GB/s": round(read_gbs, 1), "band_kernel_vs_it": round(band_gbs / read_gbs, 4)},
        "contiguous_read_probe": {"kernel": "fetiF_read_probe: each work-group streams one contiguous region of "
                                            "the same bytes (16-byte non-temporal loads)",
                                  "GB/s_by_region": probe, "band_kernel_vs_best": round(band_gbs / probe_best, 4)},
    }

    if tune is not None:
        from paper_2502_08382_amd.traffic import lookup
        rec = lookup(shape_key(tune))
        if rec is not None:
            result["roofline"]["traffic"] = int(rec["traffic_bytes"])
            result["roofline"]["traffic_source"] = (f"rocprofv3 FETCH_SIZE x {rec['fetch_factor']} + WRITE_SIZE x "
                                                    f"{rec['write_factor']} (1 GiB copy calibration)")

    # solver time: HIP events around the PCPG call on its stream
    t_solve_ms = float(np.mean([a.elapsed_time(b) for a, b in pcpg_events]))
    result["solver"]["ms"] = round(t_solve_ms, 3)
    if refine:
        # the reduced-precision solution against an FP64 one: PCPG to 1e-12
        # with the implicit FP64 operator (the factors), outside the timing
        sol64 = torch.empty_like(sol)
        with torch.cuda.stream(stream):
            r64 = ctx.pcpg(d, e, sol64, tol=1e-12, implicit=True, max_iters=20000, use_graph=False,
                           stream=stream)
        torch.cuda.synchronize()
        err = float(torch.linalg.vector_norm(sol - sol64) / torch.linalg.vector_norm(sol64))
        result["solver"]["lambda_rel_err_vs_fp64"] = err
        result["solver"]["fp64_reference"] = f"implicit FP64 PCPG to 1e-12 ({r64['iters']} iterations)"
        log(f"lambda vs the FP64 solution: rel err {err:.2e} ({r64['iters']} FP64 iterations)")
    if t_pcpg_graph is not None:
        result["solver"]["hip_graph_ms_per_iter"] = round(t_pcpg_graph / args.iters, 4)
    result["solver"]["ms_per_iter"] = round(t_solve_ms / max(1, solver[-1]["iters"]), 4)
    result["solves_with_factors_ms"] = round(ms["solves"] / K, 3)

    # ---- preprocessing with the host factorisation of the next assembly
    # group overlapping the copy and assembly of the previous one (a second
    # context with --groups groups): its wall time against the host
    # factorisation alone (factor_upload returns once the host work is done)
    t_overlap = None
    if args.groups > 0:
        ctx2 = FetiContext([subdomain_dict(s) for s in prob.subs], prob.n_lambda, device=0, f_storage=args.prec,
                           assembly_groups=args.groups)
        if atune is not None:
            ctx2.set_assembly(atune["panel"], atune["chunk"])
        if tune is not None:   # the same apply shape, so the two applies sum in the same order
            ctx2.set_apply(tune["band"], tune["rows"], tune["nontemporal"], tune["split"], tune.get("seg", 0))
        t_host, t_pipe = [], []
        with torch.cuda.stream(stream):
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx2.factor_upload(kvals, stream=stream)
                t_host.append(time.perf_counter() - t0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx2.factor_assemble(kvals, stream=stream)
                torch.cuda.synchronize()
                t_pipe.append(time.perf_counter() - t0)
            q2 = torch.empty_like(q)
            ctx.apply(lam, q, stream=stream)
            ctx2.apply(lam, q2, stream=stream)
            torch.cuda.synchronize()
        same = bool(torch.equal(q, q2))
        ngroups = ctx2.info()["assembly_groups"]
        ctx2.close()
        th, tp = min(t_host) * 1e3, min(t_pipe) * 1e3
        t_overlap = max(0.0, tp - th)
        result["pipelined_preprocessing"] = {
            "groups": ngroups, "host_factor_ms": round(th, 3), "factor_copy_assembly_wall_ms": round(tp, 3),
            "beyond_host_factor_ms": round(t_overlap, 3), "apply_bitwise_equal": same}
        log(f"pipelined factorisation + copy + assembly ({ngroups} groups): {tp:.1f} ms wall, host "
            f"factorisation alone {th:.1f} ms, apply equal to the one-group context: {same}")

    # ---- CPU oracle on the host cores, bounded samples of the workload
    if not args.no_cpu:
        cpu = cpu_oracle_leg(prob, args.cpu_sample)
        t_cpu = cpu["implicit_ms"]
        cpu_gbs = apply_bytes / (t_cpu * 1e-3) / 1e9
        result["cpu_baseline"] = {
            "value": round(cpu_gbs, 3), "unit": "GB/s", "cores": cpu["threads"], "kind": "oracle",
            "sample": cpu["implicit_sample"] + "; value = the explicit operator's algorithmic bytes per apply / "
                      "CPU time per apply",
            "ms_per_apply": round(t_cpu, 3),
            "cpu_model": cpu["cpu_model"], "host_cpus": cpu["host_cpus"],
            "implicit_1_thread_ms_per_apply": round(cpu["implicit_t1_ms"], 3),
            "implicit_1_thread_sample": cpu["implicit_t1_sample"],
            "explicit_assembly_ms": round(cpu["assembly_ms"], 1),
            "explicit_apply_ms": round(cpu["explicit_apply_ms"], 3),
            "explicit_sample": cpu["explicit_sample"]}
        result["gpu_vs_cpu_explicit"] = {
            "assembly_speedup": round(cpu["assembly_ms"] / t_asm, 1),
            "apply_speedup": round(cpu["explicit_apply_ms"] / t_apply, 1),
            "note": "CPU side: the oracle's explicit assembly (one unit solve per local multiplier with its "
                    "sparse Cholesky factor) and dense apply, on all host threads"}
        denom = t_cpu - t_apply
        result["break_even_iters"] = (math.ceil((t_upload + t_asm) / denom) if denom > 0 else None)
        result["break_even_detail"] = {"t_upload_ms": round(t_upload, 3), "t_assembly_ms": round(t_asm, 3),
                                       "t_impl_cpu_ms": round(t_cpu, 3), "t_apply_gpu_ms": round(t_apply, 4)}
        if t_overlap is not None and denom > 0:
            # the same amortisation with the copy and assembly time that the
            # pipelined preprocessing adds beyond the host factorisation
            result["break_even_iters_pipelined"] = max(1, math.ceil(t_overlap / denom))
    print(json.dumps(result), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
