"""Autotuner of the apply work decomposition (the paper's parameter
auto-configuration, Sec. V-A, applied to this library's own kernel shapes).

It times the candidate shapes of fetiF_apply with the library's HIP-event
phase timers on the caller's stream and keeps the fastest.  Results can be
cached in a JSON file keyed by a signature of the problem (subdomain count,
multiplier-count statistics, storage precision).
"""
from __future__ import annotations

import itertools
import json
import os


def signature(ctx):
    ms = sorted(ctx.m)
    return f"n{ctx.nsub}-m{ms[0]}-{ms[len(ms) // 2]}-{ms[-1]}-p{ctx.f_storage}"


def _time_apply(ctx, lam, q, reps, stream):
    import torch
    ctx.apply(lam, q, stream=stream)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    for _ in range(reps):
        ctx.apply(lam, q, stream=stream)
    ctx.profile(False)
    prof = ctx.profile_read(reset=True)
    band = prof["apply_band"][0] / max(1, prof["apply_band"][1])
    gath = prof["apply_gather"][0] / max(1, prof["apply_gather"][1])
    return band + gath, band


def group_candidates(ctx, per_cu=(2, 3, 4, 6, 8, 12)):
    """Elements per work-group that give about k work-groups per compute
    unit for the whole apply (exactly k with the equal-share split)."""
    import torch
    ncu = torch.cuda.get_device_properties(ctx.device).multi_processor_count
    total = ctx.info()["apply_elements"]
    return tuple(max(1, -(-total // (ncu * k))) for k in per_cu)


def tune_apply(ctx, lam, q, bands=None, rows=(2, 4), nontemporal=(1,), splits=(0, 1), segs=(0, 2, 3, 4, 8), reps=20,
               stream=None, cache=None, verbose=False):
    """Try every (kernel, split, band, rows, nontemporal) shape; install and
    return the best.  bands: candidate elements per work-group (default:
    group_candidates); segs: 0 the whole-row kernel, 2/3/4/8 the
    column-segmented kernel with that many chunks per segment.

    Returns dict(band=..., rows=..., nontemporal=..., split=..., seg=..., ms=..., trials=[...])."""
    if bands is None:
        bands = group_candidates(ctx)
    sig = signature(ctx)
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                hit = json.load(f).get(sig)
            if hit:
                ctx.set_apply(hit["band"], hit["rows"], hit["nontemporal"], hit.get("split", 0), hit.get("seg", 0))
                return dict(hit, cached=True)
        except (OSError, ValueError):
            pass
    trials = []
    for sg, sp, b, r, n in itertools.product(segs, splits, bands, rows, nontemporal):
        if sg == 8 and r == 4:
            continue   # no such kernel instance
        if sg == 0 and max(ctx.m) > 4096:
            continue   # the whole-row kernel holds at most 4096 columns
        ctx.set_apply(b, r, n, sp, sg)
        t, tb = _time_apply(ctx, lam, q, reps, stream)
        trials.append(dict(band=b, rows=r, nontemporal=n, split=sp, seg=sg, ms=t, band_ms=tb))
        if verbose:
            print(f"[autotune] seg={sg} split={sp} band={b} rows={r} nt={n}: apply {t * 1e3:.1f} us "
                  f"(band kernel {tb * 1e3:.1f} us)", flush=True)
    best = min(trials, key=lambda d: d["ms"])
    ctx.set_apply(best["band"], best["rows"], best["nontemporal"], best["split"], best["seg"])
    out = dict(band=best["band"], rows=best["rows"], nontemporal=best["nontemporal"], split=best["split"],
               seg=best["seg"], ms=best["ms"], trials=trials, cached=False)
    if cache:
        data = {}
        if os.path.exists(cache):
            try:
                with open(cache) as f:
                    data = json.load(f)
            except (OSError, ValueError):
                data = {}
        data[sig] = {k: out[k] for k in ("band", "rows", "nontemporal", "split", "seg", "ms")}
        with open(cache, "w") as f:
            json.dump(data, f, indent=1)
    return out


STORED_SHAPES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_apply.json")


def stored_apply_shape(ctx, cache=STORED_SHAPES):
    """The apply shape stored for this workload's signature, or None."""
    try:
        with open(cache) as f:
            return json.load(f).get(signature(ctx))
    except (OSError, ValueError):
        return None


def install_stored_apply_shape(ctx, cache=STORED_SHAPES):
    """Install the stored apply shape of this workload (what the benchmark
    runs when its tuner finds the workload in the store); returns it, or
    None when the store has no entry (the context keeps its defaults)."""
    hit = stored_apply_shape(ctx, cache)
    if hit:
        ctx.set_apply(hit["band"], hit["rows"], hit["nontemporal"], hit.get("split", 0), hit.get("seg", 0))
    return hit


def tune_assembly(ctx, panels=(32, 48, 64, 96), chunks=(16, 32, 64), reps=3, stream=None, verbose=False):
    """Try every (TRSM panel width, RHS columns per work-group) shape of the
    assembly; install and return the fastest by the TRSM phase time.  The
    context must hold uploaded factors (it is assembled once per trial)."""
    import torch
    trials = []
    for p, c in itertools.product(panels, chunks):
        ctx.set_assembly(p, c)
        ctx.assemble(stream=stream)
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_read(reset=True)
        for _ in range(reps):
            ctx.assemble(stream=stream)
        ctx.profile(False)
        prof = ctx.profile_read(reset=True)
        t = prof["trsm"][0] / max(1, prof["trsm"][1])
        trials.append(dict(panel=p, chunk=c, trsm_ms=t))
        if verbose:
            print(f"[autotune] trsm panel={p} chunk={c}: {t:.3f} ms", flush=True)
    best = min(trials, key=lambda d: d["trsm_ms"])
    ctx.set_assembly(best["panel"], best["chunk"])
    return dict(best, trials=trials)
