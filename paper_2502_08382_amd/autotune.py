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

DEFAULT_BANDS = (8192, 16384, 32768, 65536, 131072)


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


def tune_apply(ctx, lam, q, bands=DEFAULT_BANDS, rows=(1, 2), nontemporal=(0, 1), reps=20,
               stream=None, cache=None, verbose=False):
    """Try every (band, rows, nontemporal) shape; install and return the best.

    Returns dict(band=..., rows=..., nontemporal=..., ms=..., trials=[...])."""
    sig = signature(ctx)
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                hit = json.load(f).get(sig)
            if hit:
                ctx.set_apply(hit["band"], hit["rows"], hit["nontemporal"])
                return dict(hit, cached=True)
        except (OSError, ValueError):
            pass
    trials = []
    for b, r, n in itertools.product(bands, rows, nontemporal):
        ctx.set_apply(b, r, n)
        t, tb = _time_apply(ctx, lam, q, reps, stream)
        trials.append(dict(band=b, rows=r, nontemporal=n, ms=t, band_ms=tb))
        if verbose:
            print(f"[autotune] band={b} rows={r} nt={n}: apply {t * 1e3:.1f} us (band kernel {tb * 1e3:.1f} us)",
                  flush=True)
    best = min(trials, key=lambda d: d["ms"])
    ctx.set_apply(best["band"], best["rows"], best["nontemporal"])
    out = dict(band=best["band"], rows=best["rows"], nontemporal=best["nontemporal"], ms=best["ms"],
               trials=trials, cached=False)
    if cache:
        data = {}
        if os.path.exists(cache):
            try:
                with open(cache) as f:
                    data = json.load(f)
            except (OSError, ValueError):
                data = {}
        data[sig] = {k: out[k] for k in ("band", "rows", "nontemporal", "ms")}
        with open(cache, "w") as f:
            json.dump(data, f, indent=1)
    return out
