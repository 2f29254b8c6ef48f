"""Autotuner of the batched calls: the band width b of step (1) per size bucket.

The band width trades the cost of the full -> band reduction (smaller panels,
more of them) against bulge chasing and the Q2 back-transformation (about
6 b n^2 flops and (n/b)^2 reflector blocks); the best b for small problems is
not the best for large ones.  The tuner times the caller's own problems: for
each size bucket it takes a sample of up to `per_bucket` problems of the
batch, solves copies of them in one batched call with each candidate width,
and keeps the fastest.  The resulting table goes to the handle
(elsi_gpu_set_batch_band_table) and, keyed by device, buckets, candidates and
the sizes sampled, to a JSON cache file, so that a later run with the same
batch composition skips the timing.  Every solve runs in the library's kernels;
this module only chooses a setting.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import binding as B

DEFAULT_CANDIDATES = (16, 32, 48, 64)


def default_buckets(sizes) -> list[int]:
    """Upper bounds of power-of-two size buckets covering `sizes`."""
    top = max(int(x) for x in sizes)
    bounds, hi = [], 512
    while True:
        bounds.append(hi)
        if hi >= top:
            return bounds
        hi *= 2


def _sample(idx_sorted, per_bucket):
    """Up to per_bucket indices spread evenly over a bucket (sorted by size)."""
    if len(idx_sorted) <= per_bucket:
        return list(idx_sorted)
    step = len(idx_sorted) / per_bucket
    return [idx_sorted[int(i * step + step / 2)] for i in range(per_bucket)]


def _cache_key(device_name, buckets, candidates, sampled_sizes, workers):
    return json.dumps({"device": device_name, "buckets": list(buckets), "candidates": list(candidates),
                       "sizes": sampled_sizes, "workers": workers}, sort_keys=True)


def tune_batch_band_widths(handle: B.Handle, Hs, Ss, n_electrons, buckets=None,
                           candidates=DEFAULT_CANDIDATES, per_bucket: int = 8, workers: int = 8,
                           cache_path: str | None = None, log=None):
    """Choose the band width per size bucket for `handle`'s batched dm calls.

    Hs, Ss: the batch's device matrices (not modified: the timing solves copies);
    n_electrons: per problem.  Returns {"n_max": [...], "b": [...], "ms": {...},
    "tune_ms": wall time of the tuning, "cached": bool} and sets the table on
    the handle (and its worker count to `workers`).  Problems above the last
    bucket keep the handle's band width.
    """
    sizes = [int(H.shape[0]) for H in Hs]
    if not sizes:
        handle.set_batch_band_table([], [])
        return {"n_max": [], "b": [], "ms": {}, "tune_ms": 0.0, "cached": False}
    buckets = list(buckets) if buckets else default_buckets(sizes)
    candidates = [int(b) for b in candidates]
    order = sorted(range(len(sizes)), key=lambda q: sizes[q])
    samples, lo = [], 0
    for hi in buckets:
        members = [q for q in order if lo < sizes[q] <= hi]
        samples.append(_sample(members, per_bucket))
        lo = hi
    sampled_sizes = [[sizes[q] for q in s] for s in samples]
    cache_path = cache_path or os.environ.get("ELSI_GPU_TUNE_CACHE")
    dev_name = torch.cuda.get_device_name(Hs[0].device)
    key = _cache_key(dev_name, buckets, candidates, sampled_sizes, workers)
    handle.set_batch_workers(workers)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            rec = cache[key]
            handle.set_batch_band_table(rec["n_max"], rec["b"])
            return dict(rec, tune_ms=0.0, cached=True)

    t_start = time.perf_counter()
    n_max, widths, timings = [], [], {}
    for hi, sample in zip(buckets, samples):
        if not sample:
            continue
        Hc = [torch.empty_like(Hs[q]) for q in sample]
        Sc = [torch.empty_like(Ss[q]) for q in sample] if Ss is not None else None
        ne = [n_electrons[q] for q in sample]

        def solve(b):
            for a, q in zip(Hc, sample):
                a.copy_(Hs[q])
            if Sc is not None:
                for a, q in zip(Sc, sample):
                    a.copy_(Ss[q])
            handle.set_batch_band_table([hi], [b])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            handle.dm_batched(Hc, Sc, ne)
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) * 1e3

        solve(candidates[-1])   # first touch of this bucket's sizes
        ms = {b: solve(b) for b in candidates}
        best = min(candidates, key=lambda b: ms[b])
        timings[str(hi)] = {str(b): round(v, 3) for b, v in ms.items()}
        n_max.append(hi)
        widths.append(best)
        if log:
            log(f"[tune] n <= {hi}: {len(sample)} problems, ms per width {timings[str(hi)]}, b = {best}")
        del Hc, Sc
    handle.set_batch_band_table(n_max, widths)
    rec = {"n_max": n_max, "b": widths, "ms": timings}
    if cache_path:
        cache[key] = rec
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_path)
    return dict(rec, tune_ms=(time.perf_counter() - t_start) * 1e3, cached=False)
