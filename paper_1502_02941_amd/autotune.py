"""Autotuner for the batched persistent solve.

Times dg_batch_run on a size-stratified subsample of the instances for each
candidate launch shape (threads per workgroup, number of workspace slots =
workgroups, restart-length policy) and keeps the fastest.  Results are cached
in a JSON file keyed by device name, precision form and the subsample's
(degree, size) signature.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np
import torch

CACHE = os.environ.get("DGDCR_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "dgdcr", "autotune.json"))


NONE = 1 << 62


# Largest instance (unknowns) for which solving everything in the persistent
# kernel is tried: one workgroup per instance leaves larger ones running alone
# on a compute unit long after the rest (measured: 97 s instead of 3.5 s on a
# 48-instance sample reaching 98k unknowns).
PERSISTENT_ONLY_MAX_DOFS = 32768


def candidates(n_cu, max_dofs=0):
    """Stage 1: split between the persistent solve (small instances) and the
    lockstep solve (large ones); later stages in tune_batch."""
    base = dict(block_threads=256, slots=2 * n_cu, restart_min=64, restart_per_side=2.0)
    splits = (0, 16384, NONE) if max_dofs <= PERSISTENT_ONLY_MAX_DOFS else (0, 16384)
    return [dict(base, lockstep_min_dofs=t) for t in splits]


def stratified_sample(items, sizes, count, seed=0):
    """About `count` items spread evenly over the size order."""
    order = np.argsort(sizes)
    if len(order) <= count:
        return [items[i] for i in order]
    pick = order[np.linspace(0, len(order) - 1, count).round().astype(int)]
    return [items[i] for i in pick]


def _key(mixed, sample_sig):
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    h = hashlib.sha1(json.dumps(sample_sig).encode()).hexdigest()[:16]
    return "%s|%s|%s" % (dev, "mixed" if mixed else "fp64", h)


def tune_batch(api, instances, mixed, rel_tol=1e-10, inner_tol=1e-5, sample=48, reps=1, log=None, use_cache=True):
    """instances: list of (MeshArrays, Problem).  Returns the best option dict."""
    sizes = [m.T * (p.degree + 1) * (p.degree + 2) // 2 for m, p in instances]
    sub = stratified_sample(instances, sizes, sample)
    sig = sorted((p.degree, m.T) for m, p in sub)
    key = _key(mixed, sig)
    cache = {}
    if use_cache and os.path.exists(CACHE):
        try:
            cache = json.load(open(CACHE))
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        return cache[key]["best"]
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    results = []

    def measure(c):
        slots = min(c["slots"], len(sub))
        b = api.Batch(sub, mixed=mixed, rel_tol=rel_tol, inner_tol=inner_tol, block_threads=c["block_threads"],
                      slots=slots, restart_min=c["restart_min"], restart_per_side=c["restart_per_side"],
                      lockstep_min_dofs=c["lockstep_min_dofs"], log=log)
        x, rep = b.alloc()
        b.run(x, rep)
        b.wait(log)
        ok = bool((b.reports(rep)["status"] == 0).all())
        t0 = time.perf_counter()
        for _ in range(reps):
            x.zero_()
            b.run(x, rep)
            b.wait(log)
        dt = (time.perf_counter() - t0) / reps
        results.append((dt if ok else float("inf"), c))
        if log:
            log("  tune %s: %.1f ms%s" % (c, dt * 1e3, "" if ok else " (not converged)"))
        del b, x, rep
        torch.cuda.empty_cache()

    for c in candidates(n_cu, max(sizes)):
        measure(c)
    results.sort(key=lambda r: r[0])
    shape = dict(results[0][1])
    if shape["lockstep_min_dofs"] != 0:  # persistent part in use: try its other launch shape
        measure(dict(shape, block_threads=512, slots=n_cu))
        results.sort(key=lambda r: r[0])
        shape = dict(results[0][1])
    for rmin, per in ((32, 3.0), (128, 2.0)):
        measure(dict(shape, restart_min=rmin, restart_per_side=per))
    results.sort(key=lambda r: r[0])
    best = dict(results[0][1])
    cache[key] = {"best": best, "ms": results[0][0] * 1e3,
                  "all": [(r[0] * 1e3, r[1]) for r in results]}
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        json.dump(cache, open(CACHE, "w"), indent=1)
    except OSError:
        pass
    return best
