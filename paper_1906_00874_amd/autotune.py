"""Autotuner of the factorisation's tile shapes on the device it runs on.

The knobs are the tile shape of the truncation (the widest stacked factor
pair one pass takes: the K of its Gram, pivoted-Cholesky and SVD-core tiles)
and the width of the persistent launch (workgroups).  Neither changes the
method: the rank rule and tolerance stay the same, so every candidate's
factors meet the same accuracy bound; they differ from each other within
the truncation tolerance, not bit for bit.  A run is bitwise reproducible
for a fixed choice, which is what batched-versus-alone equality relies on.

The search is coordinate-wise: the stack widths first at the default launch
width, then the launch widths at the best stack width.  Every candidate is
timed by HIP events on the launch stream around whole factorisations (the
restore of the assembled matrices from their pristine copies is outside the
timed region), and the median of `reps` runs decides.  Choices can be kept
in a JSON cache keyed by the workload's signature.
"""
from __future__ import annotations

import json
import os
import time

WIDTHS = (64, 48, 40, 32)
WORKERS = (0, 192, 128)


def signature(handles, extra=""):
    """Key of a workload: the sizes and planning parameters of its matrices."""
    sizes = {}
    for h in handles:
        sizes[h.n] = sizes.get(h.n, 0) + 1
    p = handles[0].params
    parts = [f"{n}x{c}" for n, c in sorted(sizes.items())]
    return (f"n[{','.join(parts)}]-leaf{p.leaf_size}-eta{p.eta:g}-eps{p.eps_factor:g}-"
            f"cap{p.rank_cap_factor}-fix{p.fixed_rank}-prec{int(p.precision)}{extra}")


def _median(v):
    v = sorted(v)
    return v[len(v) // 2] if len(v) % 2 else 0.5 * (v[len(v) // 2 - 1] + v[len(v) // 2])


def search(measure, widths=WIDTHS, workers=WORKERS):
    """Coordinate search over (stack width, workers) with `measure(w, k)`
    returning a time in ms; returns (best (w, k), table of measured rows)."""
    table = []
    best = None
    for w in widths:
        t = measure(w, workers[0])
        table.append({"trunc_width": w, "workers": workers[0], "ms": round(t, 3)})
        if best is None or t < best[2]:
            best = (w, workers[0], t)
    for k in workers[1:]:
        t = measure(best[0], k)
        table.append({"trunc_width": best[0], "workers": k, "ms": round(t, 3)})
        if t < best[2]:
            best = (best[0], k, t)
    return (best[0], best[1]), table


def _load(cache):
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            return json.load(fh)
    return {}


def _store(cache, key, entry):
    if not cache:
        return
    data = _load(cache)
    data[key] = entry
    tmp = cache + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, cache)


def tune_batch(batch, handles, reps=2, widths=WIDTHS, workers=WORKERS, cache=None,
               log=None):
    """Pick and apply the fastest (stack width, workers) for `batch` (a
    binding.Batch over `handles`).  Returns {"trunc_width", "workers",
    "table", "signature", "cached"}."""
    import torch
    key = signature(handles, "-batch")
    hit = _load(cache).get(key)
    if hit:
        batch.set_tuning(hit["trunc_width"], hit["workers"])
        return dict(hit, signature=key, cached=True)
    stream = torch.cuda.current_stream()

    def measure(w, k):
        batch.set_tuning(w, k)
        ts = []
        for _ in range(reps):
            for h in handles:
                h.reset()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            batch.factor()
            e1.record(stream)
            batch.sync()
            ts.append(e0.elapsed_time(e1))
        t = _median(ts)
        if log:
            log(f"autotune: trunc_width {w} workers {k}: {t:.1f} ms")
        return t

    t0 = time.perf_counter()
    (w, k), table = search(measure, widths, workers)
    batch.set_tuning(w, k)
    entry = {"trunc_width": w, "workers": k, "table": table,
             "tuning_s": round(time.perf_counter() - t0, 1)}
    _store(cache, key, entry)
    return dict(entry, signature=key, cached=False)


def tune_handle(h, reps=3, widths=WIDTHS, workers=WORKERS, cache=None, log=None):
    """The same for one handle factored by the dataflow executor."""
    import torch
    key = signature([h], "-single")
    hit = _load(cache).get(key)
    if hit:
        h.set_tuning(hit["trunc_width"])
        h.set_workers(hit["workers"])
        return dict(hit, signature=key, cached=True)
    stream = torch.cuda.current_stream()

    def measure(w, k):
        h.set_tuning(w)
        h.set_workers(k)
        ts = []
        for _ in range(reps):
            h.reset()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            h.factor()
            e1.record(stream)
            h.sync()
            ts.append(e0.elapsed_time(e1))
        t = _median(ts)
        if log:
            log(f"autotune: trunc_width {w} workers {k}: {t:.1f} ms")
        return t

    t0 = time.perf_counter()
    (w, k), table = search(measure, widths, workers)
    h.set_tuning(w)
    h.set_workers(k)
    entry = {"trunc_width": w, "workers": k, "table": table,
             "tuning_s": round(time.perf_counter() - t0, 1)}
    _store(cache, key, entry)
    return dict(entry, signature=key, cached=False)
