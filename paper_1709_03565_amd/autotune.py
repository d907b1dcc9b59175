"""Autotuner for the persistent sampler's launch shape.

The sampler is compiled in a few shapes (threads per workgroup, sample slots per
workgroup, nodes per sample kept in LDS before the sample moves to the next tier) and
takes one more knob at run time, big_row (the in-degree above which the first tier hands a
sample on).  Which shape is fastest depends on the graph: the cascade-size distribution
decides how many samples outgrow the LDS visited set, and the hub rows decide how long a
workgroup can be held by one sample.  autotune() times every candidate on a pilot sketch
of the real graph (sampling only, measured with the library's own HIP events) and returns
the fastest; results are cached in a JSON file keyed by device, graph shape and a
fingerprint of the edge probabilities.

The pilot has to be about as large as the real build: a persistent launch ends with a tail
in which a few large cascades hold the last workgroups, and that tail is a fixed cost, so
on a small pilot shapes with short tails win even when they are slower per sample.  A
first pass times every shape once; the three fastest are timed again and the best of those
is refined over big_row.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import torch

from . import skis

# (threads_per_block, slots_per_block, visited_threshold, quads_per_lane) the library is compiled for
SHAPES = [(64, 4, 192, 2), (64, 4, 192, 1), (64, 4, 256, 2), (64, 4, 256, 1), (64, 2, 256, 1), (64, 3, 256, 1),
          (64, 2, 384, 1), (64, 6, 256, 2), (64, 8, 128, 2),
          (64, 8, 192, 2), (64, 8, 192, 1), (64, 8, 256, 2), (64, 12, 192, 2), (64, 16, 128, 2), (64, 16, 64, 2),
          (256, 16, 128, 2), (256, 32, 128, 2), (256, 16, 256, 2)]
BIG_ROWS = [4096, 16384, 65536]

_DEFAULT_CACHE = os.path.join(os.environ.get("SKIS_TUNE_CACHE", "/tmp"), "skis_autotune.json")


def _fingerprint(row_ptr, w) -> str:
    rp = row_ptr.cpu().numpy() if isinstance(row_ptr, torch.Tensor) else np.asarray(row_ptr)
    ww = w.cpu().numpy() if isinstance(w, torch.Tensor) else np.asarray(w)
    deg = np.diff(rp.astype(np.int64))
    h = hashlib.sha1()
    h.update(np.array([len(deg), int(deg.sum()), int(deg.max(initial=0))], np.int64).tobytes())
    h.update(np.histogram(deg, bins=32)[0].astype(np.int64).tobytes())
    h.update(np.quantile(ww.astype(np.float64), np.linspace(0, 1, 33)).tobytes() if ww.size else b"")
    return h.hexdigest()[:16]


def _device_key() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return "%s/%d" % (getattr(p, "gcnArchName", p.name), p.multi_processor_count)


def autotune(row_ptr, col, w, pilot_samples: int = 1 << 24, seed: int = 1, shapes=None, big_rows=None,
             repeats: int = 2, cache_path: str | None = _DEFAULT_CACHE, log=None) -> dict:
    """Returns the fastest options as a dict of skis_options field values, plus the timings."""
    key = "%s|%s|T=%d" % (_device_key(), _fingerprint(row_ptr, w), pilot_samples)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        return cache[key]
    shapes = shapes or SHAPES
    big_rows = big_rows or BIG_ROWS
    results = []

    def trial(opts, reps):
        best = None
        for _ in range(reps):
            sk = skis.build_sketch(row_ptr, col, w, pilot_samples, seed, build_inverse_index=0, **opts)
            inf = sk.info()
            sk.free()
            t = inf.ms_tier0 + inf.ms_tier1 + inf.ms_tier2
            best = t if best is None else min(best, t)
        results.append(dict(opts, ms=best))
        if log:
            log("autotune %s: %.2f ms" % (opts, best))
        return best

    first = []
    for (th, sl, vi, pl) in shapes:
        o = dict(threads_per_block=th, slots_per_block=sl, visited_threshold=vi, quads_per_lane=pl)
        first.append((trial(o, 1), o))
    first.sort(key=lambda x: x[0])
    best_opts, best_ms = None, None
    for _, o in first[:3]:
        t = trial(o, repeats)
        if best_ms is None or t < best_ms:
            best_opts, best_ms = o, t
    for br in big_rows:
        o = dict(best_opts, big_row=br)
        t = trial(o, repeats)
        if t < best_ms:
            best_opts, best_ms = o, t
    out = dict(best_opts, ms=best_ms, pilot_samples=pilot_samples, trials=results)
    if cache_path:
        cache[key] = out
        tmp = cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f)
        os.replace(tmp, cache_path)
    return out


def options_from(tuned: dict) -> dict:
    """The skis_options fields of an autotune() result."""
    return {k: v for k, v in tuned.items() if k in ("threads_per_block", "slots_per_block", "visited_threshold",
                                                    "quads_per_lane", "big_row")}
