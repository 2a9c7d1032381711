"""Launch-shape autotuner with a JSON cache.

For a model it times the element passes and the particle passes (forward and
adjoint) under candidate launch shapes -- threads per workgroup (element passes:
per planned element tile) and, for the particle passes, particles per thread,
i.e. the tile size -- with HIP events around every launch
(``gsim_model_set_timing``), and keeps the fastest shape of each pass.  Results
are cached per (GPU architecture, pass, size bucket) in a JSON file
(``$GSIM_AUTOTUNE_CACHE``, default ``~/.cache/gsim_autotune.json``), so later
models of a similar size reuse them without timing.

The element-pass shape never changes results; the particle-pass shape fixes the
summation tree of per-body contact gradients and losses (deterministic for a
given shape).
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import gsim

ELEMENT_CANDIDATES = ((64, 1), (128, 1), (256, 1), (512, 1))
PARTICLE_CANDIDATES = ((64, 1), (128, 1), (256, 1), (512, 1), (256, 2), (128, 4))


def cache_path():
    return os.environ.get("GSIM_AUTOTUNE_CACHE", os.path.expanduser("~/.cache/gsim_autotune.json"))


def _load_cache():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def bucket_key(model, pass_):
    arch = torch.cuda.get_device_properties(model.device).gcnArchName.split(":")[0]
    n = (model.ne + model.nt + model.nh) if pass_ == 0 else model.np
    kind = "tet" if model.ne else "shell"
    return "%s/%s/%s/2^%d/%s" % (arch, "element" if pass_ == 0 else "particle", kind, int(math.log2(max(n, 1))),
                                 "f64" if model.dtype == torch.float64 else "f32")


def _time_passes(model, params, x, v, steps, stream):
    """Average per-launch ms of (element fwd, particle fwd, element adj, particle adj)."""
    xb = torch.zeros_like(x)
    vb = torch.ones_like(v) * 1e-3
    g = model.zero_grads()
    model.set_timing()
    for _ in range(steps):
        model.step(params, x, v, 1, stream=stream)
        model.step_backward(params, x, v, xb, vb, g, stream=stream)
    torch.cuda.synchronize()
    t = model.read_timing()
    model.set_timing(())
    return {k: (ms / n if n else float("inf")) for k, (n, ms) in t.items()}


def tune(model, params, x, v, steps=6, use_cache=True, stream=None):
    """Chooses and applies the fastest launch shape of each pass; returns a report."""
    cache = _load_cache() if use_cache else {}
    exec_mode = model.get_exec()[0]
    model.set_exec(gsim.EXEC_PLAIN)
    report = {}
    for pass_, cands, names in ((0, ELEMENT_CANDIDATES, ("element_fwd", "element_adj")),
                                (1, PARTICLE_CANDIDATES, ("particle_fwd", "particle_adj"))):
        key = bucket_key(model, pass_)
        if key in cache:
            b, i = cache[key]["shape"]
            model.set_launch(pass_, b, i)
            report[key] = dict(cache[key], cached=True)
            continue
        results = {}
        for b, i in cands:
            model.set_launch(pass_, b, i)
            _time_passes(model, params, x, v, 2, stream)  # warm
            t = _time_passes(model, params, x, v, steps, stream)
            results["%dx%d" % (b, i)] = sum(t[n] for n in names)
        best = min(results, key=results.get)
        b, i = (int(s) for s in best.split("x"))
        model.set_launch(pass_, b, i)
        cache[key] = {"shape": [b, i], "ms_per_step": results[best], "candidates": results}
        report[key] = dict(cache[key], cached=False)
    model.set_exec(exec_mode)
    if use_cache:
        _save_cache(cache)
    return report
