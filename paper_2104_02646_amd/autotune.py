"""Autotuner with a JSON cache, at two levels.

``tune_model`` chooses how a batch is planned and launched: the element-tile size of
the two-pass path (elements per tile), the number of concurrent launch lanes, and the
execution (two-pass launches replayed from a captured graph, the fused path with one
workgroup per LDS-resident body, or persistent execution of the two-pass tiles with one
workgroup per body), by timing whole checkpointed gradient evaluations (rollout, loss,
adjoint) of every candidate with HIP events on the launch stream; it returns the model
built with the fastest configuration.

``tune`` chooses, for a given model, the launch shape of each pass: threads per
workgroup (element passes: per planned element tile) and, for the particle passes,
particles per thread, with HIP events around every launch
(``gsim_model_set_timing``).

Both cache their choice in a JSON file (``$GSIM_AUTOTUNE_CACHE``, default
``~/.cache/gsim_autotune.json``) per GPU architecture and size bucket, so later
models of a similar size reuse it without timing.

None of these choices changes the model: the tile size, the lanes and the element-pass
shape change only the order in which element contributions are summed (tile size) or
nothing at all (lanes, element-pass shape); the particle-pass shape fixes the
summation tree of per-body contact gradients and losses.  Each configuration is
deterministic.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import gsim

ELEMENT_CANDIDATES = ((64, 1), (128, 1), (256, 1), (512, 1))
TILE_CANDIDATES = (128, 256, 384, 512)
LANE_CANDIDATES = (1, 2, 3, 4)
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


def _arch(device):
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def model_key(bodies, dtype, T, K, device):
    n = sum(b.ne + b.nt + b.nh for b in bodies)
    return "%s/model/%d-bodies/2^%d-elements/T%d-K%d/%s" % (
        _arch(device), 2 ** int(math.log2(max(len(bodies), 1))), int(math.log2(max(n, 1))), T, K,
        "f64" if dtype == torch.float64 else "f32")


def _gradient_ms(m, bodies, T, reps, stream):
    """Median ms of one checkpointed gradient (rollout, loss, zeroed gradients, adjoint)."""
    import numpy as np
    p = m.params_from_bodies()
    x0 = gsim.soa(np.concatenate([b.x0 for b in bodies])).to(m.device)
    v0 = gsim.soa(np.concatenate([b.v0 for b in bodies])).to(m.device)
    tgt = x0 + 0.01
    xT, vT = m.empty_state()
    xb0, vb0 = m.empty_state()
    want = tuple(k for k, n in (("mu", m.ne), ("lam", m.ne), ("ktri", m.nt)) if n) + ("mass", "contact")
    g = m.zero_grads(want)

    def one():
        m.rollout(p, x0, v0, T, out=(xT, vT), stream=stream)
        loss, xb, vb = m.loss_mse(xT, tgt, stream=stream)
        for t in g.values():
            t.zero_()
        m.rollout_backward(p, T, xb, vb, g, out=(xb0, vb0), stream=stream)
    with torch.cuda.stream(stream):
        one()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(stream)
        for k in range(reps):
            one()
            ev[k + 1].record(stream)
        ev[-1].synchronize()
    return float(np.median([ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]))


def tune_model(bodies, dtype=torch.float32, max_steps=100, ckpt_every=10, reps=3, use_cache=True, device="cuda",
               stream=None, tiles=TILE_CANDIDATES, lanes=LANE_CANDIDATES, fused=True):
    """Builds the batch with every candidate (tile size, lanes, graph) and, with `fused`,
    the fused path, times a gradient of max_steps steps for each, and returns (model,
    report) for the fastest; the model is left in that configuration."""
    stream = stream or torch.cuda.Stream(device)
    T, K = int(max_steps), int(ckpt_every)
    key = model_key(bodies, dtype, T, K, device) + ("" if fused else "/two-pass")
    cache = _load_cache() if use_cache else {}

    def build(tile, n_lanes, exec_mode):
        with torch.cuda.stream(stream):
            m = gsim.Model(bodies, dtype, max_steps=T, ckpt_every=K, device=device, stream=stream, tile_elems=tile)
        m.set_exec(exec_mode)
        m.set_lanes(min(n_lanes, len(bodies)))
        return m
    if key in cache:
        c = cache[key]["choice"]
        return build(c["tile_elems"], c["lanes"], c["exec"]), dict(cache[key], cached=True)
    results = {}
    for tile in tiles:
        m = build(tile, 1, gsim.EXEC_GRAPH)
        for n_lanes in lanes:
            if n_lanes > len(bodies):
                continue
            m.set_lanes(n_lanes)
            results["tile%d/lanes%d/graph" % (tile, n_lanes)] = _gradient_ms(m, bodies, T, reps, stream)
        del m
    if fused:
        try:
            m = build(0, 1, gsim.EXEC_FUSED)
            results["fused"] = _gradient_ms(m, bodies, T, reps, stream)
            del m
        except gsim.GsimError:
            pass  # a body does not fit one workgroup's LDS
        try:
            m = build(0, 1, gsim.EXEC_PERSIST)
            results["persist"] = _gradient_ms(m, bodies, T, reps, stream)
            del m
        except gsim.GsimError:
            pass  # FP64, or a body with lift/drag
    torch.cuda.synchronize()
    best = min(results, key=results.get)
    if best in ("fused", "persist"):
        choice = {"tile_elems": gsim.TILE_DEFAULT, "lanes": 1,
                  "exec": gsim.EXEC_FUSED if best == "fused" else gsim.EXEC_PERSIST}
    else:
        t, l, _ = best.split("/")
        choice = {"tile_elems": int(t[4:]), "lanes": int(l[5:]), "exec": gsim.EXEC_GRAPH}
    entry = {"choice": choice, "ms_per_gradient": results[best], "candidates_ms": results}
    if use_cache:
        cache[key] = entry
        _save_cache(cache)
    return build(choice["tile_elems"], choice["lanes"], choice["exec"]), dict(entry, cached=False)
