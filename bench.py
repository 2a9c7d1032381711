"""Benchmark: batched forward + checkpointed adjoint of the differentiable step.

Workload (default): 256 independent tet bodies, tet counts log-uniform in
[500, 20000] (box or grid-in-sphere voxelisations), FP32, per-body materials
mu, lambda ~ U(1e4, 1e5), mass ~ U(0.5, 1.5), ground contact k_e = 1e4,
mu_f = 0.5; 100 steps of dt = 1/600 forward with a checkpoint every 10 steps,
then the checkpointed adjoint (segment recompute + adjoint steps) back to
gradients w.r.t. mu, lambda, mass and the contact parameters.  All bodies are
stepped together: two launches per simulation step cover every body, and the
whole launch sequence is replayed from a captured hipGraph.

One bench step = one system-identification gradient evaluation over the batch:
rollout (with checkpoints) + loss + zeroing of gradients + rollout_backward.
value = sum_b Ne_b * T / (seconds per bench step), element-steps/s fwd+adjoint.

Also reported: forward-only rate; the plain one-body-per-launch path (each body
its own model, plain launches, no graph); per-kernel durations from HIP events
(plain execution, one extra bench step); the roofline of the dominant kernel;
the FP64 oracle on a bounded sample of the same bodies on the host CPU, and the
FP32 gradient error of those bodies against the oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "element-steps/s fwd+adjoint (FP32, grad err ≤1e-3); served p50/p99 query latency"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(kernel, ne, np_, K):
    """Bytes one launch of `kernel` must move by the method's own arrays (FP32 / int32),
    each touched once, none of the design's intermediates (tile-particle records,
    per-tile partials, staged copies): the per-element and per-particle figures of the
    scope table's accounting, split over the two passes.
      element_fwd   64 Ne (tet record: corners 16, Dm^-1 36, volume 4, mu + lambda 8)
                    + 12 Np (positions);
      particle_fwd  52 Np (x, v, w read; x, v written);
      element_adj   64 Ne + 16 Ne / K (mu-bar, lambda-bar written once per segment)
                    + 40 Np (x, xbar+, vbar+, w);
      particle_adj  84 Np (x, v, w, xbar+, vbar+ read; xbar-, vbar- written; mass-bar
                    read-modify-write)."""
    if kernel == "element_fwd":
        return 64 * ne + 12 * np_
    if kernel == "particle_fwd":
        return 52 * np_
    if kernel == "element_adj":
        return 64 * ne + 16 * ne / K + 40 * np_
    if kernel == "particle_adj":
        return 84 * np_
    if kernel in ("element_dual", "particle_dual"):  # a shared launch: one pass of each
        return (algorithmic_bytes(kernel.replace("dual", "fwd"), ne, np_, K)
                + algorithmic_bytes(kernel.replace("dual", "adj"), ne, np_, K))
    return None


DUAL_PAIR_MIN_TILES = 2048  # the library pairs a tile's two passes from this many element tiles on


def compulsory_per_launch(kernel, ne, np_, ntp, T, K, launches, paired=True):
    """Compulsory bytes of one launch: a two-pass kernel's bytes per pass (its
    kernel_bytes over the passes of that kind in one gradient, whether they run on their
    own or in shared launches), a shared launch the sum of its two passes' (the shared
    element launch in the paired layout less one read of the element records, 64 B per
    tet: its workgroups run both passes of a tile), a fused kernel's total over its
    launches."""
    nseg = -(-T // K)
    passes = {"element_fwd": T + (T - nseg), "particle_fwd": T + (T - nseg), "element_adj": T, "particle_adj": T}
    if kernel in passes:
        return kernel_bytes(kernel, ne, np_, ntp, T, K) / passes[kernel]
    if kernel in ("element_dual", "particle_dual"):
        both = sum(compulsory_per_launch(kernel.replace("dual", x), ne, np_, ntp, T, K, None) for x in ("fwd", "adj"))
        return both - (64 * ne if kernel == "element_dual" and paired else 0)
    return kernel_bytes(kernel, ne, np_, ntp, T, K) / launches


def kernel_bytes(kernel, ne, np_, ntp, T, K):
    """Compulsory bytes of this design (FP32 / int32) that all launches of `kernel` in
    one bench step move, each array touched once per pass.  Tet bodies only;
    ntp = tile particles (sum over element tiles of the particles each touches).
      element pass, per tet: corner codes 16, D_m^-1 36, volume 4, mu + lambda 8
        (adjoint: + mu-bar, lambda-bar read-modify-write 16); per tile particle:
        record (index, run, partial slot) 12, positions 12 (adjoint: + the adjoint force
        12), partial write 12 (adjoint: 16);
      particle pass, per particle: partial count 4, x, v 24, mass 4, pinned 1, writes
        24 (adjoint: xbar+, vbar+ 24, x, v 24, mass 4, pinned 1, partial count 4,
        writes 24, mass-bar read-modify-write 8); per partial: 12 (adjoint: 16);
        checkpoint stores 24 per particle per segment."""
    nseg = -(-T // K)
    fwd_passes = T + (T - nseg)  # rollout + segment recompute
    if kernel == "element_fwd":
        return fwd_passes * (64 * ne + 36 * ntp)
    if kernel == "particle_fwd":
        return fwd_passes * (57 * np_ + 12 * ntp) + nseg * 24 * np_
    if kernel == "element_adj":
        # adjoint force handed over by the previous particle adjoint: x and fbar (24)
        # per tile particle, except for the first adjoint step (x, xbar+, vbar+, mass,
        # pinned: 41)
        return T * (80 * ne + 52 * ntp) + 17 * ntp
    if kernel == "particle_adj":
        # + the adjoint force of the previous step written (12 per particle)
        return T * (101 * np_ + 16 * ntp) - 12 * np_
    if kernel == "fused_fwd":
        # per step: tet record 56 + mu, lambda 8 + original index 4; mass, pinned 5 per particle;
        # per launch: state in 24 (+ out 24 for the rollout); stores: checkpoints, segment states
        return (fwd_passes * (68 * ne + 5 * np_) + (1 + nseg) * 24 * np_ + 24 * np_
                + nseg * 24 * np_ + (T - nseg) * 24 * np_)
    if kernel == "fused_adj":
        # per step: record 68 + mu-bar, lambda-bar read-modify-write 16 per tet; per particle:
        # state x, v 24, adjoint state read+write 48, mass, pinned 5, mass-bar read-modify-write 8
        return T * (84 * ne + 85 * np_) + nseg * 48 * np_
    raise ValueError(kernel)


# HBM bytes per launch of the two-pass kernels on the default workload, from the
# rocprofv3 FETCH_SIZE and WRITE_SIZE runs summarised in
# profiles/batch256_two_pass_kernel_stats.md (FETCH_SIZE scaled by 2.0 and WRITE_SIZE by
# 1.0, the factors a 1 GiB copy gives).  They hold for the kernel sources with this SHA-1
# (of gsim_kernels.hip followed by gsim_device.h) and 512-element tiles only; for any other
# source or tile size the traffic is reported as null.
MEASURED_TRAFFIC = {
    "source_sha1": "3d05ef10ad73b646266638641f7adf5421e2a62a",
    "workload": (256, 100, 10, 512),  # bodies, steps, checkpoint interval, elements per tile
    "per_launch": {"element_fwd": 106.21e6, "particle_fwd": 27.68e6, "element_adj": 134.20e6,
                   "particle_adj": 42.67e6, "element_dual": 206.37e6, "particle_dual": 68.50e6},
}


def measured_traffic(kernel, bodies, T, K, tile_elems=256):
    import hashlib
    h = hashlib.sha1()
    for name in ("gsim_kernels.hip", "gsim_device.h"):
        with open(os.path.join(ROOT, "paper_2104_02646_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    sha = h.hexdigest()
    if sha != MEASURED_TRAFFIC["source_sha1"] or (bodies, T, K, tile_elems) != MEASURED_TRAFFIC["workload"]:
        return None
    return MEASURED_TRAFFIC["per_launch"].get(kernel)


def step_algorithmic_bytes(ne, np_, K, nt=0, nh=0):
    """Whole-step accounting: B_f = 64 Ne + 52 Np per forward step, B_a = 64 Ne + 84 Np
    + 16 Ne/K per adjoint step; triangles add 36 B (indices 12, Dm^-1 16, area 4,
    stiffness 4) per pass and 8 Nt/K for their stiffness gradient, hinges 20 B (indices
    16, rest angle 4)."""
    bf = 64 * ne + 36 * nt + 20 * nh + 52 * np_
    ba = 64 * ne + 36 * nt + 20 * nh + 84 * np_ + (16 * ne + 8 * nt) / K
    return bf, ba


def gradient_bytes(ne, np_, T, K, nt=0, nh=0, kept=False):
    """Algorithmic bytes of one checkpointed gradient: the forward passes that run (T
    in the rollout, T - ceil(T/K) recomputed: the first state of each segment is its
    checkpoint; with `kept`, the last segment's states come from the rollout and its
    recompute does not run) times B_f, plus T adjoint steps times B_a."""
    bf, ba = step_algorithmic_bytes(ne, np_, K, nt, nh)
    nseg = -(-T // K)
    fwd_passes = T + (T - nseg) - ((T - (nseg - 1) * K - 1) if kept else 0)
    return fwd_passes * bf + T * ba, fwd_passes


def kernel_table(timing, ne, np_, ntp, T, K, paired=True):
    """Per-kernel averages from the HIP-event timing of one gradient, with the
    algorithmic and the design's compulsory bytes per launch."""
    kern = {}
    for k, (n, ms) in timing.items():
        if n:
            avg = ms / n
            alg = algorithmic_bytes(k, ne, np_, K)
            comp = compulsory_per_launch(k, ne, np_, ntp, T, K, n, paired)
            kern[k] = {"launches": n, "avg_us": avg * 1e3, "total_ms": ms, "compulsory_bytes_per_launch": comp,
                       "compulsory_GBps": comp / (avg * 1e-3) / 1e9}
            if alg is not None:
                kern[k].update(algorithmic_bytes_per_launch=alg, GBps=alg / (avg * 1e-3) / 1e9)
    return kern


def roofline(d, name, traffic):
    """Roofline object of the dominant kernel: achieved = algorithmic bytes per launch /
    average launch duration; the design's compulsory bytes and the HBM counter traffic
    (per launch, null when not taken for this source) beside it, each as a ratio to
    the algorithmic bytes."""
    alg = d["algorithmic_bytes_per_launch"]
    return {"bound": "hbm", "kernel": name, "achieved": d["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": d["GBps"] / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_over_algorithmic": None if traffic is None else traffic / alg,
            "algorithmic_bytes_per_launch": alg, "compulsory_bytes_per_launch": d["compulsory_bytes_per_launch"],
            "compulsory_over_algorithmic": d["compulsory_bytes_per_launch"] / alg, "avg_launch_us": d["avg_us"]}


def cpu_baseline(bodies, targets, T, budget_tets):
    """FP64 oracle fwd + loss + adjoint on the first bodies until budget_tets tets."""
    import oracle.oracle as orc
    orc.build(force=False)
    sample, tot = [], 0
    for i, b in enumerate(bodies):
        if tot >= budget_tets:
            break
        sample.append(i)
        tot += b.ne
    out = {}
    # one host core, like taskset -c 0: the oracle runs in this thread, pinned to core 0
    keep = os.sched_getaffinity(0)
    os.sched_setaffinity(0, {min(keep)})
    try:
        t0 = time.perf_counter()
        for i in sample:
            b = bodies[i]
            o = orc.Oracle(b.X, tets=b.tets, pinned=b.pinned, gravity=b.gravity, ground=True, plane=b.plane, dt=b.dt)
            L, g, xs, vs = o.loss_and_grad(b.params(), b.x0, b.v0, T, targets[i], want=("mu", "lam", "mass"))
            out[i] = (L, g, xs[-1])
        dt = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, keep)
    return sample, tot, dt, out, min(keep)


# The paper's timing analysis (Table 4, right): differentiable-physics steps per second
# of deformable simulation by tet count, forward and backward; hardware and precision
# not stated.  Context only.
PAPER_TABLE4_RIGHT = {"hardware": "not stated", "unit": "simulation steps/s (Hz)",
                      "rows": [{"tets": n, "fwd_hz": f, "bwd_hz": b, "fwd_elem_steps_per_s": n * f,
                                "fwd_plus_bwd_elem_steps_per_s": n / (1.0 / f + 1.0 / b)}
                               for n, f, b in ((100, 9057, 3721), (200, 9057, 3780), (400, 8751, 3750),
                                               (1000, 4174, 1644), (2000, 3967, 1655), (5000, 3871, 1553),
                                               (10000, 3721, 1429))]}


def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def gradient_line(bodies, dtype, T, K, exec_mode, lanes=1, reps=3, timing=False, targets=None, tile=0):
    """One model of `bodies`: median ms of a checkpointed gradient (rollout, loss, zeroed
    gradients, adjoint) and of a forward rollout, HIP events on the launch stream; with
    `timing`, also one gradient in plain execution with per-kernel events and the
    dominant kernel's roofline on the algorithmic bytes."""
    import torch
    from paper_2104_02646_amd import gsim
    stream = torch.cuda.Stream()
    ne = sum(b.ne for b in bodies)
    nel = sum(b.ne + b.nt + b.nh for b in bodies)
    np_ = sum(b.np for b in bodies)
    with torch.cuda.stream(stream):
        m = gsim.Model(bodies, dtype, max_steps=T, ckpt_every=K, tile_elems=tile)
        m.set_exec(exec_mode)
        m.set_lanes(min(lanes, len(bodies)))
        p = m.params_from_bodies()
        x0 = gsim.soa(np.concatenate([b.x0 for b in bodies])).to(dtype)
        v0 = gsim.soa(np.concatenate([b.v0 for b in bodies])).to(dtype)
        tgt = (gsim.soa(np.concatenate(targets)) if targets is not None else x0 + 0.01).to(dtype)
        xT, vT = m.empty_state()
        xb0, vb0 = m.empty_state()
        want = tuple(k for k, n in (("mu", m.ne), ("lam", m.ne), ("ktri", m.nt)) if n) + ("mass", "contact")
        g = m.zero_grads(want)

        def grad():
            m.rollout(p, x0, v0, T, out=(xT, vT), stream=stream)
            loss, xb, vb = m.loss_mse(xT, tgt, stream=stream)
            for t in g.values():
                t.zero_()
            m.rollout_backward(p, T, xb, vb, g, out=(xb0, vb0), stream=stream)

        def fwd():
            m.rollout(p, x0, v0, T, out=(xT, vT), stream=stream)

        def median_ms(f):
            f()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
            ev[0].record(stream)
            for k in range(reps):
                f()
                ev[k + 1].record(stream)
            ev[-1].synchronize()
            return float(np.median([ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]))
        gms, fms = median_ms(grad), median_ms(fwd)
        kept = m.keeps_last_segment()
        out = {"ms_per_gradient": gms, "us_per_sim_step": gms * 1e3 / T, "fwd_us_per_sim_step": fms * 1e3 / T,
               "value": nel * T / (gms * 1e-3), "forward_value": nel * T / (fms * 1e-3)}
        if timing:
            m.set_exec(gsim.EXEC_PLAIN)
            m.set_timing()
            grad()
            torch.cuda.synchronize()
            t = m.read_timing()
            m.set_timing(())
            etiles, tps = m.plan.tiles()[:2]
            kern = kernel_table(t, ne, np_, len(tps), T, K, len(etiles) >= DUAL_PAIR_MIN_TILES)
            dom = max((k for k in kern if "algorithmic_bytes_per_launch" in kern[k]), key=lambda k: kern[k]["total_ms"])
            out["kernels"] = kern
            out["roofline"] = roofline(kern[dom], dom, None)
            gb, passes = gradient_bytes(ne, np_, T, K, kept=kept)
            out["step_algorithmic"] = {"GBps": gb / (gms * 1e-3) / 1e9, "frac": gb / (gms * 1e-3) / 1e12 / 8.0,
                                       "forward_passes": passes}
    del m
    torch.cuda.synchronize()
    return out


def try_line(*a, **kw):
    from paper_2104_02646_amd import gsim
    try:
        return gradient_line(*a, **kw)
    except gsim.GsimError as e:
        return {"unavailable": str(e)}


def config_lines(W, log):
    """The other workloads: tiny cube (FP32 and FP64), 64 x 64 cloth, large blob, and
    the batch at 2048 bodies (working set beyond the 256 MB last-level cache), each as
    the two-pass graph path beside the plain one-launch-per-pass path (and the fused
    path where every body fits one workgroup's LDS; the tiny cube also with persistent
    execution, FP32)."""
    import torch
    from paper_2104_02646_amd import gsim
    out = {}
    cube = [W.tiny_cube(0).round_to(np.float32)]
    tc = {"workload": "tiny cube: 162 tets, 64 particles, 100 steps, checkpoints every 10", "unit": "us per step "
          "(fwd + checkpointed adjoint of one gradient, divided by its steps)"}
    for dt, name in ((torch.float32, "f32"), (torch.float64, "f64")):
        for ex, en in ((gsim.EXEC_GRAPH, "graph"), (gsim.EXEC_PERSIST, "persist"), (gsim.EXEC_FUSED, "fused"),
                       (gsim.EXEC_PLAIN, "plain")):
            tc["%s_%s" % (name, en)] = try_line(cube, dt, 100, 10, ex)
    out["tiny_cube"] = tc
    log("configs: tiny cube done")
    cl = [W.cloth(10).round_to(np.float32)]
    c1 = {"workload": "cloth 64x64: 7938 triangles, 11781 hinges, 400 steps, checkpoints every 20",
          "unit": "us per step; value in (triangle + hinge)-steps/s"}
    for ex, en in ((gsim.EXEC_GRAPH, "graph"), (gsim.EXEC_FUSED, "fused"), (gsim.EXEC_PLAIN, "plain")):
        c1[en] = try_line(cl, torch.float32, 400, 20, ex)
    out["cloth"] = c1
    log("configs: cloth done")
    from paper_2104_02646_amd import autotune

    def tuned(bodies, T, K, tiles, lanes, fused):
        """The autotuner's choice for this workload (set-up, outside every timing)."""
        t0 = time.perf_counter()
        m, rep = autotune.tune_model(bodies, torch.float32, T, K, reps=2, use_cache=False, tiles=tiles, lanes=lanes,
                                     fused=fused)
        del m
        torch.cuda.synchronize()
        return dict(rep["choice"], candidates_ms=rep["candidates_ms"], tune_s=time.perf_counter() - t0)
    blob = W.large_blob(30).round_to(np.float32)
    c3 = {"workload": "large blob: %d tets, %d particles, 1000 steps, checkpoints every 50" % (blob.ne, blob.np),
          "unit": "element-steps/s"}
    ch = tuned([blob], 1000, 50, (64, 128, 256, 512), (1,), False)
    c3["autotuned"] = ch
    c3["graph"] = gradient_line([blob], torch.float32, 1000, 50, gsim.EXEC_GRAPH, timing=True, tile=ch["tile_elems"])
    c3["plain"] = gradient_line([blob], torch.float32, 1000, 50, gsim.EXEC_PLAIN, tile=ch["tile_elems"])
    out["large_blob"] = c3
    log("configs: large blob done")
    big = [b.round_to(np.float32) for b in W.batch_bodies(20, 2048)]
    ch = tuned(big, 100, 10, (512,), (2, 3, 4), False)
    out["batch_2048"] = dict(gradient_line(big, torch.float32, 100, 10, gsim.EXEC_GRAPH, lanes=ch["lanes"], timing=True,
                                           tile=ch["tile_elems"]),
                             autotuned=ch,
                             workload="batch of 2048 tet bodies (%d tets, %d particles), 100 steps, checkpoints "
                                      "every 10: working set beyond the 256 MB last-level cache"
                                      % (sum(b.ne for b in big), sum(b.np for b in big)),
                             unit="element-steps/s")
    del big
    log("configs: 2048-body batch done")
    return out


def serving(n_measured, n_warm, ckpt_every, log):
    """Poisson stream (200 req/s) of tet / cloth gradient queries through the
    continuous-batching engine and through the one-query-per-launch FIFO path."""
    import torch
    from paper_2104_02646_amd import serve, workloads as W
    trace = W.serving_trace(40, n_measured + n_warm)
    bodies = [W.query_body(q) for q in trace]
    work = np.array([(b.ne + b.nt) * q.steps for q, b in zip(trace, bodies)], float)
    eng = serve.Engine(pool_bytes=8 << 30, max_live=256, max_tiles=1 << 18)
    lat, wall, _ = serve.replay_trace(trace, bodies, eng, ckpt_every=ckpt_every)
    st = eng.stats()
    del eng
    torch.cuda.synchronize()
    log("serving: engine done (%.1f s)" % wall)
    flat, fwall = serve.replay_fifo(trace, bodies, ckpt_every=ckpt_every)
    log("serving: fifo done (%.1f s)" % fwall)
    m = slice(n_warm, None)
    arr = np.array([q.arrival for q in trace])
    span = arr[-1] - arr[n_warm]

    def summary(l, w):
        return {"p50_ms": float(np.percentile(l[m], 50) * 1e3), "p99_ms": float(np.percentile(l[m], 99) * 1e3),
                "mean_ms": float(l[m].mean() * 1e3), "wall_s": w,
                "req_per_s": float(len(trace) / w), "element_steps_per_s": float(work.sum() / w)}
    # saturation: the first n_sat queries of the trace all submitted at once, so the
    # engine's slots stay full; throughput against the queries' algorithmic bytes
    n_sat = min(400, len(trace))
    eng = serve.Engine(pool_bytes=8 << 30, max_live=256, max_tiles=1 << 18)
    # the engine stores every state of a query whose whole trajectory fits 1/64 of its
    # pool (no recomputed segments): the algorithmic bytes count the passes it runs
    limit = eng.stats()["pool_free"] // 64
    k_run = [1 if serve.QueryBuffers(b, q.steps, 1).bytes() <= limit else ckpt_every
             for q, b in zip(trace[:n_sat], bodies[:n_sat])]
    slat, swall, _ = serve.replay_trace(trace[:n_sat], bodies[:n_sat], eng, ckpt_every=ckpt_every, time_scale=0.0)
    sst = eng.stats()
    del eng
    torch.cuda.synchronize()
    log("serving: saturation done (%.1f s)" % swall)
    sbytes = sum(gradient_bytes(b.ne, b.np, q.steps, k, b.nt, b.nh)[0]
                 for q, b, k in zip(trace[:n_sat], bodies[:n_sat], k_run))
    sat = {"queries": n_sat, "wall_s": swall, "req_per_s": n_sat / swall,
           "queries_storing_every_state": int(sum(k == 1 for k in k_run)),
           "element_steps_per_s": float(work[:n_sat].sum() / swall), "mean_live": sst["mean_live"],
           "ticks": sst["ticks"], "ms_per_tick": swall * 1e3 / max(sst["ticks"], 1),
           "algorithmic_GBps": sbytes / swall / 1e9, "frac_of_hbm_peak": sbytes / swall / 1e9 / HBM_PEAK_GBS}
    return {"queries": n_measured, "warmup_queries": n_warm, "arrival_rate": 200.0,
            "trace_span_s": float(span), "engine": dict(summary(lat, wall), mean_live=st["mean_live"],
                                                        ticks=st["ticks"], ms_per_tick=wall * 1e3 / max(st["ticks"], 1)),
            "one_query_per_launch_fifo": summary(flat, fwall), "saturation": sat}


def control_step(model, p, x0, v0, tgt, T, steps, stream, ne, n_signals=8):
    """The actuated step of the control tasks at the batch's scale: controller
    forward (per-step actuation rows for every tet), rollout driven by those rows,
    loss, adjoint with per-step actuation gradients, controller backward.  Also the
    two controller kernels alone (HIP events on the launch stream) against their
    algorithmic bytes: forward reads W once and writes T rows, backward reads W
    and T rows of act-bar and read-modify-writes W-bar."""
    import torch
    from paper_2104_02646_amd import gsim
    omega, dt, scale = 2 * np.pi * 4.0, 1.0 / 600.0, 0.05
    rng = np.random.default_rng(99)
    Wc = torch.as_tensor(rng.normal(0, 0.5, (n_signals, ne)), dtype=torch.float32, device="cuda")
    act = torch.empty(T, ne, dtype=torch.float32, device="cuda")
    gact = torch.zeros_like(act)
    gW = torch.zeros_like(Wc)
    g = model.zero_grads(("mu", "lam", "mass", "contact"))
    xT, vT = model.empty_state()
    xb0, vb0 = model.empty_state()

    def one():
        gsim.controller_forward(Wc, omega, dt, T, scale=scale, out=act, stream=stream)
        q = dict(p, act=act)
        model.rollout(q, x0, v0, T, out=(xT, vT), stream=stream)
        loss, xb, vb = model.loss_mse(xT, tgt, stream=stream)
        for t in g.values():
            t.zero_()
        gact.zero_()
        model.rollout_backward(q, T, xb, vb, dict(g, act=gact), out=(xb0, vb0), stream=stream)
        gW.zero_()
        gsim.controller_backward(Wc, gact, omega, dt, scale=scale, W_grad=gW, stream=stream)
    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    reps = 10
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(stream)
    for _ in range(reps):
        gsim.controller_forward(Wc, omega, dt, T, scale=scale, out=act, stream=stream)
    ev[1].record(stream)
    for _ in range(reps):
        gsim.controller_backward(Wc, gact, omega, dt, scale=scale, W_grad=gW, stream=stream)
    ev[2].record(stream)
    ev[2].synchronize()
    f_ms, b_ms = ev[0].elapsed_time(ev[1]) / reps, ev[1].elapsed_time(ev[2]) / reps
    f_bytes = 4 * (n_signals * ne + T * ne)
    b_bytes = 4 * (n_signals * ne + T * ne + 2 * n_signals * ne)
    return {"workload": "controller (%d sinusoids -> linear -> tanh) driving every tet of the batch, per-step "
                        "actuation rows and gradients" % n_signals,
            "value": ne * T / sec, "unit": "element-steps/s", "ms_per_step": sec * 1e3,
            "controller_fwd": {"avg_us": f_ms * 1e3, "bytes": f_bytes, "GBps": f_bytes / (f_ms * 1e-3) / 1e9},
            "controller_bwd": {"avg_us": b_ms * 1e3, "bytes": b_bytes, "GBps": b_bytes / (b_ms * 1e-3) / 1e9}}


def cloth_air_batch(steps, n_cloths=64, T=100, K=10):
    """The control-cloth step at batch scale: 64 free cloths (72 .. 2048 triangles,
    seeded sizes) under lift/drag, T steps forward with checkpoints, loss, adjoint
    with the initial-velocity gradient; the same batch without air for comparison.
    Rate: (triangles + hinges) x steps per second, forward + adjoint."""
    import torch
    from paper_2104_02646_amd import gsim, workloads as W
    out = {}
    for air in (True, False):
        bodies = [W.control_cloth(900 + i).round_to(np.float32) for i in range(n_cloths)]
        if not air:
            bodies = [b.with_params(air=False) for b in bodies]
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            m = gsim.Model(bodies, torch.float32, max_steps=T, ckpt_every=K)
            p = m.params_from_bodies()
            x0 = gsim.soa(np.concatenate([b.x0 for b in bodies]))
            v0 = gsim.soa(np.concatenate([b.v0 for b in bodies]))
            tgt = gsim.soa(np.concatenate([b.x0 + 0.3 for b in bodies]))
            xT, vT = m.empty_state()
            xb0, vb0 = m.empty_state()
            g = m.zero_grads(("ktri", "mass"))

            def one():
                m.rollout(p, x0, v0, T, out=(xT, vT), stream=stream)
                loss, xb, vb = m.loss_mse(xT, tgt, stream=stream)
                for t in g.values():
                    t.zero_()
                m.rollout_backward(p, T, xb, vb, g, out=(xb0, vb0), stream=stream)
            one()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                one()
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / steps
        n_el = sum(b.nt + b.nh for b in bodies)
        out["air" if air else "no_air"] = {"ms_per_step": sec * 1e3, "value": n_el * T / sec}
        out["workload"] = ("%d free cloths (%d triangles, %d hinges in all), %d steps fwd + checkpointed adjoint "
                           "(every %d), initial-velocity gradient" % (n_cloths, sum(b.nt for b in bodies),
                                                                      sum(b.nh for b in bodies), T, K))
    out["unit"] = "element-steps/s (triangles + hinges)"
    out["air_overhead"] = out["air"]["ms_per_step"] / out["no_air"]["ms_per_step"]
    return out


def rigid_batch_bench(steps, n_bodies=1024, T=400):
    """The rigid parameter-estimation step at batch scale: 1024 rigid bodies (boxes,
    cylinders, spheres of 8 .. 250 vertices) with vertex contact, T steps forward
    (one launch, every state stored), vertex loss, reverse pass (one launch) with
    mass, inertia, contact and initial-state gradients.  Each body's steps form one
    dependent chain inside one wavefront, so the launches are bound by that chain's
    latency, not by HBM (a body-step moves 104 bytes of state in FP32).  Run in FP64
    (the parity-bearing line: over 400 steps of bouncing contact some of these bodies'
    gradients are conditioned beyond FP32 state storage) and in FP32 beside it."""
    import torch
    from paper_2104_02646_amd import gsim, workloads as W
    bodies = [b.round_to(np.float32) for b in W.rigid_batch(80, n_bodies)]
    out = {}
    for tdt, name in ((torch.float64, "f64"), (torch.float32, "f32")):
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            m = gsim.RigidModel(bodies, tdt)
            p = m.params_from_bodies()
            s0 = m.initial_state()
            tgt = torch.as_tensor(np.concatenate([b.verts + b.s0[:3] + 0.2 for b in bodies]), dtype=tdt,
                                  device="cuda")
            traj = m.new_trajectory(T)
            g = m.zero_grads()

            def one():
                m.rollout(p, s0, T, traj=traj, stream=stream)
                loss, sbar = m.loss(traj[-1], tgt, stream=stream)
                for t in g.values():
                    t.zero_()
                return m.rollout_backward(p, traj, T, sbar, g, stream=stream)
            one()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                one()
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / steps
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record(stream)
            m.rollout(p, s0, T, traj=traj, stream=stream)
            ev[1].record(stream)
            loss, sbar = m.loss(traj[-1], tgt, stream=stream)
            m.rollout_backward(p, traj, T, sbar, g, stream=stream)
            ev[2].record(stream)
            ev[2].synchronize()
        nv = sum(b.nv for b in bodies)
        out[name] = {"ms_per_step": sec * 1e3, "body_steps_per_s": n_bodies * T / sec,
                     "vertex_steps_per_s": nv * T / sec, "forward_launch_ms": ev[0].elapsed_time(ev[1]),
                     "loss_and_adjoint_ms": ev[1].elapsed_time(ev[2])}
    out["workload"] = ("%d rigid bodies (%d vertices in all), %d steps forward + vertex loss + reverse pass; "
                       "f64 is the parity-bearing line" % (n_bodies, sum(b.nv for b in bodies), T))
    out["f64_over_f32_time"] = out["f64"]["ms_per_step"] / out["f32"]["ms_per_step"]
    return out


def raster_bench(reps=20, H=256, W=256):
    """The soft silhouette renderer on the cloth workload's mesh (64 x 64 particles,
    7938 triangles) seen by a perspective camera at H x W pixels: forward (projection
    + per-pixel pass) and backward (recomputed forward + per-triangle adjoint + vertex
    gather), HIP events over `reps` calls each."""
    import torch
    from paper_2104_02646_amd import gsim, workloads as W_
    b = W_.cloth(10)
    eye, tgt, up = np.array([1.0, 3.0, 4.0]), np.array([1.0, 0.6, 1.0]), np.array([0.0, 1.0, 0.0])
    fwd = (tgt - eye) / np.linalg.norm(tgt - eye)
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    Rm = np.stack([right, down, fwd])
    K = np.array([[1.1 * W, 0, W / 2], [0, 1.1 * W, H / 2], [0, 0, 1.0]])
    P = K @ np.concatenate([Rm, (-Rm @ eye)[:, None]], 1)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        r = gsim.Renderer(b.tris, b.np, H, W)
        x = gsim.soa(b.X)
        ib = torch.ones(H, W, device="cuda")
        xb = torch.zeros(3, b.np, device="cuda")
        img = r.forward(x, P, 1.0, stream=stream)
        r.backward(x, P, 1.0, ib, xb, stream=stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        for _ in range(reps):
            r.forward(x, P, 1.0, stream=stream)
        ev[1].record(stream)
        for _ in range(reps):
            r.backward(x, P, 1.0, ib, xb, stream=stream)
        ev[2].record(stream)
        ev[2].synchronize()
    return {"workload": "soft silhouette of the 64x64 cloth (%d triangles) at %dx%d" % (b.nt, H, W),
            "coverage": float(img.mean()), "forward_ms": ev[0].elapsed_time(ev[1]) / reps,
            "backward_ms": ev[1].elapsed_time(ev[2]) / reps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--bodies", type=int, default=256)
    ap.add_argument("--sim-steps", type=int, default=100)
    ap.add_argument("--ckpt-every", type=int, default=10)
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (tile size, lanes, execution, pass shapes) and use the flags below")
    ap.add_argument("--exec", choices=("fused", "graph", "plain", "persist"), default="graph")
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--items", type=int, default=1)
    ap.add_argument("--lanes", type=int, default=3, help="concurrent launch lanes of the two-pass path (1..4)")
    ap.add_argument("--tile", type=int, default=0, help="elements per element tile (0 = the library default)")
    ap.add_argument("--cpu-tets", type=int, default=15000, help="oracle sample size (tets)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--serve-queries", type=int, default=2000, help="measured queries of the serving trace (0 = skip)")
    ap.add_argument("--serve-warmup", type=int, default=200, help="warm-up queries before the measured ones")
    ap.add_argument("--no-configs", action="store_true", help="skip the tiny cube, cloth, blob and 2048-body lines")
    ap.add_argument("--no-control", action="store_true", help="skip the actuated (controller-driven) step")
    ap.add_argument("--no-cloth", action="store_true", help="skip the lift/drag cloth batch")
    ap.add_argument("--no-rigid", action="store_true", help="skip the rigid-body batch")
    ap.add_argument("--no-raster", action="store_true", help="skip the renderer")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device tensor copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (bodies would shard "
              "across GPUs with no exchange); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2104_02646_amd import autotune, gsim, workloads as W

    if args.calibrate_copy:
        n = 1 << 28  # 2^28 floats = 1 GiB
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_copy": 4 * n, "bytes_written_per_copy": 4 * n,
                          "copies": 3}), flush=True)
        return

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    T, K = args.sim_steps, args.ckpt_every
    t_gen = time.perf_counter()
    bodies = [b.round_to(np.float32) for b in W.batch_bodies(20, args.bodies)]
    targets = [W.synthetic_target(b, 7000 + i).astype(np.float32).astype(np.float64) for i, b in enumerate(bodies)]
    ne = sum(b.ne for b in bodies)
    np_ = sum(b.np for b in bodies)
    t_gen = time.perf_counter() - t_gen

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream()
    t_plan = time.perf_counter()
    tuned, t_tune = None, 0.0
    with torch.cuda.stream(stream):
        if args.no_tune:
            model = gsim.Model(bodies, torch.float32, max_steps=T, ckpt_every=K, device=dev, tile_elems=args.tile)
            exec_mode = {"fused": gsim.EXEC_FUSED, "graph": gsim.EXEC_GRAPH, "plain": gsim.EXEC_PLAIN,
                         "persist": gsim.EXEC_PERSIST}[args.exec]
            model.set_exec(exec_mode, args.block, args.items)
            model.set_lanes(args.lanes)
        else:
            t_tune = time.perf_counter()
            model, rep = autotune.tune_model(bodies, torch.float32, T, K, device=dev, stream=stream, use_cache=False)
            tuned = {"model": {k: rep[k] for k in ("choice", "ms_per_gradient", "candidates_ms")}}
        p = model.params_from_bodies()
        x0 = gsim.soa(np.concatenate([b.x0 for b in bodies]))
        v0 = gsim.soa(np.concatenate([b.v0 for b in bodies]))
        tgt = gsim.soa(np.concatenate(targets))
        xT, vT = model.empty_state()
        xb0, vb0 = model.empty_state()
        g = model.zero_grads(("mu", "lam", "mass", "contact"))
        if tuned is not None:
            shapes = autotune.tune(model, p, x0, v0, use_cache=False, stream=stream)
            tuned["pass_shapes"] = {k: v["shape"] for k, v in shapes.items()}
            t_tune = time.perf_counter() - t_tune
    stream.synchronize()
    t_plan = time.perf_counter() - t_plan - t_tune
    exec_mode, block, items = model.get_exec()
    args.exec = {gsim.EXEC_FUSED: "fused", gsim.EXEC_GRAPH: "graph", gsim.EXEC_PLAIN: "plain",
                 gsim.EXEC_PERSIST: "persist"}[exec_mode]
    args.block, args.items, args.lanes = block, items, model.get_lanes()
    kept = model.keeps_last_segment()  # the timed steps' backward takes the rollout's last segment
    tile_elems = model.plan.tile_elems or gsim.TILE_DEFAULT
    etiles_, tps_ = gsim.Plan(bodies, tile_elems=tile_elems).tiles()[:2]
    ntp = len(tps_)  # tile particles of the element tiles
    paired = len(etiles_) >= DUAL_PAIR_MIN_TILES

    def bench_step():
        model.rollout(p, x0, v0, T, out=(xT, vT), stream=stream)
        loss, xb, vb = model.loss_mse(xT, tgt, stream=stream)
        for t in g.values():
            t.zero_()
        model.rollout_backward(p, T, xb, vb, g, out=(xb0, vb0), stream=stream)
        return loss

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            bench_step()
        torch.cuda.synchronize()
        # every step bracketed by HIP events on the launch stream; value = the median
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        t0 = time.perf_counter()
        ev[0].record(stream)
        for k in range(args.steps):
            loss = bench_step()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        t_total = time.perf_counter() - t0
        step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
        sec = float(np.median(step_ms)) * 1e-3
        # forward-only rate (rollout with checkpoints): median of per-rollout HIP events
        torch.cuda.synchronize()
        evf = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        evf[0].record(stream)
        for k in range(args.steps):
            model.rollout(p, x0, v0, T, out=(xT, vT), stream=stream)
            evf[k + 1].record(stream)
        torch.cuda.synchronize()
        sec_fwd = float(np.median([evf[k].elapsed_time(evf[k + 1]) for k in range(args.steps)])) * 1e-3
        control = None if args.no_control else control_step(model, p, x0, v0, tgt, T, args.steps, stream, ne)
        # per-kernel durations: one more bench step with HIP events around every launch
        # (graph replay cannot carry them: the two-pass path is timed with plain launches)
        model.set_exec(gsim.EXEC_FUSED if args.exec == "fused" else gsim.EXEC_PLAIN)
        model.set_timing()
        bench_step()
        torch.cuda.synchronize()
        timing = model.read_timing()
        model.set_timing(())
        g_np = {k: t.detach().double().cpu().numpy() for k, t in g.items()}
        xT_np = gsim.aos(xT)
        # the other batched execution, same model and buffers
        other = gsim.EXEC_GRAPH if args.exec == "fused" else gsim.EXEC_FUSED
        alt = None
        try:
            model.set_exec(other)
            bench_step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                bench_step()
            torch.cuda.synchronize()
            alt = (time.perf_counter() - t0) / args.steps
        except gsim.GsimError as e:
            alt = str(e)

    value = ne * T / sec
    kern = kernel_table(timing, ne, np_, ntp, T, K, paired)
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    d = kern[dom]
    gbytes, fwd_passes = gradient_bytes(ne, np_, T, K, kept=kept)
    step_bw = gbytes / sec / 1e9
    traffic = measured_traffic(dom, len(bodies), T, K, tile_elems)

    result = {
        "metric": METRIC, "value": value, "unit": "element-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch of %d tet bodies (log-uniform 500-20000 tets), %d steps fwd + "
                               "checkpointed adjoint (every %d), ground contact + friction" % (len(bodies), T, K),
                   "bodies": len(bodies), "tets": ne, "particles": np_, "sim_steps": T, "ckpt_every": K,
                   "exec": args.exec, "block": args.block, "items": args.items, "lanes": args.lanes,
                   "tile_elems": tile_elems, "autotuned": tuned},
        "roofline": roofline(d, dom, traffic),
        "kernels": kern,
        "step_times_ms": {"median": float(np.median(step_ms)), "mean": float(step_ms.mean()),
                          "min": float(step_ms.min()), "max": float(step_ms.max())},
        "forward_elem_steps_per_s": ne * T / sec_fwd,
        "step_algorithmic": {"GBps": step_bw, "frac": step_bw / HBM_PEAK_GBS, "bytes_per_gradient": gbytes,
                             "forward_passes": fwd_passes, "adjoint_passes": T,
                             "bytes_per_elem_step": gbytes / (ne * T)},
        "setup_s": {"generate": t_gen, "plan_and_upload": t_plan, "autotune": t_tune},
    }
    name = {gsim.EXEC_GRAPH: "two_pass_graph", gsim.EXEC_FUSED: "fused"}[other]
    result[name] = ({"value": ne * T / alt, "ms_per_step": alt * 1e3} if isinstance(alt, float)
                    else {"unavailable": alt})

    # plain one-body-per-launch path on the same GPU
    if not args.no_plain:
        models = []
        for i, b in enumerate(bodies):
            m1 = gsim.Model([b], torch.float32, max_steps=T, ckpt_every=K, device=dev)
            p1 = m1.params_from_bodies()
            models.append((m1, p1, gsim.soa(b.x0), gsim.soa(b.v0), gsim.soa(targets[i]), m1.zero_grads(("mu", "lam", "mass", "contact"))))

        def plain_step():
            for m1, p1, a0, b0, t1, g1 in models:
                xa, va = m1.rollout(p1, a0, b0, T)
                l1, xb1, vb1 = m1.loss_mse(xa, t1)
                for t in g1.values():
                    t.zero_()
                m1.rollout_backward(p1, T, xb1, vb1, g1)
        plain_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain_step()
        torch.cuda.synchronize()
        sp = time.perf_counter() - t0
        result["plain_one_body_per_launch"] = {"value": ne * T / sp, "ms_per_step": sp * 1e3,
                                               "speedup_of_batched": sp / sec}
        del models

    # FP64 oracle on a bounded sample, and the FP32 gradient error of those bodies
    if not args.no_cpu:
        sample, tot, dt_cpu, ref, core = cpu_baseline(bodies, targets, T, args.cpu_tets)
        errs = {"x": 0.0, "mu": 0.0, "lam": 0.0, "mass": 0.0, "muf": 0.0}
        poffs = np.cumsum([0] + [b.np for b in bodies])
        eoffs = np.cumsum([0] + [b.ne for b in bodies])
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        for i in sample:
            L, gr, x_ref = ref[i]
            sl = slice(poffs[i], poffs[i + 1])
            se = slice(eoffs[i], eoffs[i + 1])
            errs["x"] = max(errs["x"], rel(xT_np[sl], x_ref))
            errs["mu"] = max(errs["mu"], rel(g_np["mu"][se], gr["mu"]))
            errs["lam"] = max(errs["lam"], rel(g_np["lam"][se], gr["lam"]))
            errs["mass"] = max(errs["mass"], rel(g_np["mass"][sl], gr["mass"]))
            if gr["contact"][3] != 0:
                errs["muf"] = max(errs["muf"], abs(g_np["contact"][i, 3] - gr["contact"][3]) / abs(gr["contact"][3]))
        result["cpu_baseline"] = dict({"value": tot * T / dt_cpu, "unit": "element-steps/s", "cores": 1,
                                       "kind": "oracle", "pinned_core": core,
                                       "sample": "bodies 0..%d of the batch (%d tets), %d steps fwd + loss + "
                                                 "adjoint, FP64, single thread pinned to one core"
                                                 % (sample[-1], tot, T)}, **host_info())
        result["parity_sample"] = {"bodies": len(sample), "max_rel_err": errs}
    result["paper_table4_right"] = PAPER_TABLE4_RIGHT
    if not args.no_configs:
        result["configs"] = config_lines(W, log)
    if control is not None:
        control["overhead_vs_unactuated_step"] = control["ms_per_step"] / (sec * 1e3)
        result["control"] = control
    if not args.no_cloth:
        result["control_cloth"] = cloth_air_batch(args.steps)
    if not args.no_rigid:
        result["rigid"] = rigid_batch_bench(args.steps)
    if not args.no_raster:
        result["raster"] = raster_bench()
    if args.serve_queries > 0:
        result["serving"] = serving(args.serve_queries, args.serve_warmup, K, log)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
