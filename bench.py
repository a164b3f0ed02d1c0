#!/usr/bin/env python3
"""Throughput of the Blahut-Arimoto iteration for the binary deletion channel at
n = 20 on one MI355X; prints one JSON line.

Workload: three instances n = 20, d in {0.64, 0.80, 0.95}, p_0 uniform, FP32
log-domain iterates (FP64 certification reported after the timed steps).  One
step = one BA iteration of all three instances: q = W^T p, D(x), the Blahut
reductions and the update, over all 2*3^20 - 2^20 nonzeros of W per instance.
The steps run as ba_step calls of --per-call iterations (50: ba_run's chunk between
FP64 certifications, whose first and last iterations carry the call's own launches)
after --warmup iterations that bring the device to its steady clocks.

metric: BA iterations per second, and W-nonzero terms per second =
iterations/s x nnz(W) x instances.  The default engine evaluates the two products
of each iteration stage by stage (BA_ENGINE_FACTORED) and never visits a nonzero,
so for it the terms/s figure is nonzero-equivalent (accounted, not visited); the
per-nonzero engine of the paper's method (BA_ENGINE_STREAM), which visits every
nonzero, is measured on the same workload and reported beside it.  The FP64 plain
iteration of one instance is reported too.

After the timed steps (outside the timed region) the same three instances are
run to the stopping rule of Section 2.3 (certified gap < 1e-6 bits, with an
iteration cap): certified bounds on C_20(d), the gap reached, the FP32-vs-FP64
difference of the bounds (FP64 iterates with the same floor, same iteration
counts) and the orbit check of Theorem 4 on the final laws.  The CPU baseline is
the oracle's FP64 certification of those final laws.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 20
DS = [0.64, 0.80, 0.95]
UNIT_EQUIV = "W-nonzero-equivalent terms/s (factored engine: nonzeros accounted, not visited)"
FUSE = 8  # the library default (positions per launch of the factored engine)


# HBM bytes per launch of each kernel of this workload's default plan (3 instances),
# from rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by a device copy's reading of the
# same counters (x2.0 and x1.0); a sweep's figure is their average over the launches
# of one ba_step call, weighted as the algorithmic bytes are.  Valid only for the
# kernel sources they were measured on (summary: profiles/factored_sweeps_n20_fp32_x3.md).
MEASURED_TRAFFIC = {
    "sources": ["paper_2604_05867_amd/csrc/ba_factored.hip", "paper_2604_05867_amd/csrc/ba_factored_common.h",
                "paper_2604_05867_amd/csrc/ba_part.h"],
    # of the sources concatenated
    "sha256": "49340f8670fce8520761f69ff22d7ed91b77b5fe0766735f3b28e6ed348187cb",
    "bytes": {"first8": 37780000, "first8_upd": 50450000, "fwd12": 51450000,
              "bwd12": 50960000, "d8": 63060000, "dfused": 88200000},
}


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for src in MEASURED_TRAFFIC["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(fuse, calls, backward):
    """The PMC traffic per launch of a sweep over ba_step calls of the given lengths
    (iterations) if the kernel sources are unchanged since it was taken, else None."""
    if MEASURED_TRAFFIC["sha256"] is None or kernel_source_sha() != MEASURED_TRAFFIC["sha256"]:
        return None
    kinds = []
    for iters in calls:
        k = call_launch_kinds(N, fuse, iters, backward)
        if k is None:
            return None
        kinds += k
    return int(sum(MEASURED_TRAFFIC["bytes"][k] for k in kinds) / len(kinds))


def call_lengths(iters, per_call):
    """iters iterations as ba_step calls of per_call (the last one shorter)."""
    return [min(per_call, iters - i) for i in range(0, iters, per_call)]


def step_calls(ctx, iters, per_call):
    for k in call_lengths(iters, per_call):
        ctx.step(k)


def time_kernel_calls(ctx, iters, per_call):
    """ba_time_kernels over the same calls: {kernel class: (ms, launches)} summed."""
    tot = {}
    for k in call_lengths(iters, per_call):
        for name, (ms, nl) in ctx.time_kernels(k).items():
            a = tot.get(name, (0.0, 0))
            tot[name] = (a[0] + ms, a[1] + nl)
    return tot


def stage_sizes(n):
    """Entries of the n+1 intermediate arrays of the factored products."""
    return [((2 << i) - 1) << (n - i) for i in range(n + 1)]


def sweep_launch_bytes(n, esz, nb, fuse, backward, fused_update=0.0):
    """Algorithmic HBM bytes of each launch of one sweep of the factored engine, in
    launch order: a launch covering positions i..i+t-1 reads its source stage once
    and writes its destination stage once; the last backward launch also reads
    H and log p (D is formed there, stored as log p + D for BA); the first forward
    launch, when it makes the previous iteration's update (a fraction fused_update of
    the iterations), reads log p + D instead of p and writes log p.  Launch sequence as in the library: fuse 2 =
    four positions per launch (forward: the last 1-4 positions two at a time;
    backward: the first n mod 4 positions two or one at a time), fuse 3 = as 2 with
    eight positions per backward launch while four remain after it, fuse 4 = as 3
    with the forward's last four positions in one launch (n >= 12), fuse 5 = as 4
    with the forward's first eight positions in one launch (n >= 12), fuse 6 = as 5
    with the backward at n = 20 as twelve positions then eight, fuse 7 = as 6 with
    the forward at n = 20 as eight positions then twelve, fuse 1 = two."""
    s = stage_sizes(n)
    steps = []
    if not backward and fuse >= 7 and n == 20:
        steps = [(0, 8), (8, 20)]
    elif not backward:
        i = 0
        last4 = fuse >= 4 and n >= 12
        while i < n:
            if fuse >= 5 and n >= 12 and i == 0:
                t = 8
            elif last4 and n - i == 4:
                t = 4
            elif fuse >= 2 and i + 4 < n and not (last4 and n - i < 8):
                t = 4
            else:
                t = 2 if (fuse and i + 2 <= n and not (last4 and n - i - 2 < 4)) else 1
            steps.append((i, i + t))
            i += t
    elif fuse >= 6 and n == 20:
        steps = [(20, 8), (8, 0)]
    else:
        top, lead = n, (n % 4 if (fuse >= 2 and n >= 4) else -1)
        while top > 0:
            if fuse >= 3 and lead >= 0 and n - top >= lead and top - 8 >= 4:
                t = 8
            elif lead >= 0 and n - top >= lead:
                t = 4
            else:
                t = 2 if (fuse and top >= 2 and not (lead >= 0 and n - top + 2 > lead)) else 1
            steps.append((top, top - t))
            top -= t
    out = [(s[a] + s[b]) * esz * nb for a, b in steps]
    if backward:
        out[-1] += 2 * (1 << n) * esz * nb
    else:
        out[0] += fused_update * (1 << n) * esz * nb
    return out


def call_launch_kinds(n, fuse, iters, backward):
    """Kinds of the launches of one sweep over a ba_step call of `iters` iterations at
    launch plan level 8, n = 20 (FP32), in order, else None: forward first8 (iteration
    0), first8_upd (iteration 1: the update by the max shift), then fwd12 (positions
    8-19) alone, its first eight positions made by the fused D launch before it;
    backward bwd12, then d8 (D with its record) in the first and last iterations and
    dfused (D, the next iteration's update and first eight forward positions) between."""
    if not (fuse >= 8 and n == 20):
        return None
    out = []
    for it in range(iters):
        if not backward:
            out += (["first8_upd" if it == 1 else "first8"] if it < 2 else []) + ["fwd12"]
        else:
            out += ["bwd12", "dfused" if 1 <= it < iters - 1 else "d8"]
    return out


def call_launch_bytes(n, esz, nb, fuse, iters, backward):
    """Algorithmic HBM bytes of every launch of one sweep over a ba_step call of
    `iters` iterations, in launch order: every launch reads its source stage once and
    writes its destination stage once; first8_upd reads log p + D instead of p and
    writes log p; a D launch (d8) reads B_8, H and log p and writes log p + D; the
    fused D launch (dfused) reads B_8, H and log p and writes log p and F_8.  Below
    level 8, sweep_launch_bytes per iteration (the first one without the update)."""
    s = stage_sizes(n)
    x = 1 << n
    kinds = call_launch_kinds(n, fuse, iters, backward)
    if kinds is None:
        out = []
        for it in range(iters):
            out += sweep_launch_bytes(n, esz, nb, fuse, backward, fused_update=1.0 if it else 0.0)
        return out
    size = {"first8": s[0] + s[8], "first8_upd": s[0] + s[8] + x, "fwd12": s[8] + s[20],
            "bwd12": s[20] + s[8], "d8": s[8] + s[0] + 2 * x, "dfused": 2 * s[8] + 3 * x}
    return [size[k] * esz * nb for k in kinds]


def cpu_baseline(logps, gpu_bounds):
    """The oracle's certify-only tier on this host: one FP64 evaluation (sweep 1
    over every row, sweep 2 over every row, then L, U, I) of the three n = 20
    instances at the given laws, with every row of the channel regenerated by the
    oracle's own subsequence generator.  This is one BA iteration's worth of work
    over the whole workload (3 x 6,972,520,226 nonzeros per sweep).  Its L and U
    are compared with the GPU's FP64 certification of the same laws."""
    import numpy as np

    import oracle.native as on
    from oracle import bdc

    on.lib()
    weights = [bdc.length_weights(N, d) for d in DS]
    t0 = time.perf_counter()
    cert = on.certify(N, weights, np.asarray(logps))
    el = time.perf_counter() - t0
    visited = cert["stats"]["nnz"] * len(DS)
    ln2 = math.log(2.0)
    diff = max(max(abs(cert["L"][i] / ln2 - gpu_bounds[0][i]), abs(cert["U"][i] / ln2 - gpu_bounds[1][i]))
               for i in range(len(DS)))
    return {"value": visited / el, "unit": "W-nonzero terms/s (visited)", "cores": on.num_threads(),
            "kind": "oracle", "iters_per_s": 1.0 / el,
            "sample": "one FP64 evaluation (both sweeps, L, U, I) of the whole workload: n=20, d in %s, at the "
                      "final laws of the stopping-rule run, every row regenerated on the host "
                      "(%d nonzeros visited per sweep), %.1f s" % (DS, visited, el),
            "max_abs_bound_diff_vs_gpu_certification_bits": diff,
            "cpu": platform.processor() or platform.machine()}


def orbit_deviation(lp, n):
    """Theorem 4 (Appendix A): the BA iterates from the uniform law are invariant
    under complement and reversal.  For g = complement and reversal: the largest
    |log p(g x) - log p(x)| (nats) over the inputs within 5 and within 30 nats of the
    maximum, and its mean under p."""
    import numpy as np
    x = np.arange(1 << n)
    cp = x ^ ((1 << n) - 1)
    rv = np.zeros_like(x)
    for i in range(n):
        rv |= ((x >> i) & 1) << (n - 1 - i)
    lp = lp - (lp.max() + np.log(np.exp(lp - lp.max()).sum()))
    p = np.exp(lp)
    out = {}
    for name, g in (("complement", cp), ("reversal", rv)):
        dev = np.abs(lp[g] - lp)
        out[name] = {"max_within_5_nats": float(np.max(dev[lp > lp.max() - 5.0])),
                     "max_within_30_nats": float(np.max(dev[lp > lp.max() - 30.0])),
                     "mean_under_p": float(p @ dev)}
    return out


def config5(cap, gap_bits, dev):
    """The workload run to the stopping rule: FP32 iterates, FP64 certification
    every 50 iterations, graph-replayed chunks, stop per instance when the
    certified gap of the current iterate is below gap_bits (Section 2.3) or at the
    cap.  Then: the same instances iterated in FP64 with the same floor for the
    same number of iterations (difference of the certified bounds), and the orbit
    check of Theorem 4 on the final laws.  Returns (block, final laws, bounds)."""
    import numpy as np
    import torch

    import paper_2604_05867_amd as ba

    s = torch.cuda.Stream(dev)
    ctx = ba.Context([N] * len(DS), DS, prec=ba.PREC_FP32_LOG, cert_every=50, device=dev, stream=s)
    ctx.set_graphs(True)
    with torch.cuda.stream(s):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_segments(ctx, gap_bits, cap, 25000, "config5", current=True)
        s.synchronize()
        el = time.perf_counter() - t0
        lo, hi = ctx.bounds()
        blo, bhi, its = ctx.best_bounds()
        lp = ctx.get_logp().cpu().numpy().reshape(len(DS), 1 << N)
    ctx.close()
    out = []
    t64 = 0.0
    for i, d in enumerate(DS):
        c = ba.Context(N, d, prec=ba.PREC_FP64, device=dev)
        c.set_floor(80.0)  # the FP32 iterates' floor: the comparison isolates the precision
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        c.step(its[i])
        torch.cuda.synchronize()
        t64 += time.perf_counter() - t1
        lo64, hi64 = c.bounds()
        lp64 = c.get_logp().cpu().numpy()
        c.close()
        out.append({"d": d, "iterations": its[i], "converged": hi[i] - lo[i] < gap_bits,
                    "certified_lower_bits": lo[i], "certified_upper_bits": hi[i], "gap_bits": hi[i] - lo[i],
                    "best_lower_bits": blo[i], "best_upper_bits": bhi[i],
                    "fp64_same_iterations": {"certified_lower_bits": lo64[0], "certified_upper_bits": hi64[0],
                                             "abs_dL_bits": abs(lo64[0] - lo[i]),
                                             "abs_dU_bits": abs(hi64[0] - hi[i])},
                    "orbit_abs_dlogp_nats": orbit_deviation(lp[i], N),
                    "orbit_abs_dlogp_nats_fp64_iterate": orbit_deviation(lp64, N)})
        print("config5: d=%.2f  %d iterations  [%.9f, %.9f] bits  |FP32-FP64| = %.1e / %.1e" % (
            d, its[i], lo[i], hi[i], abs(lo64[0] - lo[i]), abs(hi64[0] - hi[i])), file=sys.stderr, flush=True)
    block = {"gap_bits": gap_bits, "cap": cap, "stop_rule": "certified gap of the current iterate (Section 2.3)",
             "seconds_fp32_batched": el, "seconds_fp64_same_iterations": t64,
             "fp64_floor_nats": 80.0,
             "instances": out}
    return block, lp, (lo, hi)


def run_segments(ctx, gap_bits, cap, seg, tag, current=False):
    """ba_run in segments of `seg` iterations (continuing the same run), printing
    progress after each; returns when every instance meets gap_bits (by its best
    bounds, or with current=True by the last certification of its current
    iterate) or after cap."""
    import numpy as np
    done = 0
    while done < cap:
        k = min(seg, cap - done)
        ctx.run(gap_bits, k)
        done += k
        if current:
            lo, hi = ctx.bounds()
        else:
            lo, hi, _ = ctx.best_bounds()
        left = int(np.sum(np.array(hi) - np.array(lo) >= gap_bits))
        print("%s: %d iterations, %d instances above the gap" % (tag, done, left), file=sys.stderr, flush=True)
        if left == 0:
            break
    return done


def config3_groups(steps, warmup, per_call):
    """The iteration of each group of config 3 on its own: 32 instances of one length
    n in {10, 12, 14, 16}, d = linspace(0.64, 0.96, 32), FP32 iterates, the default
    plan (n <= 11 as one persistent launch per call); one JSON line per group with
    its sustained time per iteration (calls of per_call iterations after warmup)."""
    import numpy as np
    import torch

    import paper_2604_05867_amd as ba
    ds = [float(d) for d in np.linspace(0.64, 0.96, 32)]
    for n in (10, 12, 14, 16):
        c = ba.Context([n] * 32, ds, prec=ba.PREC_FP32_LOG, engine=ba.ENGINE_FACTORED, cert_every=per_call)
        step_calls(c, warmup, per_call)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step_calls(c, steps, per_call)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        kt = time_kernel_calls(c, steps, per_call)
        c.close()
        print(json.dumps({"group": "n=%d x 32 instances, FP32, default plan" % n, "n": n, "instances": 32,
                          "steps": steps, "ms_per_step": el / steps * 1e3, "iters_per_s": steps / el,
                          "kernel_ms_per_step": {k: round(v[0] / steps, 4) for k, v in kt.items()},
                          "launches_per_step": {k: v[1] / steps for k, v in kt.items()}}), flush=True)


def config3(cap, gap_bits, plain_limit_s, plain_graphs=False, symmetric=False, plain_floor=None):
    """Batched FP32 (one graph, 128 instances) against plain FP64 one instance at a
    time, both to a certified gap < gap_bits or the iteration cap.  Prints one JSON
    line with both wall times and the speedup at equal certified gap.  plain_floor
    (nats): floor of the plain FP64 iterates' log p (the FP32 iterates' 80 makes the
    two sides iterate the same floored map; None keeps the FP64 default, 700)."""
    import numpy as np
    import torch

    import bdc_inputs as inp
    import paper_2604_05867_amd as ba

    ns, ds = [], []
    for n in (10, 12, 14, 16):
        for d in inp.d_grid():
            ns.append(n)
            ds.append(float(d))
    s = torch.cuda.Stream()
    ctx = ba.Context(ns, ds, prec=ba.PREC_FP32_LOG, engine=ba.ENGINE_FACTORED, cert_every=50, stream=s)
    ctx.set_graphs(True)
    ctx.set_stop_rule(ba.STOP_BEST)
    if symmetric:  # p0 uniform: every iterate is complement-invariant (both sides then use it)
        ctx.set_symmetry(True)
    with torch.cuda.stream(s):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_segments(ctx, gap_bits, cap, 25000, "config3 batched")
        s.synchronize()
        t_batch = time.perf_counter() - t0
        lo_b, hi_b, it_b = ctx.best_bounds()
    ctx.close()
    print("config3: batched %.2f s" % t_batch, file=sys.stderr, flush=True)
    # plain FP64, one instance after another, each to the gap the batched run reached
    t_plain = 0.0
    plain = []
    t_start = time.perf_counter()
    # visit the instances d-major so that any prefix mixes all lengths n evenly
    order = sorted(range(len(ns)), key=lambda j: (ds[j], ns[j]))
    for count_done, i in enumerate(order):
        n, d = ns[i], ds[i]
        if time.perf_counter() - t_start > plain_limit_s:
            break
        target = max(gap_bits, hi_b[i] - lo_b[i])
        ps = torch.cuda.Stream() if plain_graphs else torch.cuda.current_stream()
        c = ba.Context(n, d, prec=ba.PREC_FP64, engine=ba.ENGINE_FACTORED, stream=ps)
        c.set_stop_rule(ba.STOP_BEST)
        if plain_floor is not None:
            c.set_floor(plain_floor)
        if symmetric:
            c.set_symmetry(True)
        c.set_graphs(plain_graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(ps):
            c.run(target * (1 + 1e-9), cap)
        torch.cuda.synchronize()
        ti = time.perf_counter() - t0
        t_plain += ti
        lo, hi, it = c.best_bounds()
        plain.append({"i": i, "n": n, "d": d, "iters": it[0], "L": lo[0], "U": hi[0], "t_s": ti,
                      "reached_batched_gap": hi[0] - lo[0] <= target * (1 + 1e-9)})
        c.close()
        print("config3: plain %d/%d n=%d d=%.3f iters=%d gap=%.2e" % (count_done + 1, len(ns), n, d, it[0],
                                                                      hi[0] - lo[0]),
              file=sys.stderr, flush=True)
    m = len(plain)
    # batched time for the same instances is not separable; scale by the instance share
    # (the timed prefix mixes all lengths, so the share is a fair estimate)
    share = m / len(ns)
    out = {
        "metric": "batched FP32 vs plain FP64 speedup at equal certified gap",
        "stop_rule": "best certified bounds so far", "plain_graphs": plain_graphs,
        "floor_nats": {"batched_fp32": 80.0, "plain_fp64": plain_floor if plain_floor is not None else 700.0},
        "kernels": ("factored, default launch plan, complement-symmetric (both sides)" if symmetric
                    else "factored, default launch plan (both sides)"),
        "gap_bits": gap_bits, "cap": cap, "instances": len(ns), "plain_instances_timed": m,
        "t_batched_s": t_batch, "t_plain_s_timed": t_plain,
        "speedup": (t_plain / share) / t_batch if m else None,
        "speedup_is_extrapolated": m < len(ns),
        "batched": [{"n": n, "d": d, "iters": it, "L": l, "U": h} for n, d, it, l, h in zip(ns, ds, it_b, lo_b, hi_b)],
        "plain": plain,
        "max_abs_L_diff_bits": max((abs(p["L"] - lo_b[p["i"]]) for p in plain), default=None),
        "max_abs_U_diff_bits": max((abs(p["U"] - hi_b[p["i"]]) for p in plain), default=None),
        "converged_batched": int(np.sum(np.array(hi_b) - np.array(lo_b) < gap_bits)),
        "plain_reached_batched_gap": int(sum(1 for p in plain if p["reached_batched_gap"])),
    }
    print(json.dumps(out))


def step_compare(cap, gap_bits, etas):
    """Iterations and time to a certified gap with the update step eta (1 = BA) on a
    batch of slow instances (FP32 iterates, one graph-replayed context per eta)."""
    import torch

    import paper_2604_05867_amd as ba

    ns, ds = [], []
    for n in (10, 12, 14, 16):
        for d in (0.64, 0.80, 0.96):
            ns.append(n)
            ds.append(d)
    res = {}
    for eta in etas:
        s = torch.cuda.Stream()
        ctx = ba.Context(ns, ds, prec=ba.PREC_FP32_LOG, engine=ba.ENGINE_FACTORED, cert_every=50, stream=s)
        ctx.set_graphs(True)
        ctx.set_stop_rule(ba.STOP_BEST)
        ctx.set_step(eta)
        with torch.cuda.stream(s):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run_segments(ctx, gap_bits, cap, 25000, "step %.2f" % eta)
            s.synchronize()
            el = time.perf_counter() - t0
            lo, hi, its = ctx.best_bounds()
        ctx.close()
        res[str(eta)] = {"seconds": el, "iters": its, "gap_bits": [h - l for l, h in zip(lo, hi)],
                         "lower_bits": lo, "converged": int(sum(1 for l, h in zip(lo, hi) if h - l < gap_bits))}
    print(json.dumps({"metric": "iterations to a certified gap vs update step", "gap_bits": gap_bits, "cap": cap,
                      "instances": [{"n": n, "d": d} for n, d in zip(ns, ds)], "results": res}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--per-call", type=int, default=50,
                    help="iterations per ba_step call (ba_run's chunk between FP64 certifications)")
    ap.add_argument("--stream-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--no-config5", action="store_true",
                    help="skip the stopping-rule run of the workload (and the CPU baseline on its laws)")
    ap.add_argument("--config5-cap", type=int, default=200000)
    ap.add_argument("--config3-groups", action="store_true",
                    help="the iteration of each config-3 group (32 instances of one n) on its own")
    ap.add_argument("--config3", action="store_true",
                    help="batched FP32 vs plain FP64 at equal certified gap (several minutes)")
    ap.add_argument("--config3-symmetric", action="store_true",
                    help="config 3 with the complement-symmetric kernels on both sides")
    ap.add_argument("--cap", type=int, default=200000)
    ap.add_argument("--gap", type=float, default=1e-6)
    ap.add_argument("--plain-limit-s", type=float, default=600.0)
    ap.add_argument("--step-compare", action="store_true",
                    help="iterations to the gap for update steps 1, 1.5, 2 (several minutes)")
    ap.add_argument("--plain-floor", type=float, default=80.0,
                    help="config3: floor (nats) of the plain FP64 iterates; <= 0 keeps the FP64 default (700)")
    ap.add_argument("--plain-graphs", action="store_true",
                    help="config3: replay the plain FP64 runs as graphs too")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="one 256 MiB device-to-device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 26, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4}))
        return
    if args.config3_groups:
        config3_groups(args.steps, args.warmup, max(1, args.per_call))
        return
    if args.config3:
        config3(args.cap, args.gap, args.plain_limit_s, args.plain_graphs, args.config3_symmetric,
                None if args.plain_floor <= 0 else args.plain_floor)
        return
    if args.step_compare:
        step_compare(args.cap, args.gap, (1.0, 1.5, 2.0))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the BA instances of this workload fit one MI355X "
              "(multi-GPU sharding is described in DESIGN.md, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2604_05867_amd as ba

    dev = torch.device("cuda:0")
    nnz = ba.nnz(N)
    nb = len(DS)
    ctx = ba.Context([N] * nb, DS, prec=ba.PREC_FP32_LOG, engine=ba.ENGINE_FACTORED, cert_every=50,
                     device=dev)
    # every step is one BA iteration; they run as ba_step calls of per_call iterations
    # (ba_run's chunk between FP64 certifications), the warm-up long enough for the
    # device to reach its steady clocks
    pc = max(1, args.per_call)
    print("bench: warmup %d" % args.warmup, file=sys.stderr, flush=True)
    step_calls(ctx, args.warmup, pc)
    torch.cuda.synchronize()
    print("bench: timing %d steps" % args.steps, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    step_calls(ctx, args.steps, pc)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = el / args.steps * 1e3
    iters_s = args.steps / el
    value = iters_s * nnz * nb

    # per-kernel-class device time (HIP events on the bound stream) over the same calls
    kt = time_kernel_calls(ctx, args.steps, pc)
    dom = max(("sweep1", "sweep2"), key=lambda k: kt[k][0])
    dom_ms, dom_launches = kt[dom]
    per_launch_ms = dom_ms / max(dom_launches, 1)
    per_launch = []
    for k in call_lengths(args.steps, pc):
        per_launch += call_launch_bytes(N, 4, nb, FUSE, k, backward=(dom == "sweep2"))
    assert len(per_launch) == dom_launches, (len(per_launch), dom_launches)
    bytes_launch = sum(per_launch) / len(per_launch)
    achieved = bytes_launch / (per_launch_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                "frac": round(achieved / 8000.0, 4),
                "traffic": measured_traffic(FUSE, call_lengths(args.steps, pc), dom == "sweep2"),
                "kernel": ("forward sweep (k_fwd_first8, k_fwd_stage12)" if dom == "sweep1"
                           else "backward sweep (k_bwd_stage12, k_bwd_stage8_p with D and the next "
                                "iteration's update and first eight forward positions)"),
                "bytes_per_launch": int(bytes_launch), "avg_launch_us": round(per_launch_ms * 1e3, 2)}

    lo, hi = ctx.bounds()
    cert = {"lower_bits": lo, "upper_bits": hi, "gap_bits": [h - l for l, h in zip(lo, hi)],
            "iterations": args.warmup + 2 * args.steps}
    kernel_ms = {k: round(v[0] / args.steps, 4) for k, v in kt.items()}
    ctx.close()

    extra = {}
    # the same workload with the complement-symmetric kernels (valid from p0 uniform)
    print("bench: symmetric kernels", file=sys.stderr, flush=True)
    csym = ba.Context([N] * nb, DS, prec=ba.PREC_FP32_LOG, engine=ba.ENGINE_FACTORED, cert_every=50, device=dev)
    csym.set_symmetry(True)
    step_calls(csym, args.warmup, pc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_calls(csym, args.steps, pc)
    torch.cuda.synchronize()
    esym = time.perf_counter() - t0
    ktsym = time_kernel_calls(csym, args.steps, pc)
    lo_s, hi_s = csym.bounds()
    extra["symmetric"] = {"value": args.steps / esym * nnz * nb, "unit": UNIT_EQUIV,
                          "iters_per_s": args.steps / esym, "ms_per_step": esym / args.steps * 1e3,
                          "kernel_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in ktsym.items()},
                          "certified_lower_bits": lo_s, "certified_upper_bits": hi_s}
    csym.close()
    if not args.no_stream and args.stream_steps > 0:
        print("bench: stream engine", file=sys.stderr, flush=True)
        cs = ba.Context([N] * nb, DS, prec=ba.PREC_FP32_LOG, engine=ba.ENGINE_STREAM, device=dev)
        cs.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cs.step(args.stream_steps)
        torch.cuda.synchronize()
        es = time.perf_counter() - t0
        kts = cs.time_kernels(1)
        extra["stream_engine"] = {"value": args.stream_steps / es * nnz * nb, "unit": "W-nonzero terms/s (visited)",
                                  "iters_per_s": args.stream_steps / es,
                                  "ms_per_step": es / args.stream_steps * 1e3,
                                  "kernel_ms_per_step": {k: round(v[0], 3) for k, v in kts.items()}}
        cs.close()
        # the same engine with sweep 1 over complement/reversal orbits (Algorithm 7;
        # valid from the uniform start by Theorem 4)
        print("bench: stream engine, orbit-reduced sweep 1", file=sys.stderr, flush=True)
        co = ba.Context([N] * nb, DS, prec=ba.PREC_FP32_LOG, engine=ba.ENGINE_STREAM, device=dev)
        co.set_symmetry(2)
        co.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        co.step(args.stream_steps)
        torch.cuda.synchronize()
        eo = time.perf_counter() - t0
        kto = co.time_kernels(1)
        extra["stream_engine_orbits"] = {"iters_per_s": args.stream_steps / eo,
                                         "ms_per_step": eo / args.stream_steps * 1e3,
                                         "kernel_ms_per_step": {k: round(v[0], 3) for k, v in kto.items()}}
        co.close()
    if not args.no_stream and args.stream_steps > 0:
        # sweep 1 in pull form (supersequence enumeration), sweep 2 as the stream engine
        print("bench: pull engine", file=sys.stderr, flush=True)
        cp = ba.Context([N] * nb, DS, prec=ba.PREC_FP32_LOG, engine=ba.ENGINE_PULL, device=dev)
        cp.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cp.step(1)
        torch.cuda.synchronize()
        ep = time.perf_counter() - t0
        ktp = cp.time_kernels(1)
        extra["pull_engine"] = {"value": nnz * nb / ep, "unit": "W-nonzero terms/s (visited; sweep 1 in pull form)",
                                "ms_per_step": ep * 1e3,
                                "kernel_ms_per_step": {k: round(v[0], 3) for k, v in ktp.items()}}
        cp.close()
    print("bench: fp64 plain", file=sys.stderr, flush=True)
    c64 = ba.Context(N, 0.80, prec=ba.PREC_FP64, engine=ba.ENGINE_FACTORED, device=dev)
    step_calls(c64, max(2, args.warmup // 5), pc)
    torch.cuda.synchronize()
    k64 = max(5, args.steps // 5)
    t0 = time.perf_counter()
    step_calls(c64, k64, pc)
    torch.cuda.synchronize()
    e64 = time.perf_counter() - t0
    extra["fp64_single"] = {"iters_per_s": k64 / e64, "value": k64 / e64 * nnz, "unit": UNIT_EQUIV,
                            "ms_per_step": e64 / k64 * 1e3}
    c64.close()

    cpu = None
    if not args.no_config5:
        print("bench: config5 (stopping rule, cap %d)" % args.config5_cap, file=sys.stderr, flush=True)
        c5, c5_lp, c5_bounds = config5(args.config5_cap, 1e-6, dev)
        extra["config5"] = c5
        if not args.no_cpu_baseline:
            print("bench: cpu baseline (oracle certification of the final laws)", file=sys.stderr, flush=True)
            cpu = cpu_baseline(c5_lp, c5_bounds)

    line = {
        "metric": "W-nonzero terms/s and BA iters/s at n=20",
        "value": value,
        "unit": UNIT_EQUIV,
        "iters_per_s": iters_s,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "BA iteration, binary deletion channel n=20, d in {0.64,0.80,0.95} "
                               "(3 instances), p0 uniform, FP32 log-domain iterates, factored engine",
                   "n": N, "d": DS, "instances": nb, "nnz_per_instance": nnz, "iterations_per_call": pc},
        "kernel_ms_per_step": kernel_ms,
        "roofline": roofline,
        "certified": cert,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    if "stream_engine" in extra:
        line["visited_terms_per_s_stream_engine"] = extra["stream_engine"]["value"]
    print(json.dumps(line))


if __name__ == "__main__":
    main()
