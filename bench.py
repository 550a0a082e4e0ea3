#!/usr/bin/env python3
"""Benchmark of the strip unpacking + three-threshold clustering path on one MI355X.

Headline step: one fused, persistent launch (sc_process_events) over a batch of 64 synthetic
full-detector events (440 FEDs x 96 channels x 256 strips each; per-event occupancy log-uniform in
[0.5%, 5%]), in the batched workload's stated form: tile shape and order chosen by the library's
autotuner on the batch, the launch replayed as a captured hipGraph; inputs resident in HBM before
the timed region, outputs written to HBM. Beside it:
  * the same batch launched eagerly, and eagerly with the caches (L2 and the Infinity Cache)
    flushed by a 512 MiB write before every launch;
  * measured read-stream and copy bandwidth of the box;
  * the plain per-event GPU path (sc_unpack then sc_cluster) and the fused kernel one event at a
    time, for the 50-FED and the full-detector single-event workloads (20 events each);
  * the 256-event stress batch (6% occupancy, heavy width tail), first with output capacities
    sized for the 64-event batch (it overflows), then again with the needed capacities;
  * the serving sweep (Poisson arrivals at 20-120% of batched capacity);
  * the oracle timed on host cores: one process, and one process per core of the box's share.

Prints one JSON line. ``--gpus`` above 1 is refused: the path runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import re
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import fedgen  # noqa: E402

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_kernel_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2101_11489_amd", "csrc", "sc_kernels.hip")
STAGE_BYTES_SMALL = 6656   # the tuning's default LDS stage (sc_tuning.stage_bytes)
STAGE_SLACK = 16           # a stage of S bytes holds FEDs of up to S - 16 bytes; larger ones
                           # are read from global memory


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(events, counts, n_fed):
    """Bytes a launch must move at least once: ZS input and FED offsets, cluster records and
    member ADCs out, and the calibration of strips holding a digi in at least one event of the
    launch (4 B noise + 1 bit bad flag per strip, 4 B gain per APV)."""
    b = 0.0
    touched = np.zeros(n_fed * 96 * 256, dtype=bool)
    for ev, (ncl, nadc) in zip(events, counts):
        b += ev.zs.size + 8 * (n_fed + 1) + 16 * ncl + 2 * nadc
        touched |= ev.dense > 0
    n_strips = int(touched.sum())
    n_apv = int(touched.reshape(-1, 128).any(axis=1).sum())
    b += n_strips * (4 + 1 / 8) + 4 * n_apv
    return b


def kernel_sha():
    """sha256[:16] of the kernel source's code: comments and white space removed, so that a
    change of comments alone keeps committed counter runs valid."""
    text = open(KERNEL_SRC).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    text = re.sub(r"\s+", "", text)
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def load_traffic(workload, tuning):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken on the
    current kernel source, this workload and this tuning; else None."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha():
        return None
    key = [tuning[k] for k in ("chunk_digis", "tile_waves", "tiles_per_cu", "fed_major")]
    for ent in t.get("entries", []):
        if (ent.get("workload") == workload and ent.get("tuning") == key and
                ent.get("stage_bytes", STAGE_BYTES_SMALL) == tuning.get("stage_bytes", STAGE_BYTES_SMALL)):
            return ent.get("hbm_bytes_per_launch")
    return None


def host_cpu():
    """The host CPU as /proc/cpuinfo names it: model name, family / model / stepping, clock."""
    fields = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                if fields:
                    break
                continue
            k, v = (x.strip() for x in line.split(":", 1))
            if k in ("model name", "cpu family", "model", "stepping", "cpu MHz") and k not in fields:
                fields[k] = v
    except OSError:
        pass
    name = fields.get("model name", "unknown")
    extra = ", ".join(f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping", "cpu MHz")
                      if k in fields)
    return f"{name} ({extra})" if extra else name


# ---- the oracle on host cores -----------------------------------------------------------------
_CPU_JOB = {}


def _oracle_worker(args):
    """Runs the oracle over events start, start+step, ... (cycling) for `seconds`; returns
    (events done, seconds)."""
    start, step, seconds = args
    import oracle
    events, cal, n_fed = _CPU_JOB["events"], _CPU_JOB["cal"], _CPU_JOB["n_fed"]
    scratch = np.empty(n_fed * 96 * 256, np.uint8)
    cl = np.empty(4_000_000, dtype=oracle.CLUSTER_DTYPE)
    adc = np.empty(8_000_000, dtype=np.uint16)
    done, k = 0, start
    t0 = time.perf_counter()
    while True:
        e = events[k % len(events)]
        oracle.process_event_raw(e.zs, e.fed_offset, cal.noise, cal.gain, cal.bad, scratch, cl, adc)
        done += 1
        k += step
        el = time.perf_counter() - t0
        if el >= seconds:
            return done, el


def cpu_baseline(events, cal, n_fed, seconds, procs, geo):
    """The oracle (single-threaded C) on the batch's events: in this process, then in `procs`
    forked processes at once (one event stream each, nothing shared). Runs before the GPU is
    touched. Also returns the oracle's clusters and hits of the first and last event, which the
    GPU results are checked against."""
    import oracle
    from oracle.hits import cluster_hits
    from oracle.nested import NestedRunner
    refs = {}
    for i in (0, len(events) - 1):
        r = oracle.process_event(events[i].zs, events[i].fed_offset, cal.noise, cal.gain, cal.bad)
        refs[i] = (r.cl, r.adc, cluster_hits(r.cl, geo))
    cm = geo.channel_module.astype(np.int64)
    joins = np.zeros(cm.size, np.uint8)
    joins[1:] = (cm[1:] == cm[:-1]) & (np.arange(1, cm.size) % 96 != 0)
    rm = oracle.process_event(events[0].zs, events[0].fed_offset, cal.noise, cal.gain, cal.bad,
                              joins=joins)
    mod_ref = (rm.cl, rm.adc)
    _CPU_JOB.update(events=events, cal=cal, n_fed=n_fed)
    done1, s1 = _oracle_worker((0, 1, seconds))
    ctx = mp.get_context("fork")
    with ctx.Pool(procs) as pool:
        res = pool.map(_oracle_worker, [(i, procs, seconds) for i in range(procs)])
    agg = sum(d for d, _ in res) / max(s for _, s in res)
    # nested parallelism (paper §3): N events in flight x M FED ranges each, N x M = procs threads
    nested = []
    for n_out, n_in in ((procs, 1), (max(1, procs // 4), 4), (1, procs)):
        d, secs, lat = NestedRunner(events, cal, n_out, n_in).run(seconds / 2)
        nested.append({"events_in_flight": n_out, "fed_ranges_per_event": n_in,
                       "threads": n_out * n_in, "events_per_s": d / secs,
                       "latency_ms_p50": 1e3 * float(np.median(lat)) if lat else None})
    return refs, mod_ref, {
        "value": agg, "unit": "events/s", "cores": procs, "kind": "oracle",
        "sample": f"the batch's {len(events)} events cycled for {seconds:.0f} s by each of {procs} "
                  f"single-threaded oracle processes (one per core of the box's share; "
                  f"{sum(d for d, _ in res)} events in total)",
        "single_core_value": done1 / s1,
        "single_core_sample": f"{done1} events in {s1:.1f} s, one process",
        "cpu_model": host_cpu(), "host_cpus_visible": os.cpu_count(),
        "nested": nested,
        "nested_sample": f"the batch's events cycled for {seconds / 2:.0f} s per split, each "
                         "event's 440 FEDs cut into M ranges run at once, N events in flight",
    }


# ---- GPU measurements ---------------------------------------------------------------------------
def time_steps(ctx, batch, steps, warmup, stream, torch, graph, flush=None):
    """K timed synchronous calls of the prepared batch (after W untimed ones). Returns wall time,
    per-step latencies and the mean of the library's HIP-event kernel times (None when the
    launch did not record them). flush: a tensor written (on the launch stream) before every
    call, to empty the caches."""
    ctx.tuning = {"use_graph": 1 if graph else 0}
    for _ in range(warmup):
        ctx.process_batch(batch)
    torch.cuda.synchronize()
    st0 = ctx.stats()
    step_ms = []
    kern = []
    with torch.cuda.stream(stream):
        t_start = time.perf_counter()
        for k in range(steps):
            if flush is not None:
                flush.fill_(k & 0xff)
                torch.cuda.synchronize()
            ts = time.perf_counter()
            ctx.process_batch(batch)
            step_ms.append((time.perf_counter() - ts) * 1e3)
            if flush is not None:
                kern.append(ctx.stats()["last_kernel_ms"])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
    st1 = ctx.stats()
    n_timed = st1["kernels_timed"] - st0["kernels_timed"]
    kern_ms = None
    if flush is not None:
        kern_ms = statistics.mean(kern) if all(k > 0 for k in kern) else None
    elif n_timed == steps:
        kern_ms = (st1["kernel_ms_total"] - st0["kernel_ms_total"]) / n_timed
    return {"elapsed_s": elapsed if flush is None else sum(step_ms) / 1e3, "step_ms": step_ms,
            "kernel_ms": kern_ms}


def stream_probe(torch, mib=2048, reps=10):
    """Measured read-stream (a reduction over `mib` MiB) and copy bandwidth, GB/s."""
    n = (mib << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    out = {}
    for name, fn, moved in (("read_stream_gbs", lambda: x.sum(), n * 4),
                            ("copy_gbs", lambda: y.copy_(x), 2 * n * 4)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = moved * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    out["bytes"] = mib << 20
    return out


def plain_line(sc, torch, stream, cfg_id, n_events, workers, tuning):
    """The plain per-event path and the fused kernel per event and per batch on one workload. The
    two paths are checked against each other here; their oracle parity on this workload is the
    GPU tests' (config 0 and full-size parity suites)."""
    cfg = fedgen.CONFIGS[cfg_id]
    cal = fedgen.make_calibration(cfg)
    evs = fedgen.make_events(cfg, cal, range(n_events), workers=workers)
    ctx = sc.Context(cal.noise, cal.gain, cal.bad, device=0, stream=stream)
    ctx.tuning = {k: tuning[k] for k in ("chunk_digis", "tile_waves", "tiles_per_cu", "fed_major")}
    ctx.tuning = {"use_graph": 0}
    d = [sc.Event(e.zs, e.fed_offset).to_device() for e in evs]
    o = [ctx.output(*sc.safe_caps(x)) for x in d]
    dense = ctx.dense_buffer()
    for x, y in zip(d[:2], o[:2]):   # warm-up of both paths
        ctx.unpack(x, dense)
        ctx.cluster(dense, y)
        ctx.process_events([x], [y])
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        tp = time.perf_counter()
        pk = []
        for x, y in zip(d, o):
            ctx.unpack(x, dense)
            ku = ctx.stats()["last_kernel_ms"]
            ctx.cluster(dense, y)
            pk.append(ku + ctx.stats()["last_kernel_ms"])
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - tp
        plain_res = [y.to_numpy()[:2] for y in o]
        tf = time.perf_counter()
        fk = []
        for x, y in zip(d, o):
            ctx.process_events([x], [y])
            fk.append(ctx.stats()["last_kernel_ms"])
        torch.cuda.synchronize()
        single_s = time.perf_counter() - tf
        same = all(np.array_equal(a[0], y.to_numpy()[0]) and np.array_equal(a[1], y.to_numpy()[1])
                   for a, y in zip(plain_res, o))
        ctx.process_events(d, o)
        tb = time.perf_counter()
        bk = []
        for _ in range(5):
            ctx.process_events(d, o)
            bk.append(ctx.stats()["last_kernel_ms"])
        torch.cuda.synchronize()
        batch_s = (time.perf_counter() - tb) / 5
    b1 = algorithmic_bytes(evs, [(y.n_cl, y.n_adc) for y in o], cfg.n_fed)
    ctx.close()
    return {
        "workload": f"{cfg.name}: {n_events} events of {cfg.n_fed} FEDs at "
                    f"{cfg.occ * 100:.1f}% occupancy",
        "plain_unpack_then_cluster_events_per_s": n_events / plain_s,
        "plain_kernel_ms_per_event": statistics.mean(pk),
        "fused_one_event_per_launch_events_per_s": n_events / single_s,
        "fused_one_event_kernel_ms": statistics.mean(fk),
        "fused_one_event_hbm_frac": (b1 / n_events) / (statistics.mean(fk) * 1e-3) / 1e9
                                    / HBM_PEAK_GBS,
        f"fused_batch_of_{n_events}_events_per_s": n_events / batch_s,
        f"fused_batch_of_{n_events}_kernel_ms": statistics.mean(bk),
        f"fused_batch_of_{n_events}_hbm_frac": b1 / (statistics.mean(bk) * 1e-3) / 1e9
                                               / HBM_PEAK_GBS,
        "cross_check": ("plain and fused paths bit-identical on every event" if same
                        else "MISMATCH"),
    }


def ingest_line(sc, torch, ctx, events, outs, batch, reps):
    """Events/s with host-resident inputs, the host link included: sc_process_pipelined over
    reps x the batch's events (page-locked, then pageable inputs), beside the same batches one
    sc_process_events call at a time (transfer, then compute) and the measured link rate."""
    pageable = [sc.Event(e.zs, e.fed_offset) for e in events]
    pinned = sc.pack_pinned(pageable)             # back to back, as in a readout ring
    scattered = [e.to_pinned() for e in pageable]  # one page-locked buffer per event
    n = len(events)
    zs_bytes = sum(int(e.zs.size) + 8 * (len(e.fed_offset)) for e in events)
    out_all = outs * reps

    def timed(fn, k=3):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(k):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    t_pin = timed(lambda: ctx.process_pipelined(pinned * reps, out_all, batch))
    t_scat = timed(lambda: ctx.process_pipelined(scattered * reps, out_all, batch))
    t_page = timed(lambda: ctx.process_pipelined(pageable * reps, out_all, batch))
    t_serial = timed(lambda: [ctx.process_events(pinned, outs) for _ in range(reps)])
    # the link alone: the same bytes, page-locked host to device, one copy
    src = torch.empty(zs_bytes, dtype=torch.uint8, pin_memory=True)
    dst = torch.empty(zs_bytes, dtype=torch.uint8, device="cuda")
    t_link = timed(lambda: [dst.copy_(src, non_blocking=True) for _ in range(reps)])
    ev_total = n * reps
    return {
        "workload": f"{ev_total} full-detector events ({reps} x the batch's {n}) from host memory "
                    f"in batches of {batch}, device outputs; pinned: the events back to back in "
                    "one page-locked buffer; scattered: one page-locked buffer per event",
        "pipelined_pinned_events_per_s": ev_total / t_pin,
        "pipelined_pinned_scattered_events_per_s": ev_total / t_scat,
        "pipelined_pageable_events_per_s": ev_total / t_page,
        "serial_pinned_events_per_s": ev_total / t_serial,
        "link_h2d_gbs": reps * zs_bytes / t_link / 1e9,
        "link_bound_events_per_s": ev_total / t_link,
        "host_bytes_per_event": zs_bytes / n,
        "best_of": 3,
    }


def stress_line(sc, torch, stream, workers, tuning, cap_cl, cap_adc, steps):
    """The 256-event stress batch at full size: one launch with output capacities sized for the
    64-event batch (overflows are reported with the needed sizes), then the batch again with
    those sizes, timed, with the headline's tuning and with the autotuner's pick for this
    distribution. Both retries are checked against launches with capacities that always suffice
    and against each other; oracle parity of this distribution is the GPU tests'."""
    cfg = fedgen.CONFIGS[4]
    t0 = time.time()
    cal = fedgen.make_calibration(cfg)
    evs = fedgen.make_events(cfg, cal, range(cfg.n_events), workers=workers)
    gen_s = time.time() - t0
    sizes = np.concatenate([np.diff(e.fed_offset.astype(np.int64)) for e in evs])
    ctx = sc.Context(cal.noise, cal.gain, cal.bad, device=0, stream=stream)
    ctx.tuning = {k: tuning[k] for k in ("chunk_digis", "tile_waves", "tiles_per_cu", "fed_major",
                                         "stage_bytes")}
    ctx.tuning = {"use_graph": 0}
    d = [sc.Event(e.zs, e.fed_offset).to_device() for e in evs]
    o = [ctx.output(cap_cl, cap_adc) for _ in d]
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        rc, sts = ctx.process_events(d, o)
        first_ms = ctx.stats()["last_kernel_ms"]
        torch.cuda.synchronize()
    n_over = sum(1 for s in sts if s == sc.SC_ERR_OVERFLOW)
    need = [(y.n_cl, y.n_adc) for y in o]
    # every 16th event in a batch of its own with capacities that always suffice (an event's
    # results do not depend on the rest of its batch)
    sample = list(range(0, len(d), 16))
    safe = [ctx.output(*sc.safe_caps(d[i])) for i in sample]
    ctx.process_events([d[i] for i in sample], safe)
    ref = [(b.to_numpy()[0], b.to_numpy()[1]) for b in safe]
    del safe
    b = algorithmic_bytes(evs, need, cfg.n_fed)

    def retry():
        """The batch with the needed capacities, timed, and checked against the safe launch."""
        out = [ctx.output(max(c, 1), max(a, 1)) for c, a in need]
        batch = ctx.batch(d, out)
        r = time_steps(ctx, batch, steps, 2, stream, torch, graph=False)
        rc2 = ctx.process_batch(batch)[0]
        torch.cuda.synchronize()
        ok = all(np.array_equal(out[i].to_numpy()[0], c) and np.array_equal(out[i].to_numpy()[1], a)
                 for i, (c, a) in zip(sample, ref))
        k = r["kernel_ms"]
        stage = ctx.tuning["stage_bytes"]
        return {"tuning": {t: ctx.tuning[t] for t in ("chunk_digis", "tile_waves", "tiles_per_cu",
                                                      "fed_major", "stage_bytes")},
                "feds_larger_than_lds_stage": float(np.mean(sizes > stage - STAGE_SLACK)),
                "status": rc2, "events_per_s": len(evs) * steps / r["elapsed_s"],
                "ms_per_step": r["elapsed_s"] / steps * 1e3, "kernel_ms": k,
                "hbm_frac": (b / (k * 1e-3) / 1e9 / HBM_PEAK_GBS) if k else None,
                "cross_check": ("bit-identical to safe-capacity launches (every 16th event)"
                                if ok else "MISMATCH")}

    headline = retry()
    t0 = time.time()
    best = ctx.autotune(d[:64])
    tune_s = time.time() - t0
    ctx.tuning = dict(best, use_graph=0)
    tuned = retry()
    tuned["tuned_by"] = f"autotuner on 64 of the stress events ({tune_s:.1f} s)"
    ctx.close()
    return {
        "workload": f"stress: {len(evs)} events x {cfg.n_fed} FEDs at 6% occupancy, width "
                    "1+Geometric(0.25) capped at 32, 1% bad strips, noise U[2,10]",
        "generation_s": gen_s,
        "zs_mb": sum(e.zs.size for e in evs) / 1e6,
        "fed_bytes_mean": float(sizes.mean()), "fed_bytes_max": int(sizes.max()),
        "clusters": int(sum(c for c, _ in need)),
        "algorithmic_bytes_per_launch": b,
        "first_launch": {"capacities": [cap_cl, cap_adc], "status": rc,
                         "events_overflowed": n_over, "kernel_ms": first_ms},
        "retry": headline,
        "retry_autotuned": tuned,
    }


def serving_sweep(sc, torch, stream, args, tuning, fracs):
    """Open-loop Poisson arrivals through the server at fractions of the batched capacity of a
    pool of full-detector events of the occupancy mix, device-resident inputs and outputs."""
    cfg3 = fedgen.CONFIGS[3]
    cal3 = fedgen.make_calibration(cfg3)
    pool = fedgen.make_events(cfg3, cal3, range(64), workers=args.workers)
    ctx3 = sc.Context(cal3.noise, cal3.gain, cal3.bad, device=0, stream=stream,
                      max_batch=64, n_streams=2)
    if tuning is not None:
        ctx3.tuning = {k: tuning[k] for k in ("chunk_digis", "tile_waves", "tiles_per_cu",
                                              "fed_major")}
    ctx3.tuning = {"use_graph": 0}
    p_dev = [sc.Event(x.zs, x.fed_offset).to_device() for x in pool]
    n_out = 256
    p_out = [ctx3.output(*sc.safe_caps(p_dev[j % len(p_dev)])) for j in range(n_out)]
    # batched capacity on this mix
    for _ in range(3):
        ctx3.process_events(p_dev, p_out[:len(p_dev)])
    torch.cuda.synchronize()
    tcap = time.perf_counter()
    for _ in range(10):
        ctx3.process_events(p_dev, p_out[:len(p_dev)])
    torch.cuda.synchronize()
    capacity = 10 * len(p_dev) / (time.perf_counter() - tcap)
    # a short replay first: the server's start-up and first batches are not a point's tail
    ctx3.serve_replay(p_dev, p_out, 200, 0.5 * capacity, seed=1)
    points = []
    for frac in fracs:
        rc, lat, eps, ph = ctx3.serve_replay(p_dev, p_out, args.serve_events,
                                             frac * capacity, seed=int(frac * 1000),
                                             phases=True)
        # where the time goes: the phases' medians over all events and their means over the
        # slowest 1 %; "other" is the launch reaching the device and completion being seen
        other = lat - ph.sum(axis=1)
        tail = lat >= np.percentile(lat, 99)
        names = ("output_slot_wait", "queue_wait", "device", "other")
        cols = [ph[:, 0], ph[:, 1], ph[:, 2], other]
        points.append({"rate_frac": frac, "offered_events_per_s": frac * capacity,
                       "achieved_events_per_s": eps,
                       "latency_us_p50": float(np.percentile(lat, 50)),
                       "latency_us_p99": float(np.percentile(lat, 99)), "status": rc,
                       "phase_us_p50": {k: round(float(np.median(v)), 1)
                                        for k, v in zip(names, cols)},
                       "phase_us_tail_mean": {k: round(float(v[tail].mean()), 1)
                                              for k, v in zip(names, cols)}})
        log(f"serve {frac:.1f}: {points[-1]}")
    st = ctx3.stats()
    serving = {"workload": f"Poisson arrivals, {args.serve_events} events per point, pool of "
                           f"{len(pool)} full-detector events of the occupancy mix, device-"
                           "resident inputs and outputs",
               "batched_capacity_events_per_s": capacity, "points": points,
               "server_batches": st["server_batches"],
               "server_budget_bytes": st["server_budget"],
               "server_held_peak_bytes": st["server_held_peak"]}
    ctx3.close()
    return serving


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--plain-events", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="seconds each oracle process of the CPU baseline runs for")
    ap.add_argument("--cpu-procs", type=int, default=min(16, os.cpu_count() or 1),
                    help="oracle processes of the CPU aggregate (the box's CPU share)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-stress", action="store_true")
    ap.add_argument("--no-cold", action="store_true")
    ap.add_argument("--no-ingest", action="store_true")
    ap.add_argument("--no-hits", action="store_true")
    ap.add_argument("--no-modules", action="store_true")
    ap.add_argument("--serve-events", type=int, default=2000,
                    help="events per arrival-rate point of the serving sweep")
    ap.add_argument("--tuning", default=None,
                    help="chunk_digis,tile_waves,tiles_per_cu,fed_major instead of the autotuner")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--serve-only", type=float, default=None, metavar="FRAC",
                    help="only run the serving replay at this fraction of the batched capacity "
                         "(default tuning) and print its JSON")
    ap.add_argument("--ingest-only", action="store_true",
                    help="only run the host-ingest measurement on the batch and print its JSON")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB 5 times (reference "
                         "for the HBM byte counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs the path on one GPU only (got --gpus {args.gpus}); events shard "
              "across GPUs with host-side dispatch and no device exchange, so per-GPU throughput "
              "is the single-GPU figure.", file=sys.stderr)
        sys.exit(2)

    if args.serve_only is not None:
        import torch
        import paper_2101_11489_amd as sc
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        print(json.dumps(serving_sweep(sc, torch, torch.cuda.Stream(), args, None,
                                       (args.serve_only,))))
        return

    # ---- workload: 64 full-detector events, occupancy log-uniform in [0.5%, 5%] -------------
    cfg = fedgen.CONFIGS[2]
    t0 = time.time()
    cal = fedgen.make_calibration(cfg)
    events = fedgen.make_events(cfg, cal, range(args.batch), workers=args.workers)
    n_fed = cfg.n_fed
    log(f"generated {len(events)} events in {time.time() - t0:.1f}s; "
        f"ZS {sum(e.zs.size for e in events) / 1e6:.1f} MB")

    # ---- CPU baseline first, before anything touches the GPU (its processes are forked) -----
    cpu, refs, mod_ref = None, None, None
    geo = fedgen.make_geometry(cfg)
    if not args.no_cpu_baseline and not args.copy_probe_mib:
        refs, mod_ref, cpu = cpu_baseline(events, cal, n_fed, args.cpu_seconds, args.cpu_procs,
                                          geo)
        log(f"cpu baseline: {cpu}")

    import torch
    import paper_2101_11489_amd as sc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev_name = torch.cuda.get_device_name(0)
    if args.copy_probe_mib:
        a = torch.ones(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel(), "copies": 5}))
        return

    stream = torch.cuda.Stream()
    ctx = sc.Context(cal.noise, cal.gain, cal.bad, device=0, stream=stream)
    devs = [sc.Event(e.zs, e.fed_offset).to_device() for e in events]
    outs = [ctx.output(*sc.safe_caps(d)) for d in devs]
    if args.ingest_only:
        ctx.tuning = {"use_graph": 0}
        print(json.dumps(ingest_line(sc, torch, ctx, events, outs, len(events), 8)))
        ctx.close()
        return
    torch.cuda.synchronize()
    if args.tuning:
        c, w, t, f = (int(x) for x in args.tuning.split(",")[:4])
        ctx.tuning = {"chunk_digis": c, "tile_waves": w, "tiles_per_cu": t, "fed_major": f}
        tuned_by = "given"
    else:
        t_at = time.time()
        ctx.autotune(devs)
        tuned_by = f"autotuner on the batch ({time.time() - t_at:.1f} s)"
    log(f"tuning: {ctx.tuning} ({tuned_by})")

    # ---- warm-up, then a sampled parity check at full size ---------------------------------
    batch = ctx.batch(devs, outs)   # argument arrays marshalled once
    ctx.tuning = {"use_graph": 1}
    for _ in range(3):
        ctx.process_batch(batch)
    torch.cuda.synchronize()
    parity = "skipped (no CPU-baseline leg, which computes the oracle's results)"
    if refs is not None:
        ok = True
        for i, (rcl, radc, _) in refs.items():
            cl, adc, _ = outs[i].to_numpy()
            ok &= np.array_equal(cl, rcl) and np.array_equal(adc, radc)
        parity = "bit-exact against the oracle (first and last event)" if ok else "MISMATCH"
    log(f"parity: {parity}")

    # ---- timed region: graph replay (the stated form), then eager, then cache-cold ----------
    g = time_steps(ctx, batch, args.steps, args.warmup, stream, torch, graph=True)
    e = time_steps(ctx, batch, args.steps, args.warmup, stream, torch, graph=False)
    counts = [(o.n_cl, o.n_adc) for o in outs]
    n_ev = len(events)
    b_alg = algorithmic_bytes(events, counts, n_fed)
    ev_per_s = n_ev * args.steps / g["elapsed_s"]
    ms_per_step = g["elapsed_s"] / args.steps * 1e3
    # The kernel's duration: the library's HIP events right around the eager launch of the
    # same kernel on the same stream (inside a replayed graph the event nodes bracket more than
    # the kernel: graph_event_bracket_ms below).
    kern = e["kernel_ms"] if e["kernel_ms"] else g["kernel_ms"]
    achieved = b_alg / (kern * 1e-3) / 1e9 if kern else None
    tuning = ctx.tuning
    tuning["use_graph"] = 1
    eager = {"graph_event_bracket_ms": g["kernel_ms"],
             "events_per_s": n_ev * args.steps / e["elapsed_s"],
             "ms_per_step": e["elapsed_s"] / args.steps * 1e3, "kernel_ms": e["kernel_ms"],
             "latency_ms_p50": float(np.percentile(e["step_ms"], 50)),
             "latency_ms_p99": float(np.percentile(e["step_ms"], 99))}
    log(f"graph: {ev_per_s:.0f} events/s, {ms_per_step:.3f} ms/step, kernel {kern} ms; "
        f"eager: {eager}")
    cold = None
    if not args.no_cold:
        flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        c = time_steps(ctx, batch, 20, 2, stream, torch, graph=False, flush=flush)
        del flush
        torch.cuda.empty_cache()
        cold = {"what": "eager launches, each after a 512 MiB write on the launch stream (L2 and "
                        "Infinity Cache emptied of the batch's inputs and calibration)",
                "kernel_ms": c["kernel_ms"],
                "hbm_frac": (b_alg / (c["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS)
                            if c["kernel_ms"] else None}
        log(f"cold: {cold}")
    probe = stream_probe(torch)
    log(f"stream probe: {probe}")

    # ---- plain per-event path: 50-FED and full-detector single events -----------------------
    plain = {}
    if not args.no_plain:
        for cid in (0, 1):
            plain[f"config{cid}"] = plain_line(sc, torch, stream, cid, args.plain_events,
                                               args.workers, tuning)
            log(f"plain config {cid}: {plain[f'config{cid}']}")

    # ---- the 256-event stress batch ------------------------------------------------------------
    # ---- clusters -> global hits over the batch's outputs (the step after the path) ---------
    hits_line = None
    if not args.no_hits:
        ctx.set_geometry(geo)
        hit_bufs = ctx.cluster_hits(outs)
        hit_bufs = [torch.empty((max(1, h.shape[0]), 4), dtype=torch.float32, device="cuda")
                    for h in hit_bufs]
        ks = []
        for _ in range(3 + 20):
            ctx.cluster_hits(outs, hits=hit_bufs)
            ks.append(ctx.stats()["last_kernel_ms"])
        k_hits = statistics.mean(ks[3:])
        n_cl_all = sum(min(o.cs.n_cl, o.cs.cap_cl) for o in outs)
        tables = geo.channel_module.size * 8 + geo.n_modules * 32
        b_hits = n_cl_all * 32 + tables
        max_err = None
        if refs is not None:
            max_err = 0.0
            for i, (_, _, rh) in refs.items():
                got = hit_bufs[i][:rh.shape[0]].cpu().numpy().astype(np.float64)
                max_err = max(max_err, float(np.max(np.abs(got - rh))))
        hits_line = {
            "workload": f"global hits of the batch's {n_cl_all} clusters ({n_ev} events) on a "
                        f"synthetic geometry of {geo.n_modules} modules, one launch",
            "kernel_ms": k_hits, "clusters_per_s": n_cl_all / (k_hits * 1e-3),
            "algorithmic_bytes_per_launch": b_hits,
            "roofline": {"bound": "hbm", "achieved": b_hits / (k_hits * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": b_hits / (k_hits * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "max_abs_err_cm_vs_oracle": max_err,
        }
        log(f"hits: {hits_line}")
        del hit_bufs

    # ---- module rows: the same batch with runs continuing across the channels of a module ---
    mod_line = None
    if not args.no_modules:
        ctx.tuning = {"use_graph": 0}
        ctx.set_modules(geo.channel_module)
        ks = []
        for _ in range(3 + 20):
            ctx.process_batch(batch)
            ks.append(ctx.stats()["last_kernel_ms"])
        torch.cuda.synchronize()
        mod_ok = None
        if mod_ref is not None:
            rcl, radc = mod_ref
            cl, adc, _ = outs[0].to_numpy()
            mod_ok = bool(np.array_equal(cl, rcl) and np.array_equal(adc, radc))
        n_cross = int(np.sum(outs[0].to_numpy()[0]["first"].astype(np.int64) +
                             outs[0].to_numpy()[0]["width"] > 256))
        ctx.set_modules(None)
        ctx.tuning = {"use_graph": 1}
        k_mod = statistics.mean(ks[3:])
        mod_line = {
            "workload": f"the {n_ev}-event batch with the synthetic module map "
                        f"({geo.n_modules} modules of 2-3 channels), eager launches",
            "kernel_ms": k_mod, "events_per_s_kernel": n_ev / (k_mod * 1e-3),
            "clusters_crossing_a_channel_edge_event0": n_cross,
            "parity": ("bit-exact against the module-aware oracle (first event)" if mod_ok
                       else "skipped" if mod_ok is None else "MISMATCH"),
        }
        log(f"modules: {mod_line}")
        # the plain results again for whatever follows
        ctx.process_batch(batch)

    ingest = None
    if not args.no_ingest:
        ctx.tuning = {"use_graph": 0}
        ingest = ingest_line(sc, torch, ctx, events, outs, n_ev, 8)
        ctx.tuning = {"use_graph": 1}
        log(f"host ingest: {ingest}")

    stress = None
    if not args.no_stress:
        cap_cl = max(c for c, _ in counts)
        cap_adc = max(a for _, a in counts)
        stress = stress_line(sc, torch, stream, args.workers, tuning, cap_cl, cap_adc, 5)
        log(f"stress: {stress}")

    # ---- serving: Poisson arrivals of the occupancy mix {0.5,1.5,3,6}% -----------------------
    serving = None
    if not args.no_serve:
        serving = serving_sweep(sc, torch, stream, args, tuning, (0.2, 0.4, 0.6, 0.8, 1.0, 1.2))

    traffic = load_traffic(f"config2-batch{n_ev}", tuning)
    line = {
        "metric": "events/s, unpack + three-threshold clustering, batched full-detector events",
        "value": ev_per_s,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": f"batched: {n_ev} full-detector events per fused persistent launch "
                        "(440 FEDs x 96 ch x 256 strips, occupancy log-uniform 0.5-5%), "
                        "hipGraph replay, autotuned tiles",
            "n_fed": n_fed, "events_per_launch": n_ev,
            "zs_mb_per_launch": round(sum(x.zs.size for x in events) / 1e6, 2),
            "clusters_per_launch": int(sum(c for c, _ in counts)),
            "tuning": tuning, "tuned_by": tuned_by, "device": dev_name,
        },
        "strips_per_s": ev_per_s * n_fed * 96 * 256,
        "digis_per_s": sum(x.n_digis for x in events) * args.steps / g["elapsed_s"],
        "latency_ms_p50": float(np.percentile(g["step_ms"], 50)),
        "latency_ms_p99": float(np.percentile(g["step_ms"], 99)),
        "kernel_ms": kern,
        "parity": parity,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": b_alg,
            "kernel": "fused_kernel",
            "measured_read_stream_gbs": probe["read_stream_gbs"],
            "measured_copy_gbs": probe["copy_gbs"],
        },
        "eager": eager,
        "cache_cold": cold,
        "plain_path": plain or None,
        "module_rows": mod_line,
        "cluster_hits": hits_line,
        "host_ingest": ingest,
        "stress": stress,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
