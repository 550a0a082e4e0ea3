"""The oracle run with nested parallelism on the host: events in flight x FED ranges per event.

TEST INFRASTRUCTURE ONLY (the CPU comparator): used by the tests and the benchmark's CPU-baseline
leg; the GPU library never imports it.

Paper §3 runs the CPU version with nested OpenMP: an outer level over events and an inner level
over the strips of an event. Here the unchanged single-threaded C oracle does the work: an event's
FEDs are cut into M ranges, each unpacked and clustered by one oracle call (FEDs are independent
and clusters never leave their FED), and N events are in flight at once. The oracle's C calls
release the GIL, so N x M Python threads keep N x M cores busy. The ranges' clusters, put back in
FED order with their channel numbers shifted, are the whole event's.
"""
from __future__ import annotations

import ctypes
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import CLUSTER_DTYPE, T_CHANNEL, T_CLUSTER, T_SEED, Clusters, lib

NCH, NS, NAPV = 96, 256, 128


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def fed_ranges(n_fed: int, m: int) -> list[tuple[int, int]]:
    b = np.linspace(0, n_fed, m + 1).round().astype(int)
    return [(int(b[i]), int(b[i + 1])) for i in range(m) if b[i + 1] > b[i]]


class _RangeBuffers:
    """Per-thread buffers for one FED range: dense ADCs, channel status, cluster output."""

    def __init__(self, n_fed: int, cap: int):
        self.adc = np.empty(n_fed * NCH * NS, np.uint8)
        self.st = np.empty(n_fed * NCH, np.uint8)
        self.cl = np.empty(cap, CLUSTER_DTYPE)
        self.out_adc = np.empty(2 * cap, np.uint16)


def run_range(zs, fo, noise, gain, bad, a, b, buf, t=(T_SEED, T_CHANNEL, T_CLUSTER)):
    """FEDs [a, b) of one event: one oracle unpack and one oracle cluster call over the range.
    Returns (unpack status, n_cl, n_adc); the clusters' channels are range-local."""
    L = lib()
    n = b - a
    zsp = zs if zs.size else np.zeros(1, np.uint8)
    st = L.oracle_unpack(_p(zsp), ctypes.c_void_p(fo.ctypes.data + 8 * a), n, _p(buf.adc),
                         _p(buf.st))
    n_cl, n_adc = ctypes.c_uint64(), ctypes.c_uint64()
    L.oracle_cluster(_p(buf.adc), n, ctypes.c_void_p(noise.ctypes.data + 4 * a * NCH * NS),
                     ctypes.c_void_p(gain.ctypes.data + 4 * a * NCH * 2),
                     ctypes.c_void_p(bad.ctypes.data + a * NCH * NS), t[0], t[1], t[2],
                     _p(buf.cl), buf.cl.size, _p(buf.out_adc), buf.out_adc.size,
                     ctypes.byref(n_cl), ctypes.byref(n_adc))
    return int(st), int(n_cl.value), int(n_adc.value)


def process_event_ranges(zs, fed_offset, noise, gain, bad, m: int) -> Clusters:
    """One event as m FED ranges, one after the other, results put back together."""
    zs = np.ascontiguousarray(zs, np.uint8)
    fo = np.ascontiguousarray(fed_offset, np.uint64)
    noise = np.ascontiguousarray(noise, np.float32)
    gain = np.ascontiguousarray(gain, np.float32)
    bad = np.ascontiguousarray(bad, np.uint8)
    n_fed = fo.size - 1
    cls, adcs, status = [], [], 0
    for a, b in fed_ranges(n_fed, m):
        buf = _RangeBuffers(b - a, max(1, int(fo[b] - fo[a])))
        st, ncl, nadc = run_range(zs, fo, noise, gain, bad, a, b, buf)
        cl = buf.cl[:ncl].copy()
        cl["channel"] += a * NCH
        cls.append(cl)
        adcs.append(buf.out_adc[:nadc].copy())
        status |= st
    return Clusters(np.concatenate(cls), np.concatenate(adcs), status)


class NestedRunner:
    """N events in flight, each split into M FED ranges processed at once, over a list of
    events cycled for a given time. run() returns (events done, seconds, per-event latencies)."""

    def __init__(self, events, cal, n_outer: int, n_inner: int):
        self.events, self.cal = events, cal
        self.n_outer, self.n_inner = n_outer, n_inner
        n_fed = events[0].fed_offset.size - 1
        self.ranges = fed_ranges(n_fed, n_inner)
        cap = max(int(np.max(np.diff(e.fed_offset.astype(np.int64)))) for e in events)
        self.bufs = [[_RangeBuffers(b - a, max(1, cap * (b - a))) for a, b in self.ranges]
                     for _ in range(n_outer)]
        self.noise = np.ascontiguousarray(cal.noise, np.float32)
        self.gain = np.ascontiguousarray(cal.gain, np.float32)
        self.bad = np.ascontiguousarray(cal.bad, np.uint8)

    def run(self, seconds: float):
        lock = threading.Lock()
        nxt = [0]
        done, lat = [0], []
        t0 = time.perf_counter()
        with ThreadPoolExecutor(self.n_outer * len(self.ranges)) as inner:
            def outer(slot):
                while True:
                    with lock:
                        k = nxt[0]
                        nxt[0] += 1
                    if time.perf_counter() - t0 >= seconds:
                        return
                    e = self.events[k % len(self.events)]
                    zs = np.ascontiguousarray(e.zs, np.uint8)
                    fo = np.ascontiguousarray(e.fed_offset, np.uint64)
                    ts = time.perf_counter()
                    futs = [inner.submit(run_range, zs, fo, self.noise, self.gain, self.bad,
                                         a, b, buf)
                            for (a, b), buf in zip(self.ranges, self.bufs[slot])]
                    for f in futs:
                        f.result()
                    te = time.perf_counter()
                    with lock:
                        done[0] += 1
                        lat.append(te - ts)
            threads = [threading.Thread(target=outer, args=(s,)) for s in range(self.n_outer)]
            for t in threads:
                t.start()
            for t in threads:
                t.join()
        return done[0], time.perf_counter() - t0, lat
