"""Python binding of libsc.so, the MI355X strip unpacking + three-threshold clustering library.

Argument marshalling only: every step of the path runs in the library's HIP kernels. PyTorch
provides device memory (``torch.empty(..., device="cuda")``) and the stream handle. The binding
refuses to work without the compiled library; there is no CPU fallback.

Entry points mirror the C ABI in include/sc.h: ``Context.unpack``, ``Context.cluster``,
``Context.process_events``, ``Context.submit`` / ``Context.poll``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsc.so")

CHANNELS_PER_FED = 96
STRIPS_PER_CHANNEL = 256

SC_OK, SC_MALFORMED, SC_PENDING = 0, 1, 2
SC_ERR_INVALID_ARG, SC_ERR_OVERFLOW, SC_ERR_BUDGET = -1, -2, -3
SC_STATIC_MAX_EVENTS, SC_STATIC_MAX_TILES = 1024, 1024 * 440   # sc_process_events_static
SC_ERR_AGAIN, SC_ERR_DEVICE, SC_ERR_NOMEM, SC_ERR_UNKNOWN_TICKET = -4, -5, -6, -7
SC_MEM_HOST, SC_MEM_DEVICE, SC_MEM_HOST_PINNED = 0, 1, 2
CH_MALFORMED, CH_FED_TRAILING = 1, 2

STATUS_NAMES = {0: "OK", 1: "MALFORMED", 2: "PENDING", -1: "INVALID_ARG", -2: "OVERFLOW",
                -3: "BUDGET", -4: "AGAIN", -5: "DEVICE", -6: "NOMEM", -7: "UNKNOWN_TICKET"}

CLUSTER_DTYPE = np.dtype([("channel", "<u4"), ("first", "<u2"), ("width", "<u2"),
                          ("charge", "<u4"), ("barycenter", "<f4")])

EXPORTED = ["sc_default_options", "sc_create", "sc_destroy", "sc_unpack", "sc_cluster",
            "sc_process_events", "sc_process_pipelined", "sc_process_events_static", "sc_submit", "sc_poll", "sc_serve_replay", "sc_get_tuning",
            "sc_set_tuning", "sc_autotune", "sc_get_stats", "sc_last_error", "sc_set_geometry",
            "sc_cluster_hits", "sc_set_modules"]


class ScError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ScCalib(ctypes.Structure):
    _fields_ = [("n_fed", ctypes.c_uint32), ("noise", ctypes.c_void_p), ("gain", ctypes.c_void_p),
                ("bad", ctypes.c_void_p), ("t_seed", ctypes.c_float),
                ("t_channel", ctypes.c_float), ("t_cluster", ctypes.c_float)]


class ScOptions(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("hbm_budget", ctypes.c_size_t), ("max_batch", ctypes.c_uint32),
                ("n_streams", ctypes.c_uint32), ("queue_depth", ctypes.c_uint32),
                ("tune_cache", ctypes.c_char_p)]


class ScEvent(ctypes.Structure):
    _fields_ = [("zs", ctypes.c_void_p), ("fed_offset", ctypes.c_void_p), ("mem", ctypes.c_int)]


class ScClusters(ctypes.Structure):
    _fields_ = [("cl", ctypes.c_void_p), ("cap_cl", ctypes.c_uint32), ("n_cl", ctypes.c_uint32),
                ("adc", ctypes.c_void_p), ("cap_adc", ctypes.c_uint32),
                ("n_adc", ctypes.c_uint32), ("chan_status", ctypes.c_void_p),
                ("mem", ctypes.c_int)]


class ScGeometry(ctypes.Structure):
    _fields_ = [("n_modules", ctypes.c_uint32), ("channel_module", ctypes.c_void_p),
                ("channel_first", ctypes.c_void_p), ("module_strips", ctypes.c_void_p),
                ("origin", ctypes.c_void_p), ("u_dir", ctypes.c_void_p), ("pitch", ctypes.c_void_p)]


class ScTuning(ctypes.Structure):
    _fields_ = [("chunk_digis", ctypes.c_uint32), ("tile_waves", ctypes.c_uint32),
                ("tiles_per_cu", ctypes.c_uint32), ("fed_major", ctypes.c_uint32),
                ("use_graph", ctypes.c_uint32), ("stage_bytes", ctypes.c_uint32)]


class ScStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("events", ctypes.c_uint64),
                ("graph_replays", ctypes.c_uint64), ("graph_captures", ctypes.c_uint64),
                ("server_batches", ctypes.c_uint64), ("server_events", ctypes.c_uint64),
                ("server_rejected_again", ctypes.c_uint64), ("last_kernel_ms", ctypes.c_double),
                ("kernel_ms_total", ctypes.c_double), ("kernels_timed", ctypes.c_uint64),
                ("allocations", ctypes.c_uint64), ("server_budget", ctypes.c_uint64),
                ("server_held_peak", ctypes.c_uint64)]


_lib = None


def lib():
    """Load libsc.so (built in-tree by build.py). Fails loudly when it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2101_11489_amd/build.py "
                              "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(LIB_PATH)
        P, st = ctypes.c_void_p, ctypes.c_int
        sig = {
            "sc_default_options": ([ctypes.POINTER(ScOptions)], None),
            "sc_create": ([ctypes.POINTER(ScCalib), ctypes.POINTER(ScOptions), ctypes.POINTER(P)], st),
            "sc_destroy": ([P], None),
            "sc_unpack": ([P, ctypes.POINTER(ScEvent), P, P, ctypes.c_int], st),
            "sc_cluster": ([P, P, ctypes.c_int, ctypes.POINTER(ScClusters)], st),
            "sc_process_events": ([P, ctypes.POINTER(ScEvent), ctypes.c_uint32,
                                   ctypes.POINTER(ScClusters), ctypes.POINTER(ctypes.c_int)], st),
            "sc_process_pipelined": ([P, ctypes.POINTER(ScEvent), ctypes.c_uint32,
                                      ctypes.POINTER(ScClusters), ctypes.c_uint32,
                                      ctypes.POINTER(ctypes.c_int)], st),
            "sc_process_events_static": ([P, ctypes.POINTER(ScEvent), ctypes.c_uint32,
                                          ctypes.POINTER(ScClusters), ctypes.POINTER(ctypes.c_int)],
                                         st),
            "sc_submit": ([P, ctypes.POINTER(ScEvent), ctypes.POINTER(ScClusters),
                           ctypes.POINTER(ctypes.c_uint64)], st),
            "sc_poll": ([P, ctypes.c_uint64, ctypes.c_int64], st),
            "sc_serve_replay": ([P, ctypes.POINTER(ScEvent), ctypes.c_uint32,
                                 ctypes.POINTER(ScClusters), ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
                                st),
            "sc_get_tuning": ([P, ctypes.POINTER(ScTuning)], st),
            "sc_set_tuning": ([P, ctypes.POINTER(ScTuning)], st),
            "sc_autotune": ([P, ctypes.POINTER(ScEvent), ctypes.c_uint32,
                             ctypes.POINTER(ScTuning)], st),
            "sc_get_stats": ([P, ctypes.POINTER(ScStats)], st),
            "sc_set_geometry": ([P, ctypes.POINTER(ScGeometry)], st),
            "sc_set_modules": ([P, ctypes.c_void_p], st),
            "sc_cluster_hits": ([P, ctypes.POINTER(ScClusters), ctypes.c_uint32,
                                 ctypes.POINTER(ctypes.c_void_p)], st),
            "sc_last_error": ([P], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


# ---- buffers: torch tensors on the GPU, numpy arrays on the host ---------------------------

def _torch():
    import torch
    return torch


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


def _is_dev(x) -> bool:
    return not isinstance(x, np.ndarray)


@dataclass
class Event:
    """One event: ZS bytes and FED offsets (u64 [n_fed+1]), both numpy (host) or both torch
    CUDA tensors (device). pinned=True marks numpy arrays that view page-locked memory (made by
    to_pinned), which the library copies to the device without staging."""
    zs: object
    fed_offset: object
    pinned: bool = False

    def __post_init__(self):
        if isinstance(self.zs, np.ndarray):
            self.zs = np.ascontiguousarray(self.zs, dtype=np.uint8)
        if isinstance(self.fed_offset, np.ndarray):
            self.fed_offset = np.ascontiguousarray(self.fed_offset, dtype=np.uint64)
        if _is_dev(self.zs) != _is_dev(self.fed_offset):
            raise ValueError("zs and fed_offset must both be host or both be device buffers")

    @property
    def mem(self) -> int:
        if _is_dev(self.zs):
            return SC_MEM_DEVICE
        return SC_MEM_HOST_PINNED if self.pinned else SC_MEM_HOST

    def to_pinned(self) -> "Event":
        """A host copy in page-locked memory (torch pin_memory), kept alive by the Event."""
        torch = _torch()
        zs = np.ascontiguousarray(self.zs, dtype=np.uint8)
        fo = np.ascontiguousarray(self.fed_offset, dtype=np.uint64)
        tz = torch.empty(max(zs.size, 1), dtype=torch.uint8, pin_memory=True)
        tf = torch.empty(fo.size, dtype=torch.int64, pin_memory=True)
        nz, nf = tz.numpy()[:zs.size], tf.numpy().view(np.uint64)
        nz[:] = zs
        nf[:] = fo
        ev = Event(nz, nf, pinned=True)
        ev._pinned_keep = (tz, tf)
        return ev

    def c(self) -> ScEvent:
        zs = self.zs
        if isinstance(zs, np.ndarray) and zs.size == 0:
            zs = np.zeros(1, np.uint8)
            self._keep = zs
        return ScEvent(_ptr(zs), _ptr(self.fed_offset), self.mem)

    def to_device(self, device="cuda") -> "Event":
        torch = _torch()
        zs = torch.from_numpy(np.ascontiguousarray(self.zs, dtype=np.uint8)).to(device)
        fo = torch.from_numpy(np.ascontiguousarray(self.fed_offset, dtype=np.uint64).view(np.int64)).to(device)
        return Event(zs, fo)


def pack_pinned(events):
    """Host copies of the events laid back to back in one page-locked buffer (the layout of a
    readout ring): consecutive events of a batch then go to the device in one transfer."""
    torch = _torch()
    zs = [np.ascontiguousarray(e.zs, dtype=np.uint8) for e in events]
    spans = [int(np.asarray(e.fed_offset, dtype=np.uint64).max()) if len(e.fed_offset) else 0
             for e in events]
    if any(sp > z.size for sp, z in zip(spans, zs)):
        raise ValueError("an event's FED offsets reach past its bytes")
    total = sum(spans)
    buf = torch.empty(max(total, 1), dtype=torch.uint8, pin_memory=True)
    flat = buf.numpy()
    out, at = [], 0
    for e, z, sp in zip(events, zs, spans):
        flat[at:at + sp] = z[:sp]
        fo = torch.empty(len(e.fed_offset), dtype=torch.int64, pin_memory=True)
        fo.numpy().view(np.uint64)[:] = np.asarray(e.fed_offset, dtype=np.uint64)
        ev = Event(flat[at:at + sp], fo.numpy().view(np.uint64), pinned=True)
        ev._pinned_keep = (buf, fo)
        out.append(ev)
        at += sp
    return out


class Batch:
    """Events and outputs of one sc_process_events call, marshalled once. Each output's count
    fields alias the batch's argument array, so the library's counts appear in the outputs."""

    def __init__(self, events, outs):
        if len(events) != len(outs):
            raise ValueError("one output per event")
        self.events, self.outs = list(events), list(outs)
        self.n = len(self.events)
        self.c_ev = (ScEvent * self.n)(*[e.c() for e in self.events])
        self.c_out = (ScClusters * self.n)(*[o.cs for o in self.outs])
        self.c_st = (ctypes.c_int * self.n)()
        for i, o in enumerate(self.outs):
            o.cs = self.c_out[i]


class Output:
    """Cluster output buffers of one event (device: torch CUDA tensors; host: numpy)."""

    def __init__(self, cap_cl: int, cap_adc: int, n_fed: int, device: bool = True,
                 chan_status: bool = False, device_name="cuda"):
        self.device = device
        if device:
            torch = _torch()
            self.cl = torch.zeros((max(cap_cl, 1), 4), dtype=torch.int32, device=device_name)
            self.adc = torch.zeros(max(cap_adc, 1), dtype=torch.int16, device=device_name)
            self.chan_status = (torch.zeros(n_fed * CHANNELS_PER_FED, dtype=torch.uint8,
                                            device=device_name) if chan_status else None)
        else:
            self.cl = np.zeros(max(cap_cl, 1), dtype=CLUSTER_DTYPE)
            self.adc = np.zeros(max(cap_adc, 1), dtype=np.uint16)
            self.chan_status = np.zeros(n_fed * CHANNELS_PER_FED, np.uint8) if chan_status else None
        self.cs = ScClusters(_ptr(self.cl), cap_cl, 0, _ptr(self.adc), cap_adc, 0,
                             _ptr(self.chan_status), SC_MEM_DEVICE if device else SC_MEM_HOST)

    @property
    def n_cl(self) -> int:
        return self.cs.n_cl

    @property
    def n_adc(self) -> int:
        return self.cs.n_adc

    def to_numpy(self):
        """(clusters CLUSTER_DTYPE[n], member ADCs uint16[n_adc], chan_status or None), limited to
        what was written."""
        ncl = min(self.cs.n_cl, self.cs.cap_cl)
        nadc = min(self.cs.n_adc, self.cs.cap_adc)
        if self.device:
            cl = self.cl[:ncl].cpu().numpy().view(CLUSTER_DTYPE).reshape(-1)
            adc = self.adc[:nadc].cpu().numpy().view(np.uint16)
            st = self.chan_status.cpu().numpy() if self.chan_status is not None else None
        else:
            cl, adc, st = self.cl[:ncl].copy(), self.adc[:nadc].copy(), self.chan_status
        return cl, adc, st


class Context:
    """A library context: resident calibration, workspaces, graphs and the server."""

    def __init__(self, noise, gain, bad, t_seed=3.0, t_channel=2.0, t_cluster=5.0, device=0,
                 stream=None, hbm_budget=0, max_batch=64, n_streams=2, queue_depth=4096,
                 tune_cache=None):
        L = lib()
        noise = np.ascontiguousarray(noise, np.float32)
        gain = np.ascontiguousarray(gain, np.float32)
        bad = np.ascontiguousarray(bad, np.uint8)
        n_strips = noise.size
        if n_strips % (CHANNELS_PER_FED * STRIPS_PER_CHANNEL):
            raise ValueError("noise size is not a whole number of FEDs")
        self.n_fed = n_strips // (CHANNELS_PER_FED * STRIPS_PER_CHANNEL)
        if gain.size != n_strips // 128 or bad.size != n_strips:
            raise ValueError("gain / bad sizes do not match noise")
        cal = ScCalib(self.n_fed, noise.ctypes.data, gain.ctypes.data, bad.ctypes.data,
                      t_seed, t_channel, t_cluster)
        torch = _torch()
        # the library works on this stream; before every call it waits for the caller's current
        # stream, so tensors torch has just filled are ready
        self.stream = stream if stream is not None else torch.cuda.Stream(device)
        opt = ScOptions()
        L.sc_default_options(ctypes.byref(opt))
        opt.device = device
        opt.stream = self.stream.cuda_stream
        opt.hbm_budget = hbm_budget
        opt.max_batch = max_batch
        opt.n_streams = n_streams
        opt.queue_depth = queue_depth
        self._tune_cache = tune_cache.encode() if tune_cache else None
        opt.tune_cache = self._tune_cache
        h = ctypes.c_void_p()
        rc = L.sc_create(ctypes.byref(cal), ctypes.byref(opt), ctypes.byref(h))
        if rc != SC_OK:
            raise ScError(rc, L.sc_last_error(None).decode())
        self._h = h
        self.device = device
        self._pending = {}

    # -- lifetime --
    def close(self):
        if getattr(self, "_h", None):
            lib().sc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def last_error(self) -> str:
        return lib().sc_last_error(self._h).decode()

    def _order(self):
        torch = _torch()
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def _check(self, rc, allowed=(SC_OK, SC_MALFORMED)):
        if rc not in allowed:
            raise ScError(rc, self.last_error())
        return rc

    # -- allocation helpers (torch memory) --
    def output(self, cap_cl, cap_adc, device=True, chan_status=False) -> Output:
        return Output(cap_cl, cap_adc, self.n_fed, device=device, chan_status=chan_status,
                      device_name=f"cuda:{self.device}")

    def dense_buffer(self, device=True):
        n = self.n_fed * CHANNELS_PER_FED * STRIPS_PER_CHANNEL
        if device:
            torch = _torch()
            return torch.zeros(n, dtype=torch.uint8, device=f"cuda:{self.device}")
        return np.zeros(n, np.uint8)

    # -- the path --
    def unpack(self, ev: Event, dense=None, chan_status=None):
        """§2 unpacking: ZS event -> dense per-strip ADCs (+ per-channel status)."""
        if dense is None:
            dense = self.dense_buffer(device=_is_dev(ev.zs))
        out_mem = SC_MEM_DEVICE if _is_dev(dense) else SC_MEM_HOST
        self._order()
        e = ev.c()
        rc = lib().sc_unpack(self._h, ctypes.byref(e), _ptr(dense), _ptr(chan_status), out_mem)
        self._check(rc)
        return dense, rc

    def cluster(self, dense, out: Output):
        """§2 clustering from dense ADCs. Returns the status (OK or OVERFLOW)."""
        in_mem = SC_MEM_DEVICE if _is_dev(dense) else SC_MEM_HOST
        self._order()
        rc = lib().sc_cluster(self._h, _ptr(dense), in_mem, ctypes.byref(out.cs))
        return self._check(rc, (SC_OK, SC_ERR_OVERFLOW))

    def process_events(self, events, outs):
        """Fused unpack + cluster of several events in one launch. Returns (status, per-event
        statuses)."""
        n = len(events)
        evs = (ScEvent * n)(*[e.c() for e in events])
        cs = (ScClusters * n)(*[o.cs for o in outs])
        sts = (ctypes.c_int * n)()
        self._order()
        rc = lib().sc_process_events(self._h, evs, n, cs, sts)
        for o, c in zip(outs, cs):
            o.cs.n_cl, o.cs.n_adc = c.n_cl, c.n_adc
        self._check(rc, (SC_OK, SC_MALFORMED, SC_ERR_OVERFLOW))
        return rc, list(sts)

    def process_pipelined(self, events, outs, batch):
        """Host ingest overlapped with compute: the events as consecutive batches of `batch`,
        batch k+1 sent to the device while batch k runs. Returns (status, per-event statuses)."""
        n = len(events)
        evs = (ScEvent * n)(*[e.c() for e in events])
        cs = (ScClusters * n)(*[o.cs for o in outs])
        sts = (ctypes.c_int * n)()
        self._order()
        rc = lib().sc_process_pipelined(self._h, evs, n, cs, batch, sts)
        for o, c in zip(outs, cs):
            o.cs.n_cl, o.cs.n_adc = c.n_cl, c.n_adc
        self._check(rc, (SC_OK, SC_MALFORMED, SC_ERR_OVERFLOW))
        return rc, list(sts)

    def batch(self, events, outs) -> "Batch":
        """Marshals events and outputs once for repeated process_batch calls (the outputs then
        read their counts from the batch's argument array)."""
        return Batch(events, outs)

    def process_batch(self, b: "Batch"):
        """process_events on a prepared Batch. Returns (status, per-event statuses)."""
        self._order()
        rc = lib().sc_process_events(self._h, b.c_ev, b.n, b.c_out, b.c_st)
        self._check(rc, (SC_OK, SC_MALFORMED, SC_ERR_OVERFLOW))
        return rc, list(b.c_st)

    def _ready_for_server(self):
        # the server runs on streams of its own: make everything queued so far finish first
        _torch().cuda.current_stream(self.device).synchronize()

    def submit(self, ev: Event, out: Output) -> int:
        self._ready_for_server()
        e = ev.c()
        t = ctypes.c_uint64()
        rc = lib().sc_submit(self._h, ctypes.byref(e), ctypes.byref(out.cs), ctypes.byref(t))
        if rc != SC_OK:
            raise ScError(rc, self.last_error())
        self._pending[t.value] = (ev, out, e)    # keep buffers alive until polled
        return t.value

    def try_submit(self, ev: Event, out: Output):
        """Like submit, but returns (status, ticket) instead of raising on AGAIN/BUDGET."""
        self._ready_for_server()
        e = ev.c()
        t = ctypes.c_uint64()
        rc = lib().sc_submit(self._h, ctypes.byref(e), ctypes.byref(out.cs), ctypes.byref(t))
        if rc == SC_OK:
            self._pending[t.value] = (ev, out, e)
        return rc, t.value

    def poll(self, ticket: int, timeout_us: int = -1) -> int:
        rc = lib().sc_poll(self._h, ticket, timeout_us)
        if rc != SC_PENDING:
            self._pending.pop(ticket, None)
        return rc

    def serve_replay(self, events, outs, n, rate_hz, seed=11489, phases=False):
        """Open-loop Poisson load on the server. Returns (status, latencies_us[n], events/s), and
        with phases=True also an [n, 3] array: arrival to submit, submit to launch, device time
        of the event's batch (microseconds)."""
        self._ready_for_server()
        evs = (ScEvent * len(events))(*[e.c() for e in events])
        cs = (ScClusters * len(outs))(*[o.cs for o in outs])
        lat = (ctypes.c_double * n)()
        ph = (ctypes.c_double * (3 * n))() if phases else None
        eps = ctypes.c_double()
        rc = lib().sc_serve_replay(self._h, evs, len(events), cs, len(outs), n, rate_hz, seed,
                                   lat, ph, ctypes.byref(eps))
        for o, c in zip(outs, cs):
            o.cs.n_cl, o.cs.n_adc = c.n_cl, c.n_adc
        self._check(rc, (SC_OK, SC_MALFORMED, SC_ERR_OVERFLOW))
        lat = np.frombuffer(lat, dtype=np.float64).copy()
        if phases:
            return rc, lat, eps.value, np.frombuffer(ph, dtype=np.float64).reshape(n, 3).copy()
        return rc, lat, eps.value

    # -- tuning / stats --
    @property
    def tuning(self) -> dict:
        t = ScTuning()
        self._check(lib().sc_get_tuning(self._h, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in ScTuning._fields_}

    @tuning.setter
    def tuning(self, d: dict):
        cur = self.tuning
        cur.update(d)
        t = ScTuning(*[cur[f] for f, _ in ScTuning._fields_])
        self._check(lib().sc_set_tuning(self._h, ctypes.byref(t)))

    def autotune(self, events) -> dict:
        n = len(events)
        evs = (ScEvent * n)(*[e.c() for e in events])
        t = ScTuning()
        self._order()
        self._check(lib().sc_autotune(self._h, evs, n, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in ScTuning._fields_}

    def set_modules(self, channel_module):
        """Module rows from the module of every FED channel (uint32 [n_fed * 96]); None turns
        them off."""
        if channel_module is None:
            self._check(lib().sc_set_modules(self._h, None))
            return
        cm = np.ascontiguousarray(channel_module, np.uint32)
        if cm.size != self.n_fed * CHANNELS_PER_FED:
            raise ValueError("channel_module must have n_fed * 96 entries")
        self._check(lib().sc_set_modules(self._h, cm.ctypes.data))

    def set_geometry(self, geom):
        """Module geometry (channel_module, channel_first, module_strips, origin [M, 3], u_dir
        [M, 3], pitch) for cluster_hits, kept on the device."""
        arrs = (np.ascontiguousarray(geom.channel_module, np.uint32),
                np.ascontiguousarray(geom.channel_first, np.uint32),
                np.ascontiguousarray(geom.module_strips, np.uint32),
                np.ascontiguousarray(geom.origin, np.float32).reshape(-1),
                np.ascontiguousarray(geom.u_dir, np.float32).reshape(-1),
                np.ascontiguousarray(geom.pitch, np.float32))
        if arrs[0].size != self.n_fed * CHANNELS_PER_FED or arrs[1].size != arrs[0].size:
            raise ValueError("channel tables must have n_fed * 96 entries")
        n_mod = arrs[2].size
        if arrs[3].size != 3 * n_mod or arrs[4].size != 3 * n_mod or arrs[5].size != n_mod:
            raise ValueError("module tables must have n_modules entries (x3 for vectors)")
        g = ScGeometry(n_mod, *[a.ctypes.data for a in arrs])
        self._check(lib().sc_set_geometry(self._h, ctypes.byref(g)))

    def cluster_hits(self, outs, hits=None):
        """Global hits of the clusters of device outputs: one float32 [n_cl, 4] tensor per output
        (x, y, z, u in cm), allocated here unless given."""
        torch = _torch()
        n = len(outs)
        if hits is None:
            hits = [torch.empty((max(1, min(o.cs.n_cl, o.cs.cap_cl)), 4), dtype=torch.float32,
                                device=self.device) for o in outs]
        cs = (ScClusters * n)(*[o.cs for o in outs])
        ptrs = (ctypes.c_void_p * n)(*[h.data_ptr() for h in hits])
        self._order()
        self._check(lib().sc_cluster_hits(self._h, cs, n, ptrs))
        return [h[:min(o.cs.n_cl, o.cs.cap_cl)] for h, o in zip(hits, outs)]

    def stats(self) -> dict:
        s = ScStats()
        self._check(lib().sc_get_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ScStats._fields_}


def safe_caps(ev: Event) -> tuple[int, int]:
    """Capacities that always suffice: clusters and member ADCs never exceed the digi count,
    which never exceeds the event's ZS bytes."""
    fo = ev.fed_offset
    span = int(fo.max()) if isinstance(fo, np.ndarray) else int(fo.max().item())
    return max(span, 1), max(span, 1)
