"""Seeded synthetic strip-tracker data: calibration tables and zero-suppressed FED buffers.

This module is the only code shared by the oracle side and the GPU side of the tests and the
benchmark. It produces inputs; it holds none of the unpacking or clustering arithmetic.

Detector organisation (paper §2, Parallelization): a FED reads 96 optical channels of 256 strips.
A readout chip (APV) serves 128 strips, so each channel holds two APVs.

Zero-suppressed (ZS) byte format written here (paper §2 describes it only as a variant of CSR
with channel = row and strip = column; Fig. 1 is not reproduced, so the concrete bytes are this
project's reading):
  * a FED buffer is its 96 channel records back to back, channel 0 first, no header or trailer;
  * a channel record is a little-endian u16 ``P`` (number of payload bytes that follow), then the
    payload: zero or more runs ``(u8 first_strip, u8 count, count x u8 ADC)`` in increasing strip
    order; runs longer than 255 strips are carried as adjacent runs.

Synthetic workload (the paper's simulated ttbar sample with 70 pile-up interactions is not
available; these distributions stand in for it):
  * calibration: noise ~ U[lo, hi] FP32 ADC counts per strip, gain ~ N(1, 0.05) FP32 per APV,
    bad ~ Bernoulli(p_bad) per strip;
  * hits: each strip starts a hit with probability ``occ``; width = min(Geometric(p), cap)
    (support >= 1); charge ~ LogNormal(ln 90, 0.5) ADC split equally over the width and cut at the
    channel end; overlapping hits add;
  * signal: x = gain(apv) * deposit + noise * N(0, 1) on every strip, ADC = clamp(rint(x), 0, 255);
  * the front end keeps a strip in the ZS record when its ADC exceeds twice its noise (FP32).

Synthetic geometry (the paper's next step converts clusters to global hit coordinates; the real
tracker geometry and cabling are not available, so this layout stands in for them):
  * modules: each block of 24 consecutive channels of a FED is cut into modules of 2 or 3
    consecutive channels (512 or 768 strips), sizes drawn at random; a channel's strips start at
    256 x (its place in the module) in module strip numbering;
  * placement: barrel-like; a module sits on one of ten layers of radius 25 to 110 cm, at a
    random azimuth phi and z in [-100, 100] cm; its strips run along z, so the measurement
    direction is the tangent (-sin phi, cos phi, 0), tilted out of the transverse plane by a
    random angle in [-0.1, 0.1] rad; pitch 80 um on the four inner layers, 120 um on the next
    three and 183 um on the outer three.

Random streams: ``numpy.random.Generator(PCG64(SeedSequence([11489, config_id, stream, index])))``
with stream 0 = calibration, stream 1 = event ``index``, stream 2 = geometry.
"""
from __future__ import annotations

import dataclasses
import math
from concurrent.futures import ProcessPoolExecutor
from typing import Iterable, Sequence

import numpy as np

CHANNELS_PER_FED = 96
STRIPS_PER_CHANNEL = 256
STRIPS_PER_APV = 128
STRIPS_PER_FED = CHANNELS_PER_FED * STRIPS_PER_CHANNEL
MAX_RUN = 255
SEED_ROOT = 11489

__all__ = [
    "CHANNELS_PER_FED", "STRIPS_PER_CHANNEL", "STRIPS_PER_APV", "STRIPS_PER_FED",
    "GenConfig", "CONFIGS", "Calibration", "Event", "make_calibration", "make_event",
    "make_events", "encode_dense", "encode_channel_runs", "assemble_feds", "rng_for",
    "Geometry", "make_geometry", "MODULE_BLOCK",
]

MODULE_BLOCK = 24   # modules never cross a multiple of 24 channels of a FED


@dataclasses.dataclass(frozen=True)
class GenConfig:
    """One synthetic workload. ``occ`` is a fixed occupancy, or None when ``occ_sampler`` draws one
    per event."""

    config_id: int
    name: str
    n_fed: int
    n_events: int
    occ: float | None = 0.01
    occ_sampler: str = "fixed"          # "fixed" | "loguniform" | "mix"
    occ_range: tuple[float, float] = (0.005, 0.05)
    occ_mix: tuple[tuple[float, float], ...] = ()
    width_p: float = 0.5
    width_cap: int = 8
    charge_median: float = 90.0
    charge_sigma_ln: float = 0.5
    noise_lo: float = 3.0
    noise_hi: float = 6.0
    gain_mu: float = 1.0
    gain_sigma: float = 0.05
    p_bad: float = 0.001
    zs_factor: float = 2.0

    @property
    def n_channels(self) -> int:
        return self.n_fed * CHANNELS_PER_FED

    @property
    def n_strips(self) -> int:
        return self.n_channels * STRIPS_PER_CHANNEL

    def with_(self, **kw) -> "GenConfig":
        return dataclasses.replace(self, **kw)


CONFIGS: dict[int, GenConfig] = {
    0: GenConfig(0, "plain-50fed", n_fed=50, n_events=20, occ=0.01),
    1: GenConfig(1, "plain-full", n_fed=440, n_events=20, occ=0.015),
    2: GenConfig(2, "batched-full", n_fed=440, n_events=64, occ=None, occ_sampler="loguniform",
                 occ_range=(0.005, 0.05)),
    3: GenConfig(3, "serving-full", n_fed=440, n_events=2000, occ=None, occ_sampler="mix",
                 occ_mix=((0.005, 0.2), (0.015, 0.4), (0.03, 0.3), (0.06, 0.1))),
    4: GenConfig(4, "stress-full", n_fed=440, n_events=256, occ=0.06, width_p=0.25, width_cap=32,
                 p_bad=0.01, noise_lo=2.0, noise_hi=10.0),
}


def rng_for(config_id: int, stream: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(
        [SEED_ROOT, int(config_id), int(stream), int(index)])))


@dataclasses.dataclass
class Calibration:
    n_fed: int
    noise: np.ndarray   # float32 [n_fed*96*256]
    gain: np.ndarray    # float32 [n_fed*96*2]
    bad: np.ndarray     # uint8   [n_fed*96*256], != 0 means flagged bad


@dataclasses.dataclass
class Event:
    zs: np.ndarray          # uint8, all FED buffers back to back
    fed_offset: np.ndarray  # uint64 [n_fed+1]; FED f is zs[fed_offset[f]:fed_offset[f+1]]
    dense: np.ndarray       # uint8 [n_fed*96*256]: ADC of strips kept by the front end, else 0
    occ: float
    index: int

    @property
    def n_fed(self) -> int:
        return len(self.fed_offset) - 1

    @property
    def n_digis(self) -> int:
        return int(np.count_nonzero(self.dense))


def make_calibration(cfg: GenConfig) -> Calibration:
    rng = rng_for(cfg.config_id, 0, 0)
    n = cfg.n_strips
    noise = rng.uniform(cfg.noise_lo, cfg.noise_hi, size=n).astype(np.float32)
    gain = rng.normal(cfg.gain_mu, cfg.gain_sigma, size=n // STRIPS_PER_APV).astype(np.float32)
    bad = (rng.random(n) < cfg.p_bad).astype(np.uint8)
    return Calibration(cfg.n_fed, noise, gain, bad)


@dataclasses.dataclass
class Geometry:
    channel_module: np.ndarray   # uint32 [n_fed*96]: module of each channel
    channel_first: np.ndarray    # uint32 [n_fed*96]: module strip number of the channel's strip 0
    module_strips: np.ndarray    # uint32 [n_modules]: 512 or 768
    origin: np.ndarray           # float32 [n_modules, 3]: module centre, cm
    u_dir: np.ndarray            # float32 [n_modules, 3]: unit vector across the strips
    pitch: np.ndarray            # float32 [n_modules]: strip pitch, cm

    @property
    def n_modules(self) -> int:
        return int(self.module_strips.size)


def make_geometry(cfg: GenConfig) -> Geometry:
    rng = rng_for(cfg.config_id, 2, 0)
    sizes = []
    for _ in range(cfg.n_fed * (CHANNELS_PER_FED // MODULE_BLOCK)):
        left = MODULE_BLOCK
        while left:
            k = left if left in (2, 3) else 2 if left == 4 else int(rng.integers(2, 4))
            sizes.append(k)
            left -= k
    sizes = np.array(sizes, dtype=np.int64)
    n_mod = sizes.size
    channel_module = np.repeat(np.arange(n_mod), sizes).astype(np.uint32)
    starts = np.cumsum(sizes) - sizes
    channel_first = ((np.arange(channel_module.size) - np.repeat(starts, sizes))
                     * STRIPS_PER_CHANNEL).astype(np.uint32)
    radii = np.linspace(25.0, 110.0, 10)
    pitches = np.array([0.0080] * 4 + [0.0120] * 3 + [0.0183] * 3)
    layer = rng.integers(0, 10, size=n_mod)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n_mod)
    z = rng.uniform(-100.0, 100.0, size=n_mod)
    tilt = rng.uniform(-0.1, 0.1, size=n_mod)
    r = radii[layer]
    origin = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1).astype(np.float32)
    u_dir = np.stack([-np.sin(phi) * np.cos(tilt), np.cos(phi) * np.cos(tilt), np.sin(tilt)],
                     axis=1).astype(np.float32)
    return Geometry(channel_module, channel_first,
                    (sizes * STRIPS_PER_CHANNEL).astype(np.uint32), origin, u_dir,
                    pitches[layer].astype(np.float32))


def _event_occupancy(cfg: GenConfig, rng: np.random.Generator) -> float:
    if cfg.occ_sampler == "fixed":
        return float(cfg.occ)
    if cfg.occ_sampler == "loguniform":
        lo, hi = cfg.occ_range
        return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))
    if cfg.occ_sampler == "mix":
        vals = np.array([v for v, _ in cfg.occ_mix])
        probs = np.array([p for _, p in cfg.occ_mix])
        return float(vals[rng.choice(len(vals), p=probs / probs.sum())])
    raise ValueError(cfg.occ_sampler)


def make_event(cfg: GenConfig, calib: Calibration, index: int) -> Event:
    rng = rng_for(cfg.config_id, 1, index)
    occ = _event_occupancy(cfg, rng)
    n = cfg.n_strips
    # hit starts, widths and charges
    starts = np.flatnonzero(rng.random(n) < occ)
    n_hits = starts.size
    widths = np.minimum(rng.geometric(cfg.width_p, size=n_hits), cfg.width_cap).astype(np.int64)
    charges = rng.lognormal(math.log(cfg.charge_median), cfg.charge_sigma_ln, size=n_hits)
    per_strip = charges / widths
    # expand each hit over its strips, dropping strips past the end of the channel
    hit_of = np.repeat(np.arange(n_hits), widths)
    within = np.arange(hit_of.size) - np.repeat(np.cumsum(widths) - widths, widths)
    strip = starts[hit_of] + within
    keep = (strip // STRIPS_PER_CHANNEL) == (starts[hit_of] // STRIPS_PER_CHANNEL)
    deposit = np.bincount(strip[keep], weights=per_strip[hit_of[keep]], minlength=n)
    # analogue signal with per-APV gain and per-strip Gaussian noise, digitised to 8 bits
    z = rng.standard_normal(n, dtype=np.float32)
    gain_strip = np.repeat(calib.gain, STRIPS_PER_APV)
    x = gain_strip * deposit.astype(np.float32) + calib.noise * z
    adc = np.clip(np.rint(x), 0, 255).astype(np.uint8)
    # front-end zero suppression
    kept = adc.astype(np.float32) > np.float32(cfg.zs_factor) * calib.noise
    dense = np.where(kept, adc, np.uint8(0)).astype(np.uint8)
    zs, fed_offset = encode_dense(dense.reshape(-1, STRIPS_PER_CHANNEL),
                                  kept.reshape(-1, STRIPS_PER_CHANNEL))
    return Event(zs, fed_offset, dense, occ, index)


def _make_event_job(args):
    cfg, calib, index = args
    return make_event(cfg, calib, index)


def make_events(cfg: GenConfig, calib: Calibration, indices: Iterable[int],
                workers: int = 1) -> list[Event]:
    indices = list(indices)
    if workers <= 1 or len(indices) <= 1:
        return [make_event(cfg, calib, i) for i in indices]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_make_event_job, [(cfg, calib, i) for i in indices]))


def encode_dense(adc: np.ndarray, mask: np.ndarray, max_run: int = MAX_RUN):
    """Encode channels (rows of 256 strips) into ZS FED buffers.

    ``adc`` u8 [n_channels, 256]; ``mask`` bool of the same shape selects the strips written.
    Maximal runs of selected strips become runs; a run longer than ``max_run`` is split into
    adjacent runs. ``n_channels`` must be a multiple of 96. Returns ``(zs u8, fed_offset u64)``.
    """
    adc = np.ascontiguousarray(adc, dtype=np.uint8)
    mask = np.ascontiguousarray(mask, dtype=bool)
    n_ch = adc.shape[0]
    assert adc.shape == (n_ch, STRIPS_PER_CHANNEL) and mask.shape == adc.shape
    assert n_ch % CHANNELS_PER_FED == 0
    assert 1 <= max_run <= 255
    m = np.zeros((n_ch, STRIPS_PER_CHANNEL + 2), dtype=np.int8)
    m[:, 1:-1] = mask
    d = np.diff(m, axis=1)
    sch, sstart = np.nonzero(d == 1)
    ech, send = np.nonzero(d == -1)
    assert np.array_equal(sch, ech)
    run_len = send - sstart
    pieces = (run_len + max_run - 1) // max_run
    run_of = np.repeat(np.arange(run_len.size), pieces)
    k = np.arange(run_of.size) - np.repeat(np.cumsum(pieces) - pieces, pieces)
    p_ch = sch[run_of]
    p_first = sstart[run_of] + k * max_run
    p_count = np.minimum(run_len[run_of] - k * max_run, max_run)
    # payload bytes per channel and byte positions
    p_bytes = 2 + p_count
    payload = np.bincount(p_ch, weights=p_bytes, minlength=n_ch).astype(np.int64)
    rec = 2 + payload
    ch_start = np.cumsum(rec) - rec
    total = int(rec.sum())
    out = np.zeros(total, dtype=np.uint8)
    out[ch_start] = (payload & 0xFF).astype(np.uint8)
    out[ch_start + 1] = (payload >> 8).astype(np.uint8)
    # position of each piece inside its channel payload (segmented exclusive scan)
    csum = np.cumsum(p_bytes) - p_bytes
    first_piece = np.searchsorted(p_ch, p_ch, side="left")
    piece_pos = ch_start[p_ch] + 2 + (csum - csum[first_piece])
    out[piece_pos] = p_first.astype(np.uint8)
    out[piece_pos + 1] = p_count.astype(np.uint8)
    # ADC bytes
    strip_in_piece = np.arange(int(p_count.sum())) - np.repeat(np.cumsum(p_count) - p_count, p_count)
    sel_ch = np.repeat(p_ch, p_count)
    sel_s = np.repeat(p_first, p_count) + strip_in_piece
    out[np.repeat(piece_pos + 2, p_count) + strip_in_piece] = adc[sel_ch, sel_s]
    fed_bytes = rec.reshape(-1, CHANNELS_PER_FED).sum(axis=1)
    fed_offset = np.zeros(fed_bytes.size + 1, dtype=np.uint64)
    fed_offset[1:] = np.cumsum(fed_bytes)
    return out, fed_offset


def encode_channel_runs(runs: Sequence[tuple[int, Sequence[int]]]) -> bytes:
    """One channel record from explicit runs ``[(first, [adc, ...]), ...]``, written as given
    (no merging, no validation), for hand-built test inputs."""
    payload = bytearray()
    for first, adcs in runs:
        payload += bytes([first & 0xFF, len(adcs) & 0xFF]) + bytes(int(a) & 0xFF for a in adcs)
    return len(payload).to_bytes(2, "little") + bytes(payload)


def assemble_feds(feds: Sequence[Sequence[bytes] | bytes]):
    """Concatenate FED buffers. Each item is either raw FED bytes or a list of channel records
    (missing channels at the end are filled with empty records). Returns ``(zs, fed_offset)``."""
    blobs = []
    for f in feds:
        if isinstance(f, (bytes, bytearray)):
            blobs.append(bytes(f))
        else:
            recs = list(f) + [b"\x00\x00"] * (CHANNELS_PER_FED - len(f))
            blobs.append(b"".join(recs))
    fed_offset = np.zeros(len(blobs) + 1, dtype=np.uint64)
    fed_offset[1:] = np.cumsum([len(b) for b in blobs])
    zs = np.frombuffer(b"".join(blobs), dtype=np.uint8).copy()
    return zs, fed_offset
