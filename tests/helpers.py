"""Input construction and exact-arithmetic helpers for tests (no clustering logic here)."""
from __future__ import annotations

from fractions import Fraction

import numpy as np

import fedgen

NCH = fedgen.CHANNELS_PER_FED
NS = fedgen.STRIPS_PER_CHANNEL


def calib_arrays(n_fed=1, noise=1.0, gain=1.0):
    n = n_fed * NCH * NS
    noise_a = np.full(n, noise, dtype=np.float32)
    gain_a = np.full(n // 128, gain, dtype=np.float32)
    bad_a = np.zeros(n, dtype=np.uint8)
    return noise_a, gain_a, bad_a


def event_from_runs(channel_runs: dict, n_fed=1):
    """channel_runs: {global_channel: [(first, [adc, ...]), ...]} -> (zs, fed_offset)."""
    feds = []
    for f in range(n_fed):
        recs = [fedgen.encode_channel_runs(channel_runs.get(f * NCH + ch, []))
                for ch in range(NCH)]
        feds.append(recs)
    return fedgen.assemble_feds(feds)


def event_from_dense(dense: np.ndarray):
    """Canonical ZS encoding of dense rows (every nonzero strip written)."""
    rows = dense.reshape(-1, NS)
    return fedgen.encode_dense(rows, rows > 0)


# ---- exact IEEE-754 binary32 rounding, for brute-force references ---------------------------

def round_f32(x: Fraction) -> np.float32:
    """Round an exact rational to the nearest binary32 (ties to even), with subnormals and
    overflow to infinity."""
    if x == 0:
        return np.float32(0.0)
    sign = -1 if x < 0 else 1
    x = abs(x)
    # exponent e with 2^e <= x < 2^(e+1)
    e = x.numerator.bit_length() - x.denominator.bit_length()
    if Fraction(2) ** e > x:
        e -= 1
    e = max(e, -126)
    q = x / (Fraction(2) ** (e - 23))          # scaled so the integer part has 24 bits
    m = q.numerator // q.denominator
    rem = q - m
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and m % 2 == 1):
        m += 1
    val = Fraction(m) * Fraction(2) ** (e - 23)
    if val >= Fraction(2) ** 128:
        return np.float32(sign * np.inf)
    return np.float32(sign * float(val))


def fmaf_exact(a: np.float32, b: np.float32, c: np.float32) -> np.float32:
    return round_f32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


# ---- golden fixture parsing ----------------------------------------------------------------

def parse_hex(spec: str) -> bytes:
    """Space-separated hex tokens; ``xx*N`` repeats a byte (or byte group) N times."""
    out = bytearray()
    for tok in spec.split():
        if "*" in tok:
            h, n = tok.split("*")
            out += bytes.fromhex(h) * int(n)
        else:
            out += bytes.fromhex(tok)
    return bytes(out)


def parse_channel_set(spec, n_max=None):
    if isinstance(spec, str):
        lo, hi = spec.split("-")
        return list(range(int(lo), int(hi) + 1))
    return list(spec)


def golden_event(case: dict):
    """(zs, fed_offset, n_fed) of a golden case given as per-channel records, per-channel runs
    or raw FED hex."""
    if "fed_hex" in case:
        blobs = [parse_hex(h) for h in case["fed_hex"]]
        zs = np.frombuffer(b"".join(blobs), dtype=np.uint8).copy()
        if "fed_offset" in case:
            fo = np.array(case["fed_offset"], dtype=np.uint64)
        else:
            fo = np.zeros(len(blobs) + 1, dtype=np.uint64)
            fo[1:] = np.cumsum([len(b) for b in blobs])
        return zs, fo, len(fo) - 1
    chans = set()
    for key in ("records", "runs"):
        chans |= {int(c) for c in case.get(key, {})}
    n_fed = max(1, (max(chans) // NCH + 1) if chans else 1)
    feds = []
    for f in range(n_fed):
        recs = []
        for ch in range(NCH):
            g = str(f * NCH + ch)
            if g in case.get("records", {}):
                recs.append(parse_hex(case["records"][g]))
            elif g in case.get("runs", {}):
                recs.append(fedgen.encode_channel_runs([(r[0], r[1]) for r in case["runs"][g]]))
            else:
                recs.append(b"\x00\x00")
        feds.append(recs)
    zs, fo = fedgen.assemble_feds(feds)
    return zs, fo, n_fed


def _f(v):
    return float(v) if not isinstance(v, str) else float(v)


def golden_calib(case: dict, n_fed: int):
    noise, gain, bad = calib_arrays(n_fed)
    for ch, first, count, val in case.get("noise", []):
        noise[ch * NS + first: ch * NS + first + count] = np.float32(_f(val))
    for apv, val in case.get("gain", []):
        gain[apv] = np.float32(_f(val))
    for ch, s in case.get("bad", []):
        bad[ch * NS + s] = 1
    return noise, gain, bad
