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


# ---- runs at the cluster threshold -----------------------------------------------------------

def sqrt_f32(x: np.float32) -> np.float32:
    """Correctly rounded binary32 square root (numpy's float32 sqrt is IEEE)."""
    return np.sqrt(np.float32(x), dtype=np.float32)


def noise_sum(noises, s=np.float32(0.0)) -> np.float32:
    """Sequential fmaf sum of the noise squares from the first strip, exact binary32 rounding."""
    for n in noises:
        s = fmaf_exact(np.float32(n), np.float32(n), s)
    return s


def bound_of(s: np.float32, t: float) -> np.float32:
    """fl(t * sqrtf(S)): the right-hand side of the cluster threshold."""
    return np.float32(np.float32(t) * sqrt_f32(s))


def threshold_runs(seed: int, t_cluster=5.0, lengths=(1, 2, 3, 4, 5, 7, 9, 15, 31, 33, 63, 64,
                                                       65, 66, 100, 129, 200, 250)):
    """One FED of runs whose charge sits at the cluster threshold: for each run the charge Q (sum
    of its ADCs) equals fl(t * sqrtf(S)) exactly, or lies one binary32 step above or below it
    (S: sequential fmaf sum of the noise squares). Noise is proportional to the ADC (n = c * a with
    c <= sqrt(L) / t < 3.2), so every strip is active and a seed for thresholds t_channel = 0.25,
    t_seed = 0.3; the last strip's noise is stepped ulp by ulp towards the wanted bound. Returns
    ({channel: [(first, adcs)]}, noise, runs) with runs as tuples (channel, first, length, Q,
    bound)."""
    rng = np.random.default_rng(seed)
    noise, _, _ = calib_arrays(1)
    chan_runs, runs = {}, []
    k = 0
    for ch in range(NCH):
        pos = 0
        while True:
            L = int(lengths[rng.integers(len(lengths))])
            if pos + L > NS:
                break
            adcs = [int(v) for v in rng.integers(1, 31, size=L)]
            q = sum(adcs)
            c = q / (t_cluster * float(np.sqrt(np.sum(np.square(adcs, dtype=np.float64)))))
            ns = [np.float32(c * a) for a in adcs]
            s_prev = noise_sum(ns[:-1])
            want = (np.float32(q) if k % 3 == 0 else
                    np.nextafter(np.float32(q), np.float32(np.inf if k % 3 == 1 else -np.inf)))
            best, best_d = None, None
            n_last = ns[-1]
            for _ in range(64):
                r = bound_of(fmaf_exact(n_last, n_last, s_prev), t_cluster)
                d = float(r) - float(want)
                if best_d is None or abs(d) < abs(best_d):
                    best, best_d = n_last, d
                if d == 0:
                    break
                n_last = np.nextafter(n_last, np.float32(-np.inf if d > 0 else np.inf))
            ns[-1] = best
            noise[ch * NS + pos: ch * NS + pos + L] = ns
            chan_runs.setdefault(ch, []).append((pos, adcs))
            runs.append((ch, pos, L, q, bound_of(fmaf_exact(best, best, s_prev), t_cluster)))
            k += 1
            pos += L + 1
    return chan_runs, noise, runs
