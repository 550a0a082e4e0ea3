"""Pins of the module-aware oracle (readings M1-M4 in oracle.c): a run of active strips goes on
across the edge between two channels of one FED that read the same module.

Pinned by hand-worked rows, a brute-force interval enumeration over windows that straddle
channel edges (exact rationals, a different algorithm), invariants on generated events with the
synthetic module map, and the reduction to the plain oracle when no channel is joined.
"""
from fractions import Fraction

import numpy as np
import pytest

import fedgen
import oracle
from helpers import NCH, NS, calib_arrays, event_from_dense, fmaf_exact, round_f32


def _run(dense, noise, gain, bad, joins):
    zs, fo = event_from_dense(dense)
    return oracle.process_event(zs, fo, noise, gain, bad, joins=joins)


def _recs(out):
    return [(int(r["channel"]), int(r["first"]), int(r["width"]), int(r["charge"]),
             float(r["barycenter"])) for r in out.cl]


def _setup(n_fed=1, noise=1.0):
    noise_a, gain_a, bad_a = calib_arrays(n_fed, noise=noise)
    dense = np.zeros(n_fed * NCH * NS, np.uint8)
    joins = np.zeros(n_fed * NCH, np.uint8)
    return dense, noise_a, gain_a, bad_a, joins


def _f32(x):
    return float(np.float32(float(Fraction(x))))


# ---- hand-worked rows (noise 1, gain 1 unless stated; thresholds 3 / 2 / 5) ---------------------

def test_run_across_a_joined_edge_is_one_cluster():
    dense, noise, gain, bad, joins = _setup()
    dense[253:256] = 10                      # channel 0, strips 253-255
    dense[NS:NS + 2] = 10                    # channel 1, strips 0-1
    joins[1] = 1                             # channel 1 continues channel 0's module
    # one run of 5 strips: Q = 50 >= 5 sqrt(5); strips 253..257 of channel 0's numbering,
    # barycenter (253.5 + ... + 257.5) / 5 = 255.5
    assert _recs(_run(dense, noise, gain, bad, joins)) == [(0, 253, 5, 50, 255.5)]
    # without the join the channel edge stops it: two clusters
    assert _recs(_run(dense, noise, gain, bad, None)) == [(0, 253, 3, 30, 254.5),
                                                          (1, 0, 2, 20, 1.0)]


def test_seed_on_the_far_side_of_the_edge():
    dense, noise, gain, bad, joins = _setup()
    dense[255] = 3            # channel 0 strip 255: active (3 > 2), no seed (3 > 3 is false)
    dense[NS] = 9             # channel 1 strip 0: seed
    joins[1] = 1
    # Q = 12 >= 5 sqrt(2); barycenter (255.5 * 3 + 256.5 * 9) / 12 = 3075 / 12 = 256.25
    assert _recs(_run(dense, noise, gain, bad, joins)) == [(0, 255, 2, 12, 256.25)]
    # unjoined: the lone strip of channel 0 has no seed; channel 1's strip stands alone
    assert _recs(_run(dense, noise, gain, bad, None)) == [(1, 0, 1, 9, 0.5)]


def test_cluster_threshold_over_the_joined_run():
    dense, noise, gain, bad, joins = _setup(noise=2.0)
    dense[255] = 7            # seed (7 > 6)
    dense[NS:NS + 2] = 6      # active, not seeds (6 > 6 is false)
    joins[1] = 1
    # joined: Q = 19, S = 4 + 4 + 4 = 12, 5 sqrt(12) = 17.32 <= 19: accepted
    # barycenter (255.5 * 7 + 256.5 * 6 + 257.5 * 6) / 19 = 4872.5 / 19 = 9745 / 38
    assert _recs(_run(dense, noise, gain, bad, joins)) == [(0, 255, 3, 19, _f32(Fraction(9745, 38)))]
    # unjoined: channel 0's run (Q = 7 < 5 sqrt(4) = 10) fails the threshold and channel 1's
    # run has no seed
    assert _recs(_run(dense, noise, gain, bad, None)) == []


def test_each_member_keeps_its_own_apv_gain():
    dense, noise, gain, bad, joins = _setup()
    gain[1] = 2.0             # channel 0, APV 1 (strips 128-255)
    gain[2] = 0.5             # channel 1, APV 0 (strips 0-127)
    dense[254:256] = 20
    dense[NS] = 20
    joins[1] = 1
    # corrected ADCs 10, 10, 40; charge 60; barycenter (254.5*10 + 255.5*10 + 256.5*40) / 60 = 256
    out = _run(dense, noise, gain, bad, joins)
    assert _recs(out) == [(0, 254, 3, 60, 256.0)]
    assert out.adc.tolist() == [10, 10, 40]


def test_module_edge_and_bad_strip_stop_the_run():
    dense, noise, gain, bad, joins = _setup()
    joins[1] = 1              # module = channels 0, 1; channel 2 starts another module
    dense[NS + 255] = 10      # channel 1 strip 255
    dense[2 * NS] = 10        # channel 2 strip 0 (not joined)
    dense[255] = 10           # channel 0 strip 255
    bad[NS] = 1               # channel 1 strip 0 is bad: the joined run stops before it
    dense[NS] = 10
    dense[NS + 1] = 10        # channel 1 strip 1
    assert _recs(_run(dense, noise, gain, bad, joins)) == [
        (0, 255, 1, 10, 255.5), (1, 1, 1, 10, 1.5), (1, 255, 1, 10, 255.5), (2, 0, 1, 10, 0.5)]


def test_full_three_channel_module():
    dense, noise, gain, bad, joins = _setup()
    dense[3 * NS:6 * NS] = 10     # channels 3, 4, 5 all active
    joins[4] = joins[5] = 1
    # one cluster of 768 strips from channel 3 strip 0: charge 7680, barycenter 384
    out = _run(dense, noise, gain, bad, joins)
    assert _recs(out) == [(3, 0, 768, 7680, 384.0)]
    assert out.adc.size == 768


def test_joins_do_not_cross_feds():
    dense, noise, gain, bad, joins = _setup(n_fed=2)
    dense[NCH * NS - 1] = 10      # FED 0, channel 95, strip 255
    dense[NCH * NS] = 10          # FED 1, channel 0, strip 0
    joins[NCH] = 1                # ignored on a FED's first channel
    assert _recs(_run(dense, noise, gain, bad, joins)) == [(95, 255, 1, 10, 255.5),
                                                           (96, 0, 1, 10, 0.5)]


def test_capacity_counts_a_wide_cluster():
    dense, noise, gain, bad, joins = _setup()
    dense[:2 * NS] = 10
    joins[1] = 1
    adc, _, _ = oracle.unpack(*event_from_dense(dense))
    out = oracle.cluster(adc, noise, gain, bad, cap_cl=1, cap_adc=100, joins=joins)
    assert out.status == -2 and out.cl.size == 1 and out.adc.size == 100


# ---- brute force over windows that straddle channel edges -----------------------------------

def _brute_force_row(a, n, g, bad, t_seed=3.0, t_ch=2.0, t_cl=5.0):
    """Every interval [l, r] of one row (consecutive channels of a module) that satisfies the
    cluster definition, exact rationals standing in for FP32 where a rounding decides."""
    L = a.size
    T_ch, T_sd, T_cl = np.float32(t_ch), np.float32(t_seed), np.float32(t_cl)

    def usable(s):
        gs = g[s // 128]
        return (bad[s] == 0 and not np.isnan(n[s]) and n[s] >= 0 and not np.isinf(n[s])
                and not np.isnan(gs) and gs > 0)

    act = [usable(s) and Fraction(int(a[s])) > Fraction(float(T_ch * n[s])) for s in range(L)]
    sd = [act[s] and Fraction(int(a[s])) > Fraction(float(T_sd * n[s])) for s in range(L)]
    out = []
    for l in range(L):
        if not act[l] or (l > 0 and act[l - 1]):
            continue
        r = l
        while r + 1 < L and act[r + 1]:
            r += 1
        if not any(sd[l:r + 1]):
            continue
        q = sum(int(x) for x in a[l:r + 1])
        S = np.float32(0)
        for s in range(l, r + 1):
            S = fmaf_exact(n[s], n[s], S)
        root = np.float32(np.sqrt(np.float64(S)))
        if not Fraction(q) >= Fraction(float(T_cl * root)):
            continue
        cs = []
        for s in range(l, r + 1):
            v = Fraction(float(round_f32(Fraction(int(a[s])) / Fraction(float(g[s // 128])))))
            fl = int(v)
            frac = v - fl
            cs.append(min(fl + (1 if frac > Fraction(1, 2) or (frac == Fraction(1, 2) and fl % 2)
                                else 0), 65535))
        tot = sum(cs)
        off = (l // NS) * NS
        bary = (Fraction(sum((2 * (s - off) + 1) * c for s, c in zip(range(l, r + 1), cs)),
                         2 * tot) if tot else Fraction(l - off) + Fraction(r - l + 1, 2))
        out.append((l // NS, l % NS, r - l + 1, tot, bary, cs))
    return out


@pytest.mark.parametrize("edge_at", [250, 253, 255])
def test_brute_force_windows_across_joined_edges(edge_at):
    """Windows of strips edge_at..255 of each channel and 0..5 of the next, over rows of two and
    three channels (the generator's module map), random ADCs around each strip's thresholds,
    random noise, gains and bad flags."""
    rng = np.random.default_rng(2000 + edge_at)
    n_fed = 2
    geo = fedgen.make_geometry(fedgen.CONFIGS[0].with_(n_fed=n_fed))
    cm = geo.channel_module.astype(np.int64)
    joins = np.zeros(n_fed * NCH, np.uint8)
    joins[1:] = (cm[1:] == cm[:-1]) & (np.arange(1, n_fed * NCH) % NCH != 0)
    noise, gain, bad = calib_arrays(n_fed)
    noise[:] = rng.choice(np.array([0.75, 1.0, 1.5, 2.0, 3.0, 1.3, 2.7], np.float32),
                          size=noise.size)
    gain[:] = rng.choice(np.array([1.0, 2.0, 0.5, 1.1, 0.9], np.float32), size=gain.size)
    dense = np.zeros(n_fed * NCH * NS, np.uint8)
    for c in range(n_fed * NCH):
        for s in list(range(edge_at, NS)) + list(range(0, 6)):
            i = c * NS + s
            nz = noise[i]
            choices = [0, int(2 * nz), int(2 * nz) + 1, int(3 * nz), int(3 * nz) + 1, 255]
            dense[i] = choices[rng.integers(len(choices))]
            bad[i] = rng.random() < 0.1
    out = _run(dense, noise, gain, bad, joins)
    have = []
    k = 0
    for rec in out.cl:
        w = int(rec["width"])
        have.append((int(rec["channel"]), int(rec["first"]), w, int(rec["charge"]),
                     np.float32(rec["barycenter"]), out.adc[k:k + w].tolist()))
        k += w
    want = []
    c = 0
    n_cross = 0
    while c < n_fed * NCH:
        c1 = c + 1
        while c1 < n_fed * NCH and joins[c1]:
            c1 += 1
        sl = slice(c * NS, c1 * NS)
        for ch, first, w, q, b, cs in _brute_force_row(dense[sl], noise[sl],
                                                       gain[2 * c:2 * c1], bad[sl]):
            want.append((c + ch, first, w, q, np.float32(float(b)), cs))
            n_cross += first + w > NS
        c = c1
    assert have == want
    assert n_cross > 0           # the windows produce clusters that do cross an edge


# ---- generated events with the synthetic module map -----------------------------------------

@pytest.mark.parametrize("cfg_id", [0, 4])
def test_generated_events_invariants(cfg_id):
    cfg = fedgen.CONFIGS[cfg_id].with_(n_fed=20)
    cal = fedgen.make_calibration(cfg)
    geo = fedgen.make_geometry(cfg)
    cm = geo.channel_module.astype(np.int64)
    joins = np.zeros(cfg.n_channels, np.uint8)
    joins[1:] = (cm[1:] == cm[:-1]) & (np.arange(1, cfg.n_channels) % NCH != 0)
    ev = fedgen.make_event(cfg, cal, 3)
    mod = oracle.process_event(ev.zs, ev.fed_offset, cal.noise, cal.gain, cal.bad, joins=joins)
    plain = oracle.process_event(ev.zs, ev.fed_offset, cal.noise, cal.gain, cal.bad)
    ch, first, width = (mod.cl[f].astype(np.int64) for f in ("channel", "first", "width"))
    last_ch = ch + (first + width - 1) // NS
    # a cluster stays inside its module, and a record's channel is where it starts
    assert np.all(cm[last_ch] == cm[ch]) and np.all(first < NS)
    crossing = last_ch > ch
    if cfg_id == 4:                 # wide, dense hits: some clusters do cross a joined edge
        assert crossing.any()
    # clusters that touch no joined edge are the plain oracle's clusters
    key = lambda r: (int(r["channel"]), int(r["first"]))
    pmap = {key(r): r for r in plain.cl}
    for r, x in zip(mod.cl, crossing):
        if x:
            continue
        c, f, w = int(r["channel"]), int(r["first"]), int(r["width"])
        touches = (f == 0 and joins[c]) or (f + w == NS and c + 1 < cfg.n_channels and joins[c + 1])
        if not touches:
            assert pmap[key(r)].tobytes() == r.tobytes()
    # member ADCs in order, and as many as the widths say
    assert mod.adc.size == int(width.sum())


def test_no_joins_is_the_plain_oracle():
    cfg = fedgen.CONFIGS[4].with_(n_fed=12)
    cal = fedgen.make_calibration(cfg)
    ev = fedgen.make_event(cfg, cal, 1)
    a = oracle.process_event(ev.zs, ev.fed_offset, cal.noise, cal.gain, cal.bad)
    b = oracle.process_event(ev.zs, ev.fed_offset, cal.noise, cal.gain, cal.bad,
                             joins=np.zeros(cfg.n_channels, np.uint8))
    assert a.cl.tobytes() == b.cl.tobytes() and a.adc.tobytes() == b.adc.tobytes()
