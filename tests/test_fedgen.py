"""Synthetic workload generator: determinism, format and distribution moments."""
import math

import numpy as np

import fedgen


def test_deterministic_and_distinct():
    cfg = fedgen.CONFIGS[0]
    c1 = fedgen.make_calibration(cfg)
    c2 = fedgen.make_calibration(cfg)
    np.testing.assert_array_equal(c1.noise, c2.noise)
    e1 = fedgen.make_event(cfg, c1, 4)
    e2 = fedgen.make_event(cfg, c1, 4)
    e3 = fedgen.make_event(cfg, c1, 5)
    np.testing.assert_array_equal(e1.zs, e2.zs)
    assert not np.array_equal(e1.dense, e3.dense)


def test_calibration_moments():
    cfg = fedgen.CONFIGS[1]
    cal = fedgen.make_calibration(cfg)
    assert cal.noise.dtype == np.float32 and cal.noise.size == 440 * 96 * 256
    assert cal.noise.min() >= 3.0 and cal.noise.max() <= 6.0
    assert abs(cal.noise.mean() - 4.5) < 0.01
    assert abs(cal.gain.mean() - 1.0) < 0.002 and abs(cal.gain.std() - 0.05) < 0.002
    assert abs(cal.bad.mean() - 0.001) < 0.0002


def test_event_sizes_match_expected_scale():
    cfg = fedgen.CONFIGS[0]
    cal = fedgen.make_calibration(cfg)
    ev = fedgen.make_event(cfg, cal, 0)
    assert ev.fed_offset.size == 51 and ev.fed_offset[-1] == ev.zs.size
    # ~1% hit starts with mean width ~2, plus ~2.2% noise-only strips above 2 sigma
    frac = ev.n_digis / cfg.n_strips
    assert 0.03 < frac < 0.05
    assert 100e3 < ev.zs.size < 180e3


def test_occupancy_samplers():
    cfg = fedgen.CONFIGS[2].with_(n_fed=2)
    occ = [fedgen._event_occupancy(cfg, fedgen.rng_for(2, 1, i)) for i in range(400)]
    assert min(occ) >= 0.005 and max(occ) <= 0.05
    assert abs(np.mean(np.log(occ)) - (math.log(0.005) + math.log(0.05)) / 2) < 0.15
    cfg3 = fedgen.CONFIGS[3].with_(n_fed=2)
    occ3 = [fedgen._event_occupancy(cfg3, fedgen.rng_for(3, 1, i)) for i in range(1000)]
    vals, counts = np.unique(occ3, return_counts=True)
    assert set(vals.tolist()) <= {0.005, 0.015, 0.03, 0.06}
    assert abs(counts[vals.tolist().index(0.015)] / 1000 - 0.4) < 0.05


def test_width_cap_and_stress_config():
    cfg = fedgen.CONFIGS[4].with_(n_fed=8)
    cal = fedgen.make_calibration(cfg)
    ev = fedgen.make_event(cfg, cal, 0)
    assert abs(cal.bad.mean() - 0.01) < 0.002
    assert cal.noise.min() >= 2.0 and cal.noise.max() <= 10.0
    assert ev.n_digis / cfg.n_strips > 0.1


def test_encode_run_splitting():
    adc = np.zeros((96, 256), np.uint8)
    mask = np.zeros((96, 256), bool)
    mask[5, 10:30] = True
    adc[5, 10:30] = 7
    zs, fo = fedgen.encode_dense(adc, mask, max_run=8)
    # 20 strips in pieces of 8, 8, 4: payload 3*2 + 20 = 26
    start = 5 * 2
    assert int(zs[start]) | (int(zs[start + 1]) << 8) == 26
    assert list(zs[start + 2:start + 4]) == [10, 8]
    assert list(zs[start + 12:start + 14]) == [18, 8]
    assert list(zs[start + 22:start + 24]) == [26, 4]
