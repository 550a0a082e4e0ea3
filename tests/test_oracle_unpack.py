"""Pins of the oracle's unpacker (paper §2: ZS data stored like CSR per FED).

* hand-built byte vectors with hand-written expected ADCs and statuses (tests/golden);
* round trips against the generator's independent encoder, including random sparse rows;
* on generated events, the decoded ADCs equal the generator's kept ADCs.
"""
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import fedgen
import oracle
from helpers import golden_event, parse_channel_set, NS

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "unpack_cases.json")
CASES = json.load(open(GOLDEN))["cases"]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_golden_unpack(case):
    zs, fo, n_fed = golden_event(case)
    adc, st, rc = oracle.unpack(zs, fo)
    expect = np.zeros(n_fed * 96 * NS, dtype=np.uint8)
    for ch, segs in case["adc"].items():
        for first, count, val in segs:
            expect[int(ch) * NS + first: int(ch) * NS + first + count] = val
    np.testing.assert_array_equal(adc, expect)
    bad = parse_channel_set(case["malformed"])
    trail = parse_channel_set(case["trailing"])
    want = np.zeros(n_fed * 96, dtype=np.uint8)
    want[bad] |= oracle.CH_MALFORMED
    want[trail] |= oracle.FED_TRAILING
    np.testing.assert_array_equal(st, want)
    assert rc == (1 if bad else 0)


def _rows(draw_rows):
    return np.array(draw_rows, dtype=np.uint8).reshape(96, NS)


@settings(max_examples=60, deadline=None)
@given(st.data())
def test_roundtrip_random_sparse_rows(data):
    rng = np.random.default_rng(data.draw(st.integers(0, 2**32 - 1)))
    density = data.draw(st.sampled_from([0.0, 0.01, 0.2, 0.5, 0.9, 1.0]))
    mask = rng.random((96, NS)) < density
    adc = rng.integers(0, 256, size=(96, NS), dtype=np.uint8)
    max_run = data.draw(st.sampled_from([255, 7, 1]))
    zs, fo = fedgen.encode_dense(adc, mask, max_run=max_run)
    out, stt, rc = oracle.unpack(zs, fo)
    np.testing.assert_array_equal(out.reshape(96, NS), np.where(mask, adc, 0))
    assert rc == 0 and not stt.any()


def test_roundtrip_generated_event():
    cfg = fedgen.CONFIGS[0]
    cal = fedgen.make_calibration(cfg)
    for i in range(2):
        ev = fedgen.make_event(cfg, cal, i)
        adc, stt, rc = oracle.unpack(ev.zs, ev.fed_offset)
        assert rc == 0 and not stt.any()
        np.testing.assert_array_equal(adc, ev.dense)
        # every strip the front end kept passes its cut, and nothing else is present
        kept = ev.dense > 0
        assert np.all(ev.dense[kept].astype(np.float32) > np.float32(2) * cal.noise[kept])


def test_full_channel_needs_two_records():
    adc = np.zeros((96, NS), dtype=np.uint8)
    adc[0] = np.arange(1, 257) % 251 + 1
    zs, fo = fedgen.encode_dense(adc, adc > 0)
    # 2 length bytes + (2 + 255) + (2 + 1) for channel 0, 2 bytes for the 95 empty channels
    assert zs.size == 2 + 260 + 95 * 2
    out, _, _ = oracle.unpack(zs, fo)
    np.testing.assert_array_equal(out.reshape(96, NS)[0], adc[0])
