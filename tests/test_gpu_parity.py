"""GPU parity: every entry point of libsc.so against the oracle on the same seeded inputs.

Bar: cluster membership, strip ranges, charges and gain-corrected ADCs bit-exact; barycenters
within 1e-6 relative (FP32).
"""
import json
import os

import numpy as np
import pytest

import fedgen
import oracle
from helpers import (calib_arrays, event_from_runs, golden_calib, golden_event,
                     parse_channel_set, threshold_runs, NS)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2101_11489_amd as sc  # noqa: E402
from gpu_common import bary_bit_exact, compare_clusters, make_ctx, run_fused  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden")
HAND = json.load(open(os.path.join(GOLD, "hand_channels.json")))["cases"]
UNPACK = json.load(open(os.path.join(GOLD, "unpack_cases.json")))["cases"]


@pytest.fixture(scope="module")
def cfg0():
    cfg = fedgen.CONFIGS[0]
    cal = fedgen.make_calibration(cfg)
    evs = [fedgen.make_event(cfg, cal, i) for i in range(6)]
    ctx = make_ctx(cal.noise, cal.gain, cal.bad)
    yield cfg, cal, evs, ctx
    ctx.close()


@pytest.mark.parametrize("case", HAND, ids=[c["name"] for c in HAND])
@pytest.mark.parametrize("device", [True, False], ids=["dev", "host"])
def test_hand_channels_fused(case, device):
    zs, fo, n_fed = golden_event(case)
    noise, gain, bad = golden_calib(case, n_fed)
    ref = oracle.process_event(zs, fo, noise, gain, bad)
    with make_ctx(noise, gain, bad) as ctx:
        (res,), rc, sts, _ = run_fused(ctx, [(zs, fo)], device=device, chan_status=True)
        cl, adc, st = res
        compare_clusters(cl, adc, ref, case["name"])
        assert bary_bit_exact(cl, ref)
        np.testing.assert_array_equal(st, ref.chan_status)
        assert rc == (sc.SC_MALFORMED if ref.status else sc.SC_OK)


@pytest.mark.parametrize("case", UNPACK, ids=[c["name"] for c in UNPACK])
def test_unpack_golden(case):
    zs, fo, n_fed = golden_event(case)
    noise, gain, bad = golden_calib({}, n_fed)
    ref_adc, ref_st, ref_rc = oracle.unpack(zs, fo)
    with make_ctx(noise, gain, bad) as ctx:
        for device in (True, False):
            ev = sc.Event(zs, fo)
            if device:
                ev = ev.to_device()
            dense = ctx.dense_buffer(device=device)
            st = (torch.zeros(n_fed * 96, dtype=torch.uint8, device="cuda") if device
                  else np.zeros(n_fed * 96, np.uint8))
            _, rc = ctx.unpack(ev, dense, st)
            d = dense.cpu().numpy() if device else dense
            s = st.cpu().numpy() if device else st
            np.testing.assert_array_equal(d, ref_adc)
            np.testing.assert_array_equal(s, ref_st)
            assert rc == (sc.SC_MALFORMED if ref_rc else sc.SC_OK)
        # fused path on the same bytes: statuses and (empty or not) clusters agree too
        ref = oracle.process_event(zs, fo, noise, gain, bad)
        (res,), rc, _, _ = run_fused(ctx, [(zs, fo)], chan_status=True)
        compare_clusters(res[0], res[1], ref, case["name"])
        np.testing.assert_array_equal(res[2], ref_st)


def test_cluster_dense_hand_channels():
    for case in HAND:
        zs, fo, n_fed = golden_event(case)
        noise, gain, bad = golden_calib(case, n_fed)
        dense, _, _ = oracle.unpack(zs, fo)
        ref = oracle.cluster(dense, noise, gain, bad)
        with make_ctx(noise, gain, bad) as ctx:
            for device in (True, False):
                out = ctx.output(4096, 8192, device=device)
                src = torch.from_numpy(dense).cuda() if device else dense
                rc = ctx.cluster(src, out)
                cl, adc, _ = out.to_numpy()
                compare_clusters(cl, adc, ref, case["name"])
                assert rc == sc.SC_OK


@pytest.mark.parametrize("waves,chunk", [(1, 1024), (2, 2880), (2, 3072), (4, 2048)])
def test_runs_at_the_cluster_threshold(waves, chunk):
    # charges equal to fl(t * sqrtf(S)) or one binary32 step beside it, runs of 1 to 250 strips
    # (across 64-digi steps): decisions the kernels cannot take from their tree-order noise sum
    thr = dict(t_seed=0.3, t_channel=0.25, t_cluster=5.0)
    for seed in (1, 2):
        chan_runs, noise, runs = threshold_runs(seed)
        _, gain, bad = calib_arrays(1)
        zs, fo = event_from_runs(chan_runs)
        ref = oracle.process_event(zs, fo, noise, gain, bad, **thr)
        with make_ctx(noise, gain, bad, **thr) as ctx:
            ctx.tuning = {"chunk_digis": chunk, "tile_waves": waves, "use_graph": 0}
            (res,), rc, _, _ = run_fused(ctx, [(zs, fo)])
            assert rc == sc.SC_OK
            compare_clusters(res[0], res[1], ref, f"seed {seed}")
            assert bary_bit_exact(res[0], ref)


@pytest.mark.parametrize("waves,chunk", [(1, 1024), (2, 2880), (4, 2048)])
def test_one_strip_runs_at_the_cluster_threshold(waves, chunk):
    # isolated strips, so that both digis of every lane end a run: digi A's run takes the
    # tree-sum test, digi B's the one-strip test. Noise at fl(a / t) and up to three binary32
    # steps beside it, and tiny (below 2^-60 the one-strip test leaves the run to the
    # sequential sum)
    thr = dict(t_seed=0.3, t_channel=0.25, t_cluster=5.0)
    rng = np.random.default_rng(11489)
    noise, gain, bad = calib_arrays(1)
    tiny = [0.0, 1e-40, 1e-30, 2.0 ** -70, 2.0 ** -63, 2.0 ** -61, 2.0 ** -60, 2.0 ** -59]
    chan_runs = {}
    for ch in range(16):   # 6.3 KB of ZS: the FED fits the LDS stage
        recs = []
        for s in range(ch % 2, 256, 2):
            a = int(rng.integers(1, 256))
            k = int(rng.integers(0, 9))
            if k < 7:
                n = np.float32(a) / np.float32(thr["t_cluster"])
                for _ in range(abs(k - 3)):
                    n = np.nextafter(n, np.float32(np.inf if k > 3 else 0.0), dtype=np.float32)
            else:
                n = np.float32(tiny[int(rng.integers(0, len(tiny)))])
            noise[ch * 256 + s] = n
            recs.append((s, [a]))
        chan_runs[ch] = recs
    zs, fo = event_from_runs(chan_runs)
    ref = oracle.process_event(zs, fo, noise, gain, bad, **thr)
    assert 0 < ref.cl.size < 16 * 128   # some runs pass the threshold and some do not
    with make_ctx(noise, gain, bad, **thr) as ctx:
        ctx.tuning = {"chunk_digis": chunk, "tile_waves": waves, "use_graph": 0}
        (res,), rc, _, _ = run_fused(ctx, [(zs, fo)])
        assert rc == sc.SC_OK
        compare_clusters(res[0], res[1], ref, "one-strip runs")
        assert bary_bit_exact(res[0], ref)


def test_generated_config0_batch(cfg0):
    cfg, cal, evs, ctx = cfg0
    refs = [oracle.process_event(e.zs, e.fed_offset, cal.noise, cal.gain, cal.bad) for e in evs]
    results, rc, sts, _ = run_fused(ctx, [(e.zs, e.fed_offset) for e in evs])
    assert rc == sc.SC_OK and all(s == sc.SC_OK for s in sts)
    for i, (res, ref) in enumerate(zip(results, refs)):
        compare_clusters(res[0], res[1], ref, f"event {i}")
        assert bary_bit_exact(res[0], ref)


def test_plain_path_unpack_then_cluster(cfg0):
    cfg, cal, evs, ctx = cfg0
    e = evs[0]
    ref = oracle.process_event(e.zs, e.fed_offset, cal.noise, cal.gain, cal.bad)
    dev = sc.Event(e.zs, e.fed_offset).to_device()
    dense, rc = ctx.unpack(dev)
    assert rc == sc.SC_OK
    np.testing.assert_array_equal(dense.cpu().numpy(), e.dense)
    out = ctx.output(*sc.safe_caps(dev))
    assert ctx.cluster(dense, out) == sc.SC_OK
    cl, adc, _ = out.to_numpy()
    compare_clusters(cl, adc, ref, "plain")


SHAPES = [(1, 1024), (1, 2048), (1, 3072), (1, 4096), (2, 2048), (2, 2880), (2, 3072), (2, 4096),
          (4, 2048), (4, 3072), (4, 4096)]


@pytest.mark.parametrize("waves,chunk", SHAPES, ids=[f"w{w}-d{d}" for w, d in SHAPES])
@pytest.mark.parametrize("fed_major", [0, 1, 2])
def test_tuning_choices_identical(cfg0, waves, chunk, fed_major):
    cfg, cal, evs, ctx = cfg0
    refs = [oracle.process_event(e.zs, e.fed_offset, cal.noise, cal.gain, cal.bad) for e in evs[:3]]
    before = ctx.tuning
    ctx.tuning = {"chunk_digis": chunk, "tile_waves": waves, "fed_major": fed_major,
                  "use_graph": 0}
    try:
        results, rc, _, _ = run_fused(ctx, [(e.zs, e.fed_offset) for e in evs[:3]])
        for res, ref in zip(results, refs):
            compare_clusters(res[0], res[1], ref, f"chunk {chunk}")
        # the dense path with the same chunk size
        dense, _ = ctx.unpack(sc.Event(evs[0].zs, evs[0].fed_offset).to_device())
        out = ctx.output(*sc.safe_caps(sc.Event(evs[0].zs, evs[0].fed_offset)))
        ctx.cluster(dense, out)
        compare_clusters(*out.to_numpy()[:2], refs[0], f"dense chunk {chunk}")
    finally:
        ctx.tuning = before


def test_unsupported_tile_shapes_are_refused(cfg0):
    cfg, cal, evs, ctx = cfg0
    before = ctx.tuning
    for t in ({"tile_waves": 3}, {"tile_waves": 8}, {"chunk_digis": 1536}, {"chunk_digis": 512},
              {"tile_waves": 2, "chunk_digis": 1024}, {"tile_waves": 4, "chunk_digis": 1024},
              {"tile_waves": 1, "chunk_digis": 2880}, {"tile_waves": 4, "chunk_digis": 2880}):
        with pytest.raises(sc.ScError):
            ctx.tuning = t
    assert ctx.tuning == before
