"""GPU: module-aware clustering (runs across the channel edges of a module row) against the
module-aware oracle. Bar as for the plain path: clusters, ranges, charges and member ADCs
bit-exact; barycenters within 1e-6 relative (and checked bit-exact where stated).
"""
import numpy as np
import pytest

import fedgen
import oracle
from helpers import NCH, NS, calib_arrays, event_from_dense

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2101_11489_amd as sc  # noqa: E402
from gpu_common import bary_bit_exact, compare_clusters, make_ctx, run_fused  # noqa: E402

MOD_SHAPES = [(1, 1024), (1, 3072), (2, 2048), (2, 2880), (2, 4096), (4, 3072)]


def _joins(cm):
    n = cm.size
    j = np.zeros(n, np.uint8)
    j[1:] = (cm[1:] == cm[:-1]) & (np.arange(1, n) % NCH != 0)
    return j


@pytest.fixture(scope="module")
def full():
    cfg = fedgen.CONFIGS[2]
    cal = fedgen.make_calibration(cfg)
    geo = fedgen.make_geometry(cfg)
    evs = fedgen.make_events(cfg, cal, range(6), workers=6)
    joins = _joins(geo.channel_module)
    refs = [oracle.process_event(e.zs, e.fed_offset, cal.noise, cal.gain, cal.bad, joins=joins)
            for e in evs]
    ctx = make_ctx(cal.noise, cal.gain, cal.bad)
    ctx.set_modules(geo.channel_module)
    yield cal, geo, evs, refs, ctx
    ctx.close()


def _crossing(cl):
    return int(np.sum(cl["first"].astype(np.int64) + cl["width"] > NS))


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("waves,chunk", MOD_SHAPES)
def test_full_detector_module_rows_exact(full, waves, chunk, order):
    cal, geo, evs, refs, ctx = full
    before = ctx.tuning
    ctx.tuning = {"use_graph": 0, "tile_waves": waves, "chunk_digis": chunk, "fed_major": order}
    try:
        results, rc, _, _ = run_fused(ctx, [(e.zs, e.fed_offset) for e in evs])
        assert rc == sc.SC_OK
        for i, (res, ref) in enumerate(zip(results, refs)):
            compare_clusters(res[0], res[1], ref, f"module rows, event {i}")
            assert bary_bit_exact(res[0], ref)
        assert sum(_crossing(r.cl) for r in refs) > 100    # the events do cross module edges
    finally:
        ctx.tuning = before


@pytest.mark.parametrize("waves,chunk", [(2, 2880), (4, 4096), (4, 6144)])
def test_module_rows_with_the_large_stage(full, waves, chunk):
    cal, geo, evs, refs, ctx = full
    before = ctx.tuning
    ctx.tuning = {"use_graph": 0, "tile_waves": waves, "chunk_digis": chunk, "stage_bytes": 10240}
    try:
        results, rc, _, _ = run_fused(ctx, [(e.zs, e.fed_offset) for e in evs[:3]])
        assert rc == sc.SC_OK
        for i, (res, ref) in enumerate(zip(results, refs[:3])):
            compare_clusters(res[0], res[1], ref, f"module rows, large stage, event {i}")
            assert bary_bit_exact(res[0], ref)
    finally:
        ctx.tuning = before


def test_graph_replay_and_rows_off_again(full):
    cal, geo, evs, refs, ctx = full
    devs = [sc.Event(e.zs, e.fed_offset).to_device() for e in evs[:3]]
    outs = [ctx.output(*sc.safe_caps(d)) for d in devs]
    ctx.tuning = {"use_graph": 1}
    for rep in range(3):
        ctx.process_events(devs, outs)
        for o, ref in zip(outs, refs[:3]):
            compare_clusters(*o.to_numpy()[:2], ref, f"graph replay {rep}")
    # rows off: the plain oracle's clusters, also through a graph (a different kernel)
    ctx.set_modules(None)
    try:
        ctx.process_events(devs, outs)
        for o, e in zip(outs, evs[:3]):
            plain = oracle.process_event(e.zs, e.fed_offset, cal.noise, cal.gain, cal.bad)
            compare_clusters(*o.to_numpy()[:2], plain, "rows off")
    finally:
        ctx.set_modules(geo.channel_module)
        ctx.tuning = {"use_graph": 0}


@pytest.mark.parametrize("waves,chunk", MOD_SHAPES)
def test_dense_path_with_module_rows(full, waves, chunk):
    cal, geo, evs, refs, ctx = full
    before = ctx.tuning
    ctx.tuning = {"use_graph": 0, "tile_waves": waves, "chunk_digis": chunk}
    try:
        ev = sc.Event(evs[1].zs, evs[1].fed_offset).to_device()
        dense, _ = ctx.unpack(ev)
        out = ctx.output(*sc.safe_caps(sc.Event(evs[1].zs, evs[1].fed_offset)))
        ctx.cluster(dense, out)
        compare_clusters(*out.to_numpy()[:2], refs[1], f"dense path, module rows {waves}x{chunk}")
    finally:
        ctx.tuning = before


def test_stress_distribution_with_module_rows():
    """Config-4 hits (6 %, widths up to 32, 1 % bad strips) on 60 FEDs: wide clusters across
    module edges, FEDs past the LDS stage and groups split into chunks at row boundaries."""
    cfg = fedgen.CONFIGS[4].with_(n_fed=60)
    cal = fedgen.make_calibration(cfg)
    geo = fedgen.make_geometry(cfg)
    joins = _joins(geo.channel_module)
    evs = fedgen.make_events(cfg, cal, range(4), workers=4)
    with make_ctx(cal.noise, cal.gain, cal.bad) as ctx:
        ctx.set_modules(geo.channel_module)
        for waves, chunk in ((2, 2880), (1, 1024), (4, 3072)):
            ctx.tuning = {"use_graph": 0, "tile_waves": waves, "chunk_digis": chunk}
            results, rc, _, _ = run_fused(ctx, [(e.zs, e.fed_offset) for e in evs])
            for i, (res, e) in enumerate(zip(results, evs)):
                ref = oracle.process_event(e.zs, e.fed_offset, cal.noise, cal.gain, cal.bad,
                                           joins=joins)
                compare_clusters(res[0], res[1], ref, f"stress {waves}x{chunk} event {i}")
                assert _crossing(ref.cl) > 0


def _hand_ctx(noise, gain, bad, cm):
    ctx = make_ctx(noise, gain, bad)
    ctx.set_modules(cm)
    return ctx


def test_hand_rows_and_saturated_moment():
    """A three-channel row fully active with corrected ADCs near 65535 (the strip moment needs
    35 bits), a seed beyond the edge, per-APV gains across the edge and a bad strip at strip 0."""
    noise, gain, bad = calib_arrays(1)
    cm = np.arange(NCH, dtype=np.uint32)
    cm[1] = cm[0]                  # row: channels 0, 1
    cm[4] = cm[5] = cm[3]          # row: channels 3, 4, 5
    cm[8] = cm[7]                  # row: channels 7, 8
    dense = np.zeros(NCH * NS, np.uint8)
    dense[250:256] = 12
    dense[NS:NS + 4] = 9
    gain[1], gain[2] = 2.0, 0.5
    rng = np.random.default_rng(3)
    dense[3 * NS:6 * NS] = rng.integers(200, 256, 3 * NS)
    gain[6:12] = 0.001             # corrected ADCs saturate at 65535
    gain[7] = 0.0037               # ... or come close: rint(adc / 0.0037)
    dense[7 * NS + 255] = 3        # active, not a seed
    dense[8 * NS] = 9              # the seed, across the edge
    bad[8 * NS + 1] = 1
    dense[8 * NS + 1] = 9
    zs, fo = event_from_dense(dense)
    ref = oracle.process_event(zs, fo, noise, gain, bad, joins=_joins(cm))
    assert ref.cl.size == 3 and int(ref.cl["width"][1]) == 768
    ctx = _hand_ctx(noise, gain, bad, cm)
    try:
        for waves, chunk in MOD_SHAPES:
            ctx.tuning = {"use_graph": 0, "tile_waves": waves, "chunk_digis": chunk}
            results, rc, _, _ = run_fused(ctx, [(zs, fo)])
            compare_clusters(results[0][0], results[0][1], ref, f"hand rows {waves}x{chunk}")
            assert bary_bit_exact(results[0][0], ref)
    finally:
        ctx.close()


def test_module_maps_and_shapes_refused(full):
    cal, geo, evs, refs, ctx = full
    n = ctx.n_fed * NCH
    bad_maps = []
    cm = np.arange(n, dtype=np.uint32)
    cm[24] = cm[23]                # crosses a multiple of 24 channels
    bad_maps.append(cm)
    cm = np.arange(n, dtype=np.uint32)
    cm[1:4] = cm[0]                # four channels
    bad_maps.append(cm)
    for m in bad_maps:
        with pytest.raises(sc.ScError):
            ctx.set_modules(m)
    with pytest.raises(ValueError):
        ctx.set_modules(np.zeros(7, np.uint32))
    with pytest.raises(sc.ScError):   # 4 waves x 2048 digis: 512 per wave, less than a row
        ctx.tuning = {"tile_waves": 4, "chunk_digis": 2048}
    # the context still has its rows and gives their clusters
    results, rc, _, _ = run_fused(ctx, [(evs[0].zs, evs[0].fed_offset)])
    compare_clusters(results[0][0], results[0][1], refs[0], "after refusals")
    with make_ctx(cal.noise, cal.gain, cal.bad) as other:
        other.tuning = {"tile_waves": 4, "chunk_digis": 2048}
        with pytest.raises(sc.ScError):
            other.set_modules(geo.channel_module)


def test_served_pipelined_and_hits_with_module_rows(full):
    cal, geo, evs, refs, ctx = full
    with make_ctx(cal.noise, cal.gain, cal.bad, max_batch=3, n_streams=2) as srv:
        srv.set_modules(geo.channel_module)
        srv.set_geometry(geo)
        devs = [sc.Event(e.zs, e.fed_offset).to_device() for e in evs]
        outs = [srv.output(*sc.safe_caps(d)) for d in devs]
        tickets = [srv.submit(d, o) for d, o in zip(devs, outs)]
        for t in tickets:
            assert srv.poll(t, -1) == sc.SC_OK
        for i, (o, ref) in enumerate(zip(outs, refs)):
            compare_clusters(*o.to_numpy()[:2], ref, f"served {i}")
        pinned = sc.pack_pinned([sc.Event(e.zs, e.fed_offset) for e in evs])
        outs2 = [srv.output(*sc.safe_caps(p)) for p in pinned]
        rc, _ = srv.process_pipelined(pinned, outs2, 2)
        for i, (o, ref) in enumerate(zip(outs2, refs)):
            compare_clusters(*o.to_numpy()[:2], ref, f"pipelined {i}")
        # hits of clusters that cross into the next channel: barycenter past 256
        from oracle.hits import cluster_hits
        h = srv.cluster_hits(outs2[:1])[0].cpu().numpy().astype(np.float64)
        want = cluster_hits(refs[0].cl, geo)
        assert np.max(np.abs(h - want)) < 1e-4
