"""GPU: full-size events, batching, graphs, overflow, edge cases and the server, against the oracle.

Bar: clusters, ranges, charges, member ADCs bit-exact; barycenters within 1e-6 relative.
"""
import numpy as np
import pytest

import fedgen
import oracle
from helpers import NS, calib_arrays, event_from_runs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2101_11489_amd as sc  # noqa: E402
from gpu_common import compare_clusters, make_ctx, run_fused  # noqa: E402


def _oracle(ev, cal):
    return oracle.process_event(ev.zs, ev.fed_offset, cal.noise, cal.gain, cal.bad)


@pytest.fixture(scope="module")
def full():
    """Config-2 detector (440 FEDs) with 8 events of uneven occupancy, and their oracle output."""
    cfg = fedgen.CONFIGS[2]
    cal = fedgen.make_calibration(cfg)
    evs = fedgen.make_events(cfg, cal, range(8), workers=8)
    refs = [_oracle(e, cal) for e in evs]
    ctx = make_ctx(cal.noise, cal.gain, cal.bad)
    yield cal, evs, refs, ctx
    ctx.close()


@pytest.mark.parametrize("waves,chunk", [(1, 3072), (1, 1024), (2, 2048), (2, 2880), (2, 4096),
                                         (4, 3072)])
def test_full_detector_batch_exact(full, waves, chunk):
    cal, evs, refs, ctx = full
    before = ctx.tuning
    ctx.tuning = {"use_graph": 0, "tile_waves": waves, "chunk_digis": chunk}
    try:
        results, rc, sts, _ = run_fused(ctx, [(e.zs, e.fed_offset) for e in evs])
        assert rc == sc.SC_OK
        for i, (res, ref) in enumerate(zip(results, refs)):
            compare_clusters(res[0], res[1], ref, f"event {i} occ {evs[i].occ:.4f}")
    finally:
        ctx.tuning = before


LARGE_STAGE = 10240   # sc_tuning.stage_bytes of the large LDS stage (FEDs up to 10224 bytes)


@pytest.mark.parametrize("waves,chunk", [(2, 2048), (2, 2880), (4, 4096), (4, 6144)])
def test_full_detector_batch_exact_large_stage(full, waves, chunk):
    cal, evs, refs, ctx = full
    before = ctx.tuning
    ctx.tuning = {"use_graph": 0, "tile_waves": waves, "chunk_digis": chunk,
                  "stage_bytes": LARGE_STAGE}
    try:
        results, rc, sts, _ = run_fused(ctx, [(e.zs, e.fed_offset) for e in evs])
        assert rc == sc.SC_OK
        for i, (res, ref) in enumerate(zip(results, refs)):
            compare_clusters(res[0], res[1], ref, f"large stage, event {i}")
    finally:
        ctx.tuning = before


@pytest.mark.parametrize("waves,chunk", [(2, 2880), (1, 3072)])
@pytest.mark.parametrize("graph", [0, 1])
def test_full_detector_per_xcd_order_exact(full, waves, chunk, graph):
    """Tile order 2 (FEDs dealt to one queue per XCD): the 8 full-size events, eager and as graph
    replays, several times in a row, give the oracle's clusters."""
    cal, evs, refs, ctx = full
    before = ctx.tuning
    ctx.tuning = {"use_graph": graph, "tile_waves": waves, "chunk_digis": chunk, "fed_major": 2}
    try:
        for rep in range(3):
            results, rc, _, _ = run_fused(ctx, [(e.zs, e.fed_offset) for e in evs])
            assert rc == sc.SC_OK
            for i, (res, ref) in enumerate(zip(results, refs)):
                compare_clusters(res[0], res[1], ref, f"order 2 call {rep} event {i}")
    finally:
        ctx.tuning = before


@pytest.mark.parametrize("batch", [1, 3, 8, 24])
@pytest.mark.parametrize("layout", ["scattered", "packed"])
def test_pipelined_host_ingest_exact(full, batch, layout):
    """sc_process_pipelined over 24 events (the 8 full-size events three times) in pageable host,
    page-locked host and device memory, mixed, with device and host outputs, in batches of
    `batch` (a ragged last batch for 3). Page-locked events are separate buffers, or back to back
    in one buffer (then consecutive ones share a transfer). Every event gives the oracle's
    clusters, and the same bytes as sc_process_events."""
    cal, evs, refs, ctx = full
    hosts = [sc.Event(e.zs, e.fed_offset) for e in evs]
    pinned = [h.to_pinned() for h in hosts] if layout == "scattered" else sc.pack_pinned(hosts)
    devs = [h.to_device() for h in hosts]
    kinds = [hosts, pinned, devs]
    order = [(i % 8, (i // 2) % 3) for i in range(24)]
    events = [kinds[k][i] for i, k in order]
    outs = [ctx.output(*sc.safe_caps(hosts[i]), device=(j % 4 != 1))
            for j, (i, _) in enumerate(order)]
    rc, sts = ctx.process_pipelined(events, outs, batch)
    assert rc == sc.SC_OK and sts == [sc.SC_OK] * 24
    for j, ((i, k), o) in enumerate(zip(order, outs)):
        compare_clusters(*o.to_numpy()[:2], refs[i], f"pipelined event {j} kind {k}")
    one = [ctx.output(*sc.safe_caps(hosts[i])) for i in range(8)]
    ctx.process_events(devs, one)
    for j, ((i, _), o) in enumerate(zip(order, outs)):
        a, b = o.to_numpy(), one[i].to_numpy()
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])


def test_pipelined_small_calls_and_host_outputs(full):
    """Batch larger than n; an odd n; host outputs with channel status; page-locked events
    through the server (copied at submit like pageable ones)."""
    cal, evs, refs, ctx = full
    hosts = [sc.Event(e.zs, e.fed_offset) for e in evs]
    pinned = sc.pack_pinned(hosts)
    o1 = [ctx.output(*sc.safe_caps(hosts[2]))]
    rc, sts = ctx.process_pipelined([pinned[2]], o1, 8)
    assert rc == sc.SC_OK and sts == [sc.SC_OK]
    compare_clusters(*o1[0].to_numpy()[:2], refs[2], "one event, batch 8")
    outs = [ctx.output(*sc.safe_caps(h), device=False, chan_status=True) for h in hosts[:5]]
    rc, sts = ctx.process_pipelined(pinned[:5], outs, 2)
    assert rc == sc.SC_OK
    for i, o in enumerate(outs):
        cl, adc, st = o.to_numpy()
        compare_clusters(cl, adc, refs[i], f"host outputs {i}")
        np.testing.assert_array_equal(st, refs[i].chan_status)
    with make_ctx(cal.noise, cal.gain, cal.bad, max_batch=2, n_streams=2) as srv:
        souts = [srv.output(*sc.safe_caps(h)) for h in hosts[:4]]
        tickets = [srv.submit(p, o) for p, o in zip(pinned[:4], souts)]
        for t in tickets:
            assert srv.poll(t, -1) == sc.SC_OK
        for i, o in enumerate(souts):
            compare_clusters(*o.to_numpy()[:2], refs[i], f"served page-locked {i}")


def test_pipelined_statuses_per_event(full):
    """An event whose outputs are too small overflows alone; the others of its batch and of the
    other batches are exact, and a second call on the same context reuses the slots."""
    cal, evs, refs, ctx = full
    pinned = sc.pack_pinned([sc.Event(e.zs, e.fed_offset) for e in evs])
    for rep in range(2):
        outs = [ctx.output(*sc.safe_caps(p)) for p in pinned]
        outs[5] = ctx.output(max(1, refs[5].cl.size // 2), refs[5].adc.size)
        rc, sts = ctx.process_pipelined(pinned, outs, 3)
        assert rc == sc.SC_ERR_OVERFLOW
        assert sts == [sc.SC_OK] * 5 + [sc.SC_ERR_OVERFLOW] + [sc.SC_OK] * 2
        assert outs[5].cs.n_cl == refs[5].cl.size
        for i in (0, 1, 2, 3, 4, 6, 7):
            compare_clusters(*outs[i].to_numpy()[:2], refs[i], f"call {rep} event {i}")


def test_event_alone_equals_event_in_any_batch(full):
    cal, evs, refs, ctx = full
    pairs = [(e.zs, e.fed_offset) for e in evs]
    alone, _, _, _ = run_fused(ctx, [pairs[3]])
    mixed, _, _, _ = run_fused(ctx, [pairs[5], pairs[3], pairs[0]])
    rev, _, _, _ = run_fused(ctx, pairs[::-1])
    for got in (alone[0], mixed[1], rev[len(pairs) - 1 - 3]):
        np.testing.assert_array_equal(got[0], alone[0][0])
        np.testing.assert_array_equal(got[1], alone[0][1])
    compare_clusters(alone[0][0], alone[0][1], refs[3], "alone")


def test_repeated_and_alternating_batches(full):
    # the same prepared batch again (descriptors already on the device), two batches of the same
    # size in turn, and a dense sc_cluster call in between (which reuses the descriptor buffer)
    cal, evs, refs, ctx = full
    devs = [sc.Event(e.zs, e.fed_offset).to_device() for e in evs]
    outs_a = [ctx.output(*sc.safe_caps(d)) for d in devs[:4]]
    outs_b = [ctx.output(*sc.safe_caps(d)) for d in devs[4:]]
    a, b = ctx.batch(devs[:4], outs_a), ctx.batch(devs[4:], outs_b)
    for g in (0, 1):
        ctx.tuning = {"use_graph": g}
        for rep, (bt, outs, rr) in enumerate([(a, outs_a, refs[:4]), (a, outs_a, refs[:4]),
                                              (b, outs_b, refs[4:]), (a, outs_a, refs[:4]),
                                              (b, outs_b, refs[4:]), (b, outs_b, refs[4:])]):
            for o in outs:
                o.cl.zero_()
                o.adc.zero_()
            rc, _ = ctx.process_batch(bt)
            assert rc == sc.SC_OK
            for o, ref in zip(outs, rr):
                compare_clusters(*o.to_numpy()[:2], ref, f"graph {g} call {rep}")
            if rep == 3:
                dense, _ = ctx.unpack(devs[0])
                out = ctx.output(*sc.safe_caps(devs[0]))
                ctx.cluster(dense, out)
                compare_clusters(*out.to_numpy()[:2], refs[0], "dense in between")
    ctx.tuning = {"use_graph": 1}


def test_graph_replays_match_eager(full):
    cal, evs, refs, ctx = full
    devs = [sc.Event(e.zs, e.fed_offset).to_device() for e in evs[:4]]
    outs = [ctx.output(*sc.safe_caps(d)) for d in devs]
    ctx.tuning = {"use_graph": 1}
    before = ctx.stats()
    for rep in range(5):
        for o in outs:                  # eager torch work between replays
            o.cl.zero_()
            o.adc.zero_()
        torch.cuda.synchronize()
        ctx.process_events(devs, outs)
        for o, ref in zip(outs, refs[:4]):
            cl, adc, _ = o.to_numpy()
            compare_clusters(cl, adc, ref, f"replay {rep}")
    after = ctx.stats()
    assert after["graph_replays"] - before["graph_replays"] == 5
    assert after["graph_captures"] - before["graph_captures"] <= 1


def test_overflow_then_regrow(full):
    cal, evs, refs, ctx = full
    ev = sc.Event(evs[1].zs, evs[1].fed_offset).to_device()
    need_cl, need_adc = refs[1].cl.size, refs[1].adc.size
    small = ctx.output(need_cl // 3, need_adc // 2)
    rc, sts = ctx.process_events([ev], [small])
    assert rc == sc.SC_ERR_OVERFLOW and sts == [sc.SC_ERR_OVERFLOW]
    assert (small.n_cl, small.n_adc) == (need_cl, need_adc)
    cl, adc, _ = small.to_numpy()
    np.testing.assert_array_equal(cl, refs[1].cl[:need_cl // 3])     # the prefix is valid
    np.testing.assert_array_equal(adc, refs[1].adc[:need_adc // 2])
    big = ctx.output(small.n_cl, small.n_adc)                          # exactly the needs
    rc, _ = ctx.process_events([ev], [big])
    assert rc == sc.SC_OK
    compare_clusters(*big.to_numpy()[:2], refs[1], "regrown")


def test_host_and_device_mixed_batch(full):
    cal, evs, refs, ctx = full
    e_dev = sc.Event(evs[2].zs, evs[2].fed_offset).to_device()
    e_host = sc.Event(evs[4].zs, evs[4].fed_offset)
    o_dev = ctx.output(*sc.safe_caps(e_host), device=True)
    o_host = ctx.output(*sc.safe_caps(e_host), device=False, chan_status=True)
    ctx.process_events([e_host, e_dev], [o_dev, o_host])
    compare_clusters(*o_dev.to_numpy()[:2], refs[4], "host event -> device output")
    cl, adc, st = o_host.to_numpy()
    compare_clusters(cl, adc, refs[2], "device event -> host output")
    assert not st.any()


def test_stress_distribution_and_overflow_batch():
    cfg = fedgen.CONFIGS[4].with_(n_fed=60)
    cal = fedgen.make_calibration(cfg)
    evs = fedgen.make_events(cfg, cal, range(6), workers=6)
    refs = [_oracle(e, cal) for e in evs]
    with make_ctx(cal.noise, cal.gain, cal.bad) as ctx:
        # capacities sized for a lighter workload: some events overflow, the rest are exact
        caps = (int(np.median([r.cl.size for r in refs])), int(np.median([r.adc.size for r in refs])))
        results, rc, sts, outs = run_fused(ctx, [(e.zs, e.fed_offset) for e in evs], caps=caps)
        assert rc == sc.SC_ERR_OVERFLOW
        for i, (st, o, ref) in enumerate(zip(sts, outs, refs)):
            assert (o.n_cl, o.n_adc) == (ref.cl.size, ref.adc.size)
            if st == sc.SC_OK:
                compare_clusters(*o.to_numpy()[:2], ref, f"stress {i}")
            else:
                assert ref.cl.size > caps[0] or ref.adc.size > caps[1]
        # retry only the overflowed events with the reported sizes
        redo = [i for i, s in enumerate(sts) if s == sc.SC_ERR_OVERFLOW]
        assert redo
        res2, rc2, _, _ = run_fused(ctx, [(evs[i].zs, evs[i].fed_offset) for i in redo])
        assert rc2 == sc.SC_OK
        for i, r in zip(redo, res2):
            compare_clusters(r[0], r[1], refs[i], f"stress retry {i}")
        # long clusters crossing wavefront words and the APV boundary are present
        allcl = np.concatenate([r.cl for r in refs])
        assert allcl["width"].max() >= 12


@pytest.mark.parametrize("waves,chunk", [(2, 2048), (2, 2880), (4, 4096), (4, 6144)])
def test_stress_distribution_large_stage(waves, chunk):
    """The stress distribution's FEDs (about 8.2 KB) are past the small stage and inside the
    large one: staged and walked in LDS there, read from global memory with the small stage; the
    same clusters either way."""
    cfg = fedgen.CONFIGS[4].with_(n_fed=60)
    cal = fedgen.make_calibration(cfg)
    evs = fedgen.make_events(cfg, cal, range(3), workers=3)
    sizes = np.concatenate([np.diff(e.fed_offset.astype(np.int64)) for e in evs])
    assert np.mean(sizes > 6640) > 0.9 and np.all(sizes <= LARGE_STAGE - 16)
    refs = [_oracle(e, cal) for e in evs]
    with make_ctx(cal.noise, cal.gain, cal.bad) as ctx:
        ctx.tuning = {"use_graph": 0, "tile_waves": waves, "chunk_digis": chunk,
                      "stage_bytes": LARGE_STAGE}
        results, rc, _, _ = run_fused(ctx, [(e.zs, e.fed_offset) for e in evs])
        assert rc == sc.SC_OK
        for i, (res, ref) in enumerate(zip(results, refs)):
            compare_clusters(res[0], res[1], ref, f"stress, large stage, event {i}")


def _edge_event(kind):
    n_fed = 3
    noise, gain, bad = calib_arrays(n_fed)
    if kind == "all_empty":
        runs = {}
        zs, fo = event_from_runs(runs, n_fed)
    elif kind == "zero_length_feds":
        zs, fo = np.zeros(0, np.uint8), np.zeros(n_fed + 1, np.uint64)
    elif kind == "full_fed":
        # every channel of FED 1 fully active with one seed: 25 KB of ZS (larger than the LDS
        # stage) and 24576 digis (many chunks)
        runs = {96 + c: [(0, [3] * 255), (255, [4])] for c in range(96)}
        zs, fo = event_from_runs(runs, n_fed)
    elif kind == "alternating_fed":
        # 128 isolated strips per channel -> 12288 clusters in one FED
        runs = {c: [(2 * k, [5]) for k in range(128)] for c in range(96)}
        zs, fo = event_from_runs(runs, n_fed)
    elif kind == "between_stages":
        # 30 full channels in FED 1: 7.9 KB of ZS (past the small stage, inside the large one)
        # and 7680 digis (several chunks)
        runs = {96 + c: [(0, [4] + [3] * 254), (255, [3])] for c in range(30)}
        zs, fo = event_from_runs(runs, n_fed)
    elif kind == "multichunk_fits_stage":
        # 20 full channels: 5 KB of ZS (fits the stage) but 5120 digis
        runs = {192 + c: [(0, [4] + [3] * 254), (255, [3])] for c in range(20)}
        zs, fo = event_from_runs(runs, n_fed)
    elif kind == "group_heads":
        # the first channel of every channel group (W = 1, 2, 4) malformed (a run of count 0)
        # and the next one empty, so that a group's first digi slot belongs to a later channel;
        # channels of 40 one-strip runs (three bytes a digi); in the first group 1,576 digis
        # (more than one chunk at up to 1,536 digis a wave) with an empty channel among the full
        # ones
        full = [(0, [4] + [3] * 254), (255, [3])]
        alt = [(2 * k, [5]) for k in range(40)]
        runs = {}
        for g in (0, 24, 48, 72):
            runs[g] = [(10, [])]
            runs[g + 2] = alt
        for c in (3, 4, 6, 7, 8, 9):
            runs[c] = full
        runs[60] = [(0, [4, 3]), (2, [3, 4])]   # adjacent runs: one cluster
        zs, fo = event_from_runs(runs, n_fed)
    elif kind == "garbage":
        rng = np.random.default_rng(7)
        zs = rng.integers(0, 256, size=30000, dtype=np.uint8)
        fo = np.array([0, 9000, 21000, 30000], np.uint64)
    else:
        raise ValueError(kind)
    return zs, fo, noise, gain, bad


@pytest.mark.parametrize("kind", ["all_empty", "zero_length_feds", "full_fed", "alternating_fed",
                                  "between_stages", "multichunk_fits_stage", "group_heads",
                                  "garbage"])
@pytest.mark.parametrize("shape", [(1024, 1, 0), (3072, 1, 0), (2048, 2, 0), (2880, 2, 0),
                                   (4096, 2, 0), (2048, 4, 0), (2880, 2, LARGE_STAGE),
                                   (4096, 4, LARGE_STAGE), (6144, 4, LARGE_STAGE)])
def test_edge_cases(kind, shape):
    zs, fo, noise, gain, bad = _edge_event(kind)
    ref = oracle.process_event(zs, fo, noise, gain, bad)
    with make_ctx(noise, gain, bad) as ctx:
        ctx.tuning = {"chunk_digis": shape[0], "tile_waves": shape[1], "stage_bytes": shape[2]}
        caps = (max(ref.cl.size, 1), max(ref.adc.size, 1))
        (res,), rc, sts, _ = run_fused(ctx, [(zs, fo)], caps=caps, chan_status=True)
        compare_clusters(res[0], res[1], ref, kind)
        np.testing.assert_array_equal(res[2], ref.chan_status)
        # plain path on the same input
        dense, _ = ctx.unpack(sc.Event(zs, fo).to_device())
        ref_dense, _, _ = oracle.unpack(zs, fo)
        np.testing.assert_array_equal(dense.cpu().numpy(), ref_dense)
        out = ctx.output(*caps)
        ctx.cluster(dense, out)
        compare_clusters(*out.to_numpy()[:2], ref, kind + " dense")


def test_server_matches_oracle_and_is_mix_independent(full):
    cal, evs, refs, _ = full
    with make_ctx(cal.noise, cal.gain, cal.bad, max_batch=4, n_streams=2) as ctx:
        devs = [sc.Event(e.zs, e.fed_offset).to_device() for e in evs]
        hosts = [sc.Event(e.zs, e.fed_offset) for e in evs]
        outs, tickets = [], []
        for i in range(len(evs)):
            ev = devs[i] if i % 2 == 0 else hosts[i]
            o = ctx.output(*sc.safe_caps(hosts[i]), device=(i % 3 != 0))
            outs.append(o)
            tickets.append(ctx.submit(ev, o))
        for t in tickets:
            assert ctx.poll(t, -1) == sc.SC_OK
        for i, (o, ref) in enumerate(zip(outs, refs)):
            compare_clusters(*o.to_numpy()[:2], ref, f"served {i}")
        # alone (one event in flight) gives the same bytes as inside the mix
        o = ctx.output(*sc.safe_caps(hosts[5]))
        t = ctx.submit(devs[5], o)
        assert ctx.poll(t, -1) == sc.SC_OK
        a, b = o.to_numpy(), outs[5].to_numpy()
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
        st = ctx.stats()
        assert st["server_events"] == len(evs) + 1 and st["server_batches"] >= 2
        assert ctx.poll(t, 0) == sc.SC_ERR_UNKNOWN_TICKET
        assert ctx.poll(123456789, 0) == sc.SC_ERR_UNKNOWN_TICKET


def test_server_under_per_xcd_tuning(full):
    """A context tuned to tile order 2 serves with order 1 (several server launches may run at
    once); results are the oracle's, and synchronous calls on it keep order 2."""
    cal, evs, refs, _ = full
    with make_ctx(cal.noise, cal.gain, cal.bad, max_batch=3, n_streams=2) as ctx:
        ctx.tuning = {"fed_major": 2, "use_graph": 0}
        devs = [sc.Event(e.zs, e.fed_offset).to_device() for e in evs]
        outs = [ctx.output(*sc.safe_caps(d)) for d in devs]
        tickets = [ctx.submit(d, o) for d, o in zip(devs, outs)]
        for t in tickets:
            assert ctx.poll(t, -1) == sc.SC_OK
        for i, (o, ref) in enumerate(zip(outs, refs)):
            compare_clusters(*o.to_numpy()[:2], ref, f"served under order 2, event {i}")
        assert ctx.tuning["fed_major"] == 2
        results, rc, _, _ = run_fused(ctx, [(e.zs, e.fed_offset) for e in evs[:3]])
        for r, ref in zip(results, refs[:3]):
            compare_clusters(r[0], r[1], ref, "synchronous after serving")


def test_server_budget_and_backpressure(full):
    cal, evs, refs, _ = full
    host = sc.Event(evs[0].zs, evs[0].fed_offset)
    cap_cl, cap_adc = refs[0].cl.size, refs[0].adc.size
    one = host.zs.size + 16 * cap_cl + 2 * cap_adc + 8 * 440 + 64
    # budget below what one host event with host outputs needs staged: refused outright
    with make_ctx(cal.noise, cal.gain, cal.bad, hbm_budget=one // 2) as ctx:
        o = ctx.output(cap_cl, cap_adc, device=False)
        rc, _ = ctx.try_submit(host, o)
        assert rc == sc.SC_ERR_BUDGET
    # budget of ~1.5 events, one batch slot, queue of 1: submissions bounce with AGAIN while
    # the queue is full, and every accepted event still completes exactly
    with make_ctx(cal.noise, cal.gain, cal.bad, hbm_budget=int(one * 1.5), n_streams=1,
                  max_batch=1, queue_depth=1) as ctx:
        dev = host.to_device()
        accepted, again = [], 0
        for _ in range(2000):
            o = ctx.output(cap_cl, cap_adc)
            rc, t = ctx.try_submit(dev, o)
            if rc == sc.SC_OK:
                accepted.append((t, o))
            else:
                assert rc == sc.SC_ERR_AGAIN
                again += 1
            if again >= 3 and len(accepted) >= 3:
                break
        assert again >= 1
        for t, o in accepted:
            assert ctx.poll(t, -1) == sc.SC_OK
            compare_clusters(*o.to_numpy()[:2], refs[0], "budgeted")


def test_server_holds_within_budget_on_mixed_sizes(full):
    """Host events and host outputs of uneven sizes in a random order, with a budget of about
    two and a half of the largest requests: every event completes exactly, and the device bytes
    the server held (its per-batch tables plus staging) never exceeded the budget."""
    cal, evs, refs, _ = full
    hosts = [sc.Event(e.zs, e.fed_offset) for e in evs]
    caps = [sc.safe_caps(h) for h in hosts]
    largest = max(h.zs.size + 16 * c + 2 * c2 + 8 * 441 + 64 * 1024 for h, (c, c2) in zip(hosts, caps))
    budget = int(2.5 * largest)
    rng = np.random.default_rng(7)
    order = rng.permutation(np.repeat(np.arange(len(evs)), 4))
    with make_ctx(cal.noise, cal.gain, cal.bad, hbm_budget=budget, max_batch=4, n_streams=2) as ctx:
        served = []
        for i in order:
            o = ctx.output(*caps[i], device=False)
            served.append((int(i), ctx.submit(hosts[i], o), o))
        for i, t, o in served:
            assert ctx.poll(t, -1) == sc.SC_OK
            compare_clusters(*o.to_numpy()[:2], refs[i], f"budgeted event {i}")
        st = ctx.stats()
        assert st["server_budget"] == budget
        assert 0 < st["server_held_peak"] <= budget
        assert st["server_events"] == len(order)
    # a budget below the per-batch tables is refused when the server starts
    with make_ctx(cal.noise, cal.gain, cal.bad, hbm_budget=4096, max_batch=64) as ctx:
        o = ctx.output(*caps[0])
        rc, _ = ctx.try_submit(hosts[0].to_device(), o)
        assert rc == sc.SC_ERR_BUDGET


def test_autotune_identical_and_cached(full, tmp_path):
    cal, evs, refs, _ = full
    cache = str(tmp_path / "tune.json")
    with make_ctx(cal.noise, cal.gain, cal.bad, tune_cache=cache) as ctx:
        devs = [sc.Event(e.zs, e.fed_offset).to_device() for e in evs[:4]]
        best = ctx.autotune(devs)
        assert best["chunk_digis"] in (1024, 2048, 2880, 3072, 4096, 6144) and best["tile_waves"] in (1, 2, 4)
        results, _, _, _ = run_fused(ctx, [(e.zs, e.fed_offset) for e in evs[:2]])
        for r, ref in zip(results, refs[:2]):
            compare_clusters(r[0], r[1], ref, "after autotune")
    with make_ctx(cal.noise, cal.gain, cal.bad, tune_cache=cache) as ctx2:
        t = ctx2.tuning
        keys = ("chunk_digis", "tile_waves", "tiles_per_cu", "fed_major", "stage_bytes")
        assert [t[k] for k in keys] == [best[k] for k in keys]


def test_serve_replay_poisson(full):
    """Open-loop Poisson arrivals through the server: every event completes with the oracle's
    clusters, output slots are reused only after completion, latencies are positive."""
    cal, evs, refs, _ = full
    with make_ctx(cal.noise, cal.gain, cal.bad, max_batch=8, n_streams=2) as ctx:
        devs = [sc.Event(e.zs, e.fed_offset).to_device() for e in evs]
        outs = [ctx.output(*sc.safe_caps(devs[j % len(devs)])) for j in range(2 * len(devs))]
        rc, lat, eps, ph = ctx.serve_replay(devs, outs, 300, rate_hz=20000.0, seed=3,
                                            phases=True)
        assert rc == sc.SC_OK
        assert lat.shape == (300,) and (lat > 0).all()
        # the phases are non-negative and together within the latency
        assert ph.shape == (300, 3) and (ph >= 0).all() and (ph[:, 2] > 0).all()
        assert (ph.sum(axis=1) <= lat + 1.0).all()
        assert eps > 0
        for j, o in enumerate(outs):
            compare_clusters(*o.to_numpy()[:2], refs[j % len(devs)], f"replay slot {j}")
