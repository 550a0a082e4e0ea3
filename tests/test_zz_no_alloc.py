"""GPU: the allocation-free batch call (sc_process_events_static) against sc_process_events.

Called through the C ABI: two calls in a row, the second with fewer events, each compared with
sc_process_events on the same device events (clusters, member ADCs, counts and statuses
bit-exact), no allocation by the library across the calls, and the refused arguments.
"""
import ctypes

import numpy as np
import pytest

import fedgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2101_11489_amd as sc  # noqa: E402
from gpu_common import compare_clusters, make_ctx  # noqa: E402


def _static(ctx, devs, outs):
    b = ctx.batch(devs, outs)
    torch.cuda.synchronize()
    rc = sc.lib().sc_process_events_static(ctx._h, b.c_ev, b.n, b.c_out, b.c_st)
    torch.cuda.synchronize()
    return rc, list(b.c_st)


def test_static_call_matches_process_events_twice():
    cfg = fedgen.CONFIGS[2].with_(n_fed=40)
    cal = fedgen.make_calibration(cfg)
    evs = [fedgen.make_event(cfg, cal, i) for i in range(6)]
    with make_ctx(cal.noise, cal.gain, cal.bad) as ctx:
        devs = [sc.Event(e.zs, e.fed_offset).to_device() for e in evs]
        for call, idx in enumerate(([0, 1, 2, 3, 4, 5], [5, 2])):   # the second call is smaller
            sel = [devs[i] for i in idx]
            ref_outs = [ctx.output(*sc.safe_caps(d)) for d in sel]
            rc_ref, st_ref = ctx.process_events(sel, ref_outs)
            torch.cuda.synchronize()
            outs = [ctx.output(*sc.safe_caps(d)) for d in sel]
            for o in outs:   # garbage where nothing is written, to catch stale reads
                o.cl.fill_(0xAB)
                o.adc.fill_(0xCD)
            allocs = ctx.stats()["allocations"]
            rc, st = _static(ctx, sel, outs)
            assert ctx.stats()["allocations"] == allocs, "the static call allocated"
            assert rc == rc_ref and st == st_ref, (call, rc, rc_ref, st, st_ref)
            for k, (o, r) in enumerate(zip(outs, ref_outs)):
                assert (o.n_cl, o.n_adc) == (r.n_cl, r.n_adc)
                cl, adc, _ = o.to_numpy()
                rcl, radc, _ = r.to_numpy()
                assert np.array_equal(cl, rcl) and np.array_equal(adc, radc), (call, k)
            # and one event against the oracle
            e = evs[idx[-1]]
            ref = oracle.process_event(e.zs, e.fed_offset, cal.noise, cal.gain, cal.bad)
            compare_clusters(*outs[-1].to_numpy()[:2], ref, f"call {call}")


def test_static_call_refusals():
    cfg = fedgen.CONFIGS[0].with_(n_fed=4)
    cal = fedgen.make_calibration(cfg)
    e = fedgen.make_event(cfg, cal, 0)
    with make_ctx(cal.noise, cal.gain, cal.bad) as ctx:
        dev = sc.Event(e.zs, e.fed_offset).to_device()
        host = sc.Event(e.zs, e.fed_offset)
        out = ctx.output(*sc.safe_caps(dev))
        b = ctx.batch([dev], [out])
        L = sc.lib()
        assert L.sc_process_events_static(ctx._h, b.c_ev, 0, b.c_out, b.c_st) == sc.SC_ERR_INVALID_ARG
        assert L.sc_process_events_static(ctx._h, b.c_ev, sc.SC_STATIC_MAX_EVENTS + 1, b.c_out,
                                          b.c_st) == sc.SC_ERR_INVALID_ARG
        assert b"SC_STATIC_MAX_EVENTS" in L.sc_last_error(ctx._h)
        hb = ctx.batch([host], [ctx.output(*sc.safe_caps(dev))])
        assert L.sc_process_events_static(ctx._h, hb.c_ev, 1, hb.c_out, hb.c_st) == sc.SC_ERR_INVALID_ARG
        assert b"device memory" in L.sc_last_error(ctx._h)
        # still usable afterwards
        rc, _ = _static(ctx, [dev], [out])
        assert rc in (sc.SC_OK, sc.SC_MALFORMED)
