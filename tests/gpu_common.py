"""Shared pieces of the GPU tests: contexts, oracle comparison with the stated tolerance."""
from __future__ import annotations

import numpy as np

import oracle
import paper_2101_11489_amd as sc

BARY_RTOL = 1e-6   # barycenter tolerance (relative, FP32); everything else must be bit-exact


def compare_clusters(got_cl, got_adc, ref: "oracle.Clusters", where=""):
    """Cluster membership, ranges, charges and member ADCs bit-exact; barycenters within 1e-6
    relative (they are in fact expected to be bit-exact, which is checked separately)."""
    assert got_cl.size == ref.cl.size, f"{where}: {got_cl.size} clusters vs {ref.cl.size}"
    for f in ("channel", "first", "width", "charge"):
        if not np.array_equal(got_cl[f], ref.cl[f]):
            bad = np.flatnonzero(got_cl[f] != ref.cl[f])[:5]
            raise AssertionError(f"{where}: field {f} differs at {bad}: {got_cl[bad]} vs {ref.cl[bad]}")
    np.testing.assert_allclose(got_cl["barycenter"], ref.cl["barycenter"], rtol=BARY_RTOL, atol=0,
                               err_msg=where)
    assert np.array_equal(got_adc, ref.adc), f"{where}: member ADCs differ"


def bary_bit_exact(got_cl, ref):
    return np.array_equal(got_cl["barycenter"].view(np.uint32), ref.cl["barycenter"].view(np.uint32))


def make_ctx(noise, gain, bad, **kw):
    return sc.Context(noise, gain, bad, device=0, **kw)


def run_fused(ctx, events_np, device=True, caps=None, chan_status=False):
    """events_np: list of (zs, fed_offset) numpy pairs -> list of (cl, adc, chan_status), rc, sts."""
    evs = [sc.Event(zs, fo) for zs, fo in events_np]
    if device:
        evs = [e.to_device() for e in evs]
    outs = []
    for e in evs:
        cc, ca = caps if caps is not None else sc.safe_caps(e)
        outs.append(ctx.output(cc, ca, device=device, chan_status=chan_status))
    rc, sts = ctx.process_events(evs, outs)
    return [o.to_numpy() for o in outs], rc, sts, outs
