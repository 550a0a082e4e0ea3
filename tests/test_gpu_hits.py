"""GPU: cluster -> global hit coordinates against the fp64 oracle.

Tolerance, from the kernel's FP32 steps (each rounds once, relative error at most 2^-24):
p = first + b, q = p - strips/2, u = q * pitch, x = fma(u, dx, ox). So
|u - u_ref| <= 2^-24 (pitch (|p| + |q|) + |u|) and |x - x_ref| <= 2^-24 |x| + |dx| |u - u_ref|,
with a 1 % margin for the second-order terms.
"""
import numpy as np
import pytest

import fedgen
import oracle
from oracle.hits import cluster_hits

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2101_11489_amd as sc  # noqa: E402
from gpu_common import make_ctx  # noqa: E402

EPS = 2.0 ** -24


def _check(got, cl, geo, where):
    ref = cluster_hits(cl, geo)
    ch = cl["channel"].astype(np.int64)
    m = geo.channel_module[ch]
    p = geo.channel_first[ch].astype(np.float64) + cl["barycenter"].astype(np.float64)
    q = p - geo.module_strips[m] / 2.0
    pitch = geo.pitch[m].astype(np.float64)
    tol_u = EPS * (pitch * (np.abs(p) + np.abs(q)) + np.abs(ref[:, 3])) * 1.01
    d = np.abs(geo.u_dir[m].astype(np.float64))
    tol = np.empty_like(ref)
    tol[:, :3] = (EPS * np.abs(ref[:, :3]) + d * tol_u[:, None]) * 1.01
    tol[:, 3] = tol_u
    err = np.abs(got.astype(np.float64) - ref)
    bad = np.argwhere(err > tol)
    assert bad.size == 0, f"{where}: {bad[:5]} got {got[bad[:5, 0]]} ref {ref[bad[:5, 0]]}"


@pytest.fixture(scope="module")
def setup():
    cfg = fedgen.CONFIGS[2]
    cal = fedgen.make_calibration(cfg)
    geo = fedgen.make_geometry(cfg)
    evs = fedgen.make_events(cfg, cal, range(4), workers=4)
    ctx = make_ctx(cal.noise, cal.gain, cal.bad)
    devs = [sc.Event(e.zs, e.fed_offset).to_device() for e in evs]
    outs = [ctx.output(*sc.safe_caps(d)) for d in devs]
    rc, _ = ctx.process_events(devs, outs)
    assert rc == sc.SC_OK
    yield cfg, cal, geo, evs, ctx, outs
    ctx.close()


def test_hits_match_oracle_full_events(setup):
    cfg, cal, geo, evs, ctx, outs = setup
    ctx.set_geometry(geo)
    hits = ctx.cluster_hits(outs)
    for i, (h, o) in enumerate(zip(hits, outs)):
        cl = o.to_numpy()[0]
        assert h.shape == (cl.size, 4) and cl.size > 100000
        _check(h.cpu().numpy(), cl, geo, f"event {i}")
        # the records are the oracle's, so the hits are those of the oracle's clusters too
        ref_cl = oracle.process_event(evs[i].zs, evs[i].fed_offset, cal.noise, cal.gain, cal.bad).cl
        np.testing.assert_array_equal(cl["channel"], ref_cl["channel"])


def test_hits_batch_equals_single_calls(setup):
    cfg, cal, geo, evs, ctx, outs = setup
    ctx.set_geometry(geo)
    together = ctx.cluster_hits(outs)
    for o, t in zip(outs, together):
        alone = ctx.cluster_hits([o])[0]
        assert torch.equal(alone, t)


def test_empty_events_and_out_of_range_channels(setup):
    cfg, cal, geo, evs, ctx, outs = setup
    ctx.set_geometry(geo)
    # an output with no clusters next to a full one, and crafted records: the last channel, the
    # first past the detector (NaN) and channel 0 at both strip edges
    empty = ctx.output(16, 16)
    empty.cs.n_cl = 0
    crafted = ctx.output(8, 8)
    recs = np.zeros(4, oracle.CLUSTER_DTYPE)
    n_ch = cfg.n_channels
    recs["channel"] = [n_ch - 1, n_ch, 0, 0]
    recs["barycenter"] = [128.5, 3.0, 0.0, 256.0]
    crafted.cl[:4].copy_(torch.from_numpy(recs.view(np.int32).reshape(4, 4).copy()))
    crafted.cs.n_cl = 4
    hits = ctx.cluster_hits([empty, outs[0], crafted])
    assert hits[0].shape == (0, 4)
    got = hits[2].cpu().numpy()
    assert np.isnan(got[1]).all()
    ok = np.array([0, 2, 3])
    _check(got[ok], recs[ok], geo, "crafted")


def test_geometry_and_argument_errors(setup):
    cfg, cal, geo, evs, ctx, outs = setup
    fresh = make_ctx(cal.noise, cal.gain, cal.bad)
    try:
        with pytest.raises(sc.ScError):
            fresh.cluster_hits(outs[:1])                    # no geometry yet
        bad = fedgen.Geometry(geo.channel_module.copy(), geo.channel_first, geo.module_strips,
                              geo.origin, geo.u_dir, geo.pitch)
        bad.channel_module[7] = geo.n_modules               # past the last module
        with pytest.raises(sc.ScError):
            fresh.set_geometry(bad)
        wide = fedgen.Geometry(geo.channel_module, geo.channel_first.copy(), geo.module_strips,
                               geo.origin, geo.u_dir, geo.pitch)
        wide.channel_first[1] = geo.module_strips[geo.channel_module[1]]   # past the module
        with pytest.raises(sc.ScError):
            fresh.set_geometry(wide)
        fresh.set_geometry(geo)
        host_out = fresh.output(8, 8, device=False)
        host_out.cs.n_cl = 1
        with pytest.raises(sc.ScError):
            fresh.cluster_hits([host_out])                  # host outputs are refused
        h = fresh.cluster_hits(outs[:1])[0]
        _check(h.cpu().numpy(), outs[0].to_numpy()[0], geo, "fresh context")
    finally:
        fresh.close()


def test_more_events_than_one_launch_covers(setup):
    """65,537 outputs (one launch covers at most 65,535 events): the first and the last carry
    full events, the rest are empty; the hits of both full ones match the oracle."""
    cfg, cal, geo, evs, ctx, outs = setup
    ctx.set_geometry(geo)
    empty = ctx.output(16, 16)
    empty.cs.n_cl = 0
    many = [outs[0]] + [empty] * 65535 + [outs[1]]
    rows = [max(1, min(o.cs.n_cl, o.cs.cap_cl)) for o in (outs[0], empty, outs[1])]
    big = torch.empty((rows[0] + 65535 * rows[1] + rows[2], 4), dtype=torch.float32, device="cuda")
    views, at = [], 0
    for k in range(len(many)):
        r = rows[0] if k == 0 else rows[2] if k == len(many) - 1 else rows[1]
        views.append(big[at:at + r])
        at += r
    got = ctx.cluster_hits(many, hits=views)
    _check(got[0].cpu().numpy(), outs[0].to_numpy()[0], geo, "first of 65537")
    _check(got[-1].cpu().numpy(), outs[1].to_numpy()[0], geo, "last of 65537")
