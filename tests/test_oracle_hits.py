"""Pins of the hit-coordinate oracle (closed forms and geometric invariants), CPU only."""
import math
from types import SimpleNamespace

import numpy as np
import pytest

import fedgen
from oracle import CLUSTER_DTYPE
from oracle.hits import cluster_hits


def _geom(channel_module, channel_first, module_strips, origin, u_dir, pitch):
    return SimpleNamespace(channel_module=np.array(channel_module, np.uint32),
                           channel_first=np.array(channel_first, np.uint32),
                           module_strips=np.array(module_strips, np.uint32),
                           origin=np.array(origin, np.float32).reshape(-1, 3),
                           u_dir=np.array(u_dir, np.float32).reshape(-1, 3),
                           pitch=np.array(pitch, np.float32))


def _cl(channels, barys):
    cl = np.zeros(len(channels), CLUSTER_DTYPE)
    cl["channel"] = channels
    cl["barycenter"] = barys
    return cl


def test_hand_example_two_channel_module():
    # one module of two channels (512 strips), centre at the origin, measuring along x with a
    # pitch of 1/64 cm (exact in binary). A cluster in the second channel at barycenter 10.5 sits
    # at module strip position 266.5, i.e. 10.5 pitches right of the centre (256): u = 10.5/64.
    g = _geom([0, 0], [0, 256], [512], [0, 0, 0], [1, 0, 0], [1 / 64])
    h = cluster_hits(_cl([1, 0, 0], [10.5, 0.5, 256.0]), g)
    np.testing.assert_array_equal(h[0], [10.5 / 64, 0, 0, 10.5 / 64])
    # first channel, strip 0 centre: 255.5 pitches left of the module centre
    np.testing.assert_array_equal(h[1], [-255.5 / 64, 0, 0, -255.5 / 64])
    # barycenter 256 in channel 0 is the module centre
    np.testing.assert_array_equal(h[2], [0, 0, 0, 0])


def test_hand_example_offset_module_along_y():
    # three-channel module (768 strips) centred at (10, 20, -5) cm measuring along +y, pitch
    # 1/128 cm: channel 2 of the module, barycenter 0.25 -> position 512.25, 128.25 pitches above
    # the centre (384) -> y = 20 + 128.25/128.
    g = _geom([0, 0, 0], [0, 256, 512], [768], [10, 20, -5], [0, 1, 0], [1 / 128])
    h = cluster_hits(_cl([2], [0.25]), g)
    np.testing.assert_array_equal(h[0], [10, 20 + 128.25 / 128, -5, 128.25 / 128])


def test_module_centre_maps_to_origin():
    geo = fedgen.make_geometry(fedgen.CONFIGS[0])
    ch = np.arange(geo.channel_module.size)
    m = geo.channel_module[ch]
    # the barycenter that puts the cluster at the module centre: half the strips minus the
    # channel's first strip, when that falls inside the channel
    b = geo.module_strips[m] / 2.0 - geo.channel_first[ch]
    sel = (b >= 0) & (b <= 256)
    h = cluster_hits(_cl(ch[sel], b[sel].astype(np.float32)), geo)
    np.testing.assert_array_equal(h[:, :3], geo.origin[m[sel]].astype(np.float64))
    np.testing.assert_array_equal(h[:, 3], 0.0)


def test_hits_lie_on_the_measurement_line_at_distance_u():
    geo = fedgen.make_geometry(fedgen.CONFIGS[0])
    rng = np.random.default_rng(5)
    ch = rng.integers(0, geo.channel_module.size, 5000)
    b = rng.uniform(0, 256, 5000).astype(np.float32)
    h = cluster_hits(_cl(ch, b), geo)
    m = geo.channel_module[ch]
    o = geo.origin[m].astype(np.float64)
    d = geo.u_dir[m].astype(np.float64)
    rel = h[:, :3] - o
    np.testing.assert_allclose(np.cross(rel, d), 0, atol=1e-12)
    np.testing.assert_allclose(np.sum(rel * d, axis=1) / np.sum(d * d, axis=1), h[:, 3],
                               rtol=1e-12, atol=1e-12)
    # |u| is at most half the module's width
    assert np.all(np.abs(h[:, 3]) <= geo.module_strips[m] / 2 * geo.pitch[m] * (1 + 1e-12))


def test_barrel_radius_identity():
    # the measurement direction of a barrel module is tangent (perpendicular to the radius in
    # the transverse plane), so x^2 + y^2 = R^2 + u^2 (dx^2 + dy^2) and z - z0 = u dz
    geo = fedgen.make_geometry(fedgen.CONFIGS[0])
    rng = np.random.default_rng(6)
    ch = rng.integers(0, geo.channel_module.size, 3000)
    h = cluster_hits(_cl(ch, rng.uniform(0, 256, 3000).astype(np.float32)), geo)
    m = geo.channel_module[ch]
    o = geo.origin[m].astype(np.float64)
    d = geo.u_dir[m].astype(np.float64)
    u = h[:, 3]
    # the generator's tangent is perpendicular to the radius up to float32 rounding
    lhs = h[:, 0] ** 2 + h[:, 1] ** 2
    rhs = o[:, 0] ** 2 + o[:, 1] ** 2 + u ** 2 * (d[:, 0] ** 2 + d[:, 1] ** 2) \
        + 2 * u * (o[:, 0] * d[:, 0] + o[:, 1] * d[:, 1])
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)
    assert np.max(np.abs(o[:, 0] * d[:, 0] + o[:, 1] * d[:, 1])) < 1e-4
    np.testing.assert_allclose(h[:, 2] - o[:, 2], u * d[:, 2], atol=1e-12)


@pytest.mark.parametrize("angle", [0.3, 1.7, -2.9])
def test_rotating_the_geometry_rotates_the_hits(angle):
    geo = fedgen.make_geometry(fedgen.CONFIGS[0])
    rng = np.random.default_rng(7)
    ch = rng.integers(0, geo.channel_module.size, 500)
    cl = _cl(ch, rng.uniform(0, 256, 500).astype(np.float32))
    c, s = math.cos(angle), math.sin(angle)
    rot = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
    # rotate in float64 and keep only geometries that stay exact in float32: rotate the hits
    # of the float32-rounded rotated geometry and compare with the rotated hits
    g2 = SimpleNamespace(**{k: getattr(geo, k) for k in
                            ("channel_module", "channel_first", "module_strips", "pitch")})
    g2.origin = (geo.origin.astype(np.float64) @ rot.T).astype(np.float32)
    g2.u_dir = (geo.u_dir.astype(np.float64) @ rot.T).astype(np.float32)
    h = cluster_hits(cl, geo)
    h2 = cluster_hits(cl, g2)
    np.testing.assert_allclose(h2[:, :3], h[:, :3] @ rot.T, atol=2e-5)
    np.testing.assert_array_equal(h2[:, 3], h[:, 3])


def test_geometry_generator_layout():
    geo = fedgen.make_geometry(fedgen.CONFIGS[0])
    n_ch = fedgen.CONFIGS[0].n_channels
    assert geo.channel_module.size == n_ch
    # modules are 2 or 3 consecutive channels inside one block of 24, numbered from 0 in order
    counts = np.bincount(geo.channel_module)
    assert set(counts.tolist()) <= {2, 3}
    assert np.all(np.diff(geo.channel_module.astype(np.int64)) >= 0)
    blocks = np.arange(n_ch) // fedgen.MODULE_BLOCK
    first_ch = np.searchsorted(geo.channel_module, np.arange(geo.n_modules))
    assert np.array_equal(blocks[first_ch], blocks[first_ch + counts - 1])
    np.testing.assert_array_equal(geo.module_strips, counts * 256)
    np.testing.assert_allclose(np.linalg.norm(geo.u_dir.astype(np.float64), axis=1), 1, rtol=1e-6)


# ---- planted mistakes: each must fail one of the pins above --------------------------------
def _mutant(kind):
    def fn(cl, geom):
        ch = np.asarray(cl["channel"], dtype=np.int64)
        m = np.asarray(geom.channel_module, dtype=np.int64)[ch]
        first = np.asarray(geom.channel_first, dtype=np.float64)[ch]
        b = np.asarray(cl["barycenter"], dtype=np.float32).astype(np.float64)
        p = b if kind == "no_channel_offset" else first + b
        if kind == "strip_index_not_centre":
            p = first + np.floor(b)
        strips = np.asarray(geom.module_strips, dtype=np.float64)[m]
        half = strips if kind == "full_not_half" else strips / 2.0
        pitch = np.asarray(geom.pitch, dtype=np.float64)[m]
        u = (p - half) * pitch
        if kind == "flipped":
            u = -u
        o = np.asarray(geom.origin, dtype=np.float64)[m]
        d = np.asarray(geom.u_dir, dtype=np.float64)[m]
        if kind == "swapped_axes":
            d = d[:, [1, 0, 2]]
        out = np.empty((ch.size, 4))
        out[:, :3] = o + u[:, None] * d
        out[:, 3] = u
        return out
    return fn


PINS = [test_hand_example_two_channel_module, test_hand_example_offset_module_along_y,
        test_module_centre_maps_to_origin, test_hits_lie_on_the_measurement_line_at_distance_u,
        test_barrel_radius_identity]


@pytest.mark.parametrize("kind", ["no_channel_offset", "strip_index_not_centre", "full_not_half",
                                  "flipped", "swapped_axes"])
def test_planted_mistakes_are_caught(kind, monkeypatch):
    failed = 0
    for pin in PINS:
        monkeypatch.setitem(globals(), "cluster_hits", _mutant(kind))
        try:
            pin()
        except AssertionError:
            failed += 1
        finally:
            monkeypatch.undo()
    assert failed >= 1, kind
