"""Global hit coordinates of clusters: plain fp64 NumPy.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's checks; the GPU library and
its Python binding never import it.

The paper names this conversion as the step that follows clustering (§5, Conclusions: clusters
are turned into global hit coordinates as input for tracking) and does not define it. Reading
used here, for planar modules with parallel strips:
  * a cluster's position across its module, in strip pitches from the module's first strip
    edge, is p = channel_first[channel] + barycenter (the barycenter is channel-local, strip s
    spanning [s, s+1));
  * the local coordinate from the module centre is u = (p - module_strips / 2) * pitch;
  * the global hit is origin + u * u_dir (the module centre plus u along the measurement
    direction); the position along the strips is not measured and taken at the centre.
Every step is in float64 on the float32 inputs.
"""
from __future__ import annotations

import numpy as np


def cluster_hits(cl: np.ndarray, geom) -> np.ndarray:
    """cl: cluster records (fields channel, barycenter); geom: channel_module, channel_first,
    module_strips, origin [M, 3], u_dir [M, 3], pitch. Returns float64 [n, 4]: x, y, z, u."""
    ch = np.asarray(cl["channel"], dtype=np.int64)
    m = np.asarray(geom.channel_module, dtype=np.int64)[ch]
    p = (np.asarray(geom.channel_first, dtype=np.float64)[ch]
         + np.asarray(cl["barycenter"], dtype=np.float32).astype(np.float64))
    half = np.asarray(geom.module_strips, dtype=np.float64)[m] / 2.0
    u = (p - half) * np.asarray(geom.pitch, dtype=np.float32).astype(np.float64)[m]
    o = np.asarray(geom.origin, dtype=np.float32).astype(np.float64)[m]
    d = np.asarray(geom.u_dir, dtype=np.float32).astype(np.float64)[m]
    out = np.empty((ch.size, 4), dtype=np.float64)
    out[:, :3] = o + u[:, None] * d
    out[:, 3] = u
    return out
