"""ctypes binding of the plain C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's CPU-baseline
leg; the GPU library and its Python binding never import it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CLUSTER_DTYPE = np.dtype([("channel", "<u4"), ("first", "<u2"), ("width", "<u2"),
                          ("charge", "<u4"), ("barycenter", "<f4")])
assert CLUSTER_DTYPE.itemsize == 16

CH_MALFORMED = 1
FED_TRAILING = 2
T_SEED, T_CHANNEL, T_CLUSTER = 3.0, 2.0, 5.0

_lib = None


GCC_FLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fno-finite-math-only",
             "-Wall", "-Wextra", "-fPIC", "-shared"]


def build(force: bool = True, src: str = SRC, out: str = LIB) -> str:
    """Compile liboracle.so with gcc (plain C99, no fast-math, no FP contraction)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-I", HERE, "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def lib():
    """The loaded oracle. ORACLE_LIB may name another build of oracle.c (the mutation test
    uses it to load deliberately broken variants)."""
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB", LIB)
        if path == LIB and not os.path.exists(LIB):
            build(force=True)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        u32, u64, f32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float
        L.oracle_unpack.argtypes = [P, P, u32, P, P]
        L.oracle_unpack.restype = ctypes.c_int
        L.oracle_flags.argtypes = [P, u32, P, P, P, f32, f32, P]
        L.oracle_flags.restype = None
        L.oracle_cluster.argtypes = [P, u32, P, P, P, f32, f32, f32, P, u64, P, u64, P, P]
        L.oracle_cluster.restype = ctypes.c_int
        L.oracle_process_event.argtypes = [P, P, u32, P, P, P, f32, f32, f32, P, P, P, u64, P,
                                           u64, P, P]
        L.oracle_cluster_modules.argtypes = [P, u32, P, P, P, f32, f32, f32, P, P, u64, P, u64,
                                             P, P]
        L.oracle_cluster_modules.restype = ctypes.c_int
        L.oracle_process_event.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Clusters:
    cl: np.ndarray       # CLUSTER_DTYPE [n_cl]
    adc: np.ndarray      # uint16 [n_adc], member ADCs cluster after cluster
    status: int = 0
    chan_status: np.ndarray | None = None

    @property
    def n_cl(self) -> int:
        return int(self.cl.size)


def unpack(zs: np.ndarray, fed_offset: np.ndarray):
    zs = np.ascontiguousarray(zs, dtype=np.uint8)
    fo = np.ascontiguousarray(fed_offset, dtype=np.uint64)
    n_fed = fo.size - 1
    adc = np.empty(n_fed * 96 * 256, dtype=np.uint8)
    st = np.empty(n_fed * 96, dtype=np.uint8)
    zsp = zs if zs.size else np.zeros(1, np.uint8)
    rc = lib().oracle_unpack(_p(zsp), _p(fo), n_fed, _p(adc), _p(st))
    return adc, st, int(rc)


def flags(adc, noise, gain, bad, t_seed=T_SEED, t_channel=T_CHANNEL):
    adc = np.ascontiguousarray(adc, dtype=np.uint8)
    n_fed = adc.size // (96 * 256)
    out = np.empty_like(adc)
    lib().oracle_flags(_p(adc), n_fed, _p(np.ascontiguousarray(noise, np.float32)),
                       _p(np.ascontiguousarray(gain, np.float32)),
                       _p(np.ascontiguousarray(bad, np.uint8)), t_seed, t_channel, _p(out))
    return out


def cluster(adc, noise, gain, bad, t_seed=T_SEED, t_channel=T_CHANNEL, t_cluster=T_CLUSTER,
            cap_cl=None, cap_adc=None, joins=None) -> Clusters:
    """Three-threshold clustering of dense ADCs; with joins (u8 per channel, nonzero: the channel
    reads the same module as the previous channel of its FED) the module-aware variant."""
    if joins is not None:
        return _cluster_modules(adc, noise, gain, bad, t_seed, t_channel, t_cluster, cap_cl,
                                cap_adc, joins)
    adc = np.ascontiguousarray(adc, dtype=np.uint8)
    n_fed = adc.size // (96 * 256)
    assert adc.size == n_fed * 96 * 256
    noise = np.ascontiguousarray(noise, np.float32)
    gain = np.ascontiguousarray(gain, np.float32)
    bad = np.ascontiguousarray(bad, np.uint8)
    n_cl = ctypes.c_uint64()
    n_adc = ctypes.c_uint64()
    # counting pass, then an exact-size pass
    lib().oracle_cluster(_p(adc), n_fed, _p(noise), _p(gain), _p(bad), t_seed, t_channel,
                         t_cluster, None, 0, None, 0, ctypes.byref(n_cl), ctypes.byref(n_adc))
    ncl = n_cl.value if cap_cl is None else cap_cl
    nadc = n_adc.value if cap_adc is None else cap_adc
    cl = np.zeros(max(ncl, 1), dtype=CLUSTER_DTYPE)
    out_adc = np.zeros(max(nadc, 1), dtype=np.uint16)
    rc = lib().oracle_cluster(_p(adc), n_fed, _p(noise), _p(gain), _p(bad), t_seed, t_channel,
                              t_cluster, _p(cl), ncl, _p(out_adc), nadc, ctypes.byref(n_cl),
                              ctypes.byref(n_adc))
    return Clusters(cl[:min(ncl, n_cl.value)], out_adc[:min(nadc, n_adc.value)], int(rc))


def _cluster_modules(adc, noise, gain, bad, t_seed, t_channel, t_cluster, cap_cl, cap_adc,
                     joins) -> Clusters:
    adc = np.ascontiguousarray(adc, dtype=np.uint8)
    n_fed = adc.size // (96 * 256)
    assert adc.size == n_fed * 96 * 256
    noise = np.ascontiguousarray(noise, np.float32)
    gain = np.ascontiguousarray(gain, np.float32)
    bad = np.ascontiguousarray(bad, np.uint8)
    joins = np.ascontiguousarray(joins, np.uint8)
    assert joins.size == n_fed * 96
    n_cl = ctypes.c_uint64()
    n_adc = ctypes.c_uint64()
    L = lib()
    L.oracle_cluster_modules(_p(adc), n_fed, _p(noise), _p(gain), _p(bad), t_seed, t_channel,
                             t_cluster, _p(joins), None, 0, None, 0, ctypes.byref(n_cl),
                             ctypes.byref(n_adc))
    ncl = n_cl.value if cap_cl is None else cap_cl
    nadc = n_adc.value if cap_adc is None else cap_adc
    cl = np.zeros(max(ncl, 1), dtype=CLUSTER_DTYPE)
    out_adc = np.zeros(max(nadc, 1), dtype=np.uint16)
    rc = L.oracle_cluster_modules(_p(adc), n_fed, _p(noise), _p(gain), _p(bad), t_seed,
                                  t_channel, t_cluster, _p(joins), _p(cl), ncl, _p(out_adc), nadc,
                                  ctypes.byref(n_cl), ctypes.byref(n_adc))
    return Clusters(cl[:min(ncl, n_cl.value)], out_adc[:min(nadc, n_adc.value)], int(rc))


def process_event(zs, fed_offset, noise, gain, bad, t_seed=T_SEED, t_channel=T_CHANNEL,
                  t_cluster=T_CLUSTER, joins=None) -> Clusters:
    adc, st, rc = unpack(zs, fed_offset)
    out = cluster(adc, noise, gain, bad, t_seed, t_channel, t_cluster, joins=joins)
    out.status = rc
    out.chan_status = st
    return out


def process_event_raw(zs, fed_offset, noise, gain, bad, scratch, cl, out_adc,
                      t_seed=T_SEED, t_channel=T_CHANNEL, t_cluster=T_CLUSTER):
    """Single C call into preallocated buffers (used to time the oracle)."""
    n_cl = ctypes.c_uint64()
    n_adc = ctypes.c_uint64()
    fo = fed_offset
    rc = lib().oracle_process_event(_p(zs), _p(fo), fo.size - 1, _p(noise), _p(gain), _p(bad),
                                    t_seed, t_channel, t_cluster, _p(scratch), None, _p(cl),
                                    cl.size, _p(out_adc), out_adc.size, ctypes.byref(n_cl),
                                    ctypes.byref(n_adc))
    return rc, n_cl.value, n_adc.value
