"""The C-ABI library loads without a GPU, exports every entry point include/sc.h declares, and
the Python binding's structures match the C layouts. No compute calls (no GPU here)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2101_11489_amd as sc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sc.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sc_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(sc.LIB_PATH):
        from paper_2101_11489_amd import build
        build.build()
    return sc.lib()


def test_every_declared_symbol_is_exported(built):
    names = declared_functions()
    assert set(names) == set(sc.EXPORTED), names
    out = subprocess.run(["nm", "-D", "--defined-only", sc.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sc_[a-z_]+)\b", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(built, n)


def test_struct_layouts_match_header(tmp_path):
    prog = tmp_path / "sizes.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "sc.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(sc_calib), sizeof(sc_options), sizeof(sc_event),
         sizeof(sc_cluster_rec), sizeof(sc_clusters), sizeof(sc_tuning), sizeof(sc_stats));
  printf("%zu %zu %zu %zu\\n", offsetof(sc_clusters, n_cl), offsetof(sc_clusters, adc),
         offsetof(sc_clusters, chan_status), offsetof(sc_clusters, mem));
  return 0;
}
""")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o",
                    str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(x) for x in lines[0].split()]
    want = [ctypes.sizeof(sc.ScCalib), ctypes.sizeof(sc.ScOptions), ctypes.sizeof(sc.ScEvent),
            sc.CLUSTER_DTYPE.itemsize, ctypes.sizeof(sc.ScClusters), ctypes.sizeof(sc.ScTuning),
            ctypes.sizeof(sc.ScStats)]
    assert sizes == want
    assert sizes[3] == 16
    offs = [int(x) for x in lines[1].split()]
    assert offs == [sc.ScClusters.n_cl.offset, sc.ScClusters.adc.offset,
                    sc.ScClusters.chan_status.offset, sc.ScClusters.mem.offset]


def test_create_without_gpu_fails_cleanly(built):
    """With no GPU the library reports an error instead of crashing, and the binding never
    falls back to a CPU path."""
    import numpy as np
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    cal = sc.ScCalib(1, np.zeros(1).ctypes.data, 0, 0, 3.0, 2.0, 5.0)
    h = ctypes.c_void_p()
    rc = built.sc_create(ctypes.byref(cal), None, ctypes.byref(h))
    assert rc == sc.SC_ERR_INVALID_ARG and not h.value
    assert built.sc_last_error(None)


def test_unknown_memory_kinds_are_refused(built):
    """sc_unpack and sc_cluster accept only SC_MEM_HOST and SC_MEM_DEVICE for the buffer they
    name; anything else is refused before any other check (no device is touched)."""
    import numpy as np
    buf = np.zeros(64, dtype=np.uint8)
    fo = np.zeros(2, dtype=np.uint64)
    ev = sc.ScEvent(buf.ctypes.data, fo.ctypes.data, sc.SC_MEM_HOST)
    for bad in (2, -1, 7):
        rc = built.sc_unpack(None, ctypes.byref(ev), buf.ctypes.data, None, bad)
        assert rc == sc.SC_ERR_INVALID_ARG
        assert b"out_mem" in built.sc_last_error(None)
        out = sc.ScClusters()
        rc = built.sc_cluster(None, buf.ctypes.data, bad, ctypes.byref(out))
        assert rc == sc.SC_ERR_INVALID_ARG
        assert b"in_mem" in built.sc_last_error(None)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(sc, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(sc, "_lib", None)
    with pytest.raises(ImportError):
        sc.lib()


def test_batch_marshals_once_and_aliases_counts(built):
    """A prepared batch holds the argument arrays of sc_process_events; each output's count
    fields are the batch's array entries, so counts the library writes there show in the
    outputs (host buffers: no GPU needed)."""
    n_fed = 2
    evs = [sc.Event(np.arange(10 + i, dtype=np.uint8), np.array([0, 4, 10 + i], np.uint64))
           for i in range(3)]
    outs = [sc.Output(5 + i, 7 + i, n_fed, device=False) for i in range(3)]
    b = sc.Batch(evs, outs)
    assert b.n == 3
    for i in range(3):
        assert b.c_ev[i].zs == evs[i].zs.ctypes.data
        assert b.c_ev[i].fed_offset == evs[i].fed_offset.ctypes.data
        assert b.c_ev[i].mem == sc.SC_MEM_HOST
        assert (b.c_out[i].cap_cl, b.c_out[i].cap_adc) == (5 + i, 7 + i)
        b.c_out[i].n_cl, b.c_out[i].n_adc = 100 + i, 200 + i   # as the library would
    assert [(o.n_cl, o.n_adc) for o in outs] == [(100, 200), (101, 201), (102, 202)]
    with pytest.raises(ValueError):
        sc.Batch(evs, outs[:2])
