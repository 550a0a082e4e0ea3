"""Code-generation checks of the gfx950 kernels (CPU only: hipcc cross-compiles to assembly).

A wavefront runs its lanes in lock step. If the compiler turns a loop into an inner loop for
some lanes and an outer one for the others (it may do so when two branches on a lane-dependent,
loop-invariant condition meet across a back edge), the lanes of the inner loop wait for work
that only the lanes outside can produce: the wavefront never finishes. In the assembly such a
loop leaves through an exec-mask update (`s_andn2_b64 exec, exec, ...`) instead of a scalar
branch. These tests require that no loop of that kind contains a barrier or a cross-lane
operation (lanes that left the loop would be missing from it), and that no kernel spills to
scratch memory.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2101_11489_amd", "csrc", "sc_kernels.hip")

CROSS_LANE = re.compile(r"\b(v_readfirstlane\w*|v_mbcnt\w*|ds_bpermute\w*|ds_permute\w*|"
                        r"ds_swizzle\w*|s_barrier)\b|wave barrier|row_\w+|quad_perm")
LOOP_EXIT_BY_EXEC = re.compile(r"^s_andn2_b64\s+exec,\s*exec,")


def _device_asm(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    from paper_2101_11489_amd import build as b
    out = tmp_path / "kernels.s"
    cmd = ["hipcc", *b.DEVICE_FLAGS, "--cuda-device-only", "-S", "-I",
           os.path.join(ROOT, "include"), "-I", os.path.dirname(SRC), SRC, "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


def _kernels(asm):
    """{kernel symbol: [lines of its body]} for every kernel entry in the assembly."""
    out, cur = {}, None
    for ln in asm.splitlines():
        m = re.match(r"^(_Z\w+):", ln)
        if m:
            cur = m.group(1)
            out[cur] = []
            continue
        if cur is not None:
            out[cur].append(ln)
            if "s_endpgm" in ln:
                cur = None
    return out


def _loops(body):
    """{loop header: instructions of the blocks whose innermost loop it is}."""
    loops, cur_loop = {}, None
    for ln in body:
        m = re.match(r"^(\.LBB\d+_\d+|; %bb\.\d+):", ln)
        if m:
            name = m.group(1).lstrip(".L")
            if re.search(r"Loop Header: Depth=", ln):
                cur_loop = name
            else:
                h = re.search(r"Header=(BB\d+_\d+) Depth=", ln)
                cur_loop = h.group(1) if h else None
            continue
        if re.search(r"Loop Header: Depth=", ln):
            # header comment on its own line right after the label
            continue
        if cur_loop is None:
            continue
        s = ln.strip()
        if s and (not s.startswith(";") or "wave barrier" in s):
            loops.setdefault(cur_loop, []).append(s)
    return loops


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    return _kernels(_device_asm(tmp_path_factory.mktemp("asm")))


def test_every_kernel_is_present(kernels):
    names = " ".join(kernels)
    for k in ("fused_kernel", "cluster_dense_kernel", "unpack_kernel", "reset_kernel",
              "derive_calib_kernel"):
        assert k in names


def test_no_lane_split_loop_holds_cross_lane_work(kernels):
    bad = []
    for name, body in kernels.items():
        for header, ins in _loops(body).items():
            if not any(LOOP_EXIT_BY_EXEC.match(i) for i in ins):
                continue
            xl = [i for i in ins if CROSS_LANE.search(i)]
            if xl:
                bad.append(f"{name} loop {header}: {xl[:3]}")
    assert not bad, "\n".join(bad)


def test_the_tile_loop_is_left_by_a_scalar_branch(kernels):
    """The persistent loop of each tile kernel holds the queue atomic; its header must not sit
    inside a loop with an exec-mask exit."""
    for name, body in kernels.items():
        if "fused_kernel" not in name and "cluster_dense_kernel" not in name:
            continue
        loops = _loops(body)
        holders = [h for h, ins in loops.items() if any(i.startswith("global_atomic_add") for i in ins)]
        assert holders, name
        for h in holders:
            assert not any(LOOP_EXIT_BY_EXEC.match(i) for i in loops[h]), f"{name} loop {h}"


def test_no_scratch(kernels, tmp_path):
    asm = _device_asm(tmp_path)
    sizes = re.findall(r"\.private_segment_fixed_size:\s+(\d+)", asm)
    assert sizes and all(int(x) == 0 for x in sizes)
