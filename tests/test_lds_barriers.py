"""Every workgroup barrier in the library's gfx950 code is preceded, on every
path into it, by a wait for the wave's own LDS operations.

hipcc has been seen to drop that wait on some paths (a loop back-edge into the
barrier at the top of the next iteration), which let one wave read LDS that
another wave had stored to but whose store had not landed: wrong values in a
few percent of the calls, and only while other launches shared the compute
units.  The kernels use a barrier helper with an explicit wait; this test
compiles every source with the library's own flags and scans the assembly."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from tests.lds_barrier_scan import kernels, unsafe_barriers


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_scan_flags_a_store_left_in_flight():
    # a loop whose last LDS store reaches the barrier at its top without a wait
    bad = """
\ts_mov_b32 s0, 0
.LBB0_1:
\ts_barrier
\tds_read_b32 v1, v0
\ts_waitcnt lgkmcnt(0)
\tv_add_f32_e32 v1, 1.0, v1
\tds_write_b32 v0, v1
\ts_add_i32 s0, s0, 1
\ts_cmp_lt_i32 s0, 4
\ts_cbranch_scc1 .LBB0_1
\ts_endpgm
""".splitlines()
    found, nbar = unsafe_barriers(bad)
    assert nbar == 1 and len(found) == 1
    good = [ln.replace("\ts_cbranch_scc1", "\ts_waitcnt lgkmcnt(0)\n\ts_cbranch_scc1") for ln in bad]
    good = "\n".join(good).splitlines()
    assert unsafe_barriers(good)[0] == []
    # a cross-lane DS instruction in flight is no LDS access
    xl = [ln.replace("ds_write_b32 v0, v1", "ds_bpermute_b32 v2, v0, v1") for ln in bad]
    assert unsafe_barriers(xl)[0] == []


def test_library_barriers_wait_for_lds():
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    from paper_1205_2584_amd import build

    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        flags = [f for f in build.FLAGS if f != "-fPIC"]

        def asm(src):
            out = os.path.join(tmp, os.path.splitext(src)[0] + ".s")
            cmd = [hipcc, *flags, "--cuda-device-only", "-S", os.path.join(build.CSRC, src), "-o", out]
            r = subprocess.run(cmd, capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-2000:]
            return src, out

        with ThreadPoolExecutor(max_workers=4) as ex:
            outs = list(ex.map(asm, build.SOURCES))
        problems, total = [], 0
        for src, path in outs:
            with open(path) as f:
                text = f.read()
            for name, lines in kernels(text):
                found, nbar = unsafe_barriers(lines)
                total += nbar
                problems += [(src, name, b, k) for b, k in found]
    assert total > 100  # the scan saw the kernels' barriers
    assert not problems, problems
