"""Build properties of the tracking kernels (compiled for gfx950 on the CPU, not run).

The tracking kernels are built for a number of waves per SIMD (FP64: four static, three
persistent; mixed: eight / six for endpoint runs, six / four otherwise); the register allocator
then moves a few rarely used values (constants of the accurate phase of the correctly rounded
functions) to scratch.  The tests bound that: no kernel other than the
tracking kernels uses scratch at all, and no tracking kernel uses more than 96 bytes per lane
(dynamic indexing of the per-lane arrays, which would put every step's state in memory, costs
more: 184 bytes in the quadtree transfer before it was written with selects).  The occupancy
floor keeps the wave counts the kernels were tuned for."""
import os
import re
import shutil
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def usage():
    sys.path.insert(0, ROOT)
    from paper_2302_13590_amd import build as B
    if not os.path.exists(B.HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    src = os.path.join(B.CSRC, "pt_kernels.hip")
    with tempfile.TemporaryDirectory() as d:
        flags = [f for f in B.FLAGS if f not in ("-shared", "-fPIC")]
        r = subprocess.run([B.HIPCC] + flags + ["-I", B.INCLUDE, "-c", src, "-o", os.path.join(d, "k.o"),
                            "-Rpass-analysis=kernel-resource-usage"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = {}
    name = None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            out[name] = {}
            continue
        m = re.search(r"remark: \s*([A-Za-z ]+?)(?: \[[^\]]*\])?: (\d+)", line)
        if name and m:
            out[name][m.group(1).strip()] = int(m.group(2))
    assert out, "no resource remarks parsed"
    return out


MAX_TRACK_SCRATCH = 96


def test_scratch_bounded(usage):
    spill = {k: v.get("ScratchSize", 0) for k, v in usage.items() if v.get("ScratchSize", 0) > 0}
    other = {k: b for k, b in spill.items() if "k_track_" not in k}
    assert not other, other
    big = {k: b for k, b in spill.items() if b > MAX_TRACK_SCRATCH}
    assert not big, big


def _waves_floor(name):
    """Waves per SIMD each tracking kernel is built for, from its template arguments
    (precision 0 = FP64, 1 = mixed; output 0 = endpoint)."""
    m = re.search(r"k_track_(static|persistent)ILi(\d)ELi(\d)ELi(\d)ELb(\d)", name)
    assert m, name
    kind, prec, out = m.group(1), int(m.group(2)), int(m.group(4))
    if kind == "static":
        return 4 if prec == 0 else (8 if out == 0 else 6)
    return 3 if prec == 0 else (6 if out == 0 else 4)


def test_tracking_kernel_occupancy(usage):
    # the careful pass (k_track_careful) runs only for the rare particles handed to it and has no
    # occupancy target
    occ = {k: v.get("Occupancy", 0) for k, v in usage.items() if re.search(r"k_track_(static|persistent)", k)}
    assert len(occ) >= 30, sorted(occ)
    low = {k: o for k, o in occ.items() if o < _waves_floor(k)}
    assert not low, low
