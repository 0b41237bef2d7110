"""The algorithmic VALU figures that bench.py reports against the ALU roofline
(wave instructions per 8-pixel row step in the main row loop of
batch_kernel<k>) must be those of the code generated from the current
sources: compile the batch kernels to gfx950 assembly and count."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1810_11518_amd import build  # noqa: E402


def _blocks(body):
    """Basic blocks of one function: (label, loop comment text, instructions)."""
    out = []
    cur = ["entry", "", []]
    for line in body.split("\n")[1:]:
        t = line.strip()
        m = re.match(r"^(\.LBB\d+_\d+):\s*(;.*)?$", t)
        if m:
            out.append(cur)
            cur = [m.group(1), m.group(2) or "", []]
        elif t.startswith(";") and not cur[2]:
            cur[1] += " " + t
        elif t and not t.startswith((".", ";")):
            cur[2].append(t.split()[0])
    out.append(cur)
    return out


def main_loop_valu(asm, k, mode, copies=1):
    """Fewest VALU instructions of any main row loop of batch_kernel<k, mode,
    copies>: the innermost loops that hold 24 LDS instructions (the
    x3-unrolled row loop, 8 per row step).  Each task layout has one such loop
    for waves whose rows all start 4-aligned and one for the rest; the aligned
    one, which most waves run, has the fewest."""
    m = re.search(r"^(_ZN3ldp12batch_kernelILi%dELi%dELi%dEEEv\w*):" % (k, mode, copies), asm,
                  re.M)
    assert m, "batch_kernel<%d, %d, %d> not found" % (k, mode, copies)
    i = m.start()
    return _loop_valu(asm[i:asm.index(".Lfunc_end", i)])


def _loop_valu(body):
    """Fewest VALU instructions of the main row loops of one function."""
    blocks = _blocks(body)
    counts = []
    for lab, com, _ in blocks:
        if "Inner Loop Header" not in com:
            continue
        hdr = lab.replace(".LBB", "BB")
        members = [b for b in blocks if b[0] == lab or ("Header=%s " % hdr) in (b[1] + " ")]
        ins = [x for b in members for x in b[2]]
        if sum(x.startswith("ds_") for x in ins) == 24:
            counts.append(sum(x.startswith("v_") for x in ins))
    assert counts, "no main row loop found"
    return min(counts)


def _function(asm, prefix):
    """The assembly of the first function whose symbol starts with `prefix`."""
    m = re.search(r"^(%s\w*):" % prefix, asm, re.M)
    assert m, prefix
    return asm[m.start():asm.index(".Lfunc_end", m.start())]


@pytest.fixture(scope="module")
def batch_asm(tmp_path_factory):
    if not os.path.exists(build.HIPCC):
        pytest.skip("hipcc not installed")
    src = os.path.join(build.CSRC, "ldp_batch.hip")
    out = str(tmp_path_factory.mktemp("isa") / "batch.s")
    cmd = [build.HIPCC] + build.COMMON + ["--cuda-device-only", "-S", src, "-o", out]
    p = subprocess.run(cmd, capture_output=True, text=True)
    assert p.returncode == 0, p.stderr[-2000:]
    return open(out).read()


def test_valu_per_row_step_matches_generated_code(batch_asm):
    asm = batch_asm
    # the kernels with one and with two LDS copies of the histograms share
    # the row loop
    for copies in (1, 2):
        for mode, table in ((0, bench.VALU_PER_ROW_STEP), (1, bench.VALU_PER_ROW_STEP_MAGNITUDE),
                            (2, bench.VALU_PER_ROW_STEP_DIRECT)):
            for k in range(1, 9):
                n = main_loop_valu(asm, k, mode, copies)
                assert table[k] * 3 == pytest.approx(n), (mode, k, copies, n)
        assert bench.VALU_PER_ROW_STEP_LBP * 3 == pytest.approx(main_loop_valu(asm, 1, 3, copies))


def test_non_temporal_stores_only_in_the_nt_kernel(batch_asm):
    """batch_kernel_nt streams its code stores and its 16-byte histogram
    flush past the caches (the `nt` cache-policy bit); the cell-grid kernels
    (one and two histogram copies) store through them."""
    nt = _function(batch_asm, "_ZN3ldp15batch_kernel_ntILi3ELi0EEEv")
    assert re.search(r"buffer_store_dword v\d+, v\d+, s\[\d+:\d+\], 0 offen.* nt", nt)
    assert re.search(r"global_store_dwordx4 .* nt", nt)
    for copies in (1, 2):
        plain = _function(batch_asm, "_ZN3ldp12batch_kernelILi3ELi0ELi%dEEEv" % copies)
        assert "buffer_store_dword" in plain and not re.search(r"_store_\w+ .* nt\b", plain)
    # the same row loop, with another cache policy on its stores
    assert _loop_valu(nt) == main_loop_valu(batch_asm, 3, 0, 1)
