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
    body = asm[i:asm.index(".Lfunc_end", i)]
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
    assert counts, "no main row loop found in batch_kernel<%d, %d>" % (k, mode)
    return min(counts)


@pytest.mark.skipif(not os.path.exists(build.HIPCC), reason="hipcc not installed")
def test_valu_per_row_step_matches_generated_code(tmp_path):
    src = os.path.join(build.CSRC, "ldp_batch.hip")
    out = str(tmp_path / "batch.s")
    cmd = [build.HIPCC] + build.COMMON + ["--cuda-device-only", "-S", src, "-o", out]
    p = subprocess.run(cmd, capture_output=True, text=True)
    assert p.returncode == 0, p.stderr[-2000:]
    asm = open(out).read()
    # the kernels with one and with two LDS copies of the histograms share
    # the row loop
    for copies in (1, 2):
        for mode, table in ((0, bench.VALU_PER_ROW_STEP), (1, bench.VALU_PER_ROW_STEP_MAGNITUDE),
                            (2, bench.VALU_PER_ROW_STEP_DIRECT)):
            for k in range(1, 9):
                n = main_loop_valu(asm, k, mode, copies)
                assert table[k] * 3 == pytest.approx(n), (mode, k, copies, n)
        assert bench.VALU_PER_ROW_STEP_LBP * 3 == pytest.approx(main_loop_valu(asm, 1, 3, copies))
