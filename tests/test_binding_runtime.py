"""The binding loads libldp.so against the HIP runtime torch uses: one HIP
runtime library in the process even when the binding is loaded before torch
is imported (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(not os.path.exists(os.path.join(ROOT, "paper_1810_11518_amd", "libldp.so")),
                    reason="libldp.so not built")
def test_one_hip_runtime_when_binding_loads_first():
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1810_11518_amd import binding\n"
        "binding.load()\n"
        "import torch\n"
        "libs = sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l})\n"
        "print(len(libs)); print(libs)\n" % ROOT)
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = p.stdout.strip().splitlines()
    assert lines[0] == "1", lines


@pytest.mark.parametrize("n", [0, 2, 8])
def test_bench_refuses_other_gpu_counts(n):
    """bench.py measures one GPU: any other --gpus value exits with status 2
    and says why, before it touches a device."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2, (p.returncode, p.stderr[-500:])
    assert "one GPU" in p.stderr and p.stdout == ""
