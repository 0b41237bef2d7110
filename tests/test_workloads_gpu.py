"""Full-size workloads in the launch configuration the benchmark times:
every image's codes and histograms bit-exact against the C oracle (run over
the images on the host's cores), plus the properties that hold at any size."""
import numpy as np
import pytest

from conftest import gpu_available
from oracle import native as oracle_c
from paper_1810_11518_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_1810_11518_amd import binding
    binding.load()
    return binding


def _run(lib, name, k, n=None):
    from paper_1810_11518_amd import autotune
    w = synth.WORKLOADS[name]
    Hs, Ws = synth.workload_sizes(name, n)
    off, strides, total = synth.layout(Hs, Ws)
    host = torch.empty(total + 64, dtype=torch.uint8, pin_memory=True)
    synth.fill(host.numpy(), off, Hs, Ws, strides, w["kind"], synth.SEEDS[name])
    img = host.cuda()
    Hc, Wc = Hs.astype(np.int64) - 2, Ws.astype(np.int64) - 2
    coff = np.concatenate([[0], np.cumsum(Hc * Wc)])
    codes = torch.empty(int(coff[-1]) + 64, dtype=torch.uint8, device="cuda")
    cy, cx = w["cells"]
    hist = torch.empty(len(Hs) * cy * cx * 256, dtype=torch.int32, device="cuda")
    descs = lib.BatchPlan.descs([img.data_ptr() + int(o) for o in off],
                                [codes.data_ptr() + int(o) for o in coff[:-1]],
                                [hist.data_ptr() + j * cy * cx * 1024 for j in range(len(Hs))],
                                [int(s) for s in strides], [int(h) for h in Hs],
                                [int(x) for x in Ws])
    tune = autotune.lookup(Hs, Ws, k, (cy, cx)) if n is None else None
    plan = lib.BatchPlan(len(Hs), int((Hs.astype(np.int64) * Ws).sum()), k, cy, cx, tune)
    plan.set(descs)
    plan.run()
    plan.run()
    torch.cuda.synchronize()
    return Hs, Ws, off, strides, host.numpy(), codes, coff, hist.view(len(Hs), cy, cx, 256), (cy, cx)


def _check_all(Hs, Ws, off, strides, host, codes, coff, hist, cells, k):
    """Every image of the batch against the oracle, element by element."""
    want_c, want_off, want_h = oracle_c.ldp_extract_batch(host, off, Hs, Ws, strides, k, *cells)
    assert (want_off == coff).all()
    got_c = codes[:int(coff[-1])].cpu().numpy()
    bad = np.flatnonzero(got_c != want_c)
    assert bad.size == 0, ("codes differ", int(np.searchsorted(coff, bad[0], side="right") - 1))
    got_h = hist.cpu().numpy().view(np.uint32)
    diff = np.flatnonzero((got_h != want_h).reshape(len(Hs), -1).any(axis=1))
    assert diff.size == 0, ("histograms differ", diff[:8].tolist())


def _check_mass(Hs, Ws, hist, k):
    h = hist.cpu().numpy().view(np.uint32).astype(np.int64)
    mass = h.sum(axis=(1, 2, 3))
    assert (mass == (Hs.astype(np.int64) - 2) * (Ws.astype(np.int64) - 2)).all()
    low = [v for v in range(256) if bin(v).count("1") < k]
    assert h[..., low].sum() == 0


def test_batch_workload_full_size(lib):
    """4096 x 490x640, k=3, 7x6 cells."""
    r = _run(lib, "batch", 3)
    Hs, Ws, hist = r[0], r[1], r[7]
    _check_all(*r, k=3)
    _check_mass(Hs, Ws, hist, 3)


def test_uneven_workload_full_size(lib):
    """10,000 images with sides uniform in [48, 1024], k=3, 7x6 cells."""
    r = _run(lib, "uneven", 3)
    Hs, Ws, hist = r[0], r[1], r[7]
    _check_all(*r, k=3)
    _check_mass(Hs, Ws, hist, 3)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_large_workload_subset(lib, k):
    """8192x8192 images of the bandwidth workload (flat patches), 16x16 cells:
    the batch path on 4 of the 64 images, all four checked against the
    oracle."""
    r = _run(lib, "large", k, n=4)
    Hs, Ws, hist = r[0], r[1], r[7]
    _check_all(*r, k=k)
    _check_mass(Hs, Ws, hist, k)


def test_large_workload_full_size_k3(lib):
    """All 64 images of 8192x8192 (4.3 G pixels), k=3, 16x16 cells, every
    image against the oracle."""
    r = _run(lib, "large", 3)
    Hs, Ws, hist = r[0], r[1], r[7]
    _check_all(*r, k=3)
    _check_mass(Hs, Ws, hist, 3)
