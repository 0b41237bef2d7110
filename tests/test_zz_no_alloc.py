"""ldp_batch_launch_noalloc through the C ABI: the same codes and histograms
as ldp_batch_launch (the existing argument-table launch on a plan) on two
calls in a row, the second with a smaller batch, outputs poisoned before each
call."""
import ctypes

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


def _batch(lib, Hs, Ws, cells, seed):
    off, strides, total = synth.layout(Hs, Ws)
    host = np.zeros(total + 64, np.uint8)
    synth.fill(host, off, Hs, Ws, strides, synth.KIND_BLUR_SP_FLAT, seed)
    dev = torch.from_numpy(host).cuda()
    n = len(Hs)
    codes = [torch.empty((int(h) - 2) * (int(w) - 2), dtype=torch.uint8, device="cuda")
             for h, w in zip(Hs, Ws)]
    hists = [torch.empty(cells + (256,), dtype=torch.int32, device="cuda") for _ in range(n)]
    descs = lib.BatchPlan.descs([dev.data_ptr() + int(o) for o in off],
                                [c.data_ptr() for c in codes], [h.data_ptr() for h in hists],
                                [int(s) for s in strides], [int(h) for h in Hs],
                                [int(w) for w in Ws])
    return dict(host=host, off=off, strides=strides, dev=dev, codes=codes, hists=hists,
                descs=descs, Hs=Hs, Ws=Ws)


def _poison(b):
    for c in b["codes"]:
        c.fill_(0xA5)
    for h in b["hists"]:
        h.fill_(-1)


def _outputs(b):
    return ([c.cpu().numpy() for c in b["codes"]],
            [h.cpu().numpy().view(np.uint32).copy() for h in b["hists"]])


@pytest.mark.parametrize("k,cells", [(3, (7, 6)), (2, (2, 70))])
def test_noalloc_matches_batch_launch_twice(lib, k, cells):
    r = np.random.default_rng(301 + k)
    # 7x6 cells: 7 items an image, 28 images = 196 items (the most); 2x70
    # cells: two runs of 35 cells per cell row, 4 items an image
    n1 = 28 if cells == (7, 6) else 20
    sizes = [(int(r.integers(cells[0] + 2, 700)), int(r.integers(cells[1] + 2, 900)))
             for _ in range(n1)]
    sizes[0] = (490, 640)
    runs = []
    for call, n in enumerate((n1, 5)):          # the second call: a smaller batch
        Hs = np.array([h for h, _ in sizes[:n]], dtype=np.int32)
        Ws = np.array([w for _, w in sizes[:n]], dtype=np.int32)
        got = _batch(lib, Hs, Ws, cells, 400 + call)
        ref = _batch(lib, Hs, Ws, cells, 400 + call)
        _poison(got)
        _poison(ref)
        lib.batch_launch_noalloc(got["descs"], k, *cells)
        plan = lib.BatchPlan(n, int((Hs.astype(np.int64) * Ws).sum()), k, *cells)
        plan.launch(ref["descs"])
        torch.cuda.synchronize()
        plan.close()
        gc, gh = _outputs(got)
        rc, rh = _outputs(ref)
        for j in range(n):
            assert (gc[j] == rc[j]).all(), (call, j)
            assert (gh[j] == rh[j]).all(), (call, j)
        # and one image of each call against the oracle
        j = n - 1
        H, W, s, o = int(Hs[j]), int(Ws[j]), int(got["strides"][j]), int(got["off"][j])
        img = got["host"][o:o + H * s].reshape(H, s)[:, :W]
        wc, wh = oracle_c.ldp_extract(img, k, *cells)
        assert (gc[j].reshape(wc.shape) == wc).all() and (gh[j] == wh).all(), call
        runs.append(n)
    assert runs == [n1, 5]


def test_noalloc_refuses_batches_past_its_limits(lib):
    Hs = np.full(29, 40, dtype=np.int32)
    Ws = np.full(29, 40, dtype=np.int32)
    b = _batch(lib, Hs, Ws, (7, 6), 402)
    with pytest.raises(lib.LdpError) as e:        # 29 images
        lib.batch_launch_noalloc(b["descs"], 3, 7, 6)
    assert e.value.status == lib.LDP_ERR_UNSUPPORTED
    few = (lib.ImageDesc * 28)(*b["descs"][:28])
    with pytest.raises(lib.LdpError) as e:        # 28 x 8 = 224 work items
        lib.batch_launch_noalloc(few, 3, 8, 6)
    assert e.value.status == lib.LDP_ERR_UNSUPPORTED


def test_noalloc_replays_under_graph_capture(lib):
    """The callers it is for: a HIP graph captured around the call, replayed
    three times with eager work (poisoning the outputs) and synchronisations
    between the replays; every replay equals the eager call."""
    cells = (7, 6)
    Hs = np.array([490, 77, 300], dtype=np.int32)
    Ws = np.array([640, 130, 411], dtype=np.int32)
    b = _batch(lib, Hs, Ws, cells, 410)
    _poison(b)
    lib.batch_launch_noalloc(b["descs"], 3, *cells)      # eager (first use on this GPU done)
    torch.cuda.synchronize()
    want_c, want_h = _outputs(b)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            lib.batch_launch_noalloc(b["descs"], 3, *cells)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        _poison(b)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got_c, got_h = _outputs(b)
        for j in range(len(Hs)):
            assert (got_c[j] == want_c[j]).all(), (rep, j)
            assert (got_h[j] == want_h[j]).all(), (rep, j)
