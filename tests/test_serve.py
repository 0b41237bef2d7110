"""Admission and batching policy of the request server, on the CPU.

The server's dry-run mode runs the real dispatcher (pool allocator, slots,
batch formation, completion) with no device work: each batch "completes" a
fixed time after launch.  Results are not computed here; the GPU tests check
them against the oracle.
"""
import time

import numpy as np
import pytest

from paper_1810_11518_amd import binding


def _drain(srv, n, timeout=20.0):
    done = []
    t0 = time.time()
    while len(done) < n and time.time() - t0 < timeout:
        done += srv.poll(wait_us=20000)
    return done


def _req(H, W, cells=(7, 6)):
    return np.zeros((H, W), np.uint8), np.zeros(cells[0] * cells[1] * 256, np.uint32)


def _bytes(H, W, cells=(7, 6), codes=False):
    r = lambda x: (x + 255) // 256 * 256
    return r(H * W) + (r((H - 2) * (W - 2)) if codes else 0) + r(cells[0] * cells[1] * 1024)


def test_admission_never_exceeds_pool_slots_or_depth():
    pool = 1 << 20
    srv = binding.Server(pool, max_inflight=12, max_batch=5, depth=2, k=3, cells_y=7, cells_x=6,
                         dry_run=True, dry_run_us=3000)
    r = np.random.default_rng(0)
    reqs = [_req(int(r.integers(9, 300)), int(r.integers(9, 300))) for _ in range(80)]
    ids = [srv.submit(im, h) for im, h in reqs]
    done = _drain(srv, len(ids))
    st = srv.stats()
    srv.close()
    assert sorted(d["id"] for d in done) == ids
    assert st["completed"] == 80 and st["rejected"] == 0
    assert st["peak_pool_bytes"] <= pool
    assert st["peak_inflight"] <= 12
    assert st["peak_batches"] <= 2
    assert st["max_batch_seen"] <= 5
    assert all(d["status"] == 0 and 1 <= d["batch_size"] <= 5 for d in done)
    # first come, first admitted
    by_id = sorted(done, key=lambda d: d["id"])
    admits = [d["t_admit"] for d in by_id]
    assert admits == sorted(admits)
    assert all(d["t_submit"] <= d["t_admit"] <= d["t_done"] for d in done)


def test_requests_that_do_not_fit_wait_instead_of_failing():
    one = _bytes(200, 200)
    srv = binding.Server(one + 100, max_inflight=64, max_batch=64, depth=4, k=3, cells_y=7,
                         cells_x=6, dry_run=True, dry_run_us=2000)
    reqs = [_req(200, 200) for _ in range(6)]
    ids = [srv.submit(im, h) for im, h in reqs]
    done = _drain(srv, 6)
    st = srv.stats()
    srv.close()
    assert len(done) == 6 and st["peak_inflight"] == 1 and st["max_batch_seen"] == 1
    assert st["launches"] == 6
    assert st["memory_waits"] == 5      # each later request waited at the head of the queue
    done.sort(key=lambda d: d["id"])
    for a, b in zip(done, done[1:]):
        assert b["t_admit"] >= a["t_done"]  # admitted only once memory came back


def test_oversize_request_is_rejected():
    srv = binding.Server(1 << 16, 8, 8, 1, 3, 7, 6, dry_run=True, dry_run_us=100)
    im, h = _req(400, 400)
    with pytest.raises(binding.LdpError) as e:
        srv.submit(im, h)
    assert e.value.status == binding.LDP_ERR_NO_MEMORY
    small = _req(20, 20)
    srv.submit(*small)
    assert len(_drain(srv, 1)) == 1
    assert srv.stats()["rejected"] == 1
    srv.close()


def test_invalid_requests_are_refused():
    srv = binding.Server(1 << 20, 8, 8, 1, 3, 7, 6, dry_run=True, dry_run_us=100)
    with pytest.raises(binding.LdpError):
        srv.submit(*_req(8, 100))            # fewer code rows than cell rows
    with pytest.raises(ValueError):
        srv.submit(np.zeros((50, 50), np.uint8), np.zeros(10, np.uint32))
    srv.close()


def test_arrivals_during_running_batches_are_admitted_then():
    """Continuous batching: a request arriving while a batch runs is admitted
    into another launch slot before that batch completes.  Eight slots: the
    four first requests take at most four launches however the dispatcher
    groups them, so a slot is always free for the late one."""
    srv = binding.Server(1 << 24, 64, 4, 8, 3, 7, 6, dry_run=True, dry_run_us=50000)
    first = [srv.submit(*_req(64, 64)) for _ in range(4)]
    time.sleep(0.01)
    later = srv.submit(*_req(64, 64))
    done = {d["id"]: d for d in _drain(srv, 5)}
    st = srv.stats()
    srv.close()
    assert done[later]["t_admit"] < done[first[0]]["t_done"]
    assert st["peak_batches"] >= 2
