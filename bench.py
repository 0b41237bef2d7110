"""Benchmark of the LDP hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batch]

One step = one pass of the whole path (codes of every interior pixel, top-k
selection, the 8-bit code, per-cell histograms) over one batch of synthetic
images already resident in device memory.  The headline is the persistent,
graph-captured batched launch over the 4096-image batch of 490x640 frames;
the same batch run as one launch per image ("plain") is timed beside it.
The other workloads (10,000 uneven images; 64 images of 8192x8192 for
k = 2, 3, 4), the two calls of the two-call path (ldp_codes, ldp_histograms),
the variants, serving and the CPU oracle are reported as secondary keys of
the same JSON line.  Prints ONE JSON line.
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LDP Mpixel/s + % HBM roofline (batched vs plain kernel); p50/p99 serve latency"
HBM_PEAK_GBS = 8000.0
# Single-issue VALU rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one wave64
# VALU instruction per SIMD per 4-cycle quad), in tera lane-instructions per
# second.  gfx950 can also issue two simple 32-bit VALU instructions in one
# quad (the SQ_ACTIVE_INST_VALU2 counter), so this is a utilisation scale,
# not a ceiling.
VALU_SINGLE_ISSUE_T = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU work of the batched kernel: wave instructions per 8-pixel row step of
# a lane (one wave covers 512 code pixels) in the main row loop of
# batch_kernel<k> as compiled for gfx950 (the x3-unrolled loop / 3; both
# histogram paths counted; the loop with the fewest instructions, which waves
# whose rows start 4-aligned run).  tests/test_isa_counts.py recompiles the
# kernel and checks these figures against the generated code.
VALU_PER_ROW_STEP = {1: 413 / 3, 2: 557 / 3, 3: 593 / 3, 4: 653 / 3, 5: 653 / 3, 6: 593 / 3,
                     7: 557 / 3, 8: 45 / 3}
# the same for ranking by response magnitude (flags LDP_RANK_MAGNITUDE), for
# responses computed mask by mask (LDP_DIRECT_MASKS) and for LBP labels
# (LDP_CODE_LBP, one kernel for every k)
VALU_PER_ROW_STEP_MAGNITUDE = {1: 767 / 3, 2: 911 / 3, 3: 947 / 3, 4: 1007 / 3, 5: 1007 / 3,
                               6: 947 / 3, 7: 911 / 3, 8: 45 / 3}
VALU_PER_ROW_STEP_DIRECT = {1: 1043 / 3, 2: 1187 / 3, 3: 1223 / 3, 4: 1283 / 3, 5: 1283 / 3,
                            6: 1223 / 3, 7: 1187 / 3, 8: 45 / 3}
VALU_PER_ROW_STEP_LBP = 287 / 3
# untimed work before the warm-up steps, so that timing starts at steady clocks
DEVICE_WARMUP_S = 0.3
# the paper's own CPU timings (Table 2, one image): the direct eight-mask LDP
# and the accelerated scheme, Python on an Intel Core i5-3230M
PAPER_CPU = {"ldp_s_per_image": 11.04, "aldp_s_per_image": 2.81, "aldp_over_ldp": 3.93,
             "hardware": "Intel Core i5-3230M @ 2.60 GHz, 6 GB RAM, Python (Table 2, Section 3.3)"}

DESC = {"batch": "4096 x 490x640 uint8, blurred noise + 8 rectangles",
        "uneven": "10000 uint8 images, H and W uniform in [48,1024], blurred noise + rectangles",
        "large": "64 x 8192x8192 uint8, blurred noise + 5% salt-and-pepper + flat patches"}


# the sources the batched kernel is built from: hardware counter figures taken
# with other sources do not describe it
BATCH_KERNEL_SOURCES = ("paper_1810_11518_amd/csrc/ldp_batch.hip",
                        "paper_1810_11518_amd/csrc/ldp_engine.hpp",
                        "paper_1810_11518_amd/csrc/ldp_device.hpp",
                        "paper_1810_11518_amd/csrc/ldp_host.hpp", "include/ldp.h")


def kernel_sources_hash(files=BATCH_KERNEL_SOURCES):
    """sha256[:16] over the batched kernel's source files."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="batch", choices=["batch", "uneven", "large"],
                    help="the timed workload (the headline is 'batch')")
    ap.add_argument("--k", type=int, default=None, help="override k of the timed workload")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-images", type=int, default=None,
                    help="images of the all-core CPU sample (single thread: a fifth of them)")
    ap.add_argument("--tune", default=None, help="JSON tune dict for the batch plan (else the "
                    "autotuner's cached choice for this batch, else defaults)")
    ap.add_argument("--autotune", type=float, default=0.0, metavar="SECONDS",
                    help="tune the batch plan on this batch for about SECONDS and cache it")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--workload-steps", type=int, default=20,
                    help="timed launches of each secondary workload (uneven, large k=2,3,4) "
                         "and of the two-call path; 0 skips them")
    ap.add_argument("--variant-steps", type=int, default=20,
                    help="timed launches of each variant path on the headline batch; 0 skips "
                         "them")
    ap.add_argument("--serve-rates", default="1000,2000,5000,10000,20000,50000",
                    help="comma-separated Poisson arrival rates (images/s) for the serving "
                         "runs; empty to skip")
    ap.add_argument("--serve-requests", type=int, default=20000,
                    help="timed requests per rate and path")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one ldp_stream_copy of this many MiB first (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    return ap.parse_args()


def algorithmic_bytes(Hs, Ws, cells):
    """Image bytes read + code bytes written + histogram bytes written."""
    H = Hs.astype(np.int64)
    W = Ws.astype(np.int64)
    return int((H * W + (H - 2) * (W - 2)).sum() + len(H) * cells[0] * cells[1] * 1024)


def hbm(nbytes, ms):
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": int(nbytes)}


def copy_rate(torch, binding, dev, mib=1024, reps=5):
    """Achievable device-memory rate: ldp_stream_copy of `mib` MiB (a kernel
    that reads and writes each byte once), best of `reps`, HIP events; GB/s
    of bytes read plus written."""
    src = torch.ones((mib << 20) // 4, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    binding.stream_copy(src, dst)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        binding.stream_copy(src, dst)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    ok = bool(torch.equal(src, dst))
    del src, dst
    return 2.0 * (mib << 20) / (best * 1e-3) / 1e9, ok


def _timed(torch, fn, steps, warmup=3, settle_s=0.0):
    """Mean ms per call of fn over `steps` calls, HIP events on the current
    stream (the stream every call here launches on)."""
    t_end = time.perf_counter() + settle_s
    while time.perf_counter() < t_end:
        fn()
        torch.cuda.synchronize()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


class Batch:
    """A workload's images generated on the host (pinned), copied to the
    device, with device code and histogram buffers and the descriptors."""

    def __init__(self, torch, binding, synth, name, n=None):
        w = synth.WORKLOADS[name]
        self.name, self.cells = name, w["cells"]
        self.Hs, self.Ws = synth.workload_sizes(name, n)
        self.off, self.strides, total = synth.layout(self.Hs, self.Ws)
        t0 = time.time()
        self.host = torch.empty(total + 64, dtype=torch.uint8, pin_memory=True)
        synth.fill(self.host.numpy(), self.off, self.Hs, self.Ws, self.strides, w["kind"],
                   synth.SEEDS[name])
        self.gen_s = time.time() - t0
        self.img = self.host.to("cuda", non_blocking=True)
        Hc = self.Hs.astype(np.int64) - 2
        Wc = self.Ws.astype(np.int64) - 2
        self.code_off = np.concatenate([[0], np.cumsum(Hc * Wc)])
        self.codes = torch.empty(int(self.code_off[-1]) + 64, dtype=torch.uint8, device="cuda")
        cy, cx = self.cells
        self.n = len(self.Hs)
        self.hist = torch.empty(self.n * cy * cx * 256, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        hb = cy * cx * 1024
        self.descs = binding.BatchPlan.descs(
            [self.img.data_ptr() + int(o) for o in self.off],
            [self.codes.data_ptr() + int(o) for o in self.code_off[:-1]],
            [self.hist.data_ptr() + j * hb for j in range(self.n)],
            [int(s) for s in self.strides], [int(h) for h in self.Hs], [int(x) for x in self.Ws])
        self.pixels = int((self.Hs.astype(np.int64) * self.Ws).sum())
        self.code_pixels = int((Hc * Wc).sum())
        self.abytes = algorithmic_bytes(self.Hs, self.Ws, self.cells)

    def image(self, j):
        hv = self.host.numpy()
        H, W, s, o = int(self.Hs[j]), int(self.Ws[j]), int(self.strides[j]), int(self.off[j])
        return hv[o:o + H * s].reshape(H, s)[:, :W]

    def outputs(self, j):
        cy, cx = self.cells
        c = self.codes[int(self.code_off[j]):int(self.code_off[j + 1])].cpu().numpy()
        h = self.hist.view(self.n, cy, cx, 256)[j].cpu().numpy().view(np.uint32).copy()
        return c, h


def traffic_for(path, key, k):
    """HBM bytes and VALU instructions per launch from the committed rocprofv3
    counters, valid only for the kernel sources they were taken with."""
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        tr = json.load(f).get(key)
    if tr and tr.get("k") == k and tr.get("kernel_sources_sha256_16") == kernel_sources_hash():
        return tr.get("bytes_per_launch"), tr.get("valu_wave_instructions_per_launch")
    return None, None


def measure_workload(torch, binding, autotune, b, k, steps, plain_steps):
    """Persistent batched launch and one launch per image on batch `b`."""
    tune = autotune.lookup(b.Hs, b.Ws, k, b.cells)
    plan = binding.BatchPlan(b.n, b.pixels, k, b.cells[0], b.cells[1], tune)
    plan.set(b.descs)
    items, grid = plan.info()
    _, _, hist_copies, _ = plan.layout()
    ms = _timed(torch, plan.run, steps, settle_s=DEVICE_WARMUP_S)
    ms_plain = _timed(torch, plan.run_per_image, plain_steps, warmup=1) if plain_steps else None
    plan.run()
    torch.cuda.synchronize()
    plan.close()
    code_pixels = b.code_pixels
    out = {"k": k, "ms": round(ms, 4), "value": round(b.pixels / (ms * 1e-3) / 1e6, 1),
           "unit": "Mpixel/s", "hbm": hbm(b.abytes, ms),
           "valu_single_issue_frac": round(VALU_PER_ROW_STEP[k] / 8.0 * code_pixels /
                                           (ms * 1e-3) / 1e12 / VALU_SINGLE_ISSUE_T, 4),
           "work_items": items, "grid_blocks": grid, "lds_histogram_copies": hist_copies,
           "tune": tune, "tune_source": "autotune cache" if tune else "default"}
    if ms_plain:
        out["plain"] = {"ms": round(ms_plain, 3),
                        "value": round(b.pixels / (ms_plain * 1e-3) / 1e6, 1),
                        "launches": "one ldp_extract per image"}
        out["batched_over_plain"] = round(ms_plain / ms, 2)
    return out


def two_call_path(torch, binding, b, k, steps):
    """The two calls the boundary names, one call per image over batch `b`:
    ldp_codes (Eqs. 1-3) and ldp_histograms (Eqs. 4-5) of its code maps."""
    cy, cx = b.cells
    imgs, code_maps, hists = [], [], []
    for j in range(b.n):
        H, W, s, o = int(b.Hs[j]), int(b.Ws[j]), int(b.strides[j]), int(b.off[j])
        imgs.append(b.img[o:o + H * s].view(H, s)[:, :W])
        code_maps.append(b.codes[int(b.code_off[j]):int(b.code_off[j + 1])].view(H - 2, W - 2))
        hists.append(b.hist.view(b.n, cy, cx, 256)[j])

    def codes_pass():
        for j in range(b.n):
            binding.codes(imgs[j], k, out=code_maps[j])

    def hist_pass():
        for j in range(b.n):
            binding.histograms(code_maps[j], cy, cx, out=hists[j])

    ms_c = _timed(torch, codes_pass, steps, warmup=2)
    ms_h = _timed(torch, hist_pass, steps, warmup=2)
    codes_pass()
    hist_pass()
    torch.cuda.synchronize()
    cbytes = b.pixels + b.code_pixels
    hbytes = b.code_pixels + b.n * cy * cx * 1024
    return {
        "what": "one call per image over the %d images of the '%s' workload, k=%d" % (b.n, b.name, k),
        "ldp_codes": {"ms": round(ms_c, 4), "value": round(b.pixels / (ms_c * 1e-3) / 1e6, 1),
                      "unit": "Mpixel/s", "hbm": hbm(cbytes, ms_c)},
        "ldp_histograms": {"ms": round(ms_h, 4),
                           "value": round(b.code_pixels / (ms_h * 1e-3) / 1e6, 1),
                           "unit": "Mpixel/s (code pixels)", "hbm": hbm(hbytes, ms_h)},
    }


def variant_bench(binding, torch, args, b, k, tune, ms_signed, sample, saved):
    """The variant paths on the headline batch.  Outputs of the sample images
    go to `saved` for the CPU leg's comparison with the oracle."""
    from paper_1810_11518_amd import autotune
    out = {}
    cy, cx = b.cells
    per = cy * cx
    n_cells = b.n * per
    nb = binding.compact_bins(k)
    # Eq. 6 compact vectors of the batch's histograms, tiled five times so
    # that the working set (1.3 GB) is far above the 256 MB last-level cache
    reps = 5
    h2 = b.hist[:n_cells * 256].view(n_cells, 256)
    big = h2.repeat(reps, 1)
    comp = torch.empty((n_cells * reps, nb), dtype=torch.int32, device=b.hist.device)
    ms = _timed(torch, lambda: binding.compact_histograms(big, k, out=comp), args.variant_steps)
    cbytes = n_cells * reps * (256 + nb) * 4
    saved["compact"] = {j: comp[j * per:(j + 1) * per].cpu().numpy().view(np.uint32).copy()
                        for j in sample}
    del big, comp
    out["compact_histograms"] = {
        "what": "Eq. 6 vectors: C(8,k) pattern-value bins + tie bin per cell, from 256-bin "
                "histograms (the batch's, tiled %dx: a working set above the last-level cache)"
                % reps, "cells": n_cells * reps, "bins": nb, "ms": round(ms, 4),
        "roofline": dict(hbm(cbytes, ms), bound="hbm")}
    plan = binding.BatchPlan(b.n, b.pixels, k, cy, cx, tune, flags=binding.LDP_RANK_MAGNITUDE)
    plan.set(b.descs)
    ms = _timed(torch, plan.run, args.variant_steps)
    plan.close()
    saved["magnitude"] = {j: b.outputs(j) for j in sample}
    lane_ops = VALU_PER_ROW_STEP_MAGNITUDE[k] / 8.0 * b.code_pixels
    out["magnitude"] = {
        "what": "the same batch ranked by |m_i| (flags LDP_RANK_MAGNITUDE)",
        "value": round(b.pixels / (ms * 1e-3) / 1e6, 1), "unit": "Mpixel/s", "ms": round(ms, 4),
        "vs_signed": round(ms / ms_signed, 3), "hbm": hbm(b.abytes, ms),
        "valu_single_issue_frac": round(lane_ops / (ms * 1e-3) / 1e12 / VALU_SINGLE_ISSUE_T, 4)}
    # windows of w x w code pixels instead of the cell grid (Section 3.2's
    # 10-100 px windows), as batch plans over the same images
    wins = []
    max_w = int(b.Ws.max())
    for w in (10, 20, 25, 50, 100):
        ny = -(-(b.Hs.astype(np.int64) - 2) // w)
        nx = -(-(b.Ws.astype(np.int64) - 2) // w)
        nbins = ny * nx * 256
        whist = torch.empty(int(nbins.sum()), dtype=torch.int32, device=b.hist.device)
        hoff = np.concatenate([[0], np.cumsum(nbins)])[:-1] * 4
        wdescs = binding.BatchPlan.descs([int(d.img) for d in b.descs],
                                         [int(d.codes) for d in b.descs],
                                         [whist.data_ptr() + int(o) for o in hoff],
                                         [int(d.stride) for d in b.descs],
                                         [int(d.H) for d in b.descs], [int(d.W) for d in b.descs])
        # the autotuner's window-plan choice for this window size, else the
        # batch's own tune
        wtune = autotune.lookup(b.Hs, b.Ws, k, (w, w), windows=True) or tune
        plan = binding.BatchPlan(b.n, b.pixels, k, w, w, wtune, windows=True, max_width=max_w)
        plan.set(wdescs)
        items, _ = plan.info()
        nt_stores = plan.layout()[3]
        ms = _timed(torch, plan.run, args.variant_steps)
        plan.close()
        wb = int((b.Hs.astype(np.int64) * b.Ws).sum() + b.code_pixels + nbins.sum() * 4)
        wins.append({"window": w, "windows_per_image": int(ny[0] * nx[0]),
                     "windows": int((ny * nx).sum()), "work_items": items, "tune": wtune,
                     "non_temporal_stores": bool(nt_stores),
                     "ms": round(ms, 4),
                     "value": round(b.pixels / (ms * 1e-3) / 1e6, 1), "unit": "Mpixel/s",
                     "hbm": hbm(wb, ms)})
        del whist
    out["windows"] = {"what": "the batch with w x w pixel windows instead of the cell grid "
                              "(batch plans with windows; rows of more than 63 windows are "
                              "split over work items)", "runs": wins}
    for name, flag, per_step, what in (
            ("direct_masks", binding.LDP_DIRECT_MASKS, VALU_PER_ROW_STEP_DIRECT[k],
             "the headline codes with every response computed as its own 8-tap mask "
             "correlation (flags LDP_DIRECT_MASKS): the unaccelerated route"),
            ("lbp", binding.LDP_CODE_LBP, VALU_PER_ROW_STEP_LBP,
             "LBP labels and histograms of the same batch (flags LDP_CODE_LBP)")):
        vtune = autotune.lookup(b.Hs, b.Ws, k, b.cells, flags=flag) or tune
        plan = binding.BatchPlan(b.n, b.pixels, k, cy, cx, vtune, flags=flag)
        plan.set(b.descs)
        ms = _timed(torch, plan.run, args.variant_steps)
        plan.close()
        saved[name] = {j: b.outputs(j) for j in sample}
        lane_ops = per_step / 8.0 * b.code_pixels
        out[name] = {
            "what": what, "value": round(b.pixels / (ms * 1e-3) / 1e6, 1), "unit": "Mpixel/s",
            "ms": round(ms, 4), "vs_signed": round(ms / ms_signed, 3), "tune": vtune,
            "hbm": hbm(b.abytes, ms),
            "valu_single_issue_frac": round(lane_ops / (ms * 1e-3) / 1e12 / VALU_SINGLE_ISSUE_T, 4)}
    return out


def host_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)),
            "cpu_model": model}


def cpu_leg(args, b, k, sample, saved, gpu_mpix, direct_over_signed):
    """The C oracle on the host, on bounded samples of the headline batch:
    single thread, and OpenMP over images on the host threads this process
    may use (at most 16).  Then the GPU outputs kept for the sample images
    (headline and variants) are compared with it."""
    from oracle import ldp as oracle_np
    from oracle import lbp as oracle_lbp
    from oracle import native
    n_all = min(args.cpu_images or 1024, b.n)
    n_one = max(1, n_all // 5)
    threads = native.default_threads()
    t0 = time.perf_counter()
    native.ldp_extract_batch(b.host.numpy(), b.off[:n_one], b.Hs[:n_one], b.Ws[:n_one],
                             b.strides[:n_one], k, *b.cells, threads=1)
    dt1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    native.ldp_extract_batch(b.host.numpy(), b.off[:n_all], b.Hs[:n_all], b.Ws[:n_all],
                             b.strides[:n_all], k, *b.cells, threads=threads)
    dtn = time.perf_counter() - t0
    px1 = int((b.Hs[:n_one].astype(np.int64) * b.Ws[:n_one]).sum())
    pxn = int((b.Hs[:n_all].astype(np.int64) * b.Ws[:n_all]).sum())
    allc = pxn / dtn / 1e6
    cpu = {"value": round(allc, 2), "unit": "Mpixel/s", "cores": threads, "kind": "oracle",
           "sample": "first %d of %d headline images, plain C oracle (direct masks, sort), "
                     "OpenMP over images on %d threads, %.1f s" % (n_all, b.n, threads, dtn),
           "single_thread": {"value": round(px1 / dt1 / 1e6, 3), "unit": "Mpixel/s",
                             "sample": "first %d images, one thread, %.1f s" % (n_one, dt1)},
           "host": host_info(),
           "gpu_over_cpu_all_cores": round(gpu_mpix / allc, 1),
           "paper": dict(PAPER_CPU, here_direct_masks_over_accelerated_gpu=direct_over_signed)}
    checks = {}
    for mode in ("signed", "magnitude", "direct_masks", "lbp"):
        if mode not in saved:
            continue
        res = []
        for j in sample:
            img = b.image(j)
            if mode == "lbp":
                wc = oracle_lbp.lbp_codes(img)
                wh = oracle_np.ldp_histograms(wc, *b.cells)
            else:
                wc, wh = native.ldp_extract(img, k, *b.cells, magnitude=(mode == "magnitude"))
            gc, gh = saved[mode][j]
            res.append(bool((gc.reshape(wc.shape) == wc).all() and (gh == wh).all()))
            if mode == "signed" and "compact" in saved:
                want = oracle_np.compact_histograms(wh, k).reshape(saved["compact"][j].shape)
                checks.setdefault("compact", []).append(bool((saved["compact"][j] == want).all()))
        checks[mode] = res
    return cpu, checks


def _drive(binding, srv, sched, imgs, outs, pool_images):
    """Open-loop driver: submit request i at scheduled host time sched[i]
    (image i % pool_images), collect completions; returns per-request
    latency (results on the host - scheduled arrival), admission delay, batch
    size, statuses, the pixels submitted, the last completion time, and the
    latency's other two parts: submission lag (submitted - scheduled) and
    service time (results on the host - admitted)."""
    n = len(sched)
    nout = len(outs)
    lat = np.zeros(n)
    adm = np.zeros(n)
    lag = np.zeros(n)
    svc = np.zeros(n)
    sizes = np.zeros(n)
    status = np.zeros(n, dtype=np.int64)
    i = done = 0
    first = None
    px = 0
    last_done = 0.0
    while done < n:
        now = binding.now()
        while i < n and sched[i] <= now:
            j = i % pool_images
            rid = srv.submit(imgs[j], outs[i % nout])
            if first is None:
                first = rid
            px += imgs[j].shape[0] * imgs[j].shape[1]
            i += 1
        for c in srv.poll(wait_us=0 if i < n else 2000):
            q = c["id"] - first
            lat[q] = c["t_done"] - sched[q]
            adm[q] = c["t_admit"] - c["t_submit"]
            lag[q] = c["t_submit"] - sched[q]
            svc[q] = c["t_done"] - c["t_admit"]
            sizes[q] = c["batch_size"]
            status[q] = c["status"]
            done += 1
            last_done = c["t_done"]
    return lat, adm, sizes, status, px, last_done, lag, svc


def serve_bench(binding, synth, torch, rates, n_req, k=3, cells=(7, 6), pool_images=256,
                warm_seconds=0.25):
    """Open-loop serving runs: Poisson arrivals of single images with sides
    log-uniform in [64, 2048] (drawn from a pool of pre-generated images),
    histogram outputs, `n_req` timed requests per rate after `warm_seconds`
    of untimed load at the same rate.  Two paths:
      in_place  page-locked images and histogram buffers that the GPU
                addresses: the kernel reads the image and writes the
                histograms over PCIe, no pool space;
      copy      pageable images and histogram buffers: every request is
                admitted into a 32 MiB pool (image + histograms) whose
                page-locked host mirror the server packs the image into and
                the kernel reads and writes in place; results are copied out
                after the batch; admission waits for pool memory under
                load."""
    _, Hs, Ws = synth.serve_stream(1000, pool_images)
    off, strides, total = synth.layout(Hs, Ws)
    keep = torch.empty(total + 64, dtype=torch.uint8, pin_memory=True)
    host_pinned = keep.numpy()
    synth.fill(host_pinned, off, Hs, Ws, strides, synth.KIND_BLUR_RECTS, synth.SEEDS["serve"])
    host_pageable = host_pinned.copy()
    nout = 2048
    hb = cells[0] * cells[1] * 256
    keep_out = torch.empty(nout * hb * 4, dtype=torch.uint8, pin_memory=True)
    paths = {
        "in_place": dict(pool=4 << 30, host=host_pinned,
                         outs=keep_out.numpy().view(np.uint32).reshape(nout, hb)),
        "copy": dict(pool=32 << 20, host=host_pageable,
                     outs=np.zeros((nout, hb), dtype=np.uint32)),
    }
    results = {}
    for pname, pc in paths.items():
        imgs = [pc["host"][int(o):int(o) + int(h) * int(st)].reshape(int(h), int(st))[:, :int(w)]
                for o, h, w, st in zip(off, Hs, Ws, strides)]
        runs = []
        for rate in rates:
            arr, _, _ = synth.serve_stream(rate, n_req)
            srv = binding.Server(pc["pool"], max_inflight=1024, max_batch=256, depth=4, k=k,
                                 cells_y=cells[0], cells_x=cells[1])
            nw = max(1, int(rate * warm_seconds))
            _drive(binding, srv, binding.now() + 0.01 + arr[:nw], imgs, pc["outs"], pool_images)
            st0 = srv.stats()
            t0 = binding.now() + 0.02
            lat, adm, sizes, status, px, last_done, lag, svc = _drive(
                binding, srv, t0 + arr, imgs, pc["outs"], pool_images)
            st = srv.stats()
            srv.close()
            span = last_done - t0
            runs.append({"rate_img_s": rate, "requests": n_req,
                         "throughput_img_s": round(n_req / span, 1),
                         "throughput_mpix_s": round(px / span / 1e6, 1),
                         "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                         "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                         "admission_p99_ms": round(float(np.percentile(adm, 99)) * 1e3, 3),
                         # the p50 latency's parts: the driver's submission lag,
                         # admission, and launch + kernel + completion
                         "submit_lag_p50_ms": round(float(np.percentile(lag, 50)) * 1e3, 3),
                         "admission_p50_ms": round(float(np.percentile(adm, 50)) * 1e3, 3),
                         "service_p50_ms": round(float(np.percentile(svc, 50)) * 1e3, 3),
                         "memory_waits": int(st["memory_waits"] - st0["memory_waits"]),
                         "peak_pool_bytes": int(st["peak_pool_bytes"]),
                         "pool_bytes": int(pc["pool"]),
                         "errors": int((status != 0).sum()),
                         "mean_batch": round(float(sizes.mean()), 2),
                         "peak_batches_in_flight": st["peak_batches"],
                         "launches": int(st["launches"] - st0["launches"])})
        results[pname] = runs
    return results


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(images would shard across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1810_11518_amd import autotune, binding, synth

    binding.load()
    dev = torch.device("cuda:0")
    if args.calib_copy_mib:
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        binding.stream_copy(src, dst)
        torch.cuda.synchronize()
        del src, dst
    b = Batch(torch, binding, synth, args.workload)
    w = synth.WORKLOADS[args.workload]
    k = args.k if args.k is not None else (w["k"] if isinstance(w["k"], int) else 3)
    cells = b.cells
    n = b.n

    tune_src = "default"
    if args.tune:
        tune, tune_src = json.loads(args.tune), "command line"
    elif args.autotune > 0:
        tune, tms = autotune.tune_batch(b.descs, b.Hs, b.Ws, k, cells, budget_s=args.autotune)
        autotune.save(b.Hs, b.Ws, k, cells, tune, tms, note="bench.py --workload %s" % args.workload)
        tune_src = "autotuned now"
    else:
        tune = autotune.lookup(b.Hs, b.Ws, k, cells)
        tune_src = "autotune cache" if tune else "default"
    plan = binding.BatchPlan(n, b.pixels, k, cells[0], cells[1], tune)
    plan.set(b.descs)
    items, grid = plan.info()
    _, lds_bytes, hist_copies, _ = plan.layout()
    stream = torch.cuda.current_stream()

    # ---- batched persistent launch (graph replays on torch's current stream)
    t_end = time.perf_counter() + DEVICE_WARMUP_S
    while time.perf_counter() < t_end:
        plan.run()
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.run()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_event = ev0.elapsed_time(ev1) / args.steps
    ms_step = max(ms_event, wall * 1000.0 / args.steps)

    # ---- plain: one launch per image
    ms_plain = None
    if args.plain_steps > 0:
        ms_plain = _timed(torch, plan.run_per_image, args.plain_steps, warmup=1)
    plan.run()
    torch.cuda.synchronize()

    # outputs of a few images, kept for the CPU leg's comparison with the oracle
    sample = [0, n // 2, n - 1]
    saved = {"signed": {j: b.outputs(j) for j in sample}}

    copy_gbs, copy_ok = copy_rate(torch, binding, dev)

    # ---- serving, on a device that so far holds only the headline batch
    serve = None
    if args.serve_rates and args.serve_rates.strip():
        rates = [int(x) for x in args.serve_rates.split(",") if x]
        serve = {"workload": "Poisson arrivals, single uint8 images, sides log-uniform in "
                             "[64,2048], k=3, 7x6 cells, histogram outputs; latency from "
                             "scheduled arrival to results on the host, after 0.25 s of "
                             "untimed load at the same rate; admission delay = admitted - "
                             "submitted; in_place: page-locked buffers the kernel reads and "
                             "writes; copy: pageable buffers through the page-locked mirror "
                             "of a 32 MiB pool",
                 "paths": serve_bench(binding, synth, torch, rates, args.serve_requests)}

    # ---- variants on the same batch (they overwrite the outputs)
    variants = None
    if args.variant_steps > 0:
        variants = variant_bench(binding, torch, args, b, k, tune, ms_event, sample, saved)

    cpu, checks = None, {}
    if not args.no_cpu:
        direct = (variants or {}).get("direct_masks", {}).get("vs_signed")
        cpu, checks = cpu_leg(args, b, k, sample, saved, b.pixels / (ms_step * 1e-3) / 1e6,
                              direct)
    if variants:
        for name, key in (("compact_histograms", "compact"), ("magnitude", "magnitude"),
                          ("direct_masks", "direct_masks"), ("lbp", "lbp")):
            variants[name]["checked_images_bit_exact"] = checks.get(key)

    # ---- the other workloads and the two-call path (headline batch freed)
    workloads, two_call = None, None
    if args.workload_steps > 0 and args.workload == "batch":
        plan.close()
        workloads = {}
        u = Batch(torch, binding, synth, "uneven")
        workloads["uneven"] = dict(measure_workload(torch, binding, autotune, u, 3,
                                                    args.workload_steps, args.plain_steps),
                                   workload=DESC["uneven"], gen_seconds=round(u.gen_s, 1))
        del u
        lg = Batch(torch, binding, synth, "large")
        workloads["large"] = {"workload": DESC["large"] + ", 16x16 cells",
                              "gen_seconds": round(lg.gen_s, 1)}
        for kk in (2, 3, 4):
            workloads["large"]["k%d" % kk] = measure_workload(torch, binding, autotune, lg, kk,
                                                              args.workload_steps, 1)
        two_call = two_call_path(torch, binding, lg, 3, max(1, args.workload_steps // 4))
        del lg

    mpix = b.pixels / (ms_step * 1e-3) / 1e6
    mpix_plain = b.pixels / (ms_plain * 1e-3) / 1e6 if ms_plain else None
    traffic, valu = traffic_for(args.traffic, args.workload if args.workload != "large"
                                else "large_k%d" % k, k)
    lane_ops = VALU_PER_ROW_STEP[k] / 8.0 * b.code_pixels  # lane instructions per launch
    valu_t = lane_ops / (ms_event * 1e-3) / 1e12
    issued_t = valu * 64 / (ms_event * 1e-3) / 1e12 if valu else None
    roof = hbm(b.abytes, ms_event)
    out = {
        "metric": METRIC,
        "value": round(mpix, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": "%s: %s, k=%d, %dx%d cells" % (args.workload, DESC[args.workload],
                                                              k, cells[0], cells[1]),
                   "images": n, "pixels": b.pixels, "k": k, "cells": list(cells),
                   "work_items": items, "grid_blocks": grid, "tune": tune, "tune_source": tune_src,
                   "device_warmup_s": DEVICE_WARMUP_S},
        "roofline": {"bound": "hbm", "achieved": roof["achieved"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": roof["frac"], "traffic": traffic,
                     "kernel": "batch_kernel<%d, 0, %d>" % (k, hist_copies),
                     "kernel_ms": round(ms_event, 4),
                     "lds_bytes_per_workgroup": lds_bytes, "lds_histogram_copies": hist_copies,
                     "algorithmic_bytes_per_launch": b.abytes,
                     "copy": {"achieved": round(copy_gbs, 1), "unit": "GB/s",
                              "frac_of_peak": round(copy_gbs / HBM_PEAK_GBS, 4),
                              "checked": copy_ok,
                              "kernel": "ldp_stream_copy, 1 GiB, best of 5, read + write bytes"},
                     "frac_of_copy": round(roof["achieved"] / copy_gbs, 4),
                     "valu": {"per_pixel": round(VALU_PER_ROW_STEP[k] / 8.0, 2),
                              "achieved": round(valu_t, 2), "unit": "T lane-instr/s",
                              "single_issue_rate": round(VALU_SINGLE_ISSUE_T, 2),
                              "single_issue_frac": round(valu_t / VALU_SINGLE_ISSUE_T, 4),
                              "issued": round(issued_t, 2) if issued_t else None,
                              "note": "main-loop VALU instructions of the compiled kernel per "
                                      "code pixel; the rate is one wave64 instruction per "
                                      "SIMD per quad-cycle, which dual issue of simple 32-bit "
                                      "ops can exceed"}},
        "plain": None if not ms_plain else {
            "value": round(mpix_plain, 1), "unit": "Mpixel/s", "ms_per_step": round(ms_plain, 3),
            "hbm_frac": round(b.abytes / (ms_plain * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "launches": "one ldp_extract per image"},
        "batched_over_plain": round(ms_plain / ms_step, 2) if ms_plain else None,
        "workloads": workloads,
        "two_call_path": two_call,
        "variants": variants,
        "cpu_baseline": cpu,
        "checked_images_bit_exact": checks.get("signed"),
        "serve": serve,
        "gen_seconds": round(b.gen_s, 1),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
