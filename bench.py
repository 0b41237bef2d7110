"""Benchmark of the LDP hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batch]

One step = one pass of the whole path (codes of every interior pixel, top-k
selection, the 8-bit code, per-cell histograms) over one batch of synthetic
images already resident in device memory.  The headline is the persistent,
graph-captured batched launch; the same batch run as one launch per image
("plain") is timed beside it.  Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LDP Mpixel/s + % HBM roofline (batched vs plain kernel); p50/p99 serve latency"
HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one wave64 VALU
# instruction per SIMD every 4 cycles), in tera lane-instructions per second
VALU_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic VALU work of the batched kernel: wave instructions per 8-pixel
# row step of a lane (one wave covers 512 code pixels) in the main row loop of
# batch_kernel<k> as compiled for gfx950 (the x3-unrolled loop / 3; both
# histogram paths counted; the loop with the fewest instructions, which waves
# whose rows start 4-aligned run).  tests/test_isa_counts.py recompiles the
# kernel and checks these figures against the generated code.
VALU_PER_ROW_STEP = {1: 413 / 3, 2: 569 / 3, 3: 605 / 3, 4: 665 / 3, 5: 665 / 3, 6: 605 / 3,
                     7: 569 / 3, 8: 45 / 3}
# the same for ranking by response magnitude (flags LDP_RANK_MAGNITUDE), for
# responses computed mask by mask (LDP_DIRECT_MASKS) and for LBP labels
# (LDP_CODE_LBP, one kernel for every k)
VALU_PER_ROW_STEP_MAGNITUDE = {1: 767 / 3, 2: 923 / 3, 3: 959 / 3, 4: 1019 / 3, 5: 1019 / 3,
                               6: 959 / 3, 7: 923 / 3, 8: 45 / 3}
VALU_PER_ROW_STEP_DIRECT = {1: 1043 / 3, 2: 1199 / 3, 3: 1235 / 3, 4: 1295 / 3, 5: 1295 / 3,
                            6: 1235 / 3, 7: 1199 / 3, 8: 45 / 3}
VALU_PER_ROW_STEP_LBP = 287 / 3
# untimed work before the warm-up steps, so that timing starts at steady clocks
DEVICE_WARMUP_S = 0.3


def kernel_sources_hash():
    import glob
    import hashlib
    src = sorted(glob.glob(os.path.join(ROOT, "paper_1810_11518_amd", "csrc", "*.hip")) +
                 glob.glob(os.path.join(ROOT, "paper_1810_11518_amd", "csrc", "*.hpp")))
    h = hashlib.sha256()
    for f in src:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="batch", choices=["batch", "uneven", "large"])
    ap.add_argument("--k", type=int, default=None, help="override k (large workload: 2, 3 or 4)")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-images", type=int, default=None)
    ap.add_argument("--tune", default=None, help="JSON tune dict for the batch plan (else the "
                    "autotuner's cached choice for this batch, else defaults)")
    ap.add_argument("--autotune", type=float, default=0.0, metavar="SECONDS",
                    help="tune the batch plan on this batch for about SECONDS and cache it")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--variant-steps", type=int, default=20,
                    help="timed launches of each variant path (magnitude ranking, Eq. 6 compact "
                         "histograms) on the same batch; 0 skips them")
    ap.add_argument("--serve-rates", default="1000,2000,10000,50000",
                    help="comma-separated Poisson arrival rates (images/s) for the serving "
                         "run; empty to skip")
    ap.add_argument("--serve-seconds", type=float, default=1.5)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    return ap.parse_args()


def make_workload(name, synth):
    w = synth.WORKLOADS[name]
    Hs, Ws = synth.workload_sizes(name)
    off, strides, total = synth.layout(Hs, Ws)
    return w, Hs, Ws, off, strides, total


def algorithmic_bytes(Hs, Ws, cells):
    H = Hs.astype(np.int64)
    W = Ws.astype(np.int64)
    return int((H * W + (H - 2) * (W - 2)).sum() + len(H) * cells[0] * cells[1] * 1024)


def copy_rate(torch, dev, mib=1024, reps=5):
    """Achievable HBM rate on this device: a plain device-to-device copy of
    `mib` MiB (torch's copy kernel), best of `reps`, HIP events; GB/s of
    bytes read plus written."""
    src = torch.ones((mib << 20) // 4, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    return 2.0 * (mib << 20) / (best * 1e-3) / 1e9


def _timed(torch, fn, steps, warmup=3):
    """Mean ms per call of fn over `steps` calls, HIP events on the current stream."""
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


def variant_bench(binding, torch, args, plan_args, descs, hist, codes, code_off, Hs, Ws,
                  ms_signed, sample, saved):
    """The variant paths on the headline batch: Eq. 6 compact vectors of its
    histograms (HBM-bound) and the whole batch ranked by response magnitude
    (VALU-bound).  Outputs of the sample images go to `saved` for the CPU
    leg's comparison with the oracle."""
    n, pixels, k, cells, tune = plan_args
    out = {}
    per = cells[0] * cells[1]
    n_cells = n * per
    nb = binding.compact_bins(k)
    h2 = hist[:n_cells * 256].view(n_cells, 256)
    comp = torch.empty((n_cells, nb), dtype=torch.int32, device=hist.device)
    ms = _timed(torch, lambda: binding.compact_histograms(h2, k, out=comp), args.variant_steps)
    cbytes = n_cells * (256 + nb) * 4
    saved["compact"] = {j: comp[j * per:(j + 1) * per].cpu().numpy().view(np.uint32).copy()
                        for j in sample}
    out["compact_histograms"] = {
        "what": "Eq. 6 vectors: C(8,k) pattern-value bins + tie bin per cell, from the batch's "
                "256-bin histograms", "cells": n_cells, "bins": nb, "ms": round(ms, 4),
        "roofline": {"bound": "hbm", "achieved": round(cbytes / (ms * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(cbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "algorithmic_bytes": cbytes}}
    plan = binding.BatchPlan(n, pixels, k, cells[0], cells[1], tune,
                             flags=binding.LDP_RANK_MAGNITUDE)
    plan.set(descs)
    ms = _timed(torch, plan.run, args.variant_steps)
    plan.close()
    code_pixels = int(((Hs.astype(np.int64) - 2) * (Ws.astype(np.int64) - 2)).sum())
    lane_ops = VALU_PER_ROW_STEP_MAGNITUDE[k] / 8.0 * code_pixels
    hist_h = hist.view(n, cells[0], cells[1], 256)
    saved["magnitude"] = {j: (codes[int(code_off[j]):int(code_off[j + 1])].cpu().numpy(),
                              hist_h[j].cpu().numpy().view(np.uint32).copy()) for j in sample}
    out["magnitude"] = {
        "what": "the same batch ranked by |m_i| (flags LDP_RANK_MAGNITUDE)",
        "value": round(pixels / (ms * 1e-3) / 1e6, 1), "unit": "Mpixel/s", "ms": round(ms, 4),
        "vs_signed": round(ms / ms_signed, 3),
        "roofline": {"bound": "alu", "unit": "T VALU lane-instr/s",
                     "achieved": round(lane_ops / (ms * 1e-3) / 1e12, 2),
                     "peak": round(VALU_PEAK_T, 2),
                     "frac": round(lane_ops / (ms * 1e-3) / 1e12 / VALU_PEAK_T, 4),
                     "per_pixel": round(VALU_PER_ROW_STEP_MAGNITUDE[k] / 8.0, 2)}}
    # windows of w x w code pixels instead of the cell grid (Section 3.2), as
    # batch plans over the same images; the histograms grow as windows shrink
    wins = []
    max_w = int(Ws.max())
    for w in (20, 25, 50, 100):
        if -(-(max_w - 2) // w) > 63:
            continue
        ny = -(-(Hs.astype(np.int64) - 2) // w)
        nx = -(-(Ws.astype(np.int64) - 2) // w)
        nbins = ny * nx * 256
        whist = torch.empty(int(nbins.sum()), dtype=torch.int32, device=hist.device)
        hoff = np.concatenate([[0], np.cumsum(nbins)])[:-1] * 4
        wdescs = binding.BatchPlan.descs([int(d.img) for d in descs], [int(d.codes) for d in descs],
                                         [whist.data_ptr() + int(o) for o in hoff],
                                         [int(d.stride) for d in descs], [int(d.H) for d in descs],
                                         [int(d.W) for d in descs])
        plan = binding.BatchPlan(n, pixels, k, w, w, tune, windows=True, max_width=max_w)
        plan.set(wdescs)
        ms = _timed(torch, plan.run, args.variant_steps)
        plan.close()
        wb = int((Hs.astype(np.int64) * Ws).sum() + code_pixels + nbins.sum() * 4)
        wins.append({"window": w, "windows": int((ny * nx).sum()), "ms": round(ms, 4),
                     "value": round(pixels / (ms * 1e-3) / 1e6, 1), "unit": "Mpixel/s",
                     "hbm": {"achieved": round(wb / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(wb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                             "algorithmic_bytes": wb}})
        del whist
    out["windows"] = {"what": "the batch with w x w pixel windows instead of the cell grid "
                              "(batch plans with windows)", "runs": wins}
    abytes = algorithmic_bytes(Hs, Ws, cells)
    for name, flag, per_step, what in (
            ("direct_masks", binding.LDP_DIRECT_MASKS, VALU_PER_ROW_STEP_DIRECT[k],
             "the headline codes with every response computed as its own 8-tap mask "
             "correlation (flags LDP_DIRECT_MASKS): the unaccelerated route"),
            ("lbp", binding.LDP_CODE_LBP, VALU_PER_ROW_STEP_LBP,
             "LBP labels and histograms of the same batch (flags LDP_CODE_LBP)")):
        from paper_1810_11518_amd import autotune
        vtune = autotune.lookup(Hs, Ws, k, cells, flags=flag) or tune
        plan = binding.BatchPlan(n, pixels, k, cells[0], cells[1], vtune, flags=flag)
        plan.set(descs)
        ms = _timed(torch, plan.run, args.variant_steps)
        plan.close()
        saved[name] = {j: (codes[int(code_off[j]):int(code_off[j + 1])].cpu().numpy(),
                           hist_h[j].cpu().numpy().view(np.uint32).copy()) for j in sample}
        lane_ops = per_step / 8.0 * code_pixels
        out[name] = {
            "what": what, "value": round(pixels / (ms * 1e-3) / 1e6, 1), "unit": "Mpixel/s",
            "ms": round(ms, 4), "vs_signed": round(ms / ms_signed, 3), "tune": vtune,
            "roofline": {"bound": "alu", "unit": "T VALU lane-instr/s",
                         "achieved": round(lane_ops / (ms * 1e-3) / 1e12, 2),
                         "peak": round(VALU_PEAK_T, 2),
                         "frac": round(lane_ops / (ms * 1e-3) / 1e12 / VALU_PEAK_T, 4),
                         "per_pixel": round(per_step / 8.0, 2),
                         "hbm": {"achieved": round(abytes / (ms * 1e-3) / 1e9, 1),
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": round(abytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}}
    return out


def cpu_leg(args, host, Hs, Ws, strides, off, k, cells, n, sample, saved):
    """The oracle on the host: timed on a bounded sample of the batch (the
    cpu_baseline figure), then compared with the GPU outputs kept for the
    sample images (headline, and the variants when they ran)."""
    from oracle import ldp as oracle_np
    from oracle import native
    hv = host.numpy()

    def image(j):
        H, W, s, o = int(Hs[j]), int(Ws[j]), int(strides[j]), int(off[j])
        return hv[o:o + H * s].reshape(H, s)[:, :W]

    # about 10 s of single-thread oracle work
    ncpu = min(args.cpu_images or {"batch": 800, "uneven": 800, "large": 4}[args.workload], n)
    t0 = time.perf_counter()
    px = 0
    for j in range(ncpu):
        native.ldp_extract(image(j), k, cells[0], cells[1])
        px += int(Hs[j]) * int(Ws[j])
    dt = time.perf_counter() - t0
    cpu = {"value": round(px / dt / 1e6, 3), "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
           "sample": "first %d of %d images, plain C oracle (direct masks, sort), "
                     "single thread, %.1f s" % (ncpu, n, dt)}
    from oracle import lbp as oracle_lbp
    checks = {}
    for mode in ("signed", "magnitude", "direct_masks", "lbp"):
        if mode not in saved:
            continue
        res = []
        for j in sample:
            if mode == "lbp":
                wc = oracle_lbp.lbp_codes(image(j))
                wh = oracle_np.ldp_histograms(wc, cells[0], cells[1])
            else:
                wc, wh = native.ldp_extract(image(j), k, cells[0], cells[1],
                                            magnitude=(mode == "magnitude"))
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
    latency (results on the host - scheduled arrival), batch size, the pixels
    submitted and the last completion time."""
    n = len(sched)
    nout = len(outs)
    lat = np.zeros(n)
    sizes = np.zeros(n)
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
            lat[c["id"] - first] = c["t_done"] - sched[c["id"] - first]
            sizes[c["id"] - first] = c["batch_size"]
            done += 1
            last_done = c["t_done"]
    return lat, sizes, px, last_done


def serve_bench(binding, synth, rates, seconds, k=3, cells=(7, 6), pool_images=256,
                warm_seconds=0.25):
    """Open-loop serving run per rate: Poisson arrivals of single images with
    sides log-uniform in [64, 2048] (drawn from a pool of pre-generated images),
    histogram outputs; latency = results on the host - scheduled arrival.
    Each rate first runs `warm_seconds` of the same arrival process untimed
    (steady state: every launch slot and pool region in use)."""
    import torch
    _, Hs, Ws = synth.serve_stream(1000, pool_images)
    off, strides, total = synth.layout(Hs, Ws)
    keep = torch.empty(total + 64, dtype=torch.uint8, pin_memory=True)
    host = keep.numpy()
    synth.fill(host, off, Hs, Ws, strides, synth.KIND_BLUR_RECTS, synth.SEEDS["serve"])
    imgs = [host[int(o):int(o) + int(h) * int(st)].reshape(int(h), int(st))[:, :int(w)]
            for o, h, w, st in zip(off, Hs, Ws, strides)]
    nout = 2048
    hb = cells[0] * cells[1] * 256
    keep_out = torch.empty(nout * hb * 4, dtype=torch.uint8, pin_memory=True)
    outs = keep_out.numpy().view(np.uint32).reshape(nout, hb)
    results = []
    for rate in rates:
        n = max(1, int(rate * seconds))
        arr, _, _ = synth.serve_stream(rate, n)
        srv = binding.Server(4 << 30, max_inflight=1024, max_batch=256, depth=4, k=k,
                             cells_y=cells[0], cells_x=cells[1])
        # untimed steady-state warm-up at the same rate (the head of the
        # timed stream's own arrival gaps)
        nw = max(1, int(rate * warm_seconds))
        _drive(binding, srv, binding.now() + 0.01 + arr[:nw], imgs, outs, pool_images)
        t0 = binding.now() + 0.02
        lat, sizes, px, last_done = _drive(binding, srv, t0 + arr, imgs, outs, pool_images)
        st = srv.stats()
        srv.close()
        span = last_done - t0
        results.append({"rate_img_s": rate, "requests": n,
                        "throughput_img_s": round(n / span, 1),
                        "throughput_mpix_s": round(px / span / 1e6, 1),
                        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                        "mean_batch": round(float(sizes.mean()), 1),
                        "peak_batches_in_flight": st["peak_batches"],
                        "launches_incl_warmup": st["launches"]})
    return results


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(images would shard across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1810_11518_amd import binding, synth

    binding.load()
    dev = torch.device("cuda:0")
    if args.calib_copy_mib:
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w, Hs, Ws, off, strides, total = make_workload(args.workload, synth)
    k = args.k if args.k is not None else (w["k"] if isinstance(w["k"], int) else 3)
    cells = w["cells"]
    n = len(Hs)
    t0 = time.time()
    host = torch.empty(total + 64, dtype=torch.uint8, pin_memory=True)
    synth.fill(host.numpy(), off, Hs, Ws, strides, w["kind"], synth.SEEDS[args.workload])
    gen_s = time.time() - t0
    img = host.to(dev, non_blocking=True)
    Hc = Hs.astype(np.int64) - 2
    Wc = Ws.astype(np.int64) - 2
    code_off = np.concatenate([[0], np.cumsum(Hc * Wc)])
    codes = torch.empty(int(code_off[-1]) + 64, dtype=torch.uint8, device=dev)
    hist = torch.empty(n * cells[0] * cells[1] * 256, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    base_i, base_c, base_h = img.data_ptr(), codes.data_ptr(), hist.data_ptr()
    hb = cells[0] * cells[1] * 256 * 4
    descs = binding.BatchPlan.descs([base_i + int(o) for o in off],
                                    [base_c + int(o) for o in code_off[:-1]],
                                    [base_h + j * hb for j in range(n)],
                                    [int(s) for s in strides], [int(h) for h in Hs],
                                    [int(x) for x in Ws])
    from paper_1810_11518_amd import autotune
    tune_src = "default"
    if args.tune:
        tune, tune_src = json.loads(args.tune), "command line"
    elif args.autotune > 0:
        tune, tms = autotune.tune_batch(descs, Hs, Ws, k, cells, budget_s=args.autotune)
        autotune.save(Hs, Ws, k, cells, tune, tms, note="bench.py --workload %s" % args.workload)
        tune_src = "autotuned now"
    else:
        tune = autotune.lookup(Hs, Ws, k, cells)
        tune_src = "autotune cache" if tune else "default"
    pixels = int((Hs.astype(np.int64) * Ws).sum())
    plan = binding.BatchPlan(n, pixels, k, cells[0], cells[1], tune)
    plan.set(descs)
    items, grid = plan.info()
    stream = torch.cuda.current_stream()

    # ---- batched persistent launch
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
        plan.run_per_image()
        torch.cuda.synchronize()
        ep0, ep1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ep0.record(stream)
        for _ in range(args.plain_steps):
            plan.run_per_image()
        ep1.record(stream)
        torch.cuda.synchronize()
        ms_plain = ep0.elapsed_time(ep1) / args.plain_steps

    # outputs of a few images, kept for the CPU leg's comparison with the oracle
    # (the timed runs all give the same results as one run)
    sample = [0, n // 2, n - 1]
    hist_h = hist.view(n, cells[0], cells[1], 256)
    saved = {"signed": {j: (codes[int(code_off[j]):int(code_off[j + 1])].cpu().numpy(),
                            hist_h[j].cpu().numpy().view(np.uint32).copy()) for j in sample}}

    # ---- serving, on a device that so far holds only the headline batch
    serve = None
    if args.serve_rates and args.serve_rates.strip():
        rates = [int(x) for x in args.serve_rates.split(",") if x]
        serve = {"workload": "Poisson arrivals, single uint8 images, sides log-uniform in "
                             "[64,2048], k=3, 7x6 cells, histogram outputs; latency from "
                             "scheduled arrival to results on the host, after 0.25 s of "
                             "untimed load at the same rate",
                 "runs": serve_bench(binding, synth, rates, args.serve_seconds)}

    # ---- variants on the same batch (they overwrite the outputs)
    variants = None
    if args.variant_steps > 0:
        variants = variant_bench(binding, torch, args, plan_args=(n, pixels, k, cells, tune),
                                 descs=descs, hist=hist, codes=codes, code_off=code_off,
                                 Hs=Hs, Ws=Ws, ms_signed=ms_event, sample=sample, saved=saved)

    abytes = algorithmic_bytes(Hs, Ws, cells)
    achieved = abytes / (ms_event * 1e-3) / 1e9
    copy_gbs = copy_rate(torch, dev)
    mpix = pixels / (ms_step * 1e-3) / 1e6
    mpix_plain = pixels / (ms_plain * 1e-3) / 1e6 if ms_plain else None

    # HBM bytes and VALU instructions per launch from the committed rocprofv3
    # counters, valid only for the kernel sources they were taken with
    traffic = valu = None
    if os.path.exists(args.traffic):
        with open(args.traffic) as f:
            tr = json.load(f).get(args.workload)
        if tr and tr.get("k") == k and tr.get("kernel_sources_sha256_16") == kernel_sources_hash():
            traffic = tr.get("bytes_per_launch")
            valu = tr.get("valu_wave_instructions_per_launch")
    code_pixels = int(((Hs.astype(np.int64) - 2) * (Ws.astype(np.int64) - 2)).sum())
    alu_lane_ops = VALU_PER_ROW_STEP[k] / 8.0 * code_pixels  # lane instructions per launch
    alu_achieved = alu_lane_ops / (ms_event * 1e-3) / 1e12
    alu_issued = valu * 64 / (ms_event * 1e-3) / 1e12 if valu else None

    cpu, checks = None, {}
    if not args.no_cpu:
        cpu, checks = cpu_leg(args, host, Hs, Ws, strides, off, k, cells, n, sample, saved)
    if variants:
        for name, key in (("compact_histograms", "compact"), ("magnitude", "magnitude"),
                          ("direct_masks", "direct_masks"), ("lbp", "lbp")):
            variants[name]["checked_images_bit_exact"] = checks.get(key)


    desc = {"batch": "4096 x 490x640 uint8, blurred noise + 8 rectangles",
            "uneven": "10000 uint8 images, H and W uniform in [48,1024], blurred noise + rectangles",
            "large": "64 x 8192x8192 uint8, blurred noise + 5% salt-and-pepper + flat patches"}
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
        "config": {"workload": "%s: %s, k=%d, %dx%d cells" % (args.workload, desc[args.workload], k,
                                                              cells[0], cells[1]),
                   "images": n, "pixels": pixels, "k": k, "cells": list(cells),
                   "work_items": items, "grid_blocks": grid, "tune": tune, "tune_source": tune_src,
                   "device_warmup_s": DEVICE_WARMUP_S},
        "roofline": {"bound": "alu", "unit": "T VALU lane-instr/s",
                     "achieved": round(alu_achieved, 2),
                     "peak": round(VALU_PEAK_T, 2),
                     "frac": round(alu_achieved / VALU_PEAK_T, 4),
                     "per_pixel": round(VALU_PER_ROW_STEP[k] / 8.0, 2),
                     "issued": round(alu_issued, 2) if alu_issued else None,
                     "traffic": traffic,
                     "hbm": {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(achieved / HBM_PEAK_GBS, 4),
                             "algorithmic_bytes_per_launch": abytes,
                             "copy_achieved": round(copy_gbs, 1),
                             "frac_of_copy": round(achieved / copy_gbs, 4),
                             "copy": "1 GiB device-to-device copy, best of 5, read + write bytes"},
                     "kernel": "batch_kernel<%d>" % k},
        "plain": None if not ms_plain else {
            "value": round(mpix_plain, 1), "unit": "Mpixel/s", "ms_per_step": round(ms_plain, 3),
            "frac": round(abytes / (ms_plain * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "launches": "one ldp_extract per image"},
        "batched_over_plain": round(ms_plain / ms_step, 2) if ms_plain else None,
        "variants": variants,
        "cpu_baseline": cpu,
        "checked_images_bit_exact": checks.get("signed"),
        "serve": serve,
        "gen_seconds": round(gen_s, 1),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
