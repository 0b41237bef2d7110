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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch", choices=["batch", "uneven", "large"])
    ap.add_argument("--k", type=int, default=None, help="override k (large workload: 2, 3 or 4)")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-images", type=int, default=None)
    ap.add_argument("--tune", default=None, help="JSON tune dict for the batch plan")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"))
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
    tune = json.loads(args.tune) if args.tune else None
    pixels = int((Hs.astype(np.int64) * Ws).sum())
    plan = binding.BatchPlan(n, pixels, k, cells[0], cells[1], tune)
    plan.set(descs)
    items, grid = plan.info()
    stream = torch.cuda.current_stream()

    # ---- batched persistent launch
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

    # results of the timed runs are the same as one run: check a few images
    check = []
    if not args.no_cpu:
        from oracle import native
        hist_h = hist.view(n, cells[0], cells[1], 256)
        for j in [0, n // 2, n - 1]:
            H, W, s, o = int(Hs[j]), int(Ws[j]), int(strides[j]), int(off[j])
            im = host.numpy()[o:o + H * s].reshape(H, s)[:, :W]
            wc, wh = native.ldp_extract(im, k, cells[0], cells[1])
            gc = codes[int(code_off[j]):int(code_off[j + 1])].cpu().numpy().reshape(wc.shape)
            gh = hist_h[j].cpu().numpy().view(np.uint32)
            check.append(bool((gc == wc).all() and (gh == wh).all()))

    abytes = algorithmic_bytes(Hs, Ws, cells)
    achieved = abytes / (ms_event * 1e-3) / 1e9
    mpix = pixels / (ms_step * 1e-3) / 1e6
    mpix_plain = pixels / (ms_plain * 1e-3) / 1e6 if ms_plain else None

    traffic = None
    if os.path.exists(args.traffic):
        with open(args.traffic) as f:
            tr = json.load(f).get(args.workload)
        if tr and tr.get("k") == k:
            traffic = tr.get("bytes_per_launch")

    cpu = None
    if not args.no_cpu:
        from oracle import native
        ncpu = args.cpu_images or {"batch": 320, "uneven": 320, "large": 2}[args.workload]
        ncpu = min(ncpu, n)
        hv = host.numpy()
        t0 = time.perf_counter()
        px = 0
        for j in range(ncpu):
            H, W, s, o = int(Hs[j]), int(Ws[j]), int(strides[j]), int(off[j])
            native.ldp_extract(hv[o:o + H * s].reshape(H, s)[:, :W], k, cells[0], cells[1])
            px += H * W
        dt = time.perf_counter() - t0
        cpu = {"value": round(px / dt / 1e6, 3), "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
               "sample": "first %d of %d images, plain C oracle (direct masks, sort), "
                         "single thread, %.1f s" % (ncpu, n, dt)}

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
                   "work_items": items, "grid_blocks": grid},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "algorithmic_bytes_per_launch": abytes},
        "plain": None if not ms_plain else {
            "value": round(mpix_plain, 1), "unit": "Mpixel/s", "ms_per_step": round(ms_plain, 3),
            "frac": round(abytes / (ms_plain * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "launches": "one ldp_extract per image"},
        "batched_over_plain": round(ms_plain / ms_step, 2) if ms_plain else None,
        "cpu_baseline": cpu,
        "checked_images_bit_exact": check,
        "gen_seconds": round(gen_s, 1),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
