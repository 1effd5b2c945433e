"""Benchmark of the Sauvola hot path on one MI355X.

Default workload: Sauvola on a 4096 x 3072 (W x H) uint8 synthetic document,
h = w = 75, k = 0.5, R = 128, writing the uint8 mask plus float32 window mean
and standard deviation (10 bytes of algorithmic HBM traffic per pixel).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu] [--pmc]

Prints ONE JSON line.  `value` is Gpix/s over the K timed steps (inputs
resident in HBM; buffer sets rotated so the 256 MB Infinity Cache cannot serve
repeats).  `roofline` prices the kernel's average duration (the timed
region's time per launch, HIP events on the stream the kernel runs on) against
the 8 TB/s HBM peak; `traffic` is the counter-derived HBM bytes per launch from
the committed profile summary, or null when that was taken on other kernel
source.
`cpu_baseline` times the CPU oracle (Algorithm 1 sweep plus the binary64
threshold, one thread) on the same page.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "Gpix/s Sauvola 4096×3072 w=75 (% HBM peak); batched & fwd+bwd vs plain"
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_sauvola_4096x3072_w75.txt")
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "counters_sauvola_4096x3072_w75.txt")
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # lane-ops per second, in T


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("box.hip", "internal.hpp"):
        with open(os.path.join(ROOT, "paper_1905_13038_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(launch_px: int):
    """Counter-derived HBM bytes per launch from the committed profile
    summary, or None if it is missing or was taken on other kernel source."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    vals = {}
    for line in open(PROFILE_TRAFFIC):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def read_counter(key: str):
    """A per-pixel figure from the committed counter summary of the headline
    kernel, or None if missing or taken on other kernel source."""
    if not os.path.exists(PROFILE_COUNTERS):
        return None
    vals = {}
    for line in open(PROFILE_COUNTERS):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(I, h, w, k, R, seconds):
    """The CPU oracle on the same page: one thread, then row bands (each with
    its halo rows, re-priming its column sums) on a thread pool of up to 16
    of the host's cores.  `value` is the pool's rate."""
    import oracle
    mpix1, reps1, dt1 = oracle.time_recursive_sauvola(I, h, w, k, R, min_seconds=seconds / 2)
    nproc = os.cpu_count() or 1
    threads = max(1, min(16, nproc))
    mpixn, repsn, dtn = oracle.time_recursive_sauvola_bands(I, h, w, k, R, threads, min_seconds=seconds / 2)
    # the oracle's other paths, one thread each, on bounded samples of their
    # workloads: the direct definition (Theta(H W h w)) on the whole 512 x 384
    # page at h = w = 32, and the sliding-histogram quantiles on the first
    # 256 rows of the 2048 x 1536 page (as a 256 x 2048 image)
    from docgen import gen_document
    others = {}
    I0 = gen_document(384, 512, 1)
    t0 = time.perf_counter()
    S1, S2 = oracle.sums_direct(I0, 32, 32)
    oracle.threshold(I0, 32, 32, oracle.SAUVOLA, 0.5, 128.0, S1=S1, S2=S2)
    dt = time.perf_counter() - t0
    others["direct_sauvola_512x384_h32"] = {"Mpix_s": round(I0.size / dt / 1e6, 3), "seconds": round(dt, 3),
                                            "threads": 1, "sample": "the whole page once"}
    Iq = np.ascontiguousarray(gen_document(1536, 2048, 3, noise=10.0, stain=True)[:256])
    for qwin in (32, 101):
        t0 = time.perf_counter()
        oracle.quantile_hist(Iq, qwin, qwin, 0.5)
        dt = time.perf_counter() - t0
        others["quantile_hist_h%d_q0.5" % qwin] = {"Mpix_s": round(Iq.size / dt / 1e6, 3), "seconds": round(dt, 3),
                                                   "threads": 1,
                                                   "sample": "rows 0-255 of the 2048x1536 page, once"}
    return {
        "value": round(mpixn / 1000.0, 6),
        "unit": "Gpix/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d full passes of the %dx%d page on %d threads (row bands with their halo rows; "
                  "Algorithm 1 sweep + binary64 threshold, %.1f s) and %d on one thread (%.1f s)"
                  % (repsn, I.shape[1], I.shape[0], threads, dtn, reps1, dt1),
        "single_thread_value": round(mpix1 / 1000.0, 6),
        "nproc": nproc,
        "cpu_model": cpu_model(),
        "other_oracle_paths": others,
    }


def warm_gpu(step, seconds=0.3):
    """Run steps for a fixed time so the clocks are up before timing."""
    import torch
    t = time.time()
    i = 0
    while time.time() - t < seconds:
        for _ in range(20):
            step(i)
            i += 1
        torch.cuda.synchronize()


def _timeit(fn, n, warm=3):
    """Median per-call time in microseconds of fn(i) over n calls (HIP events
    on the current stream around each call)."""
    import torch
    for i in range(warm):
        fn(i)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for i, (a, b) in enumerate(evs):
        a.record()
        fn(i)
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in evs])) * 1e3


def _loop_us(fn, n, warm=3):
    """Average per-call time in microseconds of n back-to-back calls between
    two events (launch-to-launch throughput)."""
    import torch
    for i in range(warm):
        fn(i)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(n):
        fn(i)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) * 1e3 / n


def ragged_batch_file(suffix: str) -> str:
    """A file under the temp directory keyed by the ragged-batch recipe."""
    import tempfile
    from docgen import batch_specs
    key = hashlib.sha256(json.dumps(batch_specs(), sort_keys=True).encode()).hexdigest()[:16]
    return os.path.join(tempfile.gettempdir(), "bz_ragged_batch_%s%s" % (key, suffix))


def ragged_batch_pages(workers: int = 8):
    """The 256 pages of the ragged-batch recipe (docgen.batch_specs), each
    generated from its own seed (docgen.gen_batch), and their parameters.

    The pages (1.16 Gpx) are kept in one file under the temp directory, keyed
    by the recipe, so that a later run maps them instead of generating them
    again: counter runs start after the profiler has initialised the GPU and
    so must not start worker processes (they pass workers=1)."""
    from docgen import batch_specs, gen_batch
    specs = batch_specs()
    path = ragged_batch_file(".npy")
    sizes = [d["H"] * d["W"] for d in specs]
    flat = None
    if os.path.exists(path):
        flat = np.load(path, mmap_mode="r")
        if flat.dtype != np.uint8 or flat.size != sum(sizes):
            flat = None
    if flat is None:
        pages = gen_batch(specs, workers=workers)
        flat = np.concatenate([p.ravel() for p in pages])
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "wb") as f:
            np.save(f, flat)
        os.replace(tmp, path)
    pages, at = [], 0
    for d, n in zip(specs, sizes):
        pages.append(np.asarray(flat[at:at + n]).reshape(d["H"], d["W"]))
        at += n
    params = [{"h": d["h"], "w": d["w"], "k": d["k"], "R": d["R"], "method": "sauvola"} for d in specs]
    return pages, params


def ragged_batch_inputs(dev, pages=None):
    """The ragged batch on the device: (images, params), one tensor per page."""
    import torch
    if pages is None:
        pages = ragged_batch_pages(workers=1)
    host, params = pages
    return [torch.from_numpy(np.ascontiguousarray(p)).to(dev) for p in host], params


def soft_workload(dev, B=32, Hs=1024, Ws=1024, win=32, tau=2.0):
    """The differentiable workload (B float32 pages, h = w = win): returns
    (fwd, bwd, workspace bytes), each call one launch sequence on the current
    stream."""
    import torch
    import paper_1905_13038_amd as bz
    from docgen import soft_batch
    lib = bz.lib
    st = torch.cuda.current_stream().cuda_stream
    I, kk, Wr = soft_batch(B, Hs, Ws)
    I = torch.from_numpy(np.ascontiguousarray(I)).to(dev)
    kd = torch.from_numpy(np.asarray(kk, dtype=np.float32)).to(dev)
    Rd = torch.tensor([128.0], dtype=torch.float32, device=dev)
    gy = torch.from_numpy(np.ascontiguousarray(Wr, dtype=np.float32)).to(dev)
    y = torch.empty_like(I)
    gI = torch.empty_like(I)
    gk = torch.empty_like(kd)
    gR = torch.empty_like(Rd)
    nb = int(lib.bz_soft_workspace_size(B, Hs, Ws))
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)

    def fwd(i=0):
        rc = lib.bz_soft_sauvola_fwd(I.data_ptr(), B, Hs, Ws, Ws, win, win, kd.data_ptr(),
                                     Rd.data_ptr(), tau, y.data_ptr(), st)
        if rc != 0:
            raise RuntimeError("status %d" % rc)

    def bwd(i=0):
        rc = lib.bz_soft_sauvola_bwd(I.data_ptr(), gy.data_ptr(), B, Hs, Ws, Ws, win, win,
                                     kd.data_ptr(), Rd.data_ptr(), tau, gI.data_ptr(),
                                     gk.data_ptr(), gR.data_ptr(), ws.data_ptr(), nb, st)
        if rc != 0:
            raise RuntimeError("status %d" % rc)
    return fwd, bwd, nb


def extras(sets, host, args, batch_pages=None):
    """The other measured workloads: window sweep, Niblack, mask-only,
    mean/std, cache-warm, ragged batch, soft fwd+bwd, quantiles, Table 1,
    host-memory streaming."""
    import torch
    import paper_1905_13038_amd as bz
    from docgen import gen_document

    lib = bz.lib
    H, W = host.shape
    px = H * W
    st = torch.cuda.current_stream().cuda_stream
    out = {}

    only = set(args.extras_only.split(",")) if args.extras_only else None

    def guarded(name, fn):
        if only is not None and name not in only:
            return
        print("extra: %s" % name, file=sys.stderr, flush=True)
        try:
            out[name] = fn()
        except Exception as e:  # report, do not abort the bench line
            out[name] = {"error": "%s: %s" % (type(e).__name__, e)}

    def page_call(method, win, stats, i):
        img, mask, m, sd = sets[i % len(sets)]
        mp = m.data_ptr() if stats else None
        sp = sd.data_ptr() if stats else None
        if method == "sauvola":
            rc = lib.bz_sauvola(img.data_ptr(), H, W, W, win, win, 0.5, 128.0, mask.data_ptr(), W,
                                mp, sp, W, st)
        else:
            rc = lib.bz_niblack(img.data_ptr(), H, W, W, win, win, -0.2, mask.data_ptr(), W,
                                mp, sp, W, st)
        if rc != 0:
            raise RuntimeError("status %d" % rc)

    def sweep():
        res = {}
        for method in ("sauvola", "niblack"):
            for win in (15, 32, 75, 151):
                us = _loop_us(lambda i: page_call(method, win, True, i), 30)
                res["%s_w%d" % (method, win)] = {"us": round(us, 2), "Gpix_s": round(px / us / 1e3, 1),
                                                 "hbm_frac": round(10.0 * px / us / 1e3 / HBM_PEAK_GBS, 4)}
        g = [v["Gpix_s"] for k, v in res.items() if k.startswith("sauvola")]
        res["sauvola_min_over_max"] = round(min(g) / max(g), 3)
        return res

    def mask_only():
        us = _loop_us(lambda i: page_call("sauvola", 75, False, i), 30)
        res = {"us": round(us, 2), "Gpix_s": round(px / us / 1e3, 1), "bytes_per_px": 2,
               "hbm_frac": round(2.0 * px / us / 1e3 / HBM_PEAK_GBS, 4)}
        ops = read_counter("mask_only_valu_lane_ops_per_px")
        if ops is not None:
            # VALU roofline: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-ops/s
            res["valu_lane_ops_per_px"] = ops
            res["valu_frac"] = round(ops * px / us / 1e6 / VALU_PEAK_TOPS, 4)
        return res

    def transposed():
        # the headline page transposed: 3072 wide, 4096 tall
        Ht, Wt = W, H
        img = torch.from_numpy(np.ascontiguousarray(host.T)).to(sets[0][0].device)
        outs = [(torch.empty((Ht, Wt), dtype=torch.uint8, device=img.device),
                 torch.empty((Ht, Wt), dtype=torch.float32, device=img.device),
                 torch.empty((Ht, Wt), dtype=torch.float32, device=img.device)) for _ in range(4)]

        def f(i):
            mk, m, sd = outs[i % 4]
            rc = lib.bz_sauvola(img.data_ptr(), Ht, Wt, Wt, 75, 75, 0.5, 128.0, mk.data_ptr(), Wt,
                                m.data_ptr(), sd.data_ptr(), Wt, st)
            if rc != 0:
                raise RuntimeError("status %d" % rc)
        us = _loop_us(f, 30)
        return {"us": round(us, 2), "Gpix_s": round(px / us / 1e3, 1),
                "hbm_frac": round(10.0 * px / us / 1e3 / HBM_PEAK_GBS, 4), "shape_HxW": [Ht, Wt]}

    def mean_std():
        def f(i):
            img, mask, m, sd = sets[i % len(sets)]
            rc = lib.bz_window_mean_std(img.data_ptr(), H, W, W, 75, 75, m.data_ptr(), sd.data_ptr(), W, st)
            if rc != 0:
                raise RuntimeError("status %d" % rc)
        us = _loop_us(f, 30)
        return {"us": round(us, 2), "Gpix_s": round(px / us / 1e3, 1), "bytes_per_px": 9}

    def cache_warm():
        us = _loop_us(lambda i: page_call("sauvola", 75, True, 0), 30)
        return {"us": round(us, 2), "Gpix_s": round(px / us / 1e3, 1), "note": "one buffer set, no rotation"}

    def fill_floor():
        n = (9 * px) // 4
        bufs = [torch.empty(n, dtype=torch.float32, device=sets[0][0].device) for _ in range(4)]
        us = _loop_us(lambda i: bufs[i % 4].fill_(1.0), 20)
        return {"us": round(us, 2), "GB_s": round(4.0 * n / us / 1e3, 1),
                "note": "torch fill_ of 9 B/px (the output bytes of one page), rotated over 4 buffers"}

    def batch():
        # the 256 ragged pages, each generated from its own seed; the timed
        # plan takes its strip heights from the autotuner's table (measured on
        # this device, or read from its cache)
        from paper_1905_13038_amd import tune
        imgs, params = ragged_batch_inputs(sets[0][0].device, batch_pages)
        tot = sum(int(t.numel()) for t in imgs)
        plan = bz.BatchPlan(imgs, params)
        outs = plan.outputs()
        default_us = _loop_us(lambda i: plan.run(), 10, warm=2)
        synth = tune.autotune()
        plan.replan(tune.strips_for(params, synth))
        synth_us = _loop_us(lambda i: plan.run(), 10, warm=2)
        table = tune.autotune_plan(plan, params)  # leaves the plan on its result
        with open(ragged_batch_file("_strips.json"), "w") as f:  # for the counter runs
            json.dump({str(c): v for c, v in table.items()}, f)

        def plain(i):
            for img, p, (mk, mn, sd) in zip(imgs, params, outs):
                Hh, Ww = img.shape
                rc = lib.bz_sauvola(img.data_ptr(), Hh, Ww, Ww, p["h"], p["w"], p["k"], p["R"],
                                    mk.data_ptr(), mk.stride(0), mn.data_ptr(), sd.data_ptr(),
                                    mn.stride(0), st)
                if rc != 0:
                    raise RuntimeError("status %d" % rc)
        plain_us = _loop_us(plain, 5, warm=1)
        run_us = _loop_us(lambda i: plan.run(), 10, warm=2)
        plan.capture()
        graph_us = _loop_us(lambda i: plan.replay(), 10, warm=2)
        return {"images": len(imgs), "Gpx": round(tot / 1e9, 4),
                "graph_replay_us": round(graph_us, 1), "persistent_run_us": round(run_us, 1),
                "persistent_run_default_strips_us": round(default_us, 1),
                "persistent_run_synthetic_table_us": round(synth_us, 1),
                "synthetic_strip_table": {str(c): s_ for c, s_ in sorted(synth.items())},
                "plain_calls_us": round(plain_us, 1),
                "graph_Gpix_s": round(tot / graph_us / 1e3, 1),
                "plain_Gpix_s": round(tot / plain_us / 1e3, 1),
                "graph_hbm_frac": round(10.0 * tot / graph_us / 1e3 / HBM_PEAK_GBS, 4),
                "strip_table": {str(c): s_ for c, s_ in sorted(table.items())},
                "inputs": "the 256 pages of the ragged-batch recipe, each generated from its own seed "
                          "(4000 + b), with the recipe's shapes, windows and k"}

    def soft():
        B, Hs, Ws, win, tau = 32, 1024, 1024, 32, 2.0
        fwd, bwd, nb = soft_workload(sets[0][0].device, B, Hs, Ws, win, tau)
        f_us = _loop_us(fwd, 10)
        b_us = _loop_us(bwd, 10)
        n = B * Hs * Ws
        return {"fwd_us": round(f_us, 1), "bwd_us": round(b_us, 1), "fwd_bwd_us": round(f_us + b_us, 1),
                "fwd_Gpix_s": round(n / f_us / 1e3, 1), "fwd_bwd_Gpix_s": round(n / (f_us + b_us) / 1e3, 1),
                "fwd_hbm_frac": round(8.0 * n / f_us / 1e3 / HBM_PEAK_GBS, 4),
                "bwd_hbm_frac": round(12.0 * n / b_us / 1e3 / HBM_PEAK_GBS, 4),
                "workspace_bytes": nb, "shape": [B, Hs, Ws], "h": win, "tau": tau}

    def quantiles():
        Hq, Wq = 1536, 2048
        dev = sets[0][0].device
        img = torch.from_numpy(gen_document(Hq, Wq, 3, noise=10.0, stain=True)).to(dev)
        Q = torch.empty_like(img)
        mk = torch.empty_like(img)
        res = {}
        for win in (32, 101):
            for q in (0.5, 0.1):
                def f(i):
                    rc = lib.bz_window_quantile(img.data_ptr(), Hq, Wq, Wq, win, win, q, Q.data_ptr(), Wq,
                                                mk.data_ptr(), Wq, st)
                    if rc != 0:
                        raise RuntimeError("status %d" % rc)
                us = _loop_us(f, 10)
                npx = Hq * Wq
                res["h%d_q%g" % (win, q)] = {"us": round(us, 1), "Gpix_s": round(npx / us / 1e3, 2),
                                            "G_updates_s": round(2.0 * win * npx / us / 1e3, 1)}
        # Bernsen's rule: the window extremes (two separable passes) and the
        # midrange decision
        mn = torch.empty_like(img)
        mx = torch.empty_like(img)
        nb = int(lib.bz_extremes_workspace_size(Hq, Wq))
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)

        def b(i):
            rc = lib.bz_bernsen(img.data_ptr(), Hq, Wq, Wq, 32, 32, 15, mk.data_ptr(), Wq, mn.data_ptr(),
                                mx.data_ptr(), Wq, ws.data_ptr(), nb, st)
            if rc != 0:
                raise RuntimeError("status %d" % rc)
        us = _loop_us(b, 10)
        res["bernsen_h32"] = {"us": round(us, 1), "Gpix_s": round(Hq * Wq / us / 1e3, 2)}
        return res

    warm_gpu(lambda i: page_call("sauvola", 75, True, i))
    def table1():
        # the other rules of Table 1 on the headline page (w = 75), mask + mean
        # + std, with the page's global-statistics record computed once
        rules = {"wolf": (0.5, 128.0), "feng": (0.9, 0.2, 0.3, 0.5, 128.0), "rais": (),
                 "nick": (-0.1,), "phansalkar": (2.0, 0.04, 0.25, 128.0)}
        recs = [bz.global_stats(s_[0]) for s_ in sets]
        res = {}
        g_us = _loop_us(lambda i: lib.bz_global_stats(sets[i % len(sets)][0].data_ptr(), H, W, W,
                                                      recs[i % len(sets)].data_ptr(), st), 20)
        res["global_stats"] = {"us": round(g_us, 2), "GB_s": round(px / g_us / 1e3, 1)}
        for name, p in rules.items():
            code = bz.TABLE1[name][0]
            pv = (ctypes.c_double * 5)(*(list(p) + [0.0] * (5 - len(p))))

            def f(i, code=code, pv=pv):
                img, mask, m, sd = sets[i % len(sets)]
                rc = lib.bz_threshold(img.data_ptr(), H, W, W, 75, 75, code, pv,
                                      recs[i % len(sets)].data_ptr(), mask.data_ptr(), W, m.data_ptr(),
                                      sd.data_ptr(), W, st)
                if rc != 0:
                    raise RuntimeError("status %d" % rc)
            us = _loop_us(f, 20)
            res[name] = {"us": round(us, 2), "Gpix_s": round(px / us / 1e3, 1),
                         "hbm_frac": round(10.0 * px / us / 1e3 / HBM_PEAK_GBS, 4)}
        return res

    def streamed():
        # the banded host-memory path: page-locked image in, mask out, the
        # call synchronous (wall clock, median); 2 bytes per pixel cross PCIe
        dev = sets[0][0].device

        def wall(fn, n):
            ts = []
            for _ in range(n):
                t0 = time.perf_counter()
                fn()
                ts.append(time.perf_counter() - t0)
            return float(np.median(ts)) * 1e6

        res = {}
        src = torch.empty((H, W), dtype=torch.uint8, pin_memory=True)
        src.copy_(torch.from_numpy(host))
        outp = torch.empty((H, W), dtype=torch.uint8, pin_memory=True)
        # row bands of 384 rows; column bands of 512, 2048 and 4096 columns
        # (the last is one band: a single 2-D copy each way)
        for band, axis in ((384, "rows"), (512, "columns"), (2048, "columns"), (4096, "columns")):
            page = lambda: bz.binarize_streamed(src, 75, 75, "sauvola", 0.5, 128.0, out=outp, band=band,
                                                axis=axis)
            page()
            us = wall(page, 5)
            res["page_%dx%d_w75_%s_band%d" % (W, H, axis, band)] = {
                "us": round(us, 1), "Gpix_s": round(px / us / 1e3, 2), "pcie_GB_s": round(2.0 * px / us / 1e3, 1)}
        d = torch.empty((H, W), dtype=torch.uint8, device=dev)

        def h2d():
            d.copy_(src, non_blocking=True)
            torch.cuda.synchronize()

        def d2h():
            outp.copy_(d, non_blocking=True)
            torch.cuda.synchronize()
        res["copy_h2d_GB_s"] = round(px / wall(h2d, 5) / 1e3, 1)
        res["copy_d2h_GB_s"] = round(px / wall(d2h, 5) / 1e3, 1)
        # scans of 32 pages' size binarized in place, in row bands: tall and
        # wide, of the default depth (slots of about 32 MiB) and of 512 rows
        for (ty, tx, band) in ((8, 4, None), (8, 4, 512), (4, 8, None)):
            Hb, Wb = ty * H, tx * W
            big = torch.empty((Hb, Wb), dtype=torch.uint8, pin_memory=True)
            big.copy_(torch.from_numpy(np.tile(host, (ty, tx))))
            scan = lambda: bz.binarize_streamed(big, 75, 75, "sauvola", 0.5, 128.0, out=big, band=band)
            scan()
            us = wall(scan, 3)
            res["scan_%dx%d_w75_in_place_band_%s" % (Wb, Hb, band or "default")] = {
                "us": round(us, 1), "Gpix_s": round(Hb * Wb / us / 1e3, 2),
                "pcie_GB_s": round(2.0 * Hb * Wb / us / 1e3, 1)}
            del big
        return res

    def haar():
        # Haar-like features on the headline page: 12 x 12 cells, and 48 x 48;
        # algorithmic bytes 1 (I) + 4 (F) per output position
        res = {}
        img = sets[0][0]
        for (a, kind) in ((12, "edge_h"), (12, "checker"), (48, "line_v")):
            code, (kv, kh) = bz.HAAR[kind]
            Hf, Wf = H - kv * a + 1, W - kh * a + 1
            F = torch.empty((Hf, Wf), dtype=torch.int32, device=img.device)
            nb = int(lib.bz_haar_workspace_size(H, W, a, code))
            ws = torch.empty(nb, dtype=torch.uint8, device=img.device)

            def f(i, a=a, code=code, F=F, ws=ws, nb=nb, Wf=Wf):
                rc = lib.bz_haar_features(sets[i % len(sets)][0].data_ptr(), H, W, W, a, a, code, F.data_ptr(), Wf,
                                          ws.data_ptr(), nb, st)
                if rc != 0:
                    raise RuntimeError("status %d" % rc)
            us = _loop_us(f, 20)
            res["%s_a%d" % (kind, a)] = {"us": round(us, 1), "Gpix_s": round(Hf * Wf / us / 1e3, 1),
                                         "hbm_frac": round(5.0 * Hf * Wf / us / 1e3 / HBM_PEAK_GBS, 4)}
        return res

    def tiling():
        # the autotuner's single-image table (measured here), and the headline
        # call with it installed against the built-in plan
        from paper_1905_13038_amd import tune
        rows = tune.autotune_plain(cache_path=None)
        base = _loop_us(lambda i: page_call("sauvola", 75, True, i), 20)
        bz.set_tile_table(rows)
        try:
            tuned = _loop_us(lambda i: page_call("sauvola", 75, True, i), 20)
        finally:
            bz.set_tile_table([])
        return {"rows": rows, "headline_builtin_us": round(base, 2), "headline_tuned_us": round(tuned, 2)}

    guarded("window_sweep", sweep)
    guarded("sauvola_w75_mask_only", mask_only)
    guarded("sauvola_w75_transposed_3072x4096", transposed)
    guarded("mean_std_w75", mean_std)
    guarded("sauvola_w75_cache_warm", cache_warm)
    guarded("write_floor_9Bpx", fill_floor)
    guarded("ragged_batch_256", batch)
    guarded("soft_fwd_bwd_32x1024x1024_h32", soft)
    guarded("quantile_2048x1536", quantiles)
    guarded("table1_4096x3072_w75", table1)
    guarded("haar_4096x3072", haar)
    guarded("tiling_autotune_plain", tiling)
    guarded("streamed_host", streamed)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--sets", type=int, default=8, help="rotated buffer sets")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extras-only", default=None,
                    help="comma-separated names of the extras to run (default: all)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (window sweep, batch, soft, quantiles)")
    ap.add_argument("--pmc", action="store_true",
                    help="counter run: 3 launches + 3 plain 1 GiB copies, no JSON")
    ap.add_argument("--pmc-workload", choices=("page", "mask_only", "batch", "soft", "quantile"),
                    default="page",
                    help="what --pmc launches: the headline page (mask + mean + std, or the mask "
                         "only), the 256-page ragged batch (one persistent launch each), the soft "
                         "forward + backward, or the 2048x1536 quantiles (q = 0.5, h = 32 and 101)")
    ap.add_argument("--win", type=int, default=75)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    # the ragged batch's pages are generated first, in worker processes,
    # before anything touches the GPU
    only = None if args.extras_only is None else set(args.extras_only.split(","))
    batch_pages = None
    if args.pmc and args.pmc_workload == "batch":
        batch_pages = ragged_batch_pages(workers=1)
    elif not args.pmc and not args.no_extras and (only is None or "ragged_batch_256" in only):
        batch_pages = ragged_batch_pages()

    import torch
    import paper_1905_13038_amd as bz
    from docgen import gen_document

    H, W, win, k, R = 3072, 4096, args.win, 0.5, 128.0
    host = gen_document(H, W, 2, noise=10.0, stain=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sets = []
    for s in range(args.sets):
        img = torch.from_numpy(host).to(dev) if s == 0 else sets[0][0].clone()
        mask = torch.empty((H, W), dtype=torch.uint8, device=dev)
        m = torch.empty((H, W), dtype=torch.float32, device=dev)
        sd = torch.empty((H, W), dtype=torch.float32, device=dev)
        sets.append((img, mask, m, sd))
    torch.cuda.synchronize()

    def step(i):
        img, mask, m, sd = sets[i % len(sets)]
        bz.sauvola(img, win, win, k=k, R=R, mask=mask, mean=m, std=sd)

    if args.pmc:
        if args.pmc_workload == "batch":
            # the strips the timed batch measured on itself (bench.py's batch
            # run leaves them in the temp directory), else the defaults
            from paper_1905_13038_amd import tune
            imgs, params = ragged_batch_inputs(dev, batch_pages)
            table = None
            if os.path.exists(ragged_batch_file("_strips.json")):
                with open(ragged_batch_file("_strips.json")) as f:
                    table = {int(c): int(v) for c, v in json.load(f).items()}
            plan = bz.BatchPlan(imgs, params, strips=tune.strips_for(params, table))
            for i in range(3):
                plan.run()
        elif args.pmc_workload == "soft":
            fwd, bwd, _ = soft_workload(dev)
            for i in range(3):
                fwd()
                bwd()
        elif args.pmc_workload == "mask_only":
            for i in range(3):
                img, mask, m, sd = sets[i % len(sets)]
                bz.sauvola(img, win, win, k=k, R=R, stats=False, mask=mask)
        elif args.pmc_workload == "quantile":
            qimg = torch.from_numpy(gen_document(1536, 2048, 3, noise=10.0, stain=True)).to(dev)
            for qwin in (32, 101):
                for i in range(3):
                    bz.window_quantile(qimg, qwin, qwin, 0.5)
        else:
            for i in range(3):
                step(i)
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("pmc workload done", flush=True)
        return

    for i in range(args.warmup):
        step(i)
    warm_gpu(step)
    stream = torch.cuda.current_stream(dev)
    # Timed region: K back-to-back steps between two events on the stream the
    # kernel runs on.  One step is one launch; the per-step time includes the
    # host launch gap between consecutive kernels.
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for i in range(args.steps):
        step(i)
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)

    # Kernel duration for the roofline: the timed region itself (one launch
    # per step; the queue stays full, so the per-step time is the kernel's
    # duration plus the device-side gap between consecutive dispatches).
    launch_ms = total_ms / args.steps
    # and the median of single launches, each between two events (the
    # events' own overhead included)
    median_us = _timeit(step, 50) if not args.pmc else None

    px = H * W
    ms_per_step = total_ms / args.steps
    value = px / (ms_per_step * 1e-3) / 1e9
    alg_bytes = 10.0 * px
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    traffic = read_traffic(px)
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32+f32",
        "data": "synthetic",
        "config": {"workload": "sauvola_4096x3072_w%d" % win, "W": W, "H": H, "h": win, "w": win,
                   "k": k, "R": R, "outputs": "mask u8 + mean f32 + std f32",
                   "buffer_sets": args.sets},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_box<MODE_SAUVOLA>",
                     "launch_us_mean": round(launch_ms * 1e3, 3),
                     "launch_us_median_single": round(median_us, 3),
                     "launch_us_source": "HIP events around the timed region's back-to-back launches",
                     "algorithmic_bytes": int(alg_bytes)},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(host, win, win, k, R, args.cpu_seconds)
    if not args.no_extras:
        out["extras"] = extras(sets, host, args, batch_pages)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
