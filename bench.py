"""Benchmark of the ROIBIN-SZ compression path on one MI355X.

Workload: a batch of 1000 CSPAD-geometry frames (32 x 185 x 388 float32,
seeded synthetic: Gaussian noise, water ring, Bragg peaks with Poisson(60)
counts and 20% non-hit frames), ROI window 17, 2x2 binning, absolute error
bound 10 ADU.  One step = one batched compression of all 1000 frames (every
kernel of the path, one launch each); frames are resident in HBM before the
timed region.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "cspad-batch"
NFRAMES = 1000
SHAPE = (32, 185, 388)
WINDOW, BIN, EB = 17, 2, 10.0


def _gen(i):
    from paper_2206_11297_amd import synth
    counts = synth.batch_peak_counts(NFRAMES)
    return synth.batch_frame(i, counts)


def generate(fn, n, workers):
    """[fn(0), ..., fn(n-1)] on a pool of threads (the generators spend their
    time in numpy, which releases the interpreter lock); no process is
    forked, before or after the GPU is initialised."""
    from concurrent.futures import ThreadPoolExecutor
    if workers <= 1:
        return [fn(i) for i in range(n)]
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(fn, range(n)))


def _gen_pool(k):
    """Frame k of the serving pool: geometries cycle over CSPAD 32x185x388,
    Jungfrau 8x512x1024 and a 1x2048x2048 panel; 0-1500 peaks each."""
    from paper_2206_11297_amd import synth
    import numpy as np
    rng = np.random.default_rng([2206, 11297, synth.W_SERVE, k])
    npk = int(rng.integers(0, 1501))
    g = k % 3
    if g == 0:
        return synth.cspad_frame(k, npeaks=npk, workload=synth.W_SERVE)
    shape = synth.JUNGFRAU4M if g == 1 else synth.SQUARE4M
    return synth.jungfrau_frame(k, shape=shape, npeaks=npk, workload=synth.W_SERVE)


def serving_section(args, torch, dev, pool):
    """Poisson-arrival serving of mixed geometries: continuous batching vs one
    frame per launch at the same offered load, plus a backlogged run.  pool:
    the resident frames (host arrays, drawn before the GPU was touched)."""
    import numpy as np
    from paper_2206_11297_amd import serve
    npool = len(pool)
    gpool = [(torch.from_numpy(f).to(dev), torch.from_numpy(p).to(dev)) for f, p in pool]
    torch.cuda.synchronize()
    out = {"workload": f"serving: Poisson arrivals, pool of {npool} resident frames cycling "
                       "32x185x388 / 8x512x1024 / 1x2048x2048 f32, 0-1500 peaks, eb from "
                       "{5,10,20} per request, window 17, bin 2x2",
           "slots": args.serve_slots, "max_batch": args.serve_batch}
    limits = serve.SlotLimits(max_frames=args.serve_batch,
                              out_bytes=args.serve_batch * (14 << 20),
                              ws_bytes=args.serve_batch * (12 << 20))
    out["hbm_budget_gb"] = round(args.serve_slots * (limits.out_bytes + limits.ws_bytes) / 1e9, 2)
    batched = serve.GpuExecutor(args.serve_slots, limits, dev)
    # one frame per launch: a slot sized for the largest request of the pool,
    # so that it carries every request the batched slots carry
    need_out = need_ws = 0
    for f, p in gpool:
        for eb in (5.0, 10.0, 20.0):
            r = serve.Request(0, 0.0, f, p, (17, 2, eb, 0))
            batched.size_request(r)
            need_out, need_ws = max(need_out, r.out_cap), max(need_ws, r.ws_bytes)
    single_lim = serve.SlotLimits(1, need_out, need_ws)
    single = serve.GpuExecutor(1, single_lim, dev)

    def requests(rate, n, seed):
        rng = np.random.default_rng([2206, 11297, 3, seed])
        t = np.cumsum(rng.exponential(1.0 / rate, n)) if rate else np.zeros(n)
        reqs = []
        for i in range(n):
            k = int(rng.integers(0, npool))
            eb = float([5.0, 10.0, 20.0][int(rng.integers(0, 3))])
            reqs.append(serve.Request(i, float(t[i]), gpool[k][0], gpool[k][1], (17, 2, eb, 0)))
        return reqs

    # warm-up of both paths
    serve.Scheduler(batched, args.serve_slots, limits).run(requests(0, 16, 1001))
    serve.Scheduler(single, 1, single_lim).run(requests(0, 4, 1002))
    for rate in args.serve_rates:
        reqs = requests(rate * 1e3, args.serve_frames, int(rate))
        rb = serve.summarize(serve.Scheduler(batched, args.serve_slots, limits).run(reqs), reqs)
        rs = serve.summarize(serve.Scheduler(single, 1, single_lim).run(reqs), reqs)
        out[f"{rate:g}kHz"] = {"continuous_batching": rb, "one_frame_per_launch": rs}
        print(f"[bench] serving {rate:g} kHz: batched p99 {rb['p99_ms']} ms, one-frame p99 "
              f"{rs['p99_ms']} ms", file=sys.stderr, flush=True)
    reqs = requests(0, args.serve_frames, 99)
    out["backlogged"] = serve.summarize(serve.Scheduler(batched, args.serve_slots, limits).run(reqs),
                                        reqs)
    return out


def decompress_section(args, torch, dev, B, sizes, host):
    """Decompression of the first frames' streams, one frame per call
    (rsz_decompress: header read, kernels, status read): per-frame latency,
    reconstructed GB/s and per-kernel times (bit-exactness against the
    oracle's reconstruction is what the GPU tests check)."""
    import numpy as np
    from paper_2206_11297_amd import rsz
    n = min(args.decompress_frames, len(sizes))
    streams = [B.stream(i, sizes).clone() for i in range(n)]
    head = streams[0][:80].cpu().numpy().tobytes()
    st, wsb = rsz.rsz_decompress_workspace_bytes(head)
    ws = rsz.workspace(wsb * 2, dev)
    out = torch.empty(SHAPE, dtype=torch.float32, device=dev)
    s = rsz._stream()
    for i in range(min(3, n)):   # warm-up
        rsz.rsz_decompress(rsz._ptr(streams[i]), streams[i].numel(), rsz._ptr(out), out.numel(),
                           rsz._ptr(ws), ws.numel(), s)
    torch.cuda.synchronize()
    rsz.rsz_profile_enable(True)
    lat = []
    for i in range(n):
        a = time.perf_counter()
        st = rsz.rsz_decompress(rsz._ptr(streams[i]), streams[i].numel(), rsz._ptr(out),
                                out.numel(), rsz._ptr(ws), ws.numel(), s)
        lat.append(time.perf_counter() - a)
        assert st == 0, f"decompress frame {i}: status {st}"
    prof = rsz.rsz_profile_read()
    rsz.rsz_profile_enable(False)
    lat_ms = np.array(lat) * 1e3
    fb = SHAPE[0] * SHAPE[1] * SHAPE[2] * 4
    del streams, ws, out
    batched = batched_decode(torch, B, sizes, args.decompress_steps, len(sizes) * fb)
    print(f"[bench] batched decompression: {batched['gbps']} GB/s", file=sys.stderr, flush=True)
    return {"frames": n, "mode": "one frame per call (synchronous)",
            "p50_ms": round(float(np.percentile(lat_ms, 50)), 4),
            "p99_ms": round(float(np.percentile(lat_ms, 99)), 4),
            "gbps": round(n * fb / (lat_ms.sum() / 1e3) / 1e9, 2),
            "kernel_ms_per_frame": {k: round(v[1] / v[0], 4) for k, v in prof.items()},
            "batched": batched}


def batched_decode(torch, B, sizes, steps, raw_bytes):
    """Every stream of batch B decoded in one batched call
    (rsz_decompress_batch: one launch of each decoder kernel for all of
    them), timed with no events; per-kernel times from a profiled pass after
    it."""
    from paper_2206_11297_amd import rsz
    D = rsz.DecodeBatch([B.stream(i, sizes) for i in range(len(sizes))])
    for _ in range(2):
        D.run()
    torch.cuda.synchronize()
    assert (D.status.cpu().numpy() == 0).all()
    t0 = time.perf_counter()
    for _ in range(steps):
        D.run()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    rsz.rsz_profile_enable(True)
    for _ in range(max(1, min(steps, 3))):
        D.run()
    torch.cuda.synchronize()
    prof = rsz.rsz_profile_read()
    rsz.rsz_profile_enable(False)
    del D
    torch.cuda.empty_cache()
    return {"frames": len(sizes), "ms_per_batch": round(el * 1e3, 4),
            "gbps": round(raw_bytes / el / 1e9, 2),
            "kernel_ms": {k: round(v[1] / v[0], 4) for k, v in prof.items()}}


def timed_steps(torch, B, steps):
    """Seconds per step of B.run() with no timing events, then per-kernel
    milliseconds from a profiled pass of up to 3 more steps."""
    from paper_2206_11297_amd import rsz
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        B.run()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    rsz.rsz_profile_enable(True)
    for _ in range(max(1, min(steps, 3))):
        B.run()
    torch.cuda.synchronize()
    prof = rsz.rsz_profile_read()
    rsz.rsz_profile_enable(False)
    return el, {k: round(v[1] / v[0], 4) for k, v in prof.items()}


def lorenzo_dims_section(args, torch, frames, peaks, prm, knobs, raw_bytes):
    """The same batch with the Lorenzo predictor in one and three dimensions
    (Sec. VI): whole-path GB/s, compression ratio and per-kernel times."""
    import numpy as np
    from paper_2206_11297_amd import rsz
    out = {}
    npix = raw_bytes // 4
    for dim in args.dims:
        B = rsz.Batch(frames, peaks, prm + (dim,), **knobs)
        for _ in range(2):
            B.run()
        torch.cuda.synchronize()
        st = B.status.cpu().numpy()
        assert (st == 0).all(), f"dim {dim}: statuses {set(st.tolist())}"
        el, kms = timed_steps(torch, B, args.dims_steps)
        sizes = B.sizes.cpu().numpy().astype(np.int64)
        out[f"dim{dim}"] = {"value": round(raw_bytes / el / 1e9, 2), "unit": "GB/s",
                            "ms_per_step": round(el * 1e3, 4), "steps": args.dims_steps,
                            "compression_ratio_u16_aggregate": round(float(npix * 2 / sizes.sum()), 3),
                            "kernel_ms": kms}
        print(f"[bench] dim {dim}: {out[f'dim{dim}']['value']} GB/s, CR "
              f"{out[f'dim{dim}']['compression_ratio_u16_aggregate']}", file=sys.stderr, flush=True)
        del B
        torch.cuda.empty_cache()
    return out


def coding_section(args, torch, frames, peaks, prm, raw_bytes, knobs, roi, run, steps, label):
    """The same batch with the ROI windows coded losslessly instead of stored
    verbatim (roi) and/or the Huffman bits' zero runs Rice coded (run):
    whole-path GB/s, compression ratio and per-kernel times."""
    import numpy as np
    from paper_2206_11297_amd import rsz
    B = rsz.Batch(frames, peaks, prm + (2, roi, run), **knobs)
    for _ in range(2):
        B.run()
    torch.cuda.synchronize()
    st = B.status.cpu().numpy()
    assert (st == 0).all(), f"{label}: statuses {set(st.tolist())}"
    el, kms = timed_steps(torch, B, steps)
    sizes = B.sizes.cpu().numpy().astype(np.int64)
    out = {"value": round(raw_bytes / el / 1e9, 2), "unit": "GB/s", "ms_per_step": round(el * 1e3, 4),
           "steps": steps,
           "compression_ratio_u16_aggregate": round(float(raw_bytes / 2 / sizes.sum()), 3),
           "kernel_ms": kms}
    # the same streams decoded in one batched call
    out["decompress_batched"] = batched_decode(torch, B, sizes, steps, raw_bytes)
    print(f"[bench] {label}: {out['value']} GB/s, CR {out['compression_ratio_u16_aggregate']}; "
          f"batched decompression {out['decompress_batched']['gbps']} GB/s",
          file=sys.stderr, flush=True)
    del B
    torch.cuda.empty_cache()
    return out


def peaks_section(args, torch, frames, prm, raw_bytes, knobs):
    """Peak finding on the GPU over the same batch (the step before the path,
    Sec. IV-B parameters), and the frames-in, streams-out pipeline: peaks found,
    counts read back, frames with fewer than 10 peaks rejected (Sec. IV),
    the hits compressed with their found peaks."""
    import numpy as np
    from paper_2206_11297_amd import rsz
    P = rsz.PeakBatch(frames, None, 1024)
    for _ in range(2):
        P.run()
    torch.cuda.synchronize()
    st = P.status.cpu().numpy()
    assert (st == 0).all(), f"peak finding failed: statuses {set(st.tolist())}"
    rsz.rsz_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.peaks_steps):
        P.run()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.peaks_steps
    prof = rsz.rsz_profile_read()
    rsz.rsz_profile_enable(False)
    km = {k: v[1] / v[0] for k, v in prof.items()}
    counts = P.counts.cpu().numpy()
    hits = [i for i, c in enumerate(counts.tolist()) if c >= 10]
    find_ms = km["k_peaks_find"]
    out = {"value": round(raw_bytes / el / 1e9, 2), "unit": "GB/s", "ms_per_step": round(el * 1e3, 4),
           "steps": args.peaks_steps, "kernel_ms": {k: round(v, 4) for k, v in km.items()},
           "roofline": {"bound": "hbm", "achieved": round(raw_bytes / (find_ms * 1e-3) / 1e9, 1),
                        "peak": 8000.0, "unit": "GB/s",
                        "frac": round(raw_bytes / (find_ms * 1e-3) / 1e9 / 8000.0, 4),
                        "traffic": (traffic_record("k_peaks_find") or {}).get("hbm_bytes_per_launch"),
                        "kernel": "k_peaks_find", "algorithmic_bytes_per_launch": raw_bytes},
           "peaks_per_frame_mean": round(float(counts.mean()), 2),
           "hits": len(hits), "frames": len(frames), "nhr_min_peaks": 10}
    if hits:
        B = rsz.Batch([frames[i] for i in hits], [P.peaks(i, counts) for i in hits], prm, **knobs)
        for _ in range(2):
            P.run()
            c2 = P.counts.cpu().numpy()
            B.run()
        torch.cuda.synchronize()
        assert (c2 == counts).all() and (B.status.cpu().numpy() == 0).all()
        t0 = time.perf_counter()
        for _ in range(args.peaks_steps):
            P.run()
            P.counts.cpu()          # the counts plan the compression
            B.run()
        torch.cuda.synchronize()
        el2 = (time.perf_counter() - t0) / args.peaks_steps
        sizes = B.sizes.cpu().numpy().astype(np.int64)
        hit_bytes = sum(frames[i].numel() * 4 for i in hits)
        out["pipeline"] = {
            "value": round(raw_bytes / el2 / 1e9, 2), "unit": "GB/s of all frames",
            "ms_per_step": round(el2 * 1e3, 4),
            "compression_ratio_u16_hits": round(float(hit_bytes / 2 / sizes.sum()), 3),
            "compression_ratio_u16_with_nhr": round(float(raw_bytes / 2 / sizes.sum()), 3)}
        del B
    print(f"[bench] peak finding: {out['value']} GB/s, {out['peaks_per_frame_mean']} peaks/frame, "
          f"{len(hits)} hits", file=sys.stderr, flush=True)
    del P
    torch.cuda.empty_cache()
    return out


def cpu_baseline(args, host, B, sizes):
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from oracle import rsz_oracle as O
    po = O.params(*SHAPE, WINDOW, BIN, EB, 0)
    out_host = B.out.cpu().numpy()
    frame_bytes = SHAPE[0] * SHAPE[1] * SHAPE[2] * 4

    def one(k):
        i = k % len(host)   # the frame-parallel leg cycles over the frames
        f, pk = host[i]
        sto, ref, _ = O.compress(po, f, pk)
        got = out_host[B.offsets[i]:B.offsets[i] + int(sizes[i])]
        return sto == 0 and np.array_equal(got, ref)

    budget = args.cpu_seconds
    n1, t1, parity = 0, 0.0, True
    while n1 < len(host) and t1 < budget / 2:
        a = time.perf_counter()
        parity &= one(n1)
        t1 += time.perf_counter() - a
        n1 += 1
    if n1 == 0:
        return None
    single = n1 * frame_bytes / t1 / 1e9
    threads = max(1, min(args.cpu_threads, os.cpu_count() or 1))
    # frames for about budget/2 of wall time at the single-thread rate x threads
    nmt = int(max(threads, threads * (budget / 2) * n1 / t1))
    a = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        oks = list(ex.map(one, range(nmt)))
    tmt = time.perf_counter() - a
    parity &= all(oks)
    return {"value": round(nmt * frame_bytes / tmt / 1e9, 4), "unit": "GB/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{nmt} frame compressions cycling over the first {min(nmt, len(host))} "
                      f"frames of the batch, one frame per thread on {threads} threads, "
                      f"{tmt:.1f}s wall; single thread: first {n1} frames, {t1:.1f}s",
            "single_thread_value": round(single, 4), "streams_equal_gpu": bool(parity)}


def _counter_rows(root, counter):
    """Per-dispatch values of one counter from rocprofv3 CSV output under root:
    {kernel name: [(grid size, value in KiB)]}."""
    import csv
    import glob
    rows = {}
    for path in glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != counter:
                    continue
                rows.setdefault(r["Kernel_Name"], []).append(
                    (int(r.get("Grid_Size") or 0), float(r["Counter_Value"])))
    return rows


# Kernels whose counter records the roofline reads: (record name, the kernel
# name in the counter output, the source file it is built from, and which of
# its dispatches to take: the largest grid).
TRAFFIC_KERNELS = [("k_bin", "k_bin_vec<2, 2>", "compress.hip"),
                   ("k_count", "k_count<true>", "compress.hip"),
                   ("k_encode", "k_encode", "compress.hip"),
                   ("k_lorenzo_dims", "k_lorenzo_dims", "compress.hip"),
                   ("k_peaks_find", "k_peaks_find", "peaks.hip")]

# The counters of the SQ passes summarised per kernel, and what is derived
# from them (SQ_*_CYCLES and SQ_BUSY_CYCLES count in units of 4 cycles on
# this chip's counter blocks; ratios of like counters need no scale).
SQ_COUNTERS = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD",
               "SQ_INSTS_VMEM_WR", "SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
               "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS",
               "SQ_LDS_BANK_CONFLICT", "MeanOccupancyPerCU"]


def counter_summary(dirs, out_path):
    """Markdown table of the SQ counter passes (rocprofv3 CSV output under
    each of dirs): per kernel and grid, the mean per dispatch of each
    counter, the share of wave time spent waiting, and LDS bank conflicts
    per LDS instruction."""
    vals = {}
    for d in dirs:
        for c in SQ_COUNTERS:
            for k, lst in _counter_rows(d, c).items():
                for g, v in lst:
                    vals.setdefault((k, g), {}).setdefault(c, []).append(v)
    mean = lambda x: sum(x) / len(x) if x else float("nan")
    head = ["kernel", "grid", "waves", "VALU insts", "SALU insts", "LDS insts", "VMEM rd",
            "VMEM wr", "wait share", "LDS conflicts / LDS inst", "mean occupancy / CU"]
    lines = ["| " + " | ".join(head) + " |", "|" + "---|" * len(head)]
    for (k, g), d in sorted(vals.items(), key=lambda t: -mean(t[1].get("SQ_WAVE_CYCLES", [0]))):
        if "rsz::" not in k:
            continue
        m = {c: mean(d.get(c, [])) for c in SQ_COUNTERS}
        wait = m["SQ_WAIT_ANY"] / m["SQ_WAVE_CYCLES"] if m["SQ_WAVE_CYCLES"] else float("nan")
        conf = m["SQ_LDS_BANK_CONFLICT"] / m["SQ_INSTS_LDS"] if m["SQ_INSTS_LDS"] else 0.0
        name = k.replace("(rsz::BatchPlan)", "").replace("void ", "")
        lines.append(f"| `{name[:48]}` | {g} | {m['SQ_WAVES']:.0f} | {m['SQ_INSTS_VALU']:.3g} | "
                     f"{m['SQ_INSTS_SALU']:.3g} | {m['SQ_INSTS_LDS']:.3g} | "
                     f"{m['SQ_INSTS_VMEM_RD']:.3g} | {m['SQ_INSTS_VMEM_WR']:.3g} | {wait:.2f} | "
                     f"{conf:.3f} | {m['MeanOccupancyPerCU']:.1f} |")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _source_sha(name):
    src = os.path.join(ROOT, "paper_2206_11297_amd", "csrc", name)
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def traffic_summary(fetch_dir, write_dir, out_dir):
    """Summary of two rocprofv3 --pmc runs of this script (FETCH_SIZE, then
    WRITE_SIZE, both with --copy-calibration): per-kernel HBM bytes per
    dispatch, scaled by what the counters read for a 1 GiB device copy (reads
    1 GiB) and a 1 GiB fill (writes 1 GiB).  Writes the JSON records read by
    the rooflines and a Markdown table."""
    fetch = _counter_rows(fetch_dir, "FETCH_SIZE")
    write = _counter_rows(write_dir, "WRITE_SIZE")
    gib_kib = float(1 << 20)

    def calib(rows, pick):
        vals = [v for k, lst in rows.items() if pick(k) for _, v in lst if v > 0.5 * gib_kib]
        if not vals:
            raise SystemExit("calibration kernel not found in the counter output")
        return gib_kib / max(vals)

    fs = calib(fetch, lambda k: "copyBuffer" in k or "copy" in k.lower())
    ws = calib(write, lambda k: "fill" in k.lower())
    table = []   # per kernel and grid
    for k in sorted(set(fetch) | set(write)):
        if "rsz::" not in k:
            continue
        for g in sorted({g for g, _ in fetch.get(k, []) + write.get(k, [])}):
            f = [v for gg, v in fetch.get(k, []) if gg == g]
            w = [v for gg, v in write.get(k, []) if gg == g]
            fk = sum(f) / max(1, len(f))
            wk = sum(w) / max(1, len(w))
            table.append((k, g, len(f), fk, fk * 1024 * fs, wk, wk * 1024 * ws))
    os.makedirs(out_dir, exist_ok=True)
    for rec_name, match, source in TRAFFIC_KERNELS:
        names = [k for k in set(fetch) & set(write) if match in k]
        if not names:
            continue
        fl = [t for k in names for t in fetch[k]]
        wl = [t for k in names for t in write[k]]
        top = max(g for g, _ in fl)
        fv = [v for g, v in fl if g == top]
        wv = [v for g, v in wl if g == top]
        fb = sum(fv) / len(fv) * 1024 * fs
        wb = sum(wv) / len(wv) * 1024 * ws
        rec = {"kernel": rec_name, "counter_name": names[0], "workload": WORKLOAD,
               "grid": top, "dispatches": len(fv), "source": source,
               "source_sha256": _source_sha(source),
               "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
               "fetch_bytes_per_launch": round(fb), "write_bytes_per_launch": round(wb),
               "hbm_bytes_per_launch": round(fb + wb)}
        with open(os.path.join(out_dir, f"{rec_name}_{WORKLOAD}_traffic.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec))
    lines = [f"fetch scale {fs:.4f} (1 GiB copy), write scale {ws:.4f} (1 GiB fill)", "",
             "| kernel | grid (work-items) | dispatches | FETCH_SIZE KiB/dispatch | read GB "
             "| WRITE_SIZE KiB/dispatch | written GB |", "|---|---|---|---|---|---|---|"]
    for k, g, nf, fk, fb, wk, wb in sorted(table, key=lambda t: -t[4]):
        lines.append(f"| `{k[:56]}` | {g} | {nf} | {fk:.0f} | {fb / 1e9:.3f} | {wk:.0f} | "
                     f"{wb / 1e9:.3f} |")
    with open(os.path.join(out_dir, f"{WORKLOAD}_traffic_table.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def traffic_record(kernel):
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{WORKLOAD}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = rec.get("source")
    if not src or rec.get("source_sha256") != _source_sha(src):
        return None
    return rec


def launch_modes(torch, B, steps):
    """The same batch as prepared once (rsz_batch_prepare) and then queued
    as kernels only (rsz_batch_launch), and as a HIP graph replay of that
    launch: ms a step of each, beside the per-step plan of `value`.  Every
    replay still recomputes every stream from the frames' contents."""
    out = {}
    B.prepare()
    for name, fn in (("prepared_launch", B.launch), ("graph_replay", None)):
        if fn is None:
            B.graph()
            fn = B.replay
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        out[name + "_ms"] = round((time.perf_counter() - t0) * 1e3 / steps, 4)
    st = B.status.cpu().numpy()
    assert (st == 0).all(), f"launch modes: statuses {set(st.tolist())}"
    return out


def _child_processes():
    """Processes this one has started that are still alive."""
    try:
        import psutil
        return len(psutil.Process().children(recursive=True))
    except Exception:
        return None


def _path_roofline(raw_bytes, out_bytes, el, kms):
    """Whole-path and dominant-kernel roofline figures of one line: the path
    must at least read every raw frame byte and write every stream byte once
    (4 + s bytes a pixel, s the output bytes a pixel); k_bin reads the raw
    frames once."""
    path_bytes = raw_bytes + out_bytes
    out = {"path_achieved_gbps": round(path_bytes / el / 1e9, 1),
           "path_frac": round(path_bytes / el / 1e9 / 8000.0, 4),
           "out_bytes_per_pixel": round(4.0 * out_bytes / raw_bytes, 5)}
    kb = kms.get("k_bin")
    if kb:
        out["k_bin_frac"] = round(raw_bytes / (kb * 1e-3) / 1e9 / 8000.0, 4)
    return out


def _line(torch, B, steps, raw_bytes, label):
    """Timed steps of batch B (already warmed up and checked): GB/s,
    roofline fractions, compression ratio and per-kernel times."""
    import numpy as np
    el, kms = timed_steps(torch, B, steps)
    sizes = B.sizes.cpu().numpy().astype(np.int64)
    out = {"value": round(raw_bytes / el / 1e9, 2), "unit": "GB/s",
           "ms_per_step": round(el * 1e3, 4), "steps": steps,
           "compression_ratio_u16_aggregate": round(float(raw_bytes / 2 / sizes.sum()), 3)}
    out.update(_path_roofline(raw_bytes, int(sizes.sum()), el, kms))
    out["kernel_ms"] = kms
    print(f"[bench] {label}: {out['value']} GB/s, path {out['path_frac']}, k_bin "
          f"{out.get('k_bin_frac')}, CR {out['compression_ratio_u16_aggregate']}",
          file=sys.stderr, flush=True)
    return out


def _warm(torch, B, label, n=2, launch=None):
    for _ in range(n):
        (launch or B.run)()
    torch.cuda.synchronize()
    st = B.status.cpu().numpy()
    assert (st == 0).all(), f"{label}: statuses {set(st.tolist())}"


def cspad_bounds_section(args, torch, frames, peaks, knobs, raw_bytes):
    """The 1000-frame CSPAD batch at the other error bounds (1, 5, 20 ADU),
    one batched launch a step."""
    from paper_2206_11297_amd import rsz
    out = {}
    for eb in (1.0, 5.0, 20.0):
        B = rsz.Batch(frames, peaks, (WINDOW, BIN, eb, rsz.RSZ_BIN_BACKGROUND), **knobs)
        _warm(torch, B, f"cspad eb {eb:g}")
        out[f"cspad-batch-{len(frames)}_eb{eb:g}"] = _line(torch, B, args.config_steps, raw_bytes,
                                                           f"cspad eb {eb:g}")
        del B
        torch.cuda.empty_cache()
    return out


def jungfrau4m_section(args, torch, dev):
    """Batches of Jungfrau-4M-like frames (8x512x1024 f32, 20-800 peaks) at
    window {11, 25} x bin {2, 4}, eb 10 ADU, each with the autotuned tile
    shape and waves per workgroup."""
    from paper_2206_11297_amd import autotune, rsz, synth
    n = args.jf4m_frames
    host = generate(lambda i: synth.jungfrau_frame(i, workload=synth.W_JF), n, args.workers)
    frames = [torch.from_numpy(f).to(dev) for f, _ in host]
    peaks = [torch.from_numpy(p).to(dev) for _, p in host]
    del host
    raw_bytes = sum(f.numel() * 4 for f in frames)
    out = {}
    for w in (11, 25):
        for b in (2, 4):
            prm = (w, b, 10.0, rsz.RSZ_BIN_BACKGROUND)
            label = f"jungfrau4m-{n}_w{w}_b{b}"
            t = autotune.tune(frames, peaks, prm, reps=3, budget_s=args.config_autotune_seconds)
            knobs = dict(zip(("tile_rows", "tile_strips", "tile_waves"), t["best"]))
            B = rsz.Batch(frames, peaks, prm, **knobs)
            _warm(torch, B, label)
            out[label] = _line(torch, B, args.config_steps, raw_bytes, label)
            out[label]["tile"] = {"best": list(t["best"]), "from_table": bool(t.get("cached")),
                                  "autotuned": not t.get("cached"),
                                  "default_ms": t.get("default_ms"), "ms": t.get("ms")}
            del B
            torch.cuda.empty_cache()
    del frames, peaks
    torch.cuda.empty_cache()
    return out


def jungfrau16m_graph_section(args, torch, dev):
    """Batches of Jungfrau-16M-like frames (16x512x1024 f32, 0-3000 peaks),
    window 11, bin 2, eb 1 and 10 ADU: the prepared batch captured in a HIP
    graph and replayed, each replay recomputing every stream; the same
    streams decoded in one batched call; and the graph of compression
    followed by the on-device verification stage (rsz_verify_*)."""
    import numpy as np
    from paper_2206_11297_amd import autotune, rsz, synth
    n = args.jf16m_frames
    host = generate(lambda i: synth.jungfrau_frame(i, shape=synth.JUNGFRAU16M,
                                                   workload=synth.W_JF16, max_peaks=3000),
                    n, args.workers)
    frames = [torch.from_numpy(f).to(dev) for f, _ in host]
    peaks = [torch.from_numpy(p).to(dev) for _, p in host]
    del host
    raw_bytes = sum(f.numel() * 4 for f in frames)
    out = {}
    for eb in (1.0, 10.0):
        label = f"jungfrau16m-{n}_graph_eb{eb:g}"
        prm = (11, 2, eb, rsz.RSZ_BIN_BACKGROUND)
        t = autotune.tune(frames, peaks, prm, reps=3, budget_s=args.config_autotune_seconds)
        B = rsz.Batch(frames, peaks, prm, *t["best"])
        B.prepare()
        B.graph()
        _warm(torch, B, label, launch=B.replay)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.config_steps):
            B.replay()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / args.config_steps
        rsz.rsz_profile_enable(True)
        for _ in range(2):
            B.launch()
        torch.cuda.synchronize()
        kms = {k: round(v[1] / v[0], 4) for k, v in rsz.rsz_profile_read().items()}
        rsz.rsz_profile_enable(False)
        sizes = B.sizes.cpu().numpy().astype(np.int64)
        line = {"value": round(raw_bytes / el / 1e9, 2), "unit": "GB/s",
                "ms_per_step": round(el * 1e3, 4), "steps": args.config_steps,
                "mode": "graph replay",
                "compression_ratio_u16_aggregate": round(float(raw_bytes / 2 / sizes.sum()), 3)}
        line.update(_path_roofline(raw_bytes, int(sizes.sum()), el, kms))
        line["kernel_ms"] = kms
        line["kernel_ms_source"] = "HIP events around every launch of 2 eager launches"
        line["tile"] = {"best": list(t["best"]), "from_table": bool(t.get("cached")),
                        "autotuned": not t.get("cached")}
        line["decompress_batched"] = batched_decode(torch, B, sizes, 3, raw_bytes)
        # the same batch with the verification stage in its graph: every
        # stream decoded and every pixel checked on the device
        V = rsz.Verify(B)
        V.graph()
        V.replay()
        torch.cuda.synchronize()
        bad = V.bad_counts()
        assert not any(bad), f"{label}: verification failed on {sum(1 for v in bad if v)} frames"
        t0 = time.perf_counter()
        for _ in range(max(1, args.config_steps // 2)):
            V.replay()
        torch.cuda.synchronize()
        el_v = (time.perf_counter() - t0) / max(1, args.config_steps // 2)
        line["with_verification"] = {
            "ms_per_step": round(el_v * 1e3, 4), "value": round(raw_bytes / el_v / 1e9, 2),
            "unit": "GB/s", "frames_verified": len(bad),
            "note": "one graph: compression, then every stream decoded on the device and every "
                    "pixel checked against its frame (ROI bit-exact, background within eb of its "
                    "bin mean)"}
        del V
        print(f"[bench] {label}: {line['value']} GB/s, path {line['path_frac']}, k_bin "
              f"{line.get('k_bin_frac')}, CR {line['compression_ratio_u16_aggregate']}; batched "
              f"decompression {line['decompress_batched']['gbps']} GB/s; with on-device "
              f"verification {line['with_verification']['ms_per_step']} ms a step",
              file=sys.stderr, flush=True)
        out[label] = line
        del B
        torch.cuda.empty_cache()
    del frames, peaks
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=NFRAMES)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="oracle time budget (half single-thread, half frame-parallel)")
    ap.add_argument("--cpu-threads", type=int, default=16)
    ap.add_argument("--autotune-seconds", type=float, default=20.0,
                    help="time budget of the tile-shape autotuner when the shipped table "
                         "has no entry for this workload (0: library default shape)")
    ap.add_argument("--tune-store", default=None,
                    help="JSON file that receives a new autotuner result")
    ap.add_argument("--traffic-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_DIR"),
                    help="summarize two rocprofv3 --pmc runs (CSV output) and exit")
    ap.add_argument("--counter-summary", nargs="+", metavar="PATH",
                    help="summarize rocprofv3 --pmc runs of the SQ counters (CSV output under "
                         "the given directories) into the Markdown file named last, and exit")
    ap.add_argument("--latency-frames", type=int, default=200)
    ap.add_argument("--read-reference", type=int, default=1,
                    help="time a plain 4 GiB streaming read as the measured read reference")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--decompress-frames", type=int, default=200,
                    help="frames decompressed one per call for the decompression figures")
    ap.add_argument("--decompress-steps", type=int, default=10,
                    help="timed batched decompressions of the whole batch")
    ap.add_argument("--serve-rates", type=float, nargs="*", default=[1.0, 2.0, 5.0, 10.0],
                    help="Poisson arrival rates in kHz for the serving section ([] skips it)")
    ap.add_argument("--serve-frames", type=int, default=10000)
    ap.add_argument("--serve-pool", type=int, default=24)
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--serve-batch", type=int, default=32)
    ap.add_argument("--dims", type=int, nargs="*", default=[1, 3],
                    help="Lorenzo dimensions timed besides 2 on the same batch")
    ap.add_argument("--dims-steps", type=int, default=10)
    ap.add_argument("--roi-steps", type=int, default=10,
                    help="steps of the ROI-coding section (0: skip it)")
    ap.add_argument("--run-steps", type=int, default=10,
                    help="steps of the run-coding sections, alone and with the ROI coded "
                         "(0: skip them)")
    ap.add_argument("--peaks-steps", type=int, default=10,
                    help="steps of the peak-finding section (0: skip it)")
    ap.add_argument("--config-steps", type=int, default=10,
                    help="steps of each line of the other workloads: the CSPAD batch at eb "
                         "1/5/20, Jungfrau-4M batches over window x bin, the Jungfrau-16M "
                         "graph replays (0: skip them)")
    ap.add_argument("--jf4m-frames", type=int, default=256)
    ap.add_argument("--jf16m-frames", type=int, default=512)
    ap.add_argument("--config-autotune-seconds", type=float, default=6.0,
                    help="autotuner budget per Jungfrau-4M line when the shipped table has "
                         "no entry for it")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    if args.counter_summary:
        counter_summary(args.counter_summary[:-1], args.counter_summary[-1])
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the compression path is not sharded across "
              "GPUs (frames are independent, so several GPUs would each run their own "
              "batches).", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    # frames are drawn before the GPU is touched (threads; nothing is forked)
    t0 = time.time()
    host = generate(_gen, args.frames, args.workers)
    serve_pool = generate(_gen_pool, args.serve_pool, args.workers) if args.serve_rates else None
    gen_s = time.time() - t0
    print(f"[bench] generated {len(host)} frames in {gen_s:.1f}s", file=sys.stderr, flush=True)

    import torch
    from paper_2206_11297_amd import rsz

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    frames = [torch.from_numpy(f).to(dev) for f, _ in host]
    peaks = [torch.from_numpy(p).to(dev) for _, p in host]
    torch.cuda.synchronize()
    prm = (WINDOW, BIN, EB, rsz.RSZ_BIN_BACKGROUND)
    tile = None
    if args.autotune_seconds > 0:
        from paper_2206_11297_amd import autotune
        tile = autotune.tune(frames, peaks, prm, reps=3, budget_s=args.autotune_seconds,
                             store_path=args.tune_store)
        print(f"[bench] autotune: best tile {tile['best']} {tile['ms']} ms "
              f"(default {tile['default_ms']} ms, {len(tile['table'])} shapes)",
              file=sys.stderr, flush=True)
    tile_rows, tile_strips, tile_waves = (list(tile["best"]) + [0])[:3] if tile else (0, 0, 0)
    knobs = dict(tile_rows=tile_rows, tile_strips=tile_strips, tile_waves=tile_waves)
    B = rsz.Batch(frames, peaks, prm, **knobs)
    raw_bytes = sum(f.numel() * 4 for f in frames)
    npix = raw_bytes // 4

    read_ref = None
    if args.read_reference:
        # a plain streaming read of 4 GiB resident in HBM on this machine (the
        # reference the kernel's read rate is compared with)
        read_ref = rsz.measure_read(1 << 32, reps=10)
        torch.cuda.empty_cache()

    if args.copy_calibration:
        # plain copy of a known size: 1 GiB read + 1 GiB written
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        B.run()
    torch.cuda.synchronize()
    st = B.status.cpu().numpy()
    assert (st == 0).all(), f"compression failed: statuses {set(st.tolist())}"

    # the timed region records HIP events around the binning kernel only (the
    # roofline's launch time); every kernel's time comes from a profiled pass
    # after it
    rsz.rsz_profile_only("k_bin")
    rsz.rsz_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = rsz.rsz_profile_read()
    rsz.rsz_profile_enable(False)
    rsz.rsz_profile_only(None)
    ms_step = elapsed * 1e3 / args.steps
    gbps = raw_bytes / (elapsed / args.steps) / 1e9
    kprof_steps = max(1, min(args.steps, 5))
    rsz.rsz_profile_enable(True)
    for _ in range(kprof_steps):
        B.run()
    torch.cuda.synchronize()
    prof_all = rsz.rsz_profile_read()
    rsz.rsz_profile_enable(False)

    sizes = B.sizes.cpu().numpy().astype(np.int64)
    modes = launch_modes(torch, B, args.steps)
    modes["plan_each_step_ms"] = round(ms_step, 4)
    modes["note"] = ("value times plan_each_step: each step plans the batch on the host and "
                     "uploads the plan, as a stream of new batches would")
    cr_u16 = (npix // len(frames)) * 2 / sizes
    kernel_ms = {k: v[1] / v[0] for k, v in prof_all.items()}
    kb_ms = prof["k_bin"][1] / prof["k_bin"][0]
    achieved = raw_bytes / (kb_ms * 1e-3) / 1e9
    tr = traffic_record("k_bin")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
            "frac": round(achieved / 8000.0, 4),
            "measured_read_reference_gbps": None if read_ref is None else round(read_ref, 1),
            "frac_of_measured_read": None if read_ref is None else round(achieved / read_ref, 4),
            "traffic": None if tr is None else tr["hbm_bytes_per_launch"],
            "kernel": "k_bin", "algorithmic_bytes_per_launch": raw_bytes,
            "avg_launch_ms": round(kb_ms, 4)}
    # the whole path against the least traffic it needs: every raw byte read
    # and every stream byte written once, in the timed step time
    path = _path_roofline(raw_bytes, int(sizes.sum()), elapsed / args.steps, {})
    roof["path_frac"] = path["path_frac"]
    roof["path_achieved_gbps"] = path["path_achieved_gbps"]
    roof["path_bytes_per_step"] = raw_bytes + int(sizes.sum())

    # one-frame-per-launch latency at the same bound (synchronous calls)
    lat = []
    p1 = rsz.params(*SHAPE, WINDOW, BIN, EB)
    stc, cap = rsz.rsz_max_compressed_bytes(p1, 1000)
    out1 = torch.empty(cap, dtype=torch.uint8, device=dev)
    ws1 = rsz.workspace(rsz.rsz_workspace_bytes(p1, 1000)[1], dev)
    s = rsz._stream()
    for i in range(min(args.latency_frames, len(frames))):
        pk = peaks[i]
        npk = pk.shape[0]
        a = time.perf_counter()
        st1, n1 = rsz.rsz_compress(p1, rsz._ptr(frames[i]), rsz._ptr(pk) if npk else None, npk,
                                   rsz._ptr(out1), cap, rsz._ptr(ws1), ws1.numel(), s)
        lat.append(time.perf_counter() - a)
        assert st1 == 0 and n1 == sizes[i]
    lat_ms = np.array(lat if lat else [float("nan")]) * 1e3

    # CPU baseline: the oracle as it is, first on one thread, then one frame
    # per thread on the host's cores (the C library runs without the GIL),
    # each for a bounded time; its streams must equal the GPU streams byte
    # for byte
    cpu = cpu_baseline(args, host, B, sizes)

    decomp = decompress_section(args, torch, dev, B, sizes, host) if args.decompress_frames else None
    serving = serving_section(args, torch, dev, serve_pool) if args.serve_rates else None
    dims = lorenzo_dims_section(args, torch, frames, peaks, prm, knobs,
                                raw_bytes) if args.dims else None
    roi = coding_section(args, torch, frames, peaks, prm, raw_bytes, knobs, 1, 0,
                         args.roi_steps, "roi coding") if args.roi_steps else None
    runs = coding_section(args, torch, frames, peaks, prm, raw_bytes, knobs, 0,
                          1, args.run_steps, "run coding") if args.run_steps else None
    both = coding_section(args, torch, frames, peaks, prm, raw_bytes, knobs, 1,
                          1, args.run_steps, "roi + run coding") if args.run_steps else None
    pk = peaks_section(args, torch, frames, prm, raw_bytes, knobs) if args.peaks_steps else None
    nfr = len(frames)
    cfg = cspad_bounds_section(args, torch, frames, peaks, knobs, raw_bytes) \
        if args.config_steps else None
    if cfg is not None:
        # the larger workloads need the CSPAD batch's memory
        del B, frames, peaks
        torch.cuda.empty_cache()
        cfg.update(jungfrau4m_section(args, torch, dev))
        cfg.update(jungfrau16m_graph_section(args, torch, dev))

    line = {
        "metric": "raw-frame GB/s compressed (1 GPU) at eb=10 ADU; compression ratio; "
                  "p99 frame latency",
        "value": round(gbps, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{WORKLOAD}-{nfr}: {nfr} frames "
                               f"{SHAPE[0]}x{SHAPE[1]}x{SHAPE[2]} f32, Poisson(60) peaks, "
                               "20% non-hit, window 17, bin 2x2, eb 10 ADU, one batched launch",
                   "frames": nfr, "raw_bytes": raw_bytes,
                   "tile": {"rows": tile_rows, "strips": tile_strips, "waves": tile_waves,
                            "autotuned": bool(tile and not tile.get("cached")),
                            "from_table": bool(tile and tile.get("cached")),
                            "default_ms": tile["default_ms"] if tile else None,
                            "shapes_timed": len(tile["table"]) if tile else 0}},
        "roofline": roof,
        "cpu_baseline": cpu,
        "compression_ratio_u16": {"mean": round(float(cr_u16.mean()), 3),
                                  "min": round(float(cr_u16.min()), 3),
                                  "max": round(float(cr_u16.max()), 3),
                                  "aggregate": round(float(npix * 2 / sizes.sum()), 3)},
        "compression_ratio_f32_aggregate": round(float(npix * 4 / sizes.sum()), 3),
        "latency_ms": {"one_frame_per_launch_p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "one_frame_per_launch_p99": round(float(np.percentile(lat_ms, 99)), 4),
                       "batched_all_frames": round(ms_step, 4)},
        "kernel_ms": {k: round(v, 4) for k, v in kernel_ms.items()},
        "launch_modes": modes,
        "kernel_ms_source": f"HIP events around every launch in {kprof_steps} steps after the "
                            "timed region (inside it, events around k_bin only)",
        "serving": serving,
        "decompress": decomp,
        "lorenzo_dims": dims,
        "roi_coding": roi,
        "run_coding": runs,
        "roi_and_run_coding": both,
        "peak_finding": pk,
        "configs": cfg,
    }
    if serving:
        top = serving.get(f"{max(args.serve_rates):g}kHz")
        if top:
            line["latency_ms"]["serving_p50"] = top["continuous_batching"]["p50_ms"]
            line["latency_ms"]["serving_p99"] = top["continuous_batching"]["p99_ms"]
            line["latency_ms"]["serving_rate_khz"] = max(args.serve_rates)
    line["procs_at_end"] = _child_processes()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
