"""Autotuner for the binning kernel's tile shape and block schedule.

The binning kernel walks tiles of `tile_rows` bin rows x `tile_strips`
64-column strips per wave, `tile_waves` waves (tiles of consecutive row
segments) per workgroup (rsz_frame_desc).  Taller tiles re-read fewer halo
rows; shorter and narrower ones give a batch more waves, which small batches
need to fill the chip; the waves per workgroup set how a panel's rows split
into segments and how many tiles share a workgroup's LDS.  The tuner times
the batched compression of one batch for each candidate, checks that every
candidate writes the same streams as the library default (the knobs may
change speed only, as the thread-count tuning of the paper's Sec. V-C
"Autotuning Configuration" leaves the output unchanged), and returns the
fastest.  Results are cached in a JSON table keyed by the batch signature
(frame shapes, bin factors, windows and a power-of-two bucket of the frame
count).
"""
import json
import os
import time

from . import rsz

ROWS = (0, 4, 8, 12, 16, 24, 32)
STRIPS = (0, 1, 2, 4)
WAVES = (0, 2, 3)   # 0: the library default (4)
CANDIDATES = [(r, s, w) for w in WAVES for r in ROWS for s in STRIPS]


def _knobs(c):
    """(rows, strips, waves) of a candidate or stored entry (older tables
    hold (rows, strips))."""
    c = list(c)
    return (int(c[0]), int(c[1]), int(c[2]) if len(c) > 2 else 0)


def signature(frames, prm):
    """Key of a batch: its distinct (shape, window, bin[, Lorenzo dimension
    when not 2]) and frame-count bucket."""
    n = len(frames)
    prm = prm if isinstance(prm, list) else [prm] * n
    dims = lambda p: (int(p[4]),) if len(p) > 4 and int(p[4]) not in (0, 2) else ()
    kinds = sorted({(tuple(f.shape), int(p[0]), int(p[1])) + dims(p) for f, p in zip(frames, prm)})
    bucket = 1
    while bucket < n:
        bucket <<= 1
    return json.dumps({"kinds": kinds, "frames": bucket}, sort_keys=True)


def _time_batch(B, reps):
    torch = rsz._torch()
    B.run()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        B.run()
    e.record()
    torch.cuda.synchronize()
    return a.elapsed_time(e) / reps


def _same_streams(B, ref_sizes, ref):
    sizes = B.sizes.cpu().tolist()
    if sizes != ref_sizes:
        return False
    torch = rsz._torch()
    return all(torch.equal(B.stream(i, sizes), ref[i]) for i in range(len(sizes)))


TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_tiles.json")


def tune(frames, peaks, prm, candidates=None, reps=5, budget_s=30.0, cache_path=TABLE,
         store_path=None, log=None):
    """Times `candidates` (default: CANDIDATES, each (rows, strips, waves))
    on this batch; returns {"best": (rows, strips, waves), "ms": ...,
    "default_ms": ..., "table": [...], "cached": False}.  Candidates whose
    streams differ from the default's raise an error: the knobs must never
    change the output.  A result stored in cache_path (default: the table
    shipped with the package, tuned on MI355X) for the same signature is
    returned without timing, with "cached": True; store_path receives new
    results."""
    key = signature(frames, prm)
    if cache_path and os.path.exists(cache_path):
        table = json.load(open(cache_path))
        if key in table:
            out = dict(table[key], cached=True)
            out["best"] = list(_knobs(out["best"]))
            return out
    torch = rsz._torch()
    base = rsz.Batch(frames, peaks, prm)
    base.run()
    torch.cuda.synchronize()
    st = base.status.cpu().tolist()
    if any(st):
        raise rsz.RszError(max(st, key=abs), "autotune: the batch does not compress")
    ref_sizes = base.sizes.cpu().tolist()
    ref = [base.stream(i, ref_sizes).clone() for i in range(len(frames))]
    default_ms = _time_batch(base, reps)
    del base
    rows = []
    t0 = time.perf_counter()
    for c in candidates or CANDIDATES:
        if time.perf_counter() - t0 > budget_s:
            break
        r, s, w = _knobs(c)
        B = rsz.Batch(frames, peaks, prm, tile_rows=r, tile_strips=s, tile_waves=w)
        ms = _time_batch(B, reps)
        if not _same_streams(B, ref_sizes, ref):
            raise RuntimeError(f"autotune: tile shape ({r}, {s}, {w}) changed the output")
        rows.append((r, s, w, round(ms, 4)))
        if log:
            log(f"tile_rows={r} tile_strips={s} tile_waves={w}: {ms:.4f} ms")
        del B
    best = min(rows, key=lambda t: t[3]) if rows else (0, 0, 0, default_ms)
    out = {"best": [best[0], best[1], best[2]], "ms": best[3], "default_ms": round(default_ms, 4),
           "table": rows, "cached": False}
    if store_path:
        table = json.load(open(store_path)) if os.path.exists(store_path) else {}
        table[key] = {k: v for k, v in out.items() if k != "cached"}
        with open(store_path, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
    return out


def _workloads():
    """The standard seeded workloads: (name, frame generator, count, params)."""
    from . import synth
    counts = synth.batch_peak_counts(1000)
    cspad = lambda i: synth.batch_frame(i, counts)
    jf = lambda i: synth.jungfrau_frame(i, workload=synth.W_JF)
    sq = lambda i: synth.jungfrau_frame(i, shape=synth.SQUARE4M, npeaks=800, workload=synth.W_SERVE)
    jf16 = lambda i: synth.jungfrau_frame(i, shape=synth.JUNGFRAU16M, workload=synth.W_JF16,
                                          max_peaks=3000)
    out = [("cspad-batch-1000", cspad, 1000, [(17, 2, 10.0, 0)]),
           ("cspad-1", cspad, 1, [(17, 2, 10.0, 0)]),
           ("jungfrau4m-1", jf, 1, [(17, 2, 10.0, 0)]),
           ("jungfrau4m-32", jf, 32, [(17, 2, 10.0, 0)]),
           ("jungfrau4m-256", jf, 256, [(w, b, 10.0, 0) for w in (11, 25) for b in (2, 4)]),
           ("square2048-1", sq, 1, [(17, 2, 10.0, 0)]),
           ("square2048-32", sq, 32, [(17, 2, 10.0, 0)]),
           ("jungfrau16m-512", jf16, 512, [(11, 2, 1.0, 0), (11, 2, 10.0, 0)])]
    return out


def main(argv=None):
    """Tunes the standard workloads on this GPU and writes their entries to a
    JSON table (the package's table is written this way on MI355X)."""
    import argparse
    from concurrent.futures import ThreadPoolExecutor
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--out", required=True, help="JSON table to write (entries are merged)")
    ap.add_argument("--only", nargs="*", help="workload names to tune (default: all)")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    torch = rsz._torch()
    dev = torch.device("cuda:0")
    for name, gen, n, prms in _workloads():
        if args.only and name not in args.only:
            continue
        with ThreadPoolExecutor(16) as ex:
            host = list(ex.map(gen, range(n)))
        frames = [torch.from_numpy(f).to(dev) for f, _ in host]
        peaks = [torch.from_numpy(p).to(dev) for _, p in host]
        for prm in prms:
            r = tune(frames, peaks, prm, reps=args.reps, budget_s=120.0, cache_path=None,
                     store_path=args.out)
            print(f"[autotune] {name} {prm}: best {r['best']} {r['ms']} ms "
                  f"(default {r['default_ms']} ms)", flush=True)
        del frames, peaks, host
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
