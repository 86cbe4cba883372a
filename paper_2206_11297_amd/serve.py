"""Continuous-batching serving loop for per-frame compression.

Frames arrive from a (simulated) detector stream at given times.  Pending
frames are admitted into free slots as soon as a slot is idle: each slot owns a
HIP stream, a workspace and an output arena sized once from an HBM budget, so
admission is bounded by memory and never allocates.  Batches on different
slots overlap on the device; a frame's latency is the time from its arrival to
the completion of the batch that carried it.

The scheduler is independent of the GPU: an executor supplies launch / poll /
finish.  `GpuExecutor` drives librsz through rsz_compress_batch on one stream
per slot and timestamps completions with HIP events; tests also run the same
scheduler against a CPU executor.
"""
import collections
import dataclasses
import gc
import time
from typing import Callable, List, Optional, Sequence


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds since the start of the run
    frame: object           # float32 [P,H,W] device tensor (GPU executor)
    peaks: object           # int32 [n,3] device tensor
    params: tuple           # (window, bin, eb, bin_mode[, dim])
    out_cap: int = 0        # worst-case stream bytes (set by the executor)
    ws_bytes: int = 0       # workspace share (bound used by admission, set by the executor)
    raw_bytes: int = 0


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    start: float            # launch time of its batch
    done: float             # completion time of its batch
    status: int
    nbytes: int
    batch: int              # batch sequence number
    slot: int
    stream: Optional[object] = None   # compressed bytes (when kept)

    @property
    def latency(self):
        return self.done - self.arrival


@dataclasses.dataclass
class SlotLimits:
    max_frames: int
    out_bytes: int
    ws_bytes: int


class Scheduler:
    """Continuous batching over `nslots` slots.

    Admission: requests are taken in arrival order into the next free slot
    while the batch stays within the slot's frame count, output arena and
    workspace (`fits(batch)` of the executor).  A request that cannot fit an
    empty slot is rejected with status -1."""

    def __init__(self, executor, nslots: int, limits: SlotLimits,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.nslots = nslots
        self.limits = limits
        self.clock = clock

    def _form_batch(self, pending):
        # running sums of each request's own bound keep admission O(batch);
        # one exact check of the formed batch follows
        lim = self.limits
        batch, out, ws = [], 0, 0
        while pending and len(batch) < lim.max_frames:
            r = pending[0]
            if out + r.out_cap > lim.out_bytes or ws + r.ws_bytes > lim.ws_bytes:
                break
            out += r.out_cap
            ws += r.ws_bytes
            batch.append(pending.popleft())
        while batch and not self.ex.fits(batch, lim):
            pending.appendleft(batch.pop())
        return batch

    def run(self, requests: Sequence[Request], keep_streams=False) -> List[Result]:
        # Python's cyclic garbage collector stays off while the loop runs: a
        # full collection over the run's request and result objects takes
        # tens of milliseconds, which would land on some frame's latency.
        gc_was_on = gc.isenabled()
        gc.disable()
        try:
            return self._run(requests, keep_streams)
        finally:
            if gc_was_on:
                gc.enable()

    def _run(self, requests: Sequence[Request], keep_streams=False) -> List[Result]:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in reqs:
            self.ex.size_request(r)
        pending = collections.deque()
        free = list(range(self.nslots))
        inflight = {}
        results = []
        nb = 0
        i = 0
        t0 = self.clock()
        self.ex.start()
        while len(results) < len(reqs):
            now = self.clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                pending.append(reqs[i])
                i += 1
            progressed = False
            while free and pending:
                slot = free[0]
                batch = self._form_batch(pending)
                if not batch:
                    r = pending.popleft()   # does not fit an empty slot
                    results.append(Result(r.rid, r.arrival, now, now, -1, 0, -1, -1))
                    progressed = True
                    continue
                free.pop(0)
                handle = self.ex.launch(slot, batch, now)
                inflight[slot] = (batch, handle, nb)
                nb += 1
                progressed = True
            for slot in list(inflight):
                batch, handle, bn = inflight[slot]
                if self.ex.done(handle):
                    st, sizes, start, done, streams = self.ex.finish(slot, handle, batch,
                                                                     keep_streams)
                    for k, r in enumerate(batch):
                        results.append(Result(r.rid, r.arrival, start, done, int(st[k]),
                                              int(sizes[k]), bn, slot,
                                              streams[k] if streams else None))
                    del inflight[slot]
                    free.append(slot)
                    free.sort()
                    progressed = True
            if not progressed:
                self.ex.idle(pending, inflight, reqs[i].arrival - now if i < len(reqs) else None)
        results.sort(key=lambda r: r.rid)
        return results


class GpuExecutor:
    """Slots on the GPU: one HIP stream, workspace and output arena each."""

    def __init__(self, nslots: int, limits: SlotLimits, device=None):
        import torch
        from . import rsz
        self.torch, self.rsz = torch, rsz
        self.dev = device or torch.device("cuda:0")
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(nslots)]
        self.ws = [torch.empty(limits.ws_bytes, dtype=torch.uint8, device=self.dev)
                   for _ in range(nslots)]
        self.out = [torch.empty(limits.out_bytes, dtype=torch.uint8, device=self.dev)
                    for _ in range(nslots)]
        self.sizes = [torch.zeros(limits.max_frames, dtype=torch.int64, device=self.dev)
                      for _ in range(nslots)]
        self.status = [torch.zeros(limits.max_frames, dtype=torch.int32, device=self.dev)
                       for _ in range(nslots)]
        self.limits = limits
        self.t_start = None

    def size_request(self, r: Request):
        rsz = self.rsz
        P, H, W = r.frame.shape
        p = rsz.params(P, H, W, *r.params)
        npk = r.peaks.shape[0]
        st, cap = rsz.rsz_max_compressed_bytes(p, npk)
        if st:
            raise rsz.RszError(st, "rsz_max_compressed_bytes")
        r.out_cap = (cap + 255) // 256 * 256
        r.raw_bytes = P * H * W * 4
        # workspace share: the larger of the frame alone and its per-frame
        # share in a large batch (the tiling, hence the layout, differs)
        d1, _ = self._descs(0, [r])
        st1, w1 = rsz.rsz_batch_workspace_bytes(d1)
        st16, w16 = rsz.rsz_batch_workspace_bytes(d1 * 16)
        if st1 or st16:
            raise rsz.RszError(st1 or st16, "rsz_batch_workspace_bytes")
        r.ws_bytes = max(w1, -(-w16 // 16)) + 4096

    def _descs(self, slot, batch):
        rsz = self.rsz
        descs, off = [], 0
        base = self.out[slot].data_ptr()
        for r in batch:
            P, H, W = r.frame.shape
            d = rsz.rsz_frame_desc()
            d.params = rsz.params(P, H, W, *r.params)
            d.frame = r.frame.data_ptr()
            d.peaks = r.peaks.data_ptr() if r.peaks.shape[0] else None
            d.npeaks = r.peaks.shape[0]
            d.tile_rows = 0
            d.out = base + off
            d.out_cap = r.out_cap
            off += r.out_cap
            descs.append(d)
        return descs, off

    def fits(self, batch, limits: SlotLimits):
        descs, out_total = self._descs(0, batch)
        if out_total > limits.out_bytes:
            return False
        st, need = self.rsz.rsz_batch_workspace_bytes(descs)
        return st == 0 and need <= limits.ws_bytes

    def start(self):
        torch = self.torch
        self.t_start = torch.cuda.Event(enable_timing=True)
        self.t_start.record(self.streams[0])
        self.host_t0 = time.perf_counter()
        for s in self.streams[1:]:
            s.wait_stream(self.streams[0])

    def launch(self, slot, batch, now):
        rsz, torch = self.rsz, self.torch
        descs, _ = self._descs(slot, batch)
        s = self.streams[slot]
        a = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        a.record(s)
        st = rsz.rsz_compress_batch(descs, rsz._ptr(self.sizes[slot]), rsz._ptr(self.status[slot]),
                                    rsz._ptr(self.ws[slot]), self.ws[slot].numel(),
                                    rsz.C.c_void_p(s.cuda_stream))
        if st:
            raise rsz.RszError(st, "rsz_compress_batch")
        e.record(s)
        return (a, e, now)

    def done(self, handle):
        return handle[1].query()

    def finish(self, slot, handle, batch, keep_streams):
        a, e, now = handle
        n = len(batch)
        st = self.status[slot][:n].cpu().numpy()
        sizes = self.sizes[slot][:n].cpu().numpy()
        start_ms = self.t_start.elapsed_time(a)
        done_ms = self.t_start.elapsed_time(e)
        streams = None
        if keep_streams:
            streams, off = [], 0
            for k, r in enumerate(batch):
                streams.append(self.out[slot][off:off + int(sizes[k])].cpu().numpy())
                off += r.out_cap
        return st, sizes, start_ms / 1e3, done_ms / 1e3, streams

    def idle(self, pending, inflight, until_next):
        # nothing launched or finished: yield briefly (keeps polling latency low)
        if until_next is not None and until_next > 2e-4 and not inflight:
            time.sleep(min(until_next, 1e-3) * 0.5)


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if len(xs) else float("nan")


def summarize(results: List[Result], requests: Sequence[Request]):
    ok = [r for r in results if r.status == 0]
    lat = [r.latency * 1e3 for r in ok]
    raw = {q.rid: q.raw_bytes for q in requests}
    tot_raw = sum(raw[r.rid] for r in ok)
    tot_out = sum(r.nbytes for r in ok)
    t_first = min(q.arrival for q in requests)
    t_last = max(r.done for r in ok) if ok else t_first
    span = max(t_last - t_first, 1e-9)
    batches = {(r.slot, r.batch) for r in ok}
    return {"frames": len(results), "ok": len(ok),
            "p50_ms": round(percentile(lat, 50), 4), "p99_ms": round(percentile(lat, 99), 4),
            "max_ms": round(max(lat), 4) if lat else None,
            "gbps": round(tot_raw / span / 1e9, 2),
            "cr_u16": round(tot_raw / 2 / tot_out, 3) if tot_out else None,
            "batches": len(batches),
            "mean_batch": round(len(ok) / max(1, len(batches)), 2)}
