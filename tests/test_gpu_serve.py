"""Continuous batching on the GPU: requests of three detector geometries and
three error bounds arrive while earlier batches run; every stream equals the
oracle's stream of the same frame compressed alone."""
import numpy as np
import pytest

from oracle import rsz_oracle as O
from paper_2206_11297_amd import serve, synth

pytestmark = pytest.mark.gpu


def test_served_streams_equal_frames_alone():
    import torch
    assert torch.cuda.is_available()
    pool = [synth.cspad_frame(11, npeaks=40), synth.jungfrau_frame(6, npeaks=200),
            synth.jungfrau_frame(7, shape=(1, 2048, 2048), npeaks=100),
            synth.tiny_case(60, (3, 50, 90), 4, "normal")]
    dev = torch.device("cuda:0")
    gpool = [(torch.from_numpy(f).to(dev), torch.from_numpy(p).to(dev)) for f, p in pool]
    rng = np.random.default_rng(12)
    t = np.cumsum(rng.exponential(1e-4, 48))
    reqs = []
    for i in range(48):
        k = int(rng.integers(0, len(pool)))
        eb = float([5.0, 10.0, 20.0][int(rng.integers(0, 3))])
        reqs.append(serve.Request(i, float(t[i]), gpool[k][0], gpool[k][1], (17, 2, eb, 0)))
        reqs[-1].pool = k
    limits = serve.SlotLimits(max_frames=8, out_bytes=160 << 20, ws_bytes=160 << 20)
    ex = serve.GpuExecutor(3, limits, dev)
    res = serve.Scheduler(ex, 3, limits).run(reqs, keep_streams=True)
    torch.cuda.synchronize()
    cache = {}
    for r, q in zip(res, reqs):
        assert r.status == 0, (r.rid, r.status)
        key = (q.pool, q.params[2])
        if key not in cache:
            f, pk = pool[q.pool]
            st, ref, _ = O.compress(O.params(*f.shape, 17, 2, q.params[2], 0), f, pk)
            cache[key] = ref
        np.testing.assert_array_equal(r.stream, cache[key])
    s = serve.summarize(res, reqs)
    assert s["ok"] == 48 and s["p99_ms"] > 0
    print(s, flush=True)
