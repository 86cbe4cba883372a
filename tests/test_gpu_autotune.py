"""The autotuner on the GPU: tune() over a small grid of tile rows x strips x
waves per workgroup, on a small mixed batch, with no table (cache_path=None).
Every candidate must write the streams of the library default (tune raises
otherwise), the best shape's streams must equal the oracle's, and a stored
result must come back from the table without timing ("cached")."""
import json

import numpy as np
import pytest

from oracle import rsz_oracle as O
from paper_2206_11297_amd import autotune, rsz, synth

pytestmark = pytest.mark.gpu

GRID = [(r, s, w) for w in (0, 1, 2, 3) for r in (0, 4, 12) for s in (0, 1, 4)]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    rsz.lib()
    return t


def test_tune_small_grid_keeps_the_bytes(torch, tmp_path):
    counts = synth.batch_peak_counts(1000)
    host = [synth.batch_frame(i, counts) for i in range(6)]
    host.append(synth.jungfrau_frame(3))
    frames = [torch.from_numpy(f).cuda() for f, _ in host]
    peaks = [torch.from_numpy(np.ascontiguousarray(p)).cuda() for _, p in host]
    prm = (11, 2, 5.0, 0)
    store = tmp_path / "tiles.json"
    r = autotune.tune(frames, peaks, prm, candidates=GRID, reps=2, budget_s=1e9, cache_path=None,
                      store_path=str(store))
    assert not r["cached"]
    assert len(r["table"]) == len(GRID)
    assert tuple(r["best"]) in GRID
    assert r["ms"] == min(t[3] for t in r["table"])
    # the best shape's streams are the oracle's
    B = rsz.Batch(frames, peaks, prm, *r["best"])
    B.run()
    torch.cuda.synchronize()
    assert B.status.cpu().tolist() == [0] * len(host)
    for i, (f, pk) in enumerate(host):
        st, ref, _ = O.compress(O.params(*f.shape, *prm), f, pk)
        assert st == O.OK
        np.testing.assert_array_equal(B.stream(i).cpu().numpy(), ref, err_msg=f"frame {i}")
    # the stored entry is read back without timing
    table = json.load(open(store))
    assert autotune.signature(frames, prm) in table
    r2 = autotune.tune(frames, peaks, prm, candidates=GRID, cache_path=str(store))
    assert r2["cached"] and list(r2["best"]) == list(r["best"])
