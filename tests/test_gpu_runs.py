"""GPU parity of the lossless run stage after the Huffman coder (per-chunk
Rice coding of the zero runs): stream bytes and decompressed frames bit for
bit against the oracle, through the C ABI, on small and ragged frames, every
Lorenzo dimension with and without the ROI coded, CSPAD and Jungfrau frames,
mixed batches with graph replays, the capacity report, and corrupt or
crafted run sections (same status as the oracle)."""
import numpy as np
import pytest

from oracle import rsz_oracle as O
from paper_2206_11297_amd import rsz, synth
from tests import streamfmt as F
from tests.test_gpu_parity import TINY
from tests.test_oracle_runs import _rebuild

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    rsz.lib()
    return t


def _gpu(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _check(torch, frame, peaks, w, b, eb, mode=0, dim=2, roi=0):
    st, ref, _ = O.compress(O.params(*frame.shape, w, b, eb, mode, dim, roi, 1), frame, peaks)
    assert st == O.OK
    got = rsz.compress(_gpu(torch, frame), _gpu(torch, peaks), w, b, eb, mode, dim=dim,
                       roi_coding=roi, run_coding=1)
    np.testing.assert_array_equal(got.cpu().numpy(), ref)
    st, yref = O.decompress(ref)
    assert st == O.OK
    y = rsz.decompress(got)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(y.cpu().numpy().view(np.uint32), yref.view(np.uint32))
    return ref


@pytest.mark.parametrize("case", TINY, ids=[f"seed{c[0]}" for c in TINY])
def test_small_frames(torch, case):
    seed, shape, npk, w, b, eb, kind = case
    frame, peaks = synth.tiny_case(seed, shape, npk, kind)
    print(f"case seed={seed} shape={shape} npk={npk} w={w}", flush=True)
    _check(torch, frame, peaks, w, b, eb)
    _check(torch, frame, peaks, w, b, eb, mode=1, roi=1)


def test_constant_frames(torch):
    # no one bit at all, and the parameter tie of two runs (0 and 1023)
    _check(torch, np.zeros((2, 64, 64), np.float32), np.zeros((0, 3), np.int32), 5, 2, 1.0)
    _check(torch, np.full((2, 64, 64), 7.0, np.float32), np.zeros((0, 3), np.int32), 5, 2, 1.0)


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("roi", [0, 1])
def test_cspad_and_jungfrau(torch, dim, roi):
    frame, peaks = synth.cspad_frame(0)
    _check(torch, frame, peaks, 17, 2, 10.0, dim=dim, roi=roi)
    frame, peaks = synth.jungfrau_frame(1)
    _check(torch, frame, peaks, 25, 4, 10.0, dim=dim, roi=roi)


def test_dense_bits_and_every_parameter(torch):
    """Fine bounds make the Huffman bits dense (small parameters), coarse
    ones sparse (large parameters): across them the chunks take many of the
    21 parameters."""
    frame, peaks = synth.cspad_frame(4)
    ks = set()
    for eb in (0.05, 1.0, 10.0, 200.0, 5000.0):
        ref = _check(torch, frame, peaks, 17, 1, eb)
        d = F.parse(ref)
        ks |= set(d["run_k"][:d["n_chunks"]].tolist())
    assert len(ks) >= 6, ks


def test_batch_mixed_coding_and_graph(torch):
    cases = [synth.cspad_frame(7), synth.tiny_case(40, (2, 50, 90), 3, "normal"),
             synth.jungfrau_frame(2), synth.cspad_frame(8, npeaks=0),
             synth.tiny_case(41, (1, 1, 1), 1, "normal"), synth.tiny_case(42, (3, 70, 33), 5, "int")]
    prm = [(17, 2, 10.0, 0, 2, 1, 1), (5, 3, 1.0, 1, 1, 1, 1), (11, 4, 10.0, 0, 2, 0, 0),
           (17, 2, 5.0, 0, 3, 0, 1), (1, 1, 1.0, 0, 2, 1, 1), (3, 1, 0.5, 0, 2, 0, 1)]
    frames = [_gpu(torch, f) for f, _ in cases]
    peaks = [_gpu(torch, p) for _, p in cases]

    def refs(cur):
        out = []
        for (f, pk), t in zip(cur, prm):
            st, ref, _ = O.compress(O.params(*f.shape, *t), f, pk)
            assert st == O.OK
            out.append(ref)
        return out

    B = rsz.Batch(frames, peaks, prm)
    B.run()
    torch.cuda.synchronize()
    assert B.status.cpu().tolist() == [0] * len(cases)
    for i, ref in enumerate(refs(cases)):
        np.testing.assert_array_equal(B.stream(i).cpu().numpy(), ref)
    B.prepare()
    B.graph()
    rng = np.random.default_rng(83)
    for rep in range(3):
        cur = []
        for (f, pk), g in zip(cases, frames):
            f2 = (f + rng.normal(0, 3, f.shape)).astype(np.float32)
            g.copy_(torch.from_numpy(f2))
            cur.append((f2, pk))
        torch.cuda.synchronize()
        B.replay()
        torch.cuda.synchronize()
        assert B.status.cpu().tolist() == [0] * len(cases)
        for i, ref in enumerate(refs(cur)):
            np.testing.assert_array_equal(B.stream(i).cpu().numpy(), ref)


def test_capacity_reports_the_coded_size(torch):
    frame, peaks = synth.cspad_frame(3)
    st, ref, need = O.compress(O.params(32, 185, 388, 17, 2, 10.0, 0, 2, 0, 1), frame, peaks)
    p = rsz.params(32, 185, 388, 17, 2, 10.0, 0, 2, 0, 1)
    g, pk = _gpu(torch, frame), _gpu(torch, peaks)
    out = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    ws = rsz.workspace(rsz.rsz_workspace_bytes(p, peaks.shape[0])[1])
    st, n = rsz.rsz_compress(p, rsz._ptr(g), rsz._ptr(pk), peaks.shape[0], rsz._ptr(out),
                             out.numel(), rsz._ptr(ws), ws.numel(), rsz._stream())
    assert st == rsz.RSZ_ERR_CAPACITY and n == need
    out = torch.empty(need, dtype=torch.uint8, device="cuda")
    st, n = rsz.rsz_compress(p, rsz._ptr(g), rsz._ptr(pk), peaks.shape[0], rsz._ptr(out),
                             out.numel(), rsz._ptr(ws), ws.numel(), rsz._stream())
    assert st == rsz.RSZ_OK and n == need
    np.testing.assert_array_equal(out.cpu().numpy(), ref)


def _status(torch, s2):
    try:
        y = rsz.decompress(_gpu(torch, s2)).cpu().numpy()
        return 0, y
    except rsz.RszError as e:
        return e.status, None


def test_corrupt_run_sections_match_oracle(torch):
    frame, peaks = synth.tiny_case(20, (2, 90, 150), 4, "normal")
    st, s1, _ = O.compress(O.params(2, 90, 150, 7, 1, 3.0, 0, 2, 0, 1), frame, peaks)
    d = F.parse(s1)
    run = d["off"]["run"]
    rng = np.random.default_rng(87)
    for t in range(120):
        s2 = s1.copy()
        pos = int(rng.integers(run, s2.size))
        s2[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        sto, yo = O.decompress(s2)
        stg, y = _status(torch, s2)
        assert stg == sto, (t, pos)
        if sto == 0:
            np.testing.assert_array_equal(y.view(np.uint32), yo.view(np.uint32))
    # crafted: a parameter above 20, a padding byte, a one bit moved from
    # chunk 1's codes to chunk 0's (same expanded bits, but past chunk 0's
    # end), a last offset beyond the words, a truncated stream
    nch = d["n_chunks"]
    roff = d["off"]["runoffs"]
    T = d["T"]
    co = [int(x) for x in d["chunk_offsets"]] + [T]
    allones = np.flatnonzero(np.array(F.bits_of(d["bit_words"], T)))
    ones = [[int(x) for x in allones if co[c] <= x < co[c + 1]] for c in range(nch)]
    moved = [list(x) for x in ones]
    moved[0].append(moved[1].pop(0))
    crafted = []
    for edit in (lambda s: s.__setitem__(run, 21), lambda s: s.__setitem__(run + nch, 1),
                 lambda s: s[roff + 4 * nch:roff + 4 * nch + 4].view(np.uint32).__setitem__(
                     0, d["Trun"] + 32)):
        s2 = s1.copy()
        edit(s2)
        crafted.append(s2)
    crafted += [_rebuild(s1, d, moved), _rebuild(s1, d, ones), s1[:-4].copy()]
    for i, s2 in enumerate(crafted):
        sto, yo = O.decompress(s2)
        stg, y = _status(torch, s2)
        assert stg == sto, i
        if i < 4 or i == 5:
            assert sto == O.ERR_CORRUPT, i
        if sto == 0:
            np.testing.assert_array_equal(y.view(np.uint32), yo.view(np.uint32))
