"""Pins of the oracle's lossless ROI coder (the windows Sec. IV keeps exactly,
coded by a predictive float coder in place of fpzip):

- an independent reader (tests/streamfmt.py) decodes the coded section back
  to the exact payload bits of the verbatim stream;
- the section's size equals the definition recomputed here with numpy
  (order-preserving map, 2D Lorenzo over the window, zigzag classes, class
  code lengths + class - 1 raw bits);
- the class code is an optimal prefix code (independent heap Huffman cost);
- decompression gives the same frame as the verbatim stream, for special
  values (NaN, infinities, -0.0, denormals), windows off the panel, and no
  peaks at all;
- corruption of the coded section decodes or is rejected."""
import heapq

import numpy as np
import pytest

from oracle import rsz_oracle as O
from paper_2206_11297_amd import synth
from tests import streamfmt as F


def _both(frame, peaks, w, b, eb, mode=0, dim=2):
    P, H, W = frame.shape
    st0, s0, n0 = O.compress(O.params(P, H, W, w, b, eb, mode, dim, 0), frame, peaks)
    st1, s1, n1 = O.compress(O.params(P, H, W, w, b, eb, mode, dim, 1), frame, peaks)
    assert st0 == O.OK and st1 == O.OK
    return s0, s1


def _classes(payload, npk, w):
    b = payload.reshape(npk, w, w).astype(np.uint64)
    M = np.where(b & 0x80000000, (~b) & 0xFFFFFFFF, b | 0x80000000).astype(np.int64)
    P = np.pad(M, ((0, 0), (1, 0), (1, 0)), constant_values=1 << 31)
    pred = (P[:, :-1, 1:] + P[:, 1:, :-1] - P[:, :-1, :-1]) & 0xFFFFFFFF
    r = (M - pred) & 0xFFFFFFFF
    r = np.where(r >= 1 << 31, r - (1 << 32), r)             # as int32
    z = np.where(r >= 0, 2 * r, -2 * r - 1)
    c = np.zeros(z.shape, np.int64)
    t = z.copy()
    while (t > 0).any():
        c += t > 0
        t >>= 1
    return c.ravel()


def _heap_cost(counts):
    h = [int(x) for x in counts if x > 0]
    if len(h) == 1:
        return h[0]
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


CASES = [
    (1, (1, 5, 7), 2, 3, 2, 1.0, "normal"),
    (2, (2, 9, 9), 3, 5, 3, 0.5, "int"),
    (5, (2, 7, 9), 2, 9, 2, 1.0, "special"),
    (10, (1, 9, 9), 2, 17, 2, 1.0, "normal"),
    (11, (3, 40, 61), 12, 7, 2, 0.5, "normal"),
    (12, (2, 30, 30), 6, 25, 1, 2.0, "int"),
    (13, (1, 20, 20), 3, 1, 2, 1.0, "const"),
]


@pytest.mark.parametrize("case", CASES, ids=[f"seed{c[0]}" for c in CASES])
def test_coded_section_matches_definition(case):
    seed, shape, npk, w, b, eb, kind = case
    frame, peaks = synth.tiny_case(seed, shape, npk, kind)
    s0, s1 = _both(frame, peaks, w, b, eb)
    d0, d1 = F.parse(s0), F.parse(s1)
    assert not d0["roi_coded"] and d1["roi_coded"]
    # the independent reader returns the verbatim payload bit for bit
    np.testing.assert_array_equal(d1["roi"], d0["roi"])
    # everything else of the stream is the same
    assert d1["T"] == d0["T"] and d1["n_out"] == d0["n_out"]
    np.testing.assert_array_equal(d1["bit_words"], d0["bit_words"])
    # size from the definition; optimal class code
    c = _classes(d0["roi"], npk, w)
    lens = d1["roi_lens"][:33].astype(np.int64)
    assert int(d1["Troi"]) == int(lens[c].sum() + np.maximum(c - 1, 0).sum())
    hist = np.bincount(c, minlength=33)
    assert int((hist * lens).sum()) == _heap_cost(hist)
    assert not d1["roi_lens"][33:].any()
    # decompression is the same frame
    st, y0 = O.decompress(s0)
    st1, y1 = O.decompress(s1)
    assert st == st1 == O.OK
    np.testing.assert_array_equal(y1.view(np.uint32), y0.view(np.uint32))


def test_special_values_and_edges():
    f = np.random.default_rng(3).normal(0.0, 3.0, (2, 20, 24)).astype(np.float32)
    f[0, 5, 5] = np.nan
    f[0, 5, 6] = np.inf
    f[0, 6, 5] = -np.inf
    f[0, 6, 6] = -0.0
    f[0, 4, 4] = np.float32(1e-45)
    f[1, :3, :3] = 0.0
    peaks = np.array([[0, 5, 5], [0, 0, 0], [1, 19, 23], [1, 1, 1], [0, 5, 5]], np.int32)
    s0, s1 = _both(f, peaks, 9, 2, 1.0)
    d0, d1 = F.parse(s0), F.parse(s1)
    np.testing.assert_array_equal(d1["roi"], d0["roi"])
    st, y1 = O.decompress(s1)
    assert st == O.OK
    np.testing.assert_array_equal(y1.view(np.uint32), O.decompress(s0)[1].view(np.uint32))
    M = F.mask_slices(f.shape, [tuple(x) for x in peaks], 9)
    np.testing.assert_array_equal(y1.view(np.uint32)[M], f.view(np.uint32)[M])


def test_no_peaks_and_cspad_frame():
    f, _ = synth.tiny_case(30, (2, 16, 16), 0, "normal")
    s0, s1 = _both(f, np.zeros((0, 3), np.int32), 5, 2, 1.0)
    d1 = F.parse(s1)
    assert d1["Troi"] == 0 and not d1["roi_lens"].any()
    assert O.decompress(s1)[0] == O.OK
    frame, peaks = synth.cspad_frame(0)
    s0, s1 = _both(frame, peaks, 17, 2, 10.0)
    assert s1.size < s0.size
    np.testing.assert_array_equal(O.decompress(s1)[1].view(np.uint32),
                                  O.decompress(s0)[1].view(np.uint32))


def test_corrupt_coded_sections():
    frame, peaks = synth.tiny_case(14, (2, 12, 16), 3, "normal", scale=200.0)
    _, s1 = _both(frame, peaks, 5, 2, 1.0)
    d = F.parse(s1)
    rsec = d["off"]["rsec"]
    rng = np.random.default_rng(8)
    rejected = 0
    for t in range(300):
        s2 = s1.copy()
        pos = int(rng.integers(rsec, s2.size))
        s2[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        st, _ = O.decompress(s2)
        assert st in (O.OK, O.ERR_CORRUPT)
        rejected += st == O.ERR_CORRUPT
    assert rejected > 0
    # a class length beyond 32, and a non-zero padding byte
    for off, val in ((rsec, 40), (rsec + 34, 1)):
        s2 = s1.copy()
        s2[off] = val
        assert O.decompress(s2)[0] == O.ERR_CORRUPT
    # a header that says verbatim but carries ROI bits
    s2 = s1.copy()
    s2[6] &= ~np.uint8(8)
    assert O.decompress(s2)[0] == O.ERR_CORRUPT
    # the coding flag needs a coded-size limit: npeaks * w * w <= 2^26
    p = O.params(1, 64, 64, 1023, 1, 1.0, 0, 2, 1)
    assert O.lib().ro_check_params(p, 65) == O.ERR_ARG
    p.roi_coding = 0
    assert O.lib().ro_check_params(p, 65) == O.OK
