"""Pins of the oracle's lossless run stage after the Huffman coder (SZ passes
its Huffman output through a lossless compressor; here a Rice coding of the
zero runs of each 4096-symbol chunk's bits):

- an independent reader (tests/streamfmt.py) expands the run section back to
  the Huffman bits of the verbatim stream, bit for bit, and every other
  section is unchanged;
- an independent string encoder written here (runs as '1' * q + '0' + k
  binary digits) gives the run bits of every chunk exactly, for the
  parameter the stream names, and that parameter gives the fewest bits of
  the 21 candidates (the first on ties);
- closed forms: an all-zero frame (one code of length 1, all bits zero) has
  no run bits and parameter 0; a constant frame with two one bits has a
  parameter tie broken towards the smaller; the section never codes more
  bits than T, and the size bound covers it;
- decompression gives the same frame as the verbatim stream across Lorenzo
  dimensions, bin modes and ROI coding;
- corruption of the run section decodes or is rejected; malformed
  parameters, offsets and sizes are rejected."""
import numpy as np
import pytest

from oracle import rsz_oracle as O
from paper_2206_11297_amd import synth
from tests import streamfmt as F


def _pair(frame, peaks, w, b, eb, mode=0, dim=2, roi=0):
    P, H, W = frame.shape
    st0, s0, _ = O.compress(O.params(P, H, W, w, b, eb, mode, dim, roi, 0), frame, peaks)
    st1, s1, _ = O.compress(O.params(P, H, W, w, b, eb, mode, dim, roi, 1), frame, peaks)
    assert st0 == O.OK and st1 == O.OK
    return s0, s1


def _string_code(bits, k):
    """The Rice code of the zero runs before each one bit, as a '0'/'1'
    string."""
    out, run = [], 0
    for x in bits:
        if x:
            out.append("1" * (run >> k) + "0" + (format(run & ((1 << k) - 1), f"0{k}b") if k else ""))
            run = 0
        else:
            run += 1
    return "".join(out)


def _check_runs(d0, d1):
    T, nch = d0["T"], d0["n_chunks"]
    bits = np.array(F.bits_of(d0["bit_words"], T), np.uint8)
    co = [int(x) for x in d0["chunk_offsets"]] + [T]
    run_bits = "".join(str(x) for x in F.bits_of(d1["run_words"], d1["Trun"]))
    offs = d1["run_offsets"]
    assert int(offs[0]) == 0
    for c in range(nch):
        seg = bits[co[c]:co[c + 1]]
        k = int(d1["run_k"][c])
        got = run_bits[int(offs[c]):int(offs[c + 1])]
        assert got == _string_code(seg, k), c
        sizes = [len(_string_code(seg, kk)) for kk in range(21)]
        assert k == int(np.argmin(sizes)) and len(got) == min(sizes)
    assert not d1["run_k"][nch:].any()
    assert d1["Trun"] <= T


CASES = [
    (1, (1, 5, 7), 2, 3, 2, 1.0, "normal", 2),
    (2, (2, 9, 9), 3, 5, 3, 0.5, "int", 1),
    (5, (2, 7, 9), 2, 9, 2, 1.0, "special", 2),
    (11, (3, 40, 61), 12, 7, 2, 0.5, "normal", 3),
    (12, (2, 30, 30), 6, 25, 1, 2.0, "int", 2),
    (20, (2, 90, 150), 4, 7, 1, 3.0, "normal", 2),
]


@pytest.mark.parametrize("case", CASES, ids=[f"seed{c[0]}" for c in CASES])
@pytest.mark.parametrize("roi", [0, 1])
def test_run_section_matches_definition(case, roi):
    seed, shape, npk, w, b, eb, kind, dim = case
    frame, peaks = synth.tiny_case(seed, shape, npk, kind)
    s0, s1 = _pair(frame, peaks, w, b, eb, dim=dim, roi=roi)
    d0, d1 = F.parse(s0), F.parse(s1)
    assert not d0["run_coded"] and d1["run_coded"]
    # the independent reader gives back the verbatim Huffman bits
    np.testing.assert_array_equal(d1["bit_words"], d0["bit_words"])
    for key in ("lens", "oidx", "ores", "chunk_offsets", "roi", "peaks"):
        np.testing.assert_array_equal(d1[key], d0[key], err_msg=key)
    assert d1["T"] == d0["T"] and d1["n_out"] == d0["n_out"]
    _check_runs(d0, d1)
    st0, y0 = O.decompress(s0)
    st1, y1 = O.decompress(s1)
    assert st0 == st1 == O.OK
    np.testing.assert_array_equal(y1.view(np.uint32), y0.view(np.uint32))


def test_constant_frames():
    # all zeros: one code (length 1, all bits zero), no run bits, parameter 0
    f = np.zeros((2, 64, 64), np.float32)
    s0, s1 = _pair(f, np.zeros((0, 3), np.int32), 5, 2, 1.0)
    d0, d1 = F.parse(s0), F.parse(s1)
    assert d0["T"] == 2 * 32 * 32 and not d0["bit_words"].any()
    assert d1["Trun"] == 0 and not d1["run_k"].any() and not d1["run_offsets"].any()
    assert s1.size == s0.size - 4 * (d0["T"] // 32) + 4 + 4 * 2
    np.testing.assert_array_equal(O.decompress(s1)[1], f)
    # all 7.0 with 2eb = 2: the first bin of each panel has q = rint(3.5) = 4
    # and the one residual that is not 0, so the two codes have length 1 and
    # the bits are zero but for bits 0 and 1024 (residual 4 sorts after 0):
    # runs 0 and 1023 in one chunk.  Bits per parameter k: (0 >> k) + (1023 >>
    # k) + 2 (k + 1), 21 for k = 8 and for k = 9, more for every other k: the
    # tie goes to 8, coded as '0' + 8 zeros, then '1110' + 8 ones
    f = np.full((2, 64, 64), 7.0, np.float32)
    s0, s1 = _pair(f, np.zeros((0, 3), np.int32), 5, 2, 1.0)
    d0, d1 = F.parse(s0), F.parse(s1)
    ones = np.flatnonzero(np.array(F.bits_of(d0["bit_words"], d0["T"])))
    assert ones.tolist() == [0, 1024]
    assert [(0 >> k) + (1023 >> k) + 2 * (k + 1) for k in (7, 8, 9, 10)] == [23, 21, 21, 22]
    assert d1["Trun"] == 21 and d1["run_k"][0] == 8
    assert d1["run_words"].tolist() == [int(("0" * 9 + "1110" + "1" * 8).ljust(32, "0"), 2)]
    np.testing.assert_array_equal(O.decompress(s1)[1], O.decompress(s0)[1])


def test_cspad_frame_and_bin_modes():
    frame, peaks = synth.cspad_frame(0)
    for mode, b in ((0, 2), (1, 1)):
        s0, s1 = _pair(frame, peaks, 17, b, 10.0, mode)
        d0, d1 = F.parse(s0), F.parse(s1)
        assert d1["Trun"] < d0["T"] // 2                  # the code-0 runs dominate
        np.testing.assert_array_equal(O.decompress(s1)[1].view(np.uint32),
                                      O.decompress(s0)[1].view(np.uint32))
    # the parameters of the first chunks, against the string encoder
    bits = np.array(F.bits_of(d0["bit_words"], d0["T"]), np.uint8)
    co = d0["chunk_offsets"]
    for c in range(3):
        seg = bits[co[c]:co[c + 1]]
        sizes = [len(_string_code(seg, k)) for k in range(21)]
        assert int(d1["run_k"][c]) == int(np.argmin(sizes))


def test_max_bytes_covers_the_run_section():
    p0 = O.params(3, 40, 61, 7, 1, 0.5)
    p1 = O.params(3, 40, 61, 7, 1, 0.5, 0, 2, 0, 1)
    nb = O.nbins(p1)
    nc = -(-nb // 4096)
    assert O.max_bytes(p1, 5)[1] == O.max_bytes(p0, 5)[1] + F.align4(nc) + 4 * (nc + 1)
    frame, peaks = synth.tiny_case(11, (3, 40, 61), 5, "normal", scale=1e6)
    st, s1, need = O.compress(p1, frame, peaks)
    assert st == O.OK and need <= O.max_bytes(p1, 5)[1]


def test_corrupt_run_sections():
    frame, peaks = synth.tiny_case(20, (2, 90, 150), 4, "normal")
    _, s1 = _pair(frame, peaks, 7, 1, 3.0)
    d = F.parse(s1)
    run = d["off"]["run"]
    nch = d["n_chunks"]
    assert nch == 7 and d["Trun"] > 0
    rng = np.random.default_rng(9)
    rejected = 0
    for t in range(300):
        s2 = s1.copy()
        pos = int(rng.integers(run, s2.size))
        s2[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        st, _ = O.decompress(s2)
        assert st in (O.OK, O.ERR_CORRUPT)
        rejected += st == O.ERR_CORRUPT
    assert rejected > 0

    def bad(edit):
        s2 = s1.copy()
        edit(s2)
        return O.decompress(s2)[0] == O.ERR_CORRUPT

    assert bad(lambda s: s.__setitem__(run, 21))                # parameter above 20
    assert bad(lambda s: s.__setitem__(run + nch, 1))           # padding byte
    roff = d["off"]["runoffs"]
    assert bad(lambda s: s[roff:roff + 4].view(np.uint32).__setitem__(0, 1))   # first offset
    # an offset that goes backwards
    o2 = int(d["run_offsets"][2])
    assert bad(lambda s: s[roff + 8:roff + 12].view(np.uint32).__setitem__(0, o2 + 40))
    # the last offset must fill the words exactly
    last = roff + 4 * nch
    assert bad(lambda s: s[last:last + 4].view(np.uint32).__setitem__(0, d["Trun"] + 32))
    # cleared flag: the sizes no longer add up
    assert bad(lambda s: s.__setitem__(6, s[6] & ~np.uint8(16)))
    # a reserved flag bit
    assert bad(lambda s: s.__setitem__(6, s[6] | np.uint8(32)))
    # a truncated stream
    assert O.decompress(s1[:-4])[0] == O.ERR_CORRUPT
    # one bit beyond a chunk's end: move a chunk offset down so that chunk
    # 0's ones no longer fit
    co = d["off"]["chunks"]
    c1 = int(d["chunk_offsets"][1])
    assert bad(lambda s: s[co + 4:co + 8].view(np.uint32).__setitem__(0, c1 - 64))


def _rebuild(s1, d, ones):
    """The stream with its run section re-coded from absolute one-bit
    positions per chunk (each chunk's parameter kept), by the string
    encoder."""
    co = d["chunk_offsets"]
    codes = []
    for c, pos in enumerate(ones):
        bits = np.zeros(max(pos) + 1 - int(co[c]) if pos else 0, np.uint8)
        bits[np.array(pos, np.int64) - int(co[c])] = 1
        codes.append(_string_code(bits, int(d["run_k"][c])))
    offs = np.cumsum([0] + [len(x) for x in codes]).astype(np.uint32)
    allbits = "".join(codes)
    padded = allbits.ljust(32 * (-(-len(allbits) // 32)), "0")
    words = np.array([int(padded[i:i + 32], 2) for i in range(0, len(padded), 32)], np.uint32)
    s2 = np.concatenate([s1[:d["off"]["runoffs"]], offs.view(np.uint8), words.view(np.uint8)])
    s2[64:72] = np.array([s2.size], np.uint64).view(np.uint8)
    return s2


def test_a_one_bit_past_its_chunk_is_rejected():
    """Moving chunk 1's first one bit into chunk 0's codes leaves the
    expanded bits unchanged, but chunk 0 then places a bit beyond its end."""
    frame, peaks = synth.tiny_case(20, (2, 90, 150), 4, "normal")
    _, s1 = _pair(frame, peaks, 7, 1, 3.0)
    d = F.parse(s1)
    T = d["T"]
    co = [int(x) for x in d["chunk_offsets"]] + [T]
    allones = np.flatnonzero(np.array(F.bits_of(d["bit_words"], T)))
    ones = [[int(x) for x in allones if co[c] <= x < co[c + 1]] for c in range(d["n_chunks"])]
    np.testing.assert_array_equal(_rebuild(s1, d, ones), s1)        # the builder itself
    moved = [list(x) for x in ones]
    moved[0].append(moved[1].pop(0))
    s2 = _rebuild(s1, d, moved)
    assert O.decompress(s2)[0] == O.ERR_CORRUPT


def test_rice_parameter_window():
    """The fact the GPU parameter search rests on.  With n runs of sum S, the
    cost f(k) = sum(r >> k) + n (1 + k) is convex in k (f(k+1) - f(k) = n -
    sum(ceil((r >> k) / 2)) never decreases), f(k+1) < f(k) while 3 n 2^k <
    S, and f(k+1) >= f(k) once n 2^k >= S.  So the smallest minimiser over
    0..20 lies in [kl, kl + 2] with kl the smallest k with 3 n 2^k >= S (then
    clamped to 20).  Checked exhaustively against the argmin on random run
    lists of many shapes, and the window is tight (every offset occurs)."""
    rng = np.random.default_rng(5)
    seen = set()
    for t in range(4000):
        n = int(rng.integers(1, 60))
        kind = t % 4
        if kind == 0:
            r = rng.geometric(1.0 / float(rng.uniform(1, 5000)), n) - 1
        elif kind == 1:
            r = rng.integers(0, 1 << int(rng.integers(0, 18)), n)
        elif kind == 2:
            r = np.where(rng.random(n) < 0.9, 0, rng.integers(0, 1 << 17, n))
        else:
            r = np.full(n, int(rng.integers(0, 1 << 17)))
        if t % 50 == 0:
            # one run of 6 * 2^j and three of 2 * 2^j: S = 3 n 2^j, so kl = j,
            # and the costs give k = j + 2 (the window's last value)
            j = int(rng.integers(0, 15))
            r, n = np.array([6 << j] + [2 << j] * 3), 4
        r = r.astype(np.int64)
        cost = [int((r >> k).sum()) + n * (1 + k) for k in range(21)]
        best = int(np.argmin(cost))
        S = int(r.sum())
        kl = 0
        while 3 * n * (1 << kl) < S:
            kl += 1
        kl = min(kl, 20)
        assert kl <= best <= min(kl + 2, 20), (n, S, kl, best)
        seen.add(best - kl)
    assert seen == {0, 1, 2}
