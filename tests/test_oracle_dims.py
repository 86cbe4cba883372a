"""Pins of the oracle's Lorenzo predictor in one and three dimensions (the
"dimension" of Sec. VI: neighbours along the row of bins, over the panel, or
across the stack of panels), against definitions written independently here:

- the residual is the composition of first differences (numpy's diff with a
  zero prepended) along each axis the predictor spans, where the oracle sums
  signed corner neighbours;
- prefix sums along the same axes give q back;
- fields the predictor is exact on give zero residuals;
- the largest residuals the quantiser allows (|r| up to 2^d (2^28 - 1))
  survive the container;
- the header carries the dimension, and the final reconstruction does not
  depend on it (it has the closed form of the 2D path).
"""
import numpy as np
import pytest

from oracle import rsz_oracle as O
from paper_2206_11297_amd import synth
from tests import streamfmt as F

NOPEAKS = np.zeros((0, 3), np.int32)


def lorenzo_by_differences(q, dim, P, Hb, Wb):
    if dim == 1:
        return np.diff(q.astype(np.int64).ravel(), prepend=0)
    x = q.astype(np.int64).reshape(P, Hb, Wb)
    x = np.diff(np.diff(x, axis=1, prepend=0), axis=2, prepend=0)
    if dim == 3:
        x = np.diff(x, axis=0, prepend=0)
    return x.ravel()


def inverse_by_prefix_sums(r, dim, P, Hb, Wb):
    if dim == 1:
        return np.cumsum(r.astype(np.int64))
    x = np.cumsum(np.cumsum(r.astype(np.int64).reshape(P, Hb, Wb), 1), 2)
    if dim == 3:
        x = np.cumsum(x, 0)
    return x.ravel()


CASES = [
    (1, (1, 5, 7), 2, 3, 2, 1.0, "normal"),
    (2, (2, 9, 9), 3, 5, 3, 0.5, "int"),
    (3, (3, 6, 8), 0, 1, 1, 1.0, "int"),
    (5, (2, 7, 9), 2, 9, 2, 1.0, "special"),
    (7, (3, 4, 5), 3, 2, 2, 1.0, "normal"),
    (8, (1, 1, 1), 1, 1, 1, 1.0, "normal"),
    (11, (4, 13, 70), 5, 3, 1, 0.5, "normal"),
    (12, (3, 1, 9), 1, 1, 1, 0.25, "normal"),
    (13, (5, 8, 1), 1, 1, 1, 0.25, "normal"),
]


@pytest.mark.parametrize("case", CASES, ids=[f"seed{c[0]}" for c in CASES])
@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("bin_mode", [0, 1])
def test_residuals_are_first_differences(case, dim, bin_mode):
    seed, shape, npk, w, b, eb, kind = case
    frame, peaks = synth.tiny_case(seed, shape, npk, kind)
    P, H, W = shape
    Hb, Wb = -(-H // b), -(-W // b)
    p = O.params(*shape, w, b, eb, bin_mode, dim)
    d = O.intermediates(p, frame, peaks)
    assert d["status"] == O.OK
    # q does not depend on the dimension
    d2 = O.intermediates(O.params(*shape, w, b, eb, bin_mode, 2), frame, peaks)
    np.testing.assert_array_equal(d["q"], d2["q"])
    np.testing.assert_array_equal(d["r"], lorenzo_by_differences(d["q"], dim, P, Hb, Wb))
    np.testing.assert_array_equal(inverse_by_prefix_sums(d["r"], dim, P, Hb, Wb), d["q"])
    # codes, outliers and histogram follow the residuals
    small = np.abs(d["r"].astype(np.int64)) < 512
    np.testing.assert_array_equal(d["codes"][small], d["r"][small] + 512)
    assert np.all(d["codes"][~small] == 0)
    np.testing.assert_array_equal(d["out_idx"], np.nonzero(~small)[0])
    np.testing.assert_array_equal(d["hist"], np.bincount(d["codes"], minlength=1024))
    # the stream decodes (independent reader) to these codes, and decompresses
    # to the closed form, whatever the dimension
    st, stream, _ = O.compress(p, frame, peaks)
    assert st == O.OK
    s = F.parse(stream)
    assert s["dim"] == dim and s["bin_mode"] == bin_mode
    syms, _ = F.decode_symbols(s["lens"], s["bit_words"], s["T"], P * Hb * Wb)
    np.testing.assert_array_equal(syms, d["codes"])
    st, y = O.decompress(stream)
    assert st == O.OK
    yc, *_ = F.closed_form_reconstruction(frame, peaks, w, b, eb, bin_mode)
    np.testing.assert_array_equal(y.view(np.uint32), yc.view(np.uint32))
    st, pi, _, _ = O.stream_info(stream)
    assert st == O.OK and pi.dim == dim


def _frame_of_q(q, eb=0.5):
    """b = 1 frame whose bins quantise to q exactly (values q * 2eb)."""
    return (q.astype(np.float64) * 2 * eb).astype(np.float32)


def test_raster_ramp_1d_versus_2d():
    """q = g (the raster index): the 1D residual is 1 after the first bin,
    across row and panel starts; the 2D residual vanishes inside each panel
    (q is bilinear there) but not on its first row and column."""
    P, H, W = 3, 4, 6
    q = np.arange(P * H * W).reshape(P, H, W)
    frame = _frame_of_q(q)
    r1 = O.intermediates(O.params(P, H, W, 1, 1, 0.5, 0, 1), frame, NOPEAKS)["r"]
    assert r1[0] == 0 and np.all(r1[1:] == 1)
    r2 = O.intermediates(O.params(P, H, W, 1, 1, 0.5, 0, 2), frame, NOPEAKS)["r"].reshape(P, H, W)
    assert np.all(r2[:, 1:, 1:] == 0)
    assert np.all(r2[:, 0, 1:] == 1) and np.all(r2[:, 1:, 0] == W)


def test_separable_field_3d_exact():
    """The 3D predictor is exact on q = f(I,J) + g(p,J) + h(p,I): zero
    residual wherever all three axes have a predecessor."""
    rng = np.random.default_rng(9)
    P, H, W = 4, 5, 7
    f = rng.integers(-50, 50, (H, W))
    g = rng.integers(-50, 50, (P, W))
    h = rng.integers(-50, 50, (P, H))
    q = f[None] + g[:, None, :] + h[:, :, None]
    r = O.intermediates(O.params(P, H, W, 1, 1, 0.5, 0, 3), _frame_of_q(q), NOPEAKS)["r"]
    r = r.reshape(P, H, W)
    assert np.all(r[1:, 1:, 1:] == 0)
    assert np.any(r[0] != 0)


def test_identical_panels_3d():
    """Panels that repeat the first one leave only the first panel's 2D
    residuals: every later panel codes as 512 (residual 0)."""
    frame, _ = synth.tiny_case(4, (1, 20, 30), 0, "normal")
    stack = np.repeat(frame, 5, axis=0)
    p3 = O.params(5, 20, 30, 1, 2, 0.5, 0, 3)
    d3 = O.intermediates(p3, stack, NOPEAKS)
    d2 = O.intermediates(O.params(5, 20, 30, 1, 2, 0.5, 0, 2), stack, NOPEAKS)
    plane = 10 * 15
    np.testing.assert_array_equal(d3["r"][:plane], d2["r"][:plane])
    assert np.all(d3["r"][plane:] == 0)
    assert d3["hist"][512] >= 4 * plane
    st3, s3, n3 = O.compress(p3, stack, NOPEAKS)
    st2, s2, n2 = O.compress(O.params(5, 20, 30, 1, 2, 0.5, 0, 2), stack, NOPEAKS)
    assert n3 < n2


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_largest_residuals_round_trip(dim):
    """A checkerboard of q = +-(2^28 - 16) (float32-exact) drives every
    residual to its largest magnitude for the dimension, 2^d (2^28 - 16); the
    outlier list carries them and decompression restores the frame."""
    P, H, W = 3, 4, 5
    A = (1 << 28) - 16
    p_, i_, j_ = np.meshgrid(np.arange(P), np.arange(H), np.arange(W), indexing="ij")
    sign = 1 - 2 * ((p_ + i_ + j_) % 2) if dim == 3 else 1 - 2 * ((i_ + j_) % 2)
    if dim == 1:
        sign = 1 - 2 * (np.arange(P * H * W) % 2).reshape(P, H, W)
    q = (A * sign).astype(np.int64)
    frame = _frame_of_q(q)
    assert np.array_equal(frame.astype(np.int64), q)
    p = O.params(P, H, W, 1, 1, 0.5, 0, dim)
    d = O.intermediates(p, frame, NOPEAKS)
    assert d["status"] == O.OK
    assert np.max(np.abs(d["r"].astype(np.int64))) == (1 << dim) * A
    st, stream, _ = O.compress(p, frame, NOPEAKS)
    assert st == O.OK
    st, y = O.decompress(stream)
    assert st == O.OK
    np.testing.assert_array_equal(y, frame)


def test_header_dimension_flags():
    frame, peaks = synth.tiny_case(21, (2, 9, 11), 3, "normal", scale=100.0)
    for dim, code in ((1, 1), (2, 0), (3, 3), (0, 0)):
        st, s, _ = O.compress(O.params(2, 9, 11, 3, 2, 1.0, 1, dim), frame, peaks)
        assert st == O.OK
        flags = int(s[6]) | int(s[7]) << 8
        assert flags == 1 | code << 1
        st, pi, _, _ = O.stream_info(s)
        assert st == O.OK and pi.dim == (dim or 2) and pi.bin_mode == 1
    # dimension code 2 and any higher flag bit are malformed
    for flags in (1 | 2 << 1, 1 << 3, 1 << 15):
        s2 = s.copy()
        s2[6], s2[7] = flags & 0xFF, flags >> 8
        assert O.stream_info(s2)[0] == O.ERR_CORRUPT
        assert O.decompress(s2)[0] == O.ERR_CORRUPT
    assert O.compress(O.params(2, 9, 11, 3, 2, 1.0, 0, 4), frame, peaks)[0] == O.ERR_ARG


def test_residual_bound_is_checked_per_dimension():
    """An outlier residual at 2^(28+d) cannot come from a valid q field and
    is rejected; the largest 3D value, 2^31 - 1, is accepted."""
    P, H, W = 1, 2, 2
    frame = _frame_of_q(np.array([[[600, 0], [0, 0]]]))
    for dim in (1, 2, 3):
        st, s, _ = O.compress(O.params(P, H, W, 1, 1, 0.5, 0, dim), frame, NOPEAKS)
        d = F.parse(s)
        assert d["n_out"] >= 1
        off = d["off"]["ores"]
        for v, ok in (((1 << (28 + dim)) - 1, True), (1 << (28 + dim), False),
                      (-(1 << (28 + dim)) + 1, True), (-(1 << (28 + dim)), False)):
            if not -(1 << 31) <= v < (1 << 31):
                continue
            s2 = s.copy()
            s2[off:off + 4] = np.frombuffer(np.int32(v).tobytes(), np.uint8)
            assert (O.decompress(s2)[0] == O.OK) == ok, (dim, v)
