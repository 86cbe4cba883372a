"""GPU parity of batched decompression (one launch of each decoder kernel for
many streams) through the C ABI: every frame bit for bit against the oracle's
decompression, across Lorenzo dimensions, bin modes, ROI and run coding and
shapes in one batch; corrupt streams get the oracle's status while the rest
of the batch decodes; host-rejected headers and too-small frames get their
status without work; graph-free repeated runs give the same frames."""
import numpy as np
import pytest

from oracle import rsz_oracle as O
from paper_2206_11297_amd import rsz, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    rsz.lib()
    return t


def _streams():
    cases = [(synth.cspad_frame(5), (17, 2, 10.0, 0, 2, 0, 0)),
             (synth.cspad_frame(6), (17, 2, 10.0, 1, 3, 1, 1)),
             (synth.tiny_case(50, (2, 50, 90), 3, "normal"), (5, 3, 1.0, 0, 1, 0, 1)),
             (synth.jungfrau_frame(3), (25, 4, 10.0, 0, 2, 1, 0)),
             (synth.tiny_case(51, (1, 1, 1), 1, "normal"), (1, 1, 1.0, 0, 2, 0, 0)),
             (synth.cspad_frame(9, npeaks=0), (17, 2, 5.0, 0, 1, 0, 1)),
             (synth.tiny_case(52, (3, 70, 33), 5, "special"), (3, 1, 0.5, 1, 2, 1, 1))]
    out = []
    for (f, pk), t in cases:
        st, s, _ = O.compress(O.params(*f.shape, *t), f, pk)
        assert st == O.OK
        out.append(s)
    return out


def _check(torch, host_streams, expect=None):
    D = rsz.DecodeBatch([torch.from_numpy(s).cuda() for s in host_streams])
    D.run()
    torch.cuda.synchronize()
    status = D.status.cpu().tolist()
    for i, s in enumerate(host_streams):
        sto, yo = O.decompress(s)
        want = sto if expect is None or expect[i] is None else expect[i]
        assert status[i] == want, (i, status[i], want)
        if want == 0:
            np.testing.assert_array_equal(D.frames[i].cpu().numpy().view(np.uint32),
                                          yo.view(np.uint32), err_msg=f"stream {i}")
    return D


def test_mixed_batch(torch):
    D = _check(torch, _streams())
    # a second run over the same workspace gives the same frames
    first = [f.clone() for f in D.frames]
    for f in D.frames:
        f.fill_(-1.0)
    D.run()
    torch.cuda.synchronize()
    assert D.status.cpu().tolist() == [0] * len(first)
    for a, b in zip(first, D.frames):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_corrupt_streams_next_to_good_ones(torch):
    good = _streams()
    rng = np.random.default_rng(91)
    batch = []
    for t in range(24):
        s = good[t % len(good)].copy()
        if t % 3:
            for _ in range(1 + t % 4):
                pos = int(rng.integers(80, s.size))
                s[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        batch.append(s)
    _check(torch, batch)


def test_rejected_headers_and_small_frames(torch):
    good = _streams()
    bad_magic = good[0].copy()
    bad_magic[0] ^= 1
    short = good[1][:-4].copy()               # the header's size exceeds the bytes given
    D = rsz.DecodeBatch([torch.from_numpy(s).cuda() for s in (good[2], bad_magic, short, good[4])])
    # frame 3 too small for its stream
    D.frames[3] = torch.empty(0, dtype=torch.float32, device="cuda")
    D.descs[3].frame_elems = 0
    D.run()
    torch.cuda.synchronize()
    assert D.status.cpu().tolist() == [0, rsz.RSZ_ERR_CORRUPT, rsz.RSZ_ERR_CORRUPT, rsz.RSZ_ERR_ARG]
    np.testing.assert_array_equal(D.frames[0].cpu().numpy().view(np.uint32),
                                  O.decompress(good[2])[1].view(np.uint32))


def test_full_cspad_batch_decodes_like_single_calls(torch):
    counts = synth.batch_peak_counts(1000)
    host = [synth.batch_frame(i, counts) for i in range(200)]
    B = rsz.Batch([torch.from_numpy(f).cuda() for f, _ in host],
                  [torch.from_numpy(p).cuda() for _, p in host], (17, 2, 10.0, 0))
    B.run()
    torch.cuda.synchronize()
    sizes = B.sizes.cpu().numpy()
    streams = [B.stream(i, sizes) for i in range(len(host))]
    print("decoding 200 CSPAD streams in one batch", flush=True)
    D = rsz.DecodeBatch(streams)
    D.run()
    torch.cuda.synchronize()
    assert (D.status.cpu().numpy() == 0).all()
    for i in (0, 1, 57, 123, 199):
        y = rsz.decompress(streams[i])
        assert torch.equal(y.view(torch.int32), D.frames[i].view(torch.int32))
        st, yo = O.decompress(streams[i].cpu().numpy())
        np.testing.assert_array_equal(D.frames[i].cpu().numpy().view(np.uint32), yo.view(np.uint32))


def test_pixel_write_paths(torch):
    """Dimension 2 writes the pixels where q becomes final: in one workgroup
    per panel when the panel's bins fit in LDS (at most 19200 of them, at
    most 1024 per row), else in the column sums.  b = 2 / 4 with W a
    multiple of b writes one float2 / float4 per pixel row of a bin, other
    shapes pixel by pixel; odd H leaves a last bin row of fewer pixel rows.
    Dimensions 1 and 3 expand in a pass of their own."""
    cases = [((2, 31, 40), 2, 2), ((3, 29, 42), 2, 2), ((2, 17, 41), 2, 2), ((2, 33, 44), 4, 2),
             ((2, 35, 46), 4, 2), ((2, 23, 39), 3, 2), ((1, 9, 4), 2, 2), ((2, 31, 40), 2, 1),
             ((3, 29, 44), 2, 3),
             # at and past the LDS limits: 19200 / 19456 bins, 1024 / 1250 bins a row
             ((2, 75, 256), 1, 2), ((1, 76, 256), 1, 2), ((1, 4, 2048), 2, 2), ((1, 3, 2500), 2, 2),
             # column sums writing the pixels: float2, pixel by pixel, float4
             ((1, 401, 202), 2, 2), ((1, 5, 2501), 2, 2), ((1, 650, 480), 4, 2)]
    streams = []
    for k, (shape, b, dim) in enumerate(cases):
        f, pk = synth.tiny_case(60 + k, shape, 3, "normal", scale=50.0)
        st, s, _ = O.compress(O.params(*shape, 3, b, 0.5, 0, dim), f, pk)
        assert st == O.OK
        streams.append(s)
    _check(torch, streams)


def test_window_widths(torch):
    """ROI windows are restored and cross-checked one wave per window, the
    lanes stepping 64 window elements at a time: widths below, at and above
    64 (a step wraps a row at most once), a width of 1, and windows clipped
    by the frame's edges or overlapping each other."""
    streams = []
    for k, w in enumerate((1, 2, 7, 63, 64, 65, 129)):
        f, pk = synth.tiny_case(80 + k, (2, 150, 170), 6, "normal", scale=50.0)
        pk[0, 1:] = (0, 0)                  # clipped at a corner
        pk[1, :] = (pk[2, 0], pk[2, 1], min(pk[2, 2] + 1, 169))   # overlaps peak 2
        st, s, _ = O.compress(O.params(2, 150, 170, w, 2, 0.5, 0, 2, k % 2), f, pk)
        assert st == O.OK, w
        streams.append(s)
    _check(torch, streams)
