"""GPU parity of the Lorenzo predictor in one and three dimensions (Sec. VI's
"dimension") against the oracle: intermediates, stream bytes and the
decompressed frame, bit for bit, on the small and ragged shapes of the 2D
parity suite, on CSPAD and Jungfrau frames (binning kernel's vector path,
several column groups per panel), for every tile shape, in mixed batches and
graph replays, and at the largest residuals the quantiser allows."""
import numpy as np
import pytest

from oracle import rsz_oracle as O
from paper_2206_11297_amd import rsz, synth
from tests.test_gpu_parity import TINY

pytestmark = pytest.mark.gpu

NOPEAKS = np.zeros((0, 3), np.int32)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    rsz.lib()
    return t


def _gpu(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _check_all(torch, frame, peaks, w, b, eb, mode, dim, intermediates=True):
    p = O.params(*frame.shape, w, b, eb, mode, dim)
    if intermediates:
        ref = O.intermediates(p, frame, peaks)
        assert ref["status"] == O.OK
        d = rsz.debug_intermediates(_gpu(torch, frame), _gpu(torch, peaks), w, b, eb, mode, dim)
        assert d["status"] == 0
        np.testing.assert_array_equal(d["q"].cpu().numpy(), ref["q"])
        np.testing.assert_array_equal(d["codes"].cpu().numpy().view(np.uint16), ref["codes"])
        np.testing.assert_array_equal(d["hist"].cpu().numpy().view(np.uint32), ref["hist"])
        np.testing.assert_array_equal(d["lens"].cpu().numpy(), ref["lens"])
        n_out = int(d["n_out"].cpu()[0])
        assert n_out == ref["n_out"]
        np.testing.assert_array_equal(d["out_idx"][:n_out].cpu().numpy().view(np.uint32),
                                      ref["out_idx"])
        np.testing.assert_array_equal(d["out_res"][:n_out].cpu().numpy(), ref["out_res"])
    st, sref, _ = O.compress(p, frame, peaks)
    assert st == O.OK
    got = rsz.compress(_gpu(torch, frame), _gpu(torch, peaks), w, b, eb, mode, dim=dim)
    np.testing.assert_array_equal(got.cpu().numpy(), sref)
    st, yref = O.decompress(sref)
    assert st == O.OK
    y = rsz.decompress(got)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(y.cpu().numpy().view(np.uint32), yref.view(np.uint32))


@pytest.mark.parametrize("case", TINY, ids=[f"seed{c[0]}" for c in TINY])
@pytest.mark.parametrize("dim", [1, 3])
@pytest.mark.parametrize("mode", [0, 1])
def test_small_frames(torch, case, dim, mode):
    seed, shape, npk, w, b, eb, kind = case
    frame, peaks = synth.tiny_case(seed, shape, npk, kind)
    print(f"case seed={seed} shape={shape} b={b} dim={dim} mode={mode}", flush=True)
    _check_all(torch, frame, peaks, w, b, eb, mode, dim)


@pytest.mark.parametrize("dim", [1, 3])
@pytest.mark.parametrize("eb", [1.0, 10.0])
def test_cspad_frame(torch, dim, eb):
    frame, peaks = synth.cspad_frame(0)
    print(f"cspad dim={dim} eb={eb}", flush=True)
    _check_all(torch, frame, peaks, 17, 2, eb, 0, dim)


@pytest.mark.parametrize("dim", [1, 3])
@pytest.mark.parametrize("w,b", [(11, 2), (25, 4), (11, 1)])
def test_jungfrau_frame(torch, dim, w, b):
    frame, peaks = synth.jungfrau_frame(1)
    print(f"jungfrau dim={dim} w={w} b={b}", flush=True)
    _check_all(torch, frame, peaks, w, b, 10.0, 0, dim, intermediates=False)


@pytest.mark.parametrize("dim", [1, 3])
def test_tile_shapes_never_change_bytes(torch, dim):
    """Row starts (dim 1) and panel columns (dim 3) cross every tile boundary
    the tile shapes put them on."""
    frame, peaks = synth.jungfrau_frame(6, npeaks=200)
    st, ref, _ = O.compress(O.params(*frame.shape, 11, 2, 10.0, 0, dim), frame, peaks)
    g, pk = _gpu(torch, frame), _gpu(torch, peaks)
    for tr, ts in ((0, 0), (1, 1), (3, 2), (8, 4), (32, 1), (5, 3)):
        print(f"dim={dim} tile_rows={tr} tile_strips={ts}", flush=True)
        B = rsz.Batch([g], [pk], (11, 2, 10.0, 0, dim), tile_rows=tr, tile_strips=ts)
        B.run()
        torch.cuda.synchronize()
        assert B.status.cpu().tolist() == [0]
        np.testing.assert_array_equal(B.stream(0).cpu().numpy(), ref)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_largest_residuals(torch, dim):
    """q = +-(2^28 - 16) in a checkerboard along the predictor's axes: every
    residual is an outlier of magnitude up to 2^d (2^28 - 16)."""
    P, H, W = 3, 40, 70
    A = (1 << 28) - 16
    p_, i_, j_ = np.meshgrid(np.arange(P), np.arange(H), np.arange(W), indexing="ij")
    par = {1: np.arange(P * H * W).reshape(P, H, W), 2: i_ + j_, 3: p_ + i_ + j_}[dim]
    frame = (A * (1 - 2 * (par % 2))).astype(np.float32)
    _check_all(torch, frame, NOPEAKS, 1, 1, 0.5, 0, dim)


def test_batch_mixed_dimensions_and_graph(torch):
    """One batch holding every dimension over different geometries equals the
    oracle frame by frame, launched eagerly and replayed from a graph with
    new frame contents in between."""
    cases = [synth.cspad_frame(7), synth.tiny_case(40, (2, 50, 90), 3, "normal"),
             synth.jungfrau_frame(2), synth.cspad_frame(8, npeaks=0),
             synth.tiny_case(41, (1, 1, 1), 1, "normal"), synth.tiny_case(42, (4, 30, 130), 5,
                                                                         "normal")]
    prm = [(17, 2, 10.0, 0, 3), (5, 3, 1.0, 1, 1), (11, 4, 10.0, 0, 1), (17, 2, 5.0, 0, 2),
           (1, 1, 1.0, 0, 3), (3, 2, 0.5, 1, 3)]
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
    rng = np.random.default_rng(78)
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


@pytest.mark.parametrize("dim", [1, 3])
def test_corrupt_streams_match_oracle_status(torch, dim):
    frame, peaks = synth.tiny_case(14, (3, 12, 16), 3, "normal", scale=200.0)
    st, s, _ = O.compress(O.params(3, 12, 16, 3, 2, 1.0, 0, dim), frame, peaks)
    rng = np.random.default_rng(50 + dim)
    for t in range(60):
        s2 = s.copy()
        pos = int(rng.integers(80, s2.size))
        s2[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        sto, yo = O.decompress(s2)
        try:
            y = rsz.decompress(_gpu(torch, s2)).cpu().numpy()
            stg = 0
        except rsz.RszError as e:
            stg = e.status
        assert stg == sto, (t, pos)
        if sto == 0:
            np.testing.assert_array_equal(y.view(np.uint32), yo.view(np.uint32))


@pytest.mark.parametrize("plane", [1, 3, 15, 16, 17, 31, 48, 4095, 4096, 4097, 20000])
def test_panel_plane_sizes_3d(torch, plane):
    """Panel planes of every size class around the 16-byte groups the 3D
    step works in (the predecessor bytes sit (-plane) mod 16 into a group;
    panel 0 ends inside a group), with a mix of small residuals and escapes
    on both sides of the panel difference."""
    rng = np.random.default_rng(plane)
    P = max(3, min(40, 60000 // plane))
    base = rng.normal(0.0, 3.0, (1, 1, plane))
    frame = (base + rng.normal(0.0, 1.0, (P, 1, plane))).astype(np.float32)
    spikes = rng.random((P, 1, plane)) < 0.05
    frame[spikes] = rng.normal(0.0, 2000.0, int(spikes.sum())).astype(np.float32)
    print(f"plane={plane} panels={P}", flush=True)
    _check_all(torch, frame, NOPEAKS, 1, 1, 0.5, 0, 3)
