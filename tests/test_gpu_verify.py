"""The on-device verification stage (rsz_verify_*): a prepared batch
captured with its verification in one HIP graph and replayed.  Every
frame's failing-pixel count must be 0, every decoding the verification
writes must equal the oracle's decompression bit for bit, every stream the
oracle's, and frames the stage cannot verify (a failed compression, the
ROI coded) must report 0xFFFFFFFF while the others still pass."""
import numpy as np
import pytest

from oracle import rsz_oracle as O
from paper_2206_11297_amd import rsz, synth

pytestmark = pytest.mark.gpu

NOT_VERIFIED = 0xFFFFFFFF


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    rsz.lib()
    return t


def _gpu(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _full(t):
    return tuple(t) + (2, 0, 0)[len(t) - 4:]


def _check_against_oracle(torch, B, V, cases, prm, skip=()):
    for i, ((f, pk), t) in enumerate(zip(cases, prm)):
        if i in skip:
            continue
        st, ref, _ = O.compress(O.params(*f.shape, *_full(t)), f, pk)
        assert st == O.OK
        np.testing.assert_array_equal(B.stream(i).cpu().numpy(), ref, err_msg=f"frame {i}")
        st, yo = O.decompress(ref)
        assert st == O.OK
        np.testing.assert_array_equal(V.frames[i].cpu().numpy().view(np.uint32),
                                      yo.view(np.uint32), err_msg=f"frame {i}")


def test_verify_graph_mixed_batch(torch):
    # shapes, bin factors (b = 3 leaves ragged bins), both bin modes, the
    # Lorenzo dimensions, no peaks, windows off the panel, outliers (eb 0.02)
    cases = [synth.cspad_frame(21), synth.jungfrau_frame(7), synth.cspad_frame(22, npeaks=0),
             synth.tiny_case(61, (3, 70, 130), 6, "normal"),
             synth.tiny_case(62, (2, 80, 300), 10, "normal"),
             synth.tiny_case(63, (2, 9, 9), 3, "int"), synth.tiny_case(64, (1, 1, 1), 1, "normal")]
    prm = [(17, 2, 10.0, 0), (25, 4, 10.0, 0), (17, 2, 5.0, 0, 1), (7, 3, 1.0, 1),
           (7, 2, 0.02, 0, 3), (5, 3, 0.5, 1), (1, 1, 1.0, 0)]
    frames = [_gpu(torch, f) for f, _ in cases]
    peaks = [_gpu(torch, p) for _, p in cases]
    B = rsz.Batch(frames, peaks, prm)
    B.prepare()
    V = rsz.Verify(B)
    V.graph()
    for rep in range(3):
        print(f"replay {rep}", flush=True)
        V.replay()
        torch.cuda.synchronize()
        assert B.status.cpu().tolist() == [0] * len(cases)
        assert V.bad_counts() == [0] * len(cases)
        _check_against_oracle(torch, B, V, cases, prm)
        # eager work between replays, then new contents for the next one
        B.run()
        torch.cuda.synchronize()
        for f in frames:
            f.mul_(1.0 + 0.25 * (rep + 1))
        cases = [(f.cpu().numpy(), p) for f, (_, p) in zip(frames, cases)]


def test_verify_reports_frames_it_cannot_check(torch):
    good, gp = synth.tiny_case(65, (2, 40, 60), 4, "normal", scale=50.0)
    cases = [(good, gp), (good, np.array([[5, 0, 0]], np.int32)), (good, gp), (good, gp)]
    prm = [(5, 2, 1.0, 0), (5, 2, 1.0, 0), (5, 2, 1.0, 0, 2, 1), (5, 2, 1.0, 0)]
    frames = [_gpu(torch, f) for f, _ in cases]
    peaks = [_gpu(torch, p) for _, p in cases]
    B = rsz.Batch(frames, peaks, prm)
    B.prepare()
    V = rsz.Verify(B)
    B.launch()
    V.launch()
    torch.cuda.synchronize()
    # frame 1: a peak outside the frame (compression fails); frame 2: ROI coded
    assert B.status.cpu().tolist() == [0, rsz.RSZ_ERR_PEAK, 0, 0]
    assert V.bad_counts() == [0, NOT_VERIFIED, NOT_VERIFIED, 0]
    _check_against_oracle(torch, B, V, cases, prm, skip=(1, 2))
