"""Determinism over poisoned memory: the workspace and the output buffers are
filled with a byte pattern (0xA5, as well as 0x00 and 0xFF) before each run,
and every run must give the same bytes, equal to the oracle's.  A kernel that
reads a word it has not written, or a race between workgroups, shows up as a
stream that changes with the pattern or between runs."""
import numpy as np
import pytest

from oracle import rsz_oracle as O
from paper_2206_11297_amd import rsz, synth

pytestmark = pytest.mark.gpu

PATTERNS = [0xA5] * 5 + [0x00, 0xFF]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    rsz.lib()
    return t


def _gpu(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_mixed_batch_over_poisoned_workspace(torch):
    # shapes, bin factors, bin modes, Lorenzo dimensions and the optional
    # ROI and run coding all in one batch
    cases = [synth.cspad_frame(11), synth.tiny_case(44, (2, 50, 90), 3, "normal"),
             synth.jungfrau_frame(5), synth.cspad_frame(12, npeaks=0),
             synth.tiny_case(45, (1, 1, 1), 1, "normal"), synth.tiny_case(46, (3, 70, 130), 6,
                                                                          "int"),
             synth.tiny_case(47, (2, 80, 300), 10, "normal")]
    prm = [(17, 2, 10.0, 0), (5, 3, 1.0, 1), (11, 4, 10.0, 0, 1), (17, 2, 5.0, 0, 3),
           (1, 1, 1.0, 0), (7, 2, 0.5, 0, 2, 1, 1), (7, 2, 0.02, 1, 2, 0, 1)]
    refs = []
    for (f, pk), t in zip(cases, prm):
        full = tuple(t) + (2, 0, 0)[len(t) - 4:]
        w, b, eb, mode, dim, roi, run = full
        st, ref, _ = O.compress(O.params(*f.shape, w, b, eb, mode, dim, roi, run), f, pk)
        assert st == O.OK
        refs.append(ref)
    frames = [_gpu(torch, f) for f, _ in cases]
    peaks = [_gpu(torch, p) for _, p in cases]
    B = rsz.Batch(frames, peaks, prm)
    for k, byte in enumerate(PATTERNS):
        print(f"mixed batch run {k} over 0x{byte:02X}", flush=True)
        B.ws.fill_(byte)
        B.out.fill_(byte)
        B.sizes.fill_(-1)
        B.status.fill_(-99)
        B.run()
        torch.cuda.synchronize()
        assert B.status.cpu().tolist() == [0] * len(cases)
        for i, ref in enumerate(refs):
            np.testing.assert_array_equal(B.stream(i).cpu().numpy(), ref,
                                          err_msg=f"run {k} frame {i}")
    # the batched decoder over a poisoned workspace and poisoned frames
    D = rsz.DecodeBatch([B.stream(i) for i in range(len(cases))])
    yrefs = []
    for ref in refs:
        st, yo = O.decompress(ref)
        assert st == O.OK
        yrefs.append(yo)
    for k, byte in enumerate(PATTERNS[:3]):
        print(f"batched decode run {k} over 0x{byte:02X}", flush=True)
        D.ws.fill_(byte)
        for f in D.frames:
            f.view(torch.uint8).fill_(byte)
        D.status.fill_(-99)
        D.run()
        torch.cuda.synchronize()
        assert D.status.cpu().tolist() == [0] * len(cases)
        for i, yo in enumerate(yrefs):
            np.testing.assert_array_equal(D.frames[i].cpu().numpy().view(np.uint32),
                                          yo.view(np.uint32), err_msg=f"run {k} frame {i}")


def test_cspad_frame_over_poisoned_workspace(torch):
    frame, peaks = synth.cspad_frame(13)
    w, b, eb = 17, 2, 10.0
    st, ref, _ = O.compress(O.params(*frame.shape, w, b, eb), frame, peaks)
    assert st == O.OK
    p = rsz.params(*frame.shape, w, b, eb)
    st, wsb = rsz.rsz_workspace_bytes(p, len(peaks))
    assert st == 0
    st, cap = rsz.rsz_max_compressed_bytes(p, len(peaks))
    assert st == 0
    g, pk = _gpu(torch, frame), _gpu(torch, peaks)
    ws = rsz.workspace(wsb)
    out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    for k, byte in enumerate(PATTERNS):
        print(f"cspad frame run {k} over 0x{byte:02X}", flush=True)
        ws.fill_(byte)
        out.fill_(byte)
        st, n = rsz.rsz_compress(p, rsz._ptr(g), rsz._ptr(pk), len(peaks), rsz._ptr(out), cap,
                                 rsz._ptr(ws), ws.numel(), rsz._stream())
        assert st == 0 and n == ref.size
        np.testing.assert_array_equal(out[:n].cpu().numpy(), ref, err_msg=f"run {k}")
