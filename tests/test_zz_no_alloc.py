"""rsz_compress_noalloc (the entry point whose workspace is the library's
static per-GPU array) against rsz_compress with a caller workspace, through
the C ABI: byte-equal streams and sizes on two calls in a row, the second
with a smaller frame (so it runs over what the first left in the array),
and a frame too large for the array refused before any work is queued."""
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


def _both(torch, frame, peaks, w, b, eb):
    """(stream of rsz_compress, stream of rsz_compress_noalloc) for one frame."""
    p = rsz.params(*frame.shape, w, b, eb)
    npk = len(peaks)
    st, cap = rsz.rsz_max_compressed_bytes(p, npk)
    assert st == 0
    st, wsb = rsz.rsz_workspace_bytes(p, npk)
    assert st == 0 and wsb <= rsz.NOALLOC_SCRATCH_BYTES
    g = torch.from_numpy(frame).cuda()
    pk = torch.from_numpy(np.ascontiguousarray(peaks)).cuda() if npk else None
    pk_ptr = rsz._ptr(pk) if npk else None
    ws = rsz.workspace(wsb)
    out_a = torch.full((cap,), 0xA5, dtype=torch.uint8, device="cuda")
    out_b = torch.full((cap,), 0x5A, dtype=torch.uint8, device="cuda")
    s = rsz._stream()
    st, na = rsz.rsz_compress(p, rsz._ptr(g), pk_ptr, npk, rsz._ptr(out_a), cap, rsz._ptr(ws),
                              wsb, s)
    assert st == 0
    st, nb = rsz.rsz_compress_noalloc(p, rsz._ptr(g), pk_ptr, npk, rsz._ptr(out_b), cap, s)
    assert st == 0
    assert na == nb
    return out_a[:na].cpu().numpy(), out_b[:nb].cpu().numpy()


def test_noalloc_matches_workspace_entry_point_twice(torch):
    # call 1: a full CSPAD-shaped frame
    frame, peaks = synth.cspad_frame(3, npeaks=60)
    a, b = _both(torch, frame, peaks, 17, 2, 10.0)
    np.testing.assert_array_equal(a, b)
    # call 2: a smaller frame, other parameters, over the first call's scratch
    frame2, peaks2 = synth.tiny_case(41, (3, 70, 90), 7, "normal", scale=50.0)
    a2, b2 = _both(torch, frame2, peaks2, 5, 3, 1.0)
    np.testing.assert_array_equal(a2, b2)
    st, ref, _ = O.compress(O.params(3, 70, 90, 5, 3, 1.0), frame2, peaks2)
    assert st == O.OK
    np.testing.assert_array_equal(b2, ref)


def test_noalloc_refuses_frames_beyond_the_scratch(torch):
    p = rsz.params(1, 4096, 4096, 17, 1, 10.0)
    st, wsb = rsz.rsz_workspace_bytes(p, 0)
    assert st == 0 and wsb > rsz.NOALLOC_SCRATCH_BYTES
    g = torch.zeros(16, dtype=torch.float32, device="cuda")
    out = torch.zeros(256, dtype=torch.uint8, device="cuda")
    st, _ = rsz.rsz_compress_noalloc(p, rsz._ptr(g), None, 0, rsz._ptr(out), 256, rsz._stream())
    assert st == rsz.RSZ_ERR_WORKSPACE
    torch.cuda.synchronize()
