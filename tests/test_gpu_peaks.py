"""GPU parity of the peak finder (the step before the path, Sec. IV-B) and of
the frames-in, streams-out pipeline with non-hit rejection (Sec. IV),
through the C ABI, against the oracle: peak lists (raster order) and counts
bit for bit, statuses, and the streams of the hits."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import rsz_oracle as O
from paper_2206_11297_amd import rsz, synth
from tests.test_oracle_peaks import spots

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


def _oracle_q(q):
    return O.peak_params(**{name: getattr(q, name) for name, _ in rsz.rsz_peak_params._fields_
                            if name != "reserved"})


def _check_batch(torch, frames, q, max_peaks=4096):
    B = rsz.PeakBatch([_gpu(torch, f) for f in frames], q, max_peaks)
    B.run()
    torch.cuda.synchronize()
    counts = B.counts.cpu().tolist()
    assert B.status.cpu().tolist() == [0] * len(frames)
    oq = _oracle_q(q)
    for i, f in enumerate(frames):
        ref, n = O.find_peaks(oq, f)
        assert counts[i] == n, f"frame {i}"
        np.testing.assert_array_equal(B.peaks(i, counts).cpu().numpy(), ref, err_msg=f"frame {i}")
    return counts


def _random_frames(seed, k):
    out = []
    for s in range(k):
        rng = np.random.default_rng([seed, s])
        shape = (int(rng.integers(1, 4)), int(rng.integers(1, 70)), int(rng.integers(1, 90)))
        n = int(rng.integers(0, 30))
        centres = [(int(rng.integers(0, shape[0])), int(rng.integers(0, shape[1])),
                    int(rng.integers(0, shape[2]))) for _ in range(n)]
        out.append(spots(shape, centres, s, noise=float(rng.choice([0.5, 2.0, 8.0])),
                         sigma=(0.4, float(rng.choice([0.8, 1.6])))))
    return out


def test_random_frames_one_batch(torch):
    """40 frames of random shapes (widths not a multiple of 4, single rows and
    columns), spots at edges and corners, in one batched launch."""
    frames = _random_frames(11, 40)
    counts = _check_batch(torch, frames, rsz.peak_params())
    assert sum(counts) > 50


@pytest.mark.parametrize("kw", [dict(pix_nsigma=0.0), dict(rank=2, ring_in=3, ring_out=6,
                                                            pix_nsigma=1.5),
                                dict(rank=1, ring_in=2, ring_out=2, pix_nsigma=5.0),
                                dict(npix_min=1, npix_max=49, amax_min=100.0, atot_min=0.0,
                                     snr_min=0.0)])
def test_other_parameters(torch, kw):
    _check_batch(torch, _random_frames(12, 12), rsz.peak_params(**kw))


def test_special_values_and_plateaus(torch):
    f = np.random.default_rng(5).normal(0.0, 1.0, (2, 40, 41)).astype(np.float32)
    f[0, 10, 10] = f[0, 10, 11] = 800.0                   # plateau
    f[0, 0, 0], f[0, 0, 1] = 900.0, 500.0                 # corner
    f[0, 30, 30], f[0, 30, 31] = 1000.0, 400.0
    f[0, 28, 28] = np.nan                                 # NaN inside that window
    f[1, 20, 20], f[1, 20, 21] = np.inf, 500.0            # infinite maximum
    f[1, 5, 35], f[1, 5, 36] = 2000.0, 900.0
    f[1, 2, 33] = -np.inf                                 # in that ring
    f[1, 39, 40], f[1, 38, 40] = 700.0, 650.0             # last pixel of the frame
    _check_batch(torch, [f], rsz.peak_params())


def test_synthetic_frames(torch):
    counts = synth.batch_peak_counts(1000)
    frames = [synth.batch_frame(i, counts)[0] for i in range(20)]
    frames += [synth.jungfrau_frame(i)[0] for i in range(3)]
    c = _check_batch(torch, frames, rsz.peak_params())
    assert max(c) >= 10


def test_capacity_and_bad_descriptors(torch):
    f = spots((1, 60, 60), [(0, 10 * a + 5, 10 * b + 5) for a in range(6) for b in range(6)], 3,
              noise=0.5, sigma=(0.5, 0.6), amp=(2000.0, 3000.0))
    ref, n = O.find_peaks(_oracle_q(rsz.peak_params()), f)
    assert n > 5
    g = _gpu(torch, f)
    B = rsz.PeakBatch([g, g, g], None, max_peaks=5)
    B.descs[2].max_peaks = 0                               # invalid for frame 2 only
    B.run()
    torch.cuda.synchronize()
    assert B.status.cpu().tolist() == [rsz.RSZ_ERR_CAPACITY, rsz.RSZ_ERR_CAPACITY, rsz.RSZ_ERR_ARG]
    assert B.counts.cpu().tolist() == [n, n, 0]
    B2 = rsz.PeakBatch([g], None, max_peaks=n)
    B2.run()
    torch.cuda.synchronize()
    assert B2.status.cpu().tolist() == [0]
    np.testing.assert_array_equal(B2.peaks(0).cpu().numpy(), ref)


def test_frames_in_streams_out(torch):
    """Peaks found on the GPU, frames with fewer than 10 rejected, the hits
    compressed with their found peaks: the hits and every stream equal the
    oracle's peak finder followed by the oracle's compressor."""
    counts = synth.batch_peak_counts(1000)
    host = [synth.batch_frame(i, counts)[0] for i in range(24)]
    frames = [_gpu(torch, f) for f in host]
    hits, B, P = rsz.compress_hits(frames, (17, 2, 10.0, 0))
    torch.cuda.synchronize()
    oq = _oracle_q(rsz.peak_params())
    ref_hits = []
    for i, f in enumerate(host):
        pk, n = O.find_peaks(oq, f)
        if n >= 10:
            ref_hits.append(i)
            st, ref, _ = O.compress(O.params(32, 185, 388, 17, 2, 10.0), f, pk)
            assert st == O.OK
            np.testing.assert_array_equal(B.stream(hits.index(i)).cpu().numpy(), ref)
    assert hits == ref_hits and len(hits) > 0
    assert (B.status.cpu().numpy() == 0).all()


def test_full_batch_1000_cspad(torch):
    """The 1000-frame CSPAD batch in one launch sequence: every frame's list
    equals the oracle's."""
    counts = synth.batch_peak_counts(1000)
    with ThreadPoolExecutor(16) as ex:
        host = list(ex.map(lambda i: synth.batch_frame(i, counts)[0], range(1000)))
    print("cspad 1000 peak finding", flush=True)
    B = rsz.PeakBatch([_gpu(torch, f) for f in host], None, 1024)
    B.run()
    torch.cuda.synchronize()
    assert (B.status.cpu().numpy() == 0).all()
    got = B.counts.cpu().tolist()
    oq = _oracle_q(rsz.peak_params())
    with ThreadPoolExecutor(16) as ex:
        refs = list(ex.map(lambda f: O.find_peaks(oq, f), host))
    for i, (ref, n) in enumerate(refs):
        assert got[i] == n, f"frame {i}"
        np.testing.assert_array_equal(B.peaks(i, got).cpu().numpy(), ref, err_msg=f"frame {i}")
    # non-hit frames have no peak at all
    assert all(got[i] == 0 for i, c in enumerate(counts) if c == 0)
