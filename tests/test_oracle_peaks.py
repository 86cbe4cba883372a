"""Pins of the oracle's peak finder (Sec. IV-B's peak_finder_v3 parameters:
7x7 local maxima, maximum >= 300 ADU, total > 600 ADU, signal to noise > 10,
2-30 peak pixels; non-hit rejection below 10 peaks, Sec. IV).

An independent definition is written here with numpy and scipy: window
maxima by explicit comparison, the peak pixels as the 4-connected component
(scipy.ndimage.label) of the cut mask, the background by numpy mean/std, the
cuts and the signal to noise with square roots.  The oracle compares squares
instead; the two agree except at exact ties of the squared forms, which
random data does not produce.  Hand-built cases pin each criterion."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import rsz_oracle as O
from paper_2206_11297_amd import synth


def reference_peaks(frame, h=3, ring_in=4, ring_out=5, npix_min=2, npix_max=30, amax=300.0,
                    atot=600.0, snr=10.0, k=3.0):
    out = []
    P, H, W = frame.shape
    four = ndimage.generate_binary_structure(2, 1)
    for p in range(P):
        x = frame[p]
        for i in range(H):
            for j in range(W):
                c = x[i, j]
                if not float(c) >= amax:
                    continue
                i0, i1, j0, j1 = max(0, i - h), min(H, i + h + 1), max(0, j - h), min(W, j + h + 1)
                win = x[i0:i1, j0:j1]
                # maximum; on a plateau the first pixel in raster order
                flat = [(u, v) for u in range(i0, i1) for v in range(j0, j1)]
                if any(x[u, v] > c for u, v in flat):
                    continue
                if any(x[u, v] == c for u, v in flat if (u, v) < (i, j)):
                    continue
                if any(np.isnan(x[u, v]) for u, v in flat):
                    continue
                uu, vv = np.mgrid[max(0, i - ring_out):min(H, i + ring_out + 1),
                                  max(0, j - ring_out):min(W, j + ring_out + 1)]
                ring = np.maximum(np.abs(uu - i), np.abs(vv - j)) >= ring_in
                bg = x[uu[ring], vv[ring]].astype(np.float64)
                if bg.size == 0:
                    continue
                mu, sd = bg.mean(), bg.std()
                cut = (win.astype(np.float64) - mu) > k * sd
                lab, _ = ndimage.label(cut, structure=four)
                lc = lab[i - i0, j - j0]
                if lc == 0:
                    continue
                comp = lab == lc
                n = int(comp.sum())
                S = float(win[comp].astype(np.float64).sum())
                num = S - n * mu
                son = np.inf if sd == 0 and num > 0 else (num / (sd * np.sqrt(n)) if sd > 0 else -np.inf)
                if npix_min <= n <= npix_max and S > atot and son > snr:
                    out.append((p, i, j))
    return np.array(out, np.int32).reshape(-1, 3)


def spots(shape, centres, seed, noise=2.0, sigma=(0.5, 0.9), amp=(300.0, 3000.0)):
    rng = np.random.default_rng(seed)
    f = rng.normal(0.0, noise, shape)
    P, H, W = shape
    yy, xx = np.mgrid[0:H, 0:W]
    for p, r, c in centres:
        s = rng.uniform(*sigma)
        a = rng.uniform(*amp)
        f[p] += a * np.exp(-((yy - r) ** 2 + (xx - c) ** 2) / (2 * s * s))
    return f.astype(np.float32)


@pytest.mark.parametrize("seed", range(12))
def test_random_spot_frames_match_reference(seed):
    rng = np.random.default_rng(100 + seed)
    shape = (int(rng.integers(1, 4)), int(rng.integers(10, 60)), int(rng.integers(10, 80)))
    n = int(rng.integers(0, 25))
    centres = [(int(rng.integers(0, shape[0])), int(rng.integers(0, shape[1])),
                int(rng.integers(0, shape[2]))) for _ in range(n)]
    frame = spots(shape, centres, seed, noise=float(rng.choice([0.5, 2.0, 8.0])),
                  sigma=(0.4, float(rng.choice([0.8, 1.6]))))
    q = O.peak_params()
    got, cnt = O.find_peaks(q, frame)
    np.testing.assert_array_equal(got, reference_peaks(frame))
    assert cnt == got.shape[0]


@pytest.mark.parametrize("k,rank,ring", [(0.0, 3, (4, 5)), (1.5, 2, (3, 6)), (5.0, 1, (2, 2))])
def test_other_parameters_match_reference(k, rank, ring):
    frame = spots((2, 50, 70), [(0, 10, 10), (0, 11, 30), (1, 0, 0), (1, 49, 69), (0, 25, 40),
                                (1, 20, 20), (1, 22, 23)], 7, noise=1.0)
    q = O.peak_params(rank=rank, ring_in=ring[0], ring_out=ring[1], pix_nsigma=k)
    got, _ = O.find_peaks(q, frame)
    np.testing.assert_array_equal(got, reference_peaks(frame, h=rank, ring_in=ring[0],
                                                       ring_out=ring[1], k=k))


def _flat(shape=(1, 30, 30), noise_seed=3, noise=1.0):
    return np.random.default_rng(noise_seed).normal(0.0, noise, shape).astype(np.float32)


def test_each_criterion():
    q = O.peak_params()
    # a compact spot: accepted at its centre
    f = _flat()
    f[0, 15, 15] = 1000.0
    f[0, 15, 16] = 400.0
    got, _ = O.find_peaks(q, f)
    assert got.tolist() == [[0, 15, 15]]
    # one pixel alone: fewer than 2 peak pixels
    f = _flat()
    f[0, 15, 15] = 1000.0
    assert O.find_peaks(q, f)[1] == 0
    # a diagonal neighbour is not 4-connected: still one peak pixel
    f = _flat()
    f[0, 15, 15] = 1000.0
    f[0, 16, 16] = 400.0
    assert O.find_peaks(q, f)[1] == 0
    # exact totals on a flat zero background: 600 is not above 600, 601 is
    f = np.zeros((1, 30, 30), np.float32)
    f[0, 15, 15] = 350.0
    f[0, 15, 16] = 250.0
    assert O.find_peaks(q, f)[1] == 0
    f[0, 15, 16] = 251.0
    assert O.find_peaks(q, f)[1] == 1
    # a maximum of exactly 300 is kept ("below 300" is rejected)
    f = np.zeros((1, 30, 30), np.float32)
    f[0, 15, 15] = 300.0
    f[0, 15, 16] = f[0, 14, 15] = 299.0
    assert O.find_peaks(q, f)[1] == 1
    # maximum below 300
    f = _flat()
    f[0, 15, 15] = 299.0
    f[0, 15, 16] = 299.0
    f[0, 14, 15] = 299.0
    assert O.find_peaks(q, f)[1] == 0
    # total not above 600: 310 + 200 + noise
    f = _flat(noise=0.001)
    f[0, 15, 15] = 310.0
    f[0, 15, 16] = 200.0
    assert O.find_peaks(q, f)[1] == 0
    f[0, 15, 16] = 300.0
    assert O.find_peaks(q, f)[1] == 1
    # more than 30 peak pixels: a broad bright blob filling the window
    f = _flat()
    f[0, 12:19, 12:19] += 500.0
    f[0, 15, 15] += 100.0
    assert O.find_peaks(q, f)[1] == 0
    # signal to noise: the same spot on a very noisy ring is rejected
    f = _flat(noise=200.0)
    f[0, 15, 15] = 1000.0
    f[0, 15, 16] = 700.0
    f[0, 10:21, 10:21] = np.clip(f[0, 10:21, 10:21], -400, 250)
    f[0, 15, 15] = 1000.0
    f[0, 15, 16] = 700.0
    ok, _ = O.find_peaks(q, f)
    assert ok.tolist() == reference_peaks(f).tolist()


def test_plateau_gives_first_pixel_and_edges():
    q = O.peak_params()
    f = _flat(noise=0.1)
    f[0, 10, 10] = f[0, 10, 11] = 800.0      # plateau: (10, 10) wins
    f[0, 0, 0] = 900.0                        # corner, clipped window and ring
    f[0, 0, 1] = 500.0
    f[0, 29, 20] = 700.0                      # bottom edge
    f[0, 28, 20] = 300.0
    got, _ = O.find_peaks(q, f)
    assert got.tolist() == [[0, 0, 0], [0, 10, 10], [0, 29, 20]]
    np.testing.assert_array_equal(got, reference_peaks(f))


def test_no_ring_no_peak_and_nan_neighbours():
    q = O.peak_params()
    f = np.zeros((1, 5, 5), np.float32)       # every pixel within distance 2 of the
    f[0, 2, 2] = 1000.0                       # centre: the ring (4..5) is empty
    f[0, 2, 3] = 500.0
    assert O.find_peaks(q, f)[1] == 0
    f = _flat()
    f[0, 15, 15] = 1000.0
    f[0, 15, 16] = 500.0
    f[0, 13, 13] = np.nan                      # a NaN in the window blocks the maximum
    assert O.find_peaks(q, f)[1] == 0


def test_synthetic_frames_every_peak_is_a_stamped_peak():
    """Noise never reaches 300 ADU on the synthetic frames, so every peak
    found sits on a stamped Bragg peak (within 2 px); non-hit frames give no
    peaks."""
    q = O.peak_params()
    counts = synth.batch_peak_counts(1000)
    for i in (0, 1, 2, 3, 4, 5):
        f, pk = synth.batch_frame(i, counts)
        got, n = O.find_peaks(q, f)
        truth = pk.tolist()
        if not truth:
            assert n == 0
        for p, r, c in got.tolist():
            assert any(t[0] == p and abs(t[1] - r) <= 2 and abs(t[2] - c) <= 2 for t in truth)


def test_capacity_and_parameter_checks():
    f = spots((1, 60, 60), [(0, 10 * a + 5, 10 * b + 5) for a in range(6) for b in range(6)], 3,
              noise=0.5, sigma=(0.5, 0.6), amp=(2000.0, 3000.0))
    q = O.peak_params()
    full, n = O.find_peaks(q, f)
    assert n == full.shape[0] > 10
    part, n2 = O.find_peaks(q, f, cap=5)
    assert n2 == n and part.shape[0] == 5
    np.testing.assert_array_equal(part, full[:5])
    assert O.check_peak_params(q) == O.OK
    for bad in (dict(rank=0), dict(rank=4), dict(ring_in=3), dict(ring_out=3, ring_in=4),
                dict(ring_out=16), dict(npix_min=31), dict(snr_min=-1.0),
                dict(pix_nsigma=float("nan"))):
        assert O.check_peak_params(O.peak_params(**bad)) == O.ERR_ARG, bad
