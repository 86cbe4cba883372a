"""Seeded synthetic detector frames and peak lists.

These stand in for the LCLS datasets the paper evaluates on (Se-SAD on a CSPAD
32x185x388 detector, lysozyme on a Jungfrau-4M 8x512x1024 detector; Sec. V-B),
which are not available.  This module only draws inputs: it holds none of the
compression arithmetic, and both the HIP path and the CPU oracle are fed the
same arrays from it.

Every frame is drawn from ``numpy.random.default_rng([2206, 11297, workload,
index])`` (PCG64), accumulated in float64 and cast to float32 once.  Peaks are
int32 (panel, row, col) triples.

Workloads (sizes from the paper's detectors):
  * ``cspad``: N(0, 2^2) noise + smooth water ring 40*exp(-(rho-300)^2/(2*30^2)),
    rho = distance from the centre of the 8x4 panel mosaic (1480 x 1552 pixels);
    Bragg peaks as 2D Gaussians, sigma in U[0.8, 1.5] px, amplitude
    log-uniform in [200, 5000] ADU, stamped within +-8 px of the centre.
  * ``jungfrau``: 40 ADU x Poisson(0.3) photons + N(0, 3^2) read noise, same
    peak shape.
"""
import math

import numpy as np

CSPAD = (32, 185, 388)
JUNGFRAU4M = (8, 512, 1024)
JUNGFRAU16M = (16, 512, 1024)
SQUARE4M = (1, 2048, 2048)

W_CSPAD, W_JF, W_BATCH, W_JF16, W_SERVE, W_TINY = 0, 2, 1, 4, 3, 99


def rng_for(workload, index):
    return np.random.default_rng([2206, 11297, int(workload), int(index)])


def _mosaic_origin(shape):
    """Panel origins when panels tile a mosaic 4 panels wide (the 8x4 CSPAD
    layout); other detectors stack panels vertically in 2 columns."""
    P, H, W = shape
    cols = 4 if P % 4 == 0 else (2 if P % 2 == 0 else 1)
    rows = P // cols
    org = [((p // cols) * H, (p % cols) * W) for p in range(P)]
    return org, rows * H, cols * W


def _ring(shape):
    P, H, W = shape
    org, MH, MW = _mosaic_origin(shape)
    cy, cx = MH / 2.0, MW / 2.0
    ii = np.arange(H, dtype=np.float64)[:, None]
    jj = np.arange(W, dtype=np.float64)[None, :]
    out = np.empty(shape, np.float64)
    for p in range(P):
        rho = np.sqrt((ii + org[p][0] - cy) ** 2 + (jj + org[p][1] - cx) ** 2)
        out[p] = 40.0 * np.exp(-((rho - 300.0) ** 2) / (2.0 * 30.0 ** 2))
    return out


_RING_CACHE = {}


def _stamp_peaks(frame, rng, npeaks):
    """Draw npeaks Bragg peaks, add them to the float64 frame, return the list."""
    P, H, W = frame.shape
    pan = rng.integers(0, P, npeaks)
    row = rng.integers(0, H, npeaks)
    col = rng.integers(0, W, npeaks)
    sig = rng.uniform(0.8, 1.5, npeaks)
    amp = np.exp(rng.uniform(math.log(200.0), math.log(5000.0), npeaks))
    for k in range(npeaks):
        i0, i1 = max(0, row[k] - 8), min(H, row[k] + 9)
        j0, j1 = max(0, col[k] - 8), min(W, col[k] + 9)
        di = (np.arange(i0, i1) - row[k])[:, None].astype(np.float64)
        dj = (np.arange(j0, j1) - col[k])[None, :].astype(np.float64)
        frame[pan[k], i0:i1, j0:j1] += amp[k] * np.exp(-(di ** 2 + dj ** 2) / (2.0 * sig[k] ** 2))
    return np.stack([pan, row, col], axis=1).astype(np.int32)


def cspad_frame(index, npeaks=60, workload=W_CSPAD, shape=CSPAD):
    """One CSPAD-like frame (float32 [P,H,W]) and its peak list (int32 [n,3])."""
    rng = rng_for(workload, index)
    f = rng.standard_normal(shape) * 2.0
    key = tuple(shape)
    if key not in _RING_CACHE:
        _RING_CACHE[key] = _ring(shape)
    f += _RING_CACHE[key]
    peaks = _stamp_peaks(f, rng, npeaks)
    return f.astype(np.float32), peaks


def jungfrau_frame(index, shape=JUNGFRAU4M, npeaks=None, workload=W_JF, max_peaks=None):
    """One Jungfrau-like frame: 40 ADU x Poisson(0.3) + N(0, 3^2), peaks stamped.

    npeaks defaults to round(exp(U[ln 20, ln 800])); with max_peaks it is
    uniform in [0, max_peaks]."""
    rng = rng_for(workload, index)
    if npeaks is None:
        if max_peaks is None:
            npeaks = int(round(math.exp(rng.uniform(math.log(20.0), math.log(800.0)))))
        else:
            npeaks = int(rng.integers(0, max_peaks + 1))
    f = 40.0 * rng.poisson(0.3, shape).astype(np.float64)
    f += rng.standard_normal(shape) * 3.0
    peaks = _stamp_peaks(f, rng, npeaks)
    return f.astype(np.float32), peaks


def batch_peak_counts(nframes, mean=60, nonhit_fraction=0.2, workload=W_BATCH):
    """Peak counts for a batch of CSPAD frames: exactly round(nonhit_fraction *
    nframes) seeded-chosen frames have 0 peaks, the others Poisson(mean)."""
    rng = np.random.default_rng([2206, 11297, int(workload), 1 << 30])
    counts = rng.poisson(mean, nframes)
    zero = rng.permutation(nframes)[: int(round(nonhit_fraction * nframes))]
    counts[zero] = 0
    return counts.astype(np.int64)


def batch_frame(index, counts):
    """Frame `index` of the 1000-frame CSPAD batch workload."""
    return cspad_frame(index, npeaks=int(counts[index]), workload=W_BATCH)


def tiny_case(seed, shape, npeaks, kind="normal", scale=20.0):
    """Small frames for brute-force checks.

    kind: 'normal' (N(0, scale^2)), 'int' (small integers: exact ties in the
    quantiser), 'special' (mix of -0.0, denormals, huge and tiny magnitudes),
    'const' (one value everywhere).  Peaks anywhere in the frame, including
    edges, corners and duplicates."""
    rng = np.random.default_rng([2206, 11297, W_TINY, int(seed)])
    P, H, W = shape
    if kind == "normal":
        f = rng.standard_normal(shape) * scale
    elif kind == "int":
        f = rng.integers(-40, 41, shape).astype(np.float64)
    elif kind == "const":
        f = np.full(shape, float(rng.integers(-100, 101)) * 0.5)
    elif kind == "special":
        pool = np.array([0.0, -0.0, 1e-45, -1e-45, 1.4e-45 * 3, 1e-38, 3.0e5, -2.5e5,
                         0.5, 1.5, 2.5, -0.5, 1e-7, 123.456, -77.25, 1e4], np.float64)
        f = pool[rng.integers(0, pool.size, shape)]
    else:
        raise ValueError(kind)
    f = f.astype(np.float32)
    pan = rng.integers(0, P, npeaks)
    row = rng.integers(0, H, npeaks)
    col = rng.integers(0, W, npeaks)
    peaks = np.stack([pan, row, col], axis=1).astype(np.int32)
    if npeaks >= 2:  # force a duplicate and a corner peak
        peaks[-1] = peaks[0]
        peaks[-2] = (P - 1, H - 1, W - 1)
    return f, peaks
