"""ctypes binding of the C oracle (librsz_oracle.so) -- TEST INFRASTRUCTURE ONLY.

Host numpy arrays in, host numpy arrays out.  Status codes are the C ones:
0 OK, -1 ARG, -2 PEAK, -3 RANGE, -4 CAPACITY, -5 CORRUPT.
"""
import ctypes as C
import os

import numpy as np

from .build import LIB, build_oracle

OK, ERR_ARG, ERR_PEAK, ERR_RANGE, ERR_CAPACITY, ERR_CORRUPT = 0, -1, -2, -3, -4, -5
NSYM = 1024
CHUNK = 4096


class Params(C.Structure):
    _fields_ = [("panels", C.c_uint32), ("height", C.c_uint32), ("width", C.c_uint32),
                ("window", C.c_uint32), ("bin", C.c_uint32), ("bin_mode", C.c_uint32),
                ("eb", C.c_double), ("dim", C.c_uint32), ("roi_coding", C.c_uint32),
                ("run_coding", C.c_uint32), ("reserved", C.c_uint32)]


class PeakParams(C.Structure):
    _fields_ = [("rank", C.c_uint32), ("ring_in", C.c_uint32), ("ring_out", C.c_uint32),
                ("npix_min", C.c_uint32), ("npix_max", C.c_uint32), ("reserved", C.c_uint32),
                ("amax_min", C.c_double), ("atot_min", C.c_double), ("snr_min", C.c_double),
                ("pix_nsigma", C.c_double)]


def peak_params(rank=3, ring_in=4, ring_out=5, npix_min=2, npix_max=30, amax_min=300.0,
                atot_min=600.0, snr_min=10.0, pix_nsigma=3.0):
    return PeakParams(rank, ring_in, ring_out, npix_min, npix_max, 0, amax_min, atot_min,
                      snr_min, pix_nsigma)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        L = C.CDLL(LIB)
        P = C.POINTER
        vp = C.c_void_p
        L.ro_check_params.argtypes = [P(Params), C.c_uint32]
        L.ro_max_bytes.argtypes = [P(Params), C.c_uint32, P(C.c_uint64)]
        L.ro_intermediates.argtypes = [P(Params), vp, vp, C.c_uint32] + [vp] * 14 + [P(C.c_uint64)]
        L.ro_compress.argtypes = [P(Params), vp, vp, C.c_uint32, vp, C.c_uint64, P(C.c_uint64)]
        L.ro_decompress.argtypes = [vp, C.c_uint64, vp, C.c_uint64]
        L.ro_stream_info.argtypes = [vp, C.c_uint64, P(Params), P(C.c_uint32), P(C.c_uint64)]
        L.ro_huffman_lengths.argtypes = [vp, vp]
        L.ro_canonical.argtypes = [vp, vp]
        L.ro_check_peak_params.argtypes = [P(PeakParams)]
        L.ro_find_peaks.argtypes = [P(PeakParams), C.c_uint32, C.c_uint32, C.c_uint32, vp, vp,
                                    C.c_uint64]
        L.ro_find_peaks.restype = C.c_uint64
        _lib = L
    return _lib


def params(panels, height, width, window, bin, eb, bin_mode=0, dim=2, roi_coding=0, run_coding=0):
    return Params(panels, height, width, window, bin, bin_mode, float(eb), dim, roi_coding,
                  run_coding, 0)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _peaks(peaks):
    pk = np.ascontiguousarray(np.asarray(peaks, dtype=np.int32).reshape(-1, 3))
    return pk, pk.shape[0]


def nbins(p):
    return p.panels * (-(-p.height // p.bin)) * (-(-p.width // p.bin))


def max_bytes(p, npeaks):
    out = C.c_uint64(0)
    st = lib().ro_max_bytes(C.byref(p), npeaks, C.byref(out))
    return st, out.value


def intermediates(p, frame, peaks):
    """All intermediates of compression as a dict (status under 'status')."""
    frame = np.ascontiguousarray(frame, dtype=np.float32)
    pk, npk = _peaks(peaks)
    nb = nbins(p)
    nc = -(-nb // CHUNK)
    wpr = -(-p.width // 32)
    d = dict(
        mask=np.zeros((p.panels, p.height, wpr), np.uint32),
        roi=np.zeros((npk, p.window, p.window), np.uint32),
        S=np.zeros(nb, np.float64), n=np.zeros(nb, np.uint32), q=np.zeros(nb, np.int32),
        r=np.zeros(nb, np.int32), codes=np.zeros(nb, np.uint16),
        out_idx=np.zeros(nb, np.uint32), out_res=np.zeros(nb, np.int32),
        hist=np.zeros(NSYM, np.uint32), lens=np.zeros(NSYM, np.uint8),
        cw=np.zeros(NSYM, np.uint32), chunk_off=np.zeros(nc, np.uint32))
    n_out = C.c_uint32(0)
    T = C.c_uint64(0)
    st = lib().ro_intermediates(
        C.byref(p), _ptr(frame), _ptr(pk), npk, _ptr(d["mask"]), _ptr(d["roi"]), _ptr(d["S"]),
        _ptr(d["n"]), _ptr(d["q"]), _ptr(d["r"]), _ptr(d["codes"]), _ptr(d["out_idx"]),
        _ptr(d["out_res"]), C.byref(n_out), _ptr(d["hist"]), _ptr(d["lens"]), _ptr(d["cw"]),
        _ptr(d["chunk_off"]), C.byref(T))
    d["status"] = st
    d["n_out"] = n_out.value
    d["out_idx"] = d["out_idx"][: n_out.value]
    d["out_res"] = d["out_res"][: n_out.value]
    d["T"] = T.value
    return d


def compress(p, frame, peaks, cap=None):
    """Returns (status, stream bytes as np.uint8 array, required size)."""
    frame = np.ascontiguousarray(frame, dtype=np.float32)
    pk, npk = _peaks(peaks)
    if cap is None:
        st, cap = max_bytes(p, npk)
        if st:
            return st, None, 0
    out = np.zeros(max(cap, 1), np.uint8)
    nbytes = C.c_uint64(0)
    st = lib().ro_compress(C.byref(p), _ptr(frame), _ptr(pk), npk, _ptr(out), cap,
                           C.byref(nbytes))
    if st:
        return st, None, nbytes.value
    return st, out[: nbytes.value].copy(), nbytes.value


def stream_info(stream):
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    p = Params()
    npk = C.c_uint32(0)
    total = C.c_uint64(0)
    st = lib().ro_stream_info(_ptr(stream), stream.size, C.byref(p), C.byref(npk),
                              C.byref(total))
    return st, p, npk.value, total.value


def decompress(stream):
    """Returns (status, frame as float32 [P,H,W] or None)."""
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    st, p, _, _ = stream_info(stream)
    if st:
        return st, None
    frame = np.zeros((p.panels, p.height, p.width), np.float32)
    st = lib().ro_decompress(_ptr(stream), stream.size, _ptr(frame), frame.size)
    return st, (frame if st == 0 else None)


def huffman_lengths(hist):
    hist = np.ascontiguousarray(hist, dtype=np.uint32)
    assert hist.size == NSYM
    lens = np.zeros(NSYM, np.uint8)
    lib().ro_huffman_lengths(_ptr(hist), _ptr(lens))
    return lens


def canonical(lens):
    lens = np.ascontiguousarray(lens, dtype=np.uint8)
    cw = np.zeros(NSYM, np.uint32)
    lib().ro_canonical(_ptr(lens), _ptr(cw))
    return cw


def check_peak_params(q):
    return lib().ro_check_peak_params(C.byref(q))


def find_peaks(q, frame, cap=1 << 16):
    """Peaks of a float32 [P,H,W] frame in raster order: (int32 [min(n,cap),3], n)."""
    frame = np.ascontiguousarray(frame, dtype=np.float32)
    P, H, W = frame.shape
    out = np.zeros((max(cap, 1), 3), np.int32)
    n = lib().ro_find_peaks(C.byref(q), P, H, W, _ptr(frame), _ptr(out), cap)
    return out[:min(n, cap)].copy(), n
