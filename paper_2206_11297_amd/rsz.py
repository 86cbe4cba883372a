"""Python binding of librsz (ctypes).  Argument marshalling only: every step of
the compression path runs in the HIP kernels of librsz.so.

Low-level functions mirror the C ABI names (include/rsz.h) and take raw device
pointers; the torch helpers below them allocate outputs and workspaces as
torch tensors on the current device and pass the current HIP stream.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsz.so")

RSZ_OK, RSZ_ERR_ARG, RSZ_ERR_PEAK, RSZ_ERR_RANGE = 0, -1, -2, -3
RSZ_ERR_CAPACITY, RSZ_ERR_CORRUPT, RSZ_ERR_WORKSPACE, RSZ_ERR_HIP = -4, -5, -6, -7
RSZ_BIN_BACKGROUND, RSZ_BIN_ALL = 0, 1

EXPORTS = ["rsz_status_string", "rsz_max_compressed_bytes", "rsz_workspace_bytes",
           "rsz_compress", "rsz_compress_noalloc", "rsz_batch_workspace_bytes",
           "rsz_compress_batch",
           "rsz_batch_prepare", "rsz_batch_launch", "rsz_batch_graph_create",
           "rsz_graph_launch", "rsz_graph_destroy",
           "rsz_verify_workspace_bytes", "rsz_verify_prepare", "rsz_verify_launch",
           "rsz_verify_graph_create",
           "rsz_stream_info", "rsz_decompress_workspace_bytes", "rsz_decompress",
           "rsz_decompress_batch_workspace_bytes", "rsz_decompress_batch",
           "rsz_debug_intermediates", "rsz_debug_codebook", "rsz_measure_read",
           "rsz_profile_enable", "rsz_profile_read", "rsz_profile_only",
           "rsz_peak_params_default",
           "rsz_find_peaks_workspace_bytes", "rsz_find_peaks_batch"]


class RszError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


class rsz_params(C.Structure):
    _fields_ = [("panels", C.c_uint32), ("height", C.c_uint32), ("width", C.c_uint32),
                ("window", C.c_uint32), ("bin", C.c_uint32), ("bin_mode", C.c_uint32),
                ("eb", C.c_double), ("dim", C.c_uint32), ("roi_coding", C.c_uint32),
                ("run_coding", C.c_uint32), ("reserved", C.c_uint32)]


class rsz_decode_desc(C.Structure):
    _fields_ = [("in", C.c_void_p), ("in_bytes", C.c_uint64), ("header", C.c_void_p),
                ("frame", C.c_void_p), ("frame_elems", C.c_uint64)]


class rsz_frame_desc(C.Structure):
    _fields_ = [("params", rsz_params), ("frame", C.c_void_p), ("peaks", C.c_void_p),
                ("npeaks", C.c_uint32), ("tile_rows", C.c_uint32), ("tile_strips", C.c_uint32),
                ("tile_waves", C.c_uint32), ("out", C.c_void_p),
                ("out_cap", C.c_uint64)]


class rsz_batch_plan(C.Structure):
    _fields_ = [("opaque", C.c_uint64 * 32)]


class rsz_verify_plan(C.Structure):
    _fields_ = [("opaque", C.c_uint64 * 32)]


class rsz_debug_bufs(C.Structure):
    _fields_ = [("mask", C.c_void_p), ("S", C.c_void_p), ("n", C.c_void_p), ("q", C.c_void_p),
                ("codes", C.c_void_p), ("hist", C.c_void_p), ("lens", C.c_void_p),
                ("cw", C.c_void_p), ("n_out", C.c_void_p), ("out_idx", C.c_void_p),
                ("out_res", C.c_void_p)]


class rsz_peak_params(C.Structure):
    _fields_ = [("rank", C.c_uint32), ("ring_in", C.c_uint32), ("ring_out", C.c_uint32),
                ("npix_min", C.c_uint32), ("npix_max", C.c_uint32), ("reserved", C.c_uint32),
                ("amax_min", C.c_double), ("atot_min", C.c_double), ("snr_min", C.c_double),
                ("pix_nsigma", C.c_double)]


class rsz_peak_desc(C.Structure):
    _fields_ = [("panels", C.c_uint32), ("height", C.c_uint32), ("width", C.c_uint32),
                ("max_peaks", C.c_uint32), ("frame", C.c_void_p), ("peaks", C.c_void_p)]


class rsz_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_uint32), ("total_ms", C.c_double)]


_lib = None


def lib():
    """Load librsz.so; fails loudly when the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P, vp, u32, u64 = C.POINTER, C.c_void_p, C.c_uint32, C.c_uint64
        L.rsz_status_string.restype = C.c_char_p
        L.rsz_status_string.argtypes = [C.c_int]
        L.rsz_max_compressed_bytes.argtypes = [P(rsz_params), u32, P(u64)]
        L.rsz_workspace_bytes.argtypes = [P(rsz_params), u32, P(u64)]
        L.rsz_compress.argtypes = [P(rsz_params), vp, vp, u32, vp, u64, P(u64), vp, u64, vp]
        L.rsz_compress_noalloc.argtypes = [P(rsz_params), vp, vp, u32, vp, u64, P(u64), vp]
        L.rsz_batch_workspace_bytes.argtypes = [u32, P(rsz_frame_desc), P(u64)]
        L.rsz_compress_batch.argtypes = [u32, P(rsz_frame_desc), vp, vp, vp, u64, vp]
        L.rsz_batch_prepare.argtypes = [u32, P(rsz_frame_desc), vp, vp, vp, u64, vp,
                                        P(rsz_batch_plan)]
        L.rsz_batch_launch.argtypes = [P(rsz_batch_plan), vp]
        L.rsz_batch_graph_create.argtypes = [P(rsz_batch_plan), vp, P(vp)]
        L.rsz_verify_workspace_bytes.argtypes = [P(rsz_batch_plan), u32, P(rsz_frame_desc),
                                                 P(u64)]
        L.rsz_verify_prepare.argtypes = [P(rsz_batch_plan), u32, P(rsz_frame_desc), P(vp), vp, vp,
                                         u64, vp, P(rsz_verify_plan)]
        L.rsz_verify_launch.argtypes = [P(rsz_verify_plan), vp]
        L.rsz_verify_graph_create.argtypes = [P(rsz_batch_plan), P(rsz_verify_plan), vp, P(vp)]
        L.rsz_graph_launch.argtypes = [vp, vp]
        L.rsz_graph_destroy.argtypes = [vp]
        L.rsz_stream_info.argtypes = [vp, u64, P(rsz_params), P(u32), P(u64)]
        L.rsz_decompress_workspace_bytes.argtypes = [vp, u64, P(u64)]
        L.rsz_decompress.argtypes = [vp, u64, vp, u64, vp, u64, vp]
        L.rsz_decompress_batch_workspace_bytes.argtypes = [u32, P(rsz_decode_desc), P(u64)]
        L.rsz_decompress_batch.argtypes = [u32, P(rsz_decode_desc), vp, vp, u64, vp]
        L.rsz_debug_intermediates.argtypes = [P(rsz_params), vp, vp, u32, P(rsz_debug_bufs), vp,
                                              u64, vp]
        L.rsz_debug_codebook.argtypes = [vp, vp, vp, vp, u64, vp]
        L.rsz_measure_read.argtypes = [vp, u64, vp, C.c_int, P(C.c_double), vp]
        L.rsz_profile_enable.argtypes = [C.c_int]
        L.rsz_profile_read.argtypes = [P(rsz_kernel_time), C.c_int, P(C.c_int)]
        L.rsz_profile_only.argtypes = [C.c_char_p]
        L.rsz_peak_params_default.restype = None
        L.rsz_peak_params_default.argtypes = [P(rsz_peak_params)]
        L.rsz_find_peaks_workspace_bytes.argtypes = [u32, P(rsz_peak_desc), P(u64)]
        L.rsz_find_peaks_batch.argtypes = [P(rsz_peak_params), u32, P(rsz_peak_desc), vp, vp, vp,
                                           u64, vp]
        _lib = L
    return _lib


def status_string(status):
    return lib().rsz_status_string(int(status)).decode()


def params(panels, height, width, window, bin, eb, bin_mode=RSZ_BIN_BACKGROUND, dim=2,
           roi_coding=0, run_coding=0):
    return rsz_params(panels, height, width, window, bin, bin_mode, float(eb), dim, roi_coding,
                      run_coding, 0)


# ------------------------------------------------------------ C ABI mirrors


def rsz_max_compressed_bytes(p, npeaks):
    out = C.c_uint64(0)
    st = lib().rsz_max_compressed_bytes(C.byref(p), npeaks, C.byref(out))
    return st, out.value


def rsz_workspace_bytes(p, npeaks):
    out = C.c_uint64(0)
    st = lib().rsz_workspace_bytes(C.byref(p), npeaks, C.byref(out))
    return st, out.value


def rsz_compress(p, d_frame, d_peaks, npeaks, d_out, out_cap, d_ws, ws_bytes, stream):
    nbytes = C.c_uint64(0)
    st = lib().rsz_compress(C.byref(p), d_frame, d_peaks, npeaks, d_out, out_cap,
                            C.byref(nbytes), d_ws, ws_bytes, stream)
    return st, nbytes.value


# RSZ_NOALLOC_SCRATCH_BYTES: the workspace size rsz_compress_noalloc holds per GPU
NOALLOC_SCRATCH_BYTES = 64 << 20


def rsz_compress_noalloc(p, d_frame, d_peaks, npeaks, d_out, out_cap, stream):
    nbytes = C.c_uint64(0)
    st = lib().rsz_compress_noalloc(C.byref(p), d_frame, d_peaks, npeaks, d_out, out_cap,
                                    C.byref(nbytes), stream)
    return st, nbytes.value


def _arr(cls, descs):
    """A C array of descriptors: `descs` itself when it already is one (the
    batch classes keep theirs, so a launch marshals nothing), else a copy."""
    if isinstance(descs, C.Array):
        return descs
    return (cls * len(descs))(*descs)


def rsz_batch_workspace_bytes(descs):
    arr = _arr(rsz_frame_desc, descs)
    out = C.c_uint64(0)
    st = lib().rsz_batch_workspace_bytes(len(descs), arr, C.byref(out))
    return st, out.value


def rsz_compress_batch(descs, d_out_bytes, d_status, d_ws, ws_bytes, stream):
    arr = _arr(rsz_frame_desc, descs)
    return lib().rsz_compress_batch(len(descs), arr, d_out_bytes, d_status, d_ws, ws_bytes,
                                    stream)


def rsz_batch_prepare(descs, d_out_bytes, d_status, d_ws, ws_bytes, stream):
    arr = _arr(rsz_frame_desc, descs)
    plan = rsz_batch_plan()
    st = lib().rsz_batch_prepare(len(descs), arr, d_out_bytes, d_status, d_ws, ws_bytes, stream,
                                 C.byref(plan))
    return st, plan


def rsz_batch_launch(plan, stream):
    return lib().rsz_batch_launch(C.byref(plan), stream)


def rsz_batch_graph_create(plan, stream):
    ex = C.c_void_p()
    st = lib().rsz_batch_graph_create(C.byref(plan), stream, C.byref(ex))
    return st, ex


def rsz_verify_workspace_bytes(plan, descs):
    arr = _arr(rsz_frame_desc, descs)
    out = C.c_uint64(0)
    st = lib().rsz_verify_workspace_bytes(C.byref(plan), len(descs), arr, C.byref(out))
    return st, out.value


def rsz_verify_prepare(plan, descs, frames_out, d_bad, d_ws, ws_bytes, stream):
    arr = _arr(rsz_frame_desc, descs)
    fo = (C.c_void_p * len(frames_out))(*frames_out)
    vplan = rsz_verify_plan()
    st = lib().rsz_verify_prepare(C.byref(plan), len(descs), arr, fo, d_bad, d_ws, ws_bytes,
                                  stream, C.byref(vplan))
    return st, vplan


def rsz_verify_launch(vplan, stream):
    return lib().rsz_verify_launch(C.byref(vplan), stream)


def rsz_verify_graph_create(plan, vplan, stream):
    ex = C.c_void_p(0)
    st = lib().rsz_verify_graph_create(C.byref(plan), C.byref(vplan), stream, C.byref(ex))
    return st, ex


def rsz_graph_launch(graph_exec, stream):
    return lib().rsz_graph_launch(graph_exec, stream)


def rsz_graph_destroy(graph_exec):
    return lib().rsz_graph_destroy(graph_exec)


def rsz_stream_info(h_bytes):
    buf = bytes(h_bytes)
    p = rsz_params()
    npk = C.c_uint32(0)
    total = C.c_uint64(0)
    st = lib().rsz_stream_info(buf, len(buf), C.byref(p), C.byref(npk), C.byref(total))
    return st, p, npk.value, total.value


def rsz_decompress_workspace_bytes(h_header):
    buf = bytes(h_header)
    out = C.c_uint64(0)
    st = lib().rsz_decompress_workspace_bytes(buf, len(buf), C.byref(out))
    return st, out.value


def rsz_decompress(d_in, in_bytes, d_frame, frame_elems, d_ws, ws_bytes, stream):
    return lib().rsz_decompress(d_in, in_bytes, d_frame, frame_elems, d_ws, ws_bytes, stream)


def _decode_descs(descs):
    arr = _arr(rsz_decode_desc, descs)
    return arr


def rsz_decompress_batch_workspace_bytes(descs):
    out = C.c_uint64(0)
    st = lib().rsz_decompress_batch_workspace_bytes(len(descs), _decode_descs(descs),
                                                    C.byref(out))
    return st, out.value


def rsz_decompress_batch(descs, d_status, d_ws, ws_bytes, stream):
    return lib().rsz_decompress_batch(len(descs), _decode_descs(descs), d_status, d_ws, ws_bytes,
                                      stream)


def rsz_debug_intermediates(p, d_frame, d_peaks, npeaks, bufs, d_ws, ws_bytes, stream):
    return lib().rsz_debug_intermediates(C.byref(p), d_frame, d_peaks, npeaks, C.byref(bufs),
                                         d_ws, ws_bytes, stream)


def debug_codebook(hist):
    """Code lengths and canonical codewords of a 1024-bin histogram from the
    GPU codebook kernel (numpy in, numpy out)."""
    import numpy as np
    torch = _torch()
    h = np.ascontiguousarray(hist, dtype=np.uint32)
    if h.size != 1024:
        raise ValueError("histogram must have 1024 bins")
    lens = np.zeros(1024, np.uint8)
    cw = np.zeros(1024, np.uint32)
    ws = workspace(16 << 10, torch.device("cuda", torch.cuda.current_device()))
    st = lib().rsz_debug_codebook(h.ctypes.data, lens.ctypes.data, cw.ctypes.data, _ptr(ws),
                                  ws.numel(), _stream())
    if st:
        raise RszError(st, "rsz_debug_codebook")
    return lens, cw


def measure_read(nbytes=1 << 32, reps=10):
    """GB/s of a plain streaming read over nbytes of device memory."""
    torch = _torch()
    buf = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda").fill_(1)
    sink = torch.zeros(1024, dtype=torch.int32, device="cuda")
    out = C.c_double(0.0)
    st = lib().rsz_measure_read(_ptr(buf), buf.numel(), _ptr(sink), int(reps), C.byref(out),
                                _stream())
    if st:
        raise RszError(st, "rsz_measure_read")
    return out.value


def rsz_profile_enable(on):
    return lib().rsz_profile_enable(1 if on else 0)


def rsz_profile_only(name=None):
    """Record only the launches of kernel `name` (None: every kernel)."""
    return lib().rsz_profile_only(name.encode() if name else None)


def rsz_profile_read(max_entries=64):
    arr = (rsz_kernel_time * max_entries)()
    n = C.c_int(0)
    st = lib().rsz_profile_read(arr, max_entries, C.byref(n))
    if st:
        raise RszError(st, "rsz_profile_read")
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms)
            for i in range(min(n.value, max_entries))}


# ------------------------------------------------------------ torch helpers


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_frame(frame, peaks):
    torch = _torch()
    if not frame.is_cuda or frame.dtype != torch.float32 or frame.dim() != 3:
        raise ValueError("frame must be a float32 [panels, height, width] GPU tensor")
    frame = frame.contiguous()
    if peaks is None:
        peaks = torch.zeros((0, 3), dtype=torch.int32, device=frame.device)
    peaks = peaks.to(device=frame.device, dtype=torch.int32).reshape(-1, 3).contiguous()
    return frame, peaks


def workspace(nbytes, device=None):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")


def compress(frame, peaks, window=17, bin=2, eb=10.0, bin_mode=RSZ_BIN_BACKGROUND, out=None,
             ws=None, dim=2, roi_coding=0, run_coding=0):
    """Compress one GPU frame; returns the stream as a uint8 GPU tensor.
    dim: Lorenzo predictor dimension (1, 2 or 3); roi_coding: 1 codes the ROI
    windows losslessly instead of storing them verbatim; run_coding: 1 Rice
    codes the zero runs of the Huffman bits."""
    torch = _torch()
    frame, peaks = _check_frame(frame, peaks)
    P, H, W = frame.shape
    p = params(P, H, W, window, bin, eb, bin_mode, dim, roi_coding, run_coding)
    npk = peaks.shape[0]
    st, cap = rsz_max_compressed_bytes(p, npk)
    if st:
        raise RszError(st, "rsz_max_compressed_bytes")
    st, wsb = rsz_workspace_bytes(p, npk)
    if st:
        raise RszError(st, "rsz_workspace_bytes")
    if out is None:
        out = torch.empty(cap, dtype=torch.uint8, device=frame.device)
    if ws is None or ws.numel() < wsb:
        ws = workspace(wsb, frame.device)
    st, nbytes = rsz_compress(p, _ptr(frame), _ptr(peaks) if npk else None, npk, _ptr(out),
                              out.numel(), _ptr(ws), ws.numel(), _stream())
    if st:
        raise RszError(st, "rsz_compress")
    return out[:nbytes]


def decompress(stream, ws=None):
    """Decompress a uint8 GPU stream; returns the float32 [P,H,W] GPU frame."""
    torch = _torch()
    stream = stream.contiguous()
    if stream.data_ptr() % 16:
        stream = stream.clone()
    head = stream[:80].cpu().numpy().tobytes()
    st, p, _, total = rsz_stream_info(head)
    if st:
        raise RszError(st, "rsz_stream_info")
    st, wsb = rsz_decompress_workspace_bytes(head)
    if st:
        raise RszError(st, "rsz_decompress_workspace_bytes")
    frame = torch.empty((p.panels, p.height, p.width), dtype=torch.float32, device=stream.device)
    if ws is None or ws.numel() < wsb:
        ws = workspace(wsb, stream.device)
    st = rsz_decompress(_ptr(stream), stream.numel(), _ptr(frame), frame.numel(), _ptr(ws),
                        ws.numel(), _stream())
    if st:
        raise RszError(st, "rsz_decompress")
    return frame


class DecodeBatch:
    """Many streams decompressed with one launch of each decoder kernel.

    streams: uint8 GPU tensors.  The headers are gathered to the host in one
    transfer; frames (float32 [P,H,W] GPU tensors), the status tensor and the
    workspace are allocated here.  run() queues the decompression
    (asynchronous); status[i] is stream i's status."""

    def __init__(self, streams):
        torch = _torch()
        self.streams = [s if s.data_ptr() % 16 == 0 else s.clone() for s in
                        (x.contiguous() for x in streams)]
        dev = self.streams[0].device
        n = len(self.streams)
        heads = torch.stack([torch.nn.functional.pad(s[:80], (0, max(0, 80 - s.numel())))
                             for s in self.streams]).cpu().numpy()
        self.headers = [C.create_string_buffer(heads[i].tobytes(), 80) for i in range(n)]
        self.frames = []
        for i, s in enumerate(self.streams):
            st, p, _, _ = rsz_stream_info(heads[i].tobytes())
            shape = (p.panels, p.height, p.width) if st == 0 else (1, 1, 1)
            self.frames.append(torch.empty(shape, dtype=torch.float32, device=dev))
        self.descs = [rsz_decode_desc(s.data_ptr(), s.numel(), C.addressof(h), f.data_ptr(),
                                      f.numel())
                      for s, h, f in zip(self.streams, self.headers, self.frames)]
        # kept as a C array: every call passes it as is
        self.descs = _arr(rsz_decode_desc, self.descs)
        st, wsb = rsz_decompress_batch_workspace_bytes(self.descs)
        if st:
            raise RszError(st, "rsz_decompress_batch_workspace_bytes")
        self.ws = workspace(wsb, dev)
        self.status = torch.zeros(n, dtype=torch.int32, device=dev)

    def run(self):
        st = rsz_decompress_batch(self.descs, _ptr(self.status), _ptr(self.ws), self.ws.numel(),
                                  _stream())
        if st:
            raise RszError(st, "rsz_decompress_batch")


def debug_intermediates(frame, peaks, window=17, bin=2, eb=10.0, bin_mode=RSZ_BIN_BACKGROUND,
                        dim=2):
    """All intermediates of compressing one frame as GPU tensors (dict)."""
    torch = _torch()
    frame, peaks = _check_frame(frame, peaks)
    P, H, W = frame.shape
    p = params(P, H, W, window, bin, eb, bin_mode, dim)
    npk = peaks.shape[0]
    Hb, Wb = -(-H // bin), -(-W // bin)
    nb = P * Hb * Wb
    dev = frame.device
    d = dict(mask=torch.zeros((P, H, -(-W // 32)), dtype=torch.int32, device=dev),
             S=torch.zeros(nb, dtype=torch.float64, device=dev),
             n=torch.zeros(nb, dtype=torch.int32, device=dev),
             q=torch.zeros(nb, dtype=torch.int32, device=dev),
             codes=torch.zeros(nb, dtype=torch.int16, device=dev),
             hist=torch.zeros(1024, dtype=torch.int32, device=dev),
             lens=torch.zeros(1024, dtype=torch.uint8, device=dev),
             cw=torch.zeros(1024, dtype=torch.int32, device=dev),
             n_out=torch.zeros(1, dtype=torch.int32, device=dev),
             out_idx=torch.zeros(max(nb, 1), dtype=torch.int32, device=dev),
             out_res=torch.zeros(max(nb, 1), dtype=torch.int32, device=dev))
    bufs = rsz_debug_bufs(*[d[k].data_ptr() for k in
                            ("mask", "S", "n", "q", "codes", "hist", "lens", "cw", "n_out",
                             "out_idx", "out_res")])
    st, wsb = rsz_workspace_bytes(p, npk)
    if st:
        raise RszError(st, "rsz_workspace_bytes")
    ws = workspace(wsb, dev)
    st = rsz_debug_intermediates(p, _ptr(frame), _ptr(peaks) if npk else None, npk, bufs,
                                 _ptr(ws), ws.numel(), _stream())
    d["status"] = st
    return d


class Batch:
    """Descriptors, output buffers and workspace for one batched launch.

    frames: list of float32 [P,H,W] GPU tensors; peaks: list of int32 [n,3]
    GPU tensors; params: list of (window, bin, eb, bin_mode[, dim[, roi_coding[,
    run_coding]]]) per frame or one tuple for all (dim, the Lorenzo dimension,
    defaults to 2; roi_coding to 0, the ROI windows verbatim; run_coding to 0,
    the Huffman bits verbatim).  Output buffers are sized by
    rsz_max_compressed_bytes and packed into one uint8 tensor."""

    def __init__(self, frames, peaks, prm, tile_rows=0, tile_strips=0, tile_waves=0):
        torch = _torch()
        self.frames = [f.contiguous() for f in frames]
        self.peaks = [pk.to(dtype=torch.int32).reshape(-1, 3).contiguous() for pk in peaks]
        n = len(self.frames)
        prm = prm if isinstance(prm, list) else [prm] * n
        self.params = []
        caps = []
        for f, pk, t in zip(self.frames, self.peaks, prm):
            P, H, W = f.shape
            p = params(P, H, W, *t)
            st, cap = rsz_max_compressed_bytes(p, pk.shape[0])
            if st:
                raise RszError(st, "rsz_max_compressed_bytes")
            self.params.append(p)
            caps.append((cap + 255) // 256 * 256)
        dev = self.frames[0].device
        self.offsets = [0]
        for c in caps:
            self.offsets.append(self.offsets[-1] + c)
        self.out = torch.empty(self.offsets[-1], dtype=torch.uint8, device=dev)
        self.caps = caps
        self.descs = []
        for i in range(n):
            d = rsz_frame_desc()
            d.params = self.params[i]
            d.frame = self.frames[i].data_ptr()
            d.peaks = self.peaks[i].data_ptr() if self.peaks[i].shape[0] else None
            d.npeaks = self.peaks[i].shape[0]
            d.tile_rows = int(tile_rows)
            d.tile_strips = int(tile_strips)
            d.tile_waves = int(tile_waves)
            d.out = self.out.data_ptr() + self.offsets[i]
            d.out_cap = caps[i]
            self.descs.append(d)
        # kept as a C array: every launch passes it as is
        self.descs = _arr(rsz_frame_desc, self.descs)
        st, wsb = rsz_batch_workspace_bytes(self.descs)
        if st:
            raise RszError(st, "rsz_batch_workspace_bytes")
        self.ws = workspace(wsb, dev)
        self.sizes = torch.zeros(n, dtype=torch.int64, device=dev)
        self.status = torch.zeros(n, dtype=torch.int32, device=dev)

    def run(self):
        """Queue one batched compression on the current stream (asynchronous)."""
        st = rsz_compress_batch(self.descs, _ptr(self.sizes), _ptr(self.status), _ptr(self.ws),
                                self.ws.numel(), _stream())
        if st:
            raise RszError(st, "rsz_compress_batch")

    def prepare(self):
        """Upload the plan once; launch() / graph() then replay only kernels."""
        st, self.plan = rsz_batch_prepare(self.descs, _ptr(self.sizes), _ptr(self.status),
                                          _ptr(self.ws), self.ws.numel(), _stream())
        if st:
            raise RszError(st, "rsz_batch_prepare")

    def launch(self):
        st = rsz_batch_launch(self.plan, _stream())
        if st:
            raise RszError(st, "rsz_batch_launch")

    def graph(self):
        """Capture the prepared batch into a HIP graph (replay with replay())."""
        torch = _torch()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        st, self.graph_exec = rsz_batch_graph_create(self.plan, C.c_void_p(side.cuda_stream))
        if st:
            raise RszError(st, "rsz_batch_graph_create")
        torch.cuda.current_stream().wait_stream(side)

    def replay(self):
        st = rsz_graph_launch(self.graph_exec, _stream())
        if st:
            raise RszError(st, "rsz_graph_launch")

    def __del__(self):
        ex = getattr(self, "graph_exec", None)
        if ex is not None and ex.value:
            try:
                rsz_graph_destroy(ex)
            except Exception:
                pass

    def stream(self, i, sizes=None):
        """Stream of frame i as a GPU uint8 view (after the stream finished)."""
        n = int(self.sizes[i]) if sizes is None else int(sizes[i])
        return self.out[self.offsets[i]:self.offsets[i] + n]


class Verify:
    """On-device verification of a prepared Batch (rsz_verify_*): every
    stream the batch writes decoded into frames of its own and every pixel
    checked against its frame.  launch() queues it after the batch's work;
    graph() captures the batch's launch and the verification into one HIP
    graph (replay()).  bad[i] (uint32 in an int32 tensor): frame i's failing
    pixels, 0xFFFFFFFF when a stage failed or the frame is not verified."""

    def __init__(self, B):
        torch = _torch()
        if getattr(B, "plan", None) is None:
            raise RuntimeError("Verify needs a prepared Batch (B.prepare())")
        self.B = B
        dev = B.frames[0].device
        self.frames = [torch.empty_like(f) for f in B.frames]
        self.bad = torch.zeros(len(B.frames), dtype=torch.int32, device=dev)
        st, wsb = rsz_verify_workspace_bytes(B.plan, B.descs)
        if st:
            raise RszError(st, "rsz_verify_workspace_bytes")
        self.ws = workspace(wsb, dev)
        st, self.vplan = rsz_verify_prepare(B.plan, B.descs, [f.data_ptr() for f in self.frames],
                                            _ptr(self.bad), _ptr(self.ws), self.ws.numel(),
                                            _stream())
        if st:
            raise RszError(st, "rsz_verify_prepare")
        self.graph_exec = None

    def launch(self):
        st = rsz_verify_launch(self.vplan, _stream())
        if st:
            raise RszError(st, "rsz_verify_launch")

    def graph(self):
        """Capture the batch's launch followed by the verification."""
        torch = _torch()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        st, self.graph_exec = rsz_verify_graph_create(self.B.plan, self.vplan,
                                                      C.c_void_p(side.cuda_stream))
        if st:
            raise RszError(st, "rsz_verify_graph_create")
        torch.cuda.current_stream().wait_stream(side)

    def replay(self):
        st = rsz_graph_launch(self.graph_exec, _stream())
        if st:
            raise RszError(st, "rsz_graph_launch")

    def bad_counts(self):
        """Per-frame failing-pixel counts as Python ints (0xFFFFFFFF: not verified)."""
        return [int(v) & 0xFFFFFFFF for v in self.bad.cpu().tolist()]

    def __del__(self):
        ex = getattr(self, "graph_exec", None)
        if ex is not None and ex.value:
            try:
                rsz_graph_destroy(ex)
            except Exception:
                pass


# ------------------------------------------------------------ peak finding


def peak_params(**kw):
    """rsz_peak_params with the library defaults (Sec. IV-B values), fields
    overridden by keyword."""
    q = rsz_peak_params()
    lib().rsz_peak_params_default(C.byref(q))
    for k, v in kw.items():
        setattr(q, k, v)
    return q


def rsz_find_peaks_workspace_bytes(descs):
    arr = _arr(rsz_peak_desc, descs)
    out = C.c_uint64(0)
    st = lib().rsz_find_peaks_workspace_bytes(len(descs), arr, C.byref(out))
    return st, out.value


def rsz_find_peaks_batch(q, descs, d_counts, d_status, d_ws, ws_bytes, stream):
    arr = _arr(rsz_peak_desc, descs)
    return lib().rsz_find_peaks_batch(C.byref(q), len(descs), arr, d_counts, d_status, d_ws,
                                      ws_bytes, stream)


class PeakBatch:
    """Peak finding over a list of float32 [P,H,W] GPU frames in one batched
    launch sequence: run() queues it; counts / status hold the per-frame
    results once the stream has finished; peaks(i) is frame i's list."""

    def __init__(self, frames, q=None, max_peaks=4096):
        torch = _torch()
        self.frames = [f.contiguous() for f in frames]
        self.q = q if q is not None else peak_params()
        n = len(self.frames)
        dev = self.frames[0].device
        self.max_peaks = int(max_peaks)
        self.out = torch.zeros((n, self.max_peaks, 3), dtype=torch.int32, device=dev)
        self.descs = []
        for i, f in enumerate(self.frames):
            d = rsz_peak_desc()
            d.panels, d.height, d.width = f.shape
            d.max_peaks = self.max_peaks
            d.frame = f.data_ptr()
            d.peaks = self.out[i].data_ptr()
            self.descs.append(d)
        # kept as a C array: every launch passes it as is
        self.descs = _arr(rsz_peak_desc, self.descs)
        st, wsb = rsz_find_peaks_workspace_bytes(self.descs)
        if st:
            raise RszError(st, "rsz_find_peaks_workspace_bytes")
        self.ws = workspace(wsb, dev)
        self.counts = torch.zeros(n, dtype=torch.int32, device=dev)
        self.status = torch.zeros(n, dtype=torch.int32, device=dev)

    def run(self):
        st = rsz_find_peaks_batch(self.q, self.descs, _ptr(self.counts), _ptr(self.status),
                                  _ptr(self.ws), self.ws.numel(), _stream())
        if st:
            raise RszError(st, "rsz_find_peaks_batch")

    def peaks(self, i, counts=None):
        n = int(self.counts[i]) if counts is None else int(counts[i])
        return self.out[i, :min(n, self.max_peaks)]


def find_peaks(frame, q=None, max_peaks=4096):
    """Peaks of one float32 [P,H,W] GPU frame, int32 [n,3] (panel, row, col) in
    raster order (synchronous)."""
    frame, _ = _check_frame(frame, None)
    B = PeakBatch([frame], q, max_peaks)
    B.run()
    st = int(B.status[0])
    if st:
        raise RszError(st, "rsz_find_peaks_batch")
    return B.peaks(0).clone()


def compress_hits(frames, prm, q=None, min_peaks=10, max_peaks=4096, **batch_kw):
    """Frames in, streams out: peaks found on the GPU, non-hit rejection
    (frames with fewer than min_peaks peaks are dropped, Sec. IV), then the
    hits compressed in one batch with their found peaks as the ROI.  Returns
    (indices of the hits, the Batch holding their streams, the PeakBatch)."""
    torch = _torch()
    P = PeakBatch(frames, q, max_peaks)
    P.run()
    counts = P.counts.cpu().tolist()
    status = P.status.cpu().tolist()
    bad = [s for s in status if s]
    if bad:
        raise RszError(bad[0], "rsz_find_peaks_batch")
    hits = [i for i, c in enumerate(counts) if c >= min_peaks]
    if not hits:
        return hits, None, P
    prm = prm if isinstance(prm, list) else [prm] * len(frames)
    B = Batch([P.frames[i] for i in hits], [P.peaks(i, counts) for i in hits],
              [prm[i] for i in hits], **batch_kw)
    B.run()
    return hits, B, P
