"""Independent reader/builder of the compressed stream layout, and brute-force
definitions used as pins.  Test code only: written from the stated format and
the paper's definitions, sharing nothing with the oracle or the HIP library.

Layout (little-endian, sections 4-byte aligned):
  header 80 B: magic 'RSZ1', u16 version 1, u16 flags (bit0 bin_mode, bits
  1-2 the Lorenzo dimension, 0 standing for 2),
  u32 P, H, W, window, bin, radius(512), f64 eb, u32 npeaks, n_out, chunk(4096),
  n_chunks, u64 T (bits), u64 stream_bytes, u64 reserved 0;
  then peaks (npeaks x 3 u16, padded to 4), ROI payload (npeaks*w*w u32),
  code lengths (1024 u8), chunk bit offsets (n_chunks u32), bitstream
  (ceil(T/32) u32, codewords MSB-first within each word), outlier indices
  (n_out u32), outlier residuals (n_out i32).
  Flag bit 3: the ROI payload is replaced by a coded ROI section at the end.
  Flag bit 4: the bitstream is replaced by a run section at the very end:
  one Rice parameter per chunk (u8, padded to 4), n_chunks + 1 u32 bit
  offsets (the last is the section's bits), then the run bits.
"""
import struct

import numpy as np

HDR = struct.Struct("<4sHHIIIIIIdIIIIQQQ")
assert HDR.size == 80


def align4(x):
    return (x + 3) & ~3


def sections(npeaks, window, n_out, n_chunks, T, roi_coded=False, Troi=0, run_coded=False,
             Trun=0):
    off = {}
    off["peaks"] = 80
    off["roi"] = 80 + align4(6 * npeaks)
    off["lens"] = off["roi"] + (0 if roi_coded else 4 * npeaks * window * window)
    off["chunks"] = off["lens"] + 1024
    off["bits"] = off["chunks"] + 4 * n_chunks
    off["oidx"] = off["bits"] + (0 if run_coded else 4 * ((T + 31) // 32))
    off["ores"] = off["oidx"] + 4 * n_out
    off["total"] = off["ores"] + 4 * n_out
    if roi_coded:
        # coded ROI section at the end: 33 class lengths (padded to 36 bytes),
        # one u32 bit offset per window, the ROI bitstream
        off["rsec"] = off["total"]
        off["roffs"] = off["rsec"] + 36
        off["rbits"] = off["roffs"] + 4 * npeaks
        off["total"] = off["rbits"] + 4 * ((Troi + 31) // 32)
    if run_coded:
        off["run"] = off["total"]
        off["runoffs"] = off["run"] + align4(n_chunks)
        off["runbits"] = off["runoffs"] + 4 * (n_chunks + 1)
        off["total"] = off["runbits"] + 4 * ((Trun + 31) // 32)
    return off


def parse(buf):
    buf = bytes(np.asarray(buf, dtype=np.uint8).tobytes())
    (magic, ver, flags, P, H, W, w, b, R, eb, npk, n_out, ch, nch, T, total, res) = \
        HDR.unpack_from(buf, 0)
    coded, runs = bool(flags & 8), bool(flags & 16)
    off = sections(npk, w, n_out, nch, T, coded, res if coded else 0)
    if runs:
        Trun = struct.unpack_from("<I", buf, sections(npk, w, n_out, nch, T, coded, res, True)
                                  ["runoffs"] + 4 * nch)[0]
        off = sections(npk, w, n_out, nch, T, coded, res, True, Trun)
    d = dict(magic=magic, version=ver, flags=flags, P=P, H=H, W=W, window=w, bin=b, radius=R,
             eb=eb, npeaks=npk, n_out=n_out, chunk=ch, n_chunks=nch, T=T, stream_bytes=total,
             reserved=res, off=off, bin_mode=flags & 1,
             dim={0: 2, 1: 1, 3: 3}.get((flags >> 1) & 3))
    d["peaks"] = np.frombuffer(buf, np.uint16, 3 * npk, off["peaks"]).reshape(-1, 3)
    d["roi_coded"] = coded
    if coded:
        d["Troi"] = res
        d["roi_lens"] = np.frombuffer(buf, np.uint8, 36, off["rsec"])
        d["roi_offsets"] = np.frombuffer(buf, np.uint32, npk, off["roffs"])
        d["roi_words"] = np.frombuffer(buf, np.uint32, (res + 31) // 32, off["rbits"])
        d["roi"] = decode_roi(d["roi_lens"], d["roi_offsets"], d["roi_words"], res, npk, w)
    else:
        d["roi"] = np.frombuffer(buf, np.uint32, npk * w * w, off["roi"])
    d["lens"] = np.frombuffer(buf, np.uint8, 1024, off["lens"])
    d["oidx"] = np.frombuffer(buf, np.uint32, n_out, off["oidx"])
    d["ores"] = np.frombuffer(buf, np.int32, n_out, off["ores"])
    d["chunk_offsets"] = np.frombuffer(buf, np.uint32, nch, off["chunks"])
    d["run_coded"] = runs
    if runs:
        d["Trun"] = Trun
        d["run_k"] = np.frombuffer(buf, np.uint8, align4(nch), off["run"])
        d["run_offsets"] = np.frombuffer(buf, np.uint32, nch + 1, off["runoffs"])
        d["run_words"] = np.frombuffer(buf, np.uint32, (Trun + 31) // 32, off["runbits"])
        d["bit_words"] = decode_runs(d["run_k"], d["run_offsets"], d["run_words"],
                                     d["chunk_offsets"], T)
    else:
        d["bit_words"] = np.frombuffer(buf, np.uint32, (T + 31) // 32, off["bits"])
    return d


def decode_runs(kpar, offsets, words, chunk_offsets, T):
    """Independent reader of the run section: per chunk, codes of a unary
    quotient (ones closed by a zero) and k remainder bits give the number of
    zero bits before each one bit; the rest of the chunk is zeros.  Returns
    the T bitstream bits packed MSB-first into u32 words."""
    Trun = int(offsets[-1])
    src = bits_of(words, Trun)
    bits = np.zeros(32 * ((T + 31) // 32), np.uint8)
    nch = len(chunk_offsets)
    for c in range(nch):
        pos, end = int(offsets[c]), int(offsets[c + 1])
        k = int(kpar[c])
        at = int(chunk_offsets[c])
        stop = int(chunk_offsets[c + 1]) if c + 1 < nch else T
        while pos < end:
            q = 0
            while src[pos]:
                q += 1
                pos += 1
            pos += 1
            r = q * (1 << k)
            for t in range(k):
                r += src[pos] << (k - 1 - t)
                pos += 1
            at += r
            assert at < stop
            bits[at] = 1
            at += 1
        assert pos == end
    return np.packbits(bits).view(">u4").astype(np.uint32)


def bits_of(words, T):
    """Stream bits as a list of 0/1, bit k = bit 31-(k%32) of word k//32."""
    out = []
    for k in range(T):
        out.append((int(words[k // 32]) >> (31 - k % 32)) & 1)
    return out


def decode_symbols(lens, words, T, nsym):
    """Bit-by-bit prefix decode with a dictionary of codewords rebuilt from the
    lengths by sorting (length, symbol) -- written independently."""
    syms = sorted((int(lens[s]), s) for s in range(1024) if lens[s] > 0)
    table = {}
    code = -1
    prev = 0
    for L, s in syms:
        code = 0 if code < 0 else (code + 1) << (L - prev)
        prev = L
        table[(L, code)] = s
    bits = bits_of(words, T)
    out, pos = [], 0
    offsets = []
    for g in range(nsym):
        if g % 4096 == 0:
            offsets.append(pos)
        c, L = 0, 0
        while True:
            c = (c << 1) | bits[pos]
            pos += 1
            L += 1
            if (L, c) in table:
                out.append(table[(L, c)])
                break
            assert L < 32
    assert pos == T
    return np.array(out, np.int64), offsets


def mask_bruteforce(shape, peaks, window):
    """Per pixel: inside the window of any peak on the same panel."""
    P, H, W = shape
    h = window // 2
    M = np.zeros(shape, bool)
    for p in range(P):
        for i in range(H):
            for j in range(W):
                for (pk, r, c) in peaks:
                    if pk == p and r - h <= i <= r - h + window - 1 and c - h <= j <= c - h + window - 1:
                        M[p, i, j] = True
                        break
    return M


def mask_slices(shape, peaks, window):
    """Same mask by numpy slice assignment."""
    P, H, W = shape
    h = window // 2
    M = np.zeros(shape, bool)
    for (pk, r, c) in peaks:
        M[pk, max(0, r - h):max(0, r - h + window), max(0, c - h):max(0, c - h + window)] = True
    return M


def unpack_bitmap(bitmap, W):
    bitmap = np.asarray(bitmap, np.uint32)
    P, H, wpr = bitmap.shape
    bits = ((bitmap[..., None] >> np.arange(32, dtype=np.uint32)) & 1).astype(bool)
    return bits.reshape(P, H, wpr * 32)[:, :, :W]


def bin_sums(frame, M, b, include_all):
    """S (fp64, raster-order accumulation) and n per bin by explicit loops
    over the b x b offsets; partial bins at the edges."""
    P, H, W = frame.shape
    Hb, Wb = -(-H // b), -(-W // b)
    S = np.zeros((P, Hb, Wb), np.float64)
    n = np.zeros((P, Hb, Wb), np.int64)
    x64 = frame.astype(np.float64)
    for di in range(b):
        for dj in range(b):
            sub = x64[:, di::b, dj::b]
            inc = np.ones(sub.shape, bool) if include_all else ~M[:, di::b, dj::b]
            hs, ws = sub.shape[1], sub.shape[2]
            S[:, :hs, :ws] = np.where(inc, S[:, :hs, :ws] + sub, S[:, :hs, :ws])
            n[:, :hs, :ws] += inc
    return S, n


def closed_form_reconstruction(frame, peaks, window, b, eb, bin_mode):
    """y = x on ROI pixels (bit-exact), else float32(rint(S/(n*2eb)) * 2eb)
    replicated over the bin, with q = 0 for an empty bin."""
    P, H, W = frame.shape
    M = mask_slices(frame.shape, peaks, window)
    S, n = bin_sums(frame, M, b, bin_mode == 1)
    den = n.astype(np.float64) * (2.0 * eb)
    with np.errstate(invalid="ignore", divide="ignore"):
        q = np.where(n > 0, np.rint(S / np.where(n > 0, den, 1.0)), 0.0)
    q = q.astype(np.int64)             # q is an integer: rint(-0.3) is the integer 0
    val = (q.astype(np.float64) * (2.0 * eb)).astype(np.float32)
    y = np.repeat(np.repeat(val, b, axis=1), b, axis=2)[:, :H, :W].copy()
    y[M] = frame[M]
    return y, M, S, n, q


def decode_roi(lens, offsets, words, Troi, npeaks, w):
    """Independent decoder of the coded ROI section: per window, class
    codewords (canonical, from the lengths sorted by (length, class)) each
    followed by class-1 raw bits of the zigzag residual; the residual is added
    to the 2D Lorenzo prediction over the window in the order-preserving
    integer domain (2^31 outside the window) and mapped back to float bits."""
    syms = sorted((int(lens[c]), c) for c in range(33) if lens[c] > 0)
    table, code, prev = {}, -1, 0
    for L, c in syms:
        code = 0 if code < 0 else (code + 1) << (L - prev)
        prev = L
        table[(L, code)] = c
    bits = bits_of(words, Troi)
    out = np.zeros((npeaks, w, w), np.uint32)
    pos = 0
    for k in range(npeaks):
        assert pos == int(offsets[k])
        M = np.zeros((w, w), np.int64)
        for u in range(w):
            for v in range(w):
                c, L = 0, 0
                while (L, c) not in table:
                    c = (c << 1) | bits[pos]
                    pos += 1
                    L += 1
                    assert L <= 32
                cls = table[(L, c)]
                z = 0 if cls == 0 else 1
                for _ in range(cls - 1):
                    z = (z << 1) | bits[pos]
                    pos += 1
                r = (z >> 1) ^ (-(z & 1) & 0xFFFFFFFF)
                up = M[u - 1, v] if u else 1 << 31
                left = M[u, v - 1] if v else 1 << 31
                ul = M[u - 1, v - 1] if u and v else 1 << 31
                M[u, v] = (up + left - ul + r) & 0xFFFFFFFF
                m = int(M[u, v])
                out[k, u, v] = (m & 0x7FFFFFFF) if m & 0x80000000 else (~m & 0xFFFFFFFF)
    assert pos == Troi
    return out.reshape(-1)
