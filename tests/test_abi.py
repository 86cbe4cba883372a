"""The C-ABI library loads and exports every symbol include/rsz.h declares, and
its host-only entry points (sizes, stream header checks, argument checks)
behave as documented.  No GPU work is launched here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import rsz_oracle as O
from paper_2206_11297_amd import rsz, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "rsz.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rsz_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_names():
    assert _declared_functions() == sorted(rsz.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = C.CDLL(rsz.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_status_strings():
    for s in range(-7, 1):
        assert rsz.status_string(s) != "unknown status"


@pytest.mark.parametrize("shape,w,b,npk", [((32, 185, 388), 17, 2, 60), ((8, 512, 1024), 25, 4, 800),
                                           ((1, 1, 1), 1, 1, 1), ((2, 9, 7), 3, 3, 5)])
def test_max_bytes_matches_oracle(shape, w, b, npk):
    p = rsz.params(*shape, w, b, 10.0)
    st, n = rsz.rsz_max_compressed_bytes(p, npk)
    sto, no = O.max_bytes(O.params(*shape, w, b, 10.0), npk)
    assert st == 0 and sto == 0 and n == no
    st, ws = rsz.rsz_workspace_bytes(p, npk)
    assert st == 0 and ws > 0


@pytest.mark.parametrize("bad", [dict(panels=0), dict(height=70000), dict(window=0),
                                 dict(window=1024), dict(bin=0), dict(bin=9), dict(eb=0.0),
                                 dict(eb=float("inf")), dict(eb=float("nan")), dict(bin_mode=2),
                                 dict(dim=4),
                                 dict(panels=65535, height=65535, width=2)])
def test_bad_params_rejected(bad):
    kw = dict(panels=2, height=8, width=8, window=3, bin=2, eb=1.0, bin_mode=0, dim=2)
    kw.update(bad)
    p = rsz.params(**kw)
    assert rsz.rsz_max_compressed_bytes(p, 1)[0] == rsz.RSZ_ERR_ARG
    assert rsz.rsz_workspace_bytes(p, 1)[0] == rsz.RSZ_ERR_ARG
    assert rsz.rsz_compress(p, None, None, 0, None, 0, None, 0, None)[0] == rsz.RSZ_ERR_ARG


def test_compress_rejects_null_and_misaligned_pointers_before_any_gpu_work():
    p = rsz.params(2, 8, 8, 3, 2, 1.0)
    st, _ = rsz.rsz_compress(p, None, None, 0, C.c_void_p(4096), 1 << 20, C.c_void_p(4096),
                             1 << 20, None)
    assert st == rsz.RSZ_ERR_ARG
    st, _ = rsz.rsz_compress(p, C.c_void_p(4100), None, 0, C.c_void_p(4096), 1 << 20,
                             C.c_void_p(4096), 1 << 20, None)
    assert st == rsz.RSZ_ERR_ARG
    st, _ = rsz.rsz_compress(p, C.c_void_p(4096), None, 0, C.c_void_p(4096), 1 << 20,
                             C.c_void_p(4096), 16, None)
    assert st == rsz.RSZ_ERR_WORKSPACE


def test_stream_info_agrees_with_oracle_streams():
    for eb in (1.0, 10.0):
        f, pk = synth.cspad_frame(2)
        st, s, n = O.compress(O.params(32, 185, 388, 17, 2, eb), f, pk)
        st, p, npk, total = rsz.rsz_stream_info(s.tobytes()[:80])
        assert st == 0 and total == n and npk == pk.shape[0]
        assert (p.panels, p.height, p.width, p.window, p.bin, p.bin_mode, p.eb) == \
            (32, 185, 388, 17, 2, 0, eb)
        assert rsz.rsz_stream_info(s.tobytes())[0] == 0
        assert rsz.rsz_stream_info(s.tobytes()[:-4])[0] == rsz.RSZ_ERR_CORRUPT
        st, wsb = rsz.rsz_decompress_workspace_bytes(s.tobytes()[:80])
        assert st == 0 and wsb >= 4 * 32 * 93 * 194


def test_stream_info_rejects_bad_headers_like_the_oracle():
    f, pk = synth.tiny_case(21, (2, 9, 11), 3, "normal", scale=100.0)
    st, s, n = O.compress(O.params(2, 9, 11, 3, 2, 1.0), f, pk)
    rng = np.random.default_rng(3)
    for t in range(400):
        s2 = s.copy()
        pos = int(rng.integers(0, 80))
        s2[pos] ^= np.uint8(1 << int(rng.integers(0, 8)))
        a = rsz.rsz_stream_info(s2.tobytes())[0]
        b = O.stream_info(s2)[0]
        assert (a == 0) == (b == 0), pos


def test_struct_layouts_match_the_header(tmp_path):
    """Every ctypes mirror in the binding has the size and field offsets the
    C compiler gives the structs of include/rsz.h."""
    import subprocess
    structs = {"rsz_peak": None, "rsz_params": rsz.rsz_params, "rsz_frame_desc": rsz.rsz_frame_desc,
               "rsz_batch_plan": rsz.rsz_batch_plan, "rsz_debug_bufs": rsz.rsz_debug_bufs,
               "rsz_kernel_time": rsz.rsz_kernel_time, "rsz_peak_params": rsz.rsz_peak_params,
               "rsz_peak_desc": rsz.rsz_peak_desc, "rsz_decode_desc": rsz.rsz_decode_desc,
               "rsz_verify_plan": rsz.rsz_verify_plan}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rsz.h"', 'int main(void) {']
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in (cls._fields_ if cls is not None else []):
            lines.append(f'  printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append('  return 0;\n}')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                           str(src)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    for name, cls in structs.items():
        if cls is None:
            assert got[(name, "size")] == 12
            continue
        assert got[(name, "size")] == C.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert got[(name, fname)] == getattr(cls, fname).offset, (name, fname)


def test_peak_params_default_and_checks():
    """Library defaults are the paper's values (Sec. IV-B) and equal the
    oracle's; bad parameters and descriptors are rejected before any launch."""
    q = rsz.peak_params()
    o = O.peak_params()
    for name, _ in rsz.rsz_peak_params._fields_:
        assert getattr(q, name) == getattr(o, name), name
    d = rsz.rsz_peak_desc(2, 8, 8, 16, None, None)
    st, n = rsz.rsz_find_peaks_workspace_bytes([d])
    assert st == 0 and n > 0
    for bad in (dict(rank=0), dict(rank=4), dict(ring_in=3), dict(ring_out=16),
                dict(npix_min=40), dict(snr_min=-1.0), dict(pix_nsigma=float("inf")),
                dict(reserved=1)):
        qb = rsz.peak_params(**bad)
        assert rsz.rsz_find_peaks_batch(qb, [d], None, None, None, 0, None) == rsz.RSZ_ERR_ARG
        assert O.check_peak_params(O.peak_params(**{k: v for k, v in bad.items()
                                                     if k != "reserved"})) == O.ERR_ARG \
            or "reserved" in bad


def test_batch_decode_workspace_on_the_host():
    """rsz_decompress_batch_workspace_bytes plans from host headers only: one
    stream needs what rsz_decompress needs, a rejected header adds no region,
    and each further stream adds its own region."""
    f, pk = synth.cspad_frame(2)
    st, s, n = O.compress(O.params(32, 185, 388, 17, 2, 10.0, 0, 2, 1, 1), f, pk)
    head = C.create_string_buffer(s.tobytes()[:80], 80)
    bad = C.create_string_buffer(b"XXXX" + s.tobytes()[4:80], 80)
    fake = 1 << 20   # device addresses are not read by the host planner

    def desc(h):
        return rsz.rsz_decode_desc(fake, n, C.addressof(h), fake, 32 * 185 * 388)

    st1, one = rsz.rsz_decompress_batch_workspace_bytes([desc(head)])
    st0, single = rsz.rsz_decompress_workspace_bytes(s.tobytes()[:80])
    assert st1 == st0 == 0 and one == single
    st, with_bad = rsz.rsz_decompress_batch_workspace_bytes([desc(head), desc(bad)])
    assert st == 0 and 0 <= with_bad - one <= 2048
    st, two = rsz.rsz_decompress_batch_workspace_bytes([desc(head), desc(head)])
    assert st == 0 and two >= 2 * one - 4096
    assert rsz.rsz_decompress_batch_workspace_bytes([])[0] == rsz.RSZ_ERR_ARG
    d = desc(head)
    d.header = None
    assert rsz.rsz_decompress_batch_workspace_bytes([d])[0] == rsz.RSZ_ERR_ARG


def test_profile_filter_on_the_host():
    """rsz_profile_only selects the kernel whose launches are timed; with no
    launch recorded the read-back is empty."""
    assert rsz.rsz_profile_only("k_bin") == 0
    assert rsz.rsz_profile_enable(True) == 0
    assert rsz.rsz_profile_read() == {}
    assert rsz.rsz_profile_enable(False) == 0
    assert rsz.rsz_profile_only(None) == 0


def test_verify_planner_on_the_host():
    """rsz_verify_workspace_bytes plans from the descriptors alone (no device
    memory is touched): every frame the stage verifies adds its decoder
    region, a frame with the ROI coded or invalid parameters only a status
    word; a plan for another frame count, or a prepare without output
    frames, is refused before any upload."""
    cases = [((32, 185, 388), (17, 2, 10.0, 0), 60), ((8, 512, 1024), (25, 4, 10.0, 0), 100),
             ((3, 70, 130), (7, 3, 1.0, 1), 6), ((1, 1, 1), (1, 1, 1.0, 0), 1)]
    fake = 1 << 20   # device addresses are not read by the host planner

    def desc(shape, prm, npk):
        d = rsz.rsz_frame_desc()
        d.params = rsz.params(*shape, *prm)
        d.frame, d.peaks, d.npeaks, d.out, d.out_cap = fake, fake if npk else None, npk, fake, 1 << 30
        return d

    descs = [desc(*c) for c in cases]
    plan = rsz.rsz_batch_plan()
    for i in range(len(plan.opaque)):
        plan.opaque[i] = len(descs)   # a frame count of 4 and non-null pointers
    st, full = rsz.rsz_verify_workspace_bytes(plan, descs)
    assert st == 0 and full > 32 * 185 * 388
    coded = list(descs)
    coded[1] = desc((8, 512, 1024), (25, 4, 10.0, 0, 2, 1), 100)
    st, less = rsz.rsz_verify_workspace_bytes(plan, coded)
    assert st == 0 and less < full - 8 * 512 * 1024 // 16
    assert rsz.rsz_verify_workspace_bytes(plan, descs[:3])[0] == rsz.RSZ_ERR_ARG
    st, _ = rsz.rsz_verify_prepare(plan, descs, [0] * 4, fake, fake, 1 << 40, None)
    assert st == rsz.RSZ_ERR_ARG
