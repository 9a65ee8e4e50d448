"""The C-ABI libraries load and export every declared symbol, and argument
checking rejects bad descriptors before any GPU work (runs without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

import paper_2604_16590_amd as la
from paper_2604_16590_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(la_[a-z_0-9]+)\s*\(", text, re.M))


@pytest.mark.parametrize("header,lib", [("la.h", B.LIB_PATH), ("la_gen.h", B.GEN_PATH)])
def test_every_declared_symbol_is_exported(header, lib):
    names = declared(os.path.join(ROOT, "include", header))
    assert names, header
    handle = ctypes.CDLL(lib)
    missing = [n for n in sorted(names) if not hasattr(handle, n)]
    assert not missing, missing


def test_headers_cover_all_exports():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        names |= declared(h)
    assert {"la_forward", "la_backward", "la_workspace_size", "la_gen_fill"} <= names


def desc(**kw):
    d = dict(B=1, H=2, N=100, d=64, in_dtype=0, out_dtype=0, in_sb=2 * 100 * 64, in_sh=100 * 64,
             in_sn=64, out_sb=2 * 100 * 64, out_sh=100 * 64, out_sn=64, feature_map=0, flags=0)
    d.update(kw)
    return B.AttnDesc(**d)


def ws_status(dsc, pass_=0):
    n = ctypes.c_size_t(0)
    return la.lib().la_workspace_size(ctypes.byref(dsc), pass_, ctypes.byref(n)), n.value


def test_status_strings():
    L = la.lib()
    assert L.la_status_string(0) == b"LA_OK"
    assert L.la_status_string(2) == b"LA_ERR_UNSUPPORTED"
    assert L.la_status_string(99) == b"LA_ERR_UNKNOWN"


def test_workspace_size_valid_and_grows_only_with_partials():
    # B2 H1 d64 bf16: 64 partial sums per head up to 64 x 16,384 tokens,
    # then one more per 16,384 tokens (no FP32 sum covers more), each
    # (d^2 + d) FP32 values; everything else is O(d^2) per head
    def ws(n):
        st, nbytes = ws_status(desc(N=n, in_sb=2 * n * 64, in_sh=n * 64,
                                    out_sb=2 * n * 64, out_sh=n * 64))
        assert st == 0 and nbytes > 0
        return nbytes
    part = 2 * (64 * 64 + 64) * 4
    small = ws(1 << 16)
    assert ws(64 * 16384) == small                      # still 64 partials
    for n in (64 * 16384 + 1, 1 << 30, (1 << 30) + 77):
        P = -(-n // 16384)
        assert abs(ws(n) - (small + (P - 64) * part)) <= 512, n
    # fp32 inputs: at most 4,096 tokens per partial
    st, f = ws_status(desc(N=1 << 20, in_dtype=1, out_dtype=1, in_sb=2 * (1 << 20) * 64,
                           in_sh=(1 << 20) * 64, out_sb=2 * (1 << 20) * 64, out_sh=(1 << 20) * 64))
    assert st == 0 and f >= 2 * 256 * (64 * 64 + 64) * 4
    assert ws_status(desc(), 1)[0] == 0
    assert ws_status(desc(), 2)[0] == 0
    assert ws_status(desc(), 3)[0] == 1


@pytest.mark.parametrize("kw,status", [
    (dict(N=0), 1), (dict(B=0), 1), (dict(H=-1), 1),
    (dict(d=48, in_sn=48, out_sn=48, in_sh=4800, out_sh=4800, in_sb=9600, out_sb=9600), 2),
    (dict(d=256, in_sn=256, out_sn=256, in_sh=25600, out_sh=25600, in_sb=51200, out_sb=51200), 2),
    (dict(in_dtype=7), 1), (dict(out_dtype=-1), 1), (dict(feature_map=3), 2),
    (dict(flags=1), 1), (dict(in_sn=60), 1), (dict(in_sn=68), 1), (dict(out_sh=-64), 1),
    (dict(in_sb=12802), 1),
])
def test_bad_descriptors_are_rejected(kw, status):
    assert ws_status(desc(**kw))[0] == status


def test_size_limits():
    # N up to 2^36 tokens per (b, h) and up to 65535 (b, h) pairs
    def big(n):
        return desc(N=n, in_sb=2 * n * 64, in_sh=n * 64, out_sb=2 * n * 64, out_sh=n * 64)
    assert ws_status(big(1 << 36))[0] == 0
    assert ws_status(big((1 << 36) + 1))[0] == 2
    assert ws_status(desc(B=65535, H=1, in_sb=6400, out_sb=6400))[0] == 0
    assert ws_status(desc(B=32768, H=2))[0] == 2


def test_forward_rejects_bad_pointers_before_gpu_work():
    L = la.lib()
    d = desc()
    ws = ctypes.c_size_t(0)
    L.la_workspace_size(ctypes.byref(d), 0, ctypes.byref(ws))
    fake = 1 << 20  # never dereferenced: every case fails validation first
    args = [fake, fake, fake, fake]
    assert L.la_forward(ctypes.byref(d), None, fake, fake, fake, None, None, fake, ws.value, None) == 1
    assert L.la_forward(ctypes.byref(d), fake + 2, fake, fake, fake, None, None, fake, ws.value, None) == 1
    assert L.la_forward(ctypes.byref(d), *args, None, None, fake + 16, ws.value, None) == 1  # ws alignment
    assert L.la_forward(ctypes.byref(d), *args, None, None, fake, ws.value - 1, None) == 3
    assert L.la_forward(ctypes.byref(d), *args, fake + 4, None, fake, ws.value, None) == 1
    assert L.la_backward(ctypes.byref(d), *args[:3], None, fake, fake, fake, fake, fake, fake,
                         ws.value, None) == 1
    assert L.la_forward(None, *args, None, None, fake, ws.value, None) == 1
    L.la_workspace_size(ctypes.byref(d), 2, ctypes.byref(ws))
    assert L.la_apply(ctypes.byref(d), fake, None, fake, fake, fake, ws.value, None) == 1
    assert L.la_apply(ctypes.byref(d), fake, fake + 4, fake, fake, fake, ws.value, None) == 1
    assert L.la_apply(ctypes.byref(d), fake, fake, fake, fake, fake, ws.value - 1, None) == 3


def test_gated_calls_reject_bad_gate_arguments_before_gpu_work():
    L = la.lib()
    d = desc()
    ws0, ws2 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    L.la_workspace_size(ctypes.byref(d), 0, ctypes.byref(ws0))
    L.la_workspace_size(ctypes.byref(d), 2, ctypes.byref(ws2))
    fake = 1 << 20  # never dereferenced: every case fails validation first
    qkv = [fake, fake, fake]
    for other, sigma, sd, status in ((None, fake, 0.5, 1), (fake + 8, fake, 0.5, 1),
                                     (fake, None, 0.5, 1), (fake, fake + 4, 0.5, 1),
                                     (fake, fake, 0.0, 1), (fake, fake, -1.0, 1),
                                     (fake, fake, float("nan"), 1), (fake, fake, float("inf"), 1)):
        assert L.la_forward_gated(ctypes.byref(d), *qkv, other, sigma, sd, fake, None, None, fake,
                                  ws0.value, None) == status
        assert L.la_apply_gated(ctypes.byref(d), fake, fake, fake, other, sigma, sd, fake, fake,
                                ws2.value, None) == status
    # good gate, then the attention's own checks
    assert L.la_forward_gated(ctypes.byref(d), None, fake, fake, fake, fake, 0.5, fake, None, None,
                              fake, ws0.value, None) == 1
    assert L.la_forward_gated(ctypes.byref(d), *qkv, fake, fake, 0.5, fake, None, None, fake,
                              ws0.value - 1, None) == 3
    assert L.la_apply_gated(ctypes.byref(d), fake, fake, fake, fake, fake, 0.5, fake, fake,
                            ws2.value - 1, None) == 3
    bad = desc(N=0)
    assert L.la_apply_gated(ctypes.byref(bad), fake, fake, fake, fake, fake, 0.5, fake, fake,
                            ws2.value, None) == 1


def test_generator_rejects_bad_arguments():
    G = B.gen_lib()
    spec = B.GenSpec(1, 0, 0, 0.0, 1.0, 0, 0, 0, 1.0, 0)
    fake = 1 << 20
    assert G.la_gen_fill(None, 0, 1, 1, 8, 16, 128, 128, 16, ctypes.byref(spec), None) == 1
    assert G.la_gen_fill(fake + 2, 0, 1, 1, 8, 16, 128, 128, 16, ctypes.byref(spec), None) == 1
    assert G.la_gen_fill(fake, 2, 1, 1, 8, 16, 128, 128, 16, ctypes.byref(spec), None) == 1
    grid = B.GenSpec(1, 0, 0, 0.0, 1.0, 2, 2, 3, 1.0, 0)  # 12 tokens != N
    assert G.la_gen_fill(fake, 0, 1, 1, 8, 16, 128, 128, 16, ctypes.byref(grid), None) == 1


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(B, "LIB_PATH", "/nonexistent/liblinattn.so")
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(RuntimeError):
        B.lib()


def test_tile_geometry_and_validation():
    L = B._tile_lib()
    n, t = ctypes.c_int64(0), ctypes.c_int64(0)
    d = B._tile_desc((3, 10, 7), (1, 3, 2), (1, 3, 2), 16, B.torch.bfloat16)
    assert L.la_tile_geometry(ctypes.byref(d), ctypes.byref(n), ctypes.byref(t)) == 0
    assert n.value == 3 * 4 * 4 and t.value == 3 * 9 * 6
    assert (n.value, (3, 9, 6)) == B.tile_geometry((3, 10, 7), (1, 3, 2), (1, 3, 2))
    for dims, core, halo, C in (((3, 10, 7), (1, 3, 2), (2, 0, 0), 16),   # halo > core
                                ((3, 10, 7), (1, 3, 2), (0, 0, 0), 12),   # C not a multiple of 8
                                ((0, 10, 7), (1, 3, 2), (0, 0, 0), 16)):
        bad = B._tile_desc(dims, core, halo, C, B.torch.float32)
        assert L.la_tile_geometry(ctypes.byref(bad), ctypes.byref(n), ctypes.byref(t)) == 1
    fake = 1 << 20
    assert L.la_tile_extract(ctypes.byref(d), fake + 8, fake, None) == 1


def test_stream_probe_rejects_bad_arguments_before_gpu_work():
    # fake but aligned device addresses: every case is refused before any
    # HIP call, so nothing is enqueued
    L = la.lib()
    L.la_stream_probe.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_uint32, ctypes.c_void_p]
    L.la_stream_probe.restype = ctypes.c_int
    a, b = 1 << 20, 1 << 24
    assert L.la_stream_probe(0, a, b, 0, 0, None) == 1          # no bytes
    assert L.la_stream_probe(2, a, b, 40, 0, None) == 1         # not a multiple of 16
    assert L.la_stream_probe(1, None, None, 64, 0, None) == 1   # no destination
    assert L.la_stream_probe(0, None, b, 64, 0, None) == 1      # read without a source
    assert L.la_stream_probe(2, a + 8, b, 64, 0, None) == 1     # misaligned source
    assert L.la_stream_probe(1, None, b + 4, 64, 0, None) == 1  # misaligned destination
    assert L.la_stream_probe(2, a, a + 16, 64, 0, None) == 1    # overlapping copy
    assert L.la_stream_probe(3, a, b, 64, 0, None) == 1         # unknown kind


def test_noalloc_forward_checks_before_touching_the_device():
    # descriptor errors, and problems whose workspace exceeds the fixed
    # scratch (LA_ERR_OOM), are reported before any HIP call
    L = la.lib()
    L.la_forward_noalloc.argtypes = [ctypes.POINTER(B.AttnDesc)] + [ctypes.c_void_p] * 7
    L.la_forward_noalloc.restype = ctypes.c_int
    fake = 1 << 20
    assert L.la_forward_noalloc(ctypes.byref(desc(N=0)), fake, fake, fake, fake, None, None, None) == 1
    N, H = 4 << 20, 64
    big = B.AttnDesc(1, H, N, 64, 0, 0, H * N * 64, N * 64, 64, H * N * 64, N * 64, 64, 0, 0)
    assert ws_status(big)[1] > (128 << 20)
    assert L.la_forward_noalloc(ctypes.byref(big), fake, fake, fake, fake, None, None, None) == 3


def test_tiled_forward_argument_checks():
    # the fused tiled step supports bf16, d <= 64 and halos of at most half
    # a core; everything else is refused before any device work
    L = la.lib()
    T3 = ctypes.c_int64 * 3
    L.la_tiled_workspace_size.argtypes = [ctypes.POINTER(B.TileDesc), ctypes.c_int64,
                                          ctypes.POINTER(ctypes.c_size_t)]
    L.la_tiled_workspace_size.restype = ctypes.c_int

    def ws(dims, core, halo, C, dtype, heads):
        d = B.TileDesc(T3(*dims), T3(*core), T3(*halo), C, dtype)
        n = ctypes.c_size_t(0)
        return L.la_tiled_workspace_size(ctypes.byref(d), heads, ctypes.byref(n)), n.value

    st, n = ws((16, 32, 64), (4, 16, 16), (2, 8, 8), 256, 0, 4)
    assert st == 0 and n > 0
    assert ws((16, 32, 64), (4, 16, 16), (2, 8, 8), 256, 1, 4)[0] == 2    # fp32
    assert ws((16, 32, 64), (4, 16, 16), (2, 8, 8), 256, 0, 2)[0] == 2    # d = 128
    assert ws((16, 32, 64), (4, 16, 16), (3, 8, 8), 256, 0, 4)[0] == 2    # halo > core / 2
    assert ws((16, 32, 64), (4, 16, 16), (2, 8, 8), 256, 0, 3)[0] == 1    # C % heads
    assert ws((16, 32, 64), (4, 16, 16), (5, 8, 8), 256, 0, 4)[0] == 1    # halo > core
    assert ws((64, 64, 64), (64, 32, 40), (0, 0, 0), 256, 0, 4)[0] == 2   # > 65,536 tokens a tile
    # a tile's t extent is one FP32 run of its column sums: at most 16,384
    assert ws((16385, 1, 1), (16385, 1, 1), (0, 0, 0), 256, 0, 4)[0] == 2
    assert ws((16384, 1, 1), (16384, 1, 1), (0, 0, 0), 256, 0, 4)[0] == 0
    # the kernels address fields with 32-bit token indices: 2^31 tokens and
    # more are refused, one fewer is accepted (nothing is allocated here)
    assert ws((2048, 1024, 1024), (8, 16, 16), (2, 4, 4), 64, 0, 4)[0] == 2
    st, n = ws((2047, 1024, 1024), (8, 16, 16), (2, 4, 4), 64, 0, 4)
    assert st == 0 and n > 0
