"""ctypes binding of liblinattn.so (include/la.h) and liblagen.so.

Argument marshalling only: every step of the attention runs in the HIP
kernels behind the C ABI.  PyTorch supplies device memory and the current
HIP stream.  There is no fallback: if the library is missing or a call
fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblinattn.so")
GEN_PATH = os.path.join(_HERE, "liblagen.so")

LA_BF16, LA_FP32 = 0, 1
LA_PHI_ELU1 = 0
STATUS = {0: "LA_OK", 1: "LA_ERR_INVALID_ARG", 2: "LA_ERR_UNSUPPORTED", 3: "LA_ERR_OOM",
          4: "LA_ERR_HIP", 5: "LA_ERR_NOT_FOUND", 6: "LA_ERR_SHUTDOWN", 7: "LA_ERR_BUSY"}


class LaError(RuntimeError):
    def __init__(self, call, status, hip_error=0):
        self.status = status
        self.hip_error = hip_error
        msg = "%s returned %s" % (call, STATUS.get(status, status))
        if hip_error:
            msg += " (hipError %d)" % hip_error
        super().__init__(msg)


class AttnDesc(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int64), ("H", ctypes.c_int64), ("N", ctypes.c_int64),
                ("d", ctypes.c_int64), ("in_dtype", ctypes.c_int32),
                ("out_dtype", ctypes.c_int32),
                ("in_sb", ctypes.c_int64), ("in_sh", ctypes.c_int64), ("in_sn", ctypes.c_int64),
                ("out_sb", ctypes.c_int64), ("out_sh", ctypes.c_int64), ("out_sn", ctypes.c_int64),
                ("feature_map", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class GenSpec(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("stream", ctypes.c_uint32),
                ("tensor_id", ctypes.c_int32), ("mean", ctypes.c_double),
                ("std", ctypes.c_double), ("grid_T", ctypes.c_int32),
                ("grid_lat", ctypes.c_int32), ("grid_lon", ctypes.c_int32),
                ("amplitude", ctypes.c_double), ("b_offset", ctypes.c_int64)]


_lib = None
_gen = None
VP = ctypes.c_void_p


def lib():
    """The attention library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblinattn.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        DP = ctypes.POINTER(AttnDesc)
        L.la_status_string.restype = ctypes.c_char_p
        L.la_status_string.argtypes = [ctypes.c_int]
        L.la_last_hip_error.restype = ctypes.c_int32
        L.la_version.argtypes = [ctypes.POINTER(ctypes.c_int32)] * 2
        L.la_workspace_size.argtypes = [DP, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.la_forward.argtypes = [DP, VP, VP, VP, VP, VP, VP, VP, ctypes.c_size_t, VP]
        L.la_backward.argtypes = [DP, VP, VP, VP, VP, VP, VP, VP, VP, VP, VP, ctypes.c_size_t, VP]
        L.la_apply.argtypes = [DP, VP, VP, VP, VP, VP, ctypes.c_size_t, VP]
        L.la_forward_gated.argtypes = [DP, VP, VP, VP, VP, VP, ctypes.c_double, VP, VP, VP, VP,
                                       ctypes.c_size_t, VP]
        L.la_apply_gated.argtypes = [DP, VP, VP, VP, VP, VP, ctypes.c_double, VP, VP,
                                     ctypes.c_size_t, VP]
        for name in ("la_version", "la_workspace_size", "la_forward", "la_backward", "la_apply",
                     "la_forward_gated", "la_apply_gated"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def gen_lib():
    global _gen
    if _gen is None:
        if not os.path.exists(GEN_PATH):
            raise RuntimeError("liblagen.so is not built (run __graft_entry__.build())")
        G = ctypes.CDLL(GEN_PATH)
        G.la_gen_fill.restype = ctypes.c_int32
        G.la_gen_fill.argtypes = [VP, ctypes.c_int32] + [ctypes.c_int64] * 7 + [
            ctypes.POINTER(GenSpec), VP]
        _gen = G
    return _gen


def _check(call, status):
    if status != 0:
        raise LaError(call, status, lib().la_last_hip_error() if status == 4 else 0)


def _dtype_code(t: torch.dtype) -> int:
    if t == torch.bfloat16:
        return LA_BF16
    if t == torch.float32:
        return LA_FP32
    raise TypeError("unsupported dtype %s (bfloat16 or float32)" % t)


def _strides(x: torch.Tensor):
    if x.dim() != 4:
        raise ValueError("expected a [B, H, N, d] tensor")
    if x.shape[3] > 1 and x.stride(3) != 1:
        raise ValueError("the feature axis must be contiguous")
    return x.stride(0), x.stride(1), x.stride(2)


def _dense(x: torch.Tensor) -> bool:
    """True if x's elements occupy distinct, gap-free storage (any order)."""
    expect = 1
    for st, n in sorted((st, n) for st, n in zip(x.stride(), x.shape) if n > 1):
        if st != expect:
            return False
        expect *= n
    return True


def make_desc(q: torch.Tensor, out: torch.Tensor) -> AttnDesc:
    B, H, N, d = q.shape
    isb, ish, isn = _strides(q)
    osb, osh, osn = _strides(out)
    return AttnDesc(B, H, N, d, _dtype_code(q.dtype), _dtype_code(out.dtype),
                    isb, ish, isn, osb, osh, osn, LA_PHI_ELU1, 0)


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def workspace_size(desc: AttnDesc, pass_: int) -> int:
    n = ctypes.c_size_t(0)
    _check("la_workspace_size", lib().la_workspace_size(ctypes.byref(desc), pass_, ctypes.byref(n)))
    return n.value


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns blocks aligned well beyond 256 bytes
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def _same_layout(ref: torch.Tensor, x: torch.Tensor, name: str):
    if x.shape != ref.shape or x.dtype != ref.dtype or x.device != ref.device:
        raise ValueError("%s must match q in shape, dtype and device" % name)
    if _strides(x) != _strides(ref):
        raise ValueError("%s must have the same strides as q" % name)


def forward(q, k, v, out_dtype=None, return_summary=False, out=None):
    """O = linear attention of (q, k, v), [B, H, N, d] tensors on the GPU.

    With return_summary=True also returns S [B,H,d,d] and z [B,H,d] (FP64).
    """
    _same_layout(q, k, "k")
    _same_layout(q, v, "v")
    if not q.is_cuda:
        raise ValueError("inputs must be GPU tensors")
    B, H, N, d = q.shape
    if out is None:
        out = torch.empty((B, H, N, d), dtype=out_dtype or q.dtype, device=q.device)
    desc = make_desc(q, out)
    ws = _workspace(workspace_size(desc, 0), q.device)
    S = z = None
    if return_summary:
        S = torch.empty((B, H, d, d), dtype=torch.float64, device=q.device)
        z = torch.empty((B, H, d), dtype=torch.float64, device=q.device)
    _check("la_forward", lib().la_forward(
        ctypes.byref(desc), q.data_ptr(), k.data_ptr(), v.data_ptr(), out.data_ptr(),
        S.data_ptr() if S is not None else None, z.data_ptr() if z is not None else None,
        ws.data_ptr(), ws.numel(), _stream(q.device)))
    return (out, S, z) if return_summary else out


def forward_noalloc(q, k, v, out, S, z):
    """la_forward_noalloc: the forward pass into caller-allocated out, S
    [B,H,d,d] and z [B,H,d] (float64), with the library's fixed device
    scratch as workspace, so the call allocates nothing."""
    _same_layout(q, k, "k")
    _same_layout(q, v, "v")
    B, H, N, d = q.shape
    if S.shape != (B, H, d, d) or z.shape != (B, H, d) or S.dtype != torch.float64 \
            or z.dtype != torch.float64 or not (S.is_contiguous() and z.is_contiguous()):
        raise ValueError("S must be [B,H,d,d] and z [B,H,d], contiguous float64")
    desc = make_desc(q, out)
    L = lib()
    if not getattr(L, "_noalloc_typed", False):
        L.la_forward_noalloc.argtypes = [ctypes.POINTER(AttnDesc), VP, VP, VP, VP, VP, VP, VP]
        L.la_forward_noalloc.restype = ctypes.c_int
        L._noalloc_typed = True
    _check("la_forward_noalloc", L.la_forward_noalloc(
        ctypes.byref(desc), q.data_ptr(), k.data_ptr(), v.data_ptr(), out.data_ptr(),
        S.data_ptr(), z.data_ptr(), _stream(q.device)))
    return out


def apply(q, S, z, out_dtype=None, out=None):
    """O from queries and a summary (S, z) computed earlier by forward()."""
    if not q.is_cuda:
        raise ValueError("inputs must be GPU tensors")
    B, H, N, d = q.shape
    if S.shape != (B, H, d, d) or z.shape != (B, H, d) or S.dtype != torch.float64 \
            or z.dtype != torch.float64:
        raise ValueError("S must be [B,H,d,d] and z [B,H,d], float64")
    S = S.contiguous()
    z = z.contiguous()
    if out is None:
        out = torch.empty((B, H, N, d), dtype=out_dtype or q.dtype, device=q.device)
    desc = make_desc(q, out)
    ws = _workspace(workspace_size(desc, 2), q.device)
    _check("la_apply", lib().la_apply(ctypes.byref(desc), q.data_ptr(), S.data_ptr(), z.data_ptr(),
                                      out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(q.device)))
    return out


def _gate_args(q, other, out, sigma):
    """Checks the other branch's output against out; sigma as a [B] float64
    device tensor (a Python number is one level for every batch element)."""
    if other.shape != out.shape or other.dtype != out.dtype or other.device != out.device:
        raise ValueError("other must match the output in shape, dtype and device")
    if _strides(other) != _strides(out):
        raise ValueError("other must have the output's strides")
    B = q.shape[0]
    if not torch.is_tensor(sigma):
        sigma = torch.full((B,), float(sigma), dtype=torch.float64, device=q.device)
    if sigma.shape != (B,) or sigma.dtype != torch.float64 or sigma.device != q.device:
        raise ValueError("sigma must be a [B] float64 tensor on q's device")
    return sigma.contiguous()


def forward_gated(q, k, v, other, sigma, sigma_data=0.5, out=None, return_summary=False):
    """Noise-gated blend g*A + (1 - g)*other of this attention A with another
    branch's output, g = sigma_data / (sigma_data + sigma[b]) per batch
    element; `other` may be `out` (in place)."""
    _same_layout(q, k, "k")
    _same_layout(q, v, "v")
    if not q.is_cuda:
        raise ValueError("inputs must be GPU tensors")
    B, H, N, d = q.shape
    if out is None:
        out = torch.empty((B, H, N, d), dtype=other.dtype, device=q.device)
    sigma = _gate_args(q, other, out, sigma)
    desc = make_desc(q, out)
    ws = _workspace(workspace_size(desc, 0), q.device)
    S = z = None
    if return_summary:
        S = torch.empty((B, H, d, d), dtype=torch.float64, device=q.device)
        z = torch.empty((B, H, d), dtype=torch.float64, device=q.device)
    _check("la_forward_gated", lib().la_forward_gated(
        ctypes.byref(desc), q.data_ptr(), k.data_ptr(), v.data_ptr(), other.data_ptr(),
        sigma.data_ptr(), float(sigma_data), out.data_ptr(),
        S.data_ptr() if S is not None else None, z.data_ptr() if z is not None else None,
        ws.data_ptr(), ws.numel(), _stream(q.device)))
    return (out, S, z) if return_summary else out


def apply_gated(q, S, z, other, sigma, sigma_data=0.5, out=None):
    """apply() blended with another branch's output as in forward_gated()."""
    if not q.is_cuda:
        raise ValueError("inputs must be GPU tensors")
    B, H, N, d = q.shape
    if S.shape != (B, H, d, d) or z.shape != (B, H, d) or S.dtype != torch.float64 \
            or z.dtype != torch.float64:
        raise ValueError("S must be [B,H,d,d] and z [B,H,d], float64")
    S = S.contiguous()
    z = z.contiguous()
    if out is None:
        out = torch.empty((B, H, N, d), dtype=other.dtype, device=q.device)
    sigma = _gate_args(q, other, out, sigma)
    desc = make_desc(q, out)
    ws = _workspace(workspace_size(desc, 2), q.device)
    _check("la_apply_gated", lib().la_apply_gated(
        ctypes.byref(desc), q.data_ptr(), S.data_ptr(), z.data_ptr(), other.data_ptr(),
        sigma.data_ptr(), float(sigma_data), out.data_ptr(), ws.data_ptr(), ws.numel(),
        _stream(q.device)))
    return out


def backward(q, k, v, S, z, dout, grad_dtype=None):
    """dQ, dK, dV of L = <O, dout> given the forward's S and z."""
    _same_layout(q, k, "k")
    _same_layout(q, v, "v")
    _same_layout(q, dout, "dout")
    B, H, N, d = q.shape
    gd = grad_dtype or q.dtype
    dq = torch.empty((B, H, N, d), dtype=gd, device=q.device)
    dk = torch.empty_like(dq)
    dv = torch.empty_like(dq)
    S = S.contiguous()
    z = z.contiguous()
    desc = make_desc(q, dq)
    ws = _workspace(workspace_size(desc, 1), q.device)
    _check("la_backward", lib().la_backward(
        ctypes.byref(desc), q.data_ptr(), k.data_ptr(), v.data_ptr(), S.data_ptr(),
        z.data_ptr(), dout.data_ptr(), dq.data_ptr(), dk.data_ptr(), dv.data_ptr(),
        ws.data_ptr(), ws.numel(), _stream(q.device)))
    return dq, dk, dv


def gen_fill(x: torch.Tensor, seed: int, stream_id: int, mean=0.0, std=1.0, grid=None,
             amplitude=1.0, tensor_id=None, b_offset=0):
    """Fill a [B,H,N,d] GPU tensor with the seeded synthetic inputs."""
    B, H, N, d = x.shape
    sb, sh, sn = _strides(x)
    T, nlat, nlon = grid if grid else (0, 0, 0)
    spec = GenSpec(seed, stream_id, stream_id if tensor_id is None else tensor_id,
                   mean, std, T, nlat, nlon, amplitude, b_offset)
    rc = gen_lib().la_gen_fill(x.data_ptr(), _dtype_code(x.dtype), B, H, N, d, sb, sh, sn,
                               ctypes.byref(spec), _stream(x.device))
    if rc != 0:
        raise LaError("la_gen_fill", rc)
    return x


class LinearAttention(torch.autograd.Function):
    """Linear global attention with the hand-written backward.

    The forward saves q, k, v and the FP64 summary (S, z); phi(Q) and phi(K)
    are recomputed in the backward, never stored.
    """

    @staticmethod
    def forward(ctx, q, k, v):
        o, S, z = forward(q, k, v, return_summary=True)
        ctx.save_for_backward(q, k, v, S, z)
        return o

    @staticmethod
    def backward(ctx, do):
        q, k, v, S, z = ctx.saved_tensors
        # The kernels read dO with q's dtype and strides.  Autograd may hand
        # over any layout (the gradient of o.sum() is an expanded tensor with
        # all strides 0, a transposed gradient has a non-unit feature
        # stride): compare the raw strides and copy into q's layout when they
        # differ, or into a dense layout for all four when q's own layout
        # overlaps itself (a broadcast q).
        if do.dtype != q.dtype or do.stride() != q.stride():
            if _dense(q):
                buf = torch.empty_strided(q.shape, q.stride(), dtype=q.dtype, device=q.device)
                do = buf.copy_(do)
            else:
                q, k, v = (t.contiguous() for t in (q, k, v))
                do = do.to(q.dtype).contiguous()
        return backward(q, k, v, S, z, do)


def linear_attention(q, k, v):
    return LinearAttention.apply(q, k, v)


def profile_enable(on: bool):
    _check("la_profile_enable", lib().la_profile_enable(1 if on else 0))


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


def profile_read():
    """{kernel name: (launches, total milliseconds)} since profile_enable(True)."""
    L = lib()
    L.la_profile_read.argtypes = [ctypes.POINTER(KernelStat), ctypes.c_int32,
                                  ctypes.POINTER(ctypes.c_int32)]
    L.la_profile_read.restype = ctypes.c_int
    cap = 64
    arr = (KernelStat * cap)()
    n = ctypes.c_int32(0)
    _check("la_profile_read", L.la_profile_read(arr, cap, ctypes.byref(n)))
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(min(n.value, cap))}


class Plan:
    """Preallocated forward + backward of one problem shape: outputs, the
    FP64 summary and both workspaces are allocated once, so repeated calls
    only enqueue kernels."""

    def __init__(self, q, k, v, dout=None, out_dtype=None):
        _same_layout(q, k, "k")
        _same_layout(q, v, "v")
        B, H, N, d = q.shape
        dev = q.device
        self.q, self.k, self.v, self.dout = q, k, v, dout
        od = out_dtype or q.dtype
        self.o = torch.empty((B, H, N, d), dtype=od, device=dev)
        self.S = torch.empty((B, H, d, d), dtype=torch.float64, device=dev)
        self.z = torch.empty((B, H, d), dtype=torch.float64, device=dev)
        self.desc = make_desc(q, self.o)
        self.ws_f = _workspace(workspace_size(self.desc, 0), dev)
        if dout is not None:
            _same_layout(q, dout, "dout")
            self.dq = torch.empty_like(self.o)
            self.dk = torch.empty_like(self.o)
            self.dv = torch.empty_like(self.o)
            self.ws_b = _workspace(workspace_size(self.desc, 1), dev)
        self.stream = _stream(dev)
        self._d = ctypes.byref(self.desc)

    def forward(self):
        _check("la_forward", lib().la_forward(
            self._d, self.q.data_ptr(), self.k.data_ptr(), self.v.data_ptr(),
            self.o.data_ptr(), self.S.data_ptr(), self.z.data_ptr(), self.ws_f.data_ptr(),
            self.ws_f.numel(), self.stream))

    def backward(self):
        _check("la_backward", lib().la_backward(
            self._d, self.q.data_ptr(), self.k.data_ptr(), self.v.data_ptr(),
            self.S.data_ptr(), self.z.data_ptr(), self.dout.data_ptr(), self.dq.data_ptr(),
            self.dk.data_ptr(), self.dv.data_ptr(), self.ws_b.data_ptr(), self.ws_b.numel(),
            self.stream))


class TileDesc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int64 * 3), ("core", ctypes.c_int64 * 3),
                ("halo", ctypes.c_int64 * 3), ("C", ctypes.c_int64), ("dtype", ctypes.c_int32)]


def _tile_desc(dims, core, halo, C, dtype):
    T3 = ctypes.c_int64 * 3
    return TileDesc(T3(*dims), T3(*core), T3(*halo), C, _dtype_code(dtype))


def _tile_lib():
    L = lib()
    if not getattr(L, "_tiles_typed", False):
        P = ctypes.POINTER
        L.la_tile_geometry.argtypes = [P(TileDesc), P(ctypes.c_int64), P(ctypes.c_int64)]
        L.la_tile_extract.argtypes = [P(TileDesc), VP, VP, VP]
        L.la_tile_blend.argtypes = [P(TileDesc), VP, VP, VP]
        for n in ("la_tile_geometry", "la_tile_extract", "la_tile_blend"):
            getattr(L, n).restype = ctypes.c_int
        L._tiles_typed = True
    return L


def tile_geometry(dims, core, halo):
    """(number of tiles, (Lt, Ly, Lx) tokens per tile)."""
    n = [-(-int(d) // int(c)) for d, c in zip(dims, core)]
    L = [int(c) + 2 * int(h) for c, h in zip(core, halo)]
    return n[0] * n[1] * n[2], tuple(L)


def tile_extract(field, core, halo):
    """Tiles [n_tiles, Lt, Ly, Lx, C] with halos of a [T, Y, X, C] field."""
    if field.dim() != 4 or not field.is_contiguous():
        raise ValueError("field must be a contiguous [T, Y, X, C] tensor")
    T, Y, X, C = field.shape
    desc = _tile_desc((T, Y, X), core, halo, C, field.dtype)
    n, L = tile_geometry((T, Y, X), core, halo)
    tiles = torch.empty((n,) + L + (C,), dtype=field.dtype, device=field.device)
    _check("la_tile_extract", _tile_lib().la_tile_extract(ctypes.byref(desc), field.data_ptr(),
                                                          tiles.data_ptr(), _stream(field.device)))
    return tiles


def tile_blend(tiles, dims, core, halo):
    """Hann-weighted overlap average of tiles back onto a [T, Y, X, C] field."""
    if not tiles.is_contiguous():
        raise ValueError("tiles must be contiguous")
    C = tiles.shape[-1]
    desc = _tile_desc(dims, core, halo, C, tiles.dtype)
    n, L = tile_geometry(dims, core, halo)
    if tiles.shape != (n,) + L + (C,):
        raise ValueError("tiles must be [n_tiles, Lt, Ly, Lx, C] = %s" % (((n,) + L + (C,)),))
    out = torch.empty(tuple(dims) + (C,), dtype=tiles.dtype, device=tiles.device)
    _check("la_tile_blend", _tile_lib().la_tile_blend(ctypes.byref(desc), tiles.data_ptr(),
                                                      out.data_ptr(), _stream(tiles.device)))
    return out


def tiled_attention(q, k, v, core, halo):
    """The paper's tiled global attention step: split the [T, Y, X, H*d]
    token fields into overlapping tiles, run linear attention inside every
    tile (tiles as the batch, heads packed in the channels), and blend the
    tile outputs with Hann weights.  q, k, v: [T, Y, X, H, d] tensors."""
    T, Y, X, H, d = q.shape
    flat = lambda t: t.reshape(T, Y, X, H * d)
    tq, tk, tv = (tile_extract(flat(t), core, halo) for t in (q, k, v))
    n = tq.shape[0]
    N = tq.shape[1] * tq.shape[2] * tq.shape[3]
    view = lambda t: t.view(n, N, H, d).permute(0, 2, 1, 3)  # [B=tiles, H, N, d] view
    to = torch.empty_like(tq)
    forward(view(tq), view(tk), view(tv), out=view(to))
    return tile_blend(to, (T, Y, X), core, halo).view(T, Y, X, H, d)


def tiled_forward(q, k, v, core, halo, out=None):
    """The tiled attention step of tiled_attention() in two fused passes
    (la_tiled_forward): q, k, v [T, Y, X, H, d] bf16 tensors, contiguous;
    no tile is materialised."""
    for t in (q, k, v):
        if t.dim() != 5 or not t.is_contiguous() or t.shape != q.shape or t.dtype != q.dtype:
            raise ValueError("q, k, v must be contiguous [T, Y, X, H, d] tensors of one shape")
    T, Y, X, H, d = q.shape
    desc = _tile_desc((T, Y, X), core, halo, H * d, q.dtype)
    L = lib()
    if not getattr(L, "_tiled_typed", False):
        P = ctypes.POINTER
        L.la_tiled_workspace_size.argtypes = [P(TileDesc), ctypes.c_int64, P(ctypes.c_size_t)]
        L.la_tiled_forward.argtypes = [P(TileDesc), ctypes.c_int64, VP, VP, VP, VP, VP,
                                       ctypes.c_size_t, VP]
        L.la_tiled_workspace_size.restype = ctypes.c_int
        L.la_tiled_forward.restype = ctypes.c_int
        L._tiled_typed = True
    n = ctypes.c_size_t(0)
    _check("la_tiled_workspace_size", L.la_tiled_workspace_size(ctypes.byref(desc), H, ctypes.byref(n)))
    ws = _workspace(n.value, q.device)
    if out is None:
        out = torch.empty_like(q)
    _check("la_tiled_forward", L.la_tiled_forward(
        ctypes.byref(desc), H, q.data_ptr(), k.data_ptr(), v.data_ptr(), out.data_ptr(),
        ws.data_ptr(), ws.numel(), _stream(q.device)))
    return out


STREAM_KINDS = {"read": 0, "write": 1, "copy": 2}


def stream_probe(kind: str, dst: torch.Tensor, src: torch.Tensor = None, pattern: int = 0):
    """One plain HBM stream over dst's bytes (read: src's bytes): "read"
    reads src (dst receives at most 16 bytes), "write" fills dst with the
    32-bit `pattern`, "copy" copies src into dst.  Contiguous device tensors;
    runs on torch's current stream."""
    k = STREAM_KINDS[kind]
    L = lib()
    if not getattr(L, "_probe_typed", False):
        L.la_stream_probe.argtypes = [ctypes.c_int32, VP, VP, ctypes.c_size_t, ctypes.c_uint32, VP]
        L.la_stream_probe.restype = ctypes.c_int
        L._probe_typed = True
    for t in (dst, src):
        if t is not None and not t.is_contiguous():
            raise ValueError("stream_probe needs contiguous tensors")
    nbytes = (src if kind == "read" else dst).numel() * (src if kind == "read" else dst).element_size()
    if kind == "copy" and src.numel() * src.element_size() != nbytes:
        raise ValueError("copy: src and dst differ in size")
    if kind == "read" and dst.numel() * dst.element_size() < 16:
        raise ValueError("read: dst must hold 16 bytes")
    _check("la_stream_probe", L.la_stream_probe(k, src.data_ptr() if src is not None else None,
                                                dst.data_ptr(), nbytes, pattern & 0xFFFFFFFF,
                                                _stream(dst.device)))
