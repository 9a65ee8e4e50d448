"""FP64 CPU oracle of kernelised linear global attention (ctypes binding).

TEST INFRASTRUCTURE ONLY: only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  The product path
never does.  The arithmetic lives in ``oracle.c``; this file only builds it
and marshals numpy arrays.

Array conventions: inputs are numpy arrays of shape [B, H, N, d] with the
feature axis contiguous.  ``uint16`` arrays hold bfloat16 bit patterns;
``float32`` and ``float64`` arrays hold their values.  Outputs are dense
float64 arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with the host compiler (gcc, OpenMP)."""
    if not force and os.path.exists(_SO):
        return _SO
    src = os.path.join(_HERE, "oracle.c")
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


class _Tensor(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("dtype", ctypes.c_int32),
                ("sb", ctypes.c_int64), ("sh", ctypes.c_int64),
                ("sn", ctypes.c_int64)]


def use_library(path):
    """Load the oracle from another build of oracle.c (the mutation tests
    compile deliberately broken copies); returns the previous handle."""
    global _lib
    prev = _lib
    _lib = None
    _load(path)
    return prev


def restore_library(handle):
    global _lib
    _lib = handle


def _load(path=None):
    global _lib
    if _lib is None:
        if path is None and not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(path or _SO)
        T = _Tensor
        i64 = ctypes.c_int64
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_phi.restype = ctypes.c_double
        lib.oracle_phi.argtypes = [ctypes.c_double]
        lib.oracle_dphi.restype = ctypes.c_double
        lib.oracle_dphi.argtypes = [ctypes.c_double]
        lib.oracle_summary.argtypes = [i64, i64, i64, i64, T, T, dp, dp]
        lib.oracle_apply.argtypes = [i64, i64, i64, i64, T, dp, dp, dp]
        lib.oracle_forward.argtypes = [i64, i64, i64, i64, T, T, T, dp, dp, dp]
        lib.oracle_backward.argtypes = [i64, i64, i64, i64, T, T, T, T,
                                        dp, dp, dp, dp, dp]
        lib.oracle_backward_query.argtypes = [i64, i64, i64, i64, T, T, dp, dp, dp, dp, dp]
        lib.oracle_backward_key.argtypes = [i64, i64, i64, i64, T, T, dp, dp, dp, dp]
        lib.oracle_threads.restype = ctypes.c_int
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_tile_extract.argtypes = [i64p, i64p, i64p, i64, dp, dp]
        lib.oracle_tile_blend.argtypes = [i64p, i64p, i64p, i64, dp, dp]
        lib.oracle_hann.restype = ctypes.c_double
        lib.oracle_hann.argtypes = [i64, i64]
        lib.oracle_noise_gate.restype = ctypes.c_double
        lib.oracle_noise_gate.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.oracle_gated_mix.argtypes = [i64, i64, i64, i64, dp, T, dp, ctypes.c_double, dp]
        _lib = lib
    return _lib


_DTYPES = {np.dtype(np.uint16): 0, np.dtype(np.float32): 1,
           np.dtype(np.float64): 2}


def _tensor(a: np.ndarray) -> _Tensor:
    if a.ndim != 4:
        raise ValueError("expected a [B, H, N, d] array")
    if a.dtype not in _DTYPES:
        raise TypeError("unsupported dtype %s" % a.dtype)
    es = a.itemsize
    st = [s // es for s in a.strides]
    if any(s * es != t for s, t in zip(st, a.strides)) or (a.shape[3] > 1 and st[3] != 1):
        raise ValueError("feature axis must be contiguous")
    return _Tensor(a.ctypes.data, _DTYPES[a.dtype], st[0], st[1], st[2])


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def phi(x: float) -> float:
    return _load().oracle_phi(float(x))


def dphi(x: float) -> float:
    return _load().oracle_dphi(float(x))


def threads() -> int:
    return int(_load().oracle_threads())


def summary(k: np.ndarray, v: np.ndarray):
    """S [B,H,d,d] and z [B,H,d] in FP64."""
    B, H, N, d = k.shape
    assert v.shape == k.shape
    S = np.empty((B, H, d, d), np.float64)
    z = np.empty((B, H, d), np.float64)
    rc = _load().oracle_summary(B, H, N, d, _tensor(k), _tensor(v), _dptr(S), _dptr(z))
    if rc:
        raise ValueError("oracle_summary rejected its arguments")
    return S, z


def apply(q: np.ndarray, S: np.ndarray, z: np.ndarray) -> np.ndarray:
    """O [B,H,N,d] from queries and a given summary."""
    B, H, N, d = q.shape
    S = np.ascontiguousarray(S, np.float64)
    z = np.ascontiguousarray(z, np.float64)
    assert S.shape == (B, H, d, d) and z.shape == (B, H, d)
    o = np.empty((B, H, N, d), np.float64)
    rc = _load().oracle_apply(B, H, N, d, _tensor(q), _dptr(S), _dptr(z), _dptr(o))
    if rc:
        raise ValueError("oracle_apply rejected its arguments")
    return o


def forward(q: np.ndarray, k: np.ndarray, v: np.ndarray, want_summary=False):
    B, H, N, d = q.shape
    assert k.shape == q.shape and v.shape == q.shape
    o = np.empty((B, H, N, d), np.float64)
    S = np.empty((B, H, d, d), np.float64)
    z = np.empty((B, H, d), np.float64)
    rc = _load().oracle_forward(B, H, N, d, _tensor(q), _tensor(k), _tensor(v),
                                _dptr(o), _dptr(S), _dptr(z))
    if rc:
        raise ValueError("oracle_forward rejected its arguments")
    return (o, S, z) if want_summary else o


def backward(q, k, v, g, want_summary=False):
    """dQ, dK, dV (FP64) of L = <O, G>; optionally dS and dz too."""
    B, H, N, d = q.shape
    for a in (k, v, g):
        assert a.shape == q.shape
    dq = np.empty((B, H, N, d), np.float64)
    dk = np.empty_like(dq)
    dv = np.empty_like(dq)
    dS = np.empty((B, H, d, d), np.float64)
    dz = np.empty((B, H, d), np.float64)
    rc = _load().oracle_backward(B, H, N, d, _tensor(q), _tensor(k), _tensor(v),
                                 _tensor(g), _dptr(dq), _dptr(dk), _dptr(dv),
                                 _dptr(dS), _dptr(dz))
    if rc:
        raise ValueError("oracle_backward rejected its arguments")
    return (dq, dk, dv, dS, dz) if want_summary else (dq, dk, dv)


def backward_query(q, g, S, z, want_dq=True):
    """dQ (or None), dS, dz for the given queries against a given (S, z)."""
    B, H, N, d = q.shape
    assert g.shape == q.shape
    S = np.ascontiguousarray(S, np.float64)
    z = np.ascontiguousarray(z, np.float64)
    dq = np.empty((B, H, N, d), np.float64) if want_dq else None
    dS = np.empty((B, H, d, d), np.float64)
    dz = np.empty((B, H, d), np.float64)
    rc = _load().oracle_backward_query(B, H, N, d, _tensor(q), _tensor(g), _dptr(S), _dptr(z),
                                       _dptr(dq) if dq is not None else None, _dptr(dS), _dptr(dz))
    if rc:
        raise ValueError("oracle_backward_query rejected its arguments")
    return dq, dS, dz


def backward_key(k, v, dS, dz):
    """dK, dV for the given keys from (dS, dz)."""
    B, H, N, d = k.shape
    assert v.shape == k.shape
    dS = np.ascontiguousarray(dS, np.float64)
    dz = np.ascontiguousarray(dz, np.float64)
    dk = np.empty((B, H, N, d), np.float64)
    dv = np.empty_like(dk)
    rc = _load().oracle_backward_key(B, H, N, d, _tensor(k), _tensor(v), _dptr(dS), _dptr(dz),
                                     _dptr(dk), _dptr(dv))
    if rc:
        raise ValueError("oracle_backward_key rejected its arguments")
    return dk, dv


def _tri(v):
    return (ctypes.c_int64 * 3)(*[int(x) for x in v])


def tile_geometry(dims, core, halo):
    n = [-(-int(d) // int(c)) for d, c in zip(dims, core)]
    L = [int(c) + 2 * int(h) for c, h in zip(core, halo)]
    return n, L


def tile_extract(x, core, halo):
    """Tiles [n_tiles, Lt, Ly, Lx, C] (FP64) of a field x [T, Y, X, C]."""
    x = np.ascontiguousarray(x, np.float64)
    T, Y, X, C = x.shape
    n, L = tile_geometry((T, Y, X), core, halo)
    tiles = np.empty((n[0] * n[1] * n[2], L[0], L[1], L[2], C), np.float64)
    rc = _load().oracle_tile_extract(_tri((T, Y, X)), _tri(core), _tri(halo), C, _dptr(x), _dptr(tiles))
    if rc:
        raise ValueError("oracle_tile_extract rejected its arguments")
    return tiles


def tile_blend(tiles, dims, core, halo):
    """Hann-weighted overlap average of tiles back onto a [T, Y, X, C] field."""
    tiles = np.ascontiguousarray(tiles, np.float64)
    C = tiles.shape[-1]
    out = np.empty(tuple(dims) + (C,), np.float64)
    rc = _load().oracle_tile_blend(_tri(dims), _tri(core), _tri(halo), C, _dptr(tiles), _dptr(out))
    if rc:
        raise ValueError("oracle_tile_blend rejected its arguments")
    return out


def hann(u, L):
    return _load().oracle_hann(int(u), int(L))


def noise_gate(sigma: float, sigma_data: float = 0.5) -> float:
    """Spatial weight g(sigma) = sigma_data / (sigma_data + sigma)."""
    return _load().oracle_noise_gate(float(sigma), float(sigma_data))


def gated_mix(a, other, sigma, sigma_data=0.5):
    """g(sigma_b) * a + (1 - g(sigma_b)) * other per batch element (FP64)."""
    a = np.ascontiguousarray(a, np.float64)
    B, H, N, d = a.shape
    assert other.shape == a.shape
    sig = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, np.float64), (B,)))
    out = np.empty_like(a)
    rc = _load().oracle_gated_mix(B, H, N, d, _dptr(a), _tensor(other), _dptr(sig),
                                  float(sigma_data), _dptr(out))
    if rc:
        raise ValueError("oracle_gated_mix rejected its arguments")
    return out
