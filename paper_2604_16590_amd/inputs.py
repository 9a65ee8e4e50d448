"""Seeded synthetic inputs (host side).

This module holds the input generator only, none of the attention
arithmetic.  The same generator exists on the device (``csrc/gen.hip``,
library ``liblagen.so``); both follow one definition:

* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
  as easy as 1, 2, 3", SC 2011): a 10-round counter-based generator, round
  multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 /
  0xBB67AE85.
* Element e of the logical [b_offset + B, H, N, d] tensor (row-major flat
  index; a generated tensor holds batches b_offset .. b_offset + B - 1) takes
  pair index p = e >> 1 and Philox block c = p >> 1: counter
  (lo32 c, hi32 c, stream, 0), key (lo32 seed, hi32 seed).  The pair uses
  output words (w0, w1) = (x0, x1) for even p and (x2, x3) for odd p:
  u1 = ((w0 >> 9) + 0.5) * 2^-23, u2 = (w1 >> 8) * 2^-24; Box-Muller in FP32
  gives r = sqrt(-2 ln u1), and with t = 2 pi u2 the element takes
  r cos t (even e) or r sin t (odd e), where cos t and sin t are the FP32
  roundings of the exact values (the device evaluates them as sinpi/cospi
  of 2 u2, which is exact in FP32).
* value = mean + std * normal (+ the optional grid structure below), all in
  FP32, then (for bfloat16) float32 -> bfloat16 round to nearest even.
* Grid structure (spatiotemporal token grids of T frames x lat x lon
  patches): token n = (t * n_lat + i) * n_lon + j, lat_i = pi((i+1/2)/n_lat
  - 1/2), lon_j = 2 pi j / n_lon.  Channel c of tensor x (0 = Q, 1 = K,
  2 = V, 3 = upstream gradient) in head h adds
  A sin(m_c lon_j + l_c lat_i + 2 pi t / T + psi), m_c = 1 + c mod 4,
  l_c = 1 + c mod 3, psi = 2 pi frac(0.6180339887 (x H d + h d + c)).

bfloat16 tensors are carried on the host as uint16 bit patterns.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF

STREAM_Q, STREAM_K, STREAM_V, STREAM_G, STREAM_PERM, STREAM_SERVE = 0, 1, 2, 3, 4, 5


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 on uint64 arrays holding 32-bit words."""
    c0, c1, c2, c3 = (np.asarray(x, np.uint64) & MASK for x in (c0, c1, c2, c3))
    k0 = np.uint64(k0 & MASK) if np.isscalar(k0) else np.asarray(k0, np.uint64) & MASK
    k1 = np.uint64(k1 & MASK) if np.isscalar(k1) else np.asarray(k1, np.uint64) & MASK
    m0, m1 = np.uint64(M0), np.uint64(M1)
    w0, w1 = np.uint64(W0), np.uint64(W1)
    mask = np.uint64(MASK)
    s32 = np.uint64(32)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + w0) & mask
            k1 = (k1 + w1) & mask
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> s32, p0 & mask
        hi1, lo1 = p1 >> s32, p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


@dataclass
class GenSpec:
    seed: int
    stream: int
    mean: float = 0.0
    std: float = 1.0
    grid: tuple | None = None      # (T, n_lat, n_lon)
    amplitude: float = 1.0
    tensor_id: int = 0
    b_offset: int = 0              # first logical batch index


def normal_values(spec: GenSpec, flat_index: np.ndarray) -> np.ndarray:
    """FP64 N(0,1) draws for the given flat element indices."""
    e = np.asarray(flat_index, np.uint64)
    p = e >> np.uint64(1)
    c = p >> np.uint64(1)
    y0, y1, y2, y3 = philox4x32_10(c & np.uint64(MASK), c >> np.uint64(32),
                                   np.full_like(c, spec.stream), np.zeros_like(c),
                                   spec.seed & MASK, (spec.seed >> 32) & MASK)
    odd_pair = (p & np.uint64(1)).astype(bool)
    x0 = np.where(odd_pair, y2, y0)
    x1 = np.where(odd_pair, y3, y1)
    f32 = np.float32
    u1 = ((x0 >> np.uint64(9)).astype(f32) + f32(0.5)) * f32(2.0 ** -23)
    u2 = (x1 >> np.uint64(8)).astype(f32) * f32(2.0 ** -24)
    r = np.sqrt(f32(-2.0) * np.log(u1))
    t = (f32(2.0) * u2).astype(np.float64) * np.pi  # 2 pi u2, rounded once below
    odd = (e & np.uint64(1)).astype(bool)
    return np.where(odd, r * np.sin(t).astype(f32), r * np.cos(t).astype(f32)).astype(f32)


def structure_values(spec: GenSpec, B, H, N, d, flat_index) -> np.ndarray:
    if spec.grid is None:
        return np.zeros(np.shape(flat_index))
    T, nlat, nlon = spec.grid
    e = np.asarray(flat_index, np.int64)
    c = e % d
    n = (e // d) % N
    h = (e // (d * N)) % H
    j = n % nlon
    i = (n // nlon) % nlat
    t = n // (nlon * nlat)
    f32 = np.float32
    pi = f32(3.14159265358979)
    lat = pi * ((i.astype(f32) + f32(0.5)) / f32(nlat) - f32(0.5))
    lon = f32(2.0) * pi * j.astype(f32) / f32(nlon)
    m = (1 + c % 4).astype(f32)
    l = (1 + c % 3).astype(f32)
    key = f32(0.6180339887) * (spec.tensor_id * H * d + h * d + c).astype(f32)
    psi = f32(2.0) * pi * (key - np.floor(key))
    arg = m * lon + l * lat + f32(2.0) * pi * t.astype(f32) / f32(T) + psi
    return (f32(spec.amplitude) * np.sin(arg)).astype(f32)


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns, round to nearest even (NaN kept)."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)
    nan = np.isnan(np.asarray(x, np.float32))
    out = r.astype(np.uint16)
    out[nan] = 0x7FC0
    return out


def bf16_bits_to_f32(u: np.ndarray) -> np.ndarray:
    return (np.asarray(u, np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def generate(spec: GenSpec, shape, dtype: str) -> np.ndarray:
    """A dense [B, H, N, d] tensor: uint16 bf16 bits or float32."""
    B, H, N, d = shape
    idx = np.arange(B * H * N * d, dtype=np.int64)
    f32 = np.float32
    val = f32(spec.mean) + f32(spec.std) * normal_values(spec, idx + spec.b_offset * H * N * d)
    if spec.grid is not None:
        val = val + structure_values(spec, B, H, N, d, idx)
    f = val.astype(np.float32).reshape(shape)
    if dtype == "bf16":
        return f32_to_bf16_bits(f)
    if dtype == "fp32":
        return f
    raise ValueError(dtype)


def as_float64(a: np.ndarray) -> np.ndarray:
    """Exact FP64 view of a stored tensor (bf16 bits or float)."""
    if a.dtype == np.uint16:
        return bf16_bits_to_f32(a).astype(np.float64)
    return a.astype(np.float64)
