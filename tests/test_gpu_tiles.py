"""Tiles with halos and Hann-weighted overlap averaging on the GPU against
the oracle, and the tiled attention step composed from them."""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_16590_amd as la
from gpu_util import TOL, as64, make_inputs, normwise, require_gpu, to_device, to_host

pytestmark = pytest.mark.gpu

GEOMS = [((1, 32, 64), (1, 16, 16), (0, 4, 4)), ((4, 9, 13), (2, 4, 5), (1, 2, 2)),
         ((2, 8, 8), (2, 8, 8), (0, 0, 0)), ((3, 10, 7), (1, 3, 2), (1, 3, 2))]


def field(dims, C, dtype, seed):
    T, Y, X = dims
    (x,) = make_inputs((1, 1, T * Y * X, C), dtype, seed, streams=(0,))
    return x.reshape(T, Y, X, C)


@pytest.mark.parametrize("dims,core,halo", GEOMS)
@pytest.mark.parametrize("dtype", ["bf16", "fp32"])
def test_extract_and_blend_match_oracle(dims, core, halo, dtype):
    dev = require_gpu()
    x = field(dims, 16, dtype, 41)
    tx = to_device(x, dev)
    tiles = la.tile_extract(tx, core, halo)
    torch.cuda.synchronize()
    ref_tiles = oracle.tile_extract(as64(x), core, halo)
    np.testing.assert_array_equal(as64(tiles), ref_tiles)  # a gather: bit-exact
    # blend arbitrary (inconsistent) tiles
    n, L = la.tile_geometry(dims, core, halo)
    (raw,) = make_inputs((1, 1, n * L[0] * L[1] * L[2], 16), dtype, 42, streams=(1,))
    raw = raw.reshape((n,) + L + (16,))
    out = la.tile_blend(to_device(raw, dev), dims, core, halo)
    torch.cuda.synchronize()
    ref = oracle.tile_blend(as64(raw), dims, core, halo)
    err = normwise(as64(out)[None, None], ref[None, None])
    assert err < (4e-3 if dtype == "bf16" else 1e-6), err
    # consistent tiles blend back to the field
    back = la.tile_blend(tiles, dims, core, halo)
    torch.cuda.synchronize()
    assert normwise(as64(back)[None, None], as64(x)[None, None]) < (4e-3 if dtype == "bf16" else 1e-6)


def test_tiled_attention_matches_oracle_composition():
    dev = require_gpu()
    T, Y, X, H, d = 2, 16, 24, 2, 32
    core, halo = (1, 8, 8), (0, 2, 3)
    q, k, v = (field((T, Y, X), H * d, "bf16", s) for s in (43, 44, 45))
    tq, tk, tv = (to_device(a, dev).view(T, Y, X, H, d) for a in (q, k, v))
    out = la.tiled_attention(tq, tk, tv, core, halo)
    torch.cuda.synchronize()
    # oracle: the same composition, in FP64
    n, L = la.tile_geometry((T, Y, X), core, halo)
    N = L[0] * L[1] * L[2]
    tiles = [oracle.tile_extract(as64(a), core, halo).reshape(n, N, H, d).transpose(0, 2, 1, 3)
             for a in (q, k, v)]
    o_tiles = oracle.forward(*(np.ascontiguousarray(t) for t in tiles))
    o_tiles = o_tiles.transpose(0, 2, 1, 3).reshape((n,) + L + (H * d,))
    ref = oracle.tile_blend(o_tiles, (T, Y, X), core, halo)
    err = normwise(as64(out).reshape(1, 1, -1), ref.reshape(1, 1, -1))
    print("tiled attention normwise", err)
    assert err < TOL["bf16"]


def test_one_tile_is_global_attention():
    dev = require_gpu()
    T, Y, X, H, d = 2, 8, 16, 2, 64
    q, k, v = (field((T, Y, X), H * d, "fp32", s) for s in (46, 47, 48))
    tq, tk, tv = (to_device(a, dev).view(T, Y, X, H, d) for a in (q, k, v))
    out = la.tiled_attention(tq, tk, tv, (T, Y, X), (0, 0, 0))
    glob = la.forward(*(t.reshape(1, T * Y * X, H, d).permute(0, 2, 1, 3) for t in (tq, tk, tv)))
    torch.cuda.synchronize()
    a = out.reshape(T * Y * X, H, d)
    b = glob[0].permute(1, 0, 2)
    assert torch.allclose(a, b, rtol=1e-6, atol=1e-7)


def oracle_tiled(q, k, v, dims, core, halo, H, d):
    """The tiled step composed in the oracle (FP64): extract, attention per
    tile (tiles as the batch, heads in the channels), Hann blend."""
    n, L = la.tile_geometry(dims, core, halo)
    N = L[0] * L[1] * L[2]
    tiles = [oracle.tile_extract(as64(a), core, halo).reshape(n, N, H, d).transpose(0, 2, 1, 3)
             for a in (q, k, v)]
    o_tiles = oracle.forward(*(np.ascontiguousarray(t) for t in tiles))
    o_tiles = o_tiles.transpose(0, 2, 1, 3).reshape((n,) + L + (H * d,))
    return oracle.tile_blend(o_tiles, dims, core, halo)


FUSED = [((2, 16, 24), (1, 8, 8), (0, 2, 3), 2, 32),     # ragged x tiles
         ((4, 9, 13), (2, 4, 5), (1, 2, 2), 3, 16),      # ragged everywhere
         ((3, 16, 32), (2, 8, 16), (1, 4, 8), 2, 64),    # halos of half a core
         ((8, 8, 16), (8, 8, 16), (0, 0, 0), 1, 64),     # one tile: global attention
         ((5, 7, 11), (3, 3, 4), (0, 1, 2), 4, 16),
         # chunks of two tiles along t (planes shared inside a chunk) with
         # halos of half a core in t
         ((32, 32, 32), (4, 8, 8), (2, 2, 2), 16, 16),
         # a footprint split in two parts (FP32 runs of 16,384 tokens)
         ((8, 64, 64), (4, 64, 64), (2, 0, 0), 1, 32),
         # cores larger than the grid: one tile per dimension, its extended
         # range clamped on both sides
         ((3, 5, 7), (4, 8, 8), (2, 2, 4), 2, 16)]


@pytest.mark.parametrize("dims,core,halo,H,d", FUSED)
def test_fused_tiled_forward_matches_oracle_composition(dims, core, halo, H, d):
    # the whole step in two passes (no tile stored) against the oracle's
    # extract -> attention per tile -> blend
    dev = require_gpu()
    T, Y, X = dims
    q, k, v = (field(dims, H * d, "bf16", s) for s in (51, 52, 53))
    tq, tk, tv = (to_device(a, dev).view(T, Y, X, H, d) for a in (q, k, v))
    print("fused tiled", dims, core, halo, H, d, flush=True)
    out = la.tiled_forward(tq, tk, tv, core, halo)
    unfused = la.tiled_attention(tq, tk, tv, core, halo)
    torch.cuda.synchronize()
    ref = oracle_tiled(q, k, v, dims, core, halo, H, d)
    err = normwise(as64(out).reshape(1, 1, -1), ref.reshape(1, 1, -1))
    err_unfused = normwise(as64(unfused).reshape(1, 1, -1), ref.reshape(1, 1, -1))
    print("  normwise: fused", err, "unfused", err_unfused, flush=True)
    assert err < TOL["bf16"]
    # the same arithmetic up to the bf16 rounding of the unfused tile outputs
    # (and S_t as its hi part here): both within a few 1e-3 of each other
    assert normwise(as64(out).reshape(1, 1, -1), as64(unfused).reshape(1, 1, -1)) < 1e-2


def random_geometries(count, seed):
    # seeded ragged geometries: any grid extent from 1, cores up to the
    # extent (ceil-divided tiles, the last one clamped), halos from 0 to
    # half a core, 1 to 4 heads of d = 16, 32 or 64
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        dims = tuple(int(rng.integers(1, m)) for m in (7, 21, 27))
        core = tuple(int(rng.integers(1, n + 1)) for n in dims)
        halo = tuple(int(rng.integers(0, c // 2 + 1)) for c in core)
        L = [c + 2 * h for c, h in zip(core, halo)]
        if L[0] * L[1] * L[2] > 65536:
            continue
        out.append((dims, core, halo, int(rng.choice([1, 2, 4])), int(rng.choice([16, 32, 64]))))
    return out


@pytest.mark.parametrize("dims,core,halo,H,d", random_geometries(12, 2026))
def test_fused_tiled_forward_random_geometries(dims, core, halo, H, d):
    # the segment-pair decomposition of the tile summaries (zero-width
    # segments when a halo is 0 or half a core, clamped border planes,
    # extents of 1) against the oracle's extract -> attention -> blend
    dev = require_gpu()
    q, k, v = (field(dims, H * d, "bf16", s) for s in (61, 62, 63))
    tq, tk, tv = (to_device(a, dev).view(*dims, H, d) for a in (q, k, v))
    print("fused tiled (random)", dims, core, halo, H, d, flush=True)
    out = la.tiled_forward(tq, tk, tv, core, halo)
    torch.cuda.synchronize()
    ref = oracle_tiled(q, k, v, dims, core, halo, H, d)
    err = normwise(as64(out).reshape(1, 1, -1), ref.reshape(1, 1, -1))
    print("  normwise", err, flush=True)
    assert err < TOL["bf16"]


def test_fused_tiled_forward_bitwise_deterministic_and_full_grid_shape():
    # the paper's per-frame 32 x 64 patch grid, 16 frames, 4 heads of d = 64
    dev = require_gpu()
    dims, core, halo, H, d = (16, 32, 64), (4, 16, 16), (2, 8, 8), 4, 64
    q, k, v = (field(dims, H * d, "bf16", s) for s in (54, 55, 56))
    tq, tk, tv = (to_device(a, dev).view(*dims, H, d) for a in (q, k, v))
    a = la.tiled_forward(tq, tk, tv, core, halo)
    b = la.tiled_forward(tq, tk, tv, core, halo)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    ref = oracle_tiled(q, k, v, dims, core, halo, H, d)
    err = normwise(as64(a).reshape(1, 1, -1), ref.reshape(1, 1, -1))
    print("fused tiled 16x32x64 normwise", err, flush=True)
    assert err < TOL["bf16"]


def test_fused_tiled_forward_full_size_sampled_positions():
    # the bench's geometry: a T256 x 64 x 128 grid, 16 heads of d = 64,
    # cores 8 x 16 x 16, halos 2 x 4 x 4 (1,024 tiles of 6,912 tokens).
    # Sampled positions (corners, borders, halo overlaps, random) of two
    # heads against the oracle, one position at a time: every covering
    # tile's extended, border-clamped token set gathered from the field,
    # the oracle's summary of it applied to the position's query, and the
    # oracle's Hann weights
    dev = require_gpu()
    dims, core, halo, H, d = (256, 64, 128), (8, 16, 16), (2, 4, 4), 16, 64
    fields = []
    for sid in range(3):
        x = torch.empty(dims + (H, d), dtype=torch.bfloat16, device=dev)
        la.gen_fill(x.view(1, 1, -1, H * d), seed=1004, stream_id=sid)
        fields.append(x)
    out = la.tiled_forward(*fields, core, halo)
    torch.cuda.synchronize()
    _, L = la.tile_geometry(dims, core, halo)
    n = [(dims[k] + core[k] - 1) // core[k] for k in range(3)]  # tiles per dimension
    rng = np.random.default_rng(9)
    positions = [(0, 0, 0), (255, 63, 127), (0, 63, 0), (255, 0, 127), (7, 15, 15), (8, 16, 16),
                 (9, 17, 18), (6, 12, 12), (128, 32, 64)]
    positions += [tuple(int(rng.integers(0, m)) for m in dims) for _ in range(5)]
    got, want = [], []
    for p in positions:
        cover = []
        for k in range(3):
            cover.append([j for j in range(n[k])
                          if j * core[k] - halo[k] <= p[k] < (j + 1) * core[k] + halo[k]])
        for h in (0, 15):
            acc, wsum = np.zeros(d), 0.0
            q = to_host(fields[0][p[0], p[1], p[2], h].reshape(1, 1, 1, d))
            for jt in cover[0]:
                for jy in cover[1]:
                    for jx in cover[2]:
                        js = (jt, jy, jx)
                        w = 1.0
                        for k in range(3):
                            w *= oracle.hann(p[k] - (js[k] * core[k] - halo[k]), L[k])
                        if w == 0.0:
                            continue
                        idx = [torch.clamp(torch.arange(L[k], device=dev) + js[k] * core[k] - halo[k],
                                           0, dims[k] - 1) for k in range(3)]
                        gt, gy, gx = torch.meshgrid(*idx, indexing="ij")
                        kt, vt = (to_host(f[gt, gy, gx, h].reshape(1, 1, -1, d)) for f in fields[1:])
                        S_t, z_t = oracle.summary(as64(kt), as64(vt))
                        acc += w * oracle.apply(as64(q), S_t, z_t)[0, 0, 0]
                        wsum += w
            want.append(acc / wsum)
            got.append(as64(out[p[0], p[1], p[2], h].reshape(d)))
    err = np.linalg.norm(np.array(got) - np.array(want)) / np.linalg.norm(np.array(want))
    print("fused tiled full size, %d sampled (position, head) outputs: normwise %.3g"
          % (len(got), err), flush=True)
    assert err < TOL["bf16"]
