"""Pins of the oracle's tile operations (tiles with halos, Hann-weighted
overlap averaging): a hand-derived example, closed forms and invariants."""
import math

import numpy as np
import pytest

import oracle


def rnd(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_hann_window_values_and_partition_of_unity():
    # sin^2(pi/8) = (2 - sqrt2)/4, sin^2(3 pi/8) = (2 + sqrt2)/4
    assert abs(oracle.hann(0, 4) - (2 - math.sqrt(2)) / 4) < 1e-15
    assert abs(oracle.hann(1, 4) - (2 + math.sqrt(2)) / 4) < 1e-15
    for L in (2, 4, 6, 10, 32):
        for u in range(L // 2):
            # Hann windows shifted by half their length sum to one
            assert abs(oracle.hann(u, L) + oracle.hann(u + L // 2, L) - 1.0) < 1e-14
        assert all(oracle.hann(u, L) > 0 for u in range(L))
        assert all(abs(oracle.hann(u, L) - oracle.hann(L - 1 - u, L)) < 1e-15 for u in range(L))


def test_hand_example_one_dimension():
    # X = 4 positions, cores of 2, halo 1: tile 0 spans [-1, 3), tile 1 [1, 5)
    a = (2 - math.sqrt(2)) / 4
    b = (2 + math.sqrt(2)) / 4
    d0 = np.array([10.0, 20.0, 30.0, 40.0])   # tile 0 at x = -1, 0, 1, 2
    d1 = np.array([50.0, 60.0, 70.0, 80.0])   # tile 1 at x = 1, 2, 3, 4
    tiles = np.stack([d0, d1]).reshape(2, 1, 1, 4, 1)
    out = oracle.tile_blend(tiles, (1, 1, 4), (1, 1, 2), (0, 0, 1)).ravel()
    expect = [20.0, (b * 30.0 + a * 50.0) / (a + b), (a * 40.0 + b * 60.0) / (a + b), 70.0]
    np.testing.assert_allclose(out, expect, rtol=1e-15)


GEOMS = [((1, 6, 8), (1, 3, 4), (0, 1, 2)), ((3, 7, 5), (2, 3, 2), (1, 1, 1)),
         ((4, 4, 4), (2, 2, 2), (2, 2, 2)), ((2, 9, 11), (2, 4, 5), (0, 0, 0)),
         ((5, 5, 5), (8, 8, 8), (0, 3, 1))]


@pytest.mark.parametrize("dims,core,halo", GEOMS)
def test_blend_of_consistent_tiles_is_the_field(dims, core, halo):
    x = rnd(dims + (3,), 1)
    t = oracle.tile_extract(x, core, halo)
    np.testing.assert_allclose(oracle.tile_blend(t, dims, core, halo), x, rtol=0, atol=1e-14)


def test_extract_clamps_at_the_borders():
    x = rnd((1, 3, 3, 2), 2)
    t = oracle.tile_extract(x, (1, 3, 3), (0, 1, 1))  # one tile, 5 x 5 with clamped ring
    assert t.shape == (1, 1, 5, 5, 2)
    inner = t[0, 0, 1:4, 1:4]
    np.testing.assert_array_equal(inner, x[0])
    np.testing.assert_array_equal(t[0, 0, 0, 1:4], x[0, 0])      # top ring = first row
    np.testing.assert_array_equal(t[0, 0, 0, 0], x[0, 0, 0])     # corner = corner value
    np.testing.assert_array_equal(t[0, 0, 4, 4], x[0, 2, 2])


def test_no_halo_blend_copies_each_core():
    dims, core, halo = (1, 4, 6), (1, 2, 3), (0, 0, 0)
    n, L = oracle.tile_geometry(dims, core, halo)
    t = rnd((n[0] * n[1] * n[2],) + tuple(L) + (2,), 3)
    out = oracle.tile_blend(t, dims, core, halo)
    for tile in range(t.shape[0]):
        i, j = tile // n[2], tile % n[2]
        np.testing.assert_array_equal(out[0, 2 * i:2 * i + 2, 3 * j:3 * j + 3], t[tile, 0])


def test_blend_is_linear_and_stays_in_the_hull():
    dims, core, halo = (2, 6, 6), (1, 3, 3), (1, 1, 1)
    n, L = oracle.tile_geometry(dims, core, halo)
    shape = (n[0] * n[1] * n[2],) + tuple(L) + (2,)
    t1, t2 = rnd(shape, 4), rnd(shape, 5)
    b = lambda t: oracle.tile_blend(t, dims, core, halo)
    np.testing.assert_allclose(b(2.5 * t1 - t2), 2.5 * b(t1) - b(t2), atol=1e-13)
    assert b(t1).max() <= t1.max() + 1e-14 and b(t1).min() >= t1.min() - 1e-14
    np.testing.assert_allclose(b(np.full(shape, 7.25)), 7.25, rtol=1e-15)


def test_bad_geometry_is_rejected():
    with pytest.raises(ValueError):
        oracle.tile_extract(np.zeros((1, 4, 4, 1)), (1, 2, 2), (0, 3, 0))  # halo > core
