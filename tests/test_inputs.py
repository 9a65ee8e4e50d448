"""The seeded input generator (host definition, paper_2604_16590_amd.inputs).

Philox4x32-10 is checked against the known-answer vectors published with
the Random123 library (Salmon et al., SC 2011); the rest against what the
definition fixes: the pair -> (block, words) mapping, the Box-Muller
moments, round-to-nearest-even bf16, and the grid term.
"""
import numpy as np

from paper_2604_16590_amd import inputs

KAT = [  # (counter, key) -> output, Philox4x32 with 10 rounds
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def test_philox_known_answers():
    for ctr, key, want in KAT:
        out = inputs.philox4x32_10(*[np.array([c], np.uint64) for c in ctr], key[0], key[1])
        assert tuple(int(o[0]) for o in out) == want


def test_pairs_share_a_block_and_use_its_two_halves():
    spec = inputs.GenSpec(seed=77, stream=3)
    e = np.arange(8)
    z = inputs.normal_values(spec, e)
    # block 0 feeds pairs 0 (words x0, x1) and 1 (x2, x3); block 1 pairs 2, 3
    x = inputs.philox4x32_10(np.array([0, 1], np.uint64), np.zeros(2, np.uint64),
                             np.full(2, 3, np.uint64), np.zeros(2, np.uint64), 77, 0)
    f32 = np.float32
    for pair, (blk, lo) in enumerate(((0, 0), (0, 2), (1, 0), (1, 2))):
        w0, w1 = int(x[lo][blk]), int(x[lo + 1][blk])
        u1 = (f32(w0 >> 9) + f32(0.5)) * f32(2.0 ** -23)
        u2 = f32(w1 >> 8) * f32(2.0 ** -24)
        r = np.sqrt(f32(-2.0) * np.log(u1))
        t = 2.0 * np.pi * float(u2)
        assert z[2 * pair] == np.float32(r * np.float32(np.cos(t)))
        assert z[2 * pair + 1] == np.float32(r * np.float32(np.sin(t)))


def test_normal_moments_and_streams_differ():
    n = 1 << 18
    a = inputs.normal_values(inputs.GenSpec(seed=1, stream=0), np.arange(n)).astype(np.float64)
    b = inputs.normal_values(inputs.GenSpec(seed=1, stream=1), np.arange(n)).astype(np.float64)
    for x in (a, b):
        assert abs(x.mean()) < 5 / np.sqrt(n)
        assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / np.sqrt(n)


def test_b_offset_selects_later_batches():
    full = inputs.generate(inputs.GenSpec(seed=9, stream=2), (3, 2, 8, 4), "fp32")
    part = inputs.generate(inputs.GenSpec(seed=9, stream=2, b_offset=1), (2, 2, 8, 4), "fp32")
    assert np.array_equal(full[1:], part)


def test_bf16_round_to_nearest_even():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9, -2.5], np.float32)
    got = inputs.bf16_bits_to_f32(inputs.f32_to_bf16_bits(x))
    # ties go to the even mantissa: 1 + 2^-8 -> 1, 1 + 3*2^-8 -> 1 + 2^-6
    assert np.array_equal(got, np.array([1.0, 1.0, 1.0 + 2.0 ** -6, 1.0, -2.5], np.float32))


def test_grid_term_closed_form():
    T, nlat, nlon = 2, 3, 4
    spec = inputs.GenSpec(seed=0, stream=0, std=0.0, grid=(T, nlat, nlon), tensor_id=1)
    B, H, N, d = 1, 2, T * nlat * nlon, 5
    g = inputs.generate(spec, (B, H, N, d), "fp32").astype(np.float64)
    for h in range(H):
        for n in range(N):
            t, i, j = n // (nlat * nlon), (n // nlon) % nlat, n % nlon
            for c in range(d):
                lat = np.pi * ((i + 0.5) / nlat - 0.5)
                lon = 2 * np.pi * j / nlon
                key = 0.6180339887 * (1 * H * d + h * d + c)
                psi = 2 * np.pi * (key - np.floor(key))
                want = np.sin((1 + c % 4) * lon + (1 + c % 3) * lat + 2 * np.pi * t / T + psi)
                assert abs(g[0, h, n, c] - want) < 1e-4
