"""Forward parity: the HIP path (through the C ABI) against the FP64 oracle.

Inputs are seeded and identical on both sides (the oracle reads the very
bf16/fp32 values the kernels read).  Tolerances, normwise per (b, h):
bf16 inputs 2e-2, fp32 inputs 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_16590_amd as la
from paper_2604_16590_amd import inputs
from gpu_util import TOL, as64, make_inputs, max_rel, normwise, require_gpu, to_device, to_host

pytestmark = pytest.mark.gpu


def run_forward(q, k, v, out_dtype=None, summary=False):
    dev = require_gpu()
    tq, tk, tv = (to_device(x, dev) for x in (q, k, v))
    res = la.forward(tq, tk, tv, out_dtype=out_dtype, return_summary=summary)
    torch.cuda.synchronize()
    return res


def check(shape, dtype, seed, out_dtype=None, std=1.0, grid=None):
    q, k, v = make_inputs(shape, dtype, seed, std=std, grid=grid)
    print("case", shape, dtype, seed, out_dtype, flush=True)
    o, S, z = run_forward(q, k, v, out_dtype=out_dtype, summary=True)
    o_ref, S_ref, z_ref = oracle.forward(q, k, v, want_summary=True)
    err = normwise(as64(o), o_ref)
    tol = TOL[dtype]
    assert err < tol, (shape, dtype, err, max_rel(as64(o), o_ref))
    # FP64 summary: FP32 partial sums combined in FP64.  The bf16 path
    # rounds phi(k) to bf16 before the matrix cores, a relative error of at
    # most the bf16 unit roundoff u = 2^-8 ~ 3.9e-3 per term (the products
    # with the exact bf16 values and their FP32 sums add ~1e-6).  z sums
    # positive terms, so its error is within u of z; S's terms have both
    # signs, and their independent roundings keep its normwise error near
    # u/sqrt(3) ~ 2.3e-3 -- 4e-3 (u plus the FP32 sums) bounds both.  fp32
    # inputs carry only the FP32 sums over partials of at most 4,096
    # tokens: relative error ~ sqrt(128 matrix-core accumulations) * 2^-24
    # ~ 7e-7 of the partials' magnitude, within 1e-5 (S) and 1e-6 (z,
    # positive terms, no cancellation).
    assert normwise(S.cpu().numpy(), S_ref) < (4e-3 if dtype == "bf16" else 1e-5)
    assert normwise(z.cpu().numpy()[..., None], z_ref[..., None]) < (4e-3 if dtype == "bf16" else 1e-6)
    return err


def test_fp32_4096_tokens_vs_quadratic_form():
    # B1 H1 N4096 d64 fp32 N(0,1), checked against the brute-force form
    q, k, v = make_inputs((1, 1, 4096, 64), "fp32", 1000)
    o = run_forward(q, k, v)
    Q, K, V = (x.astype(np.float64) for x in (q, k, v))
    ph = lambda x: np.where(x > 0, x + 1.0, np.exp(np.minimum(x, 0.0)))
    A = ph(Q[0, 0]) @ ph(K[0, 0]).T
    ref = (A @ V[0, 0]) / A.sum(1, keepdims=True)
    err = normwise(as64(o), ref[None, None])
    print("fp32 N4096 normwise error", err, "max rel", max_rel(as64(o), ref[None, None]))
    assert err < TOL["fp32"]


@pytest.mark.parametrize("d", [16, 32, 64, 128])
@pytest.mark.parametrize("dtype", ["bf16", "fp32"])
@pytest.mark.parametrize("N", [1, 3, 33, 1000, 4097])
def test_ragged_and_all_head_dims(N, d, dtype):
    check((2, 3, N, d), dtype, seed=7 + N + d)


@pytest.mark.parametrize("d", [64, 128])
def test_many_partials_and_tail(d):
    # N spans several per-wave partials plus a ragged tail
    check((1, 2, 3 * 4096 * (2 if d == 128 else 1) + 77, d), "bf16", seed=11)


@pytest.mark.parametrize("d", [64, 128])
def test_bf16_in_fp32_out(d):
    err = check((1, 2, 5000, d), "bf16", seed=12, out_dtype=torch.float32)
    assert err < 1e-3  # no bf16 rounding of the output


def test_fp32_in_bf16_out():
    q, k, v = make_inputs((1, 2, 3000, 64), "fp32", 13)
    o = run_forward(q, k, v, out_dtype=torch.bfloat16)
    assert normwise(as64(o), oracle.forward(q, k, v)) < TOL["bf16"]


def test_spatiotemporal_grid_16384_tokens_full_size():
    # T8 x 32 x 64 = 16384 tokens, B4 H16 d64, bf16, N(0,1) + grid structure
    shape, grid = (4, 16, 16384, 64), (8, 32, 64)
    q, k, v = make_inputs(shape, "bf16", 1001, grid=grid)
    o = run_forward(q, k, v)
    o_ref = oracle.forward(q, k, v)
    err = normwise(as64(o), o_ref)
    print("grid normwise", err, "max rel", max_rel(as64(o), o_ref))
    assert err < TOL["bf16"]


def test_strided_bnhd_matches_contiguous():
    dev = require_gpu()
    B, N, H, d = 2, 1500, 3, 64
    base = [to_device(x, dev) for x in make_inputs((B, N, H, d), "bf16", 14)]
    views = [x.permute(0, 2, 1, 3) for x in base]  # [B, H, N, d] views of BNHD storage
    o_view = la.forward(*views)
    o_cont = la.forward(*(x.contiguous() for x in views))
    torch.cuda.synchronize()
    assert torch.equal(o_view, o_cont)
    out = torch.empty((B, N, H, d), dtype=torch.bfloat16, device=dev).permute(0, 2, 1, 3)
    la.forward(*views, out=out)
    torch.cuda.synchronize()
    assert torch.equal(out, o_cont)


def test_bitwise_deterministic():
    dev = require_gpu()
    xs = [to_device(x, dev) for x in make_inputs((2, 4, 20000, 128), "bf16", 15)]
    a = la.forward(*xs, return_summary=True)
    b = la.forward(*xs, return_summary=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_constant_values_reproduce_the_value():
    dev = require_gpu()
    shape = (1, 2, 9000, 64)
    q, k, _ = make_inputs(shape, "bf16", 16)
    row = inputs.generate(inputs.GenSpec(seed=16, stream=9), (1, 2, 1, 64), "bf16")
    v = np.ascontiguousarray(np.broadcast_to(row, shape))
    o = run_forward(q, k, v, out_dtype=torch.float32)
    ref = np.broadcast_to(inputs.as_float64(row), shape)
    # S = z v^T exactly; hi/lo operands keep num/den = v to about 2^-16
    assert max_rel(as64(o), ref) < 1e-4


def test_constant_keys_give_mean_value():
    shape = (1, 1, 3000, 32)
    q, _, v = make_inputs(shape, "bf16", 17)
    row = inputs.generate(inputs.GenSpec(seed=17, stream=8), (1, 1, 1, 32), "bf16")
    k = np.ascontiguousarray(np.broadcast_to(row, shape))
    o = run_forward(q, k, v, out_dtype=torch.float32)
    mean = inputs.as_float64(v).mean(2, keepdims=True)
    assert np.abs(as64(o) - mean).max() < 1e-4 * np.abs(inputs.as_float64(v)).max()


def test_key_permutation_invariance():
    dev = require_gpu()
    q, k, v = make_inputs((1, 2, 4000, 64), "fp32", 18)
    perm = np.random.default_rng(18).permutation(4000)
    o1 = run_forward(q, k, v)
    o2 = run_forward(q, np.ascontiguousarray(k[:, :, perm]), np.ascontiguousarray(v[:, :, perm]))
    assert normwise(as64(o1), as64(o2)) < 1e-6


def test_token_shards_sum_to_the_whole_summary():
    # one GPU's shard of tokens: per-shard (S, z) add up to the unsharded
    # ones.  Both sides sum the same bf16-rounded phi(k) v^T terms; they
    # differ only in where the FP32 partial sums start and end.  Each run's
    # FP32 rounding is ~ sqrt(m) * 2^-24 of the partials' magnitude
    # (m = accumulations per partial element, one per 32-token step;
    # probabilistic rounding-error analysis, Higham and Mary 2019), so the
    # normwise difference should be about sqrt(2) * sqrt(m) * 2^-24 *
    # sqrt(sum_p ||S_p||^2) / ||S|| -- computed below from the data (S_p:
    # sums over the whole run's partials); the bound allows 4x that.
    q, k, v = make_inputs((1, 2, 30000, 64), "bf16", 19)
    _, S, z = run_forward(q, k, v, summary=True)
    Ss = np.zeros(S.shape)
    zs = np.zeros(z.shape)
    for a, b in ((0, 11111), (11111, 20000), (20000, 30000)):
        sl = lambda x: np.ascontiguousarray(x[:, :, a:b])
        _, S_i, z_i = run_forward(sl(q), sl(k), sl(v), summary=True)
        Ss += S_i.cpu().numpy()
        zs += z_i.cpu().numpy()
    K, V = inputs.as_float64(k), inputs.as_float64(v)
    ph = np.where(K > 0, K + 1.0, np.exp(np.minimum(K, 0.0))).astype(np.float32)
    ph = inputs.bf16_bits_to_f32(inputs.f32_to_bf16_bits(ph)).astype(np.float64)
    tw, steps = 1024, 1024 // 32  # the 30,000-token run: 30 partials of 1,024 tokens
    est_S = est_z = 0.0
    for h in range(2):
        parts = [ph[0, h, i:i + tw].T @ V[0, h, i:i + tw] for i in range(0, 30000, tw)]
        zparts = [ph[0, h, i:i + tw].sum(0) for i in range(0, 30000, tw)]
        Sh, zh = sum(parts), sum(zparts)
        e = lambda ps, tot: np.sqrt(sum(np.sum(p * p) for p in ps)) / np.linalg.norm(tot)
        est_S = max(est_S, np.sqrt(2 * steps) * 2.0 ** -24 * e(parts, Sh))
        est_z = max(est_z, np.sqrt(2 * steps) * 2.0 ** -24 * e(zparts, zh))
    eS = normwise(Ss, S.cpu().numpy())
    ez = normwise(zs[..., None], z.cpu().numpy()[..., None])
    print("shard sums: S", eS, "estimate", est_S, " z", ez, "estimate", est_z, flush=True)
    assert eS < 4 * est_S and ez < 4 * est_z


def test_generator_matches_host_definition():
    dev = require_gpu()
    cases = [((2, 3, 64, 16), None, 1.0), ((2, 3, 64, 16), (2, 4, 8), 0.7071067811865476),
             ((1, 2, 33, 6), None, 1.0)]  # d % 4 != 0: one pair per Philox call
    for dtype, tdt in (("bf16", torch.bfloat16), ("fp32", torch.float32)):
        for shape, grid, std in cases:
            x = torch.empty(shape, dtype=tdt, device=dev)
            la.gen_fill(x, seed=1234, stream_id=2, std=std, grid=grid)
            torch.cuda.synchronize()
            host = inputs.generate(inputs.GenSpec(seed=1234, stream=2, std=std, grid=grid,
                                                  tensor_id=2), shape, dtype)
            dv, hv = as64(x), inputs.as_float64(host)
            # The generator is built without contraction, so both sides round
            # the same FP32 operations; only the transcendentals of the two
            # math libraries may differ in the last bits (a few ulps of a
            # grid phase of up to ~45 rad, i.e. ~1e-6 absolute in the sine).
            # Allowed: one rounding of the stored type relative to the value,
            # plus that absolute term.
            rel = 2.0 ** -7 if dtype == "bf16" else 2.0 ** -19
            absf = (2.0 ** -18 if grid else 2.0 ** -20)
            lim = rel * np.abs(hv) * 1.01 + absf
            bad = np.abs(dv - hv) > lim
            if bad.any():
                worst = np.argsort(((np.abs(dv - hv) - lim)).ravel())[-5:]
                for w in worst:
                    print("gen mismatch", dtype, grid, np.unravel_index(w, shape),
                          dv.ravel()[w], hv.ravel()[w], flush=True)
            assert not bad.any(), (dtype, grid, int(bad.sum()))
            assert np.mean(dv == hv) > (0.97 if dtype == "bf16" else 0.5)


def test_long_context_2m_tokens_sampled_heads():
    # T256 x 64 x 128 = 2,097,152 tokens, B1 H8 d128, bf16, N(0, var 0.5),
    # in the launch configuration the benchmark times.  The oracle checks
    # two whole heads (all N keys for S, z; sampled queries for O).
    dev = require_gpu()
    B, H, N, d = 1, 8, 2097152, 128
    std = 0.5 ** 0.5
    xs = [torch.empty((B, H, N, d), dtype=torch.bfloat16, device=dev) for _ in range(3)]
    for sid, x in enumerate(xs):
        la.gen_fill(x, seed=1002, stream_id=sid, std=std)
    o, S, z = la.forward(*xs, return_summary=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1002)
    for h in (0, 7):
        kh = to_host(xs[1][:, h:h + 1])
        vh = to_host(xs[2][:, h:h + 1])
        S_ref, z_ref = oracle.summary(kh, vh)
        assert normwise(S[:, h:h + 1].cpu().numpy(), S_ref) < 4e-3
        rows = np.sort(rng.choice(N, 4096, replace=False))
        rows[-1] = N - 1
        qh = to_host(xs[0][:, h:h + 1])[:, :, rows]
        o_ref = oracle.apply(np.ascontiguousarray(qh), S_ref, z_ref)
        err = normwise(as64(o[:, h:h + 1, torch.from_numpy(rows).to(dev)]), o_ref)
        print("long-context head", h, "normwise", err, flush=True)
        assert err < TOL["bf16"]
    # convex hull of V holds at any size: min_j v <= O <= max_j v per feature
    vmin = xs[2].float().amin(dim=2, keepdim=True)
    vmax = xs[2].float().amax(dim=2, keepdim=True)
    of = o.float()
    assert bool(((of >= vmin) & (of <= vmax)).all())


def test_apply_reuses_summary_bitwise_and_for_new_queries():
    # keys/values fixed, queries change (one diffusion step after another)
    dev = require_gpu()
    shape = (2, 3, 7000, 64)
    q, k, v = make_inputs(shape, "bf16", 21)
    (q2,) = make_inputs(shape, "bf16", 22, streams=(0,))
    tq, tk, tv, tq2 = (to_device(x, dev) for x in (q, k, v, q2))
    o, S, z = la.forward(tq, tk, tv, return_summary=True)
    o_again = la.apply(tq, S, z)
    o2 = la.apply(tq2, S, z)
    torch.cuda.synchronize()
    assert torch.equal(o, o_again)
    _, S_ref, z_ref = oracle.forward(q, k, v, want_summary=True)
    assert normwise(as64(o2), oracle.apply(q2, S_ref, z_ref)) < TOL["bf16"]
