"""Backward parity: la_backward and the autograd.Function against the FP64
oracle's gradients (which are themselves pinned to finite differences and
to autograd of the quadratic form).  Tolerances, normwise per (b, h):
bf16 2e-2, fp32 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_16590_amd as la
from gpu_util import TOL, as64, make_inputs, max_rel, normwise, require_gpu, to_device, to_host

pytestmark = pytest.mark.gpu


def gpu_grads(q, k, v, g, grad_dtype=None):
    dev = require_gpu()
    tq, tk, tv, tg = (to_device(x, dev) for x in (q, k, v, g))
    _, S, z = la.forward(tq, tk, tv, return_summary=True)
    res = la.backward(tq, tk, tv, S, z, tg, grad_dtype=grad_dtype)
    torch.cuda.synchronize()
    return res


def check(shape, dtype, seed, grad_dtype=None, tol=None):
    q, k, v, g = make_inputs(shape, dtype, seed, streams=(0, 1, 2, 3))
    print("case", shape, dtype, seed, grad_dtype, flush=True)
    dq, dk, dv = gpu_grads(q, k, v, g, grad_dtype)
    rq, rk, rv = oracle.backward(q, k, v, g)
    tol = tol or TOL[dtype]
    if shape[2] == 1:
        # one token: O = v_1 whatever q and k are, so dQ = dK = 0 exactly;
        # the computed values are differences of terms of size |G||v|
        scale = np.abs(g.astype(np.float64) if g.dtype != np.uint16 else as64(g)).max() * \
            np.abs(v.astype(np.float64) if v.dtype != np.uint16 else as64(v)).max()
        assert np.abs(as64(dq)).max() < tol * scale and np.abs(as64(dk)).max() < tol * scale
        err = normwise(as64(dv), rv)
        assert err < tol, ("dv", err)
        return {"dv": err}
    errs = {name: normwise(as64(x), r) for name, x, r in (("dq", dq, rq), ("dk", dk, rk), ("dv", dv, rv))}
    print("  normwise", errs, flush=True)
    for name, e in errs.items():
        assert e < tol, (name, e)
    return errs


@pytest.mark.parametrize("d", [16, 32, 64, 128])
@pytest.mark.parametrize("dtype", ["bf16", "fp32"])
@pytest.mark.parametrize("N", [1, 5, 33, 1000, 4097])
def test_ragged_and_all_head_dims(N, d, dtype):
    check((2, 2, N, d), dtype, seed=31 + N + d)


@pytest.mark.parametrize("d", [64, 128])
def test_many_partials_and_tail(d):
    check((1, 2, 2 * 8192 * (2 if d == 128 else 1) + 45, d), "bf16", seed=32)


def test_bf16_inputs_fp32_gradients():
    errs = check((1, 2, 3000, 64), "bf16", seed=33, grad_dtype=torch.float32)
    assert max(errs.values()) < 5e-3


def test_autograd_function_matches_oracle():
    dev = require_gpu()
    q, k, v, g = make_inputs((2, 3, 2500, 64), "bf16", 34, streams=(0, 1, 2, 3))
    tq, tk, tv = (to_device(x, dev).requires_grad_(True) for x in (q, k, v))
    o = la.linear_attention(tq, tk, tv)
    (o.float() * to_device(g, dev).float()).sum().backward()
    torch.cuda.synchronize()
    rq, rk, rv = oracle.backward(q, k, v, g)
    assert normwise(as64(o), oracle.forward(q, k, v)) < TOL["bf16"]
    for x, r in ((tq.grad, rq), (tk.grad, rk), (tv.grad, rv)):
        assert normwise(as64(x), r) < TOL["bf16"]


def test_autograd_with_strided_inputs_and_fp32():
    dev = require_gpu()
    B, N, H, d = 1, 700, 2, 32
    q, k, v, g = make_inputs((B, N, H, d), "fp32", 35, streams=(0, 1, 2, 3))
    tq, tk, tv = (to_device(x, dev).permute(0, 2, 1, 3).detach().requires_grad_(True)
                  for x in (q, k, v))
    tg = to_device(g, dev).permute(0, 2, 1, 3)
    o = la.linear_attention(tq, tk, tv)
    o.backward(tg)
    torch.cuda.synchronize()
    perm = lambda a: np.ascontiguousarray(a.transpose(0, 2, 1, 3))
    rq, rk, rv = oracle.backward(perm(q), perm(k), perm(v), perm(g))
    for x, r in ((tq.grad, rq), (tk.grad, rk), (tv.grad, rv)):
        assert normwise(as64(x.contiguous()), r) < TOL["fp32"]


@pytest.mark.parametrize("d", [32, 64, 128])
def test_strided_bnhd_bf16_backward(d):
    # bf16 takes the fused query pass at these head dims; inputs are views
    # of [B, N, H, d] buffers (token stride H*d), gradients contiguous
    dev = require_gpu()
    B, N, H = 2, 1300, 3
    q, k, v, g = make_inputs((B, N, H, d), "bf16", 40 + d, streams=(0, 1, 2, 3))
    tq, tk, tv, tg = (to_device(x, dev).permute(0, 2, 1, 3) for x in (q, k, v, g))
    print("case strided bnhd bf16", B, N, H, d, flush=True)
    _, S, z = la.forward(tq, tk, tv, return_summary=True)
    dq, dk, dv = la.backward(tq, tk, tv, S, z, tg)
    torch.cuda.synchronize()
    perm = lambda a: np.ascontiguousarray(a.transpose(0, 2, 1, 3))
    rq, rk, rv = oracle.backward(perm(q), perm(k), perm(v), perm(g))
    for name, x, r in (("dq", dq, rq), ("dk", dk, rk), ("dv", dv, rv)):
        err = normwise(as64(x), r)
        assert err < TOL["bf16"], (name, err)


def test_constant_values_bf16_fused_pass():
    # constant V: dQ and dK vanish exactly; the fused pass's dS and dz
    # must cancel in dK = (dS v + dz) phi'(k) just as the two-pass ones do
    from paper_2604_16590_amd import inputs
    dev = require_gpu()
    for d in (64, 128):
        shape = (1, 2, 3000, d)
        q, k, _, g = make_inputs(shape, "bf16", 41, streams=(0, 1, 2, 3))
        row = inputs.generate(inputs.GenSpec(seed=41, stream=9), (1, 1, 1, d), "bf16")
        v = np.ascontiguousarray(np.broadcast_to(row, shape))
        print("case constant V bf16", shape, flush=True)
        dq, dk, dv = gpu_grads(q, k, v, g)
        rq, rk, rv = oracle.backward(q, k, v, g)
        # relative to the size of the terms that cancel (|dV| |v|)
        scale = np.abs(as64(dv)).max() * np.abs(as64(v)).max()
        assert np.abs(as64(dq)).max() < TOL["bf16"] * scale
        assert np.abs(as64(dk)).max() < TOL["bf16"] * scale
        assert normwise(as64(dv), rv) < TOL["bf16"]


def test_value_gradient_column_sums_equal_upstream_sums():
    q, k, v, g = make_inputs((1, 2, 30000, 64), "fp32", 36, streams=(0, 1, 2, 3))
    dq, dk, dv = gpu_grads(q, k, v, g)
    lhs = as64(dv).sum(2)
    rhs = g.astype(np.float64).sum(2)
    assert normwise(lhs[..., None], rhs[..., None]) < 1e-5


def test_constant_values_give_vanishing_query_and_key_gradients():
    from paper_2604_16590_amd import inputs
    shape = (1, 1, 5000, 64)
    q, k, _, g = make_inputs(shape, "fp32", 37, streams=(0, 1, 2, 3))
    row = inputs.generate(inputs.GenSpec(seed=37, stream=9), (1, 1, 1, 64), "fp32")
    v = np.ascontiguousarray(np.broadcast_to(row, shape))
    dq, dk, dv = gpu_grads(q, k, v, g)
    # exact gradients are 0; compare with the scale of the terms that cancel
    scale_q = np.abs(as64(dv)).max() * np.abs(v).max()
    assert np.abs(as64(dq)).max() < 1e-4 * max(scale_q, 1e-30) * 10
    assert np.abs(as64(dk)).max() < 1e-4 * max(scale_q, 1e-30) * 10


def test_backward_bitwise_deterministic():
    dev = require_gpu()
    xs = [to_device(x, dev) for x in make_inputs((1, 4, 40000, 128), "bf16", 38, streams=(0, 1, 2, 3))]
    _, S, z = la.forward(*xs[:3], return_summary=True)
    a = la.backward(*xs[:3], S, z, xs[3])
    b = la.backward(*xs[:3], S, z, xs[3])
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_fwd_bwd_d64_262144_tokens_sampled_heads():
    # N = 262,144 (T64 x 64 x 64), B2 H16 d64, bf16, upstream gradient N(0,1);
    # the oracle recomputes two whole heads.
    dev = require_gpu()
    B, H, N, d = 2, 16, 262144, 64
    xs = [torch.empty((B, H, N, d), dtype=torch.bfloat16, device=dev) for _ in range(4)]
    for sid, x in enumerate(xs):
        la.gen_fill(x, seed=1003, stream_id=sid)
    q, k, v, g = (x.detach().requires_grad_(i < 3) for i, x in enumerate(xs))
    o = la.linear_attention(q, k, v)
    o.backward(g)
    torch.cuda.synchronize()
    for b, h in ((0, 0), (1, 15)):
        host = [to_host(x[b:b + 1, h:h + 1]) for x in xs]
        rq, rk, rv = oracle.backward(*host)
        for name, x, r in (("dq", q.grad, rq), ("dk", k.grad, rk), ("dv", v.grad, rv)):
            err = normwise(as64(x[b:b + 1, h:h + 1]), r)
            print("B2 H16 N262144 d64 head", (b, h), name, err, flush=True)
            assert err < TOL["bf16"]
    # at any size: sum_j dV_j = sum_i G_i per (b, h, feature)
    lhs = v.grad.double().sum(2)
    rhs = g.double().sum(2)
    rel = ((lhs - rhs).norm(dim=-1) / rhs.norm(dim=-1)).max().item()
    print("B2 H16 N262144 d64 column-sum identity", rel)
    assert rel < TOL["bf16"]


def test_long_context_2m_tokens_fwd_bwd_sampled_rows():
    # 2,097,152 tokens, B1 H8 d128, bf16: one head checked against the
    # oracle (exact S, z, dS, dz over all tokens; dQ/dK/dV on sampled rows).
    dev = require_gpu()
    B, H, N, d = 1, 8, 2097152, 128
    xs = [torch.empty((B, H, N, d), dtype=torch.bfloat16, device=dev) for _ in range(4)]
    for sid, x in enumerate(xs):
        la.gen_fill(x, seed=1002, stream_id=sid, std=(0.5 ** 0.5 if sid < 3 else 1.0))
    _, S, z = la.forward(*xs[:3], return_summary=True)
    dq, dk, dv = la.backward(*xs[:3], S, z, xs[3])
    torch.cuda.synchronize()
    h = 5
    hq, hk, hv, hg = (to_host(x[:, h:h + 1]) for x in xs)
    S_ref, z_ref = oracle.summary(hk, hv)
    _, dS_ref, dz_ref = oracle.backward_query(hq, hg, S_ref, z_ref, want_dq=False)
    rows = np.sort(np.random.default_rng(5).choice(N, 2048, replace=False))
    sel = lambda a: np.ascontiguousarray(a[:, :, rows])
    rdq, _, _ = oracle.backward_query(sel(hq), sel(hg), S_ref, z_ref)
    rdk, rdv = oracle.backward_key(sel(hk), sel(hv), dS_ref, dz_ref)
    idx = torch.from_numpy(rows).to(dev)
    for name, x, r in (("dq", dq, rdq), ("dk", dk, rdk), ("dv", dv, rdv)):
        err = normwise(as64(x[:, h:h + 1, idx]), r)
        print("long-context bwd", name, err, max_rel(as64(x[:, h:h + 1, idx]), r), flush=True)
        assert err < TOL["bf16"]
    lhs = dv.double().sum(2)
    rhs = xs[3].double().sum(2)
    assert ((lhs - rhs).norm(dim=-1) / rhs.norm(dim=-1)).max().item() < TOL["bf16"]


@pytest.mark.parametrize("d", [64, 128])
def test_beyond_2m_tokens_partial_count_grows(d):
    # N = 4,194,381 (4 Mi + 77) tokens in one (b, h): past the point where
    # 128 (d = 128) or 64 (d = 64) partials would each sum more than 16,384
    # tokens in FP32, so the partial count grows instead (257 partials of
    # 16,384 tokens, the last one 77 tokens long).  Exact S, z, dS, dz from
    # the oracle over all tokens; O, dQ, dK, dV on sampled rows.
    dev = require_gpu()
    B, H, N = 1, 1, 4 * 1048576 + 77
    print("B1 H1 N%d d%d fwd+bwd" % (N, d), flush=True)
    xs = [torch.empty((B, H, N, d), dtype=torch.bfloat16, device=dev) for _ in range(4)]
    for sid, x in enumerate(xs):
        la.gen_fill(x, seed=1010 + d, stream_id=sid, std=(0.5 ** 0.5 if sid < 3 else 1.0))
    o, S, z = la.forward(*xs[:3], return_summary=True)
    dq, dk, dv = la.backward(*xs[:3], S, z, xs[3])
    torch.cuda.synchronize()
    hq, hk, hv, hg = (to_host(x) for x in xs)
    S_ref, z_ref = oracle.summary(hk, hv)
    assert normwise(S.cpu().numpy(), S_ref) < 4e-3
    assert normwise(z.cpu().numpy()[..., None], z_ref[..., None]) < 4e-3
    _, dS_ref, dz_ref = oracle.backward_query(hq, hg, S_ref, z_ref, want_dq=False)
    rows = np.sort(np.random.default_rng(d).choice(N, 2048, replace=False))
    rows[-1] = N - 1
    sel = lambda a: np.ascontiguousarray(a[:, :, rows])
    o_ref = oracle.apply(sel(hq), S_ref, z_ref)
    rdq, _, _ = oracle.backward_query(sel(hq), sel(hg), S_ref, z_ref)
    rdk, rdv = oracle.backward_key(sel(hk), sel(hv), dS_ref, dz_ref)
    idx = torch.from_numpy(rows).to(dev)
    for name, x, r in (("o", o, o_ref), ("dq", dq, rdq), ("dk", dk, rdk), ("dv", dv, rdv)):
        err = normwise(as64(x[:, :, idx]), r)
        print("N%d d%d" % (N, d), name, err, flush=True)
        assert err < TOL["bf16"]


def test_long_context_2m_tokens_fp32_fwd_bwd():
    # The fp32 half of the 2M-token target: B1 H8 N2,097,152 d128 fp32,
    # inputs N(0, var 0.5), upstream gradient N(0,1), in the launch
    # configuration the benchmark times (512 partials of 4,096 tokens per
    # head).  One head against the oracle at the fp32 tolerance: S and z
    # over all N tokens; O, dQ, dK, dV on 2,048 sampled rows including the
    # first and the last, their references taken from the exact dS and dz
    # over all N tokens (2,048 rows of dV = phi(K) dS and dK = (V dS^T +
    # dz) phi'(K) pin the GPU's dS and dz).
    dev = require_gpu()
    B, H, N, d = 1, 8, 2097152, 128
    print("B1 H8 N2097152 d128 fp32 fwd+bwd", flush=True)
    xs = [torch.empty((B, H, N, d), dtype=torch.float32, device=dev) for _ in range(4)]
    for sid, x in enumerate(xs):
        la.gen_fill(x, seed=1002, stream_id=sid, std=(0.5 ** 0.5 if sid < 3 else 1.0))
    o, S, z = la.forward(*xs[:3], return_summary=True)
    dq, dk, dv = la.backward(*xs[:3], S, z, xs[3])
    torch.cuda.synchronize()
    h = 3
    hq, hk, hv, hg = (to_host(x[:, h:h + 1]) for x in xs)
    S_ref, z_ref = oracle.summary(hk, hv)
    eS = normwise(S[:, h:h + 1].cpu().numpy(), S_ref)
    ez = normwise(z[:, h:h + 1].cpu().numpy()[..., None], z_ref[..., None])
    print("fp32 2M S", eS, "z", ez, flush=True)
    assert eS < TOL["fp32"] and ez < TOL["fp32"]
    _, dS_ref, dz_ref = oracle.backward_query(hq, hg, S_ref, z_ref, want_dq=False)
    rows = np.sort(np.random.default_rng(3).choice(N, 2048, replace=False))
    rows[0], rows[-1] = 0, N - 1
    sel = lambda a: np.ascontiguousarray(a[:, :, rows])
    o_ref = oracle.apply(sel(hq), S_ref, z_ref)
    rdq, _, _ = oracle.backward_query(sel(hq), sel(hg), S_ref, z_ref)
    rdk, rdv = oracle.backward_key(sel(hk), sel(hv), dS_ref, dz_ref)
    idx = torch.from_numpy(rows).to(dev)
    for name, x, r in (("o", o, o_ref), ("dq", dq, rdq), ("dk", dk, rdk), ("dv", dv, rdv)):
        err = normwise(as64(x[:, h:h + 1, idx]), r)
        print("fp32 2M", name, err, max_rel(as64(x[:, h:h + 1, idx]), r), flush=True)
        assert err < TOL["fp32"]
    # column sums of dV equal those of G at any size, every head
    lhs = dv.double().sum(2)
    rhs = xs[3].double().sum(2)
    assert ((lhs - rhs).norm(dim=-1) / rhs.norm(dim=-1)).max().item() < TOL["fp32"]


def test_autograd_sum_loss_and_transposed_upstream_gradient():
    # loss = O.sum() hands the backward an expanded gradient of ones (all
    # strides 0); a gradient held as [B, N, H, d] storage arrives as a
    # permuted view.  Both reach the kernels in q's layout.
    dev = require_gpu()
    shape = (2, 3, 1500, 64)
    q, k, v = make_inputs(shape, "bf16", 42)
    tq, tk, tv = (to_device(x, dev).requires_grad_(True) for x in (q, k, v))
    la.linear_attention(tq, tk, tv).sum().backward()
    torch.cuda.synchronize()
    ones = np.full(shape, 0x3F80, np.uint16)  # bf16 1.0
    refs = oracle.backward(q, k, v, ones)
    for name, x, r in zip(("dq", "dk", "dv"), (tq.grad, tk.grad, tv.grad), refs):
        err = normwise(as64(x), r)
        print("sum loss", name, err, flush=True)
        assert err < TOL["bf16"], (name, err)
    (g,) = make_inputs((2, 1500, 3, 64), "bf16", 43, streams=(3,))
    tg = to_device(g, dev).permute(0, 2, 1, 3)
    for t in (tq, tk, tv):
        t.grad = None
    la.linear_attention(tq, tk, tv).backward(tg)
    torch.cuda.synchronize()
    refs = oracle.backward(q, k, v, np.ascontiguousarray(g.transpose(0, 2, 1, 3)))
    for name, x, r in zip(("dq", "dk", "dv"), (tq.grad, tk.grad, tv.grad), refs):
        err = normwise(as64(x), r)
        print("transposed gradient", name, err, flush=True)
        assert err < TOL["bf16"], (name, err)
