"""Noise-gated mixing on the GPU (la_forward_gated, la_apply_gated) against
the oracle's blend of its own attention with the other branch's stored
output: out = g(sigma_b) A + (1 - g(sigma_b)) other, with
g(sigma) = sigma_data / (sigma_data + sigma).  Tolerances as for the plain
forward (normwise per (b, h): 2e-2 where inputs or output are bf16, 1e-5
for fp32 throughout); the gate's
fixed points are checked bitwise against the plain calls.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2604_16590_amd as la
from gpu_util import TOL, as64, make_inputs, max_rel, normwise, require_gpu, to_device

pytestmark = pytest.mark.gpu

SIGMAS = [0.02, 0.5, 7.0]  # one per batch element: mostly spatial, even, mostly temporal


def other_branch(shape, out_dtype, seed):
    """The other branch's stored output (seeded, in the output dtype)."""
    (x,) = make_inputs(shape, out_dtype, seed, streams=(3,))
    return x


def check_forward_gated(shape, dtype, seed, out_dtype=None):
    out_dtype = out_dtype or dtype
    dev = require_gpu()
    q, k, v = make_inputs(shape, dtype, seed)
    other = other_branch(shape, out_dtype, seed)
    sigma = SIGMAS[:shape[0]]
    print("case", shape, dtype, out_dtype, seed, flush=True)
    tq, tk, tv, to = (to_device(x, dev) for x in (q, k, v, other))
    ts = torch.tensor(sigma, dtype=torch.float64, device=dev)
    o = la.forward_gated(tq, tk, tv, to, ts, 0.5)
    torch.cuda.synchronize()
    ref = oracle.gated_mix(oracle.forward(q, k, v), other, sigma, 0.5)
    err = normwise(as64(o), ref)
    # a bf16 output carries its own rounding (about 2^-9 relative)
    tol = TOL["bf16"] if "bf16" in (dtype, out_dtype) else TOL["fp32"]
    assert err < tol, (shape, dtype, out_dtype, err, max_rel(as64(o), ref))
    return err


@pytest.mark.parametrize("d", [16, 32, 64, 128])
@pytest.mark.parametrize("dtype", ["bf16", "fp32"])
@pytest.mark.parametrize("N", [33, 4097])
def test_forward_gated_matches_oracle(N, d, dtype):
    check_forward_gated((3, 2, N, d), dtype, 300 + d + N)


@pytest.mark.parametrize("d", [64, 128])
def test_forward_gated_bf16_in_fp32_out(d):
    check_forward_gated((3, 2, 5000, d), "bf16", 310 + d, out_dtype="fp32")


@pytest.mark.parametrize("d", [32, 128])
def test_forward_gated_fp32_in_bf16_out(d):
    check_forward_gated((2, 2, 3000, d), "fp32", 320 + d, out_dtype="bf16")


@pytest.mark.parametrize("dtype", ["bf16", "fp32"])
def test_gate_fixed_points_are_exact(dtype):
    """sigma = 0 gives the plain forward bitwise; sigma = inf gives `other`."""
    dev = require_gpu()
    shape = (2, 3, 2500, 64)
    q, k, v = make_inputs(shape, dtype, 330)
    other = other_branch(shape, dtype, 331)
    tq, tk, tv, to = (to_device(x, dev) for x in (q, k, v, other))
    plain = la.forward(tq, tk, tv)
    spatial = la.forward_gated(tq, tk, tv, to, 0.0)
    temporal = la.forward_gated(tq, tk, tv, to, math.inf)
    torch.cuda.synchronize()
    assert torch.equal(spatial, plain)
    assert torch.equal(temporal, to)


def test_temporal_then_gated_spatial_in_place():
    """The layer's two branches: temporal cross-attention against a cached
    summary (apply), then spatial self-attention blended into it in place."""
    dev = require_gpu()
    shape = (2, 4, 6000, 64)
    q, k, v = make_inputs(shape, "bf16", 340)
    qt, kt, vt = make_inputs((2, 4, 3000, 64), "bf16", 341)
    (qc,) = make_inputs(shape, "bf16", 342, streams=(0,))  # the current state's cross queries
    tq, tk, tv, tqt, tkt, tvt, tqc = (to_device(x, dev) for x in (q, k, v, qt, kt, vt, qc))
    _, St, zt = la.forward(tqt, tkt, tvt, return_summary=True)  # compressed history, once
    out = la.apply(tqc, St, zt)                                    # temporal branch
    sigma = torch.tensor([0.3, 4.0], dtype=torch.float64, device=dev)
    res = la.forward_gated(tq, tk, tv, out, sigma, 0.5, out=out)  # spatial, blended in place
    torch.cuda.synchronize()
    assert res.data_ptr() == out.data_ptr()
    _, St_ref, zt_ref = oracle.forward(qt, kt, vt, want_summary=True)
    temporal = oracle.apply(qc, St_ref, zt_ref)
    ref = oracle.gated_mix(oracle.forward(q, k, v), temporal, [0.3, 4.0], 0.5)
    assert normwise(as64(out), ref) < TOL["bf16"]


@pytest.mark.parametrize("dtype", ["bf16", "fp32"])
def test_apply_gated_matches_oracle(dtype):
    dev = require_gpu()
    shape = (3, 2, 4100, 128)
    q, k, v = make_inputs(shape, dtype, 350)
    (q2,) = make_inputs(shape, dtype, 351, streams=(0,))
    other = other_branch(shape, dtype, 352)
    tq, tk, tv, tq2, to = (to_device(x, dev) for x in (q, k, v, q2, other))
    _, S, z = la.forward(tq, tk, tv, return_summary=True)
    o = la.apply_gated(tq2, S, z, to, torch.tensor(SIGMAS, dtype=torch.float64, device=dev), 0.5)
    torch.cuda.synchronize()
    _, S_ref, z_ref = oracle.forward(q, k, v, want_summary=True)
    ref = oracle.gated_mix(oracle.apply(q2, S_ref, z_ref), other, SIGMAS, 0.5)
    assert normwise(as64(o), ref) < TOL[dtype]


def test_strided_bnhd_gated_matches_contiguous():
    """q, k, v, other and the output as [B, N, H, d] storage."""
    dev = require_gpu()
    shape = (2, 3, 3000, 128)
    q, k, v = make_inputs(shape, "bf16", 360)
    other = other_branch(shape, "bf16", 361)
    B, H, N, d = shape

    def bnhd(x):
        t = to_device(np.ascontiguousarray(np.swapaxes(x, 1, 2)), dev)  # [B, N, H, d] storage
        return t.transpose(1, 2)

    tq, tk, tv, to = (bnhd(x) for x in (q, k, v, other))
    out = torch.empty((B, N, H, d), dtype=torch.bfloat16, device=dev).transpose(1, 2)
    sig = torch.tensor([0.1, 2.0], dtype=torch.float64, device=dev)
    la.forward_gated(tq, tk, tv, to, sig, 0.5, out=out)
    dense = la.forward_gated(*(to_device(x, dev) for x in (q, k, v, other)), sig, 0.5)
    torch.cuda.synchronize()
    assert torch.equal(out.contiguous(), dense)


def test_long_context_cached_apply_and_gated_in_place_sampled_rows():
    # the bench's summary-reuse and gated shapes: B1 H8, 2,097,152 tokens,
    # d = 128, bf16 N(0, 0.5).  New queries against the forward's kept
    # (S, z), then the gated apply blended in place into the other branch;
    # ~2,000 sampled rows of every head (the last row included) against the
    # oracle's apply of the same (S, z) and its gated mix
    from gpu_util import to_host
    dev = require_gpu()
    B, H, N, d = 1, 8, 2097152, 128
    xs = [torch.empty((B, H, N, d), dtype=torch.bfloat16, device=dev) for _ in range(5)]
    for sid, x in enumerate(xs):  # q, k, v, the step's new queries, the other branch
        la.gen_fill(x, seed=77, stream_id=sid, std=0.5 ** 0.5)
    _, S, z = la.forward(*xs[:3], return_summary=True)
    o2 = la.apply(xs[3], S, z)
    rows = sorted(set(np.random.default_rng(5).integers(0, N, 2048).tolist()) | {0, N - 1})
    idx = torch.tensor(rows, device=dev)
    other0 = to_host(xs[4][:, :, idx])
    sigma = torch.tensor([0.7], dtype=torch.float64, device=dev)
    gated = la.apply_gated(xs[3], S, z, xs[4], sigma, 0.5, out=xs[4])
    torch.cuda.synchronize()
    ref = oracle.apply(to_host(xs[3][:, :, idx]), S.cpu().numpy(), z.cpu().numpy())
    err = normwise(as64(o2[:, :, idx]), ref)
    ref_g = oracle.gated_mix(ref, other0, [0.7], 0.5)
    err_g = normwise(as64(gated[:, :, idx]), ref_g)
    print("long context: cached apply %.3g, gated in place %.3g" % (err, err_g), flush=True)
    assert err < TOL["bf16"] and err_g < TOL["bf16"]
    assert gated.data_ptr() == xs[4].data_ptr()
