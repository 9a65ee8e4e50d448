"""la_forward_noalloc, the forward entry point that allocates nothing,
against la_forward: the same kernels and tiling on the library's fixed
device scratch instead of a caller workspace, so the same bits.  Two calls
in a row, the second on a smaller problem (the scratch keeps what the first
left), in bf16 and fp32; a problem that needs more than the scratch is
refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2604_16590_amd as la
from paper_2604_16590_amd import _binding as B
from gpu_util import TOL, as64, normwise, require_gpu, to_host

pytestmark = pytest.mark.gpu


def noalloc(q, k, v):
    B_, H, N, d = q.shape
    o = torch.full_like(q, float("nan"))
    S = torch.full((B_, H, d, d), float("nan"), dtype=torch.float64, device=q.device)
    z = torch.full((B_, H, d), float("nan"), dtype=torch.float64, device=q.device)
    la.forward_noalloc(q, k, v, o, S, z)
    return o, S, z


def inputs(shape, dtype, seed):
    dev = require_gpu()
    xs = [torch.empty(shape, dtype=dtype, device=dev) for _ in range(3)]
    for sid, x in enumerate(xs):
        la.gen_fill(x, seed=seed, stream_id=sid, std=0.5 ** 0.5)
    return xs


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32])
def test_noalloc_forward_equals_la_forward_twice_then_smaller(dtype):
    # the long-context shape's heads at 300,007 tokens, then a smaller,
    # ragged problem at another head dim
    for shape, seed in (((1, 8, 300007, 128), 71), ((2, 3, 5003, 64), 72)):
        print("noalloc case", shape, dtype, flush=True)
        xs = inputs(shape, dtype, seed)
        o_ref, S_ref, z_ref = la.forward(*xs, return_summary=True)
        o, S, z = noalloc(*xs)
        torch.cuda.synchronize()
        assert torch.equal(o, o_ref) and torch.equal(S, S_ref) and torch.equal(z, z_ref)
        # and the oracle on one head (bf16 2e-2, fp32 1e-5 normwise)
        h = shape[1] - 1
        hq, hk, hv = (to_host(x[:1, h:h + 1]) for x in xs)
        tol = TOL["bf16" if dtype == torch.bfloat16 else "fp32"]
        assert normwise(as64(o[:1, h:h + 1]), oracle.forward(hq, hk, hv)) < tol


def test_noalloc_refuses_problems_beyond_its_scratch():
    dev = require_gpu()
    q = torch.zeros((1, 1, 16, 128), dtype=torch.bfloat16, device=dev)
    # 64 heads x 4M tokens at d = 64 need ~280 MB of partial sums: refused
    # from the descriptor alone (the pointers are never read)
    N, H = 4 << 20, 64
    desc = B.AttnDesc(1, H, N, 64, 0, 0, H * N * 64, N * 64, 64, H * N * 64, N * 64, 64, 0, 0)
    need = ctypes.c_size_t(0)
    assert B.lib().la_workspace_size(ctypes.byref(desc), 0, ctypes.byref(need)) == 0
    assert need.value > (128 << 20)
    L = B.lib()
    L.la_forward_noalloc.argtypes = [ctypes.POINTER(B.AttnDesc)] + [ctypes.c_void_p] * 7
    L.la_forward_noalloc.restype = ctypes.c_int
    p = q.data_ptr()
    assert L.la_forward_noalloc(ctypes.byref(desc), p, p, p, p, None, None, None) == 3
    # and a problem that fits still runs right after
    xs = inputs((1, 2, 1000, 32), torch.bfloat16, 73)
    o_ref = la.forward(*xs)
    o, _, _ = noalloc(*xs)
    torch.cuda.synchronize()
    assert torch.equal(o, o_ref)
