"""Serving on the GPU: a request computes the same bits alone and in a mix
of concurrent requests (split into different member slices), and matches
the FP64 oracle within the bf16 tolerance."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2604_16590_amd as la
from paper_2604_16590_amd import serve
from gpu_util import TOL, as64, normwise, require_gpu, to_host

pytestmark = pytest.mark.gpu


def fetch(res, Bm, H, N, d):
    """Copy a generated request's O, S, z out of server memory."""
    o = torch.empty((Bm, H, N, d), dtype=torch.bfloat16, device="cuda:0")
    S = torch.empty((Bm, H, d, d), dtype=torch.float64, device="cuda:0")
    z = torch.empty((Bm, H, d), dtype=torch.float64, device="cuda:0")
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    for dst, src in ((o, res.o), (S, res.s), (z, res.z)):
        assert hip.hipMemcpy(dst.data_ptr(), src, dst.numel() * dst.element_size(), 3) == 0
    return o, S, z


@pytest.mark.parametrize("cap", [0, 1])
def test_alone_equals_mix_and_matches_oracle(cap):
    # cap: slots one request may hold in the mix (0: strict FIFO; 1: the
    # requests behind the target run beside it)
    require_gpu()
    H, d = 4, 64
    target = (6, 20000)  # members, tokens
    with serve.Server(4 << 30, max_slots=4, n_streams=4) as srv:
        rid = srv.submit(serve.desc_for(target[0], H, target[1], d), gen_seed=99)
        r = srv.wait(rid)
        assert r.state == serve.DONE and r.slices == 1
        alone = fetch(r, target[0], H, target[1], d)
        srv.release(rid)
    # in a mix, with a budget and slice cap that split the target differently
    with serve.Server(2 << 30, max_slots=3, n_streams=3, max_members_per_slice=2,
                      max_slices_per_request=cap) as srv:
        others = [srv.submit(serve.desc_for(3, H, n, d), gen_seed=s)
                  for s, n in ((1, 50000), (2, 7777))]
        rid = srv.submit(serve.desc_for(target[0], H, target[1], d), gen_seed=99)
        more = [srv.submit(serve.desc_for(2, H, 30001, d), gen_seed=3)]
        r = srv.wait(rid)
        assert r.state == serve.DONE and r.slices == 3
        mixed = fetch(r, target[0], H, target[1], d)
        for x in others + more:
            assert srv.wait(x).state == serve.DONE
        c = srv.stats()
        assert c.peak_bytes_in_use <= c.budget_bytes
    for a, b in zip(alone, mixed):
        assert torch.equal(a, b)
    # parity of the served result: regenerate the inputs with the generator
    xs = [torch.empty((target[0], H, target[1], d), dtype=torch.bfloat16, device="cuda:0")
          for _ in range(3)]
    for t, x in enumerate(xs):
        la.gen_fill(x, seed=99, stream_id=t)
    torch.cuda.synchronize()
    host = [to_host(x[:2]) for x in xs]
    o_ref = oracle.forward(*host)
    assert normwise(as64(alone[0][:2]), o_ref) < TOL["bf16"]


def test_caller_owned_buffers_and_failure_isolation():
    require_gpu()
    H, N, d = 2, 9000, 128
    xs = [torch.empty((4, H, N, d), dtype=torch.bfloat16, device="cuda:0") for _ in range(3)]
    for t, x in enumerate(xs):
        la.gen_fill(x, seed=7, stream_id=t)
    ref = la.forward(*xs)
    out_a = torch.empty_like(xs[0])
    out_b = torch.empty_like(xs[0])
    with serve.Server(1 << 30, max_slots=2, n_streams=2, max_members_per_slice=1) as srv:
        desc = serve.desc_for(4, H, N, d)
        srv.pause()
        a = srv.submit(desc, *xs, out_a)
        b = srv.submit(desc, *xs, out_b)
        srv.fail_slice(b, 2)
        srv.pause(False)
        ra, rb = srv.wait(a), srv.wait(b)
    torch.cuda.synchronize()
    assert ra.state == serve.DONE
    assert rb.state == serve.FAILED
    assert torch.equal(out_a, ref)
