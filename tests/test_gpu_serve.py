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


def fetch_o(res, Bm, H, N, d, b0=0):
    """Copy members [b0, b0 + Bm) of a generated request's O out of server memory."""
    o = torch.empty((Bm, H, N, d), dtype=torch.bfloat16, device="cuda:0")
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    nbytes = o.numel() * o.element_size()
    assert hip.hipMemcpy(o.data_ptr(), res.o + b0 * (nbytes // Bm), nbytes, 3) == 0
    return o


def test_summary_reuse_equals_la_apply():
    # a member's diffusion steps: one forward, then apply-only requests with
    # new queries (of another token count) against its kept S, z; each equals
    # la_apply bitwise and matches the oracle's apply
    require_gpu()
    Bm, H, N, d = 2, 3, 5000, 64
    xs = [torch.empty((Bm, H, N, d), dtype=torch.bfloat16, device="cuda:0") for _ in range(3)]
    for t, x in enumerate(xs):
        la.gen_fill(x, seed=51, stream_id=t)
    N2 = 3001
    q2 = torch.empty((Bm, H, N2, d), dtype=torch.bfloat16, device="cuda:0")
    la.gen_fill(q2, seed=52, stream_id=0)
    o1 = torch.empty_like(xs[0])
    o2 = torch.empty_like(q2)
    with serve.Server(1 << 30, max_slots=2, n_streams=2, max_members_per_slice=1) as srv:
        owner = srv.submit(serve.desc_for(Bm, H, N, d), *xs, o1)
        step = srv.submit(serve.desc_for(Bm, H, N2, d), q=q2, o=o2, reuse_summary_of=owner)
        # generated queries: stream 0 of the step's seed
        gstep = srv.submit(serve.desc_for(Bm, H, 777, d), gen_seed=53, reuse_summary_of=owner)
        ro = srv.wait(owner)
        rs, rg = srv.wait(step), srv.wait(gstep)
        assert ro.state == rs.state == rg.state == serve.DONE
        assert not rs.s and not rg.s and rg.o
        S, z = (torch.empty((Bm, H, d, d), dtype=torch.float64, device="cuda:0"),
                torch.empty((Bm, H, d), dtype=torch.float64, device="cuda:0"))
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        for dst, src in ((S, ro.s), (z, ro.z)):
            assert hip.hipMemcpy(dst.data_ptr(), src, dst.numel() * 8, 3) == 0
        og = fetch_o(rg, Bm, H, 777, d)
        for x in (gstep, step):
            srv.release(x)
        srv.release(owner)
    torch.cuda.synchronize()
    assert torch.equal(o2, la.apply(q2, S, z))
    qg = torch.empty((Bm, H, 777, d), dtype=torch.bfloat16, device="cuda:0")
    la.gen_fill(qg, seed=53, stream_id=0)
    assert torch.equal(og, la.apply(qg, S, z))
    _, S_ref, z_ref = oracle.forward(*(to_host(x) for x in xs), want_summary=True)
    assert normwise(as64(o2), oracle.apply(to_host(q2), S_ref, z_ref)) < TOL["bf16"]


def test_late_failure_drains_before_memory_is_reused():
    # slice 1 of the victim fails after its inputs were generated on its
    # stream; the other requests, admitted into memory freed around it,
    # still compute their exact results
    require_gpu()
    H, N, d = 2, 40000, 64
    with serve.Server(3 << 30, max_slots=2, n_streams=2, max_members_per_slice=1) as srv:
        srv.pause()
        victim = srv.submit(serve.desc_for(3, H, N, d), gen_seed=61)
        srv.fail_slice(victim, 1, late=True)
        others = [srv.submit(serve.desc_for(2, H, N, d), gen_seed=62 + i) for i in range(3)]
        srv.pause(False)
        rv = srv.wait(victim)
        assert rv.state == serve.FAILED and rv.error == 4
        outs = []
        for i, x in enumerate(others):
            r = srv.wait(x)
            assert r.state == serve.DONE
            outs.append(fetch_o(r, 2, H, N, d))
            srv.release(x)
        srv.release(victim)
        assert srv.stats().bytes_in_use == 0
    for i, o in enumerate(outs):
        xs = [torch.empty((2, H, N, d), dtype=torch.bfloat16, device="cuda:0") for _ in range(3)]
        for t, x in enumerate(xs):
            la.gen_fill(x, seed=62 + i, stream_id=t)
        assert torch.equal(o, la.forward(*xs))


def test_full_size_ensemble_request_sampled_members():
    # one request of the serving workload's shape: 64 members, H16 d64 bf16,
    # 262,144 tokens, server-generated N(0,1) inputs, budget small enough to
    # split it into member slices; members 0 and 63 (two heads each) against
    # the oracle, their inputs regenerated from the request's seed
    require_gpu()
    Bm, H, N, d = 64, 16, 262144, 64
    member = H * N * d * 2
    # the kept output (64 members) plus room for about a sixth of the
    # members' generated inputs at a time
    with serve.Server(80 * member + (1 << 30), max_slots=4, n_streams=4,
                      max_slices_per_request=4) as srv:
        rid = srv.submit(serve.desc_for(Bm, H, N, d), gen_seed=4242)
        r = srv.wait(rid, timeout_s=300)
        assert r.state == serve.DONE and r.slices > 1
        print("full-size request: slices", r.slices, "attention ms", r.attn_ms, flush=True)
        got = {b: fetch_o(r, 1, H, N, d, b0=b) for b in (0, 63)}
        srv.release(rid)
    for b, o in got.items():
        xs = [torch.empty((1, H, N, d), dtype=torch.bfloat16, device="cuda:0") for _ in range(3)]
        for t, x in enumerate(xs):
            la.gen_fill(x, seed=4242, stream_id=t, b_offset=b)
        for h in (0, H - 1):
            host = [to_host(x[:, h:h + 1]) for x in xs]
            err = normwise(as64(o[:, h:h + 1]), oracle.forward(*host))
            print("member", b, "head", h, "normwise", err, flush=True)
            assert err < TOL["bf16"]
