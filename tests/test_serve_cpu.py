"""Scheduler logic of the serving loop, on the CPU.

The server runs with its fake executor: no GPU work, each admitted slice
finishes a fixed time after launch.  Admission, slicing, the HBM budget,
FIFO order, failure handling and shutdown are the same code as on the GPU.
"""
import threading
import time

import pytest

from paper_2604_16590_amd import serve
from paper_2604_16590_amd import _binding as B

MS = 1_000_000


def member_bytes(H, N, d, es=2):
    return H * N * d * es


def test_single_request_completes_with_ordered_stamps():
    with serve.Server(1 << 30, fake_slice_ns=2 * MS) as srv:
        rid = srv.submit(serve.desc_for(4, 2, 4096, 64), gen_seed=1)
        r = srv.wait(rid)
        assert r.state == serve.DONE and r.error == 0
        assert r.t_arrival_ns <= r.t_admit_ns <= r.t_done_ns
        assert r.t_done_ns - r.t_admit_ns >= 2 * MS
        assert r.slices == 1
        srv.release(rid)
        with pytest.raises(B.LaError):
            srv.poll(rid)


def test_budget_splits_members_and_is_never_exceeded():
    H, N, d = 2, 65536, 64
    per_member = member_bytes(H, N, d)
    # room for the kept output of 8 members plus about 3 members' inputs
    budget = 8 * per_member + 3 * 3 * per_member + (8 << 20)
    with serve.Server(budget, max_slots=4, fake_slice_ns=1 * MS) as srv:
        rid = srv.submit(serve.desc_for(8, H, N, d), gen_seed=2)
        r = srv.wait(rid)
        assert r.state == serve.DONE
        assert r.slices >= 3
        c = srv.stats()
        assert c.peak_bytes_in_use <= c.budget_bytes
        srv.release(rid)
        assert srv.stats().bytes_in_use == 0


def test_max_members_per_slice():
    with serve.Server(1 << 30, max_members_per_slice=3, fake_slice_ns=MS // 2) as srv:
        rid = srv.submit(serve.desc_for(10, 1, 1024, 32), gen_seed=3)
        assert srv.wait(rid).slices == 4


def test_fifo_order_with_one_slot():
    with serve.Server(1 << 30, max_slots=1, fake_slice_ns=3 * MS) as srv:
        ids = [srv.submit(serve.desc_for(1, 1, 1024, 64), gen_seed=i) for i in range(6)]
        res = [srv.wait(i) for i in ids]
        done = [r.t_done_ns for r in res]
        admit = [r.t_admit_ns for r in res]
        assert done == sorted(done) and admit == sorted(admit)
        for a, b in zip(res, res[1:]):
            assert b.t_admit_ns >= a.t_done_ns  # one slot: strictly one after another


def test_slices_overlap_with_several_slots():
    with serve.Server(1 << 30, max_slots=4, n_streams=4, fake_slice_ns=20 * MS) as srv:
        t0 = time.monotonic_ns()
        ids = [srv.submit(serve.desc_for(1, 1, 1024, 64), gen_seed=i) for i in range(4)]
        res = [srv.wait(i) for i in ids]
        wall = max(r.t_done_ns for r in res) - t0
        assert wall < 60 * MS  # four 20 ms slices ran concurrently, not back to back


@pytest.mark.parametrize("cap", [0, 1])
def test_per_request_slot_cap_lets_short_requests_pass(cap):
    # a long request of 8 one-member slices, then a short one: strict FIFO
    # (cap 0) admits the short one only after every slice of the long one;
    # with a cap of one slot per request it runs beside the long one
    with serve.Server(1 << 30, max_slots=2, max_members_per_slice=1, fake_slice_ns=10 * MS,
                      max_slices_per_request=cap) as srv:
        srv.pause()
        long_id = srv.submit(serve.desc_for(8, 1, 1024, 64), gen_seed=1)
        short_id = srv.submit(serve.desc_for(1, 1, 1024, 64), gen_seed=2)
        srv.pause(False)
        rl, rs = srv.wait(long_id), srv.wait(short_id)
        assert rl.state == serve.DONE and rs.state == serve.DONE and rl.slices == 8
        if cap:
            assert rs.t_done_ns < rl.t_done_ns
            assert rs.t_admit_ns - rl.t_admit_ns < 5 * MS  # admitted at once
        else:
            assert rs.t_admit_ns - rl.t_admit_ns >= 25 * MS  # behind three rounds of slices


def test_slot_cap_bounds_a_slice_to_its_budget_share():
    H, N, d = 2, 65536, 64
    per_member = member_bytes(H, N, d)
    budget = 64 * per_member
    with serve.Server(budget, max_slots=4, fake_slice_ns=MS, max_slices_per_request=2) as srv:
        rid = srv.submit(serve.desc_for(16, H, N, d), gen_seed=3)
        r = srv.wait(rid)
        assert r.state == serve.DONE
        # generated Q, K, V of 16 members = 48 member tensors > 64/4 = 16
        assert r.slices >= 3


def test_request_too_large_for_budget_is_rejected():
    with serve.Server(64 << 20, fake_slice_ns=MS) as srv:
        with pytest.raises(B.LaError) as e:
            srv.submit(serve.desc_for(1, 16, 1 << 20, 64), gen_seed=1)
        assert e.value.status == 3  # LA_ERR_OOM
        assert srv.stats().rejected == 1


def test_injected_failure_fails_only_its_request():
    with serve.Server(1 << 30, max_slots=1, max_members_per_slice=1, fake_slice_ns=10 * MS) as srv:
        srv.pause()
        blocker = srv.submit(serve.desc_for(1, 1, 1024, 64), gen_seed=0)
        victim = srv.submit(serve.desc_for(3, 1, 1024, 64), gen_seed=1)
        other = srv.submit(serve.desc_for(2, 1, 1024, 64), gen_seed=2)
        srv.fail_slice(victim, 1)
        srv.pause(False)
        rb, rv, ro = srv.wait(blocker), srv.wait(victim), srv.wait(other)
        assert rb.state == serve.DONE and ro.state == serve.DONE
        assert rv.state == serve.FAILED and rv.error == 4  # LA_ERR_HIP
        c = srv.stats()
        assert c.failed == 1 and c.completed == 2


def test_unknown_ids_and_busy_release():
    with serve.Server(1 << 30, fake_slice_ns=50 * MS) as srv:
        with pytest.raises(B.LaError) as e:
            srv.poll(12345)
        assert e.value.status == 5
        rid = srv.submit(serve.desc_for(1, 1, 1024, 64), gen_seed=1)
        with pytest.raises(B.LaError) as e:
            srv.release(rid)
        assert e.value.status == 7  # LA_ERR_BUSY while running
        srv.wait(rid)
        srv.release(rid)


def test_pause_holds_admission():
    with serve.Server(1 << 30, fake_slice_ns=MS) as srv:
        srv.pause()
        rid = srv.submit(serve.desc_for(1, 1, 1024, 64), gen_seed=1)
        time.sleep(0.02)
        assert srv.poll(rid).state == serve.QUEUED
        srv.pause(False)
        assert srv.wait(rid).state == serve.DONE


def test_destroy_with_work_in_flight_and_queued():
    srv = serve.Server(1 << 30, max_slots=1, fake_slice_ns=30 * MS)
    for i in range(5):
        srv.submit(serve.desc_for(1, 1, 1024, 64), gen_seed=i)
    t0 = time.monotonic()
    srv.close()  # drains the slice in flight, cancels the rest
    assert time.monotonic() - t0 < 1.0


def test_concurrent_submitters():
    with serve.Server(1 << 30, max_slots=8, n_streams=4, fake_slice_ns=MS) as srv:
        ids, lock = [], threading.Lock()

        def client(seed):
            for j in range(20):
                rid = srv.submit(serve.desc_for(2, 1, 2048, 32), gen_seed=seed * 100 + j)
                with lock:
                    ids.append(rid)

        ts = [threading.Thread(target=client, args=(i,)) for i in range(4)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        assert len(set(ids)) == 80
        for rid in ids:
            assert srv.wait(rid).state == serve.DONE
            srv.release(rid)
        c = srv.stats()
        assert c.completed == 80 and c.bytes_in_use == 0 and c.queued == 0


def test_invalid_config_and_request():
    with pytest.raises(B.LaError):
        serve.Server(1 << 30, max_slots=0, fake_slice_ns=MS)
    with pytest.raises(B.LaError):
        serve.Server(1 << 30, max_slices_per_request=-1, fake_slice_ns=MS)
    with serve.Server(1 << 30, fake_slice_ns=MS) as srv:
        bad = serve.desc_for(1, 1, 1024, 48)
        with pytest.raises(B.LaError) as e:
            srv.submit(bad, gen_seed=1)
        assert e.value.status == 2
        with pytest.raises(B.LaError):
            srv.submit(serve.desc_for(1, 1, 1024, 64), gen_seed=1, gen_std=0.0)


def test_poisson_driver_reports_latency_percentiles():
    with serve.Server(8 << 30, max_slots=4, fake_slice_ns=MS) as srv:
        res = serve.run_poisson(srv, 30, 500.0, seed=1, H=2, d=32, members=2,
                                n_min=1024, n_max=8192)
    assert res["completed"] == 30 and res["failed"] == 0
    assert res["p50_ms"] <= res["p99_ms"] <= res["max_ms"]
    assert res["p50_ms"] >= 1.0  # at least the slice time


def test_late_failure_keeps_the_slice_memory_until_its_work_drains():
    # a slice that fails after its inputs were enqueued: the work already on
    # its stream may still write the slice's block, so the block (and the
    # request's FAILED state) wait until that work has drained
    H, N, d = 1, 4096, 64
    with serve.Server(1 << 30, max_slots=2, max_members_per_slice=1, fake_slice_ns=150 * MS) as srv:
        srv.pause()
        rid = srv.submit(serve.desc_for(2, H, N, d), gen_seed=1)
        srv.fail_slice(rid, 0, late=True)
        srv.pause(False)
        time.sleep(0.03)
        c = srv.stats()
        kept = H * N * d * 2 * 2 + 2 * H * d * d * 8  # generated O of 2 members + S
        assert c.in_flight_slices == 2            # the failed slice is still held
        assert c.bytes_in_use > kept + 3 * H * N * d * 2
        assert srv.poll(rid).state == serve.RUNNING
        r = srv.wait(rid)
        assert r.state == serve.FAILED and r.error == 4
        assert r.t_done_ns - r.t_admit_ns >= 150 * MS
        c = srv.stats()
        assert c.in_flight_slices == 0 and c.failed == 1
        srv.release(rid)
        assert srv.stats().bytes_in_use == 0


def test_early_failure_releases_at_once():
    with serve.Server(1 << 30, max_slots=1, fake_slice_ns=200 * MS) as srv:
        srv.pause()
        rid = srv.submit(serve.desc_for(1, 1, 1024, 64), gen_seed=1)
        srv.fail_slice(rid, 0)
        srv.pause(False)
        r = srv.wait(rid, timeout_s=5)
        assert r.state == serve.FAILED and r.t_done_ns - r.t_admit_ns < 150 * MS


def test_summary_reuse_waits_for_its_owner_and_pins_it():
    # one member's diffusion steps: the forward once, then apply-only steps
    # against its summary; the owner cannot be released while steps are
    # pending, and steps start only after the owner is DONE
    with serve.Server(1 << 30, max_slots=4, fake_slice_ns=20 * MS,
                      max_slices_per_request=1) as srv:
        owner = srv.submit(serve.desc_for(2, 2, 4096, 64), gen_seed=10)
        steps = [srv.submit(serve.desc_for(2, 2, 1000 + i, 64), gen_seed=11 + i,
                            reuse_summary_of=owner) for i in range(3)]
        with pytest.raises(B.LaError) as e:
            srv.release(owner)
        assert e.value.status == 7
        ro = srv.wait(owner)
        assert ro.state == serve.DONE                   # (fake executor: no device pointers)
        res = [srv.wait(s) for s in steps]
        for r in res:
            assert r.state == serve.DONE
            assert r.t_admit_ns >= ro.t_done_ns         # after the summary exists
        for s in steps:
            srv.release(s)
        srv.release(owner)                              # now allowed
        assert srv.stats().bytes_in_use == 0


def test_summary_reuse_errors_and_failed_owner():
    with serve.Server(1 << 30, max_slots=1, fake_slice_ns=5 * MS) as srv:
        with pytest.raises(B.LaError) as e:
            srv.submit(serve.desc_for(1, 1, 1024, 64), gen_seed=1, reuse_summary_of=999)
        assert e.value.status == 5                      # unknown owner
        srv.pause()
        owner = srv.submit(serve.desc_for(2, 1, 1024, 64), gen_seed=1)
        for bad in (serve.desc_for(3, 1, 1024, 64), serve.desc_for(2, 2, 1024, 64),
                    serve.desc_for(2, 1, 1024, 32), serve.desc_for(2, 1, 1024, 64, dtype=1)):
            with pytest.raises(B.LaError) as e:
                srv.submit(bad, gen_seed=2, reuse_summary_of=owner)
            assert e.value.status == 1                  # B, H, d, dtype must match
        step = srv.submit(serve.desc_for(2, 1, 5000, 64), gen_seed=2, reuse_summary_of=owner)
        with pytest.raises(B.LaError):                  # no chains of reuse
            srv.submit(serve.desc_for(2, 1, 64, 64), gen_seed=3, reuse_summary_of=step)
        srv.fail_slice(owner, 0)
        srv.pause(False)
        assert srv.wait(owner).state == serve.FAILED
        r = srv.wait(step)
        assert r.state == serve.FAILED and r.error == 4  # the owner's error
        srv.release(step)
        srv.release(owner)
        with pytest.raises(B.LaError):                  # a FAILED owner is refused
            owner2 = srv.submit(serve.desc_for(1, 1, 1024, 64), gen_seed=4)
            srv.fail_slice(owner2, 0)
            srv.wait(owner2)
            srv.submit(serve.desc_for(1, 1, 1024, 64), gen_seed=5, reuse_summary_of=owner2)


def test_destroy_cancels_pending_reusers():
    srv = serve.Server(1 << 30, max_slots=1, fake_slice_ns=30 * MS)
    owner = srv.submit(serve.desc_for(1, 1, 1024, 64), gen_seed=1)
    for i in range(3):
        srv.submit(serve.desc_for(1, 1, 1024, 64), gen_seed=2 + i, reuse_summary_of=owner)
    t0 = time.monotonic()
    srv.close()
    assert time.monotonic() - t0 < 1.0


def test_reuse_loop_driver_reports_step_percentiles():
    with serve.Server(1 << 30, max_slots=2, fake_slice_ns=MS) as srv:
        res = serve.run_reuse_loop(srv, steps=12, members=2, H=2, N=4096, d=32)
        assert res["completed"] == 12 and res["failed"] == 0
        assert MS / 1e6 <= res["step_p50_ms"] <= res["step_p99_ms"] <= res["step_max_ms"]
        assert srv.stats().bytes_in_use == 0


class _Ptr:
    def __init__(self, p):
        self.p = p

    def data_ptr(self):
        return self.p


def fake_pool(H, d, T):
    pool = serve.InputPool.__new__(serve.InputPool)
    pool.H, pool.d, pool.T = H, d, T
    pool.t = {n: _Ptr((i + 1) << 40) for i, n in enumerate(("q", "k", "v", "o"))}
    return pool


@pytest.mark.parametrize("members,N", [(64, 4096), (64, 1000), (64, 262144), (64, 262145),
                                       (64, 1048576), (1, 5000), (3, 16777206)])
def test_input_pool_windows_stay_inside_the_pool(members, N):
    # every member's window [base + b*s, base + b*s + N) lies in the pool;
    # windows are disjoint while members * N fits, and the strides describe
    # an [H, T, d] tensor
    import numpy as np
    H, d, T = 16, 64, 64 * 262144
    pool = fake_pool(H, d, T)
    rng = np.random.default_rng(3)
    for _ in range(50):
        desc, q, k, v, o = pool.request(members, N, rng)
        assert (desc.B, desc.H, desc.N, desc.d) == (members, H, N, d)
        assert desc.in_sh == desc.out_sh == T * d and desc.in_sn == desc.out_sn == d
        assert desc.in_sb == desc.out_sb and desc.in_sb % d == 0
        s = desc.in_sb // d
        base = (q - pool.t["q"].p) // (2 * d)
        assert (q - pool.t["q"].p) % (2 * d) == 0
        for name, p in zip(("k", "v", "o"), (k, v, o)):
            assert p - pool.t[name].p == base * 2 * d
        assert base >= 0 and base + (members - 1) * s + N <= T
        if members * N <= T:
            assert s == N
        else:
            assert 0 < s < N


def test_input_pool_rejects_a_request_larger_than_the_pool():
    import numpy as np
    with pytest.raises(ValueError):
        fake_pool(2, 64, 1000).request(1, 1001, np.random.default_rng(0))


def test_poisson_and_reuse_drivers_with_caller_owned_pool():
    pool = fake_pool(2, 32, 64 * 8192)
    with serve.Server(8 << 30, max_slots=4, fake_slice_ns=MS) as srv:
        res = serve.run_poisson(srv, 20, 500.0, seed=1, H=2, d=32, members=4,
                                n_min=1024, n_max=8192, pool=pool)
        assert res["completed"] == 20 and res["failed"] == 0
        assert res["attention_TB_s"] > 0
        loop = serve.run_reuse_loop(srv, steps=5, members=4, H=2, N=4096, d=32, pool=pool)
        assert loop["completed"] == 5
        assert srv.stats().bytes_in_use == 0
