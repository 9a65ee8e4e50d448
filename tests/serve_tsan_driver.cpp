// Scheduler stress driver for the thread-sanitizer run of the serving loop
// (tests/test_serve_tsan.py builds this with la_serve.cpp under
// -fsanitize=thread).  Everything runs on the server's fake executor: no
// device work, so every interleaving of the scheduler thread with client
// threads (submit, poll, release, pause, failure hooks, summary reuse,
// shutdown) is exercised on the host.  Exits non-zero on a broken
// invariant; the sanitizer reports races on its own.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "../include/la.h"

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(2);                                                     \
    }                                                                   \
  } while (0)

static la_request gen_request(int64_t B, int64_t H, int64_t N, int64_t d, uint64_t seed,
                              uint64_t reuse = 0) {
  la_request r{};
  r.desc.B = B; r.desc.H = H; r.desc.N = N; r.desc.d = d;
  r.desc.in_dtype = LA_BF16; r.desc.out_dtype = LA_BF16;
  r.desc.in_sn = d; r.desc.in_sh = N * d; r.desc.in_sb = H * N * d;
  r.desc.out_sn = d; r.desc.out_sh = N * d; r.desc.out_sb = H * N * d;
  r.generate = 1;
  r.gen_seed = seed;
  r.gen_std = 1.0;
  r.reuse_summary_of = reuse;
  return r;
}

static la_server* make_server(uint64_t budget, int slots, int cap, int64_t slice_ns) {
  la_server_config c{};
  c.hbm_budget_bytes = budget;
  c.max_slots = slots;
  c.n_streams = 3;
  c.max_members_per_slice = 2;
  c.fake_executor = 1;
  c.fake_slice_ns = slice_ns;
  c.max_slices_per_request = cap;
  la_server* s = nullptr;
  CHECK(la_serve_create(&c, &s) == LA_OK);
  return s;
}

static int32_t wait_done(la_server* s, uint64_t id) {
  for (;;) {
    la_result r{};
    CHECK(la_serve_poll(s, id, &r) == LA_OK);
    if (r.state == LA_REQ_DONE || r.state == LA_REQ_FAILED) return r.state;
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
}

int main() {
  for (int cap : {0, 2}) {
    la_server* s = make_server(64u << 20, 4, cap, 300000);
    std::atomic<int> done_ok{0}, done_failed{0};
    std::atomic<bool> stop{false};
    // a thread that keeps toggling admission and reading the counters
    std::thread pauser([&] {
      int k = 0;
      while (!stop.load()) {
        CHECK(la_serve_debug_pause(s, (k++ & 1)) == LA_OK);
        la_serve_counters c{};
        CHECK(la_serve_stats(s, &c) == LA_OK);
        CHECK(c.bytes_in_use <= c.budget_bytes);
        std::this_thread::sleep_for(std::chrono::microseconds(300));
      }
      CHECK(la_serve_debug_pause(s, 0) == LA_OK);
    });
    std::vector<std::thread> clients;
    for (int t = 0; t < 4; ++t) {
      clients.emplace_back([&, t] {
        for (int j = 0; j < 60; ++j) {
          uint64_t owner = 0;
          la_request r = gen_request(3, 2, 1024 + 64 * j, 32, 1000 * t + j);
          CHECK(la_serve_submit(s, &r, &owner) == LA_OK);
          if (j % 5 == 1) (void)la_serve_debug_fail_slice(s, owner, 1);
          if (j % 5 == 2) (void)la_serve_debug_fail_slice_late(s, owner, 0);
          // two diffusion steps against the owner's summary
          uint64_t steps[2];
          for (int k = 0; k < 2; ++k) {
            la_request q = gen_request(3, 2, 512 + 32 * k, 32, 50000 + 100 * t + j, owner);
            const la_status st = la_serve_submit(s, &q, &steps[k]);
            CHECK(st == LA_OK || st == LA_ERR_INVALID_ARG);  // the owner may have failed already
            if (st != LA_OK) steps[k] = 0;
          }
          const la_status rel = la_serve_release(s, owner);
          CHECK(rel == LA_ERR_BUSY || rel == LA_OK);
          const bool released = rel == LA_OK;
          for (uint64_t id : steps) {
            if (!id) continue;
            const int32_t st = wait_done(s, id);
            (st == LA_REQ_DONE ? done_ok : done_failed).fetch_add(1);
            CHECK(la_serve_release(s, id) == LA_OK);
          }
          if (!released) {
            const int32_t st = wait_done(s, owner);
            (st == LA_REQ_DONE ? done_ok : done_failed).fetch_add(1);
            CHECK(la_serve_release(s, owner) == LA_OK);
          }
        }
      });
    }
    for (auto& c : clients) c.join();
    stop.store(true);
    pauser.join();
    la_serve_counters c{};
    CHECK(la_serve_stats(s, &c) == LA_OK);
    CHECK(c.bytes_in_use == 0 && c.in_flight_slices == 0 && c.queued == 0);
    CHECK(done_failed.load() > 0 && done_ok.load() > 0);
    // shutdown with work queued and in flight, while a client still polls
    std::vector<uint64_t> ids;
    for (int j = 0; j < 12; ++j) {
      uint64_t id = 0;
      la_request r = gen_request(4, 2, 2048, 64, 777 + j);
      CHECK(la_serve_submit(s, &r, &id) == LA_OK);
      ids.push_back(id);
    }
    std::thread poller([&] {
      la_result r{};
      for (int k = 0; k < 50; ++k) {
        (void)la_serve_poll(s, ids[k % ids.size()], &r);
        std::this_thread::sleep_for(std::chrono::microseconds(100));
      }
    });
    poller.join();
    CHECK(la_serve_destroy(s) == LA_OK);
  }
  std::printf("serve tsan driver: ok\n");
  return 0;
}
