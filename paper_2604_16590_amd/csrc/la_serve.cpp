// la_serve.cpp -- continuous-batching request loop (include/la.h, la_serve_*).
//
// One scheduler thread per server.  Each tick it retires finished slices,
// then admits slices of the oldest request while a slot is free and the
// slice's device memory fits the free part of the HBM budget (with a
// per-request cap on slots, the next requests in arrival order take the
// slots the oldest one may not).  A slice is a
// contiguous run of the request's members (ensemble members are independent
// problems with the same N, H, d), so the members of a large request can
// run as memory frees up while other requests' slices overlap on the
// device.  The budget is one device allocation carved by a first-fit
// allocator, so admission never calls hipMalloc.
//
// Summary reuse: a request may name an earlier request whose FP64 summary
// S and normaliser z the server still holds; it then runs the apply only
// (la_apply of its own queries against them), the per-step work of the
// paper's temporal cross-attention against a fixed compressed history
// (Sec. III-B) over the diffusion steps of an ensemble member (Sec. V).
// It starts once that request is DONE, and that request cannot be released
// while requests reusing it are pending.
//
// Only the HIP runtime API is used here (no device code), so the file also
// builds as plain host C++ for the thread-sanitizer run of the scheduler.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/la.h"
#include "../../include/la_gen.h"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over [0, size) with coalescing of freed blocks.
class Arena {
 public:
  void init(size_t size) {
    size_ = size;
    free_.clear();
    if (size) free_[0] = size;
    in_use_ = peak_ = 0;
  }
  bool alloc(size_t n, size_t* off) {
    n = align_up(n ? n : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, start = it->first + n;
        free_.erase(it);
        if (rest) free_[start] = rest;
        in_use_ += n;
        peak_ = std::max(peak_, in_use_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align_up(n ? n : 1);
    in_use_ -= n;
    auto it = free_.emplace(off, n).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  size_t size() const { return size_; }
  size_t in_use() const { return in_use_; }
  size_t peak() const { return peak_; }

 private:
  size_t size_ = 0, in_use_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

struct Slice {
  uint64_t req;
  int index;
  int64_t b0, m;       // members [b0, b0 + m)
  size_t off, bytes;   // transient block: generated inputs + workspace
  int stream;
  hipEvent_t start, gen, done;  // timed events: slice start, inputs ready, done
  uint64_t t_fake_done;
  bool fail;           // test hook: fails before anything is enqueued
  bool fail_late;      // test hook: fails after its inputs are enqueued
  bool failed_launch;  // its launch failed after work was enqueued: it is
                       // retired (as failed) only once that work drained
};

struct Request {
  la_request spec;
  int32_t state = LA_REQ_QUEUED;
  la_status error = LA_OK;
  uint64_t t_arrival = 0, t_admit = 0, t_done = 0;
  int64_t next_member = 0;
  int slices_started = 0, slices_done = 0;
  bool failed = false;
  size_t keep_off = 0, keep_bytes = 0;  // S, z (+ O when generated)
  double gen_ms = 0.0, attn_ms = 0.0;    // device time summed over slices
  bool keep_held = false;
  void* o = nullptr;
  double* s = nullptr;  // this request's S, z (the owner's when reusing)
  double* z = nullptr;
  int reusers = 0;      // pending requests that apply this one's S, z
};

bool reuses(const la_request& r) { return r.reuse_summary_of != 0; }

int64_t esize(int32_t dt) { return dt == LA_BF16 ? 2 : 4; }

size_t member_tensor_bytes(const la_attn_desc& d, int32_t dt) {
  return (size_t)(d.H * d.N * d.d * esize(dt));
}

}  // namespace

struct la_server {
  la_server_config cfg{};
  char* base = nullptr;  // device memory of the budget (null with the fake executor)
  Arena arena;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;  // pool
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> fifo;
  std::unordered_map<uint64_t, Request> reqs;
  std::vector<Slice> inflight;
  std::set<std::pair<uint64_t, int>> fail_at, fail_late_at;
  std::thread th;
  bool stopping = false;
  bool paused = false;
  uint64_t next_id = 1;
  uint64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_rejected = 0;
  int next_stream = 0;
};

namespace {

// Transient bytes of a slice of m members: generated inputs (Q, K, V; Q
// only when reusing a summary) plus the workspace of the forward (apply).
// Kept bytes of a request: S, z (not when reusing) and a generated O.
size_t slice_bytes(const la_request& r, int64_t m) {
  la_attn_desc d = r.desc;
  d.B = m;
  if (r.generate) {
    d.in_sh = d.N * d.d; d.in_sb = d.H * d.in_sh; d.in_sn = d.d;
    d.out_sh = d.N * d.d; d.out_sb = d.H * d.out_sh; d.out_sn = d.d;
  }
  size_t ws = 0;
  la_workspace_size(&d, reuses(r) ? 2 : 0, &ws);
  size_t b = align_up(ws);
  const size_t n_gen = reuses(r) ? 1 : 3;
  if (r.generate) b += n_gen * align_up(member_tensor_bytes(d, d.in_dtype) * (size_t)m);
  return b;
}

size_t keep_bytes(const la_request& r) {
  const la_attn_desc& d = r.desc;
  size_t b = 0;
  if (!reuses(r))
    b += align_up((size_t)(d.B * d.H * d.d * d.d) * 8) + align_up((size_t)(d.B * d.H * d.d) * 8);
  if (r.generate) b += align_up(member_tensor_bytes(d, d.out_dtype) * (size_t)d.B);
  return std::max<size_t>(b, 1);
}

// A request reaches DONE or FAILED: stamps, counters, and the owner of a
// reused summary has one pending reuser less.
void complete_request(la_server* s, Request& rq, bool failed, la_status err) {
  rq.t_done = now_ns();
  rq.state = failed ? LA_REQ_FAILED : LA_REQ_DONE;
  if (failed) rq.error = err;
  if (failed) s->n_failed += 1; else s->n_completed += 1;
  if (reuses(rq.spec)) {
    auto ot = s->reqs.find(rq.spec.reuse_summary_of);
    if (ot != s->reqs.end()) ot->second.reusers -= 1;
  }
}

hipEvent_t take_event(la_server* s) {
  if (!s->events.empty()) {
    hipEvent_t e = s->events.back();
    s->events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (s->cfg.fake_executor) return e;
  if (hipEventCreateWithFlags(&e, hipEventDefault) != hipSuccess) return nullptr;
  return e;
}

// Enqueue one slice on its stream (called with the lock held).  On
// failure *enqueued tells whether work was already put on the stream (it
// may still write the slice's memory).
la_status launch_slice(la_server* s, Request& rq, Slice& sl, bool* enqueued) {
  *enqueued = false;
  if (sl.fail) return LA_ERR_HIP;  // injected device failure
  if (s->cfg.fake_executor) {
    sl.t_fake_done = now_ns() + (uint64_t)s->cfg.fake_slice_ns;
    if (sl.fail_late) {  // its (simulated) inputs are on the way
      *enqueued = true;
      return LA_ERR_HIP;
    }
    return LA_OK;
  }
  const la_request& r = rq.spec;
  la_attn_desc d = r.desc;
  d.B = sl.m;
  hipStream_t st = s->streams[sl.stream];
  char* blk = s->base + sl.off;
  const void *q, *k, *v;
  void* o;
  if (hipEventRecord(sl.start, st) != hipSuccess) return LA_ERR_HIP;
  *enqueued = true;
  const int n_gen = reuses(r) ? 1 : 3;
  if (r.generate) {
    d.in_sh = d.N * d.d; d.in_sb = d.H * d.in_sh; d.in_sn = d.d;
    d.out_sh = d.N * d.d; d.out_sb = d.H * d.out_sh; d.out_sn = d.d;
    const size_t tb = align_up(member_tensor_bytes(d, d.in_dtype) * (size_t)sl.m);
    char* gq = blk;
    char* gk = blk + tb;
    char* gv = blk + 2 * tb;
    char* bufs[3] = {gq, gk, gv};
    for (int t = 0; t < n_gen; ++t) {
      la_gen_spec g{};
      g.seed = r.gen_seed;
      g.stream = (uint32_t)t;
      g.tensor_id = t;
      g.mean = 0.0;
      g.std = r.gen_std;
      g.amplitude = 0.0;
      g.b_offset = sl.b0;
      if (la_gen_fill(bufs[t], d.in_dtype, d.B, d.H, d.N, d.d, d.in_sb, d.in_sh, d.in_sn, &g, st) != 0)
        return LA_ERR_HIP;
    }
    q = gq; k = gk; v = gv;
    o = (char*)rq.o + (size_t)sl.b0 * member_tensor_bytes(d, d.out_dtype);
    blk += n_gen * tb;
  } else {
    const int64_t ie = esize(d.in_dtype), oe = esize(d.out_dtype);
    q = (const char*)r.q + sl.b0 * d.in_sb * ie;
    k = (const char*)r.k + sl.b0 * d.in_sb * ie;
    v = (const char*)r.v + sl.b0 * d.in_sb * ie;
    o = (char*)r.o + sl.b0 * d.out_sb * oe;
  }
  if (sl.fail_late) return LA_ERR_HIP;  // injected failure after the inputs
  if (hipEventRecord(sl.gen, st) != hipSuccess) return LA_ERR_HIP;
  size_t ws = 0;
  la_workspace_size(&d, reuses(r) ? 2 : 0, &ws);
  double* S = rq.s + (size_t)sl.b0 * d.H * d.d * d.d;
  double* z = rq.z + (size_t)sl.b0 * d.H * d.d;
  const la_status st2 = reuses(r) ? la_apply(&d, q, S, z, o, blk, ws, st)
                                  : la_forward(&d, q, k, v, o, S, z, blk, ws, st);
  if (st2 != LA_OK) return st2;
  if (hipEventRecord(sl.done, st) != hipSuccess) return LA_ERR_HIP;
  return LA_OK;
}

void finish_slice(la_server* s, Slice& sl, bool ok) {
  s->arena.release(sl.off, sl.bytes);
  auto it = s->reqs.find(sl.req);
  if (ok && it != s->reqs.end() && sl.start && sl.gen && sl.done) {
    float g = 0.f, a = 0.f;
    if (hipEventElapsedTime(&g, sl.start, sl.gen) == hipSuccess &&
        hipEventElapsedTime(&a, sl.gen, sl.done) == hipSuccess) {
      it->second.gen_ms += g;
      it->second.attn_ms += a;
    }
  }
  for (hipEvent_t e : {sl.start, sl.gen, sl.done})
    if (e) s->events.push_back(e);
  if (it == s->reqs.end()) return;
  Request& rq = it->second;
  rq.slices_done += 1;
  if (!ok && !rq.failed) {
    rq.failed = true;
    rq.error = LA_ERR_HIP;
  }
  const bool all_admitted = rq.next_member >= rq.spec.desc.B;
  if (all_admitted && rq.slices_done == rq.slices_started)
    complete_request(s, rq, rq.failed, rq.error);
}

// Retire finished slices; returns how many finished.
int retire(la_server* s) {
  int n = 0;
  const uint64_t t = now_ns();
  for (size_t i = 0; i < s->inflight.size();) {
    Slice& sl = s->inflight[i];
    bool done = false, ok = true;
    if (s->cfg.fake_executor) {
      done = t >= sl.t_fake_done;
    } else {
      const hipError_t e = hipEventQuery(sl.done);
      if (e == hipSuccess) done = true;
      else if (e != hipErrorNotReady) { done = true; ok = false; }
    }
    if (done) {
      finish_slice(s, sl, ok && !sl.failed_launch);
      s->inflight[i] = s->inflight.back();
      s->inflight.pop_back();
      ++n;
    } else {
      ++i;
    }
  }
  return n;
}

// Admit slices in arrival order while a slot and budget allow.  With a cap
// on slices per request, a request holding its cap is passed over for the
// next one in the queue; budget shortage always stops admission (so a large
// request is never starved by smaller ones behind it).
int admit(la_server* s) {
  int n = 0;
  if (s->paused && !s->stopping) return 0;
  const int cap = s->cfg.max_slices_per_request;
  auto fit = s->fifo.begin();
  while (fit != s->fifo.end() && (int)s->inflight.size() < s->cfg.max_slots) {
    const uint64_t id = *fit;
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) { fit = s->fifo.erase(fit); continue; }
    Request& rq = it->second;
    if (cap > 0 && rq.slices_started - rq.slices_done >= cap) { ++fit; continue; }
    const la_request& r = rq.spec;
    if (reuses(r)) {
      // the owner cannot be released while this request is pending
      const Request& ow = s->reqs.at(r.reuse_summary_of);
      if (ow.state == LA_REQ_FAILED) {  // nothing to apply: fail, nothing started
        rq.next_member = r.desc.B;
        complete_request(s, rq, true, ow.error);
        fit = s->fifo.erase(fit);
        ++n;
        continue;
      }
      if (ow.state != LA_REQ_DONE) {  // its summary is not complete yet
        if (cap > 0) { ++fit; continue; }
        break;
      }
      rq.s = ow.s;
      rq.z = ow.z;
    }
    if (!rq.keep_held) {
      size_t off;
      if (!s->arena.alloc(keep_bytes(r), &off)) break;
      rq.keep_held = true;
      rq.keep_off = off;
      rq.keep_bytes = keep_bytes(r);
      char* p = s->base ? s->base + off : nullptr;
      const la_attn_desc& d = r.desc;
      const size_t sz = reuses(r) ? 0 : align_up((size_t)(d.B * d.H * d.d * d.d) * 8) +
                                            align_up((size_t)(d.B * d.H * d.d) * 8);
      if (!reuses(r)) {
        rq.s = (double*)p;
        rq.z = (double*)(p ? p + align_up((size_t)(d.B * d.H * d.d * d.d) * 8) : nullptr);
      }
      if (r.generate)
        rq.o = p ? p + sz : nullptr;
      else
        rq.o = r.o;
    }
    // largest member count that fits the biggest free block (and, with a
    // per-request cap, this request's share of the budget)
    int64_t left = r.desc.B - rq.next_member;
    int64_t m = left;
    if (s->cfg.max_members_per_slice > 0) m = std::min<int64_t>(m, s->cfg.max_members_per_slice);
    size_t room = s->arena.largest_free();
    if (cap > 0) {
      const size_t share = std::max<size_t>(s->cfg.hbm_budget_bytes / s->cfg.max_slots, slice_bytes(r, 1));
      room = std::min(room, share);
    }
    while (m > 0 && slice_bytes(r, m) > room) m = m > 8 ? m * 3 / 4 : m - 1;
    if (m <= 0) break;
    Slice sl{};
    sl.req = id;
    sl.index = rq.slices_started;
    sl.b0 = rq.next_member;
    sl.m = m;
    sl.bytes = slice_bytes(r, m);
    if (!s->arena.alloc(sl.bytes, &sl.off)) break;
    sl.stream = s->next_stream;
    s->next_stream = (s->next_stream + 1) % std::max(1, (int)s->streams.size());
    sl.start = take_event(s);
    sl.gen = take_event(s);
    sl.done = take_event(s);
    sl.fail = s->fail_at.count({id, sl.index}) > 0;
    sl.fail_late = s->fail_late_at.count({id, sl.index}) > 0;
    if (!s->cfg.fake_executor && !(sl.start && sl.gen && sl.done)) {
      for (hipEvent_t e : {sl.start, sl.gen, sl.done})
        if (e) s->events.push_back(e);
      s->arena.release(sl.off, sl.bytes);
      break;
    }
    if (rq.state == LA_REQ_QUEUED) {
      rq.state = LA_REQ_RUNNING;
      rq.t_admit = now_ns();
    }
    rq.next_member += m;
    rq.slices_started += 1;
    const bool all_admitted = rq.next_member >= r.desc.B;
    bool enqueued = false;
    const la_status st = launch_slice(s, rq, sl, &enqueued);
    if (st == LA_OK) {
      s->inflight.push_back(sl);
    } else if (!enqueued) {
      finish_slice(s, sl, false);
    } else {
      // Work already on the slice's stream may still write its memory:
      // keep the block until that work has drained (a marker event behind
      // it; without one, wait here), then retire the slice as failed.
      sl.failed_launch = true;
      if (!s->cfg.fake_executor) {
        hipStream_t stm = s->streams[sl.stream];
        if (hipEventRecord(sl.done, stm) != hipSuccess) {
          (void)hipStreamSynchronize(stm);
          finish_slice(s, sl, false);
          if (all_admitted) fit = s->fifo.erase(fit);
          ++n;
          continue;
        }
      }
      s->inflight.push_back(sl);
    }
    if (all_admitted) fit = s->fifo.erase(fit);
    ++n;
  }
  return n;
}

void scheduler(la_server* s) {
  if (!s->cfg.fake_executor) (void)hipSetDevice(s->cfg.device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    const int changed = retire(s) + admit(s);
    if (s->stopping && s->inflight.empty()) break;
    if (changed) {
      s->cv.notify_all();
      continue;
    }
    // idle: wake on new work, or poll the device every 20 us
    s->cv.wait_for(lk, std::chrono::microseconds(s->inflight.empty() ? 2000 : 20));
  }
  s->cv.notify_all();
}

}  // namespace

extern "C" {

la_status la_serve_create(const la_server_config* cfg, la_server** out) {
  if (!cfg || !out) return LA_ERR_INVALID_ARG;
  if (cfg->max_slots < 1 || cfg->n_streams < 1 || cfg->hbm_budget_bytes < kAlign ||
      cfg->max_members_per_slice < 0 || cfg->fake_slice_ns < 0 ||
      cfg->max_slices_per_request < 0)
    return LA_ERR_INVALID_ARG;
  la_server* s = new la_server();
  s->cfg = *cfg;
  s->arena.init(cfg->hbm_budget_bytes);
  if (!cfg->fake_executor) {
    hipError_t e = hipSetDevice(cfg->device);
    if (e == hipSuccess) e = hipMalloc((void**)&s->base, cfg->hbm_budget_bytes);
    if (e != hipSuccess) {
      delete s;
      return e == hipErrorOutOfMemory ? LA_ERR_OOM : LA_ERR_HIP;
    }
    for (int i = 0; i < cfg->n_streams; ++i) {
      hipStream_t st = nullptr;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        for (auto x : s->streams) (void)hipStreamDestroy(x);
        (void)hipFree(s->base);
        delete s;
        return LA_ERR_HIP;
      }
      s->streams.push_back(st);
    }
  } else {
    s->streams.resize(cfg->n_streams, nullptr);
  }
  s->th = std::thread(scheduler, s);
  *out = s;
  return LA_OK;
}

la_status la_serve_destroy(la_server* s) {
  if (!s) return LA_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
    // queued members are cancelled; admitted slices finish
    for (uint64_t id : s->fifo) {
      auto it = s->reqs.find(id);
      if (it == s->reqs.end()) continue;
      Request& rq = it->second;
      rq.next_member = rq.spec.desc.B;
      if (rq.slices_started == rq.slices_done) {
        complete_request(s, rq, true, LA_ERR_SHUTDOWN);
      } else {
        rq.failed = true;
        rq.error = LA_ERR_SHUTDOWN;
      }
    }
    s->fifo.clear();
  }
  s->cv.notify_all();
  s->th.join();
  if (!s->cfg.fake_executor) {
    for (auto e : s->events) (void)hipEventDestroy(e);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    (void)hipFree(s->base);
  }
  delete s;
  return LA_OK;
}

la_status la_serve_submit(la_server* s, const la_request* r, uint64_t* id) {
  if (!s || !r || !id) return LA_ERR_INVALID_ARG;
  la_request req = *r;
  la_attn_desc& d = req.desc;
  const bool reuse = reuses(req);
  if (req.generate) {
    if (r->q || r->k || r->v || r->o) return LA_ERR_INVALID_ARG;
    if (!(req.gen_std > 0.0)) return LA_ERR_INVALID_ARG;
    d.in_sn = d.d; d.in_sh = d.N * d.d; d.in_sb = d.H * d.in_sh;
    d.out_sn = d.d; d.out_sh = d.N * d.d; d.out_sb = d.H * d.out_sh;
  } else if (reuse) {
    if (r->k || r->v) return LA_ERR_INVALID_ARG;  // the owner's summary stands for them
    if (!s->cfg.fake_executor && (!r->q || !r->o)) return LA_ERR_INVALID_ARG;
  } else if (!s->cfg.fake_executor && (!r->q || !r->k || !r->v || !r->o)) {
    return LA_ERR_INVALID_ARG;
  }
  size_t ws = 0;
  la_status st = la_workspace_size(&d, reuse ? 2 : 0, &ws);
  if (st != LA_OK) return st;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return LA_ERR_SHUTDOWN;
  Request* owner = nullptr;
  if (reuse) {
    auto ot = s->reqs.find(req.reuse_summary_of);
    if (ot == s->reqs.end()) return LA_ERR_NOT_FOUND;
    owner = &ot->second;
    const la_attn_desc& od = owner->spec.desc;
    if (reuses(owner->spec) || owner->state == LA_REQ_FAILED || od.B != d.B || od.H != d.H ||
        od.d != d.d || od.in_dtype != d.in_dtype)
      return LA_ERR_INVALID_ARG;
  }
  if (keep_bytes(req) + slice_bytes(req, 1) > s->arena.size()) {
    s->n_rejected += 1;
    return LA_ERR_OOM;
  }
  const uint64_t rid = s->next_id++;
  if (owner) owner->reusers += 1;
  Request rq;
  rq.spec = req;
  rq.t_arrival = req.t_arrival_ns ? req.t_arrival_ns : now_ns();
  s->reqs.emplace(rid, rq);
  s->fifo.push_back(rid);
  s->n_submitted += 1;
  *id = rid;
  s->cv.notify_all();
  return LA_OK;
}

la_status la_serve_poll(la_server* s, uint64_t id, la_result* out) {
  if (!s || !out) return LA_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return LA_ERR_NOT_FOUND;
  const Request& rq = it->second;
  la_result r{};
  r.state = rq.state;
  r.error = rq.state == LA_REQ_FAILED ? rq.error : LA_OK;
  r.t_arrival_ns = rq.t_arrival;
  r.t_admit_ns = rq.t_admit;
  r.t_done_ns = rq.t_done;
  r.slices = rq.slices_started;
  r.o = rq.o;
  // a reusing request reports no S, z of its own (its owner's stay with it)
  r.s = reuses(rq.spec) ? nullptr : rq.s;
  r.z = reuses(rq.spec) ? nullptr : rq.z;
  r.gen_ms = rq.gen_ms;
  r.attn_ms = rq.attn_ms;
  *out = r;
  return LA_OK;
}

la_status la_serve_release(la_server* s, uint64_t id) {
  if (!s) return LA_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return LA_ERR_NOT_FOUND;
  Request& rq = it->second;
  if (rq.state != LA_REQ_DONE && rq.state != LA_REQ_FAILED) return LA_ERR_BUSY;
  if (rq.reusers > 0) return LA_ERR_BUSY;  // its S, z are still to be applied
  if (rq.keep_held) s->arena.release(rq.keep_off, rq.keep_bytes);
  s->reqs.erase(it);
  s->cv.notify_all();
  return LA_OK;
}

la_status la_serve_stats(la_server* s, la_serve_counters* out) {
  if (!s || !out) return LA_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  la_serve_counters r{};
  r.submitted = s->n_submitted;
  r.completed = s->n_completed;
  r.failed = s->n_failed;
  r.rejected = s->n_rejected;
  r.queued = (int64_t)s->fifo.size();
  r.in_flight_slices = (int64_t)s->inflight.size();
  r.bytes_in_use = s->arena.in_use();
  r.peak_bytes_in_use = s->arena.peak();
  r.budget_bytes = s->arena.size();
  *out = r;
  return LA_OK;
}

la_status la_serve_debug_fail_slice(la_server* s, uint64_t id, int32_t slice) {
  if (!s || slice < 0) return LA_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return LA_ERR_NOT_FOUND;
  if (it->second.slices_started > slice) return LA_ERR_BUSY;  // already launched
  s->fail_at.insert({id, slice});
  return LA_OK;
}

la_status la_serve_debug_fail_slice_late(la_server* s, uint64_t id, int32_t slice) {
  if (!s || slice < 0) return LA_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return LA_ERR_NOT_FOUND;
  if (it->second.slices_started > slice) return LA_ERR_BUSY;  // already launched
  s->fail_late_at.insert({id, slice});
  return LA_OK;
}

la_status la_serve_debug_pause(la_server* s, int32_t paused) {
  if (!s) return LA_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->paused = paused != 0;
  }
  s->cv.notify_all();
  return LA_OK;
}

}  // extern "C"
