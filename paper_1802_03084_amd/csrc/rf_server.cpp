// Serving runtime: segments of different shapes are admitted by an HBM
// budget and searched concurrently on slot streams (continuous batching).
//
// The paper's system streams overlapping segments from the correlator to
// search nodes (Law et al. 2018, section 3.2); on one GPU the analogue is a
// request loop: a segment is released (submitted) when its last integration
// has arrived, waits until a slot and enough device memory are free, is copied
// host to device on the slot's stream, searched by rf_search_segment, and its
// candidates are copied back.  Requests that arrive while others run are
// admitted as soon as a slot and memory free up, so their work overlaps on the
// device.
//
// Memory: the caller hands the server one device arena; each admitted request
// takes one block of it (segment copy, search workspace, candidate rows and
// count) from a first-fit allocator and returns it when done.  The library
// allocates no device memory.  Admission is in arrival order among the
// requests that fit: a later, smaller request may start while an earlier,
// larger one waits for memory.
#include "rf_internal.h"

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

namespace {

constexpr size_t kAlign = 256;
inline size_t aup(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t ticket = 0;
  const rf_plan *plan = nullptr;
  const void *h_vis = nullptr;
  size_t vis_bytes = 0, ws_bytes = 0, bytes = 0;
  int32_t cap = 0, flags = 0;
  Clock::time_point released, started, done_at;
  size_t off = 0;  // arena block
  std::vector<rf_candidate> cand;
  int32_t ncand = 0;
  rf_status status = RF_OK;
  bool done = false;
};

// First-fit allocator over [0, size): free blocks kept sorted by offset and
// merged on release.
struct Arena {
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(size_t n) {
    size = n;
    free_.clear();
    if (n) free_[0] = n;
  }
  bool alloc(size_t n, size_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

}  // namespace

struct rf_server {
  int device = 0;
  char *arena_base = nullptr;
  Arena arena;
  int nslots = 0;
  std::vector<std::thread> workers;
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> pending;        // released, not yet admitted (arrival order)
  std::map<int64_t, Request *> tickets;  // every request not yet collected by wait
  int64_t next_ticket = 1;
  int running = 0;
  bool stopping = false;
  Clock::time_point t0 = Clock::now();
};

namespace {

// Layout of one request's block: segment copy, workspace, candidates, count.
void request_layout(const rf_plan *p, int32_t cap, size_t *vis, size_t *ws, size_t *total) {
  const size_t sb = p->vis_dtype == RF_CF32 ? 8 : 4;
  *vis = (size_t)p->nint * p->nbl * p->nchan * p->npol * sb;
  *ws = segment_ws_bytes(p);
  *total = aup(*vis) + aup(*ws) + aup(sizeof(rf_candidate) * (size_t)std::max(cap, 1)) +
           aup(sizeof(int32_t));
}

// Runs one admitted request on stream s; returns its status.
rf_status serve_one(rf_server *sv, Request *r, hipStream_t s) {
  char *base = sv->arena_base + r->off;
  void *d_vis = base;
  void *d_ws = base + aup(r->vis_bytes);
  rf_candidate *d_cand = (rf_candidate *)(base + aup(r->vis_bytes) + aup(r->ws_bytes));
  int32_t *d_ncand =
      (int32_t *)((char *)d_cand + aup(sizeof(rf_candidate) * (size_t)std::max(r->cap, 1)));
  RF_HIP_TRY(hipMemcpyAsync(d_vis, r->h_vis, r->vis_bytes, hipMemcpyHostToDevice, s));
  if (r->flags & RF_SERVE_SUBTRACT_MEAN) {
    const rf_status sm = launch_mean_subtract(r->plan, d_vis, s);
    if (sm != RF_OK) return sm;
  }
  if (r->flags & RF_SERVE_FAIL_AFTER_COPY) return RF_EHIP;  // fault injection (tests)
  const rf_status st = rf_search_segment(r->plan, d_vis, d_cand, r->cap, d_ncand, nullptr, d_ws,
                                         r->ws_bytes, s);
  if (st != RF_OK) return st;
  RF_HIP_TRY(hipMemcpyAsync(&r->ncand, d_ncand, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  RF_HIP_TRY(hipStreamSynchronize(s));
  const int32_t n = std::min(r->ncand, r->cap);
  r->cand.resize((size_t)std::max(n, 0));
  if (n > 0) {
    RF_HIP_TRY(hipMemcpyAsync(r->cand.data(), d_cand, sizeof(rf_candidate) * (size_t)n,
                              hipMemcpyDeviceToHost, s));
    RF_HIP_TRY(hipStreamSynchronize(s));
  }
  return RF_OK;
}

void worker(rf_server *sv) {
  hipStream_t s = nullptr;
  const bool ok = hipSetDevice(sv->device) == hipSuccess &&
                  hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
  for (;;) {
    Request *r = nullptr;
    {
      std::unique_lock<std::mutex> lk(sv->m);
      for (;;) {
        if (sv->stopping && sv->pending.empty()) break;
        // the first request, in arrival order, whose block fits
        for (auto it = sv->pending.begin(); it != sv->pending.end(); ++it) {
          size_t off = 0;
          if (sv->arena.alloc((*it)->bytes, &off)) {
            r = *it;
            r->off = off;
            sv->pending.erase(it);
            break;
          }
        }
        if (r) break;
        sv->cv_work.wait(lk);
      }
      if (!r) break;
      ++sv->running;
      r->started = Clock::now();
    }
    const rf_status st = ok ? serve_one(sv, r, s) : RF_EHIP;
    // A request that failed part way may still have a copy or kernels in
    // flight on s (the search joins its own lane streams before it returns):
    // drain s before its block goes back to the arena, so that no later
    // request is admitted into memory that is still being written.
    if (st != RF_OK && s) (void)hipStreamSynchronize(s);
    {
      std::lock_guard<std::mutex> lk(sv->m);
      sv->arena.release(r->off, r->bytes);
      r->status = st;
      r->done_at = Clock::now();
      r->done = true;
      --sv->running;
    }
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();  // memory came free
  }
  if (s) (void)hipStreamDestroy(s);
}

}  // namespace

extern "C" {

rf_status rf_server_request_bytes(const rf_plan *p, int32_t cap, size_t *bytes) {
  if (!p || !bytes) return RF_EINVAL;
  if (cap < 0) return RF_ERANGE;
  size_t v, w;
  request_layout(p, cap, &v, &w, bytes);
  return RF_OK;
}

rf_status rf_server_create(void *d_arena, size_t arena_bytes, int32_t nslots, rf_server **out) {
  if (!out) return RF_EINVAL;
  *out = nullptr;
  if (!d_arena || arena_bytes == 0) return RF_EINVAL;
  if (nslots < 1 || nslots > 16) return RF_ERANGE;
  if ((uintptr_t)d_arena % kAlign) return RF_EINVAL;
  int dev = 0;
  RF_HIP_TRY(hipGetDevice(&dev));
  rf_server *sv = new rf_server();
  sv->device = dev;
  sv->arena_base = (char *)d_arena;
  sv->arena.init(arena_bytes & ~(kAlign - 1));
  sv->nslots = nslots;
  for (int k = 0; k < nslots; ++k) sv->workers.emplace_back(worker, sv);
  *out = sv;
  return RF_OK;
}

rf_status rf_server_submit(rf_server *sv, const rf_plan *p, const void *h_vis, int32_t cap,
                           int32_t flags, int64_t *ticket) {
  if (!sv || !p || !h_vis || !ticket) return RF_EINVAL;
  if (cap < 0) return RF_ERANGE;
  if (flags & ~(RF_SERVE_SUBTRACT_MEAN | RF_SERVE_FAIL_AFTER_COPY)) return RF_EINVAL;
  Request *r = new Request();
  r->plan = p;
  r->h_vis = h_vis;
  r->cap = cap;
  r->flags = flags;
  request_layout(p, cap, &r->vis_bytes, &r->ws_bytes, &r->bytes);
  {
    std::lock_guard<std::mutex> lk(sv->m);
    if (sv->stopping || r->bytes > sv->arena.size) {  // could never be admitted
      delete r;
      return sv->stopping ? RF_EINVAL : RF_EWORKSPACE;
    }
    r->ticket = sv->next_ticket++;
    r->released = Clock::now();
    sv->pending.push_back(r);
    sv->tickets[r->ticket] = r;
    *ticket = r->ticket;
  }
  sv->cv_work.notify_all();
  return RF_OK;
}

rf_status rf_server_wait(rf_server *sv, int64_t ticket, rf_candidate *h_cand, int32_t cap,
                         int32_t *ncand, rf_serve_times *times) {
  if (!sv || !ncand || (cap > 0 && !h_cand)) return RF_EINVAL;
  if (cap < 0) return RF_ERANGE;
  Request *r = nullptr;
  {
    std::unique_lock<std::mutex> lk(sv->m);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return RF_EINVAL;  // unknown, or already claimed
    r = it->second;
    sv->tickets.erase(it);  // claimed: this call frees it
    sv->cv_done.wait(lk, [&] { return r->done; });
  }
  const rf_status st = r->status;
  *ncand = r->ncand;
  const size_t n = std::min(r->cand.size(), (size_t)cap);
  if (n) std::memcpy(h_cand, r->cand.data(), sizeof(rf_candidate) * n);
  if (times) {
    auto sec = [&](Clock::time_point t) {
      return std::chrono::duration<double>(t - sv->t0).count();
    };
    times->released_s = sec(r->released);
    times->started_s = sec(r->started);
    times->done_s = sec(r->done_at);
    times->latency_s = std::chrono::duration<double>(r->done_at - r->released).count();
  }
  delete r;
  return st;
}

rf_status rf_server_destroy(rf_server *sv) {
  if (!sv) return RF_EINVAL;
  {
    std::lock_guard<std::mutex> lk(sv->m);
    sv->stopping = true;  // pending requests still run; then the workers exit
  }
  sv->cv_work.notify_all();
  for (auto &t : sv->workers) t.join();
  for (auto &kv : sv->tickets) delete kv.second;  // finished but never collected
  delete sv;
  return RF_OK;
}

}  // extern "C"
