// Serving scheduler: continuous batching of independent solves.
//
// Requests queue in FIFO order; a request is admitted when a slot (one HIP
// stream) and enough of the caller's device arena for its solver workspace
// are free.  Each in-flight solve advances on its own stream: the scheduler
// launches its next batch of iterations (and the copy of its flags) as soon
// as the previous one has landed, which it learns from an event recorded
// after the flag copy, so a solve on a small lattice never waits for the
// iterations of a large one.  Finished solves give back their slot and arena
// memory and the next queued requests move in at once.  The per-RHS
// arithmetic of a solve does not depend on what else runs, so a result is
// the same alone and in the mix.  Calls on one server must not overlap
// (single host thread).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "wd_internal.h"

namespace {

// First-fit allocator over [0, size) with 256-byte granularity.
class Arena {
 public:
  explicit Arena(size_t size) { free_.push_back({0, size}); }
  bool alloc(size_t n, size_t* off) {
    n = (n + 255) / 256 * 256;
    for (size_t i = 0; i < free_.size(); ++i) {
      if (free_[i].size >= n) {
        *off = free_[i].off;
        free_[i].off += n;
        free_[i].size -= n;
        if (free_[i].size == 0) free_.erase(free_.begin() + i);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) / 256 * 256;
    free_.push_back({off, n});
    std::sort(free_.begin(), free_.end(), [](const Blk& a, const Blk& b) { return a.off < b.off; });
    std::vector<Blk> merged;
    for (const Blk& b : free_) {
      if (!merged.empty() && merged.back().off + merged.back().size == b.off) merged.back().size += b.size;
      else merged.push_back(b);
    }
    free_.swap(merged);
  }
 private:
  struct Blk {
    size_t off, size;
  };
  std::vector<Blk> free_;
};

enum class State { Queued, Active, Done };

struct Request {
  int64_t id;
  int32_t kind;
  const wd_gauge* g;
  double kappa;
  double* x;
  const double* b;
  wd_solve_params prm;
  size_t need;
  State state = State::Queued;
  size_t off = 0;
  int slot = -1;
  wd_solver* h = nullptr;
  bool issued = false;  // iterations launched whose flags have not been read yet
  wd_status status = WD_OK;
  std::vector<wd_solve_info> info;
};

}  // namespace

struct wd_server {
  char* arena_base;
  size_t arena_bytes;
  Arena arena;
  wd_serve_params prm;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;  // per slot: recorded after the issued work's flag copy
  std::vector<int64_t> slot_req;  // request in each slot, -1 if free
  std::deque<int64_t> queue;
  std::map<int64_t, Request> reqs;
  int64_t next_id = 1;
  wd_server(char* base, size_t bytes, const wd_serve_params& p) : arena_base(base), arena_bytes(bytes), arena(bytes), prm(p) {}
};

using namespace wd;

namespace {

void finish(wd_server* s, Request& r) {
  r.info.assign(r.prm.nrhs, wd_solve_info{});
  r.status = wd_solver_end(r.h, r.info.data());
  r.h = nullptr;
  r.state = State::Done;
  s->arena.release(r.off, r.need);
  s->slot_req[r.slot] = -1;
  r.slot = -1;
}

wd_status admit(wd_server* s) {
  while (!s->queue.empty()) {
    const auto free_slot = std::find(s->slot_req.begin(), s->slot_req.end(), (int64_t)-1);
    if (free_slot == s->slot_req.end()) break;
    Request& r = s->reqs.at(s->queue.front());
    size_t off = 0;
    if (!s->arena.alloc(r.need, &off)) break;  // wait for memory (FIFO order)
    s->queue.pop_front();
    const int slot = (int)(free_slot - s->slot_req.begin());
    r.off = off;
    r.slot = slot;
    const wd_status st = wd_solver_begin(r.kind, r.g, r.kappa, r.x, r.b, &r.prm, s->arena_base + off,
                                         r.need, s->streams[slot], &r.h);
    if (st != WD_OK) {  // e.g. a NaN source: the request ends at once
      r.status = st;
      r.state = State::Done;
      r.info.assign(r.prm.nrhs, wd_solve_info{});
      s->arena.release(off, r.need);
      r.slot = -1;
      continue;
    }
    r.state = State::Active;
    s->slot_req[slot] = r.id;
  }
  return WD_OK;
}

}  // namespace

extern "C" {

wd_status wd_server_create(void* arena, size_t arena_bytes, const wd_serve_params* params, wd_server** out) {
  set_error("");
  if (!out) return fail(WD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!params) return fail(WD_EINVAL, "params is NULL");
  if (!arena || reinterpret_cast<uintptr_t>(arena) % 256) return fail(WD_EINVAL, "arena must be 256-byte aligned");
  if (params->max_slots < 1 || params->max_slots > 64) return fail(WD_EINVAL, "max_slots must be in [1, 64]");
  if (params->iters_per_pump < 1) return fail(WD_EINVAL, "iters_per_pump must be >= 1");
  wd_server* s = new (std::nothrow) wd_server(static_cast<char*>(arena), arena_bytes, *params);
  if (!s) return fail(WD_ENOMEM, "host allocation failed");
  for (int i = 0; i < params->max_slots; ++i) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) {
      s->streams.push_back(st);
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) s->events.push_back(ev);
    }
    if (e != hipSuccess) {
      for (hipStream_t t : s->streams) (void)hipStreamDestroy(t);
      for (hipEvent_t t : s->events) (void)hipEventDestroy(t);
      delete s;
      return fail(WD_EDEVICE, std::string("stream creation: ") + hipGetErrorString(e));
    }
  }
  s->slot_req.assign(params->max_slots, -1);
  *out = s;
  return WD_OK;
}

wd_status wd_server_submit(wd_server* s, int32_t solver, const wd_gauge* g, double kappa, double* x,
                           const double* b, const wd_solve_params* params, int64_t* request_id) {
  set_error("");
  if (!s || !g || !params || !request_id) return fail(WD_EINVAL, "NULL argument");
  const size_t need = wd_solve_workspace_bytes(&g->lat, params, solver);
  if (need == 0) return fail(WD_EINVAL, "invalid solve parameters");
  if ((need + 255) / 256 * 256 > s->arena_bytes)
    return fail(WD_ENOMEM, "request workspace (" + std::to_string(need) + " bytes) exceeds the arena");
  Request r;
  r.id = s->next_id++;
  r.kind = solver;
  r.g = g;
  r.kappa = kappa;
  r.x = x;
  r.b = b;
  r.prm = *params;
  r.need = need;
  s->reqs.emplace(r.id, r);
  s->queue.push_back(r.id);
  *request_id = r.id;
  return WD_OK;
}

wd_status wd_server_pump(wd_server* s, int32_t* n_active, int32_t* n_queued) {
  set_error("");
  if (!s) return fail(WD_EINVAL, "server is NULL");
  admit(s);
  // Each round: launch the next iterations of every in-flight solve that has
  // none outstanding, then complete whichever solves have landed (at least
  // one; the host polls the slots' events meanwhile), releasing finished
  // ones and admitting queued requests into their slots.
  for (int round = 0; round < s->prm.iters_per_pump; ++round) {
    bool outstanding = false;
    for (size_t slot = 0; slot < s->slot_req.size(); ++slot) {
      if (s->slot_req[slot] < 0) continue;
      Request& r = s->reqs.at(s->slot_req[slot]);
      if (!r.issued && solver_finished(r.h)) {  // e.g. converged at prepare: release at once
        finish(s, r);
        continue;
      }
      if (!r.issued) {
        hipError_t e = solver_issue(r.h);
        if (e == hipSuccess) e = hipEventRecord(s->events[slot], s->streams[slot]);
        if (e != hipSuccess) return fail(WD_EDEVICE, std::string("serve issue: ") + hipGetErrorString(e));
        r.issued = true;
      }
      outstanding |= r.issued;
    }
    if (!outstanding) {  // nothing in flight: admit what the released slots allow
      admit(s);
      break;
    }
    int completed = 0;
    while (completed == 0) {
      for (size_t slot = 0; slot < s->slot_req.size(); ++slot) {
        if (s->slot_req[slot] < 0) continue;
        Request& r = s->reqs.at(s->slot_req[slot]);
        if (!r.issued) continue;
        const hipError_t q = hipEventQuery(s->events[slot]);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return fail(WD_EDEVICE, std::string("serve wait: ") + hipGetErrorString(q));
        r.issued = false;
        ++completed;
        const wd_status st = solver_complete(r.h);
        if (st < 0 && st != WD_EBREAKDOWN) return st;
        if (solver_finished(r.h)) finish(s, r);
      }
      if (completed == 0) std::this_thread::yield();
    }
    admit(s);
  }
  int na = 0;
  for (int64_t id : s->slot_req) na += id >= 0;
  if (n_active) *n_active = na;
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  return WD_OK;
}

wd_status wd_server_poll(wd_server* s, int64_t request_id, int32_t* done, int32_t* status, wd_solve_info* info) {
  set_error("");
  if (!s || !done) return fail(WD_EINVAL, "NULL argument");
  auto it = s->reqs.find(request_id);
  if (it == s->reqs.end()) return fail(WD_EINVAL, "unknown request id");
  const Request& r = it->second;
  *done = r.state == State::Done ? 1 : 0;
  if (*done) {
    if (status) *status = r.status;
    if (info)
      for (size_t k = 0; k < r.info.size(); ++k) info[k] = r.info[k];
  }
  return WD_OK;
}

wd_status wd_server_destroy(wd_server* s) {
  set_error("");
  if (!s) return WD_OK;
  // finish what is in flight so no kernel still uses the arena
  for (int guard = 0; guard < 1000000; ++guard) {
    bool any = false;
    for (int64_t id : s->slot_req) any |= id >= 0;
    if (!any) break;
    s->queue.clear();
    if (wd_server_pump(s, nullptr, nullptr) != WD_OK) break;
  }
  for (auto& kv : s->reqs)
    if (kv.second.h) wd_solver_end(kv.second.h, nullptr);
  for (hipStream_t t : s->streams) (void)hipStreamDestroy(t);
  for (hipEvent_t t : s->events) (void)hipEventDestroy(t);
  delete s;
  return WD_OK;
}

}  // extern "C"
