// Serving engine: continuous admission of states-merging recursions
// (Algorithm 1 body, one sqc_recurse each) onto concurrent HIP streams.
//
// The engine is host code layered on the public interface: each slot is a
// stream with its own context; a request gets a block of the engine's
// workspace of its footprint (first fit over a free list), its context is
// pointed at that block, sqc_recurse enqueues the recursion on the slot's
// stream and an event marks its end.  Retiring a finished request frees its
// slot and block; waiting requests are then admitted in arrival order,
// skipping those that do not fit yet.
#include <hip/hip_runtime.h>

#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/sqc.h"

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kMinBlock = 4096;  // a context's control region

size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Circuit {
  std::vector<sqc_tensor> att;
  std::vector<sqc_cut> cuts;
  std::vector<int32_t> n_bits;
};

struct Pending {
  uint64_t ticket;
  sqc_request req;
  std::vector<sqc_masks> scope;
  size_t footprint;
};

struct Slot {
  hipStream_t stream = nullptr;
  sqc_ctx *ctx = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  uint64_t ticket = 0;
  size_t off = 0, len = 0;  // workspace block of the running request
};

enum State { kWaiting = 0, kRunning = 1, kDone = 2, kFailed = 3 };

}  // namespace

struct sqc_server {
  int device = 0;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  std::map<size_t, size_t> free_blocks;  // offset -> length
  std::vector<Slot> slots;
  std::vector<Circuit> circuits;
  std::deque<Pending> waiting;
  std::deque<uint64_t> finished;  // completion queue
  std::unordered_map<uint64_t, int> state;
  std::unordered_map<uint64_t, std::string> failure;
  uint64_t next_ticket = 1;
  sqc_serve_stats st{};
  std::string err;
};

namespace {

sqc_status fail(sqc_server *s, sqc_status code, const std::string &msg) {
  if (s) s->err = msg;
  return code;
}

bool take_block(sqc_server *s, size_t need, size_t &off) {
  for (auto it = s->free_blocks.begin(); it != s->free_blocks.end(); ++it) {
    if (it->second >= need) {
      off = it->first;
      const size_t rest = it->second - need;
      s->free_blocks.erase(it);
      if (rest) s->free_blocks[off + need] = rest;
      return true;
    }
  }
  return false;
}

void give_block(sqc_server *s, size_t off, size_t len) {
  auto it = s->free_blocks.emplace(off, len).first;
  // merge with the next and the previous free block
  auto nx = std::next(it);
  if (nx != s->free_blocks.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    s->free_blocks.erase(nx);
  }
  if (it != s->free_blocks.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      s->free_blocks.erase(it);
    }
  }
}

size_t footprint_of(sqc_server *s, const sqc_request &r, const sqc_masks *scope) {
  if (r.circuit < 0 || r.circuit >= (int)s->circuits.size()) return 0;
  const Circuit &c = s->circuits[r.circuit];
  const int n_sub = (int)c.att.size();
  std::vector<sqc_masks> m(n_sub);
  if (sqc_assign_bins(n_sub, c.n_bits.data(), scope, r.max_bins_M, m.data()) != SQC_OK) return 0;
  const size_t b = sqc_recurse_workspace_bytes(c.att.data(), n_sub, c.cuts.data(), (int32_t)c.cuts.size(),
                                               m.data(), r.prec);
  if (!b) return 0;
  return round_up(b < kMinBlock ? kMinBlock : b);
}

// Retire finished requests; admit waiting ones that fit.
sqc_status pump(sqc_server *s) {
  for (auto &sl : s->slots) {
    if (!sl.busy) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return fail(s, SQC_E_DEVICE, std::string("request failed on the device: ") +
                                                          hipGetErrorString(q));
    s->state[sl.ticket] = kDone;
    s->finished.push_back(sl.ticket);
    give_block(s, sl.off, sl.len);
    s->st.workspace_bytes -= sl.len;
    sl.busy = false;
    s->st.running -= 1;
    s->st.completed += 1;
  }
  for (auto it = s->waiting.begin(); it != s->waiting.end();) {
    Slot *idle = nullptr;
    for (auto &sl : s->slots)
      if (!sl.busy) {
        idle = &sl;
        break;
      }
    if (!idle) break;
    size_t off = 0;
    if (!take_block(s, it->footprint, off)) {
      ++it;  // a later, smaller request may fit
      continue;
    }
    const Circuit &c = s->circuits[it->req.circuit];
    // point the slot's context at the block (a host-side pointer update)
    sqc_status rc = sqc_ctx_set_workspace(idle->ctx, s->ws + off, it->footprint);
    if (rc == SQC_OK) {
      const sqc_masks *scope = it->scope.empty() ? nullptr : it->scope.data();
      rc = sqc_recurse(idle->ctx, c.att.data(), (int32_t)c.att.size(), c.cuts.data(),
                       (int32_t)c.cuts.size(), scope, it->req.max_bins_M, it->req.top_r, it->req.prec,
                       it->req.bins_dev, it->req.bins_prec, it->req.masks_out, it->req.topr_dev,
                       it->req.sum_dev);
    }
    if (rc == SQC_OK && hipEventRecord(idle->done, idle->stream) != hipSuccess) rc = SQC_E_DEVICE;
    if (rc != SQC_OK) {
      give_block(s, off, it->footprint);
      s->state[it->ticket] = kFailed;
      s->failure[it->ticket] = sqc_last_error(idle->ctx);
    } else {
      idle->busy = true;
      idle->ticket = it->ticket;
      idle->off = off;
      idle->len = it->footprint;
      s->state[it->ticket] = kRunning;
      s->st.admitted += 1;
      s->st.running += 1;
      s->st.workspace_bytes += it->footprint;
      if (s->st.workspace_bytes > s->st.workspace_peak) s->st.workspace_peak = s->st.workspace_bytes;
      if (s->st.running > s->st.max_running) s->st.max_running = s->st.running;
    }
    it = s->waiting.erase(it);
  }
  s->st.queued = (int32_t)s->waiting.size();
  return SQC_OK;
}

}  // namespace

extern "C" {

sqc_status sqc_serve_create(int device, int32_t n_slots, void *workspace_dev, size_t workspace_bytes,
                            sqc_server **out) {
  if (!out || !workspace_dev || n_slots < 1 || n_slots > 64) return SQC_E_ARG;
  if (reinterpret_cast<uintptr_t>(workspace_dev) % kAlign || workspace_bytes < kMinBlock) return SQC_E_ARG;
  if (hipSetDevice(device) != hipSuccess) return SQC_E_DEVICE;
  sqc_server *s = new sqc_server();
  s->device = device;
  s->ws = static_cast<char *>(workspace_dev);
  s->ws_bytes = workspace_bytes / kAlign * kAlign;
  s->free_blocks[0] = s->ws_bytes;
  s->slots.resize(n_slots);
  for (auto &sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        sqc_ctx_create(device, sl.stream, &sl.ctx) != SQC_OK) {
      sqc_serve_destroy(s);
      return SQC_E_DEVICE;
    }
  }
  *out = s;
  return SQC_OK;
}

sqc_status sqc_serve_destroy(sqc_server *s) {
  if (!s) return SQC_E_ARG;
  for (auto &sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.ctx) sqc_ctx_destroy(sl.ctx);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  delete s;
  return SQC_OK;
}

sqc_status sqc_serve_register(sqc_server *s, const sqc_tensor *attributed, int32_t n_sub,
                              const sqc_cut *cuts, int32_t n_cuts, int32_t *circuit_id) {
  if (!s || !attributed || !circuit_id || n_sub < 1 || (n_cuts > 0 && !cuts) || n_cuts < 0)
    return fail(s, SQC_E_ARG, "invalid argument to sqc_serve_register");
  Circuit c;
  c.att.assign(attributed, attributed + n_sub);
  c.cuts.assign(cuts, cuts + n_cuts);
  for (int i = 0; i < n_sub; ++i) {
    if (attributed[i].layout != SQC_LAYOUT_ATTRIBUTED || !attributed[i].data)
      return fail(s, SQC_E_SHAPE, "registered tensors must be attributed tensors with data");
    c.n_bits.push_back(attributed[i].n_bits);
  }
  // the full-state footprint validates the graph and the tensors
  sqc_request probe{};
  probe.max_bins_M = 1;
  probe.prec = SQC_F64;
  s->circuits.push_back(c);
  probe.circuit = (int32_t)s->circuits.size() - 1;
  if (!footprint_of(s, probe, nullptr)) {
    s->circuits.pop_back();
    return fail(s, SQC_E_SHAPE, "the circuit's tensors and cuts do not form a valid compute graph");
  }
  *circuit_id = probe.circuit;
  return SQC_OK;
}

size_t sqc_serve_footprint(sqc_server *s, const sqc_request *req) {
  if (!s || !req) return 0;
  return footprint_of(s, *req, req->scope);
}

sqc_status sqc_serve_submit(sqc_server *s, const sqc_request *req, uint64_t *ticket) {
  if (!s || !req || !ticket) return fail(s, SQC_E_ARG, "invalid argument to sqc_serve_submit");
  if (req->circuit < 0 || req->circuit >= (int)s->circuits.size())
    return fail(s, SQC_E_ARG, "unknown circuit id");
  if (!req->bins_dev || !req->topr_dev || !req->sum_dev)
    return fail(s, SQC_E_ARG, "request output buffers must be set");
  if (req->top_r < 1 || req->top_r > SQC_MAX_TOPR) return fail(s, SQC_E_ARG, "top_r must be in [1, 64]");
  const size_t need = footprint_of(s, *req, req->scope);
  if (!need) return fail(s, SQC_E_ARG, "the request is not valid for its circuit");
  if (need > s->ws_bytes) return fail(s, SQC_E_NOMEM, "the request's footprint exceeds the server workspace");
  Pending p;
  p.ticket = s->next_ticket++;
  p.req = *req;
  if (req->scope) p.scope.assign(req->scope, req->scope + s->circuits[req->circuit].att.size());
  p.req.scope = nullptr;
  p.footprint = need;
  s->state[p.ticket] = kWaiting;
  s->waiting.push_back(std::move(p));
  s->st.submitted += 1;
  *ticket = s->next_ticket - 1;
  return pump(s);
}

sqc_status sqc_serve_poll(sqc_server *s, uint64_t ticket, int32_t *state) {
  if (!s || !state) return fail(s, SQC_E_ARG, "invalid argument to sqc_serve_poll");
  const sqc_status rc = pump(s);
  if (rc != SQC_OK) return rc;
  auto it = s->state.find(ticket);
  if (it == s->state.end()) return fail(s, SQC_E_ARG, "unknown ticket");
  if (it->second == kFailed) return fail(s, SQC_E_ARG, s->failure[ticket]);
  *state = it->second;
  return SQC_OK;
}

sqc_status sqc_serve_wait(sqc_server *s, uint64_t ticket) {
  if (!s) return SQC_E_ARG;
  while (true) {
    int32_t st = 0;
    const sqc_status rc = sqc_serve_poll(s, ticket, &st);
    if (rc != SQC_OK) return rc;
    if (st == kDone) return SQC_OK;
    // block on the running request that holds the ticket, else on any slot
    hipEvent_t ev = nullptr;
    for (auto &sl : s->slots)
      if (sl.busy && (sl.ticket == ticket || !ev)) ev = sl.done;
    if (!ev) return fail(s, SQC_E_ARG, "request can never be admitted");
    if (hipEventSynchronize(ev) != hipSuccess) return fail(s, SQC_E_DEVICE, "hipEventSynchronize failed");
  }
}

sqc_status sqc_serve_completed(sqc_server *s, uint64_t *tickets, int32_t cap, int32_t *n) {
  if (!s || !n || cap < 0 || (cap > 0 && !tickets)) return fail(s, SQC_E_ARG, "invalid argument to sqc_serve_completed");
  const sqc_status rc = pump(s);
  if (rc != SQC_OK) return rc;
  int32_t k = 0;
  while (k < cap && !s->finished.empty()) {
    tickets[k++] = s->finished.front();
    s->state.erase(s->finished.front());
    s->finished.pop_front();
  }
  *n = k;
  return SQC_OK;
}

sqc_status sqc_serve_get_stats(sqc_server *s, sqc_serve_stats *out) {
  if (!s || !out) return SQC_E_ARG;
  *out = s->st;
  return SQC_OK;
}

const char *sqc_serve_last_error(const sqc_server *s) { return s ? s->err.c_str() : "no server"; }

}  // extern "C"
