// Serving engine: continuous batching of states-merging recursions (one
// Algorithm 1 body each) onto concurrent HIP streams.
//
// A request is validated and planned when it is submitted (bin masks,
// contraction plan, workspace footprint).  Whenever a slot (a stream with its
// own context) is idle, the engine forms a batch from the waiting requests in
// arrival order (skipping those that do not fit yet), takes one block of the
// workspace for the batch's job table and the requests' workspaces (first fit
// over a free list), and enqueues the batch: its job table is copied to the
// device and every request's merges, GEMM steps and top-R selection run in
// shared launches (one per pass, per GEMM level and kernel specialisation).
// An event marks the batch's end; retiring it frees the slot and the block.
// Batches on different slots overlap on the device, so requests that arrive
// while others run are admitted as slots and memory free up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/sqc.h"
#include "batch.hpp"
#include "common.hpp"

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kMinWorkspace = 4096;
constexpr size_t kStagingBytes = size_t(2) << 20;  // pinned job-table image per slot
constexpr int kMaxBatch = 128;                      // requests per batch
// A request passed over this many times (it did not fit while later ones
// did) stops later requests from being admitted until it runs, so the
// memory the running batches free up goes to it (aging: no starvation).
constexpr int kMaxSkips = 8;

size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Pending {
  uint64_t ticket = 0;
  sqc::PreparedPtr prep;
  size_t ws = 0, table = 0;  // workspace and job-table bytes (rounded)
  int skips = 0;             // batches formed without it although it waited
};

struct Slot {
  hipStream_t stream = nullptr;
  sqc_ctx *ctx = nullptr;
  hipEvent_t done = nullptr;
  void *staging = nullptr;  // pinned host image of the batch's job table
  bool busy = false;
  std::vector<Pending> batch;
  size_t off = 0, len = 0;  // workspace block of the running batch
};

enum State { kWaiting = 0, kRunning = 1, kDone = 2, kFailed = 3 };

}  // namespace

struct sqc_server {
  int device = 0;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  std::map<size_t, size_t> free_blocks;  // offset -> length
  std::vector<Slot> slots;
  std::vector<std::shared_ptr<const sqc::CircuitTopo>> circuits;
  std::deque<Pending> waiting;
  std::deque<uint64_t> finished;  // completion queue
  std::unordered_map<uint64_t, int> state;
  std::unordered_map<uint64_t, std::string> failure;
  uint64_t next_ticket = 1;
  int max_batch = kMaxBatch;
  sqc_serve_stats st{};
  std::string err;
};

namespace {

sqc_status fail(sqc_server *s, sqc_status code, const std::string &msg) {
  if (s) s->err = msg;
  return code;
}

size_t largest_free(const sqc_server *s) {
  size_t m = 0;
  for (auto &kv : s->free_blocks) m = std::max(m, kv.second);
  return m;
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

// Workspace block of a batch: the job table (when it holds more than one
// request), then each request's workspace.
size_t batch_bytes(size_t table, size_t ws_sum, int count) { return (count > 1 ? table : 0) + ws_sum; }

// The batching policy (host only, no device state): from the waiting
// requests in arrival order, take requests while they fit `room` (job tables
// within `staging`), up to `target`; a request that does not fit may be
// passed by later ones, and each pass counts against it; one passed over
// kMaxSkips times stops the scan (nothing behind it is admitted first).
// When a batch is formed, every request passed over gains one skip.  Returns
// the count taken; `picked` gets their positions (ascending), `held` 1 when
// an aged request stopped the scan, `table` / `ws_sum` the batch's sums.
int pick_batch(const size_t *ws, const size_t *tab, int32_t *skips, int32_t n, size_t room, size_t staging,
               int target, int32_t *picked, int32_t *held, size_t *table_out, size_t *ws_out) {
  size_t table = 0, ws_sum = 0;
  int count = 0;
  std::vector<int32_t> passed;
  *held = 0;
  for (int32_t k = 0; k < n && count < target; ++k) {
    const size_t t2 = table + tab[k], w2 = ws_sum + ws[k];
    if (batch_bytes(t2, w2, count + 1) <= room && t2 <= staging) {
      table = t2;
      ws_sum = w2;
      picked[count++] = k;
    } else if (skips[k] >= kMaxSkips) {
      *held = 1;  // aged: nothing behind it goes first
      break;
    } else {
      passed.push_back(k);  // a later, smaller request may fit
    }
  }
  if (count)
    for (int32_t k : passed) skips[k] += 1;
  *table_out = table;
  *ws_out = ws_sum;
  return count;
}

// Enqueue the slot's batch into the block at `off`.
void launch_batch(sqc_server *s, Slot &sl, size_t off) {
  char *base = s->ws + off;
  const int n = (int)sl.batch.size();
  if (n == 1) {
    sqc::enqueue_prepared(sl.ctx, *sl.batch[0].prep, base);
  } else {
    size_t table = 0;
    for (auto &p : sl.batch) table += p.table;
    std::vector<sqc::PreparedRecursion *> ps;
    std::vector<char *> wss;
    size_t at = table;
    for (auto &p : sl.batch) {
      ps.push_back(p.prep.get());
      wss.push_back(base + at);
      at += p.ws;
    }
    sqc::enqueue_batch(sl.ctx, ps.data(), n, wss.data(), base, table, sl.staging, kStagingBytes);
  }
  if (hipEventRecord(sl.done, sl.stream) != hipSuccess)
    throw sqc::Error{SQC_E_DEVICE, "hipEventRecord failed"};
}

// Retire finished batches; admit waiting requests in batches.
// (`want`: a batch size to aim for at least, when enough requests wait)
sqc_status pump(sqc_server *s, int want = 0) {
  for (auto &sl : s->slots) {
    if (!sl.busy) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess)
      return fail(s, SQC_E_DEVICE, std::string("request failed on the device: ") + hipGetErrorString(q));
    for (auto &p : sl.batch) {
      s->state[p.ticket] = kDone;
      s->finished.push_back(p.ticket);
    }
    give_block(s, sl.off, sl.len);
    s->st.workspace_bytes -= sl.len;
    s->st.running -= (int32_t)sl.batch.size();
    s->st.completed += sl.batch.size();
    sl.batch.clear();
    sl.busy = false;
  }
  while (!s->waiting.empty()) {
    int idle = 0;
    Slot *slot = nullptr;
    for (auto &sl : s->slots)
      if (!sl.busy) {
        ++idle;
        if (!slot) slot = &sl;
      }
    if (!slot) break;
    // share the waiting requests among the idle slots
    const int target =
        std::min<int>(s->max_batch, std::max<int>(want, (int)((s->waiting.size() + idle - 1) / idle)));
    const size_t room = largest_free(s);
    size_t table = 0, ws_sum = 0;
    int count = 0;
    std::vector<size_t> wsz, tsz;
    std::vector<int32_t> skips;
    for (const Pending &p : s->waiting) {
      wsz.push_back(p.ws);
      tsz.push_back(p.table);
      skips.push_back(p.skips);
    }
    std::vector<int32_t> picked(s->waiting.size());
    int32_t held = 0;
    count = pick_batch(wsz.data(), tsz.data(), skips.data(), (int32_t)wsz.size(), room, kStagingBytes, target,
                       picked.data(), &held, &table, &ws_sum);
    s->st.aged_holds += held;
    if (!count) break;
    {
      // move the picked requests into the slot's batch (in arrival order)
      std::deque<Pending> rest;
      size_t k = 0, q = 0;
      for (auto &p : s->waiting) {
        p.skips = skips[k];
        if (q < (size_t)count && picked[q] == (int32_t)k) {
          slot->batch.push_back(std::move(p));
          ++q;
        } else {
          rest.push_back(std::move(p));
        }
        ++k;
      }
      s->waiting.swap(rest);
    }
    const size_t len = batch_bytes(table, ws_sum, count);
    size_t off = 0;
    take_block(s, len, off);  // fits: len <= the largest free block
    const double t0 = now_s();
    try {
      launch_batch(s, *slot, off);
      s->st.launch_seconds += now_s() - t0;
    } catch (const sqc::Error &e) {
      s->st.launch_seconds += now_s() - t0;
      give_block(s, off, len);
      for (auto &p : slot->batch) {
        s->state[p.ticket] = kFailed;
        s->failure[p.ticket] = e.msg;
      }
      slot->batch.clear();
      continue;
    }
    slot->busy = true;
    slot->off = off;
    slot->len = len;
    for (auto &p : slot->batch) s->state[p.ticket] = kRunning;
    s->st.admitted += count;
    s->st.batches += 1;
    s->st.running += count;
    s->st.max_running = std::max(s->st.max_running, s->st.running);
    s->st.max_batch = std::max(s->st.max_batch, (int32_t)count);
    s->st.workspace_bytes += len;
    s->st.workspace_peak = std::max(s->st.workspace_peak, s->st.workspace_bytes);
  }
  s->st.queued = (int32_t)s->waiting.size();
  return SQC_OK;
}

sqc_status prepare(sqc_server *s, const sqc_request *req, Pending &p) {
  if (req->circuit < 0 || req->circuit >= (int)s->circuits.size())
    return fail(s, SQC_E_ARG, "unknown circuit id");
  const double t0 = now_s();
  try {
    p.prep = sqc::prepare_recursion(s->circuits[req->circuit], req->scope, req->max_bins_M, req->top_r,
                                    req->prec, req->bins_dev, req->bins_prec, req->topr_dev, req->sum_dev);
  } catch (const sqc::Error &e) {
    s->st.plan_seconds += now_s() - t0;
    return fail(s, e.code, e.msg);
  }
  s->st.plan_seconds += now_s() - t0;
  p.ws = round_up(sqc::prepared_workspace(*p.prep));
  p.table = round_up(sqc::prepared_table_bytes(*p.prep));
  return SQC_OK;
}

}  // namespace

extern "C" {

sqc_status sqc_serve_create(int device, int32_t n_slots, void *workspace_dev, size_t workspace_bytes,
                            sqc_server **out) {
  if (!out || !workspace_dev || n_slots < 1 || n_slots > 64) return SQC_E_ARG;
  if (reinterpret_cast<uintptr_t>(workspace_dev) % kAlign || workspace_bytes < kMinWorkspace) return SQC_E_ARG;
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
        hipHostMalloc(&sl.staging, kStagingBytes, hipHostMallocDefault) != hipSuccess ||
        sqc_ctx_create(device, sl.stream, &sl.ctx) != SQC_OK) {
      sqc_serve_destroy(s);
      return SQC_E_DEVICE;
    }
  }
  *out = s;
  return SQC_OK;
}

sqc_status sqc_serve_set_max_batch(sqc_server *s, int32_t max_batch) {
  if (!s || max_batch < 1 || max_batch > kMaxBatch) return fail(s, SQC_E_ARG, "max_batch must be in [1, 128]");
  s->max_batch = max_batch;
  return SQC_OK;
}

sqc_status sqc_serve_destroy(sqc_server *s) {
  if (!s) return SQC_E_ARG;
  for (auto &sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.ctx) sqc_ctx_destroy(sl.ctx);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.staging) (void)hipHostFree(sl.staging);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  delete s;
  return SQC_OK;
}

sqc_status sqc_serve_register(sqc_server *s, const sqc_tensor *attributed, int32_t n_sub,
                              const sqc_cut *cuts, int32_t n_cuts, int32_t *circuit_id) {
  if (!s || !circuit_id) return fail(s, SQC_E_ARG, "invalid argument to sqc_serve_register");
  try {
    s->circuits.push_back(sqc::make_circuit(attributed, n_sub, cuts, n_cuts));
  } catch (const sqc::Error &e) {
    return fail(s, e.code, e.msg);
  }
  *circuit_id = (int32_t)s->circuits.size() - 1;
  return SQC_OK;
}

size_t sqc_serve_footprint(sqc_server *s, const sqc_request *req) {
  if (!s || !req) return 0;
  Pending p;
  if (prepare(s, req, p) != SQC_OK) return 0;
  return p.ws + p.table;
}

sqc_status sqc_serve_submit(sqc_server *s, const sqc_request *req, uint64_t *ticket) {
  if (!s || !req || !ticket) return fail(s, SQC_E_ARG, "invalid argument to sqc_serve_submit");
  Pending p;
  const sqc_status rc = prepare(s, req, p);
  if (rc != SQC_OK) return rc;
  if (p.ws + p.table > s->ws_bytes || p.table > kStagingBytes)
    return fail(s, SQC_E_NOMEM, "the request's footprint exceeds the server workspace");
  if (req->masks_out) {
    const int n = sqc::circuit_n_sub(*s->circuits[req->circuit]);
    std::copy(sqc::prepared_masks(*p.prep), sqc::prepared_masks(*p.prep) + n, req->masks_out);
  }
  p.ticket = s->next_ticket++;
  s->state[p.ticket] = kWaiting;
  *ticket = p.ticket;
  s->waiting.push_back(std::move(p));
  s->st.submitted += 1;
  return pump(s);
}

sqc_status sqc_serve_submit_many(sqc_server *s, const sqc_request *reqs, int32_t n, uint64_t *tickets) {
  if (!s || n < 0 || (n > 0 && (!reqs || !tickets)))
    return fail(s, SQC_E_ARG, "invalid argument to sqc_serve_submit_many");
  std::vector<Pending> ps(n);
  for (int32_t k = 0; k < n; ++k) {
    const sqc_status rc = prepare(s, &reqs[k], ps[k]);
    if (rc != SQC_OK) return rc;
    if (ps[k].ws + ps[k].table > s->ws_bytes || ps[k].table > kStagingBytes)
      return fail(s, SQC_E_NOMEM, "a request's footprint exceeds the server workspace");
  }
  // queue the burst in shares of one batch per slot, advancing after each so
  // that the first batches run while the rest are formed
  const int share = std::max<int>(1, std::min<int>(s->max_batch, (int)((n + s->slots.size() - 1) / s->slots.size())));
  for (int32_t k = 0; k < n; ++k) {
    const sqc_request *req = &reqs[k];
    Pending &p = ps[k];
    if (req->masks_out) {
      const int ns = sqc::circuit_n_sub(*s->circuits[req->circuit]);
      std::copy(sqc::prepared_masks(*p.prep), sqc::prepared_masks(*p.prep) + ns, req->masks_out);
    }
    p.ticket = s->next_ticket++;
    s->state[p.ticket] = kWaiting;
    tickets[k] = p.ticket;
    s->waiting.push_back(std::move(p));
    s->st.submitted += 1;
    if ((k + 1) % share == 0 && k + 1 < n) {
      const sqc_status rc = pump(s, share);
      if (rc != SQC_OK) return rc;
    }
  }
  return pump(s, share);
}

sqc_status sqc_serve_poll(sqc_server *s, uint64_t ticket, int32_t *state) {
  if (!s || !state) return fail(s, SQC_E_ARG, "invalid argument to sqc_serve_poll");
  const sqc_status rc = pump(s);
  if (rc != SQC_OK) return rc;
  auto it = s->state.find(ticket);
  if (it == s->state.end()) return fail(s, SQC_E_ARG, "unknown ticket");
  if (it->second == kFailed) return fail(s, SQC_E_DEVICE, s->failure[ticket]);
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
    // block on the batch that holds the ticket, else on any running batch
    hipEvent_t ev = nullptr;
    for (auto &sl : s->slots) {
      if (!sl.busy) continue;
      bool mine = false;
      for (auto &p : sl.batch) mine = mine || p.ticket == ticket;
      if (mine || !ev) ev = sl.done;
    }
    if (!ev) return fail(s, SQC_E_ARG, "request can never be admitted");
    if (hipEventSynchronize(ev) != hipSuccess) return fail(s, SQC_E_DEVICE, "hipEventSynchronize failed");
  }
}

sqc_status sqc_serve_completed(sqc_server *s, uint64_t *tickets, int32_t cap, int32_t *n) {
  if (!s || !n || cap < 0 || (cap > 0 && !tickets))
    return fail(s, SQC_E_ARG, "invalid argument to sqc_serve_completed");
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

sqc_status sqc_serve_pick_batch(const size_t *workspace_bytes, const size_t *table_bytes, int32_t *skips,
                                int32_t n, size_t room, int32_t max_batch, int32_t *picked, int32_t *n_picked,
                                int32_t *held) {
  if (n < 0 || max_batch < 1 || !n_picked || !held || (n > 0 && (!workspace_bytes || !table_bytes || !skips ||
                                                                   !picked)))
    return SQC_E_ARG;
  size_t table = 0, ws = 0;
  *n_picked = pick_batch(workspace_bytes, table_bytes, skips, n, room, kStagingBytes, max_batch, picked, held,
                         &table, &ws);
  return SQC_OK;
}

}  // extern "C"
