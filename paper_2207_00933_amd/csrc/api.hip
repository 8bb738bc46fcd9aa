// C entry points of libsqc that use the GPU: context and workspace,
// attribution, merging, contraction, one recursion and the search loop.
#include <algorithm>
#include <cstring>
#include <sstream>

#include "batch.hpp"
#include "common.hpp"

#include <climits>
#include <map>
#include <mutex>

namespace sqc {

namespace {

// The one-element tensor of a single-subcircuit contraction: FP64 1.0, then
// FP32 1.0 in the low half of the second word.  Each device holds its own
// copy; its address on a device comes from hipGetSymbolAddress.
__device__ __align__(16) uint64_t unit_const[2] = {0x3FF0000000000000ull, 0x000000003F800000ull};

// Workspace of sqc_recurse_noalloc: a file-scope device array, so that call
// allocates nothing.  Each device holds its own copy from the first load of
// the library until the process ends; every call on a device shares it.
__device__ __align__(256) unsigned char scratch[SQC_NOALLOC_SCRATCH_BYTES];

__global__ void cast_copy(const void *src, int src_f32, void *dst, int dst_f32, int64_t n) {
  for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
       q += int64_t(gridDim.x) * blockDim.x) {
    double v = src_f32 ? (double)static_cast<const float *>(src)[q] : static_cast<const double *>(src)[q];
    if (dst_f32) static_cast<float *>(dst)[q] = (float)v;
    else static_cast<double *>(dst)[q] = v;
  }
}

}  // namespace

}  // namespace sqc

using namespace sqc;

struct sqc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  std::string err;
  void *pinned = nullptr;  // host staging for small device results
  double *unit = nullptr;  // device address of unit_const on this context's device
  // stage timing
  uint32_t timing_mask = 0;
  uint32_t saved_mask = 0;  // timing mask suspended while a graph is recorded
  bool recording = false;
  void *plan_cache = nullptr;  // PlanCache of the recursions planned on this context
  double tol = 1e-6;           // per-bin absolute error the precision selector keeps
  sqc_prec auto_choice = SQC_F64;
  double auto_bound = -1.0;    // (-1: no SQC_AUTO recursion yet)
  struct Mark {
    int stage;
    hipEvent_t a, b;
    double bytes, flops;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  struct Tot {
    double ms = 0, bytes = 0, flops = 0;
    int64_t n = 0;
  } tot[5];
};

namespace {

// Control region at the start of the workspace.
constexpr size_t kCtlBytes = 4096;
// Pinned host buffer of a context: small device results (search) and the
// job tables of a subset query's batches.
constexpr size_t kPinnedBytes = 2 << 20;
constexpr size_t kOffSearchTop = 256;    // SQC_MAX_TOPR x 16 bytes
constexpr size_t kOffSearchSum = 256 + 16 * SQC_MAX_TOPR;

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

struct Bump {
  size_t off = kCtlBytes;
  size_t take(size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  }
};

[[noreturn]] void raise(sqc_status c, const std::string &m) { throw Error{c, m}; }

void check_hip(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    std::ostringstream s;
    s << what << ": " << hipGetErrorString(e);
    raise(SQC_E_DEVICE, s.str());
  }
}

void use_device(sqc_ctx *ctx) { check_hip(hipSetDevice(ctx->device), "hipSetDevice"); }

void after_launch(const char *what) { check_hip(hipGetLastError(), what); }

int elem_bytes(sqc_prec p) { return p == SQC_F64 ? 8 : 4; }

void check_storage_prec(sqc_prec p, const char *name) {
  if (p != SQC_F64 && p != SQC_F32) {
    std::ostringstream s;
    s << name << " must be SQC_F64 or SQC_F32";
    raise(SQC_E_ARG, s.str());
  }
}

void check_path_prec(sqc_prec p) {
  if (p != SQC_F64 && p != SQC_F32 && p != SQC_BF16X3) raise(SQC_E_ARG, "unknown contraction precision");
}

void check_masks(const sqc_masks &m, int d, int i) {
  uint64_t dmask = d == 64 ? ~0ull : ((uint64_t(1) << d) - 1);
  std::ostringstream s;
  if ((m.fixed & m.active) || (m.fixed & m.merged) || (m.active & m.merged)) {
    s << "masks of subcircuit " << i << " overlap";
    raise(SQC_E_SHAPE, s.str());
  }
  if ((m.fixed | m.active | m.merged) != dmask) {
    s << "masks of subcircuit " << i << " do not cover exactly its " << d << " data bits";
    raise(SQC_E_SHAPE, s.str());
  }
  if (m.fixed_val & ~m.fixed) {
    s << "fixed_val of subcircuit " << i << " has bits outside fixed";
    raise(SQC_E_SHAPE, s.str());
  }
}

void check_size(int lbits, int dbits) {
  if (lbits + dbits > 40) raise(SQC_E_UNSUPPORTED, "tensor larger than 2^40 elements");
}

int stage_index(uint32_t bit) {
  for (int q = 0; q < 5; ++q)
    if (bit == (1u << q)) return q;
  return -1;
}

hipEvent_t take_event(sqc_ctx *ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  hipEvent_t e;
  check_hip(hipEventCreate(&e), "hipEventCreate");
  return e;
}

// Bracket one launch of `stage` with events when timing is on for it.
struct StageMark {
  sqc_ctx *ctx;
  uint32_t stage;
  bool on;
  bool external;
  hipEvent_t a{}, b{};
  double bytes, flops;
  // by_launch: the launch itself records a and b (hipExtLaunchKernel), so
  // the span is the kernel's execution without the gap before its dispatch
  StageMark(sqc_ctx *c, uint32_t st, double by, double fl, bool by_launch = false)
      : ctx(c), stage(st), on((c->timing_mask & st) != 0), external(by_launch), bytes(by), flops(fl) {
    if (on) {
      a = take_event(ctx);
      b = take_event(ctx);
      if (!external) check_hip(hipEventRecord(a, ctx->stream), "hipEventRecord");
    }
  }
  hipEvent_t start() const { return on && external ? a : nullptr; }
  hipEvent_t stop() const { return on && external ? b : nullptr; }
  void done() {
    if (!on) return;
    if (!external) check_hip(hipEventRecord(b, ctx->stream), "hipEventRecord");
    ctx->marks.push_back(sqc_ctx::Mark{stage_index(stage), a, b, bytes, flops});
    on = false;
  }
};

void settle_timing(sqc_ctx *ctx) {
  for (auto &m : ctx->marks) {
    check_hip(hipEventSynchronize(m.b), "hipEventSynchronize");
    float ms = 0.f;
    check_hip(hipEventElapsedTime(&ms, m.a, m.b), "hipEventElapsedTime");
    auto &t = ctx->tot[m.stage];
    t.ms += ms;
    t.n += 1;
    t.bytes += m.bytes;
    t.flops += m.flops;
    ctx->pool.push_back(m.a);
    ctx->pool.push_back(m.b);
  }
  ctx->marks.clear();
}

// Device addresses of the library's file-scope device arrays, per device,
// taken once with that device current (each device holds its own copies).
struct DeviceStatics {
  void *unit = nullptr;
  char *scratch = nullptr;  // the device address of `scratch` (never its host-side name)
};
constexpr int kMaxDevices = 64;
std::mutex statics_mu;
DeviceStatics statics[kMaxDevices];

// The current device must be `device`.  Null when a lookup fails.
const DeviceStatics *device_statics(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(statics_mu);
  DeviceStatics &d = statics[device];
  if (!d.unit) {
    void *u = nullptr, *w = nullptr;
    if (hipGetSymbolAddress(&u, HIP_SYMBOL(unit_const)) != hipSuccess || !u) return nullptr;
    if (hipGetSymbolAddress(&w, HIP_SYMBOL(scratch)) != hipSuccess || !w) return nullptr;
    d.unit = u;
    d.scratch = static_cast<char *>(w);
  }
  return &d;
}

// ---------------------------------------------------------------------------
// shared pieces of merge / contract / recurse
// ---------------------------------------------------------------------------

MergeArgs merge_args(const sqc_tensor &at, const sqc_masks &mk, void *out, int out_f32,
                     double *partial) {
  MergeArgs a{};
  a.in = at.data;
  a.out = out;
  a.partial = partial;
  a.in_f32 = at.prec == SQC_F32;
  a.out_f32 = out_f32;
  a.d = at.n_bits;
  a.lbits = 2 * at.n_labels;
  a.in_lbits = a.lbits;
  a.lab_fixed = 0;
  a.lab_keep = (uint64_t(1) << a.lbits) - 1;
  a.abits = __builtin_popcountll(mk.active);
  a.mbits = __builtin_popcountll(mk.merged);
  a.fixed_val = mk.fixed_val;
  a.active = mk.active;
  a.merged = mk.merged;
  auto run_lo = [](uint64_t m) -> int {
    if (!m) return 0;
    const int lo = __builtin_ctzll(m);
    const uint64_t r = m >> lo;
    return (r & (r + 1)) == 0 ? lo : -1;
  };
  a.act_lo = run_lo(mk.active);
  a.mrg_lo = run_lo(mk.merged);
  return a;
}

// Algorithmic bytes of one merge: every attributed entry in scope read once,
// every merged entry written once.
double merge_bytes(const MergeArgs &a) {
  const double in_b = a.in_f32 ? 4 : 8, out_b = a.out_f32 ? 4 : 8;
  return std::ldexp(1.0, a.lbits + a.abits + a.mbits) * in_b + std::ldexp(1.0, a.lbits + a.abits) * out_b;
}

// Enqueue merges (one launch per pass for all of them).
void enqueue_merges(sqc_ctx *ctx, const std::vector<MergeArgs> &jobs) {
  double bytes = 0, reads = 0;
  for (const MergeArgs &a : jobs) {
    bytes += merge_bytes(a);
    reads += std::ldexp(1.0, a.lbits + a.abits + a.mbits);
  }
  StageMark mark(ctx, SQC_STAGE_MERGE, bytes, reads);
  launch_merges(jobs.data(), (int)jobs.size(), ctx->stream);
  after_launch("merge kernel launch");
  mark.done();
}

size_t merge_ws(const sqc_tensor &at, const sqc_masks &mk) {
  int64_t e = merge_partial_elems(__builtin_popcountll(mk.active), 2 * at.n_labels,
                                  __builtin_popcountll(mk.merged));
  return (size_t)e * sizeof(double);
}

// Merged tensors then one partial buffer per merge (the merges run together).
struct MergeLayout {
  std::vector<size_t> merged_off, partial_off;
};
MergeLayout layout_merges(Bump &b, const sqc_tensor *att, const sqc_masks *masks, int n_sub, int eb) {
  MergeLayout L;
  // (an input already in the merged layout is read in place: no buffers)
  for (int i = 0; i < n_sub; ++i)
    L.merged_off.push_back(att[i].layout == SQC_LAYOUT_MERGED
                               ? 0
                               : b.take(((size_t)1 << (2 * att[i].n_labels + __builtin_popcountll(masks[i].active))) * eb));
  for (int i = 0; i < n_sub; ++i) {
    const size_t part = att[i].layout == SQC_LAYOUT_MERGED ? 0 : merge_ws(att[i], masks[i]);
    L.partial_off.push_back(part ? b.take(part) : 0);
  }
  return L;
}

// Inputs already in the merged layout (sqc_attribute_all_merged) serve a
// recursion that keeps every data bit of their subcircuit active, in the
// path's operand precision; returns whether there is any.
bool check_merged_inputs(const sqc_tensor *att, const sqc_masks *masks, int n_sub, sqc_prec prec) {
  bool any = false;
  for (int i = 0; i < n_sub; ++i) {
    if (att[i].layout != SQC_LAYOUT_MERGED) continue;
    any = true;
    const uint64_t all = att[i].n_bits >= 64 ? ~0ull : ((1ull << att[i].n_bits) - 1);
    std::ostringstream m;
    if (masks[i].fixed != 0 || masks[i].merged != 0 || masks[i].active != all) {
      m << "tensor " << i << " is in the merged layout, which serves only a recursion that keeps every data bit "
        << "of its subcircuit active (nothing fixed or merged)";
      raise(SQC_E_ARG, m.str());
    }
    if (att[i].prec != (prec == SQC_F64 ? SQC_F64 : SQC_F32)) {
      m << "tensor " << i << " is in the merged layout and must then be stored in the path's operand precision "
        << "(FP64 for SQC_F64, FP32 for the other paths)";
      raise(SQC_E_ARG, m.str());
    }
  }
  return any;
}

struct Contraction {
  Plan plan;
  int path_f32 = 1;
  bool unit = false;  // single subcircuit: contract with a one-element tensor
};

Contraction plan_for(const Graph &g, const std::vector<int> &bits, sqc_prec prec) {
  Contraction c;
  c.path_f32 = prec != SQC_F64;
  c.plan = make_plan(g, bits, nullptr, c.path_f32 ? 4 : 8);
  c.unit = c.plan.steps.empty();
  return c;
}

GemmArgs step_args(const Contraction &c, size_t si, const std::vector<const void *> &inputs,
                   char *ws, size_t inter_base, void *bins, int bins_f32, const void *unit) {
  GemmArgs g{};
  const Plan &p = c.plan;
  if (c.unit) {
    g.A = inputs[0];
    g.B = unit;
    g.C = bins;
    g.mbits = p.tensors[0].elems() > 1 ? p.out_bits : 0;
    g.nbits = g.kbits = 0;
    if (g.mbits) {
      g.m.nruns = 1;
      g.m.bits[0] = g.mbits;
      g.m.sx[0] = 1;
      g.m.sy[0] = 1;
      g.m.lx[0] = 0;
      g.m.ly[0] = 0;
    }
    g.out_f32 = bins_f32;
    g.final_step = 1;
    return g;
  }
  const Step &st = p.steps[si];
  auto ptr = [&](int t) -> const void * {
    const PTensor &pt = p.tensors[t];
    if (pt.input_sub >= 0) return inputs[pt.input_sub];
    return ws + inter_base + pt.ws_offset;
  };
  g.A = ptr(st.a);
  g.B = ptr(st.b);
  bool last = si + 1 == p.steps.size();
  g.C = last ? bins : (void *)(ws + inter_base + p.tensors[st.c].ws_offset);
  g.mbits = st.mbits;
  g.nbits = st.nbits;
  g.kbits = st.kbits;
  g.m = st.m;
  g.n = st.n;
  g.k = st.k;
  g.out_f32 = last ? bins_f32 : c.path_f32;
  g.final_step = last ? 1 : 0;
  return g;
}

// Workspace needed after the control region: intermediates + statistics.
size_t contraction_ws(const Contraction &c, int top_r, bool stats, int prec) {
  (void)prec;
  size_t b = align256(c.plan.inter_bytes);
  if (stats) {
    GemmArgs dummy{};
    if (c.unit) {
      dummy.mbits = c.plan.out_bits;
    } else {
      const Step &st = c.plan.steps.back();
      dummy.mbits = st.mbits;
      dummy.nbits = st.nbits;
    }
    const size_t nsub = 4 * (size_t)gemm_tiles(dummy);
    b += align256(nsub * sizeof(double));             // sub-tile maxima
    b += align256(3 * kMaxGemmGroups * sizeof(double));  // work-group statistics
    b += align256(kTopRSlots * sizeof(int)) + align256(64);   // slot counts, threshold and sum
    b += 2 * align256(kTopRSlots * (size_t)top_r * 8);       // slot values and indices

  }
  return b;
}

// Algorithmic bytes of one GEMM step: each operand element read once, each
// result written once (a slice's final step instead writes its FP64 running
// sum and compensation, reads them unless it is the first slice, and the last
// slice writes the result as well).
double gemm_bytes(const GemmArgs &g, int path_f32) {
  const double eb = path_f32 ? 4 : 8, ob = g.out_f32 ? 4 : 8;
  const double per_out = g.acc_mode == 1 ? 16 : g.acc_mode == 2 ? 32 : g.acc_mode == 3 ? 16 + ob : ob;
  return (std::ldexp(1.0, g.mbits + g.kbits) + std::ldexp(1.0, g.nbits + g.kbits)) * eb +
         std::ldexp(1.0, g.mbits + g.nbits) * per_out;
}
double gemm_flops(const GemmArgs &g) { return std::ldexp(2.0, g.mbits + g.nbits + g.kbits); }

// Every launch of a contraction (or of a whole recursion): the merges, the
// GEMM steps with their kernel specialisations and work-group counts, and the
// top-R selection after the final step.  Built once, then enqueued either
// directly or as part of a batch of recursions; both give the same results.
struct Launches {
  std::vector<MergeArgs> merges;
  std::vector<GemmArgs> steps;
  std::vector<GemmSpec> specs;
  std::vector<int> groups;
  // dependency level of each step: 0 when it reads only merged inputs, else
  // one more than the steps whose results it reads (steps of one level are
  // independent and write distinct intermediates: they may share a launch)
  std::vector<int> level;
  bool topr = false;
  TopRArgs t{};
  int path_f32 = 1;
};

// One slice of a sliced contraction: how its final step adds into the FP64
// running sums (GemmArgs::acc_mode; 0 = not sliced).
struct SliceAcc {
  int mode = 0;
  double *sum = nullptr, *comp = nullptr;
};

// GEMM steps of a contraction whose intermediates start at ws + base.  With
// `top_dev` non-null, the final step gathers statistics for the top-R stage.
void describe_contraction(Launches &L, const Contraction &c, const std::vector<const void *> &inputs,
                          char *ws, const double *unit2, size_t base, void *bins, int bins_f32,
                          sqc_prec prec, int top_r, void *top_dev, void *sum_dev,
                          const SliceAcc &acc = SliceAcc{}) {
  const void *unit = reinterpret_cast<const char *>(unit2) + (c.path_f32 ? 8 : 0);
  L.path_f32 = c.path_f32;
  size_t inter_base = base;
  size_t stats_base = base + align256(c.plan.inter_bytes);
  size_t nsteps = c.unit ? 1 : c.plan.steps.size();
  std::vector<int> tdepth(c.plan.tensors.size(), 0);  // inputs 0, results 1 + their step's level
  for (size_t si = 0; si < nsteps; ++si) {
    if (c.unit) {
      L.level.push_back(0);
    } else {
      const Step &st = c.plan.steps[si];
      const int lv = std::max(tdepth[st.a], tdepth[st.b]);
      L.level.push_back(lv);
      tdepth[st.c] = lv + 1;
    }
    GemmArgs g = step_args(c, si, inputs, ws, inter_base, bins, bins_f32, unit);
    g.nmajor = gemm_nmajor(g);
    if (g.mbits > 31 || g.nbits > 31 || g.kbits > 31)
      raise(SQC_E_UNSUPPORTED, "a contraction dimension exceeds 2^31");
    const bool last = si + 1 == nsteps;
    Bump bp;
    bp.off = stats_base;
    size_t nsub = 0;
    if (last && top_dev) {
      nsub = 4 * (size_t)gemm_tiles(g);
      g.stats = 1;
      g.blk_max = reinterpret_cast<double *>(ws + bp.take(nsub * sizeof(double)));
      g.wg_stats = reinterpret_cast<double *>(ws + bp.take(3 * kMaxGemmGroups * sizeof(double)));
    }
    if (last && acc.mode) {
      if (acc.mode != 3 && g.stats) raise(SQC_E_ARG, "internal: statistics of a slice that is not the last");
      g.acc_mode = acc.mode;
      g.acc_sum = acc.sum;
      g.acc_comp = acc.comp;
    }
    const GemmSpec base = prepare_gemm(g, prec);
    GemmSpec sp = gemm_default_spec(g, base);
    int groups = gemm_groups(g, sp);
    GemmTuning tu;
    if (gemm_tuned(g, base, tu)) {  // (keyed by the base specialisation)
      sp = base;
      if (tu.narrow && gemm_narrow_ok(g, base)) sp.reg = 4;
      groups = (int)std::min<int64_t>(std::min<int64_t>(tu.groups, gemm_tiles(g)), kMaxGemmGroups);
      g.nmajor = (g.mbits > 6 && g.nbits > 6) ? tu.nmajor : 0;
    }
    L.steps.push_back(g);
    L.specs.push_back(sp);
    L.groups.push_back(groups);
    if (last && top_dev) {
      TopRArgs &t = L.t;
      L.topr = true;
      t.C = bins;
      t.out_f32 = bins_f32;
      t.mbits = g.mbits;
      t.nbits = g.nbits;
      t.m = g.m;
      t.n = g.n;
      t.nsub = (int)nsub;
      t.blk_max = g.blk_max;
      t.wg_stats = g.wg_stats;
      t.ngroups = groups;
      t.nmajor = g.nmajor;
      t.slot_n = reinterpret_cast<int *>(ws + bp.take(kTopRSlots * sizeof(int)));
      char *misc = ws + bp.take(64);
      t.tau_sum = reinterpret_cast<double *>(misc);
      t.slot_val = reinterpret_cast<double *>(ws + bp.take(kTopRSlots * (size_t)top_r * 8));
      t.slot_idx = reinterpret_cast<uint64_t *>(ws + bp.take(kTopRSlots * (size_t)top_r * 8));
      t.top_r = top_r;
      t.gather_groups = topr_gather_groups(t.nsub);
      t.top_out = static_cast<double *>(top_dev);
      t.sum_out = static_cast<double *>(sum_dev);
    }
  }
}

// Enqueue the launches one by one on the context's stream, with no stage
// timing (no events taken): the allocation-free recursion.
void run_untimed(sqc_ctx *ctx, const Launches &L) {
  if (!L.merges.empty()) {
    launch_merges(L.merges.data(), (int)L.merges.size(), ctx->stream);
    after_launch("merge kernel launch");
  }
  for (size_t si = 0; si < L.steps.size(); ++si) {
    launch_gemm_spec(L.steps[si], L.specs[si], L.groups[si], ctx->stream);
    after_launch("contraction kernel launch");
  }
  if (L.topr) {
    launch_topr(L.t, ctx->stream);
    after_launch("top-R kernel launch");
  }
}

// Enqueue the launches one by one on the context's stream (with stage timing).
void run_direct(sqc_ctx *ctx, const Launches &L) {
  if (!L.merges.empty()) enqueue_merges(ctx, L.merges);
  const size_t n = L.steps.size();
  for (size_t si = 0; si < n; ++si) {
    const GemmArgs &g = L.steps[si];
    StageMark mark(ctx, si + 1 == n ? SQC_STAGE_FINAL : SQC_STAGE_CONTRACT, gemm_bytes(g, L.path_f32),
                   gemm_flops(g), true);
    launch_gemm_spec(g, L.specs[si], L.groups[si], ctx->stream, mark.start(), mark.stop());
    after_launch("contraction kernel launch");
    mark.done();
  }
  if (L.topr) {
    StageMark mark(ctx, SQC_STAGE_TOPR, 0.0, 0.0);
    launch_topr(L.t, ctx->stream);
    after_launch("top-R kernel launch");
    mark.done();
  }
}

void enqueue_contraction(sqc_ctx *ctx, const Contraction &c, const std::vector<const void *> &inputs,
                         size_t base, void *bins, int bins_f32, sqc_prec prec, int top_r,
                         void *top_dev, void *sum_dev) {
  Launches L;
  describe_contraction(L, c, inputs, ctx->ws, ctx->unit, base, bins, bins_f32, prec, top_r, top_dev,
                       sum_dev);
  run_direct(ctx, L);
}

void need_ws(sqc_ctx *ctx, size_t bytes) {
  if (!ctx->ws) raise(SQC_E_NOMEM, "no workspace: call sqc_ctx_set_workspace first");
  if (bytes > ctx->ws_bytes) {
    std::ostringstream s;
    s << "workspace of " << ctx->ws_bytes << " bytes is smaller than the " << bytes
      << " bytes this call needs";
    raise(SQC_E_NOMEM, s.str());
  }
}

std::vector<int> degrees_match(const Graph &g, const sqc_tensor *t, int layout) {
  std::vector<int> bits(g.n_sub);
  for (int i = 0; i < g.n_sub; ++i) {
    std::ostringstream s;
    if (!t[i].data) {
      s << "tensor " << i << " has no data";
      raise(SQC_E_ARG, s.str());
    }
    const bool ok = layout >= 0 ? t[i].layout == layout
                                : (t[i].layout == SQC_LAYOUT_ATTRIBUTED || t[i].layout == SQC_LAYOUT_MERGED);
    if (!ok) {
      s << "tensor " << i << " has the wrong layout";
      raise(SQC_E_SHAPE, s.str());
    }
    if (t[i].n_labels != (int)g.subs[i].inc.size()) {
      s << "tensor " << i << " has " << t[i].n_labels << " labels but subcircuit " << i
        << " has degree " << g.subs[i].inc.size();
      raise(SQC_E_SHAPE, s.str());
    }
    if (t[i].n_bits < 0 || t[i].n_bits > SQC_MAX_DATA_BITS) {
      s << "tensor " << i << " bit count out of range";
      raise(SQC_E_SHAPE, s.str());
    }
    check_storage_prec(t[i].prec, "tensor precision");
    check_size(2 * t[i].n_labels, t[i].n_bits);
    bits[i] = t[i].n_bits;
  }
  return bits;
}

struct RecursePlan {
  std::vector<sqc_masks> masks;
  std::vector<int> abits;
  Contraction con;
  MergeLayout ml;
  size_t con_base = 0, total = 0;
};

// Contraction plans of one compute graph by active-bit counts and precision
// (a recursion's plan depends on nothing else), for callers that plan many
// recursions of the same graph.
struct PlanCache {
  std::mutex mu;
  std::map<std::vector<int>, Contraction> plans;  // key: topology, active bits, precision
};

PlanCache *ctx_plans(sqc_ctx *ctx) {
  if (!ctx->plan_cache) ctx->plan_cache = new PlanCache();
  return static_cast<PlanCache *>(ctx->plan_cache);
}

RecursePlan plan_recursion(const Graph &g, const sqc_tensor *att, const sqc_masks *scope,
                           uint64_t M, int top_r, sqc_prec prec, PlanCache *cache = nullptr) {
  RecursePlan rp;
  std::vector<int> d(g.n_sub);
  for (int i = 0; i < g.n_sub; ++i) d[i] = att[i].n_bits;
  rp.masks.resize(g.n_sub);
  assign_bins(g.n_sub, d.data(), scope, M, rp.masks.data());
  rp.abits.resize(g.n_sub);
  for (int i = 0; i < g.n_sub; ++i) rp.abits[i] = __builtin_popcountll(rp.masks[i].active);
  if (cache) {
    std::vector<int> key{g.n_sub, (int)prec};
    for (const auto &c : g.cuts) {
      key.push_back(c.up_sub);
      key.push_back(c.down_sub);
    }
    key.insert(key.end(), rp.abits.begin(), rp.abits.end());
    std::lock_guard<std::mutex> lk(cache->mu);
    auto it = cache->plans.find(key);
    if (it == cache->plans.end()) {
      if (cache->plans.size() >= 512) cache->plans.clear();  // bounded
      it = cache->plans.emplace(key, plan_for(g, rp.abits, prec)).first;
    }
    rp.con = it->second;
  } else {
    rp.con = plan_for(g, rp.abits, prec);
  }
  Bump b;
  rp.ml = layout_merges(b, att, rp.masks.data(), g.n_sub, prec == SQC_F64 ? 8 : 4);
  rp.con_base = b.off;
  rp.total = b.off + contraction_ws(rp.con, top_r, true, prec);
  return rp;
}

// The plan of a recursion with the given masks (the bins of each subcircuit
// fixed by them rather than derived from a scope and M).
RecursePlan plan_from_masks(const Graph &g, const sqc_tensor *att, const sqc_masks *masks, int top_r,
                            sqc_prec prec) {
  RecursePlan rp;
  rp.masks.assign(masks, masks + g.n_sub);
  rp.abits.resize(g.n_sub);
  for (int i = 0; i < g.n_sub; ++i) rp.abits[i] = __builtin_popcountll(masks[i].active);
  rp.con = plan_for(g, rp.abits, prec);
  Bump b;
  rp.ml = layout_merges(b, att, rp.masks.data(), g.n_sub, prec == SQC_F64 ? 8 : 4);
  rp.con_base = b.off;
  rp.total = b.off + contraction_ws(rp.con, top_r, true, prec);
  return rp;
}

// The launches of one recursion whose workspace starts at ws.
Launches describe_recursion(const RecursePlan &rp, const sqc_tensor *att, sqc_prec prec, char *ws,
                            const double *unit2, void *bins, sqc_prec bins_prec, int top_r,
                            void *top_dev, void *sum_dev) {
  const int n_sub = (int)rp.masks.size();
  std::vector<const void *> inputs(n_sub);
  const int path_f32 = prec != SQC_F64;
  Launches L;
  for (int i = 0; i < n_sub; ++i) {
    if (att[i].layout == SQC_LAYOUT_MERGED) {  // (checked by check_merged_inputs)
      inputs[i] = att[i].data;
      continue;
    }
    void *out = ws + rp.ml.merged_off[i];
    L.merges.push_back(merge_args(att[i], rp.masks[i], out, path_f32,
                                  reinterpret_cast<double *>(ws + rp.ml.partial_off[i])));
    inputs[i] = out;
  }
  describe_contraction(L, rp.con, inputs, ws, unit2, rp.con_base, bins, bins_prec == SQC_F32, prec,
                       top_r, top_dev, sum_dev);
  return L;
}

// ---- memory-driven first-level slicing of a recursion (Sec. 6.3) ----

// A recursion whose contraction is split over the label values of some cuts:
// each slice merges, straight from the attributed tensors, only the label rows
// it keeps (so the whole merged tensors never exist), contracts the network
// without the sliced cuts, and its final step adds the slice's bins into FP64
// running sums; the last slice writes sum + compensation and the statistics
// for top-R.  Subcircuits with no sliced cut are merged once.
struct SlicedRecursion {
  RecursePlan rp;            // masks and active bits
  std::vector<int> sliced;   // cut ids; slice digit j belongs to sliced[j]
  Contraction con;           // the network without the sliced cuts
  // per subcircuit: (digit position in its sigma, index in `sliced`) of each
  // incident sliced cut, ascending digit position
  std::vector<std::vector<std::pair<int, int>>> fixed;
  std::vector<size_t> merged_off, partial_off;
  size_t sum_off = 0, comp_off = 0, con_base = 0, total = 0;
};

SlicedRecursion layout_sliced(const Graph &g, const sqc_tensor *att, const RecursePlan &rp,
                              const std::vector<int> &sliced, sqc_prec prec, int top_r) {
  SlicedRecursion sr;
  sr.rp = rp;
  sr.sliced = sliced;
  std::vector<int> which(g.cuts.size(), -1);
  for (size_t q = 0; q < sliced.size(); ++q) which[sliced[q]] = (int)q;
  std::vector<sqc_cut> rest;
  for (size_t k = 0; k < g.cuts.size(); ++k)
    if (which[k] < 0) rest.push_back(g.cuts[k]);
  const Graph g2 = build_topology(g.n_sub, rest.data(), (int32_t)rest.size());
  sr.con = plan_for(g2, rp.abits, prec);
  const size_t eb = prec == SQC_F64 ? 8 : 4;
  Bump b;
  sr.fixed.resize(g.n_sub);
  for (int i = 0; i < g.n_sub; ++i) {
    const std::vector<int> &inc = g.subs[i].inc;
    for (size_t j = 0; j < inc.size(); ++j)
      if (which[inc[j]] >= 0) sr.fixed[i].push_back({(int)j, which[inc[j]]});
    const int kept = (int)inc.size() - (int)sr.fixed[i].size();
    sr.merged_off.push_back(b.take((size_t(1) << (2 * kept + rp.abits[i])) * eb));
  }
  for (int i = 0; i < g.n_sub; ++i) {
    const int kept = (int)g.subs[i].inc.size() - (int)sr.fixed[i].size();
    const int64_t pe = merge_partial_elems(rp.abits[i], 2 * kept, __builtin_popcountll(rp.masks[i].merged));
    sr.partial_off.push_back(pe ? b.take((size_t)pe * sizeof(double)) : 0);
  }
  int abits = 0;
  for (int a : rp.abits) abits += a;
  sr.sum_off = b.take((size_t(1) << abits) * sizeof(double));
  sr.comp_off = b.take((size_t(1) << abits) * sizeof(double));
  sr.con_base = b.off;
  sr.total = b.off + contraction_ws(sr.con, top_r, true, prec);
  return sr;
}

// The cuts a recursion slices to fit `budget` bytes of workspace: none when
// the unsliced plan fits, else, as Sec. 6.3 does for memory, repeatedly the
// cut whose removal shrinks the merged inputs' total size the most until the
// sliced layout fits.  Ties go to the higher cut id: label digits follow the
// incident cuts in id order, so the higher digits are sliced first and each
// slice's label rows stay long contiguous runs of the attributed tensors
// (labels are their fastest index).  SQC_E_NOMEM when SQC_MAX_SLICED cuts
// do not suffice.
std::vector<int> choose_slices(const Graph &g, const sqc_tensor *att, const RecursePlan &rp, sqc_prec prec,
                               int top_r, size_t budget, size_t *need) {
  std::vector<int> sliced;
  *need = rp.total;
  if (rp.total <= budget) return sliced;
  std::vector<std::vector<int>> labs(g.n_sub);
  for (int i = 0; i < g.n_sub; ++i) labs[i] = g.subs[i].inc;
  std::vector<bool> gone(g.cuts.size(), false);
  auto floats = [&](int drop) {
    double t = 0;
    for (int i = 0; i < g.n_sub; ++i) {
      int c = 0;
      for (int k : labs[i]) c += !gone[k] && k != drop;
      t += std::ldexp(1.0, 2 * c + rp.abits[i]);
    }
    return t;
  };
  while (sliced.size() < (size_t)SQC_MAX_SLICED) {
    int best = -1;
    double best_t = 0;
    for (size_t k = 0; k < g.cuts.size(); ++k) {
      if (gone[k]) continue;
      const double t = floats((int)k);
      if (best < 0 || t <= best_t) {  // (k ascending: the higher id wins a tie)
        best = (int)k;
        best_t = t;
      }
    }
    if (best < 0) break;
    gone[best] = true;
    sliced.push_back(best);
    const size_t n = layout_sliced(g, att, rp, sliced, prec, top_r).total;
    *need = n;
    if (n <= budget) return sliced;
  }
  std::ostringstream m;
  m << "the recursion needs " << rp.total << " bytes of workspace unsliced and " << *need << " with "
    << sliced.size() << " sliced cut(s), above the " << budget << " bytes available";
  raise(SQC_E_NOMEM, m.str());
}

// Enqueue a sliced recursion: 4^s slices, each its merges and contraction.
void enqueue_sliced_recursion(sqc_ctx *ctx, const SlicedRecursion &sr, const sqc_tensor *att, sqc_prec prec,
                              void *bins, sqc_prec bins_prec, int top_r, void *top_dev, void *sum_dev) {
  const int n_sub = (int)sr.rp.masks.size();
  const int path_f32 = prec != SQC_F64;
  const int64_t nslices = int64_t(1) << (2 * sr.sliced.size());
  std::vector<const void *> inputs(n_sub);
  for (int i = 0; i < n_sub; ++i) inputs[i] = ctx->ws + sr.merged_off[i];
  for (int64_t q = 0; q < nslices; ++q) {
    Launches L;
    for (int i = 0; i < n_sub; ++i) {
      const auto &fx = sr.fixed[i];
      if (fx.empty() && q > 0) continue;  // merged once
      MergeArgs a = merge_args(att[i], sr.rp.masks[i], ctx->ws + sr.merged_off[i], path_f32,
                               reinterpret_cast<double *>(ctx->ws + sr.partial_off[i]));
      if (!fx.empty()) {
        // output label s' keeps the unsliced digits in order; the sliced
        // digits take this slice's values
        const int deg = att[i].n_labels;
        a.lbits = 2 * (deg - (int)fx.size());
        a.lab_fixed = 0;
        a.lab_keep = (uint64_t(1) << (2 * deg)) - 1;
        for (const auto &f : fx) {
          a.lab_fixed |= (uint64_t)((q >> (2 * f.second)) & 3) << (2 * f.first);
          a.lab_keep &= ~(uint64_t(3) << (2 * f.first));
        }
      }
      L.merges.push_back(a);
    }
    SliceAcc acc;
    acc.mode = q == 0 ? 1 : q == nslices - 1 ? 3 : 2;
    acc.sum = reinterpret_cast<double *>(ctx->ws + sr.sum_off);
    acc.comp = reinterpret_cast<double *>(ctx->ws + sr.comp_off);
    const bool last = q == nslices - 1;
    describe_contraction(L, sr.con, inputs, ctx->ws, ctx->unit, sr.con_base, bins, bins_prec == SQC_F32, prec,
                         top_r, last ? top_dev : nullptr, last ? sum_dev : nullptr, acc);
    run_direct(ctx, L);
  }
}

// ---- precision selection: the certified bound B >= max_x sum_sigma prod_i
// |T_i[sigma, x_i]| of a recursion ----

// Relative factors of the a-priori error bound per contraction path, and the
// rounding of FP32-stored bins.
constexpr double kRelBF16x3 = 0x1p-13, kRelF32 = 0x1p-20, kRelStoreF32 = 0x1p-24;

// Workspace of the selector for this scope (FP32 merged tensors, row maxima,
// the label-only FP64 contraction and its result).
size_t selector_ws(const Graph &g, const sqc_tensor *att, const sqc_masks *scope, uint64_t M, PlanCache *cache,
                   RecursePlan *rp_out = nullptr, Contraction *c0_out = nullptr, size_t *m_off = nullptr,
                   size_t *res_off = nullptr, size_t *c0_base = nullptr) {
  RecursePlan rp = plan_recursion(g, att, scope, M, 1, SQC_F32, cache);
  Bump b;
  b.off = rp.con_base;  // after the merged tensors and their partial sums
  std::vector<size_t> mo(g.n_sub);
  for (int i = 0; i < g.n_sub; ++i) mo[i] = b.take((size_t(1) << (2 * att[i].n_labels)) * sizeof(double));
  const size_t ro = b.take(sizeof(double));
  Contraction c0 = plan_for(g, std::vector<int>(g.n_sub, 0), SQC_F64);
  const size_t base = b.off;
  const size_t total = base + contraction_ws(c0, 1, false, SQC_F64);
  if (rp_out) *rp_out = rp;
  if (c0_out) *c0_out = c0;
  if (m_off) std::copy(mo.begin(), mo.end(), m_off);
  if (res_off) *res_off = ro;
  if (c0_base) *c0_base = base;
  return total;
}

sqc_prec select_precision(sqc_ctx *ctx, const Graph &g, const sqc_tensor *att, const sqc_masks *scope, uint64_t M,
                          double *bound) {
  if (ctx->recording) raise(SQC_E_ARG, "precision selection waits for the device and cannot be recorded");
  RecursePlan rp;
  Contraction c0;
  std::vector<size_t> mo(g.n_sub);
  size_t ro = 0, base = 0;
  const size_t need = selector_ws(g, att, scope, M, ctx_plans(ctx), &rp, &c0, mo.data(), &ro, &base);
  need_ws(ctx, need);
  use_device(ctx);
  std::vector<MergeArgs> merges(g.n_sub);
  std::vector<const void *> inputs(g.n_sub);
  for (int i = 0; i < g.n_sub; ++i) {
    void *out = ctx->ws + rp.ml.merged_off[i];
    merges[i] = merge_args(att[i], rp.masks[i], out, 1, reinterpret_cast<double *>(ctx->ws + rp.ml.partial_off[i]));
  }
  enqueue_merges(ctx, merges);
  for (int i = 0; i < g.n_sub; ++i) {
    const int64_t rows = int64_t(1) << (2 * att[i].n_labels);
    const int64_t cols = int64_t(1) << rp.abits[i];
    double *m = reinterpret_cast<double *>(ctx->ws + mo[i]);
    launch_row_absmax(ctx->ws + rp.ml.merged_off[i], 1, m, rows, cols, ctx->stream);
    after_launch("row maximum kernel launch");
    inputs[i] = m;
  }
  double *res = reinterpret_cast<double *>(ctx->ws + ro);
  enqueue_contraction(ctx, c0, inputs, base, res, 0, SQC_F64, 0, nullptr, nullptr);
  check_hip(hipMemcpyAsync(ctx->pinned, res, sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
            "hipMemcpyAsync of the bound");
  check_hip(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  const double B = *static_cast<const double *>(ctx->pinned);
  if (bound) *bound = B;
  if (!std::isfinite(B)) {
    std::ostringstream m;
    m << "precision selection: the merged inputs hold a non-finite value (bound " << B << ")";
    raise(SQC_E_NUMERIC, m.str());
  }
  if ((kRelBF16x3 + kRelStoreF32) * B <= ctx->tol) return SQC_BF16X3;
  if ((kRelF32 + kRelStoreF32) * B <= ctx->tol) return SQC_F32;
  return SQC_F64;
}

void enqueue_recursion(sqc_ctx *ctx, const RecursePlan &rp, const sqc_tensor *att, sqc_prec prec,
                       void *bins, sqc_prec bins_prec, int top_r, void *top_dev, void *sum_dev) {
  run_direct(ctx, describe_recursion(rp, att, prec, ctx->ws, ctx->unit, bins, bins_prec, top_r, top_dev,
                                     sum_dev));
}

}  // namespace

// ---------------------------------------------------------------------------
// requests planned ahead and batched launches (used by the serving engine)
// ---------------------------------------------------------------------------

namespace sqc {

// The launches of one recursion shape, with every pointer relative: a
// workspace offset (>= kCtlBytes), an offset into the device's unit constant
// (< kCtlBytes, GEMM operands only), or null for the request's outputs, and
// the fixed bits' values zero.  A request of that shape copies them and
// fills in its workspace, outputs and fixed values (relocate()).
struct RecursionTemplate {
  RecursePlan rp;
  Launches L;
};

struct CircuitTopo {
  Graph g;
  std::vector<sqc_tensor> att;
  mutable PlanCache plans;
  // templates by shape: precision, bins precision, top_r, the launch
  // tuning's version and every subcircuit's (fixed, active, merged) masks
  mutable std::mutex tmu;
  mutable std::map<std::vector<uint64_t>, std::shared_ptr<const RecursionTemplate>> templates;
};

struct PreparedRecursion {
  std::shared_ptr<const CircuitTopo> c;
  std::shared_ptr<const RecursionTemplate> t;
  std::vector<sqc_masks> masks;
  sqc_prec prec, bins_prec;
  void *bins, *top, *sum;
  int top_r;
};

void PreparedDeleter::operator()(PreparedRecursion *p) const { delete p; }

std::shared_ptr<const CircuitTopo> make_circuit(const sqc_tensor *att, int n_sub, const sqc_cut *cuts,
                                                int n_cuts) {
  auto c = std::make_shared<CircuitTopo>();
  c->g = build_topology(n_sub, cuts, n_cuts);
  if (!att) raise(SQC_E_ARG, "NULL argument");
  degrees_match(c->g, att, SQC_LAYOUT_ATTRIBUTED);
  c->att.assign(att, att + n_sub);
  return c;
}

int circuit_n_sub(const CircuitTopo &c) { return c.g.n_sub; }

PreparedPtr prepare_recursion(std::shared_ptr<const CircuitTopo> c, const sqc_masks *scope, uint64_t M,
                              int top_r, sqc_prec prec, void *bins, sqc_prec bins_prec, void *top_dev,
                              void *sum_dev) {
  if (!bins || !top_dev || !sum_dev) raise(SQC_E_ARG, "request output buffers must be set");
  check_path_prec(prec);
  check_storage_prec(bins_prec, "bins_prec");
  if (top_r < 1 || top_r > SQC_MAX_TOPR) raise(SQC_E_ARG, "top_r must be in [1, 64]");
  PreparedPtr p(new PreparedRecursion());
  const int n_sub = c->g.n_sub;
  std::vector<int> d(n_sub);
  for (int i = 0; i < n_sub; ++i) d[i] = c->att[i].n_bits;
  p->masks.resize(n_sub);
  assign_bins(n_sub, d.data(), scope, M, p->masks.data());
  std::vector<uint64_t> key{(uint64_t)prec, (uint64_t)bins_prec, (uint64_t)top_r, gemm_tune_version()};
  for (const sqc_masks &m : p->masks) {
    key.push_back(m.fixed);
    key.push_back(m.active);
    key.push_back(m.merged);
  }
  {
    std::lock_guard<std::mutex> lk(c->tmu);
    auto it = c->templates.find(key);
    if (it != c->templates.end()) p->t = it->second;
  }
  if (!p->t) {
    auto t = std::make_shared<RecursionTemplate>();
    t->rp = plan_recursion(c->g, c->att.data(), scope, M, top_r, prec, &c->plans);
    for (sqc_masks &m : t->rp.masks) m.fixed_val = 0;
    // outputs: null bins; top-R and sum marked by their own non-null values
    // (describe_contraction adds the top-R stage only for a non-null top)
    t->L = describe_recursion(t->rp, c->att.data(), prec, nullptr, nullptr, nullptr, bins_prec, top_r,
                              reinterpret_cast<void *>(uintptr_t(16)), reinterpret_cast<void *>(uintptr_t(32)));
    for (MergeArgs &a : t->L.merges) merge_shape(a);  // (depends on the shape only)
    std::lock_guard<std::mutex> lk(c->tmu);
    if (c->templates.size() >= 4096) c->templates.clear();  // bounded
    p->t = c->templates.emplace(key, std::move(t)).first->second;
  }
  p->c = std::move(c);
  p->prec = prec;
  p->bins_prec = bins_prec;
  p->bins = bins;
  p->top = top_dev;
  p->sum = sum_dev;
  p->top_r = top_r;
  return p;
}

size_t prepared_workspace(const PreparedRecursion &p) { return align256(p.t->rp.total); }

size_t prepared_table_bytes(const PreparedRecursion &p) {
  const size_t n_sub = p.t->rp.masks.size();
  const size_t steps = p.t->rp.con.unit ? 1 : p.t->rp.con.plan.steps.size();
  return n_sub * sizeof(MergeArgs) + steps * sizeof(GemmArgs) + sizeof(TopRArgs) +
         sizeof(int) * (3 * n_sub + 2 * steps + 8) + 256 * (2 * steps + 8);
}

const sqc_masks *prepared_masks(const PreparedRecursion &p) { return p.masks.data(); }

namespace {

// A template record made the request's: workspace offsets become addresses
// at ws, offsets below kCtlBytes addresses in the device's unit constant,
// output markers the request's outputs, and the fixed bits their values.
void relocate_merge(MergeArgs &a, const PreparedRecursion &p, char *ws, size_t k) {
  a.out = ws + reinterpret_cast<uintptr_t>(a.out);
  a.partial = reinterpret_cast<double *>(ws + reinterpret_cast<uintptr_t>(a.partial));
  a.fixed_val = p.masks[k].fixed_val;
}

void relocate_gemm(GemmArgs &g, const PreparedRecursion &p, char *ws, const char *unit, bool last) {
  auto operand = [&](const void *rel) -> const void * {
    const uintptr_t v = reinterpret_cast<uintptr_t>(rel);
    return v < kCtlBytes ? static_cast<const void *>(unit + v) : static_cast<const void *>(ws + v);
  };
  g.A = operand(g.A);
  g.B = operand(g.B);
  g.C = last ? p.bins : static_cast<void *>(ws + reinterpret_cast<uintptr_t>(g.C));
  if (g.stats) {
    g.blk_max = reinterpret_cast<double *>(ws + reinterpret_cast<uintptr_t>(g.blk_max));
    g.wg_stats = reinterpret_cast<double *>(ws + reinterpret_cast<uintptr_t>(g.wg_stats));
  }
}

void relocate_topr(TopRArgs &t, const PreparedRecursion &p, char *ws) {
  auto at = [ws](const void *rel) -> char * { return ws + reinterpret_cast<uintptr_t>(rel); };
  t.C = p.bins;
  t.blk_max = reinterpret_cast<const double *>(at(t.blk_max));
  t.wg_stats = reinterpret_cast<const double *>(at(t.wg_stats));
  t.tau_sum = reinterpret_cast<double *>(at(t.tau_sum));
  t.slot_n = reinterpret_cast<int *>(at(t.slot_n));
  t.slot_val = reinterpret_cast<double *>(at(t.slot_val));
  t.slot_idx = reinterpret_cast<uint64_t *>(at(t.slot_idx));
  t.top_out = static_cast<double *>(p.top);
  t.sum_out = static_cast<double *>(p.sum);
}

// The request's launches: its shape's template made the request's.
Launches describe_prepared(sqc_ctx *ctx, const PreparedRecursion &p, char *ws) {
  Launches L = p.t->L;
  for (size_t i = 0; i < L.merges.size(); ++i) relocate_merge(L.merges[i], p, ws, i);
  const char *unit = reinterpret_cast<const char *>(ctx->unit);
  for (size_t si = 0; si < L.steps.size(); ++si) relocate_gemm(L.steps[si], p, ws, unit, si + 1 == L.steps.size());
  if (L.topr) relocate_topr(L.t, p, ws);
  return L;
}

// Host image of a batch's job tables (arrays 256-byte aligned).
struct TableImage {
  char *host;
  size_t cap, off = 0;
  // room for n records of T, written in place by the caller
  template <class T>
  size_t reserve(size_t n) {
    const size_t at = align256(off);
    const size_t bytes = n * sizeof(T);
    if (at + bytes > cap) raise(SQC_E_NOMEM, "batch job table exceeds its staging buffer");
    off = at + bytes;
    return at;
  }
  template <class T>
  T *rec(size_t at) {
    return reinterpret_cast<T *>(host + at);
  }
  template <class T>
  size_t put(const T *v, size_t n) {
    const size_t at = reserve<T>(n);
    std::memcpy(host + at, v, n * sizeof(T));
    return at;
  }
};

// One grouped launch: kind 0 merge pass `code`, 1 GEMM of spec `spec`, 2 top-R.
struct GroupedDesc {
  int kind, code;
  GemmSpec spec;
  size_t jobs, start;
  int n, total;
};

// Work-group prefix of jobs in one pass; fails when it does not fit a grid.
std::vector<int> block_prefix(const std::vector<int64_t> &blocks) {
  std::vector<int> start(blocks.size() + 1, 0);
  int64_t acc = 0;
  for (size_t k = 0; k < blocks.size(); ++k) {
    start[k] = (int)acc;
    acc += blocks[k];
    if (acc > INT_MAX) raise(SQC_E_UNSUPPORTED, "a batched launch exceeds 2^31 work-groups");
  }
  start[blocks.size()] = (int)acc;
  return start;
}

}  // namespace

void enqueue_prepared(sqc_ctx *ctx, const PreparedRecursion &p, char *ws) {
  use_device(ctx);
  run_direct(ctx, describe_prepared(ctx, p, ws));
}

void enqueue_batch(sqc_ctx *ctx, PreparedRecursion *const *p, int n, char *const *ws, char *table_dev,
                   size_t table_bytes, void *staging, size_t staging_bytes) {
  use_device(ctx);
  // every record goes from the request's template straight to its place in
  // the staging image, made the request's there (one copy per record)
  TableImage tab{static_cast<char *>(staging), std::min(table_bytes, staging_bytes)};
  std::vector<GroupedDesc> descs;
  const char *unit = reinterpret_cast<const char *>(ctx->unit);
  auto T = [&](int i) -> const Launches & { return p[i]->t->L; };

  // merges: every subcircuit of every request, one launch per pass (shapes
  // were set when the template was made)
  struct Ref {
    int i, k;
    int64_t blocks;
  };
  std::vector<Ref> tiles, rows;
  for (int i = 0; i < n; ++i)
    for (size_t k = 0; k < T(i).merges.size(); ++k) {
      const MergeArgs &a = T(i).merges[k];
      const int64_t b0 = merge_pass_blocks(a, 0);
      if (b0) tiles.push_back(Ref{i, (int)k, b0});
      else rows.push_back(Ref{i, (int)k, merge_pass_blocks(a, 1)});
    }
  // larger jobs first: their work-groups start first and the launch ends sooner
  auto larger = [](const Ref &a, const Ref &b) { return a.blocks > b.blocks; };
  std::stable_sort(tiles.begin(), tiles.end(), larger);
  std::stable_sort(rows.begin(), rows.end(), larger);
  auto put_merges = [&](const std::vector<Ref> &refs) {
    const size_t at = tab.reserve<MergeArgs>(refs.size());
    MergeArgs *d = tab.rec<MergeArgs>(at);
    for (size_t q = 0; q < refs.size(); ++q) {
      d[q] = T(refs[q].i).merges[refs[q].k];
      relocate_merge(d[q], *p[refs[q].i], ws[refs[q].i], refs[q].k);
    }
    return at;
  };
  auto merge_pass = [&](const std::vector<Ref> &refs, int pass, size_t at) {
    const MergeArgs *d = tab.rec<MergeArgs>(at);
    std::vector<int64_t> nb(refs.size());
    for (size_t q = 0; q < refs.size(); ++q) nb[q] = merge_pass_blocks(d[q], pass);
    const std::vector<int> start = block_prefix(nb);
    descs.push_back(GroupedDesc{0, pass, GemmSpec{}, at, tab.put(start.data(), start.size()),
                                (int)refs.size(), start.back()});
  };
  if (!tiles.empty()) merge_pass(tiles, 0, put_merges(tiles));
  if (!rows.empty()) {
    const size_t at = put_merges(rows);
    merge_pass(rows, 1, at);
    merge_pass(rows, 2, at);
  }

  // GEMM steps level by level (a step reads only results of lower levels),
  // one launch per kernel specialisation within a level: independent steps
  // of one request share it as well as those of different requests
  int levels = 0;
  for (int i = 0; i < n; ++i)
    for (int lv : T(i).level) levels = std::max(levels, lv + 1);
  for (int lv = 0; lv < levels; ++lv) {
    std::map<int, std::vector<Ref>> by_spec;  // spec id -> (request, step, work-groups)
    for (int i = 0; i < n; ++i) {
      const Launches &L = T(i);
      for (size_t si = 0; si < L.steps.size(); ++si)
        if (L.level[si] == lv) by_spec[gemm_spec_id(L.specs[si])].push_back(Ref{i, (int)si, L.groups[si]});
    }
    for (auto &kv : by_spec) {
      std::vector<Ref> &refs = kv.second;
      std::stable_sort(refs.begin(), refs.end(), larger);
      const size_t at = tab.reserve<GemmArgs>(refs.size());
      GemmArgs *d = tab.rec<GemmArgs>(at);
      std::vector<int64_t> nb(refs.size());
      for (size_t q = 0; q < refs.size(); ++q) {
        const Launches &L = T(refs[q].i);
        d[q] = L.steps[refs[q].k];
        relocate_gemm(d[q], *p[refs[q].i], ws[refs[q].i], unit, refs[q].k + 1 == (int)L.steps.size());
        nb[q] = refs[q].blocks;
      }
      const std::vector<int> start = block_prefix(nb);
      const Ref &f = refs[0];
      descs.push_back(GroupedDesc{1, kv.first, T(f.i).specs[f.k], at, tab.put(start.data(), start.size()),
                                  (int)refs.size(), start.back()});
    }
  }

  // top-R of every request, one launch per bins precision
  for (int outf = 0; outf < 2; ++outf) {
    std::vector<Ref> refs;
    for (int i = 0; i < n; ++i)
      if (T(i).topr && T(i).t.out_f32 == outf) refs.push_back(Ref{i, 0, T(i).t.nsub});
    if (refs.empty()) continue;
    std::stable_sort(refs.begin(), refs.end(), larger);
    const size_t at = tab.reserve<TopRArgs>(refs.size());
    TopRArgs *d = tab.rec<TopRArgs>(at);
    std::vector<int64_t> nb(refs.size());
    for (size_t q = 0; q < refs.size(); ++q) {
      d[q] = T(refs[q].i).t;
      relocate_topr(d[q], *p[refs[q].i], ws[refs[q].i]);
      nb[q] = d[q].gather_groups;
    }
    const std::vector<int> start = block_prefix(nb);
    descs.push_back(GroupedDesc{2, outf, GemmSpec{}, at, tab.put(start.data(), start.size()), (int)refs.size(),
                                start.back()});
  }

  check_hip(hipMemcpyAsync(table_dev, staging, tab.off, hipMemcpyHostToDevice, ctx->stream),
            "hipMemcpyAsync of the batch job table");
  for (const GroupedDesc &d : descs) {
    if (d.kind == 0)
      launch_merge_grouped(d.code, reinterpret_cast<const MergeArgs *>(table_dev + d.jobs),
                           reinterpret_cast<const int *>(table_dev + d.start), d.n, d.total, ctx->stream);
    else if (d.kind == 1)
      launch_gemm_grouped(d.spec, reinterpret_cast<const GemmArgs *>(table_dev + d.jobs),
                          reinterpret_cast<const int *>(table_dev + d.start), d.n, d.total, ctx->stream);
    else
      launch_topr_grouped(reinterpret_cast<const TopRArgs *>(table_dev + d.jobs),
                          reinterpret_cast<const int *>(table_dev + d.start), d.n, d.total, d.code, ctx->stream);
    after_launch("batched kernel launch");
  }
}

}  // namespace sqc

#define SQC_TRY(ctx)          \
  try {                       \
    if (!(ctx)) raise(SQC_E_ARG, "ctx is NULL");
#define SQC_CATCH(ctx)                              \
  }                                                 \
  catch (const Error &e) {                          \
    if (ctx) (ctx)->err = e.msg;                    \
    else set_thread_error(e.msg);                   \
    return e.code;                                  \
  }                                                 \
  catch (const std::exception &e) {                 \
    if (ctx) (ctx)->err = e.what();                 \
    else set_thread_error(e.what());                \
    return SQC_E_ARG;                               \
  }

// ---- first-level index slicing (Sec. 6.3) ----

namespace {

// A sliced contraction: the network without the sliced cuts, how each
// subcircuit's rows are gathered for a slice, and the workspace layout
// (after the sliced network's intermediates: gathered operands, FP64 running
// sums and their compensations, which the final step of every slice adds
// into).
struct SlicedPlan {
  std::vector<sqc_cut> rest;
  Contraction con;
  // per subcircuit: (digit position in its sigma, index in the sliced list)
  // of each incident sliced cut, ascending digit position
  std::vector<std::vector<std::pair<int, int>>> fixed;
  std::vector<int> degree;
  std::vector<size_t> gather_off;
  size_t sum_off = 0, comp_off = 0, total = 0;
  int64_t nbins = 0;
};

SlicedPlan plan_sliced(const sqc_tensor *merged, int32_t n_sub, const sqc_cut *cuts, int32_t n_cuts,
                       const int32_t *sliced, int32_t n_sliced, sqc_prec prec) {
  Graph g = build_topology(n_sub, cuts, n_cuts);
  if (!merged) raise(SQC_E_ARG, "NULL argument");
  if (n_sliced < 0 || n_sliced > SQC_MAX_SLICED) raise(SQC_E_ARG, "n_sliced outside [0, SQC_MAX_SLICED]");
  if (n_sliced > 0 && !sliced) raise(SQC_E_ARG, "sliced is NULL");
  std::vector<int> which(n_cuts, -1);
  for (int q = 0; q < n_sliced; ++q) {
    const int k = sliced[q];
    if (k < 0 || k >= n_cuts) raise(SQC_E_ARG, "a sliced cut id is out of range");
    if (which[k] >= 0) raise(SQC_E_ARG, "a cut is listed twice in sliced");
    which[k] = q;
  }
  std::vector<int> bits = degrees_match(g, merged, SQC_LAYOUT_MERGED);
  SlicedPlan sp;
  for (int k = 0; k < n_cuts; ++k)
    if (which[k] < 0) sp.rest.push_back(cuts[k]);
  Graph g2 = build_topology(n_sub, sp.rest.data(), (int32_t)sp.rest.size());
  sp.con = plan_for(g2, bits, prec);
  int abits = 0;
  for (int b : bits) abits += b;
  if (abits > 40) raise(SQC_E_UNSUPPORTED, "more than 2^40 bins");
  const size_t elem = prec == SQC_F64 ? 8 : 4;
  Bump b;
  b.off = kCtlBytes + align256(contraction_ws(sp.con, 1, false, prec));
  sp.fixed.resize(n_sub);
  sp.degree.resize(n_sub);
  sp.gather_off.assign(n_sub, 0);
  for (int i = 0; i < n_sub; ++i) {
    const std::vector<int> &inc = g.subs[i].inc;
    sp.degree[i] = (int)inc.size();
    for (size_t j = 0; j < inc.size(); ++j)
      if (which[inc[j]] >= 0) sp.fixed[i].push_back({(int)j, which[inc[j]]});
    if (!sp.fixed[i].empty()) {
      const int kept = sp.degree[i] - (int)sp.fixed[i].size();
      sp.gather_off[i] = b.take((size_t(1) << (2 * kept + bits[i])) * elem);
    }
  }
  sp.nbins = int64_t(1) << abits;
  if (n_sliced > 0) {
    sp.sum_off = b.take((size_t)sp.nbins * 8);
    sp.comp_off = b.take((size_t)sp.nbins * 8);
  }
  sp.total = b.off;
  return sp;
}

// Rows of subcircuit i's merged tensor kept by slice `q`.
SliceArgs slice_args(const SlicedPlan &sp, int i, const sqc_tensor &t, void *out, int64_t q, size_t elem) {
  SliceArgs a{};
  a.in = t.data;
  a.out = out;
  const auto &fx = sp.fixed[i];
  const int kept = sp.degree[i] - (int)fx.size();
  a.rows = int64_t(1) << (2 * kept);
  a.row_bytes_log2 = t.n_bits + (elem == 8 ? 3 : 2);
  for (const auto &f : fx) a.fixed += ((q >> (2 * f.second)) & 3) << (2 * f.first);
  // runs of kept digits: output digits [o, o + n) read input digits [p, p + n)
  int o = 0, p = 0;
  for (size_t r = 0; r <= fx.size(); ++r) {
    const int end = r < fx.size() ? fx[r].first : sp.degree[i];
    if (end > p) {
      a.lo[a.nruns] = 2 * o;
      a.len[a.nruns] = 2 * (end - p);
      a.pos[a.nruns] = 2 * p;
      a.nruns++;
      o += end - p;
    }
    p = end + 1;
  }
  return a;
}

}  // namespace

// ---- arbitrary-subset queries (Sec. 3) ----

namespace {

constexpr size_t kQueryStaging = kPinnedBytes / 2;  // per batch in flight (two)
constexpr int kQueryMaxBatch = 128;

// Every data bit fixed: the bin of one state.
std::vector<sqc_masks> state_scope(const std::vector<int> &d, uint64_t state) {
  std::vector<sqc_masks> sc(d.size());
  int off = 0;
  for (size_t i = 0; i < d.size(); ++i) {
    const uint64_t all = d[i] >= 64 ? ~uint64_t(0) : ((uint64_t(1) << d[i]) - 1);
    sc[i].fixed = all;
    sc[i].fixed_val = off < 64 ? (state >> off) & all : 0;
    sc[i].active = 0;
    sc[i].merged = 0;
    off += d[i];
  }
  return sc;
}

struct QueryPlan {
  std::shared_ptr<const CircuitTopo> c;
  std::vector<int> d;
  int total_bits = 0;
  int batch = 1;
  size_t req_ws = 0, table = 0, outs = 0;
  size_t slot = 0;   // workspace of one batch in flight (job table, requests)
  size_t total = 0;  // the control region and two slots
};

QueryPlan plan_query(const sqc_tensor *att, int32_t n_sub, const sqc_cut *cuts, int32_t n_cuts, sqc_prec prec) {
  QueryPlan q;
  q.c = make_circuit(att, n_sub, cuts, n_cuts);
  for (int i = 0; i < n_sub; ++i) {
    q.d.push_back(att[i].n_bits);
    q.total_bits += att[i].n_bits;
  }
  if (q.total_bits > 64) raise(SQC_E_UNSUPPORTED, "more than 64 data bits in total");
  // one representative request (the shape is the same for every state)
  std::vector<sqc_masks> sc = state_scope(q.d, 0);
  char dummy[64];
  PreparedPtr p = prepare_recursion(q.c, sc.data(), 1, 1, prec, dummy, SQC_F64, dummy, dummy);
  q.req_ws = prepared_workspace(*p);
  const size_t tb = prepared_table_bytes(*p);
  q.batch = (int)std::max<size_t>(1, std::min<size_t>(kQueryMaxBatch, kQueryStaging / tb));
  q.table = align256(tb * q.batch);
  q.outs = 256;  // per request: top-1 record and sum
  q.slot = align256(q.table + (size_t)q.batch * (q.req_ws + q.outs));
  q.total = kCtlBytes + 2 * q.slot;
  return q;
}

}  // namespace

// ---- Algorithm 1 on the device: the search loop without host waits ----
//
// A recursion's shape (the fixed, active and merged bit positions of every
// subcircuit, hence its contraction plan and launches) depends only on its
// depth below the first recursion: Algorithm 2 sees how many states the
// popped bin holds, which its depth fixes; only the fixed values (which bin)
// come from the data.  The host plans every depth once and writes, per
// depth, an image of the job tables that a recursion's grouped launches read
// ("live" tables at fixed addresses, one layout for every depth, grids sized
// for the largest).  All recursions are then enqueued back to back; after
// each, search_step (one work-group) does what the host loop does (records
// the recursion, appends its R largest bins to L or to the solutions, sorts
// and truncates L, pops the best bin), then copies the popped bin's depth
// image into the live tables and writes the bin's fixed values into their
// merge jobs.  When L is empty the remaining launches find depth -1 and do
// nothing.

namespace {

struct SearchState {
  int depth;  // depth of the recursion about to run (-1: finished)
  int nL, nsol, nrec, bank;
  double parent;
};

struct SearchPatch {  // one field of the live tables written per recursion
  uint32_t off;       // byte offset in the live tables
  int32_t kind;       // 0: fixed_val of subcircuit `sub`, 1: top-R output, 2: sum output
  int32_t sub;
};

struct SearchDepth {
  int leaf;   // every bin a single state
  int a;      // active bits in total
  int patch0, npatch;
};

struct SearchArgs {
  SearchState *st;
  uint64_t *F;             // [n_sub] fixed values of the recursion about to run
  double *Lp;              // [2][2R] probability
  int *Lr, *Ld;            // [2][2R] recursion, depth
  uint64_t *Lb;            // [2][2R] bin
  uint64_t *LF;            // [2][2R][n_sub] fixed values of the bin's children
  const SearchDepth *dep;  // [D]
  const int *abits;        // [D][n_sub]
  const uint64_t *active;  // [D][n_sub]
  const SearchPatch *patch;
  const unsigned char *images;  // [D][live_bytes]
  unsigned char *live;
  int64_t live_bytes;
  double *res_top;         // [R + 1][2R] value, index bits
  double *res_sum;         // [R + 1]
  sqc_recursion_info *info;  // [R]
  sqc_found *sols;           // [max_sol]
  uint64_t *sol_states;      // [max_sol][n_sub]
  int n_sub, R, max_sol, D;
};

__device__ uint64_t deposit_dev(uint64_t v, uint64_t mask) {
  uint64_t out = 0;
  for (uint64_t m = mask; m; m &= m - 1) {
    if (v & 1) out |= m & (~m + 1);
    v >>= 1;
  }
  return out;
}

constexpr int kStepThreads = 256;
constexpr int kStepMaxSub = 64;  // subcircuits the step stages in LDS
constexpr int kStepMaxDepth = 32;  // depth records prefetched with everything else

// After recursion r (the slot's index): update L and the solutions, pop the
// next bin and set up its recursion's tables (unless r is the last slot).
// The inputs are staged in LDS by all threads at once (a single thread's
// chain of dependent loads would cost microseconds each); L is ordered by
// ranking each entry against all others (the order is strict: every entry
// has its own (recursion, bin)).
__global__ __launch_bounds__(kStepThreads) void search_step(SearchArgs a, int r, int last) {
  constexpr int L2max = 2 * SQC_MAX_TOPR;
  __shared__ double kp[L2max];
  __shared__ int kr[L2max], kd[L2max], src[L2max];
  __shared__ uint64_t kb[L2max];
  __shared__ double tv[SQC_MAX_TOPR];
  __shared__ uint64_t ti[SQC_MAX_TOPR];
  __shared__ int tslot[SQC_MAX_TOPR];  // where entry q goes (L or solutions), -1: skipped
  __shared__ uint64_t F[kStepMaxSub], act[kStepMaxSub];
  __shared__ int ab[kStepMaxSub], ab0[kStepMaxSub];
  __shared__ SearchState st;
  __shared__ SearchDepth D;
  __shared__ int n_app, n_sol_new, pop, nkeep;
  __shared__ double kp2[L2max];  // the other bank's keys (read before the bank is known)
  __shared__ int kr2[L2max], kd2[L2max];
  __shared__ uint64_t kb2[L2max];
  __shared__ SearchDepth deps[kStepMaxDepth];
  __shared__ uint64_t actd[kStepMaxDepth * 8];
  __shared__ int abd[kStepMaxDepth * 8];
  __shared__ double rsum;
  const int tid = threadIdx.x;
  const int R = a.R, ns = a.n_sub, L2 = 2 * R;
  // one round of loads: everything the step may read, for both banks of L
  // and every depth when they are small (most searches), before the state
  // says which
  if (tid == 0) {
    st = *a.st;
    rsum = a.res_sum[r];
  }
  const double *top = a.res_top + (int64_t)r * 2 * R;
  if (tid < R) {
    tv[tid] = top[2 * tid];
    ti[tid] = reinterpret_cast<const uint64_t *>(top)[2 * tid + 1];
  }
  if (tid < ns) F[tid] = a.F[tid];
  const bool small = a.D <= kStepMaxDepth && ns <= 8;
  if (small) {
    if (tid < a.D) deps[tid] = a.dep[tid];
    if (tid < a.D * ns) {
      actd[tid] = a.active[tid];
      abd[tid] = a.abits[tid];
    }
  }
  for (int e = tid; e < 2 * L2; e += kStepThreads) {
    const bool first = e < L2;
    const int k = first ? e : e - L2;
    (first ? kp : kp2)[k] = a.Lp[e];
    (first ? kr : kr2)[k] = a.Lr[e];
    (first ? kd : kd2)[k] = a.Ld[e];
    (first ? kb : kb2)[k] = a.Lb[e];
  }
  __syncthreads();
  if (st.depth < 0) return;  // finished: nothing to record (every thread returns)
  const int d = st.depth, b = st.bank, nb = 1 - b;
  if (tid == 0) D = small ? deps[d] : a.dep[d];
  if (tid < ns) {
    act[tid] = small ? actd[d * ns + tid] : a.active[d * ns + tid];
    ab[tid] = small ? abd[d * ns + tid] : a.abits[d * ns + tid];
  }
  if (b == 1)
    for (int e = tid; e < st.nL; e += kStepThreads) {
      kp[e] = kp2[e];
      kr[e] = kr2[e];
      kd[e] = kd2[e];
      kb[e] = kb2[e];
    }
  for (int e = tid; e < st.nL; e += kStepThreads) src[e] = e;  // entry e of bank b
  __syncthreads();
  // the recursion's record; where each of its R largest bins goes
  if (tid == 0) {
    sqc_recursion_info inf;
    inf.bins_sum = rsum;
    inf.parent_prob = st.parent;
    inf.top_prob = tv[0];
    inf.active_bits = D.a;
    inf.leaf = D.leaf;
    a.info[r] = inf;
    int o = 0;
    for (int i = 0; i < ns; ++i) {
      ab0[i] = o;
      o += ab[i];
    }
    const uint64_t nbins = D.a >= 63 ? ~0ull : (1ull << D.a);
    const int take = (uint64_t)R < nbins ? R : (int)nbins;
    int napp = 0, nsol = 0;
    for (int q = 0; q < R; ++q) {
      const double v = tv[q];
      int slot = -1;
      if (q < take && v == v && v != -INFINITY) {
        if (!D.leaf) slot = st.nL + napp++;
        else if (st.nsol + nsol < a.max_sol) slot = st.nsol + nsol++;
      }
      tslot[q] = slot;
    }
    n_app = napp;
    n_sol_new = nsol;
  }
  __syncthreads();
  // children's fixed values (and the appended keys), one (bin, subcircuit) per thread
  for (int e = tid; e < R * ns; e += kStepThreads) {
    const int q = e / ns, i = e % ns;
    const int slot = tslot[q];
    if (slot < 0) continue;
    const uint64_t bin = ti[q];
    const int sh = ab0[i], ai = ab[i];
    const uint64_t beta = sh >= 64 ? 0 : (bin >> sh) & (ai >= 64 ? ~0ull : ((1ull << ai) - 1));
    const uint64_t fc = F[i] | deposit_dev(beta, act[i]);
    if (!D.leaf) a.LF[((int64_t)b * L2 + slot) * ns + i] = fc;
    else a.sol_states[(int64_t)slot * ns + i] = fc;
    if (i == 0) {
      if (!D.leaf) {
        kp[slot] = tv[q];
        kr[slot] = r;
        kd[slot] = d;
        kb[slot] = bin;
        src[slot] = slot;
      } else {
        sqc_found f;
        f.prob = tv[q];
        f.recursion = r;
        f.pad = 0;
        f.bin = bin;
        a.sols[slot] = f;
      }
    }
  }
  __syncthreads();
  // rank every entry of L (probability descending, then earlier recursion,
  // then lower bin index); keep the R best
  const int nL = st.nL + n_app;
  __shared__ int at_rank[L2max];
  for (int e = tid; e < nL; e += kStepThreads) {
    int rank = 0;
    for (int f = 0; f < nL; ++f)
      rank += (kp[f] > kp[e] || (kp[f] == kp[e] && (kr[f] < kr[e] || (kr[f] == kr[e] && kb[f] < kb[e])))) ? 1 : 0;
    at_rank[rank] = e;
  }
  __syncthreads();
  if (tid == 0) {
    const int kept = nL < R ? nL : R;
    pop = 0;
    if (kept == 0) {
      st.depth = -1;
    } else if (!last) {
      pop = 1;
      const int e = at_rank[0];
      st.depth = kd[e] + 1;
      st.parent = kp[e];
      if (st.depth >= a.D) st.depth = -1;  // (cannot happen: a leaf depth ends every branch)
    }
    nkeep = kept - pop;
    st.nL = nkeep;
    st.nsol += n_sol_new;
    st.nrec = r + 1;
    st.bank = nb;
  }
  __syncthreads();
  // the kept entries, sorted, into the other bank; the popped bin's
  // children's fixed values become the next recursion's
  for (int j = tid; j < nkeep; j += kStepThreads) {
    const int e = at_rank[j + pop];
    a.Lp[nb * L2 + j] = kp[e];
    a.Lr[nb * L2 + j] = kr[e];
    a.Ld[nb * L2 + j] = kd[e];
    a.Lb[nb * L2 + j] = kb[e];
  }
  for (int x = tid; x < nkeep * ns; x += kStepThreads) {
    const int j = x / ns, i = x % ns;
    a.LF[((int64_t)nb * L2 + j) * ns + i] = a.LF[((int64_t)b * L2 + src[at_rank[j + pop]]) * ns + i];
  }
  if (pop)
    for (int i = tid; i < ns; i += kStepThreads) {
      const uint64_t fn = a.LF[((int64_t)b * L2 + src[at_rank[0]]) * ns + i];
      a.F[i] = fn;
      act[i] = fn;  // (LDS copy for the patches below: act is not needed any more)
    }
  if (tid == 0) *a.st = st;
  if (!pop || st.depth < 0) return;
  __syncthreads();
  // the next recursion's tables: its depth's image, then its fixed values
  // and output slots
  const int dn = st.depth;
  const uint4 *srcimg = reinterpret_cast<const uint4 *>(a.images + (int64_t)dn * a.live_bytes);
  uint4 *dst = reinterpret_cast<uint4 *>(a.live);
  for (int64_t q = tid; q < a.live_bytes / 16; q += kStepThreads) dst[q] = srcimg[q];
  __syncthreads();
  const SearchDepth Dn = a.dep[dn];
  for (int q = tid; q < Dn.npatch; q += kStepThreads) {
    const SearchPatch pt = a.patch[Dn.patch0 + q];
    unsigned char *f = a.live + pt.off;
    if (pt.kind == 0) *reinterpret_cast<uint64_t *>(f) = act[pt.sub];
    else if (pt.kind == 1) *reinterpret_cast<double **>(f) = a.res_top + (int64_t)(r + 1) * 2 * R;
    else *reinterpret_cast<double **>(f) = a.res_sum + (r + 1);
  }
}

// One grouped launch of the live tables: merge pass 0 / 1 / 2, a GEMM, or
// the top-R stages; its jobs and work-group prefixes per depth.
struct LiveGroup {
  int kind;   // 0 merge tiles, 1 merge rows (passes 1 and 2), 2 GEMM, 3 top-R
  int level;  // GEMM level (step index)
  GemmSpec spec;
  int spec_id = -1;
  int cap = 0;           // jobs slots
  size_t jobs = 0, start[2] = {0, 0};
  int grid0[2] = {0, 0}, grid1[2] = {0, 0};  // grids: first recursion, later ones
};

struct SearchPlan {
  std::vector<RecursePlan> rp;  // per depth
  std::vector<Launches> L;
  std::vector<LiveGroup> groups;
  size_t live_bytes = 0;
  size_t rec_ws = 0;  // recursion workspace (the largest depth's)
  // search region, offsets from its base
  size_t o_live, o_images, o_patch, o_dep, o_abits, o_active, o_state, o_F, o_L, o_res, o_info, o_sols, o_states,
      region;
  int D = 0, max_sol = 0;
  std::vector<unsigned char> upload;  // live .. F
  char *base = nullptr;               // the search region on the device
};

// jobs of a depth's launches split by live group
struct DepthJobs {
  std::vector<std::pair<MergeArgs, int>> tiles, rows;  // (shaped job, subcircuit)
};

DepthJobs split_merges(const Launches &L) {
  DepthJobs j;
  for (size_t i = 0; i < L.merges.size(); ++i) {
    MergeArgs a = L.merges[i];
    merge_shape(a);
    (merge_pass_blocks(a, 0) ? j.tiles : j.rows).push_back({a, (int)i});
  }
  return j;
}

SearchPlan plan_search(sqc_ctx *ctx, const Graph &g, const sqc_tensor *att, uint64_t M, int R, sqc_prec prec,
                       void *bins_dev, sqc_prec bins_prec, int max_solutions) {
  SearchPlan sp;
  const int n_sub = g.n_sub;
  // every depth: depth d + 1 is the scope of a bin of depth d (bin 0: the
  // fixed values are written on the device)
  std::vector<sqc_masks> scope;
  for (int d = 0; d < R; ++d) {
    sp.rp.push_back(plan_recursion(g, att, d ? scope.data() : nullptr, M, R, prec, ctx_plans(ctx)));
    bool leaf = true;
    for (int i = 0; i < n_sub; ++i)
      if (sp.rp.back().masks[i].merged) leaf = false;
    if (leaf) break;
    scope.assign(n_sub, sqc_masks{});
    if (sqc_bin_scope(n_sub, sp.rp.back().masks.data(), 0, scope.data()) != SQC_OK) raise(SQC_E_ARG, thread_error());
  }
  sp.D = (int)sp.rp.size();
  for (const RecursePlan &rp : sp.rp) sp.rec_ws = std::max(sp.rec_ws, rp.total);
  // placeholders for the output slots (patched per recursion)
  for (const RecursePlan &rp : sp.rp)
    sp.L.push_back(describe_recursion(rp, att, prec, ctx->ws, ctx->unit, bins_dev, bins_prec, R, ctx->ws, ctx->ws));

  // live groups: merges, GEMM (level, specialisation), top-R
  std::vector<DepthJobs> dj;
  for (const Launches &L : sp.L) dj.push_back(split_merges(L));
  LiveGroup mt{0, -1, GemmSpec{}}, mr{1, -1, GemmSpec{}};
  for (auto &j : dj) {
    mt.cap = std::max<int>(mt.cap, (int)j.tiles.size());
    mr.cap = std::max<int>(mr.cap, (int)j.rows.size());
  }
  if (mt.cap) sp.groups.push_back(mt);
  if (mr.cap) sp.groups.push_back(mr);
  // GEMM groups by (level, specialisation), as many job slots as the most
  // steps of that key in one depth's recursion
  std::map<std::pair<int, int>, std::pair<GemmSpec, int>> gkeys;
  for (const Launches &L : sp.L) {
    std::map<std::pair<int, int>, int> count;
    for (size_t s = 0; s < L.steps.size(); ++s) ++count[{L.level[s], gemm_spec_id(L.specs[s])}];
    for (size_t s = 0; s < L.steps.size(); ++s) {
      const std::pair<int, int> key{L.level[s], gemm_spec_id(L.specs[s])};
      auto &e = gkeys.emplace(key, std::make_pair(L.specs[s], 0)).first->second;
      e.second = std::max(e.second, count[key]);
    }
  }
  for (auto &kv : gkeys) {
    LiveGroup gg{2, kv.first.first, kv.second.first};
    gg.spec_id = kv.first.second;
    gg.cap = kv.second.second;
    sp.groups.push_back(gg);
  }
  LiveGroup tg{3, -1, GemmSpec{}};
  tg.cap = 1;
  sp.groups.push_back(tg);
  // layout of the live tables
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  for (LiveGroup &lg : sp.groups) {
    const size_t jb = lg.kind <= 1 ? sizeof(MergeArgs) : lg.kind == 2 ? sizeof(GemmArgs) : sizeof(TopRArgs);
    lg.jobs = take(jb * lg.cap);
    lg.start[0] = take(sizeof(int) * (lg.cap + 1));
    if (lg.kind == 1) lg.start[1] = take(sizeof(int) * (lg.cap + 1));
  }
  sp.live_bytes = align256(off);

  // search region
  sp.max_sol = std::max(0, std::min(max_solutions, R * R));
  off = 0;
  sp.o_live = take(sp.live_bytes);
  sp.o_images = take(sp.live_bytes * sp.D);
  std::vector<SearchPatch> patches;
  std::vector<SearchDepth> deps(sp.D);
  std::vector<std::vector<unsigned char>> images(sp.D, std::vector<unsigned char>(sp.live_bytes, 0));
  for (int d = 0; d < sp.D; ++d) {
    const Launches &L = sp.L[d];
    unsigned char *img = images[d].data();
    deps[d].patch0 = (int)patches.size();
    int a = 0;
    bool leaf = true;
    for (int i = 0; i < n_sub; ++i) {
      a += sp.rp[d].abits[i];
      if (sp.rp[d].masks[i].merged) leaf = false;
    }
    deps[d].a = a;
    deps[d].leaf = leaf ? 1 : 0;
    for (LiveGroup &lg : sp.groups) {
      int *st0 = reinterpret_cast<int *>(img + lg.start[0]);
      int *st1 = lg.kind == 1 ? reinterpret_cast<int *>(img + lg.start[1]) : nullptr;
      int total0 = 0, total1 = 0;
      if (lg.kind <= 1) {
        const auto &jobs = lg.kind == 0 ? dj[d].tiles : dj[d].rows;
        for (size_t k = 0; k < jobs.size(); ++k) {
          std::memcpy(img + lg.jobs + k * sizeof(MergeArgs), &jobs[k].first, sizeof(MergeArgs));
          patches.push_back(SearchPatch{(uint32_t)(lg.jobs + k * sizeof(MergeArgs) + offsetof(MergeArgs, fixed_val)),
                                        0, jobs[k].second});
          st0[k] = total0;
          total0 += (int)merge_pass_blocks(jobs[k].first, lg.kind == 0 ? 0 : 1);
          if (st1) {
            st1[k] = total1;
            total1 += (int)merge_pass_blocks(jobs[k].first, 2);
          }
        }
        for (int k = (int)jobs.size(); k <= lg.cap; ++k) {
          st0[k] = total0;
          if (st1) st1[k] = total1;
        }
      } else if (lg.kind == 2) {
        // this depth's steps of the group's level and specialisation, the
        // larger launches first
        std::vector<int> mine;
        for (size_t s = 0; s < L.steps.size(); ++s)
          if (L.level[s] == lg.level && gemm_spec_id(L.specs[s]) == lg.spec_id) mine.push_back((int)s);
        std::stable_sort(mine.begin(), mine.end(), [&](int a, int b) { return L.groups[a] > L.groups[b]; });
        for (size_t k = 0; k < mine.size(); ++k) {
          std::memcpy(img + lg.jobs + k * sizeof(GemmArgs), &L.steps[mine[k]], sizeof(GemmArgs));
          st0[k] = total0;
          total0 += L.groups[mine[k]];
        }
        for (int k = (int)mine.size(); k <= lg.cap; ++k) st0[k] = total0;
      } else {
        TopRArgs t = L.t;
        std::memcpy(img + lg.jobs, &t, sizeof(TopRArgs));
        patches.push_back(SearchPatch{(uint32_t)(lg.jobs + offsetof(TopRArgs, top_out)), 1, 0});
        patches.push_back(SearchPatch{(uint32_t)(lg.jobs + offsetof(TopRArgs, sum_out)), 2, 0});
        total0 = t.gather_groups;
        st0[0] = 0;
        st0[1] = total0;
      }
      int *g0 = d == 0 ? lg.grid0 : lg.grid1;
      g0[0] = std::max(g0[0], total0);
      g0[1] = std::max(g0[1], total1);
    }
    deps[d].npatch = (int)patches.size() - deps[d].patch0;
  }
  sp.o_patch = take(sizeof(SearchPatch) * std::max<size_t>(1, patches.size()));
  sp.o_dep = take(sizeof(SearchDepth) * sp.D);
  sp.o_abits = take(sizeof(int) * sp.D * n_sub);
  sp.o_active = take(sizeof(uint64_t) * sp.D * n_sub);
  sp.o_state = take(sizeof(SearchState));
  sp.o_F = take(sizeof(uint64_t) * n_sub);
  const size_t upload_end = off;
  sp.o_L = take((8 + 4 + 4 + 8) * 2 * 2 * (size_t)R + 8 * 2 * 2 * (size_t)R * n_sub + 4 * 256);
  sp.o_res = take(8 * (size_t)(R + 1) * (2 * R + 1));
  sp.o_info = take(sizeof(sqc_recursion_info) * R);
  sp.o_sols = take(sizeof(sqc_found) * std::max(1, sp.max_sol));
  sp.o_states = take(sizeof(uint64_t) * std::max(1, sp.max_sol) * n_sub);
  sp.region = off;

  // the upload image: live tables (depth 0, first recursion's slots), the
  // depth images, patches, depth records, masks, state, fixed values
  sp.upload.assign(upload_end, 0);
  unsigned char *U = sp.upload.data();
  std::memcpy(U + sp.o_live, images[0].data(), sp.live_bytes);
  for (int d = 0; d < sp.D; ++d) std::memcpy(U + sp.o_images + d * sp.live_bytes, images[d].data(), sp.live_bytes);
  if (!patches.empty()) std::memcpy(U + sp.o_patch, patches.data(), sizeof(SearchPatch) * patches.size());
  std::memcpy(U + sp.o_dep, deps.data(), sizeof(SearchDepth) * sp.D);
  for (int d = 0; d < sp.D; ++d)
    for (int i = 0; i < n_sub; ++i) {
      reinterpret_cast<int *>(U + sp.o_abits)[d * n_sub + i] = sp.rp[d].abits[i];
      reinterpret_cast<uint64_t *>(U + sp.o_active)[d * n_sub + i] = sp.rp[d].masks[i].active;
    }
  SearchState st0{};
  st0.depth = 0;
  st0.parent = 1.0;
  std::memcpy(U + sp.o_state, &st0, sizeof(st0));
  // the search region follows the recursions' workspace; the first
  // recursion's output slots are set here (later ones by search_step)
  sp.base = ctx->ws + align256(sp.rec_ws);
  double *res_top = reinterpret_cast<double *>(sp.base + sp.o_res);
  double *res_sum = res_top + (size_t)(R + 1) * 2 * R;
  for (int q = 0; q < deps[0].npatch; ++q) {
    const SearchPatch &pt = patches[deps[0].patch0 + q];
    unsigned char *f = U + sp.o_live + pt.off;
    if (pt.kind == 1) std::memcpy(f, &res_top, sizeof(res_top));
    else if (pt.kind == 2) std::memcpy(f, &res_sum, sizeof(res_sum));
  }
  return sp;
}

}  // namespace

extern "C" {

const char *sqc_version(void) { return "sqc 0.1.0 (gfx950)"; }

const char *sqc_last_error(const sqc_ctx *ctx) {
  return ctx ? ctx->err.c_str() : thread_error();
}

sqc_status sqc_ctx_create(int device, void *hip_stream, sqc_ctx **out) {
  try {
    if (!out) raise(SQC_E_ARG, "out is NULL");
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) raise(SQC_E_DEVICE, "no HIP device is available");
    if (device < 0 || device >= n) raise(SQC_E_ARG, "device index out of range");
    check_hip(hipSetDevice(device), "hipSetDevice");
    hipDeviceProp_t prop;
    check_hip(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
      std::ostringstream s;
      s << "device " << device << " is " << prop.gcnArchName << "; this build targets gfx950";
      raise(SQC_E_DEVICE, s.str());
    }
    sqc_ctx *c = new sqc_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipHostMalloc(&c->pinned, kPinnedBytes, hipHostMallocDefault) != hipSuccess) {
      delete c;
      raise(SQC_E_DEVICE, "hipHostMalloc of the staging buffer failed");
    }
    const DeviceStatics *ds = device_statics(device);
    if (!ds) {
      (void)hipHostFree(c->pinned);
      delete c;
      raise(SQC_E_DEVICE, "hipGetSymbolAddress of the library's device constants failed");
    }
    c->unit = static_cast<double *>(ds->unit);
    *out = c;
    return SQC_OK;
  } catch (const Error &e) {
    set_thread_error(e.msg);
    return e.code;
  }
}

sqc_status sqc_ctx_destroy(sqc_ctx *ctx) {
  if (!ctx) return SQC_E_ARG;
  (void)hipSetDevice(ctx->device);
  for (auto &m : ctx->marks) {
    (void)hipEventSynchronize(m.b);
    (void)hipEventDestroy(m.a);
    (void)hipEventDestroy(m.b);
  }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete static_cast<PlanCache *>(ctx->plan_cache);
  delete ctx;
  return SQC_OK;
}

sqc_status sqc_ctx_set_stream(sqc_ctx *ctx, void *hip_stream) {
  SQC_TRY(ctx)
  if (ctx->recording) raise(SQC_E_ARG, "the stream cannot change while a graph is recorded");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return SQC_OK;
  SQC_CATCH(ctx)
}

// ---- HIP graphs of enqueued work ----

struct sqc_graph {
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

sqc_status sqc_graph_begin(sqc_ctx *ctx) {
  SQC_TRY(ctx)
  if (!ctx->stream) raise(SQC_E_ARG, "graph recording needs a created stream (not the default stream)");
  if (ctx->recording) raise(SQC_E_ARG, "a graph is already being recorded on this context");
  use_device(ctx);
  check_hip(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
  ctx->saved_mask = ctx->timing_mask;
  ctx->timing_mask = 0;
  ctx->recording = true;
  return SQC_OK;
  SQC_CATCH(ctx)
}

sqc_status sqc_graph_end(sqc_ctx *ctx, sqc_graph **out) {
  SQC_TRY(ctx)
  if (!ctx->recording) raise(SQC_E_ARG, "no graph is being recorded on this context");
  use_device(ctx);
  ctx->recording = false;
  ctx->timing_mask = ctx->saved_mask;
  hipGraph_t graph = nullptr;
  check_hip(hipStreamEndCapture(ctx->stream, &graph), "hipStreamEndCapture");
  if (!out) {
    (void)hipGraphDestroy(graph);
    raise(SQC_E_ARG, "out is NULL");
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  check_hip(e, "hipGraphInstantiate");
  sqc_graph *g = new sqc_graph();
  g->exec = exec;
  g->device = ctx->device;
  *out = g;
  return SQC_OK;
  SQC_CATCH(ctx)
}

sqc_status sqc_graph_launch(sqc_ctx *ctx, const sqc_graph *g) {
  SQC_TRY(ctx)
  if (!g || !g->exec) raise(SQC_E_ARG, "graph is NULL");
  if (g->device != ctx->device) raise(SQC_E_ARG, "graph was recorded on another device");
  use_device(ctx);
  check_hip(hipGraphLaunch(g->exec, ctx->stream), "hipGraphLaunch");
  return SQC_OK;
  SQC_CATCH(ctx)
}

sqc_status sqc_graph_destroy(sqc_graph *g) {
  if (!g) return SQC_E_ARG;
  if (g->exec) {
    (void)hipSetDevice(g->device);
    (void)hipGraphExecDestroy(g->exec);
  }
  delete g;
  return SQC_OK;
}

sqc_status sqc_ctx_set_timing(sqc_ctx *ctx, uint32_t stage_mask) {
  SQC_TRY(ctx)
  ctx->timing_mask = stage_mask & 31u;
  return SQC_OK;
  SQC_CATCH(ctx)
}

sqc_status sqc_ctx_timing(sqc_ctx *ctx, uint32_t stage, int32_t reset, sqc_stage_time *out) {
  SQC_TRY(ctx)
  if (ctx->recording) raise(SQC_E_ARG, "stage timing cannot be read while a graph is recorded");
  int q = stage_index(stage);
  if (q < 0 || !out) raise(SQC_E_ARG, "stage must be one SQC_STAGE_* bit and out non-NULL");
  use_device(ctx);
  settle_timing(ctx);
  out->ms = ctx->tot[q].ms;
  out->launches = ctx->tot[q].n;
  out->bytes = ctx->tot[q].bytes;
  out->flops = ctx->tot[q].flops;
  if (reset)
    for (auto &t : ctx->tot) t = sqc_ctx::Tot{};
  return SQC_OK;
  SQC_CATCH(ctx)
}

sqc_status sqc_ctx_set_workspace(sqc_ctx *ctx, void *dev, size_t bytes) {
  SQC_TRY(ctx)
  if (!dev || bytes < kCtlBytes) raise(SQC_E_ARG, "workspace must be at least 4096 bytes");
  if (reinterpret_cast<uintptr_t>(dev) % 256) raise(SQC_E_ARG, "workspace must be 256-byte aligned");
  ctx->ws = static_cast<char *>(dev);
  ctx->ws_bytes = bytes;
  return SQC_OK;
  SQC_CATCH(ctx)
}

size_t sqc_attribute_bytes(const sqc_sub *subs, int32_t n_sub, int32_t sub_id,
                           const sqc_cut *cuts, int32_t n_cuts, sqc_prec out_prec) {
  try {
    Graph g = build_graph(subs, n_sub, cuts, n_cuts);
    if (sub_id < 0 || sub_id >= n_sub) return 0;
    if (out_prec != SQC_F64 && out_prec != SQC_F32) return 0;
    const SubInfo &s = g.subs[sub_id];
    if (2 * (int)s.inc.size() + s.d > 40) return 0;
    return ((size_t)1 << (2 * s.inc.size() + s.d)) * elem_bytes(out_prec);
  } catch (const Error &e) {
    set_thread_error(e.msg);
    return 0;
  }
}

namespace {

// Arguments of one subcircuit's attribution (validates the output tensor).
AttrArgs attr_args(const Graph &g, int sub_id, const void *variants_dev, sqc_prec in_prec,
                   const sqc_tensor *out, bool merged = false) {
  if (!variants_dev) raise(SQC_E_ARG, "variants_dev is NULL");
  if (!out || !out->data) raise(SQC_E_ARG, "out or out->data is NULL");
  check_storage_prec(in_prec, "in_prec");
  check_storage_prec(out->prec, "out->prec");
  const SubInfo &s = g.subs[sub_id];
  const int c = (int)s.inc.size();
  check_size(2 * c, s.d);
  AttrArgs a{};
  a.var = variants_dev;
  a.out = out->data;
  a.in_f32 = in_prec == SQC_F32;
  a.out_f32 = out->prec == SQC_F32;
  a.w = s.w;
  a.d = s.d;
  a.c = c;
  int64_t place = 1;
  for (int q = 0; q < c; ++q) {
    a.place[q] = place;
    if (s.role[q] == 0) {
      a.in_pos[a.n_in++] = q;
      place *= 4;
    } else {
      a.out_wire[a.n_out] = g.cuts[s.inc[q]].up_wire;
      a.out_pos[a.n_out++] = q;
      place *= 3;
    }
  }
  for (int j = 0; j < s.d; ++j) a.data_wire[j] = s.data_wire[j];
  a.scale = std::ldexp(1.0, -a.n_out);
  a.out_merged = merged ? 1 : 0;
  return a;
}

// Algorithmic bytes of one attribution: every variant entry read once, every
// attributed entry written once.
double attr_bytes(const Graph &g, int sub_id, const AttrArgs &a, double *reads) {
  const SubInfo &s = g.subs[sub_id];
  const double nvar = double(s.variants) * std::ldexp(1.0, s.w);
  const double nout = std::ldexp(1.0, 2 * a.c + s.d);
  *reads += nvar;
  return nvar * (a.in_f32 ? 4 : 8) + nout * (a.out_f32 ? 4 : 8);
}

void finish_attr_out(const AttrArgs &a, sqc_tensor *out) {
  out->n_labels = a.c;
  out->n_bits = a.d;
  out->layout = a.out_merged ? SQC_LAYOUT_MERGED : SQC_LAYOUT_ATTRIBUTED;
}

}  // namespace

sqc_status sqc_attribute(sqc_ctx *ctx, const sqc_sub *subs, int32_t n_sub, int32_t sub_id,
                         const sqc_cut *cuts, int32_t n_cuts, const void *variants_dev,
                         sqc_prec in_prec, sqc_tensor *out) {
  SQC_TRY(ctx)
  Graph g = build_graph(subs, n_sub, cuts, n_cuts);
  if (sub_id < 0 || sub_id >= n_sub) raise(SQC_E_ARG, "sub_id out of range");
  const AttrArgs a = attr_args(g, sub_id, variants_dev, in_prec, out);
  use_device(ctx);
  double reads = 0;
  const double bytes = attr_bytes(g, sub_id, a, &reads);
  StageMark mark(ctx, SQC_STAGE_ATTRIBUTE, bytes, reads);
  launch_attributes(&a, 1, ctx->stream);
  after_launch("attribution kernel launch");
  mark.done();
  finish_attr_out(a, out);
  return SQC_OK;
  SQC_CATCH(ctx)
}

namespace {

sqc_status attribute_all(sqc_ctx *ctx, const sqc_sub *subs, int32_t n_sub, const sqc_cut *cuts, int32_t n_cuts,
                         const void *const *variants_dev, sqc_prec in_prec, sqc_tensor *outs, bool merged) {
  SQC_TRY(ctx)
  Graph g = build_graph(subs, n_sub, cuts, n_cuts);
  if (!variants_dev || !outs) raise(SQC_E_ARG, "NULL argument");
  std::vector<AttrArgs> jobs;
  double bytes = 0, reads = 0;
  for (int i = 0; i < n_sub; ++i) {
    jobs.push_back(attr_args(g, i, variants_dev[i], in_prec, &outs[i], merged));
    bytes += attr_bytes(g, i, jobs.back(), &reads);
  }
  use_device(ctx);
  StageMark mark(ctx, SQC_STAGE_ATTRIBUTE, bytes, reads);
  launch_attributes(jobs.data(), n_sub, ctx->stream);
  after_launch("attribution kernel launch");
  mark.done();
  for (int i = 0; i < n_sub; ++i) finish_attr_out(jobs[i], &outs[i]);
  return SQC_OK;
  SQC_CATCH(ctx)
}

}  // namespace

sqc_status sqc_attribute_all(sqc_ctx *ctx, const sqc_sub *subs, int32_t n_sub, const sqc_cut *cuts,
                             int32_t n_cuts, const void *const *variants_dev, sqc_prec in_prec,
                             sqc_tensor *outs) {
  return attribute_all(ctx, subs, n_sub, cuts, n_cuts, variants_dev, in_prec, outs, false);
}

sqc_status sqc_attribute_all_merged(sqc_ctx *ctx, const sqc_sub *subs, int32_t n_sub, const sqc_cut *cuts,
                                    int32_t n_cuts, const void *const *variants_dev, sqc_prec in_prec,
                                    sqc_tensor *outs) {
  return attribute_all(ctx, subs, n_sub, cuts, n_cuts, variants_dev, in_prec, outs, true);
}

size_t sqc_merge_workspace_bytes(const sqc_tensor *attributed, const sqc_masks *masks) {
  if (!attributed || !masks) return 0;
  return kCtlBytes + merge_ws(*attributed, *masks);
}

sqc_status sqc_merge(sqc_ctx *ctx, const sqc_tensor *attributed, const sqc_masks *masks,
                     sqc_tensor *out) {
  SQC_TRY(ctx)
  if (!attributed || !masks || !out || !out->data || !attributed->data)
    raise(SQC_E_ARG, "NULL argument");
  if (attributed->layout != SQC_LAYOUT_ATTRIBUTED) raise(SQC_E_SHAPE, "input is not an attributed tensor");
  check_storage_prec(attributed->prec, "attributed->prec");
  check_storage_prec(out->prec, "out->prec");
  if (attributed->n_labels < 0 || attributed->n_labels > SQC_MAX_DEGREE)
    raise(SQC_E_SHAPE, "label count out of range");
  if (attributed->n_bits < 0 || attributed->n_bits > SQC_MAX_DATA_BITS)
    raise(SQC_E_SHAPE, "bit count out of range");
  check_size(2 * attributed->n_labels, attributed->n_bits);
  check_masks(*masks, attributed->n_bits, 0);
  size_t part = merge_ws(*attributed, *masks);
  if (part) need_ws(ctx, kCtlBytes + part);
  use_device(ctx);
  enqueue_merges(ctx, {merge_args(*attributed, *masks, out->data, out->prec == SQC_F32,
                                  part ? reinterpret_cast<double *>(ctx->ws + kCtlBytes) : nullptr)});
  out->n_labels = attributed->n_labels;
  out->n_bits = __builtin_popcountll(masks->active);
  out->layout = SQC_LAYOUT_MERGED;
  return SQC_OK;
  SQC_CATCH(ctx)
}

size_t sqc_contract_workspace_bytes(const sqc_tensor *merged, int32_t n_sub, const sqc_cut *cuts,
                                    int32_t n_cuts, sqc_prec prec) {
  try {
    Graph g = build_topology(n_sub, cuts, n_cuts);
    if (!merged) return 0;
    std::vector<int> bits = degrees_match(g, merged, SQC_LAYOUT_MERGED);
    Contraction c = plan_for(g, bits, prec);
    return kCtlBytes + contraction_ws(c, 1, false, prec);
  } catch (const Error &e) {
    set_thread_error(e.msg);
    return 0;
  }
}

sqc_status sqc_contract(sqc_ctx *ctx, const sqc_tensor *merged, int32_t n_sub, const sqc_cut *cuts,
                        int32_t n_cuts, sqc_prec prec, void *bins_dev, sqc_prec bins_prec) {
  SQC_TRY(ctx)
  Graph g = build_topology(n_sub, cuts, n_cuts);
  if (!merged || !bins_dev) raise(SQC_E_ARG, "NULL argument");
  check_path_prec(prec);
  check_storage_prec(bins_prec, "bins_prec");
  std::vector<int> bits = degrees_match(g, merged, SQC_LAYOUT_MERGED);
  for (int i = 0; i < n_sub; ++i) {
    bool want_f64 = prec == SQC_F64;
    if ((merged[i].prec == SQC_F64) != want_f64)
      raise(SQC_E_ARG, "merged tensors must be FP64 for the FP64 path and FP32 otherwise");
  }
  Contraction c = plan_for(g, bits, prec);
  need_ws(ctx, kCtlBytes + contraction_ws(c, 1, false, prec));
  use_device(ctx);
  std::vector<const void *> inputs(n_sub);
  for (int i = 0; i < n_sub; ++i) inputs[i] = merged[i].data;
  enqueue_contraction(ctx, c, inputs, kCtlBytes, bins_dev, bins_prec == SQC_F32, prec, 0, nullptr,
                      nullptr);
  return SQC_OK;
  SQC_CATCH(ctx)
}

size_t sqc_contract_sliced_workspace_bytes(const sqc_tensor *merged, int32_t n_sub, const sqc_cut *cuts,
                                           int32_t n_cuts, const int32_t *sliced, int32_t n_sliced,
                                           sqc_prec prec) {
  try {
    return plan_sliced(merged, n_sub, cuts, n_cuts, sliced, n_sliced, prec).total;
  } catch (const Error &e) {
    set_thread_error(e.msg);
    return 0;
  }
}

sqc_status sqc_contract_sliced(sqc_ctx *ctx, const sqc_tensor *merged, int32_t n_sub, const sqc_cut *cuts,
                               int32_t n_cuts, const int32_t *sliced, int32_t n_sliced, sqc_prec prec,
                               void *bins_dev, sqc_prec bins_prec) {
  SQC_TRY(ctx)
  if (!bins_dev) raise(SQC_E_ARG, "NULL argument");
  check_path_prec(prec);
  check_storage_prec(bins_prec, "bins_prec");
  SlicedPlan sp = plan_sliced(merged, n_sub, cuts, n_cuts, sliced, n_sliced, prec);
  for (int i = 0; i < n_sub; ++i)
    if ((merged[i].prec == SQC_F64) != (prec == SQC_F64))
      raise(SQC_E_ARG, "merged tensors must be FP64 for the FP64 path and FP32 otherwise");
  need_ws(ctx, sp.total);
  use_device(ctx);
  const size_t elem = prec == SQC_F64 ? 8 : 4;
  double *sum = reinterpret_cast<double *>(ctx->ws + sp.sum_off);
  double *comp = reinterpret_cast<double *>(ctx->ws + sp.comp_off);
  const int64_t nslices = int64_t(1) << (2 * n_sliced);
  std::vector<const void *> inputs(n_sub);
  if (nslices == 1) {  // nothing sliced: the plain contraction
    for (int i = 0; i < n_sub; ++i) inputs[i] = merged[i].data;
    enqueue_contraction(ctx, sp.con, inputs, kCtlBytes, bins_dev, bins_prec == SQC_F32, prec, 0, nullptr, nullptr);
    return SQC_OK;
  }
  for (int64_t q = 0; q < nslices; ++q) {
    {
      StageMark mark(ctx, SQC_STAGE_MERGE, 0.0, 0.0);
      for (int i = 0; i < n_sub; ++i) {
        if (sp.fixed[i].empty()) {
          inputs[i] = merged[i].data;
          continue;
        }
        const SliceArgs a = slice_args(sp, i, merged[i], ctx->ws + sp.gather_off[i], q, elem);
        launch_slice_rows(a, ctx->stream);
        after_launch("slice gather launch");
        inputs[i] = a.out;
      }
      mark.done();
    }
    SliceAcc acc;
    acc.mode = q == 0 ? 1 : q == nslices - 1 ? 3 : 2;
    acc.sum = sum;
    acc.comp = comp;
    Launches L;
    describe_contraction(L, sp.con, inputs, ctx->ws, ctx->unit, kCtlBytes, bins_dev, bins_prec == SQC_F32, prec, 0,
                         nullptr, nullptr, acc);
    run_direct(ctx, L);
  }
  return SQC_OK;
  SQC_CATCH(ctx)
}

size_t sqc_query_states_workspace_bytes(const sqc_tensor *attributed, int32_t n_sub, const sqc_cut *cuts,
                                        int32_t n_cuts, sqc_prec prec) {
  try {
    return plan_query(attributed, n_sub, cuts, n_cuts, prec).total;
  } catch (const Error &e) {
    set_thread_error(e.msg);
    return 0;
  }
}

sqc_status sqc_query_states(sqc_ctx *ctx, const sqc_tensor *attributed, int32_t n_sub, const sqc_cut *cuts,
                            int32_t n_cuts, const uint64_t *states, int64_t n_states, sqc_prec prec,
                            void *probs_dev, sqc_prec probs_prec) {
  SQC_TRY(ctx)
  if (ctx->recording) raise(SQC_E_ARG, "sqc_query_states waits for the device and cannot be recorded");
  if (n_states < 0) raise(SQC_E_ARG, "n_states must be >= 0");
  if (n_states > 0 && (!states || !probs_dev)) raise(SQC_E_ARG, "NULL argument");
  check_storage_prec(probs_prec, "probs_prec");
  QueryPlan q = plan_query(attributed, n_sub, cuts, n_cuts, prec);
  for (int64_t j = 0; j < n_states; ++j)
    if (q.total_bits < 64 && (states[j] >> q.total_bits) != 0) {
      std::ostringstream m;
      m << "state " << states[j] << " (entry " << j << ") is outside [0, 2^" << q.total_bits << ")";
      raise(SQC_E_ARG, m.str());
    }
  if (n_states == 0) return SQC_OK;
  need_ws(ctx, q.total);
  use_device(ctx);
  const size_t elem = probs_prec == SQC_F32 ? 4 : 8;
  // two batches in flight: batch k uses half k % 2 of the pinned staging
  // buffer and slot k % 2 of the workspace, and the host forms batch k + 1
  // while the device runs batch k; a half is rewritten only once the batch
  // two before has finished with it (its event)
  struct Events {  // returned to the pool on every exit
    sqc_ctx *c;
    hipEvent_t e[2];
    ~Events() {
      c->pool.push_back(e[0]);
      c->pool.push_back(e[1]);
    }
  } ev{ctx, {take_event(ctx), take_event(ctx)}};
  int64_t k = 0;
  for (int64_t j0 = 0; j0 < n_states; j0 += q.batch, ++k) {
    const int half = (int)(k & 1);
    if (k >= 2) check_hip(hipEventSynchronize(ev.e[half]), "hipEventSynchronize");
    char *table = ctx->ws + kCtlBytes + half * q.slot;
    char *reqs = table + q.table;
    char *staging = static_cast<char *>(ctx->pinned) + half * kQueryStaging;
    const int n = (int)std::min<int64_t>(q.batch, n_states - j0);
    std::vector<PreparedPtr> ps;
    std::vector<PreparedRecursion *> raw;
    std::vector<char *> ws;
    for (int r = 0; r < n; ++r) {
      std::vector<sqc_masks> sc = state_scope(q.d, states[j0 + r]);
      char *w = reqs + (size_t)r * (q.req_ws + q.outs);
      char *o = w + q.req_ws;
      ps.push_back(prepare_recursion(q.c, sc.data(), 1, 1, prec, static_cast<char *>(probs_dev) + (j0 + r) * elem,
                                     probs_prec, o, o + 2 * sizeof(double)));
      raw.push_back(ps.back().get());
      ws.push_back(w);
    }
    enqueue_batch(ctx, raw.data(), n, ws.data(), table, q.table, staging, kQueryStaging);
    check_hip(hipEventRecord(ev.e[half], ctx->stream), "hipEventRecord");
  }
  check_hip(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  return SQC_OK;
  SQC_CATCH(ctx)
}

size_t sqc_recurse_workspace_bytes(const sqc_tensor *attributed, int32_t n_sub, const sqc_cut *cuts,
                                   int32_t n_cuts, const sqc_masks *masks, sqc_prec prec) {
  try {
    Graph g = build_topology(n_sub, cuts, n_cuts);
    if (!attributed || !masks) return 0;
    degrees_match(g, attributed, -1);
    // the masks given fix the bin counts: use them as the scope with M large
    std::vector<int> abits(n_sub);
    for (int i = 0; i < n_sub; ++i) abits[i] = __builtin_popcountll(masks[i].active);
    const bool autop = prec == SQC_AUTO;
    if (autop) {
      for (int i = 0; i < n_sub; ++i)
        if (attributed[i].layout == SQC_LAYOUT_MERGED)
          raise(SQC_E_ARG, "precision selection (SQC_AUTO) needs attributed tensors, not merged-layout ones");
      prec = SQC_F64;  // the largest of the choices
    }
    check_merged_inputs(attributed, masks, n_sub, prec);
    Bump b;
    layout_merges(b, attributed, masks, n_sub, prec == SQC_F64 ? 8 : 4);
    Contraction c = plan_for(g, abits, prec);
    size_t need = b.off + contraction_ws(c, SQC_MAX_TOPR, true, prec);
    if (autop) {
      // the selector's own pass: FP32 merged tensors, row maxima, label-only contraction
      Bump b2;
      layout_merges(b2, attributed, masks, n_sub, 4);
      for (int i = 0; i < n_sub; ++i) b2.take((size_t(1) << (2 * attributed[i].n_labels)) * sizeof(double));
      b2.take(sizeof(double));
      need = std::max(need, b2.off + contraction_ws(plan_for(g, std::vector<int>(n_sub, 0), SQC_F64), 1, false,
                                                    SQC_F64));
    }
    return need;
  } catch (const Error &e) {
    set_thread_error(e.msg);
    return 0;
  }
}

sqc_status sqc_recurse(sqc_ctx *ctx, const sqc_tensor *attributed, int32_t n_sub, const sqc_cut *cuts,
                       int32_t n_cuts, const sqc_masks *scope, uint64_t max_bins_M, int32_t top_r,
                       sqc_prec prec, void *bins_dev, sqc_prec bins_prec, sqc_masks *masks_out,
                       void *topr_dev, void *sum_dev) {
  SQC_TRY(ctx)
  Graph g = build_topology(n_sub, cuts, n_cuts);
  if (!attributed || !bins_dev || !topr_dev || !sum_dev) raise(SQC_E_ARG, "NULL argument");
  if (prec == SQC_AUTO) {
    check_storage_prec(bins_prec, "bins_prec");
    if (top_r < 1 || top_r > SQC_MAX_TOPR) raise(SQC_E_ARG, "top_r must be in [1, 64]");
    degrees_match(g, attributed, -1);
    for (int i = 0; i < n_sub; ++i)
      if (attributed[i].layout == SQC_LAYOUT_MERGED)
        raise(SQC_E_ARG, "precision selection (SQC_AUTO) needs attributed tensors, not merged-layout ones");
    double B = 0.0;
    prec = select_precision(ctx, g, attributed, scope, max_bins_M, &B);
    ctx->auto_choice = prec;
    ctx->auto_bound = B;
  }
  check_path_prec(prec);
  check_storage_prec(bins_prec, "bins_prec");
  if (top_r < 1 || top_r > SQC_MAX_TOPR) raise(SQC_E_ARG, "top_r must be in [1, 64]");
  degrees_match(g, attributed, -1);
  RecursePlan rp = plan_recursion(g, attributed, scope, max_bins_M, top_r, prec, ctx_plans(ctx));
  const bool pre_merged = check_merged_inputs(attributed, rp.masks.data(), n_sub, prec);
  if (!ctx->ws) need_ws(ctx, rp.total);
  size_t need = 0;
  const std::vector<int> sl = choose_slices(g, attributed, rp, prec, top_r, ctx->ws_bytes, &need);
  if (!sl.empty() && pre_merged)
    raise(SQC_E_ARG, "the recursion needs slicing to fit the workspace, which merges label rows from attributed "
                     "tensors; merged-layout inputs cannot be sliced");
  use_device(ctx);
  if (sl.empty())
    enqueue_recursion(ctx, rp, attributed, prec, bins_dev, bins_prec, top_r, topr_dev, sum_dev);
  else
    enqueue_sliced_recursion(ctx, layout_sliced(g, attributed, rp, sl, prec, top_r), attributed, prec, bins_dev,
                             bins_prec, top_r, topr_dev, sum_dev);
  if (masks_out) std::copy(rp.masks.begin(), rp.masks.end(), masks_out);
  return SQC_OK;
  SQC_CATCH(ctx)
}

sqc_status sqc_recurse_slices(const sqc_tensor *attributed, int32_t n_sub, const sqc_cut *cuts, int32_t n_cuts,
                              const sqc_masks *masks, sqc_prec prec, int32_t top_r, size_t workspace_bytes,
                              int32_t *sliced, int32_t *n_sliced, size_t *need_bytes) {
  try {
  Graph g = build_topology(n_sub, cuts, n_cuts);
  if (!attributed || !masks || !sliced || !n_sliced) raise(SQC_E_ARG, "NULL argument");
  check_path_prec(prec);
  if (top_r < 1 || top_r > SQC_MAX_TOPR) raise(SQC_E_ARG, "top_r must be in [1, 64]");
  degrees_match(g, attributed, SQC_LAYOUT_ATTRIBUTED);
  RecursePlan rp = plan_from_masks(g, attributed, masks, top_r, prec);
  size_t need = 0;
  const std::vector<int> sl = choose_slices(g, attributed, rp, prec, top_r, workspace_bytes, &need);
  std::copy(sl.begin(), sl.end(), sliced);
  *n_sliced = (int32_t)sl.size();
  if (need_bytes) *need_bytes = need;
  set_thread_error("");
  return SQC_OK;
  } catch (const Error &e) {
    set_thread_error(e.msg);
    return e.code;
  }
}

sqc_status sqc_ctx_set_tolerance(sqc_ctx *ctx, double max_abs_error) {
  SQC_TRY(ctx)
  if (!(max_abs_error > 0.0) || max_abs_error == INFINITY) raise(SQC_E_ARG, "the tolerance must be finite and > 0");
  ctx->tol = max_abs_error;
  return SQC_OK;
  SQC_CATCH(ctx)
}

sqc_status sqc_select_precision(sqc_ctx *ctx, const sqc_tensor *attributed, int32_t n_sub, const sqc_cut *cuts,
                                int32_t n_cuts, const sqc_masks *scope, uint64_t max_bins_M, sqc_prec *chosen,
                                double *bound) {
  SQC_TRY(ctx)
  Graph g = build_topology(n_sub, cuts, n_cuts);
  if (!attributed || !chosen) raise(SQC_E_ARG, "NULL argument");
  degrees_match(g, attributed, SQC_LAYOUT_ATTRIBUTED);
  *chosen = select_precision(ctx, g, attributed, scope, max_bins_M, bound);
  return SQC_OK;
  SQC_CATCH(ctx)
}

sqc_status sqc_ctx_auto_choice(const sqc_ctx *ctx, sqc_prec *chosen, double *bound) {
  if (!ctx || !chosen) return SQC_E_ARG;
  *chosen = ctx->auto_choice;
  if (bound) *bound = ctx->auto_bound;
  return ctx->auto_bound < 0 ? SQC_E_ARG : SQC_OK;
}

sqc_status sqc_recurse_noalloc(sqc_ctx *ctx, const sqc_tensor *attributed, int32_t n_sub, const sqc_cut *cuts,
                               int32_t n_cuts, const sqc_masks *scope, uint64_t max_bins_M, int32_t top_r,
                               sqc_prec prec, void *bins_dev, sqc_prec bins_prec, sqc_masks *masks_out,
                               void *topr_dev, void *sum_dev) {
  SQC_TRY(ctx)
  Graph g = build_topology(n_sub, cuts, n_cuts);
  if (!attributed || !bins_dev || !topr_dev || !sum_dev) raise(SQC_E_ARG, "NULL argument");
  check_path_prec(prec);
  check_storage_prec(bins_prec, "bins_prec");
  if (top_r < 1 || top_r > SQC_MAX_TOPR) raise(SQC_E_ARG, "top_r must be in [1, 64]");
  degrees_match(g, attributed, SQC_LAYOUT_ATTRIBUTED);
  RecursePlan rp = plan_recursion(g, attributed, scope, max_bins_M, top_r, prec, ctx_plans(ctx));
  if (rp.total > SQC_NOALLOC_SCRATCH_BYTES) {
    std::ostringstream s;
    s << "this recursion needs " << rp.total << " bytes of workspace; the allocation-free recursion has "
      << SQC_NOALLOC_SCRATCH_BYTES << " (use sqc_recurse with a caller workspace)";
    raise(SQC_E_NOMEM, s.str());
  }
  char *ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(statics_mu);
    ws = ctx->device >= 0 && ctx->device < kMaxDevices ? statics[ctx->device].scratch : nullptr;
  }
  if (!ws) raise(SQC_E_DEVICE, "the device scratch of this context's device has no address");
  use_device(ctx);
  run_untimed(ctx, describe_recursion(rp, attributed, prec, ws, ctx->unit, bins_dev, bins_prec, top_r, topr_dev,
                                      sum_dev));
  if (masks_out) std::copy(rp.masks.begin(), rp.masks.end(), masks_out);
  return SQC_OK;
  SQC_CATCH(ctx)
}

sqc_status sqc_autotune(sqc_ctx *ctx, const sqc_tensor *attributed, int32_t n_sub, const sqc_cut *cuts,
                        int32_t n_cuts, const sqc_masks *scope, uint64_t max_bins_M, sqc_prec prec,
                        void *bins_dev, sqc_prec bins_prec, int32_t reps, sqc_tune_report *report) {
  SQC_TRY(ctx)
  if (ctx->recording) raise(SQC_E_ARG, "sqc_autotune waits for the device and cannot be recorded");
  Graph g = build_topology(n_sub, cuts, n_cuts);
  if (!attributed || !bins_dev) raise(SQC_E_ARG, "NULL argument");
  if (reps < 1 || reps > 100) raise(SQC_E_ARG, "reps must be in [1, 100]");
  check_path_prec(prec);
  check_storage_prec(bins_prec, "bins_prec");
  degrees_match(g, attributed, SQC_LAYOUT_ATTRIBUTED);
  RecursePlan rp = plan_recursion(g, attributed, scope, max_bins_M, 1, prec, ctx_plans(ctx));
  need_ws(ctx, rp.total);
  use_device(ctx);
  void *top_dev = ctx->ws + kOffSearchTop;
  void *sum_dev = ctx->ws + kOffSearchSum;
  // one full recursion leaves every step's inputs in place
  Launches L = describe_recursion(rp, attributed, prec, ctx->ws, ctx->unit, bins_dev, bins_prec, 1, top_dev,
                                  sum_dev);
  run_direct(ctx, L);
  struct Events {  // returned to the pool on every exit
    sqc_ctx *c;
    hipEvent_t a, b;
    ~Events() {
      c->pool.push_back(a);
      c->pool.push_back(b);
    }
  } ev{ctx, take_event(ctx), take_event(ctx)};
  hipEvent_t e0 = ev.a, e1 = ev.b;
  sqc_tune_report rep{};
  for (size_t si = 0; si < L.steps.size(); ++si) {
    const GemmArgs base = L.steps[si];
    const GemmSpec &used = L.specs[si];
    GemmSpec sp = used;  // the specialisation the tuning table is keyed by
    if (sp.reg == 4) sp.reg = 0;
    const int64_t tiles = gemm_tiles(base);
    // candidates: the tile shapes that apply, for each work-group counts
    // around that kernel's resident capacity, both tile orders when there are
    // several m and n panels
    std::vector<int> shapes{0};
    if (gemm_narrow_ok(base, sp)) shapes.push_back(1);
    std::vector<int> orders{base.nmajor};
    if (base.mbits > 6 && base.nbits > 6) orders.push_back(1 - base.nmajor);
    double best = 0.0, dflt = 0.0;
    GemmTuning pick{L.groups[si], base.nmajor, used.reg == 4 ? 1 : 0};
    for (int nw : shapes) {
      GemmSpec ks = sp;
      if (nw) ks.reg = 4;
      const int cap = gemm_resident_cap(ks);
      std::vector<int> counts;
      for (int64_t c : {int64_t(cap) / 4, int64_t(cap) / 2, int64_t(cap), int64_t(cap) * 2, tiles}) {
        const int v = (int)std::max<int64_t>(1, std::min<int64_t>({c, tiles, int64_t(kMaxGemmGroups)}));
        if (std::find(counts.begin(), counts.end(), v) == counts.end()) counts.push_back(v);
      }
      for (int nm : orders)
        for (int cnt : counts) {
          GemmArgs gg = base;
          gg.nmajor = nm;
          launch_gemm_spec(gg, ks, cnt, ctx->stream);  // warm
          check_hip(hipEventRecord(e0, ctx->stream), "hipEventRecord");
          for (int r = 0; r < reps; ++r) launch_gemm_spec(gg, ks, cnt, ctx->stream);
          check_hip(hipEventRecord(e1, ctx->stream), "hipEventRecord");
          after_launch("tuning launch");
          check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
          float ms = 0.f;
          check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
          const double us = 1e3 * ms / reps;
          const bool is_default = ks.reg == used.reg && nm == base.nmajor && cnt == L.groups[si];
          if (is_default) dflt = us;
          ++rep.candidates;
          if (best == 0.0 || us < best) {
            best = us;
            pick = GemmTuning{cnt, nm, nw};
          }
        }
    }
    if (si < 64) {
      rep.step_tile[si] = pick.narrow;
      rep.step_groups[si] = pick.groups;
      rep.step_nmajor[si] = pick.nmajor;
    }
    gemm_tune_store(base, sp, pick);
    rep.default_us += dflt;
    rep.tuned_us += best;
    ++rep.steps;
  }
  // leave the outputs of the tuned launches
  run_direct(ctx, describe_recursion(rp, attributed, prec, ctx->ws, ctx->unit, bins_dev, bins_prec, 1, top_dev,
                                     sum_dev));
  if (report) *report = rep;
  return SQC_OK;
  SQC_CATCH(ctx)
}

sqc_status sqc_autotune_reset(void) {
  gemm_tune_reset();
  return SQC_OK;
}

int32_t sqc_autotune_entries(void) { return (int32_t)gemm_tune_size(); }

size_t sqc_search_workspace_bytes(const sqc_tensor *attributed, int32_t n_sub, const sqc_cut *cuts,
                                  int32_t n_cuts, uint64_t max_bins_M, int32_t max_recursions, sqc_prec prec,
                                  int32_t max_solutions) {
  try {
    Graph g = build_topology(n_sub, cuts, n_cuts);
    if (!attributed) return 0;
    if (max_recursions < 1 || max_recursions > SQC_MAX_TOPR) raise(SQC_E_ARG, "max_recursions must be in [1, 64]");
    check_path_prec(prec);
    degrees_match(g, attributed, SQC_LAYOUT_ATTRIBUTED);
    sqc_ctx probe;  // sizes only: no device memory is touched
    char *fake = reinterpret_cast<char *>(uintptr_t(1) << 40);
    probe.ws = fake;
    probe.unit = reinterpret_cast<double *>(fake);
    SearchPlan sp = plan_search(&probe, g, attributed, max_bins_M, max_recursions, prec, fake, SQC_F64,
                                max_solutions);
    delete static_cast<PlanCache *>(probe.plan_cache);
    return align256(sp.rec_ws) + sp.region;
  } catch (const Error &e) {
    set_thread_error(e.msg);
    return 0;
  }
}

sqc_status sqc_search(sqc_ctx *ctx, const sqc_tensor *attributed, int32_t n_sub, const sqc_cut *cuts,
                      int32_t n_cuts, uint64_t max_bins_M, int32_t max_recursions, sqc_prec prec,
                      void *bins_dev, sqc_prec bins_prec, sqc_found *solutions,
                      uint64_t *solution_states, int32_t max_solutions, int32_t *n_solutions,
                      sqc_recursion_info *info, int32_t *n_recursions) {
  SQC_TRY(ctx)
  if (ctx->recording) raise(SQC_E_ARG, "sqc_search waits for the device and cannot be recorded");
  Graph g = build_topology(n_sub, cuts, n_cuts);
  if (!attributed || !bins_dev || !n_solutions || !n_recursions) raise(SQC_E_ARG, "NULL argument");
  if (max_solutions > 0 && (!solutions || !solution_states)) raise(SQC_E_ARG, "NULL solution buffers");
  check_path_prec(prec);
  check_storage_prec(bins_prec, "bins_prec");
  const int R = max_recursions;
  if (R < 1 || R > SQC_MAX_TOPR) raise(SQC_E_ARG, "max_recursions must be in [1, 64]");
  degrees_match(g, attributed, SQC_LAYOUT_ATTRIBUTED);
  if (!ctx->ws) raise(SQC_E_NOMEM, "no workspace: call sqc_ctx_set_workspace first");
  if (n_sub > kStepMaxSub) raise(SQC_E_UNSUPPORTED, "the search supports up to 64 subcircuits");
  use_device(ctx);
  SearchPlan sp = plan_search(ctx, g, attributed, max_bins_M, R, prec, bins_dev, bins_prec, max_solutions);
  need_ws(ctx, align256(sp.rec_ws) + sp.region);
  char *B = sp.base;
  check_hip(hipMemcpyAsync(B, sp.upload.data(), sp.upload.size(), hipMemcpyHostToDevice, ctx->stream),
            "hipMemcpyAsync of the search tables");
  SearchArgs a{};
  a.st = reinterpret_cast<SearchState *>(B + sp.o_state);
  a.F = reinterpret_cast<uint64_t *>(B + sp.o_F);
  char *Lb = B + sp.o_L;
  const size_t L2 = 2 * (size_t)R;
  a.Lp = reinterpret_cast<double *>(Lb);
  a.Lb = reinterpret_cast<uint64_t *>(Lb + 8 * 2 * L2);
  a.LF = reinterpret_cast<uint64_t *>(Lb + 16 * 2 * L2);
  a.Lr = reinterpret_cast<int *>(Lb + (16 + 8 * (size_t)n_sub) * 2 * L2);
  a.Ld = a.Lr + 2 * L2;
  a.dep = reinterpret_cast<const SearchDepth *>(B + sp.o_dep);
  a.abits = reinterpret_cast<const int *>(B + sp.o_abits);
  a.active = reinterpret_cast<const uint64_t *>(B + sp.o_active);
  a.patch = reinterpret_cast<const SearchPatch *>(B + sp.o_patch);
  a.images = reinterpret_cast<const unsigned char *>(B + sp.o_images);
  a.live = reinterpret_cast<unsigned char *>(B + sp.o_live);
  a.live_bytes = (int64_t)sp.live_bytes;
  a.res_top = reinterpret_cast<double *>(B + sp.o_res);
  a.res_sum = a.res_top + (size_t)(R + 1) * 2 * R;
  a.info = reinterpret_cast<sqc_recursion_info *>(B + sp.o_info);
  a.sols = reinterpret_cast<sqc_found *>(B + sp.o_sols);
  a.sol_states = reinterpret_cast<uint64_t *>(B + sp.o_states);
  a.n_sub = n_sub;
  a.R = R;
  a.max_sol = sp.max_sol;
  a.D = sp.D;
  // every recursion back to back: the grouped launches read the live tables
  for (int r = 0; r < R; ++r) {
    for (const LiveGroup &lg : sp.groups) {
      const int *grid = r == 0 ? lg.grid0 : lg.grid1;
      const char *J = B + sp.o_live + lg.jobs;
      const int *S0 = reinterpret_cast<const int *>(B + sp.o_live + lg.start[0]);
      const int *S1 = reinterpret_cast<const int *>(B + sp.o_live + lg.start[1]);
      if (lg.kind <= 1) {
        if (grid[0] > 0)
          launch_merge_grouped(lg.kind == 0 ? 0 : 1, reinterpret_cast<const MergeArgs *>(J), S0, lg.cap, grid[0],
                               ctx->stream);
        if (lg.kind == 1 && grid[1] > 0)
          launch_merge_grouped(2, reinterpret_cast<const MergeArgs *>(J), S1, lg.cap, grid[1], ctx->stream);
      } else if (lg.kind == 2) {
        if (grid[0] > 0)
          launch_gemm_grouped(lg.spec, reinterpret_cast<const GemmArgs *>(J), S0, lg.cap, grid[0], ctx->stream);
      } else if (grid[0] > 0) {
        launch_topr_grouped(reinterpret_cast<const TopRArgs *>(J), S0, lg.cap, grid[0], bins_prec == SQC_F32,
                            ctx->stream);
      }
    }
    hipLaunchKernelGGL(search_step, dim3(1), dim3(kStepThreads), 0, ctx->stream, a, r, r == R - 1 ? 1 : 0);
    after_launch("search kernel launch");
  }
  // one wait: the records, the solutions and the counts
  std::vector<unsigned char> back(sp.region - sp.o_info);
  SearchState st{};
  check_hip(hipMemcpyAsync(back.data(), B + sp.o_info, back.size(), hipMemcpyDeviceToHost, ctx->stream),
            "hipMemcpyAsync of the search results");
  check_hip(hipMemcpyAsync(&st, B + sp.o_state, sizeof(st), hipMemcpyDeviceToHost, ctx->stream),
            "hipMemcpyAsync of the search state");
  check_hip(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  const unsigned char *bk = back.data();
  if (info)
    std::memcpy(info, bk, sizeof(sqc_recursion_info) * st.nrec);
  const int nsol = std::min(st.nsol, std::max(0, max_solutions));
  if (nsol > 0) {
    std::memcpy(solutions, bk + (sp.o_sols - sp.o_info), sizeof(sqc_found) * nsol);
    std::memcpy(solution_states, bk + (sp.o_states - sp.o_info), sizeof(uint64_t) * nsol * n_sub);
  }
  *n_solutions = nsol;
  *n_recursions = st.nrec;
  return SQC_OK;
  SQC_CATCH(ctx)
}

}  // extern "C"
