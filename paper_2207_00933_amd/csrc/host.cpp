// Host-side logic of libsqc: compute-graph validation, Algorithm 2 as bit
// masks, the Sec. 6.2 cost model, the pairwise contraction planner and the
// Sec. 6.3 slicing heuristic.  Nothing here touches the GPU.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <set>
#include <sstream>

#include "common.hpp"

namespace sqc {

static thread_local std::string g_thread_err;
void set_thread_error(const std::string &m) { g_thread_err = m; }
const char *thread_error() { return g_thread_err.c_str(); }

[[noreturn]] static void raise(sqc_status c, const std::string &m) { throw Error{c, m}; }

static int popcount64(uint64_t v) { return __builtin_popcountll(v); }

uint64_t deposit_bits(uint64_t v, uint64_t mask) {
  uint64_t out = 0;
  for (int b = 0; mask; ++b) {
    uint64_t low = mask & (~mask + 1);
    if ((v >> b) & 1) out |= low;
    mask ^= low;
  }
  return out;
}

uint64_t extract_bits(uint64_t x, uint64_t mask) {
  uint64_t out = 0;
  int b = 0;
  while (mask) {
    uint64_t low = mask & (~mask + 1);
    if (x & low) out |= uint64_t(1) << b;
    ++b;
    mask ^= low;
  }
  return out;
}

Graph build_topology(int n_sub, const sqc_cut *cuts, int n_cuts) {
  Graph g;
  if (n_sub < 1 || n_sub > 64) raise(SQC_E_ARG, "n_sub must be in [1, 64]");
  if (n_cuts < 0) raise(SQC_E_ARG, "n_cuts must be >= 0");
  if (n_cuts > 0 && !cuts) raise(SQC_E_ARG, "cuts is NULL");
  g.n_sub = n_sub;
  g.n_cuts = n_cuts;
  g.cuts.assign(cuts, cuts + n_cuts);
  g.subs.resize(n_sub);
  for (int k = 0; k < n_cuts; ++k) {
    const sqc_cut &c = cuts[k];
    if (c.up_sub < 0 || c.up_sub >= n_sub || c.down_sub < 0 || c.down_sub >= n_sub) {
      std::ostringstream s;
      s << "cut " << k << " names a subcircuit outside [0, " << n_sub << ")";
      raise(SQC_E_SHAPE, s.str());
    }
    if (c.up_sub == c.down_sub) {
      std::ostringstream s;
      s << "cut " << k << " joins subcircuit " << c.up_sub << " to itself";
      raise(SQC_E_SHAPE, s.str());
    }
  }
  for (int k = 0; k < n_cuts; ++k) {
    SubInfo &up = g.subs[cuts[k].up_sub];
    up.inc.push_back(k);
    up.role.push_back(1);
    up.n_out++;
    SubInfo &dn = g.subs[cuts[k].down_sub];
    dn.inc.push_back(k);
    dn.role.push_back(0);
    dn.n_in++;
  }
  for (int i = 0; i < n_sub; ++i) {
    SubInfo &s = g.subs[i];
    if ((int)s.inc.size() > SQC_MAX_DEGREE) {
      std::ostringstream m;
      m << "subcircuit " << i << " has degree " << s.inc.size() << " > "
        << SQC_MAX_DEGREE;
      raise(SQC_E_SHAPE, m.str());
    }
    s.variants = 1;
    for (int r : s.role) s.variants *= (r == 0 ? 4 : 3);
  }
  return g;
}

Graph build_graph(const sqc_sub *subs, int n_sub, const sqc_cut *cuts, int n_cuts) {
  if (!subs) raise(SQC_E_ARG, "subs is NULL");
  Graph g = build_topology(n_sub, cuts, n_cuts);
  for (int i = 0; i < n_sub; ++i) {
    const sqc_sub &s = subs[i];
    SubInfo &si = g.subs[i];
    std::ostringstream m;
    if (s.n_wires < 1 || s.n_wires > kMaxWires) {
      m << "subcircuit " << i << ": n_wires " << s.n_wires << " outside [1, " << kMaxWires << "]";
      raise(SQC_E_SHAPE, m.str());
    }
    if (s.n_data < 0 || s.n_data > s.n_wires || s.n_data > SQC_MAX_DATA_BITS) {
      m << "subcircuit " << i << ": n_data " << s.n_data << " invalid";
      raise(SQC_E_SHAPE, m.str());
    }
    if (s.n_data > 0 && !s.data_wire) {
      m << "subcircuit " << i << ": data_wire is NULL";
      raise(SQC_E_ARG, m.str());
    }
    si.w = s.n_wires;
    si.d = s.n_data;
    si.data_wire.assign(s.data_wire, s.data_wire + s.n_data);
  }
  for (int i = 0; i < n_sub; ++i) {
    SubInfo &si = g.subs[i];
    std::vector<int> role(si.w, 0);  // 1 data, 2 out-cut
    std::vector<int> init(si.w, 0);
    for (int j = 0; j < si.d; ++j) {
      int t = si.data_wire[j];
      if (t < 0 || t >= si.w || role[t]) {
        std::ostringstream m;
        m << "subcircuit " << i << ": data wire " << t << " out of range or repeated";
        raise(SQC_E_SHAPE, m.str());
      }
      role[t] = 1;
    }
    for (size_t j = 0; j < si.inc.size(); ++j) {
      const sqc_cut &c = g.cuts[si.inc[j]];
      if (si.role[j] == 1) {
        int t = c.up_wire;
        if (t < 0 || t >= si.w || role[t]) {
          std::ostringstream m;
          m << "cut " << si.inc[j] << ": up_wire " << t
            << " out of range, a data wire, or measured twice";
          raise(SQC_E_SHAPE, m.str());
        }
        role[t] = 2;
      } else {
        int t = c.down_wire;
        if (t < 0 || t >= si.w || init[t]) {
          std::ostringstream m;
          m << "cut " << si.inc[j] << ": down_wire " << t
            << " out of range or initialised twice";
          raise(SQC_E_SHAPE, m.str());
        }
        init[t] = 1;
      }
    }
    for (int t = 0; t < si.w; ++t) {
      if (!role[t]) {
        std::ostringstream m;
        m << "subcircuit " << i << ": wire " << t
          << " is neither a data wire nor measured into a cut";
        raise(SQC_E_SHAPE, m.str());
      }
    }
  }
  return g;
}

void assign_bins(int n_sub, const int *n_data, const sqc_masks *scope, uint64_t M,
                 sqc_masks *out) {
  if (n_sub < 1 || !n_data || !out) raise(SQC_E_ARG, "assign_bins: bad arguments");
  if (M < 1) raise(SQC_E_ARG, "max_bins_M must be >= 1");
  int logM = 63 - __builtin_clzll(M);
  std::vector<uint64_t> unfixed(n_sub);
  std::vector<int> e(n_sub);
  for (int i = 0; i < n_sub; ++i) {
    if (n_data[i] < 0 || n_data[i] > SQC_MAX_DATA_BITS) raise(SQC_E_SHAPE, "n_data out of range");
    uint64_t dmask = n_data[i] == 64 ? ~0ull : ((uint64_t(1) << n_data[i]) - 1);
    uint64_t fixed = 0;
    if (scope) {
      fixed = scope[i].fixed;
      if ((fixed & ~dmask) || (scope[i].fixed_val & ~fixed)) {
        std::ostringstream m;
        m << "scope of subcircuit " << i << " has bits outside its data bits";
        raise(SQC_E_SHAPE, m.str());
      }
    }
    unfixed[i] = dmask & ~fixed;
    e[i] = popcount64(unfixed[i]);
  }
  int total = 0;
  for (int v : e) total += v;
  while (total > logM) {
    int im = 0;
    for (int i = 1; i < n_sub; ++i)
      if (e[i] > e[im]) im = i;
    e[im] -= 1;  // ceil(2^e / 2) = 2^(e-1) for e >= 1; total > logM >= 0 so e[im] >= 1
    total -= 1;
  }
  for (int i = 0; i < n_sub; ++i) {
    uint64_t act = 0, rest = unfixed[i];
    for (int k = 0; k < e[i]; ++k) {
      uint64_t low = rest & (~rest + 1);
      act |= low;
      rest ^= low;
    }
    out[i].fixed = scope ? scope[i].fixed : 0;
    out[i].fixed_val = scope ? scope[i].fixed_val : 0;
    out[i].active = act;
    out[i].merged = rest;
  }
}

// ---------------------------------------------------------------------------
// planner
// ---------------------------------------------------------------------------

static int64_t axis_stride(const PTensor &t, size_t j) {
  int sh = 0;
  for (size_t q = 0; q < j; ++q) sh += t.axes[q].bits;
  return int64_t(1) << sh;
}

static int find_axis(const PTensor &t, int kind, int id) {
  for (size_t j = 0; j < t.axes.size(); ++j)
    if (t.axes[j].kind == kind && t.axes[j].id == id) return (int)j;
  return -1;
}

static int min_bins_sub(const PTensor &t) {
  int best = std::numeric_limits<int>::max();
  for (auto &a : t.axes)
    if (a.kind == 0) best = std::min(best, a.id);
  return best;
}

static void push_run(IndexMap &m, int bits, int64_t sx, int64_t sy) {
  if (bits == 0) return;
  if (m.nruns > 0) {
    int r = m.nruns - 1;
    if (m.sx[r] << m.bits[r] == sx && m.sy[r] << m.bits[r] == sy) {
      m.bits[r] += bits;
      return;
    }
  }
  if (m.nruns == kMaxRuns) raise(SQC_E_UNSUPPORTED, "contraction step needs too many index runs");
  m.bits[m.nruns] = bits;
  m.sx[m.nruns] = sx;
  m.sy[m.nruns] = sy;
  m.lx[m.nruns] = (int32_t)(63 - __builtin_clzll((unsigned long long)sx));
  m.ly[m.nruns] = (int32_t)(63 - __builtin_clzll((unsigned long long)sy));
  m.nruns++;
}

double PTensor::elems_d() const { return std::ldexp(1.0, bits()); }

struct PairEval {
  double result_elems;
  double mults;
  int shared;
};

static PairEval eval_pair(const PTensor &A, const PTensor &B) {
  int sh = 0, shared_bits = 0;
  for (auto &a : A.axes)
    if (a.kind == 1 && find_axis(B, 1, a.id) >= 0) {
      sh++;
      shared_bits += a.bits;
    }
  int bitsA = 0, bitsB = 0;
  for (auto &a : A.axes) bitsA += a.bits;
  for (auto &b : B.axes) bitsB += b.bits;
  PairEval e;
  e.shared = sh;
  e.result_elems = std::ldexp(1.0, bitsA + bitsB - 2 * shared_bits);
  e.mults = std::ldexp(1.0, bitsA + bitsB - shared_bits);
  return e;
}

Plan make_plan(const Graph &g, const std::vector<int> &bits, const int *order,
               int elem_bytes) {
  Plan p;
  for (int i = 0; i < g.n_sub; ++i) {
    PTensor t;
    t.input_sub = i;
    if (bits[i] > 0) t.axes.push_back(Axis{0, i, bits[i]});
    for (int k : g.subs[i].inc) t.axes.push_back(Axis{1, k, 2});
    p.tensors.push_back(t);
  }
  std::vector<int> work;
  for (int i = 0; i < g.n_sub; ++i) work.push_back(i);
  // depth of each tensor in the contraction tree (inputs 0): steps whose
  // operands are all below a depth can share one launch
  std::vector<int> depth(g.n_sub, 0);
  int64_t ws = 0;
  int step_no = 0;
  while (work.size() > 1) {
    int wi = -1, wj = -1;
    if (order) {
      wi = order[2 * step_no];
      wj = order[2 * step_no + 1];
      if (wi < 0 || wj < 0 || wi >= (int)work.size() || wj >= (int)work.size() || wi == wj)
        raise(SQC_E_ARG, "contraction order names an invalid position");
    } else {
      // greedy: connected pairs first, then smallest result, then fewest
      // mults.  Results of at most kSmallStep elements count as one size: a
      // step that small costs its launch latency, not its size, so among
      // them the pair of shallowest operands goes first, which keeps the
      // tree shallow (a chain contracts as a balanced tree rather than a
      // sweep) and lets independent steps share launches.
      constexpr double kSmallStep = 65536.0;
      bool best_conn = false;
      double best_eff = 0, best_size = 0, best_m = 0;
      int best_depth = 0;
      for (size_t i = 0; i < work.size(); ++i)
        for (size_t j = i + 1; j < work.size(); ++j) {
          PairEval e = eval_pair(p.tensors[work[i]], p.tensors[work[j]]);
          bool conn = e.shared > 0;
          const double eff = std::max(e.result_elems, kSmallStep);
          const int dep = std::max(depth[work[i]], depth[work[j]]);
          bool better = false;
          if (wi < 0) better = true;
          else if (conn != best_conn) better = conn;
          else if (eff != best_eff) better = eff < best_eff;
          else if (dep != best_depth) better = dep < best_depth;
          else if (e.result_elems != best_size) better = e.result_elems < best_size;
          else if (e.mults != best_m) better = e.mults < best_m;
          if (better) {
            wi = (int)i;
            wj = (int)j;
            best_conn = conn;
            best_eff = eff;
            best_depth = dep;
            best_size = e.result_elems;
            best_m = e.mults;
          }
        }
    }
    int ta = work[wi], tb = work[wj];
    // GEMM "A" role: the operand holding the lowest subcircuit's bins, so the
    // result's fastest axis comes from the m side
    if (min_bins_sub(p.tensors[tb]) < min_bins_sub(p.tensors[ta])) std::swap(ta, tb);
    const PTensor A = p.tensors[ta];
    const PTensor B = p.tensors[tb];
    PTensor C;
    std::vector<Axis> bins_ax, lab_ax;
    std::set<int> shared;
    for (auto &a : A.axes) {
      if (a.kind == 0) bins_ax.push_back(a);
      else if (find_axis(B, 1, a.id) >= 0) shared.insert(a.id);
      else lab_ax.push_back(a);
    }
    for (auto &b : B.axes) {
      if (b.kind == 0) bins_ax.push_back(b);
      else if (!shared.count(b.id)) lab_ax.push_back(b);
    }
    std::sort(bins_ax.begin(), bins_ax.end(), [](const Axis &x, const Axis &y) { return x.id < y.id; });
    std::sort(lab_ax.begin(), lab_ax.end(), [](const Axis &x, const Axis &y) { return x.id < y.id; });
    C.axes = bins_ax;
    C.axes.insert(C.axes.end(), lab_ax.begin(), lab_ax.end());
    if (elem_bytes > 0 && (C.bits() > 40 || A.bits() > 40 || B.bits() > 40))
      raise(SQC_E_UNSUPPORTED, "contraction needs a tensor larger than 2^40 elements");
    Step st;
    st.a = ta;
    st.b = tb;
    st.mbits = st.nbits = st.kbits = 0;
    for (size_t j = 0; j < A.axes.size(); ++j) {
      const Axis &a = A.axes[j];
      if (a.kind == 1 && shared.count(a.id)) continue;
      int jc = find_axis(C, a.kind, a.id);
      if (elem_bytes > 0) push_run(st.m, a.bits, axis_stride(A, j), axis_stride(C, jc));
      st.mbits += a.bits;
    }
    for (size_t j = 0; j < B.axes.size(); ++j) {
      const Axis &b = B.axes[j];
      if (b.kind == 1 && shared.count(b.id)) continue;
      int jc = find_axis(C, b.kind, b.id);
      if (elem_bytes > 0) push_run(st.n, b.bits, axis_stride(B, j), axis_stride(C, jc));
      st.nbits += b.bits;
    }
    for (int id : shared) {
      int ja = find_axis(A, 1, id), jb = find_axis(B, 1, id);
      if (elem_bytes > 0) push_run(st.k, 2, axis_stride(A, ja), axis_stride(B, jb));
      st.kbits += 2;
    }
    st.mults = std::ldexp(1.0, st.mbits + st.nbits + st.kbits);
    p.mults += st.mults;
    p.max_step_operands = std::max(p.max_step_operands, A.elems_d() + B.elems_d());
    bool last = work.size() == 2;
    if (!last) {
      if (elem_bytes > 0) {
        C.ws_offset = ws;
        ws += ((C.elems() * elem_bytes + 255) / 256) * 256;
      }
      p.max_intermediate = std::max(p.max_intermediate, C.elems_d());
    }
    int tc = (int)p.tensors.size();
    p.tensors.push_back(C);
    depth.push_back(std::max(depth[ta], depth[tb]) + 1);
    st.c = tc;
    p.steps.push_back(st);
    // working list: result replaces position wi, position wj is removed
    work[wi] = tc;
    work.erase(work.begin() + wj);
    ++step_no;
  }
  p.inter_bytes = ws;
  int ob = 0;
  for (auto &a : p.tensors[work[0]].axes) {
    if (a.kind != 0) raise(SQC_E_SHAPE, "a cut label was left uncontracted");
    ob += a.bits;
  }
  p.out_bits = ob;
  return p;
}

}  // namespace sqc

// ---------------------------------------------------------------------------
// host-only C entry points
// ---------------------------------------------------------------------------
using namespace sqc;

#define SQC_HOST_TRY try {
#define SQC_HOST_CATCH                         \
  }                                            \
  catch (const Error &e) {                     \
    set_thread_error(e.msg);                   \
    return e.code;                             \
  }                                            \
  catch (const std::exception &e) {            \
    set_thread_error(e.what());                \
    return SQC_E_ARG;                          \
  }

extern "C" sqc_status sqc_check_graph(const sqc_sub *subs, int32_t n_sub,
                                      const sqc_cut *cuts, int32_t n_cuts) {
  SQC_HOST_TRY
  build_graph(subs, n_sub, cuts, n_cuts);
  set_thread_error("");
  return SQC_OK;
  SQC_HOST_CATCH
}

extern "C" sqc_status sqc_assign_bins(int32_t n_sub, const int32_t *n_data,
                                      const sqc_masks *scope, uint64_t max_bins_M,
                                      sqc_masks *out) {
  SQC_HOST_TRY
  std::vector<int> nd(n_data, n_data + (n_sub > 0 ? n_sub : 0));
  assign_bins(n_sub, nd.data(), scope, max_bins_M, out);
  return SQC_OK;
  SQC_HOST_CATCH
}

extern "C" sqc_status sqc_bin_scope(int32_t n_sub, const sqc_masks *masks, uint64_t bin,
                                    sqc_masks *scope_out) {
  SQC_HOST_TRY
  if (n_sub < 1 || !masks || !scope_out) raise(SQC_E_ARG, "bin_scope: bad arguments");
  int total = 0;
  for (int i = 0; i < n_sub; ++i) total += popcount64(masks[i].active);
  if (total < 64 && (bin >> total) != 0) raise(SQC_E_ARG, "bin index exceeds the bin count");
  uint64_t rem = bin;
  for (int i = 0; i < n_sub; ++i) {
    int a = popcount64(masks[i].active);
    uint64_t beta = a == 64 ? rem : (rem & ((uint64_t(1) << a) - 1));
    rem = a == 64 ? 0 : (rem >> a);
    scope_out[i].fixed = masks[i].fixed | masks[i].active;
    scope_out[i].fixed_val = masks[i].fixed_val | deposit_bits(beta, masks[i].active);
    scope_out[i].active = 0;
    scope_out[i].merged = masks[i].merged;
  }
  return SQC_OK;
  SQC_HOST_CATCH
}

extern "C" sqc_status sqc_plan_cost(int32_t n_sub, const int32_t *out_bits,
                                    const sqc_cut *cuts, int32_t n_cuts,
                                    const int32_t *order, sqc_cost *out) {
  SQC_HOST_TRY
  if (!out_bits || !out) raise(SQC_E_ARG, "plan_cost: NULL argument");
  if (n_sub > 65) raise(SQC_E_UNSUPPORTED, "plan_cost: at most 65 subcircuits");
  Graph g = build_topology(n_sub, cuts, n_cuts);
  std::vector<int> bits(out_bits, out_bits + n_sub);
  for (int b : bits)
    if (b < 0 || b > SQC_MAX_DATA_BITS) raise(SQC_E_SHAPE, "out_bits out of range");
  Plan p = make_plan(g, bits, order, 0);
  std::memset(out, 0, sizeof(*out));
  double inputs = 0;
  for (int i = 0; i < n_sub; ++i) inputs += p.tensors[i].elems_d();
  out->input_floats = inputs;
  out->plan_mults = p.mults;
  out->max_step_operand_floats = p.max_step_operands;
  out->max_intermediate_floats = p.max_intermediate;
  double per_term = 0, acc = std::ldexp(1.0, bits[0]);
  for (int i = 1; i < n_sub; ++i) {
    per_term += acc * std::ldexp(1.0, bits[i]);
    acc *= std::ldexp(1.0, bits[i]);
  }
  out->naive_mults = std::ldexp(per_term, 2 * n_cuts);
  out->n_steps = (int)p.steps.size();
  // record the order as positions in the working list
  std::vector<int> work;
  for (int i = 0; i < n_sub; ++i) work.push_back(i);
  for (size_t s = 0; s < p.steps.size() && s < 64; ++s) {
    int pa = -1, pb = -1;
    for (size_t q = 0; q < work.size(); ++q) {
      if (work[q] == p.steps[s].a) pa = (int)q;
      if (work[q] == p.steps[s].b) pb = (int)q;
    }
    int lo = std::min(pa, pb), hi = std::max(pa, pb);
    out->order[2 * s] = lo;
    out->order[2 * s + 1] = hi;
    work[lo] = p.steps[s].c;
    work.erase(work.begin() + hi);
  }
  return SQC_OK;
  SQC_HOST_CATCH
}

extern "C" sqc_status sqc_slice_plan(int32_t n_sub, const int32_t *out_bits,
                                     const sqc_cut *cuts, int32_t n_cuts,
                                     double budget_floats, int32_t *sliced,
                                     int32_t *n_sliced) {
  SQC_HOST_TRY
  if (!out_bits || !n_sliced || (n_cuts > 0 && !sliced)) raise(SQC_E_ARG, "slice_plan: NULL argument");
  Graph g = build_topology(n_sub, cuts, n_cuts);
  std::vector<std::set<int>> labs(n_sub);
  for (int i = 0; i < n_sub; ++i) labs[i].insert(g.subs[i].inc.begin(), g.subs[i].inc.end());
  auto total = [&](const std::vector<std::set<int>> &L) {
    double t = 0;
    for (int i = 0; i < n_sub; ++i) t += std::ldexp(1.0, 2 * (int)L[i].size() + out_bits[i]);
    return t;
  };
  int cnt = 0;
  std::vector<bool> gone(n_cuts, false);
  while (total(labs) > budget_floats && cnt < SQC_MAX_SLICED) {
    int best = -1;
    double best_t = 0;
    for (int e = 0; e < n_cuts; ++e) {
      if (gone[e]) continue;
      auto L2 = labs;
      for (auto &s : L2) s.erase(e);
      double t = total(L2);
      if (best < 0 || t < best_t) {
        best = e;
        best_t = t;
      }
    }
    if (best < 0) break;
    gone[best] = true;
    for (auto &s : labs) s.erase(best);
    sliced[cnt++] = best;
  }
  *n_sliced = cnt;
  if (total(labs) > budget_floats) {
    std::ostringstream m;
    m << "slice_plan: " << cnt << " sliced cut(s) leave " << total(labs) << " input floats, above the budget "
      << budget_floats << (cnt == SQC_MAX_SLICED ? " (at most SQC_MAX_SLICED cuts are sliced)" : "");
    raise(SQC_E_NOMEM, m.str());
  }
  return SQC_OK;
  SQC_HOST_CATCH
}

// ---------------------------------------------------------------------------
// cut search (Sec. 5): partition the two-qubit-gate DAG
// ---------------------------------------------------------------------------

namespace {

struct CutSearch {
  int n = 0, n_sub = 0, cap = 0;
  std::vector<std::vector<int>> pred;  // pred[v]: tail gates of v's in-edges (with repeats)
  std::vector<std::vector<int>> adj;   // adj[v]: both ends' other gate, one entry per edge
  std::vector<int> assign, count, deg;
  int L = 0, cut = 0, used = 0;
  std::vector<int> best;
  int best_L = 0, best_cut = 0;
  bool have = false;
  int64_t nodes = 0, max_nodes = 0;
  bool stopped = false;

  bool better(int l, int c) const { return !have || l < best_L || (l == best_L && c < best_cut); }

  // (L, cut edges) of a full assignment; false when it breaks Eq. 2 or
  // leaves a subcircuit empty
  bool score(const std::vector<int> &a, int &l, int &c) const {
    std::vector<int> d(n_sub, 0), cnt(n_sub, 0);
    c = 0;
    for (int v = 0; v < n; ++v) {
      cnt[a[v]]++;
      for (int u : pred[v])
        if (a[u] != a[v]) {
          d[a[u]]++;
          d[a[v]]++;
          c++;
        }
    }
    for (int k : cnt)
      if (k < 1 || k > cap) return false;
    l = 0;
    for (int x : d) l = std::max(l, x);
    return true;
  }

  void evaluate(const std::vector<int> &a) {
    int l, c;
    if (score(a, l, c) && better(l, c)) {
      best = a;
      best_L = l;
      best_cut = c;
      have = true;
    }
  }

  // Single-gate moves that lower (L, cut edges), first improving move per
  // gate, until a sweep moves nothing (at most `passes` sweeps).  A move is
  // scored incrementally: it changes the degrees of at most the two
  // subcircuits involved and those of v's neighbours, and a histogram of
  // degree values gives the new maximum, so one trial costs O(deg v).
  // With more than 32 subcircuits only the neighbours' subcircuits are
  // tried as targets.
  void improve(std::vector<int> &a, int passes) const {
    int l, c;
    if (!score(a, l, c)) return;
    std::vector<int> d(n_sub, 0), cnt(n_sub, 0);
    for (int v = 0; v < n; ++v) {
      cnt[a[v]]++;
      for (int u : pred[v])
        if (a[u] != a[v]) {
          d[a[u]]++;
          d[a[v]]++;
        }
    }
    int top = 0;
    for (int x : d) top = std::max(top, x);
    std::vector<int> hist((size_t)4 * n + 8, 0);  // a degree is at most 4 n
    for (int x : d) hist[x]++;
    // pending degree changes of one trial move (sub, delta), at most 2 + 2|adj|
    std::vector<std::pair<int, int>> ch;
    auto add = [&](int s, int delta) {
      for (auto &p : ch)
        if (p.first == s) {
          p.second += delta;
          return;
        }
      ch.push_back({s, delta});
    };
    std::vector<int> targets;
    for (int p = 0; p < passes; ++p) {
      bool moved = false;
      for (int v = 0; v < n; ++v) {
        const int from = a[v];
        if (cnt[from] <= 1) continue;  // a subcircuit may not become empty
        targets.clear();
        if (n_sub <= 32) {
          for (int t = 0; t < n_sub; ++t) targets.push_back(t);
        } else {
          for (int u : adj[v])
            if (std::find(targets.begin(), targets.end(), a[u]) == targets.end()) targets.push_back(a[u]);
          std::sort(targets.begin(), targets.end());
        }
        for (int to : targets) {
          if (to == from || cnt[to] >= cap) continue;
          ch.clear();
          int dc = 0;
          for (int u : adj[v]) {
            const int s = a[u];
            if (s != from) {  // edge cut now: uncut or re-cut after the move
              add(s, -1);
              add(from, -1);
              dc--;
            }
            if (s != to) {
              add(s, +1);
              add(to, +1);
              dc++;
            }
          }
          // new maximum: changed subcircuits' new degrees, else the largest
          // degree value still held by some unchanged subcircuit
          int nl = 0;
          for (auto &q : ch) {
            hist[d[q.first]]--;
            nl = std::max(nl, d[q.first] + q.second);
          }
          int h = top;
          while (h > nl && hist[h] == 0) --h;
          nl = std::max(nl, h);
          for (auto &q : ch) hist[d[q.first]]++;
          if (nl < l || (nl == l && c + dc < c)) {
            for (auto &q : ch) {
              hist[d[q.first]]--;
              d[q.first] += q.second;
              hist[d[q.first]]++;
            }
            top = std::max(top, nl);
            while (top > 0 && hist[top] == 0) --top;
            cnt[from]--;
            cnt[to]++;
            a[v] = to;
            l = nl;
            c += dc;
            moved = true;
            break;
          }
        }
      }
      if (!moved) break;
    }
  }

  // Branch and bound over the gates in circuit order with an explicit stack
  // (one frame per placed gate), so the depth is bounded by memory, not by
  // the thread's call stack.  Frame k holds the candidate subcircuits of
  // gate k in the order tried (fewest new cut edges first), the one being
  // tried, and what placing it changed.
  struct Frame {
    int next = 0, ncand = 0, chosen = -1;
    int saveL = 0, saveCut = 0, saveUsed = 0;
    int ntouched = 0;
    int touched[2] = {0, 0};
  };

  void dfs() {
    std::vector<Frame> st(n + 1);
    std::vector<int> pool;  // frame v's candidates at [v n_sub, v n_sub + ncand)
    auto fill = [&](int v) {
      Frame &f = st[v];
      f.next = 0;
      f.ncand = 0;
      f.chosen = -1;
      const int top = std::min(used, n_sub - 1);
      std::vector<std::pair<int, int>> cs;
      for (int c = 0; c <= top; ++c) {
        if (count[c] >= cap) continue;
        const int opened = used + (c == used ? 1 : 0);
        if (n - v - 1 < n_sub - opened) continue;  // too few gates left to open the rest
        int add = 0;
        for (int u : pred[v]) add += assign[u] != c;
        cs.push_back({add, c});
      }
      std::stable_sort(cs.begin(), cs.end());
      for (size_t i = 0; i < cs.size(); ++i) pool[(size_t)v * n_sub + i] = cs[i].second;
      f.ncand = (int)cs.size();
    };
    auto undo = [&](int v) {
      Frame &f = st[v];
      if (f.chosen < 0) return;
      const int c = f.chosen;
      count[c]--;
      assign[v] = -1;
      for (int i = 0; i < f.ntouched; ++i) {
        deg[f.touched[i]]--;
        deg[c]--;
      }
      L = f.saveL;
      cut = f.saveCut;
      used = f.saveUsed;
      f.chosen = -1;
    };
    pool.assign((size_t)(n + 1) * n_sub, 0);
    int v = 0;
    if (max_nodes > 0 && ++nodes > max_nodes) {
      stopped = true;
      return;
    }
    fill(0);
    while (v >= 0) {
      Frame &f = st[v];
      undo(v);
      bool descended = false;
      while (f.next < f.ncand) {
        const int c = pool[(size_t)v * n_sub + f.next++];
        int l = L, nt = 0, tt[2] = {0, 0};
        for (int u : pred[v])
          if (assign[u] != c) {
            tt[nt++] = assign[u];
            deg[assign[u]]++;
            deg[c]++;
            l = std::max(l, std::max(deg[assign[u]], deg[c]));
          }
        const int ncut = cut + nt;
        if (!better(l, ncut)) {  // (L, cut) only grow: the subtree cannot win
          for (int i = 0; i < nt; ++i) {
            deg[tt[i]]--;
            deg[c]--;
          }
          continue;
        }
        f.saveL = L;
        f.saveCut = cut;
        f.saveUsed = used;
        f.ntouched = nt;
        f.touched[0] = tt[0];
        f.touched[1] = tt[1];
        f.chosen = c;
        assign[v] = c;
        count[c]++;
        if (c == used) used++;
        L = l;
        cut = ncut;
        if (max_nodes > 0 && ++nodes > max_nodes) {
          stopped = true;
          return;
        }
        if (v + 1 == n) {
          if (used == n_sub && better(L, cut)) {
            best = assign;
            best_L = L;
            best_cut = cut;
            have = true;
          }
          undo(v);
          continue;
        }
        ++v;
        fill(v);
        descended = true;
        break;
      }
      if (!descended) --v;
    }
  }
};

}  // namespace

extern "C" sqc_status sqc_find_cuts(int32_t n_qubits, const int32_t *gates, int32_t n_gates, int32_t n_sub,
                                    double alpha, int64_t max_nodes, int32_t *assign, int32_t *L,
                                    int32_t *n_cut_edges, int32_t *optimal) {
  SQC_HOST_TRY
  if (!gates || !assign || !L || !n_cut_edges || !optimal) raise(SQC_E_ARG, "NULL argument");
  if (n_gates < 1 || n_gates > (1 << 20)) raise(SQC_E_ARG, "n_gates must be in [1, 2^20]");
  if (n_sub < 1 || n_sub > n_gates) raise(SQC_E_ARG, "n_sub must be in [1, n_gates]");
  if (n_qubits < 2) raise(SQC_E_ARG, "n_qubits must be >= 2");
  if (!(alpha > 0.0) || !(alpha <= 1.0)) raise(SQC_E_ARG, "alpha must be in (0, 1]");
  CutSearch s;
  s.n = n_gates;
  s.n_sub = n_sub;
  s.cap = (int)std::floor(alpha * n_gates + 1e-9);
  if ((int64_t)s.cap * n_sub < n_gates || s.cap < 1)
    raise(SQC_E_SHAPE, "no partition meets the load constraint alpha |V|");
  s.pred.resize(n_gates);
  s.adj.resize(n_gates);
  std::vector<int> last(n_qubits, -1);
  for (int v = 0; v < n_gates; ++v) {
    const int a = gates[2 * v], b = gates[2 * v + 1];
    if (a < 0 || a >= n_qubits || b < 0 || b >= n_qubits) raise(SQC_E_ARG, "gate qubit id out of range");
    if (a == b) raise(SQC_E_ARG, "a two-qubit gate acts on one qubit twice");
    for (int q : {a, b}) {
      if (last[q] >= 0) {
        s.pred[v].push_back(last[q]);
        s.adj[v].push_back(last[q]);
        s.adj[last[q]].push_back(v);
      }
      last[q] = v;
    }
  }
  // starts: the contiguous split of the gate order into n_sub blocks, and
  // qubit bands (a gate goes to the band of its lowest qubit), each improved
  // by single-gate moves; the best is the incumbent of the exact search
  const int passes = n_gates <= 4096 ? 64 : 4;
  std::vector<int> a0(n_gates), a1(n_gates);
  for (int v = 0; v < n_gates; ++v) {
    a0[v] = (int)((int64_t)v * n_sub / n_gates);
    const int q = std::min(gates[2 * v], gates[2 * v + 1]);
    a1[v] = (int)((int64_t)q * n_sub / n_qubits);
  }
  s.evaluate(a0);
  s.evaluate(a1);
  s.improve(a0, passes);
  s.evaluate(a0);
  s.improve(a1, passes);
  s.evaluate(a1);
  // iterated local search: perturb the best partition (a few gates moved to
  // random subcircuits, fixed-seed xorshift so results are reproducible),
  // improve it again, keep it when it wins
  if (s.have && n_sub > 1) {
    uint64_t x = 0x9E3779B97F4A7C15ull;
    auto rnd = [&]() {
      x ^= x << 13;
      x ^= x >> 7;
      x ^= x << 17;
      return x;
    };
    const int rounds = n_gates <= 512 ? 200 : 16;
    for (int r = 0; r < rounds; ++r) {
      std::vector<int> a = s.best;
      const int kick = 2 + (int)(rnd() % 4);
      for (int t = 0; t < kick; ++t) a[rnd() % n_gates] = (int)(rnd() % n_sub);
      s.improve(a, passes);
      s.evaluate(a);
    }
  }
  s.assign.assign(n_gates, -1);
  s.count.assign(n_sub, 0);
  s.deg.assign(n_sub, 0);
  s.max_nodes = max_nodes;
  s.dfs();
  if (!s.have) raise(SQC_E_SHAPE, "no partition meets the load constraint alpha |V|");
  for (int v = 0; v < n_gates; ++v) assign[v] = s.best[v];
  *L = s.best_L;
  *n_cut_edges = s.best_cut;
  *optimal = s.stopped ? 0 : 1;
  set_thread_error("");
  return SQC_OK;
  SQC_HOST_CATCH
}
