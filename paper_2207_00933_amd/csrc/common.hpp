// Internal declarations of libsqc: graph bookkeeping, the contraction planner,
// kernel argument blocks and launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sqc.h"

namespace sqc {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error {
  sqc_status code;
  std::string msg;
};

// Per-thread message for context-less calls.
void set_thread_error(const std::string &m);
const char *thread_error();

// ---------------------------------------------------------------------------
// compute graph
// ---------------------------------------------------------------------------
struct SubInfo {
  int w = 0;                    // wires
  int d = 0;                    // data bits
  std::vector<int> data_wire;   // data bit j -> wire
  std::vector<int> inc;         // incident cut ids, global order
  std::vector<int> role;        // per incident cut: 0 = in (down), 1 = out (up)
  int n_in = 0, n_out = 0;
  int64_t variants = 1;         // 4^n_in * 3^n_out
};

struct Graph {
  int n_sub = 0;
  int n_cuts = 0;
  std::vector<sqc_cut> cuts;
  std::vector<SubInfo> subs;
};

// Topology only (cut endpoints, incident lists, degree cap).  Throws Error.
Graph build_topology(int n_sub, const sqc_cut *cuts, int n_cuts);
// Full validation including wires and data wires.  Throws Error.
Graph build_graph(const sqc_sub *subs, int n_sub, const sqc_cut *cuts, int n_cuts);

// Algorithm 2 as masks (see sqc_assign_bins).  Throws Error.
void assign_bins(int n_sub, const int *n_data, const sqc_masks *scope, uint64_t M,
                 sqc_masks *out);
uint64_t deposit_bits(uint64_t v, uint64_t mask);
uint64_t extract_bits(uint64_t x, uint64_t mask);

// ---------------------------------------------------------------------------
// contraction plan
// ---------------------------------------------------------------------------
constexpr int kMaxRuns = 12;

// One index space (m, n or k) split into runs of bits; each run has a stride in
// two operands (X and Y).  index -> offset_X = sum_r ((idx >> shift_r) &
// (2^bits_r - 1)) * sx[r], the same with sy for operand Y.
struct IndexMap {
  int nruns = 0;
  int bits[kMaxRuns] = {0};
  int64_t sx[kMaxRuns] = {0};
  int64_t sy[kMaxRuns] = {0};
  // log2 of sx / sy: every stride is a product of power-of-two dimensions
  int32_t lx[kMaxRuns] = {0};
  int32_t ly[kMaxRuns] = {0};
};

struct Axis {
  int kind;  // 0 = bins of subcircuit `id`, 1 = label of cut `id`
  int id;
  int bits;
};

struct PTensor {
  std::vector<Axis> axes;  // memory order, fastest first
  int input_sub = -1;      // >= 0: merged input tensor of this subcircuit
  int64_t ws_offset = -1;  // intermediate: byte offset in the workspace
  int bits() const {
    int b = 0;
    for (auto &a : axes) b += a.bits;
    return b;
  }
  // element count (only for tensors that exist: at most 2^40 elements)
  int64_t elems() const { return int64_t(1) << bits(); }
  double elems_d() const;
};

struct Step {
  int a, b, c;       // tensor table indices; a plays the GEMM "A" role
  int mbits, nbits, kbits;
  IndexMap m, n, k;  // m: (A, C), n: (B, C), k: (A, B)
  double mults;      // product of all dimensions involved (Sec. 6.2)
};

struct Plan {
  std::vector<PTensor> tensors;  // inputs first (n_sub), then step results
  std::vector<Step> steps;
  int out_bits = 0;
  double mults = 0, max_intermediate = 0, max_step_operands = 0;
  int64_t inter_bytes = 0;  // workspace for intermediates at the plan's element size
};

// Build the greedy pairwise plan for merged tensors with `bits[i]` active bits.
// If `order` is non-null it gives the pairs to use (positions in a working list).
// elem_bytes > 0 sizes the workspace for intermediates (and rejects plans whose
// intermediates exceed 2^40 elements); elem_bytes == 0 only costs the plan.
Plan make_plan(const Graph &g, const std::vector<int> &bits, const int *order,
               int elem_bytes);

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
constexpr int kMaxWires = 32;  // outcome indices fit 32 bits
constexpr int kMaxIncident = SQC_MAX_DEGREE;

struct AttrArgs {
  const void *var;   // [V][2^w]
  void *out;         // [2^d][4^c], or [4^c][2^d] when out_merged
  int in_f32, out_f32;
  int w, d, c;
  int n_in, n_out;
  int xt_bits;                 // log2 of the x-tile
  int in_pos[kMaxIncident];    // incident position of the j-th in-cut
  int out_pos[kMaxIncident];   // incident position of the j-th out-cut
  int64_t place[kMaxIncident]; // variant mixed-radix place value per incident cut
  int out_wire[kMaxIncident];  // wire of the j-th out-cut
  int data_wire[64];
  double scale;                // 2^-n_out
  // 1: written in the merged layout of a recursion that keeps every data bit
  // active ([4^c][2^d], bins fastest): the attribution and that recursion's
  // merge (a transposition) in one pass
  int out_merged;
};
// Enqueue the attribution of n subcircuits (those that fit the LDS stage
// share launches of up to kAttrJobs jobs).
constexpr int kAttrJobs = 4;
void launch_attributes(const AttrArgs *jobs, int n, hipStream_t s);

struct MergeArgs {
  const void *in;   // attributed [2^d][L]
  void *out;        // merged [L][2^a] (or partials [P][2^a][L] when P > 1)
  double *partial;  // workspace for y-split partials
  int in_f32, out_f32;
  int d, lbits;     // L = 2^lbits = 4^c
  int abits, mbits; // active, merged bit counts
  uint64_t fixed_val, active, merged;
  int act_lo;       // active bits form one run starting here (-1: not a run)
  int mrg_lo;       // merged bits form one run starting here (-1: not a run)
  int ysplit_bits;  // P = 2^ysplit_bits
  int tb_bits;      // log2 of the b-tile
  int ts_bits;      // log2 of the sigma-tile
  int64_t grid_x;   // work-groups along the outputs (set by the launcher)
  int64_t blocks;   // work-groups of the main pass
  int64_t fin_blocks;  // work-groups of the partial-sum pass (0: none)
  // label rows of one slice (first-level slicing): the input rows hold
  // 2^in_lbits labels, and output label s reads input label
  // lab_fixed | deposit(s, lab_keep).  Unsliced: in_lbits = lbits,
  // lab_fixed = 0, lab_keep = 2^lbits - 1.
  int in_lbits;
  uint64_t lab_fixed, lab_keep;
};
// Labels a merge_rows thread reads as one vector: 4 consecutive output labels
// are 4 consecutive input labels when the lowest label digit is kept.
__host__ __device__ inline int merge_vec(const MergeArgs &a) {
  return a.lbits >= 2 && (a.in_lbits == a.lbits || (a.lab_keep & 3) == 3) ? 4 : 1;
}
// Merges launched together (at most this many per launch; more are split).
constexpr int kMergeJobs = 8;
// Enqueue n merges; jobs with merged bits >= 6 need their own partial buffer.
void launch_merges(const MergeArgs *jobs, int n, hipStream_t s);
// For batched launches from a device table: set a job's grid shape (as
// launch_merges does), its work-groups in pass 0 (merged bits < 6), 1 (the
// streaming reduction, merged bits >= 6) or 2 (its partial sums), and launch
// one pass over n shaped jobs, job j taking work-groups [start[j], start[j + 1]).
void merge_shape(MergeArgs &a);
int64_t merge_pass_blocks(const MergeArgs &a, int pass);
void launch_merge_grouped(int pass, const MergeArgs *jobs_dev, const int *start_dev, int n, int total,
                          hipStream_t s);
// out[r] = max_c |in[r * cols + c]| (FP64) for a merged tensor [rows][cols].
void launch_row_absmax(const void *in, int in_f32, double *out, int64_t rows, int64_t cols, hipStream_t s);
// FP64 partial-sum elements the merge of these bit counts needs (0: none).
int64_t merge_partial_elems(int abits, int lbits, int mbits);

struct GemmArgs {
  const void *A;
  const void *B;
  void *C;
  int mbits, nbits, kbits;
  IndexMap m, n, k;
  int out_f32;           // output element type (intermediates follow the path)
  int final_step;        // 1: compensated FP64 fold of the FP32 sums of K stages
  int nmajor;            // tile order: 0 = m panels outer (A panel read once), 1 = n panels outer
  // statistics of every 32 x 32 sub-tile (final step of a recursion)
  int stats;
  double *blk_max;       // [4 * tiles] largest stored bin of each 32 x 32 sub-tile
  double *wg_stats;      // [3 * work-groups] per work-group: FP64 sum, its
                         // compensation, largest stored bin (work-group g owns
                         // a contiguous chunk of the tiles, chunks in order)
  // slices of a sliced contraction (final step only): the result is added
  // into FP64 running sums acc_sum/acc_comp (laid out as C) with Neumaier
  // compensation.  1: the first slice starts them; 2: a later slice adds;
  // 3: the last slice adds and writes sum + compensation to C (statistics
  // from the written values).  0: plain store.
  int acc_mode;
  double *acc_sum, *acc_comp;
  // filled by launch_gemm: offsets of the low index bits the kernel adds to
  // a wave's origin (index maps are linear in disjoint bit fields)
  int64_t koff_a[16];    // A offset of k = 0..15
  int64_t koff_b[16];    // B offset of k = 0..15
  int64_t coff_n[16];    // C offset of each accumulator element's n
  int64_t coff_m16;      // C offset of m = 16
};
// 64 x 64 output tiles of a GEMM (sub-tile statistics: 4 per tile).
int64_t gemm_tiles(const GemmArgs &g);
// Tile order reading the larger operand once (the other one's panels are
// re-read, from L2 when small).
int gemm_nmajor(const GemmArgs &g);
// Work-groups launch_gemm uses at most (size of wg_stats).
constexpr int kMaxGemmGroups = 4096;
// Enqueue; returns the number of work-groups launched.
int launch_gemm(const GemmArgs &g, int prec, hipStream_t s);
// The same in parts, for callers that batch GEMMs: the kernel specialisation
// (precision path, FP64 fold of K stages, FP32 output, regular shape)...
struct GemmSpec {
  int prec;
  bool fold, outf;
  int reg;  // 0 general, 1 regular shape, 2 regular with single-run index
            // maps, 3 general with the slice-accumulating epilogue, 4 general
            // with K <= 16 staged 16 deep (the narrow tile)
};
// ...chosen after filling g's offset tables,
GemmSpec prepare_gemm(GemmArgs &g, int prec);
// a dense id of it (0 .. 59),
int gemm_spec_id(const GemmSpec &sp);
// the work-groups launch_gemm would use (results, including the work-group
// statistics, depend on this count),
int gemm_groups(const GemmArgs &g, const GemmSpec &sp);
// the resident work-group capacity of the specialisation (at most
// kMaxGemmGroups),
int gemm_resident_cap(const GemmSpec &sp);
// one launch (with start / stop events recorded by the dispatch itself when
// given: they time the kernel's execution, without the launch gap),
void launch_gemm_spec(const GemmArgs &g, const GemmSpec &sp, int groups, hipStream_t s,
                      hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// and n GEMMs of one specialisation in one launch from a device table: job j
// takes work-groups [start[j], start[j + 1]) of `total` = start[n].
void launch_gemm_grouped(const GemmSpec &sp, const GemmArgs *jobs_dev, const int *start_dev, int n,
                         int total, hipStream_t s);

// Launch choices of a GEMM shape found by the tuner (process-wide table keyed
// by specialisation, dimensions and index maps; pointers are not part of the
// key): work-group count and tile order.
struct GemmTuning {
  int groups;
  int nmajor;
  int narrow;  // 1: the 16-deep K tile (K <= 16 only)
};
// The 16-deep K tile applies to this step (K <= 16, general index maps, a
// plain store epilogue).
bool gemm_narrow_ok(const GemmArgs &g, const GemmSpec &sp);
// The launch choices a step takes untuned (the tile from the measured
// default rule, the work-group count from the occupancy of that kernel).
GemmSpec gemm_default_spec(const GemmArgs &g, const GemmSpec &sp);
uint64_t gemm_tune_key(const GemmArgs &g, const GemmSpec &sp);
bool gemm_tuned(const GemmArgs &g, const GemmSpec &sp, GemmTuning &out);
void gemm_tune_store(const GemmArgs &g, const GemmSpec &sp, const GemmTuning &t);
void gemm_tune_reset();
size_t gemm_tune_size();
// Changes whenever the tuned launch choices do (cached launch descriptions
// built before are stale).
uint64_t gemm_tune_version();

// Top-R selection over the final bins after a GEMM with statistics: the
// compensated total sum and the R best bins (value descending, lower index
// first); deterministic, no atomics.
struct TopRArgs {
  const void *C;        // final bins (dense, index = offset)
  int out_f32;
  int mbits, nbits;
  IndexMap m, n;        // geometry of the final GEMM (sub-tile addressing)
  int nsub;             // sub-tiles (4 per GEMM tile)
  const double *blk_max;
  const double *wg_stats;
  int ngroups;          // work-groups of the final GEMM
  int nmajor;           // its tile order
  double *tau_sum;      // [2] threshold, total sum
  int *slot_n;          // [kTopRSlots]
  double *slot_val;     // [kTopRSlots][top_r]
  uint64_t *slot_idx;   // [kTopRSlots][top_r]
  int top_r;            // 1 .. SQC_MAX_TOPR
  int gather_groups;    // work-groups of the gather stage (topr_gather_groups)
  double *top_out;      // top_r x {double, uint64}
  double *sum_out;
};
// Work-groups of the gather stage at most; each leaves its R best in a slot.
constexpr int kTopRSlots = 64;
// Gather work-groups for a GEMM with nsub sub-tiles (about one per 64).
int topr_gather_groups(int64_t nsub);
void launch_topr(const TopRArgs &t, hipStream_t s);
// n top-R selections from a device table of n TopRArgs, in two launches;
// job j's gather takes work-groups [start[j], start[j + 1]) of total.
void launch_topr_grouped(const TopRArgs *jobs_dev, const int *start_dev, int n, int total, int out_f32,
                         hipStream_t s);

void launch_zero(void *p, size_t bytes, hipStream_t s);

// ---- first-level index slicing (slice.hip) ----
// Rows of a merged tensor kept by one slice: output row r (of `rows`) reads
// input row fixed + sum_j ((r >> lo[j]) & (2^len[j] - 1)) << pos[j]; a row is
// 2^row_bytes_log2 bytes (>= 4).
struct SliceArgs {
  const void *in;
  void *out;
  int64_t rows;
  int64_t fixed;
  int row_bytes_log2;
  int row_shift;  // set by the launcher
  int nruns;
  int lo[SQC_MAX_SLICED + 1], len[SQC_MAX_SLICED + 1], pos[SQC_MAX_SLICED + 1];
};
void launch_slice_rows(const SliceArgs &a, hipStream_t s);

}  // namespace sqc
