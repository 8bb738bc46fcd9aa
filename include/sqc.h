/*
 * sqc.h -- cut-circuit reconstruction on one AMD Instinct MI355X (gfx950).
 *
 * C interface of libsqc.  The library reconstructs the output distribution of
 * a quantum circuit that was cut into subcircuits (ScaleQC, arXiv 2207.00933)
 * from the measured outputs of the subcircuit variants:
 *
 *   attribution  (Sec. 2.1, Eq. 1 and Fig. 1): variant probabilities ->
 *                per-subcircuit entries T_i[sigma, x] for every I/X/Y/Z label
 *                assignment sigma of the subcircuit's cuts;
 *   merging      (Sec. 4, Algorithm 2): sum the entries of the data states that
 *                fall into one bin;
 *   contraction  (Sec. 6.1-6.2): contract the compute graph -- a tensor network
 *                whose cut indices have dimension 4 -- into the 2^a bin vector;
 *   recursion    (Sec. 3, Algorithm 1): bin assignment, merge, contraction,
 *                top-R bins and the bin-sum invariant for one states-merging
 *                recursion, and the whole search loop.
 *
 * Conventions used by every call
 * ------------------------------
 * Subcircuit i has n_wires wires; wire t is bit t of its measured outcome
 * index.  Every wire ends either in a circuit output (a data wire, listed in
 * data_wire[]) or in an out-cut (measured into a cut).  Data bit j of the
 * subcircuit is wire data_wire[j].
 *
 * A cut joins wire up_wire of subcircuit up_sub (measured) to wire down_wire
 * of subcircuit down_sub (initialised).  The cuts incident to a subcircuit are
 * taken in the order of the cuts[] array; the first incident cut is the least
 * significant digit of:
 *   - the variant index: radix 4 for in-cuts (preparations |0>,|1>,|+>,|+i>
 *     numbered 0..3) and radix 3 for out-cuts (measurement bases Z, X, Y
 *     numbered 0..2; outcome bit 0 is the +1 eigenvalue);
 *   - the label index sigma: radix 4, labels I, X, Y, Z numbered 0..3.
 *
 * Reconstructed bins are indexed subcircuit-major: subcircuit 0's active bits
 * are the least significant, and within a subcircuit active data bits keep
 * their ascending order.  Mapping to original qubit order is the caller's
 * (each data bit's qubit is known to it).
 *
 * The normalisation 2^-K of the K-cut sum is folded into attribution as a
 * factor 1/2 per out-cut of each subcircuit (exact in floating point).
 *
 * Ownership and asynchrony
 * ------------------------
 * Every device buffer that a call reads or writes is allocated by the
 * caller (the Python binding uses PyTorch's allocator); the library itself
 * allocates no device memory (its constants are file-scope device arrays,
 * present on every device from the library's load).  Device pointers are plain addresses on the context's
 * device.  Calls validate their arguments synchronously on the host; on any
 * error nothing is enqueued, outputs are untouched, and a message is kept for
 * sqc_last_error().  Calls that launch kernels enqueue them on the context's
 * stream and return without waiting, unless documented otherwise.  No call
 * keeps a caller pointer after it returns, except the context's workspace.
 * A context is used by one host thread at a time; distinct contexts are
 * independent.
 */
#ifndef SQC_H
#define SQC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SQC_OK = 0,
  SQC_E_ARG = 1,         /* null pointer, bad enum value, bad count          */
  SQC_E_SHAPE = 2,       /* inconsistent graph or tensor shape; degree > 15  */
  SQC_E_NOMEM = 3,       /* workspace or buffer too small for the request    */
  SQC_E_DEVICE = 4,      /* HIP runtime error, or no usable GPU              */
  SQC_E_NUMERIC = 5,     /* non-finite input found by precision selection   */
  SQC_E_BUSY = 6,        /* serving engine: no free slot for a request       */
  SQC_E_UNSUPPORTED = 7  /* valid input outside this build's limits          */
} sqc_status;

typedef enum {
  SQC_F64 = 0,     /* IEEE binary64                                         */
  SQC_F32 = 1,     /* IEEE binary32; as a contraction precision: FP32 MFMA  */
  SQC_BF16X3 = 2,  /* contraction only: each FP32 operand split into bf16
                      hi + lo, three bf16 MFMA products (hi*hi + hi*lo +
                      lo*hi) accumulated in FP32                            */
  SQC_AUTO = 3     /* sqc_recurse only: the library picks SQC_BF16X3,
                      SQC_F32 or SQC_F64 by sqc_select_precision first     */
} sqc_prec;

/* Largest compute-graph degree (cuts on one subcircuit), Sec. 6.2. */
#define SQC_MAX_DEGREE 15
/* Largest number of data bits of one subcircuit. */
#define SQC_MAX_DATA_BITS 62
/* Largest top-R of one recursion. */
#define SQC_MAX_TOPR 64

typedef struct {
  int32_t up_sub, up_wire;      /* measured side (upstream)                 */
  int32_t down_sub, down_wire;  /* initialised side (downstream)            */
} sqc_cut;

typedef struct {
  int32_t n_wires;              /* wires of the subcircuit (<= 32)          */
  int32_t n_data;               /* wires that end in a circuit output       */
  const int32_t *data_wire;     /* n_data wire indices; data bit j = wire   */
} sqc_sub;

/* Bit masks over one subcircuit's data bits (bit j = data bit j).  fixed,
 * active and merged are disjoint and cover all data bits; fixed_val holds the
 * values of the fixed bits (zero elsewhere).  A bin is the set of data states
 * with x & fixed == fixed_val and a given value of the active bits. */
typedef struct {
  uint64_t fixed, fixed_val, active, merged;
} sqc_masks;

/* Tensor layouts. */
#define SQC_LAYOUT_ATTRIBUTED 0 /* [2^n_bits][4^n_labels]: element (sigma, x)
                                   at x * 4^n_labels + sigma                */
#define SQC_LAYOUT_MERGED 1     /* [4^n_labels][2^n_bits]: element (sigma, b)
                                   at sigma * 2^n_bits + b                  */

typedef struct {
  void *data;          /* device buffer owned by the caller                 */
  int32_t n_labels;    /* c_i: incident cuts                                */
  int32_t n_bits;      /* data bits (attributed) or active bits (merged)    */
  sqc_prec prec;       /* storage: SQC_F64 or SQC_F32                       */
  int32_t layout;      /* SQC_LAYOUT_*                                      */
} sqc_tensor;

typedef struct sqc_ctx sqc_ctx;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device` using `hip_stream` (a hipStream_t,
 * NULL = the default stream).  Fails with SQC_E_DEVICE when no GPU is usable. */
sqc_status sqc_ctx_create(int device, void *hip_stream, sqc_ctx **out);
sqc_status sqc_ctx_destroy(sqc_ctx *ctx);
/* Replace the stream later calls enqueue on. */
sqc_status sqc_ctx_set_stream(sqc_ctx *ctx, void *hip_stream);
/* Give the context a caller-owned device workspace used by merge, contract,
 * recurse and search for intermediates and scratch.  The context keeps the
 * pointer until it is replaced or the context is destroyed; the caller must
 * keep the buffer alive that long.  Nothing is launched: the buffer needs no
 * initialisation, and the call is cheap enough to make before every request. */
sqc_status sqc_ctx_set_workspace(sqc_ctx *ctx, void *dev, size_t bytes);
/* Stage timing.  With a non-zero mask, every kernel launch of the selected
 * stages is bracketed by HIP events on the context's stream (for the
 * contraction stages, events recorded by the kernel's dispatch itself through
 * hipExtLaunchKernel, so they span its execution only), and the library
 * adds the launch's algorithmic bytes (inputs read once, outputs written once)
 * and useful flops (2 M N K per GEMM) to the stage's totals. */
#define SQC_STAGE_ATTRIBUTE 1u
#define SQC_STAGE_MERGE 2u
#define SQC_STAGE_CONTRACT 4u    /* contraction steps before the last     */
#define SQC_STAGE_FINAL 8u       /* last contraction step (bins written)  */
#define SQC_STAGE_TOPR 16u
typedef struct {
  double ms;          /* summed event time of the stage's launches         */
  int64_t launches;
  double bytes;       /* summed algorithmic bytes                          */
  double flops;       /* summed useful floating-point operations           */
} sqc_stage_time;
sqc_status sqc_ctx_set_timing(sqc_ctx *ctx, uint32_t stage_mask);
/* Wait for the recorded events and report the totals of one stage (one bit
 * of the mask) since the last reset; `reset` clears every stage afterwards. */
sqc_status sqc_ctx_timing(sqc_ctx *ctx, uint32_t stage, int32_t reset,
                          sqc_stage_time *out);

/* Message describing the last error of this context (or of the calling
 * thread's last context-less call when ctx is NULL).  Never NULL. */
const char *sqc_last_error(const sqc_ctx *ctx);
/* Library version string. */
const char *sqc_version(void);

/* ---- host-only helpers (no GPU needed) ------------------------------------ */

/* Validate a compute graph: cut ids and wires in range, every wire is either a
 * data wire or measured into exactly one cut, at most one cut initialises a
 * wire, no cut joins a subcircuit to itself, degree <= SQC_MAX_DEGREE. */
sqc_status sqc_check_graph(const sqc_sub *subs, int32_t n_sub,
                           const sqc_cut *cuts, int32_t n_cuts);

/* Algorithm 2 (states assignment) as masks.  `scope` gives, per subcircuit,
 * the states under analysis as fixed / fixed_val (NULL: recursion 0, nothing
 * fixed).  Each subcircuit starts with l_i = 2^(unfixed bits) bins; while the
 * product exceeds M, the largest l'_i (lowest index on ties) is halved.  The
 * resulting per-subcircuit masks keep the scope's fixed bits, make the lowest
 * log2(l'_i) unfixed bits active and the remaining unfixed bits merged (the
 * bins of the printed rule "state j goes to bin j mod l'_i" over states in
 * ascending order).  `n_data[i]` is d_i.  Writes n_sub masks to `out`. */
sqc_status sqc_assign_bins(int32_t n_sub, const int32_t *n_data,
                           const sqc_masks *scope, uint64_t max_bins_M,
                           sqc_masks *out);

/* Scope (fixed / fixed_val) of bin `bin` (subcircuit-major index) of a
 * recursion run with `masks`: fixed' = fixed | active, fixed_val' = fixed_val
 * with the bin's active bits deposited.  Writes n_sub masks (active = 0,
 * merged = unfixed bits) to `scope_out`. */
sqc_status sqc_bin_scope(int32_t n_sub, const sqc_masks *masks, uint64_t bin,
                         sqc_masks *scope_out);

/* Cost model of Sec. 6.2 for contracting a compute graph whose subcircuit i
 * has out_bits[i] output bits (2^out_bits entries per label assignment).
 * Only up_sub / down_sub of the cuts are used.  `order` gives n_sub-1 pairs
 * (2*(n_sub-1) ints) of positions in a working list (the result replaces the
 * first position, the second is removed), or NULL for the library's planner.
 * Results: input floats, total multiplications of the plan (product of all
 * dimensions of each pairwise step), the largest step's operand floats, the
 * largest intermediate, and the multiplications of evaluating Eq. 1 directly
 * (4^K times the successive outer products). */
typedef struct {
  double input_floats;
  double plan_mults;
  double max_step_operand_floats;
  double max_intermediate_floats;
  double naive_mults;
  int32_t n_steps;
  int32_t order[2 * 64]; /* the pairs used (planner's or the given ones)   */
} sqc_cost;
sqc_status sqc_plan_cost(int32_t n_sub, const int32_t *out_bits,
                         const sqc_cut *cuts, int32_t n_cuts,
                         const int32_t *order, sqc_cost *out);

/* First-level index slicing heuristic of Sec. 6.3: repeatedly write out the
 * cut whose removal reduces the total input floats the most (lowest cut id on
 * ties) until the total is <= budget_floats, slicing at most SQC_MAX_SLICED
 * cuts (the most sqc_contract_sliced takes).  Writes the chosen cut ids to
 * `sliced` (capacity min(n_cuts, SQC_MAX_SLICED)) and their count to
 * `n_sliced`.  Errors: SQC_E_ARG for NULL pointers or a bad graph;
 * SQC_E_NOMEM when the budget is still unmet after slicing every cut or
 * SQC_MAX_SLICED of them (sliced/n_sliced then hold that best effort). */
sqc_status sqc_slice_plan(int32_t n_sub, const int32_t *out_bits,
                          const sqc_cut *cuts, int32_t n_cuts,
                          double budget_floats, int32_t *sliced,
                          int32_t *n_sliced);

/* Cut search (Sec. 5, MIP model, constraints and objective), host only.  The
 * circuit's two-qubit gates, in circuit order, are gates[2 v], gates[2 v + 1]
 * (qubit ids in [0, n_qubits)); they are the DAG's vertices, and each qubit
 * line between two consecutive two-qubit gates on that qubit is an edge
 * (input and output vertices are left out).  The call assigns every gate to
 * one of n_sub subcircuits, each holding at least one and at most
 * floor(alpha * n_gates) gates (Eq. 2), minimising the largest number of cut
 * edges on one subcircuit, L = max_c (I_c + O_c) (Eq. 3), with the total
 * number of cut edges as the tie-break.  Method: two starts (the gate order
 * cut into n_sub blocks; bands of qubits, a gate in the band of its lowest
 * qubit) improved by single-gate moves (each scored incrementally in
 * O(gate degree); with more than 32 subcircuits only the neighbours'
 * subcircuits are tried), then iterated local search (a few gates moved at
 * random with a fixed seed, improved again, kept when better), then branch
 * and bound over the gates in circuit order (subcircuit ids opened in
 * order) from that incumbent, on an explicit stack of one frame per gate,
 * pruned by the running (L, cut edges), which only grow; it stops after
 * max_nodes search nodes (<= 0: no limit) and returns the best partition
 * found (*optimal = 1 when the search completed).  Host memory
 * O(n_gates * n_sub).  Writes
 * assign[n_gates], *L and *n_cut_edges.  Errors: SQC_E_ARG for NULL
 * pointers, n_sub outside [1, n_gates], a qubit id out of range or a gate on
 * one qubit; SQC_E_SHAPE when no partition meets Eq. 2. */
sqc_status sqc_find_cuts(int32_t n_qubits, const int32_t *gates, int32_t n_gates,
                         int32_t n_sub, double alpha, int64_t max_nodes,
                         int32_t *assign, int32_t *L, int32_t *n_cut_edges,
                         int32_t *optimal);

/* ---- attribution (Sec. 2.1, Fig. 1) ---------------------------------------- */

/* Bytes of subcircuit sub_id's attributed tensor: 4^c * 2^d elements of
 * out_prec.  Returns 0 on invalid input. */
size_t sqc_attribute_bytes(const sqc_sub *subs, int32_t n_sub, int32_t sub_id,
                           const sqc_cut *cuts, int32_t n_cuts,
                           sqc_prec out_prec);

/* Attribute the variants of subcircuit sub_id.  `variants_dev` holds
 * [V][2^n_wires] probabilities of in_prec (SQC_F64 or SQC_F32), V = product
 * over incident cuts of 4 (in) or 3 (out).  `out->data` must hold
 * sqc_attribute_bytes() bytes and `out->prec` selects the stored precision
 * (SQC_F64 or SQC_F32); the call fills the other fields of *out.  Arithmetic
 * is FP64.  For every label assignment sigma of the incident cuts and data
 * state x:
 *   T[sigma, x] = 2^-out * sum_s prod_in c(sigma_e, s_e)
 *                         * sum_b prod_out g(sigma_e, b_e) * p_(s, beta(sigma))(x, b)
 * with c(I) = (1,1,0,0), c(X) = (-1,-1,2,0), c(Y) = (-1,-1,0,2),
 * c(Z) = (1,-1,0,0) over the preparations, beta(I) = beta(Z) = Z,
 * beta(X) = X, beta(Y) = Y, and g(I, b) = 1, g(X|Y|Z, b) = (-1)^b.
 * Output layout SQC_LAYOUT_ATTRIBUTED. */
sqc_status sqc_attribute(sqc_ctx *ctx, const sqc_sub *subs, int32_t n_sub,
                         int32_t sub_id, const sqc_cut *cuts, int32_t n_cuts,
                         const void *variants_dev, sqc_prec in_prec,
                         sqc_tensor *out);
/* All subcircuits at once: variants_dev[i] holds subcircuit i's variants,
 * outs[i] its output (data and prec set by the caller; the other fields are
 * filled as by sqc_attribute).  Subcircuits that fit the on-chip stage share
 * one launch, so the small ones overlap the large ones. */
sqc_status sqc_attribute_all(sqc_ctx *ctx, const sqc_sub *subs, int32_t n_sub,
                             const sqc_cut *cuts, int32_t n_cuts,
                             const void *const *variants_dev, sqc_prec in_prec,
                             sqc_tensor *outs);
/* The attribution written straight in the merged layout (Sec. 2.1 and Sec. 4
 * in one pass): outs[i] receives subcircuit i's tensor as sqc_merge would
 * produce it for a recursion that keeps every data bit of the subcircuit
 * active (nothing fixed or merged), [4^c][2^d] with the bins fastest, layout
 * SQC_LAYOUT_MERGED, each value exactly the one sqc_attribute_all followed
 * by that merge stores.  Such a tensor can be contracted by sqc_contract or
 * passed to sqc_recurse for a recursion whose masks keep all its data bits
 * active (a full-output recursion: M at least the product of the 2^d_i), in
 * the path's operand precision (out->prec FP64 for SQC_F64, FP32 for the
 * other paths); that recursion then reads it in place and runs no merge for
 * it.  Other recursions, SQC_AUTO, slicing, the search, queries and serving
 * need the attributed layout (SQC_E_ARG or SQC_E_SHAPE otherwise).
 * Arguments as for sqc_attribute_all. */
sqc_status sqc_attribute_all_merged(sqc_ctx *ctx, const sqc_sub *subs, int32_t n_sub,
                                    const sqc_cut *cuts, int32_t n_cuts,
                                    const void *const *variants_dev, sqc_prec in_prec,
                                    sqc_tensor *outs);

/* ---- merging (Sec. 4) ------------------------------------------------------ */

/* Merge an attributed tensor over the bins described by `masks`:
 *   out[sigma, b] = sum over x with x & fixed == fixed_val, the active bits
 *                   of x equal to b (compacted, ascending), of T[sigma, x].
 * `out->data` must hold 4^c * 2^popcount(active) elements of out->prec;
 * the call fills the other fields (layout SQC_LAYOUT_MERGED).  Sums are
 * accumulated in FP64 in a fixed order (deterministic).  May use the
 * context workspace (sqc_merge_workspace_bytes). */
size_t sqc_merge_workspace_bytes(const sqc_tensor *attributed,
                                 const sqc_masks *masks);
sqc_status sqc_merge(sqc_ctx *ctx, const sqc_tensor *attributed,
                     const sqc_masks *masks, sqc_tensor *out);

/* ---- contraction (Sec. 6.1-6.2) ---------------------------------------------- */

/* Contract merged tensors (one per subcircuit, layout SQC_LAYOUT_MERGED,
 * n_labels equal to each subcircuit's degree) over every cut label into the
 * 2^(sum of n_bits) bin vector `bins_dev` (bins_prec SQC_F64 or SQC_F32).
 * `prec` selects the arithmetic of the pairwise GEMMs: SQC_F64 (FP64 MFMA,
 * FP64 tensors), SQC_F32 (FP32 MFMA) or SQC_BF16X3; for the last two the
 * final step sums its K axis in FP32 chunks added into FP64 accumulators with
 * Neumaier compensation.  Order: the library's planner (greedy pairwise,
 * Sec. 6.4 notes any order gives the same result up to rounding).
 * Intermediates live in the context workspace
 * (sqc_contract_workspace_bytes). */
size_t sqc_contract_workspace_bytes(const sqc_tensor *merged, int32_t n_sub,
                                    const sqc_cut *cuts, int32_t n_cuts,
                                    sqc_prec prec);
sqc_status sqc_contract(sqc_ctx *ctx, const sqc_tensor *merged, int32_t n_sub,
                        const sqc_cut *cuts, int32_t n_cuts, sqc_prec prec,
                        void *bins_dev, sqc_prec bins_prec);

/* Sliced contraction (Sec. 6.3, first-level index slicing): the result of
 * sqc_contract, computed as a sum over slices.  `sliced` lists n_sliced
 * distinct cut ids (0 <= n_sliced <= SQC_MAX_SLICED, each id in [0, n_cuts));
 * a slice is one label assignment of those cuts, numbered with the first
 * listed cut as the least significant radix-4 digit.  For each of the
 * 4^n_sliced slices, in ascending order: every merged tensor incident to a
 * sliced cut is restricted to the slice's labels (its rows gathered into the
 * workspace, the remaining labels keeping their order), the network without
 * the sliced cuts is contracted as by sqc_contract (same `prec`), and its
 * final step adds the slice's bins into FP64 running sums with Neumaier
 * compensation (no slice vector is stored); the last slice's final step
 * writes sum + compensation to `bins_dev` (2^a elements of bins_prec, a = sum
 * of n_bits).  The contraction's intermediates are those of the sliced
 * network (4x smaller per sliced label they would carry); the call adds the
 * gathered operands and two 2^a FP64 vectors (sums, compensations) to the
 * workspace (sqc_contract_sliced_workspace_bytes).  n_sliced = 0 is the
 * plain contraction.  Merged tensors and cuts as for sqc_contract.  Stage
 * timing books the gathers under SQC_STAGE_MERGE.  Errors: SQC_E_ARG for a
 * repeated or out-of-range cut id or n_sliced outside [0, SQC_MAX_SLICED],
 * SQC_E_NOMEM for a small workspace, else as sqc_contract. */
#define SQC_MAX_SLICED 8
size_t sqc_contract_sliced_workspace_bytes(const sqc_tensor *merged, int32_t n_sub,
                                           const sqc_cut *cuts, int32_t n_cuts,
                                           const int32_t *sliced, int32_t n_sliced,
                                           sqc_prec prec);
sqc_status sqc_contract_sliced(sqc_ctx *ctx, const sqc_tensor *merged, int32_t n_sub,
                               const sqc_cut *cuts, int32_t n_cuts,
                               const int32_t *sliced, int32_t n_sliced, sqc_prec prec,
                               void *bins_dev, sqc_prec bins_prec);

/* ---- one states-merging recursion (Algorithm 1 body) ------------------------- */

/* One recursion: sqc_assign_bins on `scope` (NULL at recursion 0), merge of
 * every attributed tensor, contraction into `bins_dev` (2^a elements of
 * bins_prec, a = sum of active bits), then on the device the top_r largest
 * bins (value descending, lower index first on ties) and the FP64
 * (compensated) sum of all bins.  Results go to `topr_dev` (top_r records of
 * {double value; uint64_t index}) and `sum_dev` (one double).  The masks used
 * are written to `masks_out` (host, n_sub entries) before the call returns;
 * the device results are ready when the stream reaches them.
 * `attributed[i].prec` may differ from `prec` (SQC_F64 attributed with an
 * FP32 path is allowed).  A tensor may instead be in the merged layout
 * (sqc_attribute_all_merged) when the recursion keeps every data bit of its
 * subcircuit active and it is stored in the path's operand precision: it is
 * then read in place and not merged (else SQC_E_ARG).  prec = SQC_AUTO
 * selects the precision first (sqc_select_precision: waits for the device,
 * not while recording a graph; attributed layout only); its workspace query
 * covers every choice.
 *
 * Memory-driven slicing (Sec. 6.3): when the context's workspace is smaller
 * than the unsliced recursion needs (sqc_recurse_workspace_bytes), the call
 * slices cuts, chosen as sqc_recurse_slices reports: repeatedly the cut whose
 * removal shrinks the merged tensors' total size the most (the higher id on
 * ties: the higher label digit, so that a slice reads long contiguous runs of
 * labels), until the sliced layout fits, at most SQC_MAX_SLICED cuts, else
 * SQC_E_NOMEM.  Each of the 4^s slices merges, straight from the attributed
 * tensors, only the label rows it keeps (subcircuits with no sliced cut are
 * merged once), contracts the network without the sliced cuts, and its
 * final step adds the slice into FP64 running sums (Neumaier); the last
 * slice writes the bins and the top-R statistics.  Slices are added in
 * ascending order (the first chosen cut the least significant radix-4
 * digit), so results are deterministic; they equal the unsliced results up
 * to rounding.  The sliced workspace holds each subcircuit's slice of merged
 * rows, the sliced network's intermediates and two 2^a FP64 vectors.  With
 * SQC_AUTO the precision selector's own pass must fit unsliced; a recursion
 * with merged-layout inputs is not sliced (SQC_E_ARG when it would need to
 * be). */
size_t sqc_recurse_workspace_bytes(const sqc_tensor *attributed, int32_t n_sub,
                                   const sqc_cut *cuts, int32_t n_cuts,
                                   const sqc_masks *masks, sqc_prec prec);
/* The cuts a recursion with these masks (prec SQC_F64, SQC_F32 or
 * SQC_BF16X3, top_r in [1, 64]) slices under a workspace of workspace_bytes:
 * writes them to `sliced` (capacity SQC_MAX_SLICED; none when the unsliced
 * plan fits) in slice-digit order, their count to `n_sliced` and the bytes
 * the chosen layout needs to *need_bytes (optional).  Host only.  Errors:
 * SQC_E_ARG for NULL pointers or bad arguments, SQC_E_SHAPE for an
 * inconsistent graph, SQC_E_NOMEM when SQC_MAX_SLICED cuts do not make it
 * fit. */
sqc_status sqc_recurse_slices(const sqc_tensor *attributed, int32_t n_sub,
                              const sqc_cut *cuts, int32_t n_cuts,
                              const sqc_masks *masks, sqc_prec prec, int32_t top_r,
                              size_t workspace_bytes, int32_t *sliced,
                              int32_t *n_sliced, size_t *need_bytes);
sqc_status sqc_recurse(sqc_ctx *ctx, const sqc_tensor *attributed, int32_t n_sub,
                       const sqc_cut *cuts, int32_t n_cuts,
                       const sqc_masks *scope, uint64_t max_bins_M,
                       int32_t top_r, sqc_prec prec, void *bins_dev,
                       sqc_prec bins_prec, sqc_masks *masks_out,
                       void *topr_dev, void *sum_dev);

/* Precision selection (Eq. 1's terms summed in the path's arithmetic).  A
 * bin computed as a sum over label assignments of products of the merged
 * entries is off by at most c_path * u * S(x), S(x) = sum_sigma prod_i
 * |T_i[sigma, x_i]| (the a-priori bound of a sum of products), with
 * c * u = 2^-13 for split-BF16x3 (each operand kept to 2^-16 relative, lo*lo
 * dropped), 2^-20 for FP32 MFMA, plus 2^-24 |bin| when bins are stored in
 * FP32.  The call bounds max_x S(x) from above without forming S: it merges
 * the attributed tensors for the recursion on `scope` (FP32, as the fast
 * paths contract them), takes each label row's largest |entry| m_i[sigma]
 * (row_absmax), and contracts the m_i over the cut graph in FP64 (labels
 * only, one number): B = sum_sigma prod_i m_i[sigma|_i] >= S(x) for every x.
 * It then picks SQC_BF16X3 when (2^-13 + 2^-24) B <= the context's
 * tolerance, else SQC_F32 when (2^-20 + 2^-24) B <= it, else SQC_F64, and
 * returns the choice and B.  Enqueued on the context's stream; waits for the
 * device (it cannot be recorded into a graph).  Workspace as sqc_recurse
 * with SQC_AUTO.  The tolerance (an absolute error per bin) is 1e-6 unless
 * set by sqc_ctx_set_tolerance (> 0).  sqc_recurse with prec = SQC_AUTO
 * calls this first and keeps the choice and bound for
 * sqc_ctx_auto_choice.  This is also the library's check for non-finite
 * input: a NaN or infinity in a merged tensor (or a bound that overflows)
 * makes B non-finite, and the call (or sqc_recurse with SQC_AUTO, before
 * any contraction) fails with SQC_E_NUMERIC, *bound set to that B. */
sqc_status sqc_ctx_set_tolerance(sqc_ctx *ctx, double max_abs_error);
sqc_status sqc_select_precision(sqc_ctx *ctx, const sqc_tensor *attributed, int32_t n_sub,
                                const sqc_cut *cuts, int32_t n_cuts,
                                const sqc_masks *scope, uint64_t max_bins_M,
                                sqc_prec *chosen, double *bound);
sqc_status sqc_ctx_auto_choice(const sqc_ctx *ctx, sqc_prec *chosen, double *bound);

/* Allocation-free recursion, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same work, kernels and results as sqc_recurse (bitwise),
 * with the workspace taken from a device array inside the library instead of
 * the context's workspace (sqc_ctx_set_workspace is not needed).  The array
 * holds SQC_NOALLOC_SCRATCH_BYTES (64 MiB) on each device the library runs
 * on, from the library's load until the process ends; its address is taken
 * once per device by sqc_ctx_create.  A recursion whose workspace
 * (sqc_recurse_workspace_bytes) exceeds it fails with SQC_E_NOMEM and
 * enqueues nothing.  The call allocates nothing (no hipMalloc, no events:
 * stage timing does not apply).  Every call on one device shares that
 * device's array, and the array keeps the last call's contents (nothing in
 * it needs to start at zero: every byte a call reads, the same call wrote
 * first); calls that overlap on one device, on any streams or contexts, race
 * and give undefined results, so the caller orders them (one stream, or
 * events).  Arguments, outputs and the other errors as sqc_recurse. */
#define SQC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
sqc_status sqc_recurse_noalloc(sqc_ctx *ctx, const sqc_tensor *attributed, int32_t n_sub,
                               const sqc_cut *cuts, int32_t n_cuts,
                               const sqc_masks *scope, uint64_t max_bins_M,
                               int32_t top_r, sqc_prec prec, void *bins_dev,
                               sqc_prec bins_prec, sqc_masks *masks_out,
                               void *topr_dev, void *sum_dev);

/* Probabilities of chosen output states (Sec. 3: an arbitrary subset of
 * states evaluated in one recursion without merging into bins).  states[j]
 * (host array, n_states entries) is a full output index, subcircuit-major as
 * the bins of a recursion with every data bit active (subcircuit 0's data
 * bits least significant), each < 2^(sum of d_i).  For every state the
 * attributed tensors are restricted to that state's data bits (a merge with
 * every data bit fixed) and the cut indices are contracted as in sqc_recurse
 * with M = 1; probs_dev[j] (probs_prec) receives the reconstructed value.
 * States are processed in batches whose merges, contraction steps and
 * selections share launches (job tables staged through the context's pinned
 * buffer); two batches are in flight at most (the host forms one while the
 * device runs the other, and waits before reusing a batch's staging), and the
 * call returns once the last batch has finished, so it cannot be recorded
 * into a graph.  Repeated states are allowed.  Workspace:
 * sqc_query_states_workspace_bytes (independent of n_states).  Errors:
 * SQC_E_ARG for a NULL buffer, a state out of range or while recording, else
 * as sqc_recurse. */
size_t sqc_query_states_workspace_bytes(const sqc_tensor *attributed, int32_t n_sub,
                                        const sqc_cut *cuts, int32_t n_cuts,
                                        sqc_prec prec);
sqc_status sqc_query_states(sqc_ctx *ctx, const sqc_tensor *attributed, int32_t n_sub,
                            const sqc_cut *cuts, int32_t n_cuts, const uint64_t *states,
                            int64_t n_states, sqc_prec prec, void *probs_dev,
                            sqc_prec probs_prec);

/* ---- HIP graphs of enqueued work (not part of the paper) ----------------------- */

/* Record the work later calls enqueue on the context's stream (sqc_attribute,
 * sqc_attribute_all, sqc_merge, sqc_contract, sqc_contract_sliced,
 * sqc_recurse) into a HIP graph instead of running it, then replay it with one
 * launch.  For repeated
 * queries whose buffers do not change (the graph keeps every pointer and
 * argument of the recorded calls, including the workspace, so the caller
 * keeps them alive and unchanged in size until sqc_graph_destroy).  The
 * context must use a created stream (stream capture is not allowed on the
 * default stream).  Stage timing is suspended while recording; calls that
 * wait for the device (sqc_search, sqc_autotune, sqc_ctx_timing) and
 * sqc_ctx_set_stream fail with SQC_E_ARG while recording.  The recorded work
 * contains no memset nodes.  A failed call while recording leaves the capture
 * invalid: sqc_graph_end then fails. */
typedef struct sqc_graph sqc_graph;
sqc_status sqc_graph_begin(sqc_ctx *ctx);
sqc_status sqc_graph_end(sqc_ctx *ctx, sqc_graph **out);
/* Enqueue one replay on the context's stream. */
sqc_status sqc_graph_launch(sqc_ctx *ctx, const sqc_graph *graph);
sqc_status sqc_graph_destroy(sqc_graph *graph);

/* ---- launch tuning (not part of the paper) ------------------------------------ */

/* A project-side autotuner of the contraction launches.  For the recursion
 * described as in sqc_recurse (its workspace from sqc_recurse_workspace_bytes),
 * it runs the recursion once, then times every GEMM step of it (`reps`
 * launches each, HIP events on the context's stream, waiting for the device)
 * over candidate launch choices: two tile shapes when the step contracts at
 * most 16 labels (K staged 64 deep, or 16 deep: the narrow tile), work-group
 * counts of 1/4, 1/2, 1 and 2 times each kernel's resident capacity and one
 * per tile, and both tile orders when the step has several m and n panels.
 * Untuned, a step with K <= 16 takes the narrow tile.  The fastest choice of
 * each step is stored in a
 * process-wide table keyed by the step's kernel specialisation, dimensions
 * and index maps, and every later launch of the same shape (sqc_contract,
 * sqc_recurse, sqc_search, the serving engine) uses it.  Tile order changes
 * no result; the work-group count changes how the bin sum is split, so sums
 * may differ in the last bits from an untuned run (every run with the same
 * table gives the same bits).  The recursion is run once more at the end, so
 * `bins_dev` holds its bins.  Blocks the calling thread.  `report` (optional)
 * receives the steps tuned, candidates timed, the summed step times with
 * the default and the chosen launches, and per step (the first 64) the
 * chosen tile (0: 64 deep, 1: 16 deep), work-group count and tile order. */
typedef struct {
  int32_t steps, candidates;
  double default_us, tuned_us;
  int32_t step_tile[64], step_groups[64], step_nmajor[64];
} sqc_tune_report;
sqc_status sqc_autotune(sqc_ctx *ctx, const sqc_tensor *attributed, int32_t n_sub,
                        const sqc_cut *cuts, int32_t n_cuts, const sqc_masks *scope,
                        uint64_t max_bins_M, sqc_prec prec, void *bins_dev,
                        sqc_prec bins_prec, int32_t reps, sqc_tune_report *report);
/* Forget every tuned choice (launches return to the default heuristics). */
sqc_status sqc_autotune_reset(void);
/* Number of tuned shapes in the table. */
int32_t sqc_autotune_entries(void);

/* ---- the search loop (Algorithm 1) ------------------------------------------- */

typedef struct {
  double prob;          /* reconstructed probability of the bin            */
  int32_t recursion;    /* recursion that produced it                      */
  int32_t pad;
  uint64_t bin;         /* bin index within that recursion                 */
} sqc_found;

typedef struct {
  double bins_sum;      /* FP64 sum of the recursion's bins                */
  double parent_prob;   /* probability of the expanded bin (1 at r = 0)    */
  double top_prob;      /* largest bin                                     */
  int32_t active_bits;  /* a = log2 of the bin count                       */
  int32_t leaf;         /* 1 when every bin is a single state              */
} sqc_recursion_info;

/* Algorithm 1 with R = max_recursions: run recursions while r < R and the
 * list L of candidate bins is not empty.  After each recursion the R largest
 * bins that still hold more than one state are appended to L, L is sorted
 * (probability descending, then earlier recursion, then lower bin index) and
 * truncated to R, and the first entry is popped for the next recursion.  Bins
 * of single states are reported as solutions (the R largest of each leaf
 * recursion).  The whole loop runs on the device: a recursion's shape
 * depends only on its depth below the first one (Algorithm 2 sees only how
 * many states the popped bin holds), so every depth is planned once, all R
 * recursions are enqueued back to back, and after each a one-work-group
 * kernel updates L, pops the next bin and sets up its recursion's job tables;
 * once L is empty the remaining launches do nothing.  The call waits for the
 * device once, at the end.  Workspace: sqc_search_workspace_bytes (the
 * largest recursion's workspace, then the search's tables and results).
 * `solutions` / `solution_states` receive up to max_solutions entries (at
 * most R * R); for solution k, solution_states[k * n_sub + i] is subcircuit
 * i's data state.  `info` (optional) receives one record per recursion run
 * (capacity max_recursions).  `bins_dev` must hold 2^a elements of bins_prec
 * for the largest a the search uses (at most floor(log2 M)); it holds the
 * last recursion's bins.  The search does not slice (its recursions are
 * laid out once, unsliced); a graph whose recursions fit only sliced is
 * searched by calling sqc_recurse per recursion.  Errors: SQC_E_NOMEM when
 * the workspace is too small, SQC_E_UNSUPPORTED above 64 subcircuits, else
 * as sqc_recurse. */
size_t sqc_search_workspace_bytes(const sqc_tensor *attributed, int32_t n_sub,
                                  const sqc_cut *cuts, int32_t n_cuts, uint64_t max_bins_M,
                                  int32_t max_recursions, sqc_prec prec,
                                  int32_t max_solutions);
sqc_status sqc_search(sqc_ctx *ctx, const sqc_tensor *attributed, int32_t n_sub,
                      const sqc_cut *cuts, int32_t n_cuts, uint64_t max_bins_M,
                      int32_t max_recursions, sqc_prec prec, void *bins_dev,
                      sqc_prec bins_prec, sqc_found *solutions,
                      uint64_t *solution_states, int32_t max_solutions,
                      int32_t *n_solutions, sqc_recursion_info *info,
                      int32_t *n_recursions);

/* ---- serving (an engine around sqc_recurse; not part of the paper) -------------
 *
 * A server keeps registered circuits' attributed tensors resident (the caller
 * keeps the buffers alive until sqc_serve_destroy) and runs requests, each one
 * states-merging recursion exactly as sqc_recurse computes it.  It owns
 * n_slots HIP streams (default priority), one context each, and the caller's
 * workspace buffer.  Requests are validated and planned by sqc_serve_submit.
 * Whenever a slot is idle, the waiting requests (in arrival order; a later
 * request that fits may pass an earlier one that does not, but once a
 * request has been passed over 8 times nothing behind it is admitted before
 * it: aging, so a large request is not starved) are shared among the idle
 * slots as batches, each limited by the largest free block of the
 * workspace; a batch runs as one set of launches whose kernels read the
 * requests' jobs from a table in device memory (merges, each GEMM level per
 * kernel specialisation, top-R), so a batch costs a few launches however many
 * requests it holds.  Batches on different slots overlap on the device, and
 * requests that arrive while others run are admitted as slots and memory free
 * up.  Each result is bitwise the same as the same sqc_recurse call made
 * alone.  The engine advances (retires finished batches, admits waiting
 * requests) inside sqc_serve_submit, _poll, _wait and _completed; it is not
 * thread-safe.  Output buffers must not be touched by other streams while a
 * request runs: the engine's streams do not wait for other work. */
typedef struct sqc_server sqc_server;

typedef struct {
  int32_t circuit;            /* id from sqc_serve_register                  */
  int32_t top_r;              /* 1 .. SQC_MAX_TOPR                           */
  uint64_t max_bins_M;        /* M of Algorithm 2                            */
  const sqc_masks *scope;     /* n_sub masks of the expanded bin, or NULL at
                                 recursion 0; copied by sqc_serve_submit     */
  sqc_prec prec;              /* contraction path                            */
  sqc_prec bins_prec;         /* storage of bins_dev                         */
  void *bins_dev;             /* 2^a elements, caller-owned                  */
  void *topr_dev;             /* top_r {double, uint64} records              */
  void *sum_dev;              /* one double                                  */
  sqc_masks *masks_out;       /* optional, n_sub entries, written by submit  */
} sqc_request;

typedef struct {
  uint64_t submitted, admitted, completed;
  int32_t running, queued;
  int32_t max_running;        /* most requests on the device at once         */
  int32_t max_batch;          /* most requests in one batch                  */
  uint64_t workspace_bytes, workspace_peak;  /* bytes in use, at most        */
  uint64_t batches;           /* batches launched                            */
  double plan_seconds;        /* host time planning requests (submit)        */
  double launch_seconds;      /* host time forming and enqueuing batches     */
  uint64_t aged_holds;        /* batches cut short behind an aged request    */
} sqc_serve_stats;

/* Create a server on `device` with n_slots (1..64) streams using the caller's
 * workspace (256-byte aligned device buffer; it is split among the running
 * requests). */
sqc_status sqc_serve_create(int device, int32_t n_slots, void *workspace_dev,
                            size_t workspace_bytes, sqc_server **out);
/* Largest batch (1 .. 128, default 128); 1 runs every request on its own
 * launches, as sqc_recurse does. */
sqc_status sqc_serve_set_max_batch(sqc_server *srv, int32_t max_batch);
/* Wait for running requests, then release the streams and contexts. */
sqc_status sqc_serve_destroy(sqc_server *srv);
/* Register a circuit: its attributed tensors and cut list (copied; the tensor
 * buffers stay the caller's). */
sqc_status sqc_serve_register(sqc_server *srv, const sqc_tensor *attributed, int32_t n_sub,
                              const sqc_cut *cuts, int32_t n_cuts, int32_t *circuit_id);
/* Workspace bytes the request needs, its share of a batch's job table
 * included (0 on invalid input). */
size_t sqc_serve_footprint(sqc_server *srv, const sqc_request *req);
/* Validate, plan and queue a request; SQC_E_NOMEM when its footprint exceeds
 * the whole workspace.  `ticket` identifies it in sqc_serve_poll / _wait. */
sqc_status sqc_serve_submit(sqc_server *srv, const sqc_request *req, uint64_t *ticket);
/* Submit n requests at once (a burst of arrivals): each is validated and
 * planned as by sqc_serve_submit, then they are queued in order in shares
 * of one batch per slot (the burst size over the slot count, at most the
 * batch cap), the engine advancing after each share, so the burst leaves in
 * full batches instead of the first requests leaving alone, and the first
 * batches run while the rest are formed.  tickets[k] identifies
 * reqs[k].  On an error (that of the first failing request) nothing is
 * queued. */
sqc_status sqc_serve_submit_many(sqc_server *srv, const sqc_request *reqs, int32_t n,
                                 uint64_t *tickets);
/* state: 0 waiting, 1 running, 2 done; an admission error is returned here. */
sqc_status sqc_serve_poll(sqc_server *srv, uint64_t ticket, int32_t *state);
/* Block until the request is done. */
sqc_status sqc_serve_wait(sqc_server *srv, uint64_t ticket);
/* Advance the engine, then hand out the tickets of requests that finished
 * since the last call (a completion queue, oldest first): up to `cap` go to
 * `tickets`, their count to `n`; the rest stay queued for the next call.
 * A ticket handed out here is forgotten: later polls of it fail. */
sqc_status sqc_serve_completed(sqc_server *srv, uint64_t *tickets, int32_t cap, int32_t *n);
sqc_status sqc_serve_get_stats(sqc_server *srv, sqc_serve_stats *out);
/* The engine's batching policy on its own (host only, no server needed), for
 * tools and tests: n waiting requests in arrival order with their workspace
 * and job-table bytes and skip counts; the batch takes requests while they
 * fit `room` bytes (a batch of one needs no job table), at most max_batch; a
 * request that does not fit may be passed by later ones, and one passed over
 * 8 times or more stops the scan (*held = 1): nothing behind it is admitted
 * first.  When a batch is formed, each request passed over gains one skip
 * (skips is updated in place).  Writes the positions taken (ascending) to
 * `picked` (capacity n) and their count to *n_picked (0: no batch).  Errors:
 * SQC_E_ARG for NULL pointers, n < 0 or max_batch < 1. */
sqc_status sqc_serve_pick_batch(const size_t *workspace_bytes, const size_t *table_bytes,
                                int32_t *skips, int32_t n, size_t room, int32_t max_batch,
                                int32_t *picked, int32_t *n_picked, int32_t *held);
const char *sqc_serve_last_error(const sqc_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* SQC_H */
