// Library-internal interface of the serving engine to the recursion path:
// validated, planned requests and their enqueueing alone or as a batch whose
// launches are shared by all requests (job tables in device memory).
#pragma once

#include <memory>
#include <vector>

#include "../../include/sqc.h"

namespace sqc {

// A registered circuit: its compute graph and attributed tensors.
struct CircuitTopo;
// One recursion request with its bin masks and workspace plan.
struct PreparedRecursion;
struct PreparedDeleter {
  void operator()(PreparedRecursion *p) const;
};
using PreparedPtr = std::unique_ptr<PreparedRecursion, PreparedDeleter>;

// Validate the tensors against the cut list (throws Error).
std::shared_ptr<const CircuitTopo> make_circuit(const sqc_tensor *att, int n_sub, const sqc_cut *cuts,
                                                int n_cuts);
int circuit_n_sub(const CircuitTopo &c);

// Validate and plan one recursion (throws Error).
PreparedPtr prepare_recursion(std::shared_ptr<const CircuitTopo> c, const sqc_masks *scope, uint64_t M,
                              int top_r, sqc_prec prec, void *bins, sqc_prec bins_prec, void *top_dev,
                              void *sum_dev);
// Workspace bytes of the request (from a 256-byte aligned base).
size_t prepared_workspace(const PreparedRecursion &p);
// Upper bound of the request's share of a batch's job table.
size_t prepared_table_bytes(const PreparedRecursion &p);
// The bin masks the recursion uses (n_sub entries).
const sqc_masks *prepared_masks(const PreparedRecursion &p);

// Enqueue one request on the context's stream with its workspace at `ws`.
void enqueue_prepared(sqc_ctx *ctx, const PreparedRecursion &p, char *ws);
// Enqueue n requests as one batch on the context's stream: request i uses
// the workspace at ws[i]; the job tables are written to `staging` (pinned
// host memory of staging_bytes, untouched by the caller until the stream has
// passed this batch) and copied to `table_dev` (table_bytes).  Each request's
// results are bitwise the same as enqueue_prepared's.  Throws Error.
void enqueue_batch(sqc_ctx *ctx, PreparedRecursion *const *p, int n, char *const *ws, char *table_dev,
                   size_t table_bytes, void *staging, size_t staging_bytes);

}  // namespace sqc
