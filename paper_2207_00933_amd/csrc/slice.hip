// First-level index slicing (Sec. 6.3): the contraction over every cut label
// is split into slices, one per label assignment of the sliced cuts, whose
// bin vectors add up to the full result.
//
// slice_rows: restrict a merged tensor [sigma][b] to one slice.  The rows
// kept are those whose sliced label digits hold the slice's values; they are
// written in ascending order of the remaining digits, which is the merged
// layout of the same subcircuit with the sliced cuts removed.  Row r of the
// output reads row  fixed + sum_j ((r >> lo_j) & (2^len_j - 1)) << pos_j
// of the input (runs of kept label bits).  Rows are contiguous runs of
// 2^n_bits elements: copied in 16-byte units when a row holds at least 16
// bytes, else in 4-byte words.
//
// The slices' bin vectors are added by the final contraction step itself
// (its slice-accumulating epilogue), so no slice vector is stored.
#include "common.hpp"

namespace sqc {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int64_t source_row(const SliceArgs &a, int64_t r) {
  int64_t src = a.fixed;
  for (int j = 0; j < a.nruns; ++j)
    src += ((r >> a.lo[j]) & ((int64_t(1) << a.len[j]) - 1)) << a.pos[j];
  return src;
}

__global__ __launch_bounds__(kThreads) void slice_rows16(SliceArgs a) {
  // units of 16 bytes; a row holds 2^row_shift of them
  const int64_t total = a.rows << a.row_shift;
  const uint4 *in = static_cast<const uint4 *>(a.in);
  uint4 *out = static_cast<uint4 *>(a.out);
  for (int64_t u = int64_t(blockIdx.x) * kThreads + threadIdx.x; u < total;
       u += int64_t(gridDim.x) * kThreads) {
    const int64_t r = u >> a.row_shift, w = u & ((int64_t(1) << a.row_shift) - 1);
    out[u] = in[(source_row(a, r) << a.row_shift) + w];
  }
}

__global__ __launch_bounds__(kThreads) void slice_rows4(SliceArgs a) {
  // units of 4 bytes
  const int64_t total = a.rows << a.row_shift;
  const uint32_t *in = static_cast<const uint32_t *>(a.in);
  uint32_t *out = static_cast<uint32_t *>(a.out);
  for (int64_t u = int64_t(blockIdx.x) * kThreads + threadIdx.x; u < total;
       u += int64_t(gridDim.x) * kThreads) {
    const int64_t r = u >> a.row_shift, w = u & ((int64_t(1) << a.row_shift) - 1);
    out[u] = in[(source_row(a, r) << a.row_shift) + w];
  }
}

int grid_for(int64_t units) {
  const int64_t g = (units + kThreads - 1) / kThreads;
  return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

}  // namespace

void launch_slice_rows(const SliceArgs &a, hipStream_t s) {
  if (a.rows <= 0) return;
  if (a.row_bytes_log2 >= 4) {
    SliceArgs b = a;
    b.row_shift = a.row_bytes_log2 - 4;
    hipLaunchKernelGGL(slice_rows16, dim3(grid_for(b.rows << b.row_shift)), dim3(kThreads), 0, s, b);
  } else {
    SliceArgs b = a;
    b.row_shift = a.row_bytes_log2 - 2;
    hipLaunchKernelGGL(slice_rows4, dim3(grid_for(b.rows << b.row_shift)), dim3(kThreads), 0, s, b);
  }
}

}  // namespace sqc
