// States merging (Sec. 4, Algorithm 2): sum the attributed entries of the data
// states that share a bin.
//
//   out[sigma][b] = sum_y T[x(b, y)][sigma],
//   x(b, y) = fixed_val | deposit(b, active) | deposit(y, merged)
//
// The attributed tensor is stored [x][sigma] (labels fastest), so every state
// x contributes one contiguous row of 4^c labels: a wave reads 64 consecutive
// labels of one row and the reduction over y is a walk down rows.  For the
// masks Algorithm 2 produces (fixed bits lowest, then active, then merged) the
// rows of consecutive b are consecutive in memory at recursion 0.
//
// A work-group owns a tile of TB bins x TS labels.  Each thread accumulates in
// FP64 in ascending y; thread rows that split y are combined in LDS in a fixed
// order, and a y range split over work-groups (P > 1) goes through an FP64
// partial buffer summed in ascending partial order, so results are
// deterministic.  The tile is written [sigma][b] through LDS so that each
// label row is written as a run of TB consecutive bins.
#include "common.hpp"

#include <vector>

namespace sqc {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 2048;  // outputs per work-group

__device__ __forceinline__ double ld(const void *p, int64_t i, int f32) {
  return f32 ? (double)static_cast<const float *>(p)[i] : static_cast<const double *>(p)[i];
}

__device__ __forceinline__ uint64_t deposit(uint64_t v, uint64_t mask) {
  uint64_t out = 0;
  for (int b = 0; mask; ++b) {
    uint64_t low = mask & (~mask + 1);
    if ((v >> b) & 1) out |= low;
    mask ^= low;
  }
  return out;
}

// deposit() of a value into a mask that is one contiguous run starting at lo
__device__ __forceinline__ uint64_t deposit_run(uint64_t v, uint64_t mask, int lo) {
  return lo >= 0 ? (v << lo) : deposit(v, mask);
}

__device__ __forceinline__ void merge_tiles_body(const MergeArgs &a, int64_t tile_id, int p,
                                                 double *tile) {
  const int TS = 1 << a.ts_bits;
  const int TB = 1 << a.tb_bits;
  const int R = kThreads >> a.ts_bits;        // thread rows
  const int RB = R < TB ? R : TB;             // rows that own distinct bins
  const int YG = R / RB;                      // rows that split y inside the group
  const int BPT = TB / RB;                    // bins per thread
  // LDS row stride: one pad entry per row of 32 or more labels, so the
  // transposed reads (consecutive lanes on consecutive rows) fall on distinct
  // banks (at most 2048 / 32 = 64 pads: the tile's spare)
  const int TSP = TS + (TS >= 32 ? 1 : 0);
  const int tid = threadIdx.x;
  const int sl = tid & (TS - 1);
  const int r = tid >> a.ts_bits;
  const int brow = r % RB;
  const int g = r / RB;

  const int64_t L = int64_t(1) << a.lbits;
  const int64_t Lin = int64_t(1) << a.in_lbits;
  const int lsig_tiles = a.lbits - a.ts_bits;
  const int st = (int)(tile_id & ((int64_t(1) << lsig_tiles) - 1));
  const int64_t bt = tile_id >> lsig_tiles;
  const int64_t sigma = (int64_t(st) << a.ts_bits) + sl;
  const int64_t sigma_in = a.in_lbits == a.lbits ? sigma : (int64_t)(a.lab_fixed | deposit((uint64_t)sigma, a.lab_keep));
  const int64_t b0 = bt << a.tb_bits;

  const int64_t ny = int64_t(1) << (a.mbits - a.ysplit_bits);  // y per work-group
  const int64_t y0 = int64_t(p) * ny;
  const uint64_t nmerged = ~a.merged;

  // the thread's BPT <= kMaxBPT bins: states without the merged bits
  constexpr int kMaxBPT = kTile / kThreads;
  uint64_t xb[kMaxBPT];
  double acc[kMaxBPT];
#pragma unroll
  for (int i = 0; i < kMaxBPT; ++i) {
    const int64_t b = b0 + brow + RB * i;
    xb[i] = i < BPT ? a.fixed_val | deposit_run((uint64_t)b, a.active, a.act_lo) : 0;
    acc[i] = 0.0;
  }
  // y = y0 + g, y0 + g + YG, ...: walk the merged bits' subsets in order; the
  // loads of one y are issued together (clamped offsets, no branches)
  uint64_t z = deposit_run((uint64_t)(y0 + g), a.merged, a.mrg_lo);
  for (int64_t y = g; y < ny; y += YG) {
    int64_t off[kMaxBPT];
#pragma unroll
    for (int i = 0; i < kMaxBPT; ++i) off[i] = i < BPT ? (int64_t)(xb[i] | z) * Lin + sigma_in : 0;
    if (a.in_f32) {
      const float *in = static_cast<const float *>(a.in);
      float v[kMaxBPT];
#pragma unroll
      for (int i = 0; i < kMaxBPT; ++i) v[i] = in[off[i]];
#pragma unroll
      for (int i = 0; i < kMaxBPT; ++i) acc[i] += (double)v[i];
    } else {
      const double *in = static_cast<const double *>(a.in);
      double v[kMaxBPT];
#pragma unroll
      for (int i = 0; i < kMaxBPT; ++i) v[i] = in[off[i]];
#pragma unroll
      for (int i = 0; i < kMaxBPT; ++i) acc[i] += v[i];
    }
    for (int s = 0; s < YG; ++s) z = ((z | nmerged) + 1) & a.merged;
  }
#pragma unroll
  for (int i = 0; i < kMaxBPT; ++i)
    if (i < BPT) tile[(g * TB + brow + RB * i) * TSP + sl] = acc[i];
  __syncthreads();
  // combine the y groups in order; result at tile[bl * TSP + sl]
  if (YG > 1) {
    for (int q = tid; q < TB * TS; q += kThreads) {
      const int row = q >> a.ts_bits, col = q & (TS - 1);
      double s = tile[row * TSP + col];
      for (int gg = 1; gg < YG; ++gg) s += tile[(gg * TB + row) * TSP + col];
      tile[row * TSP + col] = s;
    }
    __syncthreads();
  }
  // write: [sigma][b] with b fastest, or partial[p][b][sigma] with sigma fastest
  const int64_t nb = int64_t(1) << a.abits;
  if (a.ysplit_bits == 0) {
    for (int q = tid; q < TB * TS; q += kThreads) {
      int bl = q & (TB - 1);
      int s = q >> a.tb_bits;
      double v = tile[bl * TSP + s];
      int64_t o = ((int64_t(st) << a.ts_bits) + s) * nb + b0 + bl;
      if (a.out_f32) __builtin_nontemporal_store((float)v, static_cast<float *>(a.out) + o);
      else static_cast<double *>(a.out)[o] = v;
    }
  } else {
    for (int q = tid; q < TB * TS; q += kThreads) {
      int s = q & (TS - 1);
      int bl = q >> a.ts_bits;
      a.partial[(int64_t(p) * nb + b0 + bl) * L + (int64_t(st) << a.ts_bits) + s] = tile[bl * TSP + s];
    }
  }
}

// Large reductions: a thread owns V consecutive output columns c = b * L +
// sigma (same bin, consecutive labels) and walks its share of the merged
// states, four rows per iteration so that several loads are in flight.  The
// work-group's FP64 partial sums go to partial[p][c].
__device__ __forceinline__ void merge_rows_body(const MergeArgs &a, int64_t bx, int p) {
  const int V = merge_vec(a);
  const int64_t L = int64_t(1) << a.lbits;
  const int64_t NC = int64_t(1) << (a.abits + a.lbits);
  const int64_t c0 = (bx * kThreads + threadIdx.x) * V;
  if (c0 >= NC) return;
  const int64_t b = c0 >> a.lbits;
  const int64_t sigma_out = c0 & (L - 1);
  // input label of the first of the V labels (the V are consecutive there)
  const int64_t sigma =
      a.in_lbits == a.lbits ? sigma_out : (int64_t)(a.lab_fixed | deposit((uint64_t)sigma_out, a.lab_keep));
  const int64_t Lin = int64_t(1) << a.in_lbits;
  const uint64_t xb = a.fixed_val | deposit_run((uint64_t)b, a.active, a.act_lo);
  const int64_t ny = int64_t(1) << (a.mbits - a.ysplit_bits);
  const uint64_t nmerged = ~a.merged;
  uint64_t z = deposit_run((uint64_t)(int64_t(p) * ny), a.merged, a.mrg_lo);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t y = 0;
  if (a.in_f32) {
    const float *in = static_cast<const float *>(a.in);
    for (; y + 4 <= ny; y += 4) {
      int64_t r[4];
      for (int u = 0; u < 4; ++u) {
        r[u] = (int64_t)(xb | z) * Lin + sigma;
        z = ((z | nmerged) + 1) & a.merged;
      }
      if (V == 4) {
        float4 v[4];
        for (int u = 0; u < 4; ++u) v[u] = *reinterpret_cast<const float4 *>(in + r[u]);
        for (int u = 0; u < 4; ++u) {
          acc[0] += v[u].x; acc[1] += v[u].y; acc[2] += v[u].z; acc[3] += v[u].w;
        }
      } else {
        float v[4];
        for (int u = 0; u < 4; ++u) v[u] = in[r[u]];
        for (int u = 0; u < 4; ++u) acc[0] += v[u];
      }
    }
    for (; y < ny; ++y) {
      int64_t r0 = (int64_t)(xb | z) * Lin + sigma;
      z = ((z | nmerged) + 1) & a.merged;
      for (int q = 0; q < V; ++q) acc[q] += in[r0 + q];
    }
  } else {
    const double *in = static_cast<const double *>(a.in);
    for (; y + 4 <= ny; y += 4) {
      int64_t r[4];
      for (int u = 0; u < 4; ++u) {
        r[u] = (int64_t)(xb | z) * Lin + sigma;
        z = ((z | nmerged) + 1) & a.merged;
      }
      if (V == 4) {
        double2 v[4][2];
        for (int u = 0; u < 4; ++u) {
          v[u][0] = *reinterpret_cast<const double2 *>(in + r[u]);
          v[u][1] = *reinterpret_cast<const double2 *>(in + r[u] + 2);
        }
        for (int u = 0; u < 4; ++u) {
          acc[0] += v[u][0].x; acc[1] += v[u][0].y; acc[2] += v[u][1].x; acc[3] += v[u][1].y;
        }
      } else {
        double v[4];
        for (int u = 0; u < 4; ++u) v[u] = in[r[u]];
        for (int u = 0; u < 4; ++u) acc[0] += v[u];
      }
    }
    for (; y < ny; ++y) {
      int64_t r0 = (int64_t)(xb | z) * Lin + sigma;
      z = ((z | nmerged) + 1) & a.merged;
      for (int q = 0; q < V; ++q) acc[q] += in[r0 + q];
    }
  }
  double *dst = a.partial + int64_t(p) * NC + c0;
  for (int q = 0; q < V; ++q) dst[q] = acc[q];
}

// Sum the partials of every column in ascending partial order and write
// out[sigma][b] (columns are read contiguously; the output is small).
__device__ __forceinline__ void merge_finish_body(const MergeArgs &a, int64_t blk, int64_t nblk) {
  const int64_t NC = int64_t(1) << (a.abits + a.lbits);
  const int64_t L = int64_t(1) << a.lbits;
  const int64_t nb = int64_t(1) << a.abits;
  const int P = 1 << a.ysplit_bits;
  for (int64_t c = blk * kThreads + threadIdx.x; c < NC; c += nblk * kThreads) {
    // partials added in ascending order; eight loads in flight at a time
    double s = 0.0;
    int q = 0;
    for (; q + 8 <= P; q += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = a.partial[int64_t(q + u) * NC + c];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; q < P; ++q) s += a.partial[int64_t(q) * NC + c];
    int64_t o = (c & (L - 1)) * nb + (c >> a.lbits);
    if (a.out_f32) static_cast<float *>(a.out)[o] = (float)s;
    else static_cast<double *>(a.out)[o] = s;
  }
}

// Grid shape of one merge (work-groups of each pass) and its y split.
void shape_merge(MergeArgs &a) {
  if (a.mbits >= 6) {
    // streaming reduction over many merged states, then the partial sums
    const int V = merge_vec(a);
    int64_t NC = int64_t(1) << (a.abits + a.lbits);
    int64_t bx = (NC / V + kThreads - 1) / kThreads;
    int ys = 0;
    while (bx * (int64_t(2) << ys) <= 1024 && a.mbits - (ys + 1) >= 4) ++ys;
    a.ysplit_bits = ys;
    a.grid_x = bx;
    a.blocks = bx << ys;
    int64_t fin = (NC + kThreads - 1) / kThreads;
    a.fin_blocks = fin > 65536 ? 65536 : fin;
    return;
  }
  a.ysplit_bits = 0;
  a.ts_bits = a.lbits < 6 ? a.lbits : 6;
  int tb = 11 - a.ts_bits;  // kTile = 2^11 outputs
  if (tb > a.abits) tb = a.abits;
  a.tb_bits = tb;
  a.blocks = (int64_t(1) << (a.lbits - a.ts_bits)) * (int64_t(1) << (a.abits - tb));
  a.grid_x = a.blocks;
  a.fin_blocks = 0;
}

// Several merges in one launch: work-group w belongs to the job j with
// start[j] <= w < start[j + 1] (a uniform scan over at most kMergeJobs
// entries), and runs that job's pass with its local index.
struct MergeBatch {
  int n;
  int64_t start[kMergeJobs + 1];
  MergeArgs job[kMergeJobs];
};

__device__ __forceinline__ int batch_job(const MergeBatch &b, int64_t w) {
  int j = 0;
  while (j + 1 < b.n && w >= b.start[j + 1]) ++j;
  return j;
}

__global__ __launch_bounds__(kThreads) void merge_tiles(MergeBatch b) {
  __shared__ double tile[kTile + 64];
  const int j = batch_job(b, blockIdx.x);
  merge_tiles_body(b.job[j], int64_t(blockIdx.x) - b.start[j], 0, tile);
}

__global__ __launch_bounds__(kThreads) void merge_rows(MergeBatch b) {
  const int j = batch_job(b, blockIdx.x);
  const MergeArgs &a = b.job[j];
  const int64_t w = int64_t(blockIdx.x) - b.start[j];
  merge_rows_body(a, w % a.grid_x, (int)(w / a.grid_x));
}

__global__ __launch_bounds__(kThreads) void merge_finish(MergeBatch b) {
  const int j = batch_job(b, blockIdx.x);
  merge_finish_body(b.job[j], int64_t(blockIdx.x) - b.start[j], b.job[j].fin_blocks);
}

// Job j of a device table with work-group prefix `start` (n + 1 entries,
// start[0] = 0): the largest j with start[j] <= w (a uniform binary search).
__device__ __forceinline__ int find_job(const int *__restrict__ start, int n, int w) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// The same passes over a device table of shaped jobs (requests batched by the
// serving engine).
// (work-groups past start[n] do nothing: a launch may size its grid for the
// largest of several tables that its jobs are later copied from)
__global__ __launch_bounds__(kThreads) void merge_tiles_grouped(const MergeArgs *__restrict__ jobs,
                                                                 const int *__restrict__ start, int n) {
  __shared__ double tile[kTile + 64];
  if ((int)blockIdx.x >= start[n]) return;
  const int j = find_job(start, n, blockIdx.x);
  merge_tiles_body(jobs[j], int64_t(blockIdx.x) - start[j], 0, tile);
}

__global__ __launch_bounds__(kThreads) void merge_rows_grouped(const MergeArgs *__restrict__ jobs,
                                                                const int *__restrict__ start, int n) {
  if ((int)blockIdx.x >= start[n]) return;
  const int j = find_job(start, n, blockIdx.x);
  const MergeArgs &a = jobs[j];
  const int64_t w = int64_t(blockIdx.x) - start[j];
  merge_rows_body(a, w % a.grid_x, (int)(w / a.grid_x));
}

__global__ __launch_bounds__(kThreads) void merge_finish_grouped(const MergeArgs *__restrict__ jobs,
                                                                  const int *__restrict__ start, int n) {
  if ((int)blockIdx.x >= start[n]) return;
  const int j = find_job(start, n, blockIdx.x);
  merge_finish_body(jobs[j], int64_t(blockIdx.x) - start[j], jobs[j].fin_blocks);
}

// Largest |entry| of every label row of a merged tensor [rows][cols]: one
// work-group per row at a time, FP64 result.  The precision selector
// contracts these maxima into a certified bound of the bins' sums of |terms|.
// max that keeps a NaN (fmax drops it), so a NaN entry reaches the bound
__device__ inline double nan_max(double m, double a) { return (a > m || a != a) ? a : m; }

__global__ __launch_bounds__(kThreads) void row_absmax(const void *in, int in_f32, double *out, int64_t rows,
                                                       int64_t cols) {
  __shared__ double part[kThreads / 64];
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    double m = 0.0;
    for (int64_t c = threadIdx.x; c < cols; c += kThreads) {
      const double v = in_f32 ? (double)static_cast<const float *>(in)[r * cols + c]
                              : static_cast<const double *>(in)[r * cols + c];
      m = nan_max(m, fabs(v));
    }
    for (int off = 32; off >= 1; off >>= 1) m = nan_max(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double x = part[0];
      for (int w = 1; w < kThreads / 64; ++w) x = nan_max(x, part[w]);
      out[r] = x;
    }
    __syncthreads();
  }
}

enum Pass { kTiles, kRows, kFinish };

int64_t pass_blocks(const MergeArgs &a, Pass p) { return p == kFinish ? a.fin_blocks : a.blocks; }

void launch_pass(const std::vector<MergeArgs> &jobs, Pass p, hipStream_t s) {
  MergeBatch b{};
  auto flush = [&]() {
    if (!b.n) return;
    const unsigned grid = (unsigned)b.start[b.n];
    if (p == kTiles) hipLaunchKernelGGL(merge_tiles, dim3(grid), dim3(kThreads), 0, s, b);
    else if (p == kRows) hipLaunchKernelGGL(merge_rows, dim3(grid), dim3(kThreads), 0, s, b);
    else hipLaunchKernelGGL(merge_finish, dim3(grid), dim3(kThreads), 0, s, b);
    b = MergeBatch{};
  };
  for (const MergeArgs &a : jobs) {
    const int64_t nb = pass_blocks(a, p);
    if (b.n == kMergeJobs || b.start[b.n] + nb > (int64_t(1) << 31) - 1) flush();
    b.job[b.n] = a;
    b.start[b.n + 1] = b.start[b.n] + nb;
    ++b.n;
  }
  flush();
}

}  // namespace

int64_t merge_partial_elems(int abits, int lbits, int mbits) {
  if (mbits < 6) return 0;
  MergeArgs a{};
  a.abits = abits;
  a.lbits = lbits;
  a.in_lbits = lbits;  // vector loads: the most partials a slice's merge takes
  a.mbits = mbits;
  shape_merge(a);
  return (int64_t(1) << (abits + lbits)) << a.ysplit_bits;
}

void merge_shape(MergeArgs &a) { shape_merge(a); }

int64_t merge_pass_blocks(const MergeArgs &a, int pass) {
  const bool rows = a.mbits >= 6;
  if (pass == kTiles) return rows ? 0 : a.blocks;
  if (pass == kRows) return rows ? a.blocks : 0;
  return rows ? a.fin_blocks : 0;
}

void launch_merge_grouped(int pass, const MergeArgs *jobs, const int *start, int n, int total,
                          hipStream_t s) {
  if (pass == kTiles)
    hipLaunchKernelGGL(merge_tiles_grouped, dim3((unsigned)total), dim3(kThreads), 0, s, jobs, start, n);
  else if (pass == kRows)
    hipLaunchKernelGGL(merge_rows_grouped, dim3((unsigned)total), dim3(kThreads), 0, s, jobs, start, n);
  else
    hipLaunchKernelGGL(merge_finish_grouped, dim3((unsigned)total), dim3(kThreads), 0, s, jobs, start, n);
}

void launch_row_absmax(const void *in, int in_f32, double *out, int64_t rows, int64_t cols, hipStream_t s) {
  const int64_t g = rows < 4096 ? rows : 4096;
  if (g > 0) hipLaunchKernelGGL(row_absmax, dim3((unsigned)g), dim3(kThreads), 0, s, in, in_f32, out, rows, cols);
}

void launch_merges(const MergeArgs *jobs, int n, hipStream_t s) {
  std::vector<MergeArgs> tiles, rows;
  for (int i = 0; i < n; ++i) {
    MergeArgs a = jobs[i];
    shape_merge(a);
    (a.mbits >= 6 ? rows : tiles).push_back(a);
  }
  if (!tiles.empty()) launch_pass(tiles, kTiles, s);
  if (!rows.empty()) {
    launch_pass(rows, kRows, s);
    launch_pass(rows, kFinish, s);
  }
}

}  // namespace sqc
