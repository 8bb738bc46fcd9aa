// Pairwise contraction of compute-graph tensors (Sec. 6.1: contracting two
// subcircuit tensors over their shared cut indices is the matrix product
// C = A B) as a strided-tensor GEMM on MFMA:
//
//   C[offC_m(m) + offC_n(n)] = sum_k A[offA_m(m) + offA_k(k)] * B[offB_n(n) + offB_k(k)]
//
// m runs over A's free axes, n over B's free axes, k over the shared cut
// labels; every dimension is a power of two and each offset is a sum of
// per-run shifted bit fields (IndexMap), so operands are read in place,
// whatever axis order the previous step left them in.
//
// Precisions: F64 (v_mfma_f64_16x16x4f64 on FP64 tensors), F32
// (v_mfma_f32_32x32x2f32) and BF16X3 (each FP32 operand split into bf16
// hi + lo by round-to-nearest-even conversions when staged into LDS;
// lo*hi + hi*lo + hi*hi on v_mfma_f32_32x32x16_bf16, FP32 accumulation).  On
// the last step of a contraction whose K spans several stages of 64 labels
// the FP32 sum of each stage is folded into FP64 with Neumaier compensation; every wave writes the FP64 sum and the maximum of its
// 32 x 32 sub-tile for the top-R selection.
//
// Schedule: a work-group (4 waves, 64 x 64 output tile, waves 32 x 32) is
// persistent over a contiguous share of the tiles; tiles of one XCD's
// work-groups are adjacent so A row panels are shared through that XCD's L2.
// With a single K stage the staged A panel stays in LDS across the n tiles of
// one m panel.  The operands of the next (tile, K stage) are loaded into
// registers while the current one is multiplied and stored.  The MFMA
// operands are swapped (B feeds the instruction's A side) so the lanes of a
// result store run along m, the contiguous output axis.
#include "common.hpp"

namespace sqc {

namespace {

constexpr int kThreads = 256;
constexpr int BM = 64;
constexpr int BN = 64;
constexpr int BK = 64;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// Offsets by index map: strides are powers of two, so each run is a shift.
// Indices of one GEMM dimension fit 31 bits (checked on the host).
__device__ __forceinline__ int64_t map_x(const IndexMap &m, uint32_t idx) {
  int64_t off = 0;
  for (int r = 0; r < m.nruns; ++r) {
    off += int64_t(idx & ((1u << m.bits[r]) - 1u)) << m.lx[r];
    idx >>= m.bits[r];
  }
  return off;
}

__device__ __forceinline__ int64_t map_y(const IndexMap &m, uint32_t idx) {
  int64_t off = 0;
  for (int r = 0; r < m.nruns; ++r) {
    off += int64_t(idx & ((1u << m.bits[r]) - 1u)) << m.ly[r];
    idx >>= m.bits[r];
  }
  return off;
}

__device__ __forceinline__ void neumaier(double &s, double &c, double x) {
  double t = s + x;
  if (fabs(s) >= fabs(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

// lexicographic "better": larger value, then lower index
__device__ __forceinline__ bool better(double v1, uint64_t i1, double v2, uint64_t i2) {
  return v1 > v2 || (v1 == v2 && i1 < i2);
}

__device__ __forceinline__ void wave_argmax(double &v, uint64_t &i) {
  for (int off = 32; off >= 1; off >>= 1) {
    double ov = __shfl_xor(v, off);
    uint64_t oi = __shfl_xor(i, off);
    if (better(ov, oi, v, i)) {
      v = ov;
      i = oi;
    }
  }
}

// Block-wide argmax (all threads get the result); sv / si hold one entry per wave.
__device__ __forceinline__ void block_argmax(double &v, uint64_t &i, double *sv, uint64_t *si) {
  wave_argmax(v, i);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sv[w] = v;
    si[w] = i;
  }
  __syncthreads();
  v = sv[0];
  i = si[0];
  for (int q = 1; q < (int)(blockDim.x >> 6); ++q)
    if (better(sv[q], si[q], v, i)) {
      v = sv[q];
      i = si[q];
    }
}

// Inclusive scan of one int per thread over the block (Hillis-Steele).
__device__ int block_scan_incl(int v, int *buf) {
  const int tid = threadIdx.x;
  buf[tid] = v;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    int add = tid >= off ? buf[tid - off] : 0;
    __syncthreads();
    buf[tid] += add;
    __syncthreads();
  }
  return buf[tid];
}

// Per-wave accumulators.  The MFMA operands are swapped (B feeds the
// instruction's A side), so result rows run over n and columns over m:
//   F32, BF16X3: one 32 x 32 block, element r of lane l at
//                m = l % 32, n = 8 (r / 4) + 4 (l / 32) + r % 4
//   F64:         2 x 2 blocks of 16 x 16, block (jn, im), element r of lane l
//                at m = 16 im + l % 16, n = 16 jn + l / 16 + 4 r
// so the lanes of one store cover consecutive m: whole 128-byte lines when m
// is the contiguous axis of C.
template <int PREC>
struct Tr {
  typedef float T;
  typedef v16f Acc;
  static constexpr int NACC = 1;
};
template <>
struct Tr<SQC_F64> {
  typedef double T;
  typedef v4d Acc;
  static constexpr int NACC = 4;
};

struct Sched {
  int first, end;  // this work-group's tiles: [first, end)
};

// Contiguous chunks of tiles per work-group; work-groups are dispatched
// round-robin over 8 XCDs, so chunk order follows (XCD, work-group within the
// XCD) and the chunks of one XCD are adjacent (shared A panels stay in its L2).
__device__ __forceinline__ Sched schedule(int ntiles) {
  const int G = gridDim.x, b = blockIdx.x;
  const int lb = (G & 7) == 0 ? (b & 7) * (G >> 3) + (b >> 3) : b;
  Sched s;
  s.first = (int)((int64_t)lb * ntiles / G);
  s.end = (int)((int64_t)(lb + 1) * ntiles / G);
  return s;
}

// Index maps are linear in the index bits: map(a | b) = map(a) + map(b) for
// disjoint a and b.  Every offset below is split into a part shared by the
// wave (tile origin, K stage, row block: scalar registers) and a per-lane
// part computed once.
//
// FOLD: the final K axis spans several K stages; the FP32 sum of each stage
// (one chunk of 2^6 labels) is folded into FP64 with Neumaier compensation.
// Otherwise the FP32 accumulator is the result.
template <int PREC, bool FOLD>
__global__ __launch_bounds__(kThreads) void gemm(GemmArgs g) {
  typedef typename Tr<PREC>::T T;
  typedef typename Tr<PREC>::Acc Acc;
  constexpr int NACC = Tr<PREC>::NACC;
  constexpr bool SPLIT = PREC == SQC_BF16X3;
  constexpr int PAD = 8;    // bf16 row padding (keeps rows 16-byte aligned)
  constexpr int LDK = BK + PAD;
  constexpr int NJ = 16;    // staged elements per thread per operand
  // F32/F64: As[k][m], Bs[k][n]; BF16X3: Ah, Al [m][k], Bh, Bl [n][k]
  constexpr int kHalf = SPLIT ? (2 * BM * LDK * 2) : (BK * BM * (int)sizeof(T));
  __shared__ __attribute__((aligned(16))) unsigned char lds[2 * kHalf];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 1, wn = wave >> 1;
  const uint32_t M = 1u << g.mbits;
  const uint32_t N = 1u << g.nbits;
  const uint32_t K = 1u << g.kbits;
  const int lnt = g.nbits > 6 ? g.nbits - 6 : 0;        // log2 of the n-tile count
  const int lmt = g.mbits > 6 ? g.mbits - 6 : 0;
  const int nks = g.kbits > 6 ? 1 << (g.kbits - 6) : 1;  // K stages of BK

  const Sched sc = schedule(1 << (lmt + lnt));
  if (sc.first >= sc.end) return;

  // staging: the thread holds column `lane` (m of A, n of B) of the tile at
  // the 16 k rows 16 wave + j
  const int64_t a_lane = map_x(g.m, lane);
  const int64_t b_lane = map_x(g.n, lane);
  const int64_t a_kw = map_x(g.k, 16 * wave);
  const int64_t b_kw = map_y(g.k, 16 * wave);
  T av[NJ], bv[NJ];
  auto load_a = [&](int tile, int ks) {
    const uint32_t m0 = (uint32_t)(tile >> lnt) << 6;
    const uint32_t k0 = (uint32_t)ks << 6;
    const T *base = static_cast<const T *>(g.A) + (map_x(g.m, m0) + map_x(g.k, k0) + a_kw);
    const bool ok = m0 + lane < M;
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      av[j] = (ok && k0 + 16 * wave + j < K) ? base[g.koff_a[j] + a_lane] : T(0);
  };
  auto load_b = [&](int tile, int ks) {
    const uint32_t n0 = (uint32_t)(tile & ((1 << lnt) - 1)) << 6;
    const uint32_t k0 = (uint32_t)ks << 6;
    const T *base = static_cast<const T *>(g.B) + (map_x(g.n, n0) + map_y(g.k, k0) + b_kw);
    const bool ok = n0 + lane < N;
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      bv[j] = (ok && k0 + 16 * wave + j < K) ? base[g.koff_b[j] + b_lane] : T(0);
  };
  auto stage = [&](const T *v, unsigned char *dst, int ld) {
    if constexpr (!SPLIT) {
      T *S = reinterpret_cast<T *>(dst);
#pragma unroll
      for (int j = 0; j < NJ; ++j) S[(16 * wave + j) * ld + lane] = v[j];
    } else {
      // 16 consecutive k of one column: two 16-byte rows of hi and of lo
      v8bf h0, h1, l0, l1;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const __bf16 a = (__bf16)v[j], b = (__bf16)v[j + 8];
        h0[j] = a;
        h1[j] = b;
        l0[j] = (__bf16)(v[j] - (float)a);
        l1[j] = (__bf16)(v[j + 8] - (float)b);
      }
      __bf16 *H = reinterpret_cast<__bf16 *>(dst) + lane * LDK + 16 * wave;
      __bf16 *L = H + BM * LDK;
      *reinterpret_cast<v8bf *>(H) = h0;
      *reinterpret_cast<v8bf *>(H + 8) = h1;
      *reinterpret_cast<v8bf *>(L) = l0;
      *reinterpret_cast<v8bf *>(L + 8) = l1;
    }
  };

  Acc acc[NACC];
  constexpr int NE = NACC * (PREC == SQC_F64 ? 4 : 16);  // result elements per lane
  double S[FOLD ? NE : 1], Cc[FOLD ? NE : 1];
  auto reset = [&]() {
    for (int q = 0; q < NACC; ++q) acc[q] = Acc{};
    if constexpr (FOLD) {
      for (int e = 0; e < NE; ++e) S[e] = Cc[e] = 0.0;
    }
  };
  auto fold = [&]() {
    if constexpr (FOLD) {
      for (int q = 0; q < NACC; ++q)
        for (int r = 0; r < NE / NACC; ++r) neumaier(S[q * (NE / NACC) + r], Cc[q * (NE / NACC) + r], (double)acc[q][r]);
      for (int q = 0; q < NACC; ++q) acc[q] = Acc{};
    }
  };
  // one MFMA k step (KSTEP labels) of this wave's 32 x 32 result
  constexpr int KSTEP = PREC == SQC_F64 ? 4 : (SPLIT ? 16 : 2);
  auto mfma_step = [&](int kk) {
    if constexpr (PREC == SQC_F64) {
      const double *As = reinterpret_cast<const double *>(lds);
      const double *Bs = reinterpret_cast<const double *>(lds + kHalf);
      const int kr = kk * 4 + (lane >> 4);
      double a[2], b[2];
      for (int i = 0; i < 2; ++i) a[i] = As[kr * BM + wm * 32 + i * 16 + (lane & 15)];
      for (int j = 0; j < 2; ++j) b[j] = Bs[kr * BN + wn * 32 + j * 16 + (lane & 15)];
      for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 2; ++i)
          acc[2 * j + i] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[j], a[i], acc[2 * j + i], 0, 0, 0);
    } else if constexpr (!SPLIT) {
      const float *As = reinterpret_cast<const float *>(lds);
      const float *Bs = reinterpret_cast<const float *>(lds + kHalf);
      const int kr = kk * 2 + (lane >> 5);
      const float a = As[kr * BM + wm * 32 + (lane & 31)];
      const float b = Bs[kr * BN + wn * 32 + (lane & 31)];
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(b, a, acc[0], 0, 0, 0);
    } else {
      const __bf16 *Ah = reinterpret_cast<const __bf16 *>(lds);
      const __bf16 *Al = Ah + BM * LDK;
      const __bf16 *Bh = reinterpret_cast<const __bf16 *>(lds + kHalf);
      const __bf16 *Bl = Bh + BN * LDK;
      const int kc = kk * 16 + 8 * (lane >> 5);
      const int ra = (wm * 32 + (lane & 31)) * LDK + kc;
      const int rb = (wn * 32 + (lane & 31)) * LDK + kc;
      const v8bf ah = *reinterpret_cast<const v8bf *>(Ah + ra);
      const v8bf al = *reinterpret_cast<const v8bf *>(Al + ra);
      const v8bf bh = *reinterpret_cast<const v8bf *>(Bh + rb);
      const v8bf bl = *reinterpret_cast<const v8bf *>(Bl + rb);
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bl, ah, acc[0], 0, 0, 0);
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bh, al, acc[0], 0, 0, 0);
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bh, ah, acc[0], 0, 0, 0);
    }
  };

  // per-lane parts of the result offsets
  int64_t c_lane_m, c_lane_n;
  if constexpr (PREC == SQC_F64) {
    c_lane_m = map_y(g.m, lane & 15);
    c_lane_n = map_y(g.n, lane >> 4);
  } else {
    c_lane_m = map_y(g.m, lane & 31);
    c_lane_n = map_y(g.n, 4 * (lane >> 5));
  }
  reset();

  // A stays staged while consecutive tiles share the m panel (single stage);
  // B stays staged when there is a single n tile and a single stage.
  const bool reuse_a = nks == 1;
  const bool reuse_b = nks == 1 && lnt == 0;
  int tile = sc.first, ks = 0;
  bool need_a = true, need_b = true;
  load_a(tile, ks);
  load_b(tile, ks);
  while (true) {
    if (need_a) stage(av, lds, BM);
    if (need_b) stage(bv, lds + kHalf, BN);
    __syncthreads();
    // ---- prefetch the next (tile, stage) into registers ----
    const int cur_tile = tile, cur_ks = ks;
    bool more;
    if (ks + 1 < nks) {
      ++ks;
      more = true;
    } else {
      ks = 0;
      ++tile;
      more = tile < sc.end;
    }
    need_a = !(reuse_a && (tile >> lnt) == (cur_tile >> lnt));
    need_b = !reuse_b;
    if (more) {
      if (need_a) load_a(tile, ks);
      if (need_b) load_b(tile, ks);
    }
    // ---- MFMA on the staged stage ----
    const uint32_t k0 = (uint32_t)cur_ks << 6;
    const int kend = (K - k0) < (uint32_t)BK ? (int)(K - k0) : BK;
    if (kend == BK) {
#pragma unroll
      for (int kk = 0; kk < BK / KSTEP; ++kk) mfma_step(kk);
    } else {
      for (int kk = 0; kk * KSTEP < kend; ++kk) mfma_step(kk);
    }
    fold();  // one FP32 chunk per K stage
    // ---- epilogue after the tile's last stage ----
    if (cur_ks == nks - 1) {
      const uint32_t mw = ((uint32_t)(cur_tile >> lnt) << 6) + wm * 32;  // wave origin
      const uint32_t nw = ((uint32_t)(cur_tile & ((1 << lnt) - 1)) << 6) + wn * 32;
      double lsum = 0.0, lmax = -INFINITY;
      if (mw < M && nw < N) {
        const int64_t cw = map_y(g.m, mw) + map_y(g.n, nw);
        auto put = [&](uint32_t mloc, uint32_t nloc, int64_t o, double v) {
          if (mw + mloc >= M || nw + nloc >= N) return;
          double stored;
          if (g.out_f32) {
            const float f = (float)v;
            static_cast<float *>(g.C)[o] = f;
            stored = (double)f;
          } else {
            static_cast<double *>(g.C)[o] = v;
            stored = v;
          }
          lsum += v;
          lmax = fmax(lmax, stored);
        };
        if constexpr (PREC == SQC_F64) {
#pragma unroll
          for (int jn = 0; jn < 2; ++jn)
#pragma unroll
            for (int im = 0; im < 2; ++im)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const uint32_t nl = 16 * jn + 4 * r;
                const int64_t o = cw + (im ? g.coff_m16 : 0) + g.coff_n[4 * jn + r] + c_lane_m + c_lane_n;
                put(16 * im + (lane & 15), nl + (lane >> 4), o, acc[2 * jn + im][r]);
              }
        } else {
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const uint32_t nl = 8 * (r >> 2) + (r & 3);
            const int64_t o = cw + g.coff_n[r] + c_lane_m + c_lane_n;
            double v;
            if constexpr (FOLD) v = S[r] + Cc[r];
            else v = (double)acc[0][r];
            put(lane & 31, nl + 4 * (lane >> 5), o, v);
          }
        }
      }
      if (g.stats) {
        for (int off = 32; off >= 1; off >>= 1) {
          lsum += __shfl_xor(lsum, off);
          lmax = fmax(lmax, __shfl_xor(lmax, off));
        }
        if (lane == 0) {
          g.blk_sum[(int64_t)cur_tile * 4 + wave] = lsum;
          g.blk_max[(int64_t)cur_tile * 4 + wave] = lmax;
        }
      }
      reset();
    }
    if (!more) break;
    __syncthreads();  // LDS is rewritten by the next stage
  }
}

// ---------------------------------------------------------------------------
// top-R selection over the final bins.  The unit is the 32 x 32 sub-tile of
// one wave (sub-tile s = tile * 4 + wave), whose FP64 sum and maximum the
// final GEMM wrote.
// ---------------------------------------------------------------------------

constexpr int kSelThreads = 1024;
constexpr int kSelWaves = kSelThreads / 64;
constexpr int kRankCap = 2048;   // entries ranked in LDS

__device__ __forceinline__ void sub_origin(const TopRArgs &t, int64_t s, int64_t &m0, int64_t &n0) {
  const int64_t N = int64_t(1) << t.nbits;
  const int64_t nt = N > BN ? N / BN : 1;
  const int64_t tile = s >> 2;
  const int w = (int)(s & 3);
  m0 = (tile / nt) * BM + (w & 1) * 32;
  n0 = (tile % nt) * BN + (w >> 1) * 32;
}

constexpr int kGroups = 256;     // groups of sub-tiles ranked for the threshold
constexpr int kPerThread = 16;   // sub-tile statistics a thread keeps in registers

// Total sum; threshold tau; ordered list of the sub-tiles whose maximum reaches
// tau.  The sub-tiles are split into G contiguous groups (4 threads each); tau
// is the R-th largest group maximum.  R groups hold a value >= tau each, so tau
// is no larger than the R-th largest bin, and every one of the R largest bins
// lies in a sub-tile whose maximum reaches tau.
__global__ __launch_bounds__(kSelThreads) void topr_select(TopRArgs t) {
  __shared__ double ps[kSelThreads], pc[kSelThreads];
  __shared__ double gmax[kGroups];
  __shared__ int scan[kSelThreads];
  __shared__ double s_tau;
  const int tid = threadIdx.x;
  const int nsub = t.nsub;
  const int R = t.top_r;
  const int per = (nsub + kSelThreads - 1) / kSelThreads;
  const int b0 = tid * per < nsub ? tid * per : nsub;
  const int b1 = (b0 + per < nsub) ? b0 + per : nsub;
  // statistics of this thread's sub-tiles: the first kPerThread in registers
  double mx[kPerThread];
  double s = 0.0, c = 0.0, tmax = -INFINITY;
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) mx[q] = (b0 + q < b1) ? t.blk_max[b0 + q] : -INFINITY;
#pragma unroll
  for (int q = 0; q < kPerThread; ++q)
    if (b0 + q < b1) neumaier(s, c, t.blk_sum[b0 + q]);
  for (int b = b0 + kPerThread; b < b1; ++b) {
    neumaier(s, c, t.blk_sum[b]);
    const double v = t.blk_max[b];
    tmax = v > tmax ? v : tmax;
  }
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) tmax = mx[q] > tmax ? mx[q] : tmax;
  ps[tid] = s;
  pc[tid] = c;
  // group maximum over 4 consecutive threads
  double gm = tmax;
  gm = fmax(gm, __shfl_xor(gm, 1));
  gm = fmax(gm, __shfl_xor(gm, 2));
  if ((tid & 3) == 0) gmax[tid >> 2] = gm;
  if (tid == 0) s_tau = -INFINITY;
  __syncthreads();
  for (int h = kSelThreads / 2; h >= 1; h >>= 1) {
    if (tid < h) {
      const double a = ps[tid], bb = ps[tid + h];
      const double sum = a + bb;
      const double err = fabs(a) >= fabs(bb) ? (a - sum) + bb : (bb - sum) + a;
      ps[tid] = sum;
      pc[tid] += pc[tid + h] + err;
    }
    __syncthreads();
  }
  // groups that hold at least one sub-tile
  const int groups = (nsub + 4 * per - 1) / (4 * per);
  if (groups >= R && tid < groups) {
    const double v = gmax[tid];
    int rank = 0;
    for (int q = 0; q < groups; ++q) {
      const double o = gmax[q];
      rank += (o > v || (o == v && q < tid)) ? 1 : 0;
    }
    if (rank == R - 1) s_tau = v;
  }
  __syncthreads();
  const double tau = s_tau;  // -inf with fewer groups than R
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) cnt += (b0 + q < b1 && mx[q] >= tau) ? 1 : 0;
  for (int b = b0 + kPerThread; b < b1; ++b) cnt += t.blk_max[b] >= tau ? 1 : 0;
  const int incl = block_scan_incl(cnt, scan);
  int pos = incl - cnt;
#pragma unroll
  for (int q = 0; q < kPerThread; ++q)
    if (b0 + q < b1 && mx[q] >= tau) t.cand[pos++] = b0 + q;
  for (int b = b0 + kPerThread; b < b1; ++b)
    if (t.blk_max[b] >= tau) t.cand[pos++] = b;
  if (tid == kSelThreads - 1) *t.cand_count = incl;
  if (tid == 0) {
    t.tau_sum[0] = tau;
    t.tau_sum[1] = ps[0] + pc[0];
  }
}

// Bins >= tau of each listed sub-tile (its R best when it holds more) into
// the sub-tile's slot of R entries.
__global__ __launch_bounds__(kThreads) void topr_gather(TopRArgs t) {
  __shared__ double red_v[4];
  __shared__ uint64_t red_i[4];
  __shared__ int s_cnt[4];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const double tau = t.tau_sum[0];
  const int R = t.top_r;
  const int ncand = *t.cand_count;
  const int64_t M = int64_t(1) << t.mbits;
  const int64_t N = int64_t(1) << t.nbits;
  for (int c = blockIdx.x; c < ncand; c += gridDim.x) {
    int64_t m0, n0;
    sub_origin(t, t.cand[c], m0, n0);
    double v[4];
    uint64_t ix[4];
    int cnt = 0;
    for (int q = 0; q < 4; ++q) {
      const int e = tid + kThreads * q;  // 1024 bins of the 32 x 32 sub-tile
      const int64_t m = m0 + (e & 31), n = n0 + (e >> 5);
      v[q] = -INFINITY;
      ix[q] = ~uint64_t(0);
      if (m < M && n < N) {
        const int64_t o = map_y(t.m, m) + map_y(t.n, n);
        const double x = t.out_f32 ? (double)static_cast<const float *>(t.C)[o]
                                   : static_cast<const double *>(t.C)[o];
        if (x == x && x >= tau) {
          v[q] = x;
          ix[q] = (uint64_t)o;
          ++cnt;
        }
      }
    }
    int wc = cnt;
    for (int off = 32; off >= 1; off >>= 1) wc += __shfl_xor(wc, off);
    __syncthreads();
    if (lane == 0) s_cnt[wave] = wc;
    __syncthreads();
    const int total = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
    double *sv = t.slot_val + int64_t(c) * R;
    uint64_t *si = t.slot_idx + int64_t(c) * R;
    if (total <= R) {
      int incl = cnt;
      for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
      }
      int pos = incl - cnt;
      for (int q = 0; q < wave; ++q) pos += s_cnt[q];
      for (int q = 0; q < 4; ++q)
        if (ix[q] != ~uint64_t(0)) {
          sv[pos] = v[q];
          si[pos] = ix[q];
          ++pos;
        }
      if (tid == 0) t.slot_n[c] = total;
    } else {
      double pv = INFINITY;
      uint64_t pi = 0;
      for (int r = 0; r < R; ++r) {
        double bv = -INFINITY;
        uint64_t bi = ~uint64_t(0);
        for (int q = 0; q < 4; ++q) {
          if (ix[q] == ~uint64_t(0)) continue;
          const bool below = r == 0 || better(pv, pi, v[q], ix[q]);
          if (below && better(v[q], ix[q], bv, bi)) {
            bv = v[q];
            bi = ix[q];
          }
        }
        block_argmax(bv, bi, red_v, red_i);
        if (tid == 0) {
          sv[r] = bv;
          si[r] = bi;
        }
        pv = bv;
        pi = bi;
      }
      if (tid == 0) t.slot_n[c] = R;
    }
  }
}

// Rank the gathered entries (an entry's rank is the number of better
// entries); ranks below R give the output positions.
__global__ __launch_bounds__(kSelThreads) void topr_rank(TopRArgs t) {
  __shared__ double sv[kRankCap];
  __shared__ uint64_t si[kRankCap];
  __shared__ int scan[kSelThreads];
  __shared__ double red_v[kSelWaves];
  __shared__ uint64_t red_i[kSelWaves];
  const int tid = threadIdx.x;
  const int R = t.top_r;
  const int ncand = *t.cand_count;
  for (int r = tid; r < R; r += kSelThreads) {
    t.top_out[2 * r] = -INFINITY;
    reinterpret_cast<uint64_t *>(t.top_out)[2 * r + 1] = ~uint64_t(0);
  }
  const int per = (ncand + kSelThreads - 1) / kSelThreads;
  const int c0 = tid * per < ncand ? tid * per : ncand;
  const int c1 = (c0 + per < ncand) ? c0 + per : ncand;
  int cnt = 0;
  for (int c = c0; c < c1; ++c) cnt += t.slot_n[c];
  const int incl = block_scan_incl(cnt, scan);
  const int n = scan[kSelThreads - 1];
  __syncthreads();
  if (n <= kRankCap) {
    int pos = incl - cnt;
    for (int c = c0; c < c1; ++c)
      for (int j = 0; j < t.slot_n[c]; ++j) {
        sv[pos] = t.slot_val[int64_t(c) * R + j];
        si[pos] = t.slot_idx[int64_t(c) * R + j];
        ++pos;
      }
    __syncthreads();
    for (int e = tid; e < n; e += kSelThreads) {
      const double v = sv[e];
      const uint64_t i = si[e];
      int rank = 0;
      for (int q = 0; q < n; ++q) rank += better(sv[q], si[q], v, i) ? 1 : 0;
      if (rank < R) {
        t.top_out[2 * rank] = v;
        reinterpret_cast<uint64_t *>(t.top_out)[2 * rank + 1] = i;
      }
    }
  } else {
    // many ties at tau: R rounds of block argmax over the slots in memory
    double pv = INFINITY;
    uint64_t pi = 0;
    for (int r = 0; r < R; ++r) {
      double bv = -INFINITY;
      uint64_t bi = ~uint64_t(0);
      for (int c = 0; c < ncand; ++c)
        for (int j = tid; j < t.slot_n[c]; j += kSelThreads) {
          const double v = t.slot_val[int64_t(c) * R + j];
          const uint64_t i = t.slot_idx[int64_t(c) * R + j];
          const bool below = r == 0 || better(pv, pi, v, i);
          if (below && better(v, i, bv, bi)) {
            bv = v;
            bi = i;
          }
        }
      block_argmax(bv, bi, red_v, red_i);
      if (tid == 0) {
        t.top_out[2 * r] = bv;
        reinterpret_cast<uint64_t *>(t.top_out)[2 * r + 1] = bi;
      }
      pv = bv;
      pi = bi;
    }
  }
  if (tid == 0) *t.sum_out = t.tau_sum[1];
}

__global__ void zero_bytes(unsigned int *p, size_t nwords) {
  for (size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x; q < nwords;
       q += size_t(gridDim.x) * blockDim.x)
    p[q] = 0u;
}

}  // namespace

int64_t gemm_tiles(const GemmArgs &g) {
  const int64_t mt = g.mbits > 6 ? (int64_t(1) << (g.mbits - 6)) : 1;
  const int64_t nt = g.nbits > 6 ? (int64_t(1) << (g.nbits - 6)) : 1;
  return mt * nt;
}

int64_t host_map(const IndexMap &m, uint32_t idx, bool y) {
  int64_t off = 0;
  for (int r = 0; r < m.nruns; ++r) {
    off += int64_t(idx & ((1u << m.bits[r]) - 1u)) << (y ? m.ly[r] : m.lx[r]);
    idx >>= m.bits[r];
  }
  return off;
}

// Work-groups of one kernel resident on the device at once.
template <int PREC, bool FOLD>
int resident_groups() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (!cached[dev]) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gemm<PREC, FOLD>, kThreads, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 2;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    cached[dev] = per_cu * cus;
  }
  return cached[dev];
}

template <int PREC, bool FOLD>
void launch_gemm_t(const GemmArgs &g, hipStream_t s) {
  const int64_t tiles = gemm_tiles(g);
  const int64_t cap = resident_groups<PREC, FOLD>();
  const dim3 grid((unsigned)(tiles < cap ? tiles : cap));
  hipLaunchKernelGGL((gemm<PREC, FOLD>), grid, dim3(kThreads), 0, s, g);
}

void launch_gemm(const GemmArgs &g_in, int prec, hipStream_t s) {
  GemmArgs g = g_in;
  for (int j = 0; j < 16; ++j) {
    g.koff_a[j] = host_map(g.k, j, false);
    g.koff_b[j] = host_map(g.k, j, true);
  }
  // accumulator element -> n within the wave's 32 x 32 block
  for (int r = 0; r < 16; ++r) {
    const uint32_t nl = prec == SQC_F64 ? 16 * (r >> 2) + 4 * (r & 3) : 8 * (r >> 2) + (r & 3);
    g.coff_n[r] = host_map(g.n, nl, true);
  }
  g.coff_m16 = host_map(g.m, 16, true);
  // fold FP32 chunks into FP64 only when the final K spans several chunks;
  // a chunk is one K stage
  const bool fold = g.final_step && g.kbits > 6;
  if (prec == SQC_F64) launch_gemm_t<SQC_F64, false>(g, s);
  else if (prec == SQC_F32) fold ? launch_gemm_t<SQC_F32, true>(g, s) : launch_gemm_t<SQC_F32, false>(g, s);
  else fold ? launch_gemm_t<SQC_BF16X3, true>(g, s) : launch_gemm_t<SQC_BF16X3, false>(g, s);
}

void launch_topr(const TopRArgs &t, hipStream_t s) {
  hipLaunchKernelGGL(topr_select, dim3(1), dim3(kSelThreads), 0, s, t);
  const int g = t.nsub < 128 ? t.nsub : 128;
  hipLaunchKernelGGL(topr_gather, dim3((unsigned)g), dim3(kThreads), 0, s, t);
  hipLaunchKernelGGL(topr_rank, dim3(1), dim3(kSelThreads), 0, s, t);
}

void launch_zero(void *p, size_t bytes, hipStream_t s) {
  size_t words = bytes / 4;
  size_t blocks = (words + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) return;
  hipLaunchKernelGGL(zero_bytes, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<unsigned int *>(p), words);
}

}  // namespace sqc
