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
  int id;          // its place in tile order
};

// Contiguous chunks of tiles per work-group; work-groups are dispatched
// round-robin over 8 XCDs, so chunk order follows (XCD, work-group within the
// XCD) and the chunks of one XCD are adjacent (shared A panels stay in its L2).
__device__ __forceinline__ Sched schedule(int ntiles) {
  const int G = gridDim.x, b = blockIdx.x;
  const int lb = (G & 7) == 0 ? (b & 7) * (G >> 3) + (b >> 3) : b;
  Sched s;
  s.id = lb;
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
  // work-group statistics: running compensated sum and maximum of its waves
  __shared__ double wg_part[3][4];
  double wsum = 0.0, wcmp = 0.0, wmax = -INFINITY;
  auto write_wg_stats = [&]() {
    if (!g.stats) return;
    if (lane == 0) {
      wg_part[0][wave] = wsum;
      wg_part[1][wave] = wcmp;
      wg_part[2][wave] = wmax;
    }
    __syncthreads();
    if (tid == 0) {
      double s = 0.0, c = 0.0, mx = -INFINITY;
      for (int w = 0; w < 4; ++w) {
        neumaier(s, c, wg_part[0][w]);
        c += wg_part[1][w];
        mx = fmax(mx, wg_part[2][w]);
      }
      g.wg_stats[3 * sc.id] = s;
      g.wg_stats[3 * sc.id + 1] = c;
      g.wg_stats[3 * sc.id + 2] = mx;
    }
  };
  if (sc.first >= sc.end) {
    write_wg_stats();
    return;
  }

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
        if (lane == 0) g.blk_max[(int64_t)cur_tile * 4 + wave] = lmax;
        neumaier(wsum, wcmp, lsum);
        wmax = fmax(wmax, lmax);
      }
      reset();
    }
    if (!more) break;
    __syncthreads();  // LDS is rewritten by the next stage
  }
  write_wg_stats();
}

// ---------------------------------------------------------------------------
// top-R selection over the final bins.  The final GEMM wrote the maximum of
// every 32 x 32 sub-tile (sub-tile s = tile * 4 + wave) and, per work-group,
// the compensated sum and maximum of its contiguous range of tiles.  One
// work-group of 1024 threads:
//   1. total sum over the work-group sums; threshold tau = the R-th largest
//      work-group maximum (R groups hold a bin >= tau each, so tau is no
//      larger than the R-th largest bin); list of the sub-tiles of groups
//      whose maximum reaches tau, kept where the sub-tile's own maximum does
//      (every one of the R largest bins lies in one of them);
//   2. the listed sub-tiles' bins are streamed in batches; bins that can
//      still enter the top R are buffered in LDS, and a full buffer is cut
//      back to its R best by ranking (rank = number of better entries under
//      the strict order: larger value, then lower index);
//   3. the final ranking writes the R best.
// Deterministic: the only atomics are integer histogram counts in LDS.  The
// number of passes grows only when many bins tie at the threshold.
// ---------------------------------------------------------------------------

constexpr int kSelThreads = 1024;
constexpr int kSelWaves = kSelThreads / 64;
constexpr int kCandCap = 4096;            // listed sub-tiles held in LDS
constexpr int kBufCap = 2048;             // buffered entries
constexpr int kBatch = 16;                // sub-tiles per streamed batch

// Exclusive prefix of v over the work-group; `total` gets the sum.
__device__ __forceinline__ int block_scan_excl(int v, int *wsum, int &total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int before = 0;
  total = 0;
  for (int q = 0; q < kSelWaves; ++q) {
    const int x = wsum[q];
    before += q < w ? x : 0;
    total += x;
  }
  __syncthreads();  // wsum is reused by the next scan
  return before + incl - v;
}

__device__ __forceinline__ void two_sum_merge(double &s, double &c, double s2, double c2) {
  const double t = s + s2;
  const double err = fabs(s) >= fabs(s2) ? (s - t) + s2 : (s2 - t) + s;
  s = t;
  c += c2 + err;
}

// Order-preserving map of doubles to unsigned keys (NaN lowest).
__device__ __forceinline__ uint64_t order_key(double v) {
  if (v != v) return 0;
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double key_value(uint64_t k) {
  return __longlong_as_double((long long)((k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k));
}

__global__ __launch_bounds__(kSelThreads) void topr(TopRArgs t) {
  __shared__ double ps[kSelWaves], pc[kSelWaves];
  __shared__ int hist[256];
  __shared__ int s_sel[2];
  __shared__ int wsum[kSelWaves];
  __shared__ int cand[kCandCap];
  __shared__ int64_t boff[kBatch];
  __shared__ double bval[kBufCap];
  __shared__ uint64_t bidx[kBufCap];
  __shared__ double lval[SQC_MAX_TOPR];
  __shared__ uint64_t lidx[SQC_MAX_TOPR];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int nsub = t.nsub;
  const int R = t.top_r;
  const int G = t.ngroups;                 // work-groups of the final GEMM
  const int ntiles = nsub >> 2;

  // ---- 1. work-group statistics; group g belongs to thread g % 1024 ----
  constexpr int kGPT = kMaxGemmGroups / kSelThreads;
  double gm[kGPT];
  double s = 0.0, c = 0.0;
  {
    double gs[kGPT], gc[kGPT];
#pragma unroll
    for (int q = 0; q < kGPT; ++q) {
      const int gi = tid + q * kSelThreads;
      const int gg = gi < G ? gi : 0;
      gs[q] = t.wg_stats[3 * gg];
      gc[q] = t.wg_stats[3 * gg + 1];
      gm[q] = t.wg_stats[3 * gg + 2];
    }
#pragma unroll
    for (int q = 0; q < kGPT; ++q)
      if (tid + q * kSelThreads < G) {
        neumaier(s, c, gs[q]);
        c += gc[q];
      }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    const double s2 = __shfl_xor(s, off), c2 = __shfl_xor(c, off);
    two_sum_merge(s, c, s2, c2);
  }
  if (lane == 0) {
    ps[wave] = s;
    pc[wave] = c;
  }

  // threshold: the R-th largest work-group maximum (radix select on keys,
  // 8 bits per pass; histogram counts are order independent)
  double tau = -INFINITY;
  if (G >= R) {
    uint64_t prefix = 0, hi = 0;
    int need = R;
    for (int pass = 0; pass < 8; ++pass) {
      const int sh = 56 - 8 * pass;
      if (tid < 256) hist[tid] = 0;
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kGPT; ++q) {
        const uint64_t k = order_key(gm[q]);
        if (tid + q * kSelThreads < G && (k & hi) == prefix) atomicAdd(&hist[(k >> sh) & 255], 1);
      }
      __syncthreads();
      if (wave == 0) {
        int h[4], tot = 0;
        for (int j = 0; j < 4; ++j) {
          h[j] = hist[255 - 4 * lane - j];  // digits in descending order
          tot += h[j];
        }
        int incl = tot;
        for (int off = 1; off < 64; off <<= 1) {
          const int o = __shfl_up(incl, off);
          if (lane >= off) incl += o;
        }
        int cum = incl - tot;
        for (int j = 0; j < 4; ++j) {
          if (cum < need && need <= cum + h[j]) {
            s_sel[0] = 255 - 4 * lane - j;
            s_sel[1] = need - cum;
          }
          cum += h[j];
        }
      }
      __syncthreads();
      prefix |= (uint64_t)s_sel[0] << sh;
      hi |= (uint64_t)255 << sh;
      need = s_sel[1];
    }
    tau = key_value(prefix);
    if (tau != tau) tau = -INFINITY;  // fewer than R groups hold a number
  }

  // ---- sub-tiles of the groups whose maximum reaches tau ----
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < kGPT; ++q) {
    const int gi = tid + q * kSelThreads;
    if (gi < G && gm[q] >= tau)
      cnt += 4 * (int)(((int64_t)(gi + 1) * ntiles / G) - ((int64_t)gi * ntiles / G));
  }
  int nlist;
  int pos = block_scan_excl(cnt, wsum, nlist);
  bool listed = nlist <= kCandCap;  // else every sub-tile is streamed
  int ncand = 0;
  if (listed) {
#pragma unroll
    for (int q = 0; q < kGPT; ++q) {
      const int gi = tid + q * kSelThreads;
      if (gi < G && gm[q] >= tau) {
        const int f = (int)((int64_t)gi * ntiles / G), e = (int)((int64_t)(gi + 1) * ntiles / G);
        for (int sb = 4 * f; sb < 4 * e; ++sb) cand[pos++] = sb;
      }
    }
    __syncthreads();
    // keep the listed sub-tiles whose own maximum reaches tau
    constexpr int kLPT = kCandCap / kSelThreads;
    int sbv[kLPT];
    int keep = 0;
#pragma unroll
    for (int q = 0; q < kLPT; ++q) {
      const int e = tid + q * kSelThreads;
      sbv[q] = e < nlist ? cand[e] : -1;
    }
    double mxv[kLPT];
#pragma unroll
    for (int q = 0; q < kLPT; ++q) mxv[q] = t.blk_max[sbv[q] >= 0 ? sbv[q] : 0];
#pragma unroll
    for (int q = 0; q < kLPT; ++q) keep += (sbv[q] >= 0 && mxv[q] >= tau) ? 1 : 0;
    int at = block_scan_excl(keep, wsum, ncand);  // also orders the reads above before the writes
#pragma unroll
    for (int q = 0; q < kLPT; ++q)
      if (sbv[q] >= 0 && mxv[q] >= tau) cand[at++] = sbv[q];
  }
  const int nstream = listed ? ncand : nsub;
  __syncthreads();

  // ---- 2. stream the bins; thread tid reads bin (tid % 32, tid / 32) of each sub-tile ----
  const uint32_t M = 1u << t.mbits, N = 1u << t.nbits;
  const int lnt = t.nbits > 6 ? t.nbits - 6 : 0;
  const uint32_t ml = tid & 31, nl = tid >> 5;
  const int64_t o_lane = map_y(t.m, ml) + map_y(t.n, nl);
  int nbuf = 0;
  bool have_bar = false;  // R entries kept: a new entry must beat the R-th
  double bar_v = 0.0;
  uint64_t bar_i = 0;

  // cut the buffer back to its R best (in order, at its front)
  auto cut = [&]() {
    for (int e = tid; e < nbuf; e += kSelThreads) {
      const double v = bval[e];
      const uint64_t i = bidx[e];
      int rank = 0;
#pragma unroll 8
      for (int q = 0; q < nbuf; ++q) rank += better(bval[q], bidx[q], v, i) ? 1 : 0;
      if (rank < R) {
        lval[rank] = v;
        lidx[rank] = i;
      }
    }
    __syncthreads();
    const int kept = nbuf < R ? nbuf : R;
    if (tid < kept) {
      bval[tid] = lval[tid];
      bidx[tid] = lidx[tid];
    }
    __syncthreads();
    nbuf = kept;
    if (kept == R) {
      have_bar = true;
      bar_v = lval[R - 1];
      bar_i = lidx[R - 1];
    }
  };

  // a sub-tile's bin (ml, nl) exists iff the sub-tile origin and (ml, nl)
  // both lie inside the M x N result (origins are multiples of 32)
  const bool lane_ok = ml < M && nl < N;
  for (int cb = 0; cb < nstream; cb += kBatch) {
    // origin offsets of the batch's sub-tiles, one thread each (-1: skipped)
    if (tid < kBatch) {
      const int ci = cb + tid;
      int64_t o = -1;
      if (ci < nstream) {
        const int sb = listed ? cand[ci] : ci;
        const int tile = sb >> 2, w = sb & 3;
        const uint32_t m0 = ((uint32_t)(tile >> lnt) << 6) + (w & 1) * 32;
        const uint32_t n0 = ((uint32_t)(tile & ((1 << lnt) - 1)) << 6) + (w >> 1) * 32;
        if (m0 < M && n0 < N && (listed || t.blk_max[sb] >= tau)) o = map_y(t.m, m0) + map_y(t.n, n0);
      }
      boff[tid] = o;
    }
    __syncthreads();
    double v[kBatch];
    uint64_t ix[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int64_t o = boff[u];
      ix[u] = (o >= 0 && lane_ok) ? (uint64_t)(o + o_lane) : ~uint64_t(0);
    }
    // loads with a clamped offset, all in flight together
    if (t.out_f32) {
      const float *Cf = static_cast<const float *>(t.C);
#pragma unroll
      for (int u = 0; u < kBatch; ++u) v[u] = (double)Cf[ix[u] == ~uint64_t(0) ? 0 : ix[u]];
    } else {
      const double *Cd = static_cast<const double *>(t.C);
#pragma unroll
      for (int u = 0; u < kBatch; ++u) v[u] = Cd[ix[u] == ~uint64_t(0) ? 0 : ix[u]];
    }
    // entries that can still enter the top R
    auto qualifies = [&](int u) {
      return ix[u] != ~uint64_t(0) && v[u] == v[u] && v[u] >= tau &&
             (!have_bar || better(v[u], ix[u], bar_v, bar_i));
    };
    int k = 0;
#pragma unroll
    for (int u = 0; u < kBatch; ++u) k += qualifies(u) ? 1 : 0;
    int total;
    int at = block_scan_excl(k, wsum, total);
    if (nbuf + total > kBufCap && nbuf > R) {
      cut();
      k = 0;
#pragma unroll
      for (int u = 0; u < kBatch; ++u) k += qualifies(u) ? 1 : 0;
      at = block_scan_excl(k, wsum, total);
    }
    if (nbuf + total <= kBufCap) {
      at += nbuf;
#pragma unroll
      for (int u = 0; u < kBatch; ++u)
        if (qualifies(u)) {
          bval[at] = v[u];
          bidx[at] = ix[u];
          ++at;
        }
      nbuf += total;
      __syncthreads();
    } else {
      // many ties: one sub-tile at a time (at most 1024 entries each); the
      // entry is picked from registers by selects (no indexed register array)
      for (int u = 0; u < kBatch; ++u) {
        double vu = v[0];
        uint64_t iu = ix[0];
#pragma unroll
        for (int q = 1; q < kBatch; ++q) {
          vu = u == q ? v[q] : vu;
          iu = u == q ? ix[q] : iu;
        }
        auto qual1 = [&]() {
          return iu != ~uint64_t(0) && vu == vu && vu >= tau && (!have_bar || better(vu, iu, bar_v, bar_i));
        };
        int one = qual1() ? 1 : 0;
        int tot1;
        int at1 = block_scan_excl(one, wsum, tot1);
        if (nbuf + tot1 > kBufCap) {
          cut();
          one = qual1() ? 1 : 0;
          at1 = block_scan_excl(one, wsum, tot1);
        }
        if (one) {
          bval[nbuf + at1] = vu;
          bidx[nbuf + at1] = iu;
        }
        nbuf += tot1;
        __syncthreads();
      }
    }
  }

  // ---- 3. final ranking ----
  cut();
  if (tid < R) {
    t.top_out[2 * tid] = tid < nbuf ? bval[tid] : -INFINITY;
    reinterpret_cast<uint64_t *>(t.top_out)[2 * tid + 1] = tid < nbuf ? bidx[tid] : ~uint64_t(0);
  }
  if (tid == 0) {
    double S = ps[0], Cc = pc[0];
    for (int q = 1; q < kSelWaves; ++q) two_sum_merge(S, Cc, ps[q], pc[q]);
    *t.sum_out = S + Cc;
  }
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
int launch_gemm_t(const GemmArgs &g, hipStream_t s) {
  const int64_t tiles = gemm_tiles(g);
  int64_t cap = resident_groups<PREC, FOLD>();
  if (cap > kMaxGemmGroups) cap = kMaxGemmGroups;
  const int G = (int)(tiles < cap ? tiles : cap);
  hipLaunchKernelGGL((gemm<PREC, FOLD>), dim3((unsigned)G), dim3(kThreads), 0, s, g);
  return G;
}

int launch_gemm(const GemmArgs &g_in, int prec, hipStream_t s) {
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
  if (prec == SQC_F64) return launch_gemm_t<SQC_F64, false>(g, s);
  if (prec == SQC_F32) return fold ? launch_gemm_t<SQC_F32, true>(g, s) : launch_gemm_t<SQC_F32, false>(g, s);
  return fold ? launch_gemm_t<SQC_BF16X3, true>(g, s) : launch_gemm_t<SQC_BF16X3, false>(g, s);
}

void launch_topr(const TopRArgs &t, hipStream_t s) {
  hipLaunchKernelGGL(topr, dim3(1), dim3(kSelThreads), 0, s, t);
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
