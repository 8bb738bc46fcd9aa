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

#include <rocprim/warp/warp_reduce.hpp>
#include <rocprim/warp/warp_scan.hpp>

#include <hip/hip_ext.h>

#include <mutex>
#include <type_traits>
#include <unordered_map>

namespace sqc {

namespace {

constexpr int kThreads = 256;
constexpr int BM = 64;
constexpr int BN = 64;
constexpr int BK = 64;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

// Offsets by index map: strides are powers of two, so each run is a shift.
// Indices of one GEMM dimension fit 31 bits (checked on the host).  The first
// four runs are evaluated unconditionally (runs past nruns are all-zero, so
// they add nothing), which lets their parameters be fetched together instead
// of one dependent scalar read per run; longer maps continue in a loop.
template <bool Y>
__device__ __forceinline__ int64_t map_off(const IndexMap &m, uint32_t idx) {
  int64_t off = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    off += int64_t(idx & ((1u << m.bits[r]) - 1u)) << (Y ? m.ly[r] : m.lx[r]);
    idx >>= m.bits[r];
  }
  for (int r = 4; r < m.nruns; ++r) {
    off += int64_t(idx & ((1u << m.bits[r]) - 1u)) << (Y ? m.ly[r] : m.lx[r]);
    idx >>= m.bits[r];
  }
  return off;
}
__device__ __forceinline__ int64_t map_x(const IndexMap &m, uint32_t idx) { return map_off<false>(m, idx); }
__device__ __forceinline__ int64_t map_y(const IndexMap &m, uint32_t idx) { return map_off<true>(m, idx); }

__device__ __forceinline__ void neumaier(double &s, double &c, double x) {
  double t = s + x;
  if (fabs(s) >= fabs(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

// Merge a compensated pair (s2, c2) into (s, c).
__device__ __forceinline__ void two_sum_merge(double &s, double &c, double s2, double c2) {
  const double t = s + s2;
  const double err = fabs(s) >= fabs(s2) ? (s - t) + s2 : (s2 - t) + s;
  s = t;
  c += c2 + err;
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

// Contiguous chunks of tiles per work-group (the first ntiles % G chunks one
// tile longer); work-groups are dispatched round-robin over 8 XCDs, so chunk
// order follows (XCD, work-group within the XCD) and the chunks of one XCD are
// adjacent (shared A panels stay in its L2).  32-bit quotient and remainder:
// a 64-bit division costs a long scalar sequence per work-group.
__device__ __forceinline__ Sched schedule(int ntiles, int b, int G) {
  const int lb = (G & 7) == 0 ? (b & 7) * (G >> 3) + (b >> 3) : b;
  const int q = ntiles / G, r = ntiles - q * G;
  Sched s;
  s.id = lb;
  s.first = lb * q + (lb < r ? lb : r);
  s.end = s.first + q + (lb < r ? 1 : 0);
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
// OUTF: FP32 result (else FP64).
// REG (1 or 2): M, N, K >= 64 and the lowest run of k spans >= 4 bits, so no tile,
// row or element needs a bound check and k rows are shifts.
// One work-group `blk` of G working on the GEMM `g`.
// REG = 2 adds: every index map is a single run of bits, so each offset is
// one shift (no loop over runs in the per-tile address arithmetic).
// REG = 3: general index maps, and the final step of one slice of a sliced
// contraction adds its result into FP64 running sums (GemmArgs::acc_mode).
// REG = 4: general index maps with K <= 16, staged as one K stage of 16
// labels instead of 64 (a narrower tile in K: a quarter of the staging
// loads, LDS and barrier time of a short contraction).
// s_waitcnt operand of vmcnt(0) alone (expcnt and lgkmcnt at their maxima)
constexpr int kWaitVmem0 = 0x0F70;

template <int PREC, bool FOLD, bool OUTF, int REG>
__device__ __forceinline__ void gemm_body(const GemmArgs &g, int blk, int G) {
  constexpr bool ACC = REG == 3;     // slice-accumulating epilogue
  constexpr bool NARROW = REG == 4;  // K <= 16: one K stage of 16 labels
  constexpr int RG = (ACC || NARROW) ? 0 : REG;  // index-map class
  constexpr bool SIMPLE = RG == 2;
  auto mx = [&](const IndexMap &mp, uint32_t v) -> int64_t {
    if constexpr (SIMPLE) return (int64_t)v << mp.lx[0];
    else return map_x(mp, v);
  };
  auto my = [&](const IndexMap &mp, uint32_t v) -> int64_t {
    if constexpr (SIMPLE) return (int64_t)v << mp.ly[0];
    else return map_y(mp, v);
  };
  typedef typename Tr<PREC>::T T;
  typedef typename Tr<PREC>::Acc Acc;
  constexpr int NACC = Tr<PREC>::NACC;
  constexpr bool SPLIT = PREC == SQC_BF16X3;
  constexpr int KB = NARROW ? 16 : BK;  // staged K depth
  constexpr int PAD = 8;    // bf16 row padding (keeps rows 16-byte aligned)
  constexpr int LDK = KB + PAD;
  constexpr int NJ = KB / 4;  // staged elements per thread per operand (rows NJ wave + j)
  // F32/F64: As[k][m], Bs[k][n]; BF16X3: Ah, Al [m][k], Bh, Bl [n][k]
  constexpr int kHalf = SPLIT ? (2 * BM * LDK * 2) : (KB * BM * (int)sizeof(T));
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

  // tile -> (m panel, n panel)
  const int nmaj = g.nmajor;
  auto tile_m = [&](int t) -> uint32_t { return nmaj ? (uint32_t)(t & ((1 << lmt) - 1)) : (uint32_t)(t >> lnt); };
  auto tile_n = [&](int t) -> uint32_t { return nmaj ? (uint32_t)(t >> lmt) : (uint32_t)(t & ((1 << lnt) - 1)); };
  const Sched sc = schedule(1 << (lmt + lnt), blk, G);
  // work-group statistics: each lane keeps a compensated running sum of its
  // elements over the work-group's tiles (merged across lanes and waves once,
  // at the end) and the maximum of the sub-tiles it took part in
  __shared__ double wg_part[3][4];
  double wsum = 0.0, wcmp = 0.0, wmax = -INFINITY;
  auto write_wg_stats = [&]() {
    if (!g.stats) return;
    double s = wsum, c = wcmp;
    for (int off = 32; off >= 1; off >>= 1) {
      const double s2 = __shfl_xor(s, off), c2 = __shfl_xor(c, off);
      two_sum_merge(s, c, s2, c2);
    }
    if (lane == 0) {
      wg_part[0][wave] = s;
      wg_part[1][wave] = c;
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
  const int64_t a_lane = mx(g.m, lane);
  const int64_t b_lane = mx(g.n, lane);
  const int64_t a_kw = mx(g.k, NJ * wave);
  const int64_t b_kw = my(g.k, NJ * wave);
  T av[NJ], bv[NJ];
  // k offsets of rows j = 0..NJ-1: shifts when the lowest run of k spans
  // them (the usual case), else a table staged in LDS
  const bool kfast = RG || (g.k.nruns >= 1 && (1 << g.k.bits[0]) >= NJ);
  const int sa = g.k.lx[0], sb = g.k.ly[0];
  __shared__ int64_t ktab[2][NJ];
  if (!kfast) {
    if (tid < NJ) {
      ktab[0][tid] = g.koff_a[tid];
      ktab[1][tid] = g.koff_b[tid];
    }
    __syncthreads();
  }
  // a full K stage needs no per-row bound; rows past K (K < KB) read offset 0
  const bool kfull = RG || (1 << g.kbits) >= KB;
  auto load_rows = [&](const T *p, T *v, int which, int s_shift, uint32_t k0) {
    if (kfull && kfast) {
      // (the row step passes an empty asm statement, so its 16 multiples are
      // formed here rather than hoisted into scalar registers for the whole
      // kernel, which spills them)
      int64_t step = (int64_t)1 << s_shift;
      asm volatile("" : "+s"(step));
#pragma unroll
      for (int j = 0; j < NJ; ++j) v[j] = p[j * step];
    } else {
      const int kr = (int)(k0 + NJ * wave);
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const bool in = (uint32_t)(kr + j) < K;
        const int64_t o = kfast ? ((int64_t)j << s_shift) : ktab[which][j];
        v[j] = p[in ? o : 0];
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        if ((uint32_t)(kr + j) >= K) v[j] = T(0);
    }
  };
  auto load_a = [&](int tile, int ks) {
    const uint32_t m0 = tile_m(tile) << 6;
    const uint32_t k0 = (uint32_t)ks << 6;
    const bool ok = RG || m0 + lane < M;  // columns past M read the column origin
    const T *p = static_cast<const T *>(g.A) + (mx(g.m, m0) + mx(g.k, k0) + a_kw) + (ok ? a_lane : 0);
    load_rows(p, av, 0, sa, k0);
    if (!ok)
#pragma unroll
      for (int j = 0; j < NJ; ++j) av[j] = T(0);
  };
  auto load_b = [&](int tile, int ks) {
    const uint32_t n0 = tile_n(tile) << 6;
    const uint32_t k0 = (uint32_t)ks << 6;
    const bool ok = RG || n0 + lane < N;
    const T *p = static_cast<const T *>(g.B) + (mx(g.n, n0) + my(g.k, k0) + b_kw) + (ok ? b_lane : 0);
    load_rows(p, bv, 1, sb, k0);
    if (!ok)
#pragma unroll
      for (int j = 0; j < NJ; ++j) bv[j] = T(0);
  };
  auto stage = [&](const T *v, unsigned char *dst, int ld) {
    if constexpr (!SPLIT) {
      T *S = reinterpret_cast<T *>(dst);
#pragma unroll
      for (int j = 0; j < NJ; ++j) S[(NJ * wave + j) * ld + lane] = v[j];
    } else if constexpr (NARROW) {
      // 4 consecutive k of one column: 8 bytes of hi and of lo
      v4bf h, l;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const __bf16 a = (__bf16)v[j];
        h[j] = a;
        l[j] = (__bf16)(v[j] - (float)a);
      }
      __bf16 *H = reinterpret_cast<__bf16 *>(dst) + lane * LDK + 4 * wave;
      *reinterpret_cast<v4bf *>(H) = h;
      *reinterpret_cast<v4bf *>(H + BM * LDK) = l;
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
  // FP32 results of a tile go out one tile late, after the next tile is
  // staged: their writes then drain while that tile is multiplied instead of
  // holding up its staging (a wait for the staged loads counts every
  // vector-memory operation still in flight, stores included)
  constexpr bool DEFER = OUTF && !ACC && !FOLD && PREC != SQC_F64;
  float pend[DEFER ? 16 : 1];
  float *pendC = nullptr;
  uint32_t pmw = 0, pnw = 0;
  double pmax = 0.0;  // the sub-tile maximum, stored with the results
  int ptile = 0;
  bool pend_c = false, pend_max = false;
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
    c_lane_m = my(g.m, lane & 15);
    c_lane_n = my(g.n, lane >> 4);
  } else {
    c_lane_m = my(g.m, lane & 31);
    c_lane_n = my(g.n, 4 * (lane >> 5));
  }
  reset();
  // the deferred stores of the last tile (the same elements and order as
  // the epilogue's stores)
  auto flush_pending = [&]() {
    if constexpr (DEFER) {
      const bool whole = RG || (g.mbits >= 5 && g.nbits >= 5);
      int64_t nstep = (int64_t)1 << g.n.ly[0];
      asm volatile("" : "+s"(nstep));
      if (pend_c) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const uint32_t nl = 8 * (r >> 2) + (r & 3);
          const uint32_t mloc = lane & 31, nloc = nl + 4 * (lane >> 5);
          if (!whole && (pmw + mloc >= M || pnw + nloc >= N)) continue;
          __builtin_nontemporal_store(pend[r], pendC + (SIMPLE ? (int64_t)nl * nstep : g.coff_n[r]));
        }
      }
      if (pend_max && lane == 0) g.blk_max[(int64_t)ptile * 4 + wave] = pmax;
      pend_c = pend_max = false;
    }
  };

  // with a single K stage an operand panel stays staged while consecutive
  // tiles share it
  int tile = sc.first, ks = 0;
  bool need_a = true, need_b = true;
  load_a(tile, ks);
  load_b(tile, ks);
  while (true) {
    if (need_a) stage(av, lds, BM);
    if (need_b) stage(bv, lds + kHalf, BN);
    if constexpr (DEFER) {
      // every load issued so far has been staged: say so to the compiler,
      // whose own waits assume a skipped staging leaves loads in flight and
      // would hold the next loads behind the deferred stores
      __builtin_amdgcn_s_waitcnt(kWaitVmem0);
    }
    __syncthreads();
    if constexpr (DEFER) {
      if (pend_c || pend_max) flush_pending();
    }
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
    need_a = !(nks == 1 && tile_m(tile) == tile_m(cur_tile));
    need_b = !(nks == 1 && tile_n(tile) == tile_n(cur_tile));
    if (more) {
      if (need_a) load_a(tile, ks);
      if (need_b) load_b(tile, ks);
    }
    // ---- MFMA on the staged stage ----
    const uint32_t k0 = (uint32_t)cur_ks << 6;
    const int kend = (RG || (K - k0) >= (uint32_t)KB) ? KB : (int)(K - k0);
    if (kend == KB) {
#pragma unroll
      for (int kk = 0; kk < KB / KSTEP; ++kk) mfma_step(kk);
    } else {
      for (int kk = 0; kk * KSTEP < kend; ++kk) mfma_step(kk);
    }
    fold();  // one FP32 chunk per K stage
    // ---- epilogue after the tile's last stage ----
    if (cur_ks == nks - 1) {
      const uint32_t mw = (tile_m(cur_tile) << 6) + wm * 32;  // wave origin
      const uint32_t nw = (tile_n(cur_tile) << 6) + wn * 32;
      typedef typename std::conditional<OUTF, float, double>::type O;
      double lsum = 0.0;
      O lmax = -INFINITY;
      if (RG || (mw < M && nw < N)) {
        const int64_t cw = my(g.m, mw) + my(g.n, nw);
        O *C = static_cast<O *>(g.C) + cw + c_lane_m + c_lane_n;
        double *AS = nullptr, *AC = nullptr;
        if constexpr (ACC) {
          AS = g.acc_sum + cw + c_lane_m + c_lane_n;
          AC = g.acc_comp + cw + c_lane_m + c_lane_n;
        }
        // with M, N >= 32 every element of a wave inside the result is inside
        const bool whole = RG || (g.mbits >= 5 && g.nbits >= 5);
        O omax = -INFINITY;
        // FP32 results go out as non-temporal stores (the FP32 and
        // split-BF16x3 steps measured faster so), FP64 results as ordinary
        // stores (non-temporal measured slower there)
        int pr = 0;  // the element's index in pend
        auto put = [&](uint32_t mloc, uint32_t nloc, int64_t o, double v) {
          if (!whole && (mw + mloc >= M || nw + nloc >= N)) return;
          if constexpr (ACC) {
            if (g.acc_mode == 1) {
              AS[o] = v;
              AC[o] = 0.0;
              return;
            }
            double sm = AS[o], cp = AC[o];
            neumaier(sm, cp, v);
            if (g.acc_mode == 2) {
              AS[o] = sm;
              AC[o] = cp;
              return;
            }
            v = sm + cp;
          }
          const O st = (O)v;
          if constexpr (DEFER) pend[pr] = st;
          else if constexpr (OUTF) __builtin_nontemporal_store(st, C + o);
          else C[o] = st;
          lsum += v;
          omax = fmax(omax, st);
        };
        if constexpr (PREC == SQC_F64) {
#pragma unroll
          for (int jn = 0; jn < 2; ++jn)
#pragma unroll
            for (int im = 0; im < 2; ++im)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const uint32_t nl = 16 * jn + 4 * r;
                const int64_t om = SIMPLE ? (int64_t)(16 * im) << g.m.ly[0] : (im ? g.coff_m16 : 0);
                const int64_t on = SIMPLE ? (int64_t)nl << g.n.ly[0] : g.coff_n[4 * jn + r];
                put(16 * im + (lane & 15), nl + (lane >> 4), om + on, acc[2 * jn + im][r]);
              }
        } else {
          int64_t nstep = (int64_t)1 << g.n.ly[0];  // (formed per tile, as above)
          asm volatile("" : "+s"(nstep));
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const uint32_t nl = 8 * (r >> 2) + (r & 3);
            double v;
            if constexpr (FOLD) v = S[r] + Cc[r];
            else v = (double)acc[0][r];
            pr = r;
            put(lane & 31, nl + 4 * (lane >> 5), SIMPLE ? (int64_t)nl * nstep : g.coff_n[r], v);
          }
          if constexpr (DEFER) {
            pendC = reinterpret_cast<float *>(C);
            pmw = mw;
            pnw = nw;
            pend_c = true;
          }
        }
        lmax = omax;
      }
      if (g.stats) {
        // sub-tile maximum in the stored type, reduced by rocPRIM's wave
        // reduction (DPP lane moves; fmax keeps NaN out); valid in lane 0,
        // the only lane that uses it
        {
          using WaveMax = rocprim::warp_reduce<O, 64>;
          __shared__ typename WaveMax::storage_type max_st[4];
          O m;
          WaveMax().reduce(lmax, m, max_st[wave], [](O x, O y) { return fmax(x, y); });
          lmax = m;
        }
        if constexpr (DEFER) {
          pmax = (double)lmax;
          ptile = cur_tile;
          pend_max = true;
        } else if (lane == 0) {
          g.blk_max[(int64_t)cur_tile * 4 + wave] = (double)lmax;
        }
        neumaier(wsum, wcmp, lsum);
        wmax = fmax(wmax, (double)lmax);
      }
      reset();
    }
    if (!more) break;
    __syncthreads();  // LDS is rewritten by the next stage
  }
  if constexpr (DEFER) {
    if (pend_c || pend_max) flush_pending();
  }
  write_wg_stats();
}

// Waves per SIMD the compiler must leave registers for: four (all that the
// work-group's LDS allows) for the split-BF16x3 regular shapes with FP32
// results, whose values held for the late stores would otherwise cost one.
template <int PREC, bool FOLD, bool OUTF, int REG>
constexpr int gemm_waves() {
  return (PREC == SQC_BF16X3 && !FOLD && OUTF && (REG == 1 || REG == 2)) ? 4 : 1;
}

template <int PREC, bool FOLD, bool OUTF, int REG>
__global__ __launch_bounds__(kThreads, (gemm_waves<PREC, FOLD, OUTF, REG>())) void gemm(GemmArgs g) {
  gemm_body<PREC, FOLD, OUTF, REG>(g, blockIdx.x, gridDim.x);
}

// Job j of a table with work-group prefix `start` (start[0] = 0, n + 1
// entries): the largest j with start[j] <= w (a uniform binary search).
__device__ __forceinline__ int find_job(const int *__restrict__ start, int n, int w) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// Several GEMMs of one specialisation in one launch (requests batched by the
// serving engine): job j owns work-groups [start[j], start[j + 1]) and runs
// exactly as the single launch with start[j + 1] - start[j] work-groups.
template <int PREC, bool FOLD, bool OUTF, int REG>
__global__ __launch_bounds__(kThreads, (gemm_waves<PREC, FOLD, OUTF, REG>())) void gemm_grouped(const GemmArgs *__restrict__ jobs,
                                                          const int *__restrict__ start, int n) {
  if ((int)blockIdx.x >= start[n]) return;  // (a grid sized for a larger table)
  const int j = find_job(start, n, blockIdx.x);
  const int s0 = start[j];
  gemm_body<PREC, FOLD, OUTF, REG>(jobs[j], (int)blockIdx.x - s0, start[j + 1] - s0);
}

// ---------------------------------------------------------------------------
// top-R selection over the final bins.  The final GEMM wrote the maximum of
// every 32 x 32 sub-tile (sub-tile s = tile * 4 + wave) and, per work-group,
// the compensated sum and maximum of its contiguous range of tiles.
//   gather (t.gather_groups <= kTopRSlots work-groups, about one per 64
//     sub-tiles): the GEMM's work-groups are joined
//     into at most 256 groups of consecutive work-groups; threshold tau = the
//     R-th largest group maximum (R groups hold a bin >= tau each, so tau is
//     no larger than the R-th largest bin), found by counting, for every
//     group, the groups better than it.
//     Work-group w then visits the sub-tiles of its runs (runs w,
//     w + gather_groups, ...; 64 to 256 sub-tiles each, so that every
//     work-group has one when there are few) whose maximum reaches tau (and
//     the running R-th best), best first; where many do, those whose maximum
//     R others in the run provably beat are skipped.  It keeps its R best bins
//     in an LDS buffer: a bin enters when it reaches tau and beats the
//     buffer's R-th best so far, which is fixed as soon as R bins are in; a
//     full buffer is cut back to its R best by counting.  Its R best go to
//     slot w.
//   rank (one work-group): the slots are merged the same way.
// The order is strict (larger value, then lower index), so the result is
// unique: deterministic, no atomics.  Ties at the top cost no more than
// distinct values: tied bins beyond the R lowest indices are dropped at once.
// The code is kept compact (loops, not unrolled copies): these are small
// grids whose instruction fetch is not amortised.
// ---------------------------------------------------------------------------

constexpr int kTW = 4;                    // waves of the top-R work-groups
constexpr int kTThreads = 64 * kTW;
constexpr int kNG = kTThreads;            // groups of GEMM work-groups
// Buffered entries per work-group: a full buffer is cut back to the R best
// by counting (each thread ranks one entry against all), which needs at most
// one entry per thread; many small cuts that raise the running R-th best
// early cost far less than sorting a large buffer when the top is flat (many
// tied bins).  (+4: the counting loop reads four entries at a time.)
constexpr int kCutAt = kTThreads;
constexpr int kBufCap = kCutAt + 4;

// Exclusive prefix of v over the work-group; `total` gets the sum.  The wave
// prefix is rocPRIM's (cross-lane DPP moves, no LDS round trips).
__device__ int block_scan_excl(int v, int *wsum, int &total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  using WaveScan = rocprim::warp_scan<int, 64>;
  __shared__ typename WaveScan::storage_type scan_st[kTW];
  int incl;
  WaveScan().inclusive_scan(v, incl, scan_st[w]);
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int before = 0;
  total = 0;
  for (int q = 0; q < kTW; ++q) {
    const int x = wsum[q];
    before += q < w ? x : 0;
    total += x;
  }
  __syncthreads();  // wsum is reused by the next scan
  return before + incl - v;
}


// origin (m0, n0) of sub-tile sb of a GEMM with 2^lmt m tiles and 2^lnt n
// tiles in the given tile order
__device__ __forceinline__ void sub_origin(int sb, int lmt, int lnt, int nmaj, uint32_t &m0, uint32_t &n0) {
  const int tile = sb >> 2, w = sb & 3;
  const uint32_t mt = nmaj ? (uint32_t)(tile & ((1 << lmt) - 1)) : (uint32_t)(tile >> lnt);
  const uint32_t nt = nmaj ? (uint32_t)(tile >> lmt) : (uint32_t)(tile & ((1 << lnt) - 1));
  m0 = (mt << 6) + (w & 1) * 32;
  n0 = (nt << 6) + (w >> 1) * 32;
}

// Offset of bin (ml, nl) of a sub-tile, or ~0 when it lies outside the result.
struct SubTileBins {
  uint32_t M, N;
  int lmt, lnt, nmaj;
  bool shifts;        // both maps are single runs: offsets are shifts
  int lym, lyn;
  int64_t o_lane[4];  // thread's bins: (tid % 32, 4 (tid / 32) + q)
  bool ok[4];
  uint64_t span;      // largest offset of a bin from its sub-tile's origin
  __device__ void init(const TopRArgs &t) {
    M = 1u << t.mbits;
    N = 1u << t.nbits;
    lnt = t.nbits > 6 ? t.nbits - 6 : 0;
    lmt = t.mbits > 6 ? t.mbits - 6 : 0;
    nmaj = t.nmajor;
    shifts = t.m.nruns == 1 && t.n.nruns == 1;
    lym = t.m.ly[0];
    lyn = t.n.ly[0];
    // a thread holds four consecutive rows: o_lane[q] = o(ml, 4 nl0) + o(q)
    // (nl0 = tid / 32 < 8 for 256 threads, disjoint bits), so in thread
    // order the buffer fills row block by row block: the lowest bin indices
    // of a sub-tile come first (on a flat top, where many bins tie, the first
    // cut then already holds the best)
    const uint32_t ml = threadIdx.x & 31, nl0 = threadIdx.x >> 5;
    const int64_t o0 = offset(t, ml, 4 * nl0);
    const int64_t r1 = offset(t, 0, 1), r2 = offset(t, 0, 2);
    o_lane[0] = o0;
    o_lane[1] = o0 + r1;
    o_lane[2] = o0 + r2;
    o_lane[3] = o0 + r1 + r2;
#pragma unroll
    for (int q = 0; q < 4; ++q) ok[q] = ml < M && 4 * nl0 + q < N;
    span = (uint64_t)offset(t, (M < 32 ? M : 32) - 1, (N < 32 ? N : 32) - 1);
  }
  // index of the sub-tile's origin bin, the lowest index in it, or ~0 for a
  // sub-tile wholly outside the result (distinct for distinct sub-tiles that
  // hold bins: the maps are injective on disjoint bits)
  __device__ int64_t offset(const TopRArgs &t, uint32_t m0, uint32_t n0) const {
    return shifts ? ((int64_t)m0 << lym) + ((int64_t)n0 << lyn) : map_y(t.m, m0) + map_y(t.n, n0);
  }
  __device__ uint64_t origin(const TopRArgs &t, int sb) const {
    uint32_t m0, n0;
    sub_origin(sb, lmt, lnt, nmaj, m0, n0);
    if (m0 >= M || n0 >= N) return ~uint64_t(0);
    return (uint64_t)offset(t, m0, n0);
  }
  // origins are multiples of 32: a bin exists iff the origin and (ml, nl) do.
  // The bins' type is a template parameter: the loads of several sub-tiles
  // stay in flight together (no branch between a load and its conversion).
  // (an inactive call reads bin 0 and marks every entry absent: no branch
  // around the loads, whose results must not be waited for one by one)
  template <bool OUTF>
  __device__ void load(const TopRArgs &t, int sb, bool active, double v[4], uint64_t ix[4]) const {
    uint32_t m0, n0;
    sub_origin(sb, lmt, lnt, nmaj, m0, n0);
    const bool sub_ok = active && m0 < M && n0 < N;
    const int64_t o0 = sub_ok ? offset(t, m0, n0) : 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) ix[q] = (sub_ok && ok[q]) ? (uint64_t)(o0 + o_lane[q]) : ~uint64_t(0);
    typedef typename std::conditional<OUTF, float, double>::type O;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = (double)static_cast<const O *>(t.C)[ix[q] == ~uint64_t(0) ? 0 : ix[q]];
  }
};

// A work-group's running R best: entries [0, n) of val / idx in LDS.
struct TopBuf {
  double *val;
  uint64_t *idx;
  int n = 0;
  bool have_bar = false;  // R entries kept: a new entry must beat the R-th
  double bar_v = 0.0;
  uint64_t bar_i = 0;
  __device__ bool wants(double v, uint64_t i, double tau) const {
    return i != ~uint64_t(0) && v == v && v >= tau && (!have_bar || better(v, i, bar_v, bar_i));
  }
  double *tv;      // [SQC_MAX_TOPR] staging of a small selection
  uint64_t *ti;
  // keep the R best, in order (better first): the buffer never holds more
  // than one entry per thread, and each thread ranks its entry by counting
  // the better ones
  __device__ void cut(int R) {
    {
      const int e = threadIdx.x;
      double v = 0.0;
      uint64_t i = 0;
      int rank = R;
      if (e < n) {
        v = val[e];
        i = idx[e];
        rank = 0;
        // (entries past n compare as worse: the loop reads 4 at a time)
        for (int q = 0; q < n; q += 4) {
          double vq[4];
          uint64_t iq[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            vq[u] = val[q + u];
            iq[u] = idx[q + u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) rank += (q + u < n && better(vq[u], iq[u], v, i)) ? 1 : 0;
        }
      }
      if (rank < R) {
        tv[rank] = v;
        ti[rank] = i;
      }
      __syncthreads();
      const int kept = n < R ? n : R;
      if (e < kept) {
        val[e] = tv[e];
        idx[e] = ti[e];
      }
      __syncthreads();
    }
    n = n < R ? n : R;
    if (n == R) {
      have_bar = true;
      bar_v = val[R - 1];
      bar_i = idx[R - 1];
    }
    __syncthreads();
  }
  // add the wanted entries of the thread's first nu of NU groups of 4 (one
  // scan when they fit; otherwise the buffer is cut to its R best, which
  // raises the bar, and what still qualifies is appended as room allows,
  // bit `done` marking the entries taken)
  template <int NU>
  __device__ void add_many(const double (&v)[NU][4], const uint64_t (&ix)[NU][4], int nu, double tau, int R,
                           int *wsum, bool early_bar) {
    static_assert(4 * NU <= 32, "one bit per entry");
    uint32_t done = 0;
    for (;;) {
      // the entries this thread appends, one bit each (a per-lane register,
      // not a lane mask per entry kept across the scan)
      uint32_t want = 0;
#pragma unroll
      for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          want |= (u < nu && wants(v[u][q], ix[u][q], tau) ? 1u : 0u) << (4 * u + q);
      want &= ~done;
      int total;
      int at = block_scan_excl(__builtin_popcount(want), wsum, total);
      if (total == 0) break;
      if (n + total > kCutAt && n > R) {
        cut(R);
        continue;
      }
      const int room = kCutAt - n;
      at += n;
#pragma unroll
      for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if ((want >> (4 * u + q)) & 1) {
            if (at < kCutAt) {
              val[at] = v[u][q];
              idx[at] = ix[u][q];
              done |= 1u << (4 * u + q);
            }
            ++at;
          }
      n += total < room ? total : room;
      __syncthreads();
      if (early_bar && !have_bar && n >= R) cut(R);  // a bar as early as possible
      if (total <= room) break;
    }
  }
};

constexpr int kVisit = 8;  // sub-tiles whose loads are in flight together

template <bool OUTF>
__device__ __forceinline__ void topr_gather_body(const TopRArgs &t, int bid, int nb) {
  __shared__ double sv[kNG];
  __shared__ int wsum[kTW];
  __shared__ double ps[kTW], pc[kTW];
  __shared__ double s_tau;
  __shared__ double bval[kBufCap];
  __shared__ uint64_t bidx[kBufCap];
  __shared__ double tval[SQC_MAX_TOPR];
  __shared__ uint64_t tidx[SQC_MAX_TOPR];
  __shared__ int list[kTThreads];
  __shared__ double lmx[kTThreads];
  __shared__ uint64_t lorg[kTThreads];
  __shared__ double wmax[kTW];
  __shared__ double sw[kTThreads];  // work-group maxima that reach tau
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int R = t.top_r;
  const int G = t.ngroups;
  const int ng = G < kNG ? G : kNG;  // group g: GEMM work-groups [g G / ng, (g+1) G / ng)
  // the first run's sub-tile maxima, loaded now so that their latency hides
  // behind the threshold
  // runs of `run` sub-tiles (64 to 256: as many work-groups as there are
  // take part in the visits when the bins are few)
  int run = 64;
  while (run < kTThreads && (int64_t)run * nb < t.nsub) run <<= 1;
  const int sb_first = bid * run + tid;
  const double mx_first = tid < run && sb_first < t.nsub ? t.blk_max[sb_first] : -INFINITY;

  // ---- group maxima (and, in work-group 0, the total sum) ----
  double s = 0.0, c = 0.0, gm = -INFINITY;
  double wm[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};  // the group's work-group maxima
  if (tid < ng) {
    const int w0 = tid * G / ng, w1 = (tid + 1) * G / ng;
    for (int w = w0; w < w1; w += 4) {
      double x[4][3];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 3; ++k) x[j][k] = t.wg_stats[3 * (w + j < w1 ? w + j : w0) + k];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (w + j < w1) {
          neumaier(s, c, x[j][0]);
          c += x[j][1];
          gm = fmax(gm, x[j][2]);
          if (w == w0) wm[j] = x[j][2];
        }
    }
  }
  if (bid == 0) {
    for (int off = 32; off >= 1; off >>= 1) {
      const double s2 = __shfl_xor(s, off), c2 = __shfl_xor(c, off);
      two_sum_merge(s, c, s2, c2);
    }
    if (lane == 0) {
      ps[wave] = s;
      pc[wave] = c;
    }
  }

  // ---- threshold tau: the R-th largest maximum of nc groups, each 2^cs
  // consecutive groups above (coarser when R is small: R groups still hold a
  // bin >= tau each).  Group g counts the maxima >= its own; tau is the
  // largest maximum reached by at least R of them. ----
  int cs = 0;
  while (cs < 2 && (ng >> (cs + 1)) >= 4 * R) ++cs;
  const int nc = (ng + (1 << cs) - 1) >> cs;
  double cm = gm;  // -inf past the ng groups
  for (int off = 1; off < (1 << cs); off <<= 1) cm = fmax(cm, __shfl_xor(cm, off));
  if ((tid & ((1 << cs) - 1)) == 0) sv[tid >> cs] = cm;
  __syncthreads();
  double cand = -INFINITY;
  if (nc >= R && tid < nc) {
    const double me = sv[tid];
    int cnt = 0;
#pragma unroll 8
    for (int j = 0; j < nc; ++j) cnt += sv[j] >= me ? 1 : 0;
    if (cnt >= R) cand = me;
  }
  {
    using WaveMax = rocprim::warp_reduce<double, 64>;
    __shared__ typename WaveMax::storage_type max_st[kTW];
    double m;
    WaveMax().reduce(cand, m, max_st[wave], rocprim::maximum<double>());
    cand = m;  // lane 0 holds the wave's maximum
  }
  if (lane == 0) wmax[wave] = cand;
  __syncthreads();
  if (tid == 0) {
    double m = wmax[0];
    for (int q = 1; q < kTW; ++q) m = fmax(m, wmax[q]);
    s_tau = m;  // -inf with fewer groups than R
  }
  __syncthreads();
  double tau = s_tau;  // -inf with fewer groups than R
  // ---- refinement: the R-th largest GEMM work-group maximum, a tighter
  // threshold (R work-groups hold a bin >= it each) when the top is flat and
  // many groups reach tau.  Every work-group maximum that reaches tau is
  // collected (at least R do) and ranked by counting, as above; skipped when
  // a group holds more than four work-groups or more than kTThreads reach
  // tau (tau stays valid). ----
  if (G <= 4 * ng && tau > -INFINITY) {
    int keepw = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) keepw += wm[j] >= tau ? 1 : 0;
    int nw;
    int at = block_scan_excl(keepw, wsum, nw);
    if (nw <= kTThreads) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (wm[j] >= tau) sw[at++] = wm[j];
      __syncthreads();
      double cand2 = -INFINITY;
      if (tid < nw) {
        const double me = sw[tid];
        int cnt = 0;
        for (int j = 0; j < nw; ++j) cnt += sw[j] >= me ? 1 : 0;
        if (cnt >= R) cand2 = me;
      }
      {
        using WaveMax = rocprim::warp_reduce<double, 64>;
        __shared__ typename WaveMax::storage_type max_st2[kTW];
        double m;
        WaveMax().reduce(cand2, m, max_st2[wave], rocprim::maximum<double>());
        cand2 = m;
      }
      if (lane == 0) wmax[wave] = cand2;
      __syncthreads();
      double m = wmax[0];
      for (int q = 1; q < kTW; ++q) m = fmax(m, wmax[q]);
      tau = fmax(tau, m);
      __syncthreads();  // (wmax and sw are not read again)
    }
  }
  if (bid == 0 && tid == 0) {
    double S = ps[0], Cc = pc[0];
    for (int q = 1; q < kTW; ++q) two_sum_merge(S, Cc, ps[q], pc[q]);
    t.tau_sum[0] = tau;
    t.tau_sum[1] = S + Cc;
  }

  // ---- this work-group's sub-tiles whose maximum reaches tau (and the
  // running R-th best): listed kTThreads at a time, then visited ----
  TopBuf buf;
  buf.val = bval;
  buf.idx = bidx;
  buf.tv = tval;
  buf.ti = tidx;
  SubTileBins stb;
  stb.init(t);
  // A sub-tile can hold a bin that beats the running R-th best only if its
  // maximum is larger, or equal with its lowest bin index (its origin's:
  // offsets grow with both coordinates) below the R-th best's index.
  auto may_improve = [&](double mxq, uint64_t orgq) -> bool {
    if (!buf.have_bar || mxq > buf.bar_v) return true;
    return mxq == buf.bar_v && orgq < buf.bar_i;
  };
  for (int base = bid * run; base < t.nsub; base += nb * run) {
    const int sb = base + tid;
    const uint64_t org = tid < run && sb < t.nsub ? stb.origin(t, sb) : ~uint64_t(0);
    const bool holds = org != ~uint64_t(0);
    const double mx = !holds ? -INFINITY : (base == bid * run ? mx_first : t.blk_max[sb]);
    const int keep = (holds && mx >= tau && may_improve(mx, org)) ? 1 : 0;
    int total;
    const int at = block_scan_excl(keep, wsum, total);
    if (keep) {
      list[at] = sb;
      lmx[at] = mx;
      lorg[at] = org;
    }
    __syncthreads();
    if (total > 2 * R) {
      // Many candidates (a flat top).  Sub-tile T's maximum is a bin that
      // beats every bin of sub-tile S when it is larger than S's maximum, or
      // equal to it with T's last bin below S's origin; a sub-tile beaten so
      // by R others holds none of the R best.  Every sub-tile that beats a
      // listed one is listed itself, so the count runs over the list.
      int keep2 = 0, sbk = 0;
      double mk = 0.0;
      uint64_t gk = 0;
      if (tid < total) {
        sbk = list[tid];
        mk = lmx[tid];
        gk = lorg[tid];
        int beaten = 0;
        for (int j = 0; j < total; ++j) {
          const double xj = lmx[j];
          beaten += (xj > mk || (xj == mk && lorg[j] + stb.span < gk)) ? 1 : 0;
        }
        keep2 = beaten < R ? 1 : 0;
      }
      int total2;
      const int at2 = block_scan_excl(keep2, wsum, total2);  // (its barriers end the reads above)
      if (keep2) {
        list[at2] = sbk;
        lmx[at2] = mk;
        lorg[at2] = gk;
      }
      total = total2;
      __syncthreads();
    }
    if (total > 1) {
      // visit the candidates best first (larger maximum, then lower origin)
      // so that the running R-th best rises fast and prunes the rest
      int rank = 0, sbk = 0;
      double mk = 0.0;
      uint64_t gk = 0;
      if (tid < total) {
        sbk = list[tid];
        mk = lmx[tid];
        gk = lorg[tid];
        for (int j = 0; j < total; ++j) rank += better(lmx[j], lorg[j], mk, gk) ? 1 : 0;
      }
      __syncthreads();
      if (tid < total) {
        list[rank] = sbk;
        lmx[rank] = mk;
        lorg[rank] = gk;
      }
      __syncthreads();
    }
    // up to kVisit sub-tiles' loads in flight together (a long list starts
    // with one, to set an R-th best); each listed sub-tile is checked again
    // against the running R-th best
    for (int q = 0; q < total;) {
      // the list is in visiting order (larger maximum, then lower origin): once
      // one cannot beat the running R-th best, none after it can
      if (!may_improve(lmx[q], lorg[q])) break;
      const int nl = min((buf.have_bar || q > 0 || total <= kVisit) ? kVisit : 1, total - q);
      double v[kVisit][4];
      uint64_t ix[kVisit][4];
      bool go[kVisit];
      int sbv[kVisit];
#pragma unroll
      for (int u = 0; u < kVisit; ++u) {
        const int qu = q + u < total ? q + u : q;
        go[u] = u < nl && may_improve(lmx[qu], lorg[qu]);
        sbv[u] = list[qu];
      }
#pragma unroll
      for (int u = 0; u < kVisit; ++u) stb.template load<OUTF>(t, sbv[u], go[u], v[u], ix[u]);
      buf.add_many(v, ix, nl, tau, R, wsum, true);
      q += nl;
    }
    __syncthreads();  // list is rewritten by the next round
  }
  if (buf.n > R) buf.cut(R);  // the slot need not be sorted
  if (tid < R) {
    t.slot_val[(int64_t)bid * R + tid] = tid < buf.n ? bval[tid] : -INFINITY;
    t.slot_idx[(int64_t)bid * R + tid] = tid < buf.n ? bidx[tid] : ~uint64_t(0);
  }
  if (tid == 0) t.slot_n[bid] = buf.n;
}

__device__ __forceinline__ void topr_rank_body(const TopRArgs &t) {
  __shared__ int wsum[kTW];
  __shared__ double bval[kBufCap];
  __shared__ uint64_t bidx[kBufCap];
  __shared__ double tval[SQC_MAX_TOPR];
  __shared__ uint64_t tidx[SQC_MAX_TOPR];
  const int tid = threadIdx.x;
  const int R = t.top_r;
  const double tau = t.tau_sum[0];
  TopBuf buf;
  buf.val = bval;
  buf.idx = bidx;
  buf.tv = tval;
  buf.ti = tidx;
  // slot entries f = w R + j, j < slot_n[w]
  const int npos = t.gather_groups * R;
  for (int f0 = 0; f0 < npos; f0 += 4 * kTThreads) {
    double v[1][4];
    uint64_t ix[1][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = f0 + q * kTThreads + tid, ff = f < npos ? f : 0;
      const int cn = t.slot_n[ff / R];
      v[0][q] = t.slot_val[ff];
      ix[0][q] = t.slot_idx[ff];
      if (!(f < npos && ff % R < cn)) ix[0][q] = ~uint64_t(0);
    }
    buf.add_many(v, ix, 1, tau, R, wsum, false);
  }
  buf.cut(R);
  if (tid < R) {
    t.top_out[2 * tid] = tid < buf.n ? bval[tid] : -INFINITY;
    reinterpret_cast<uint64_t *>(t.top_out)[2 * tid + 1] = tid < buf.n ? bidx[tid] : ~uint64_t(0);
  }
  if (tid == 0) *t.sum_out = t.tau_sum[1];
}

template <bool OUTF>
__global__ __launch_bounds__(kTThreads) void topr_gather(TopRArgs t) {
  topr_gather_body<OUTF>(t, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kTThreads) void topr_rank(TopRArgs t) { topr_rank_body(t); }

// Batched top-R: job j's gather takes work-groups [start[j], start[j + 1]),
// then one rank work-group per job.
template <bool OUTF>
__global__ __launch_bounds__(kTThreads) void topr_gather_grouped(const TopRArgs *__restrict__ jobs,
                                                                 const int *__restrict__ start, int n) {
  if ((int)blockIdx.x >= start[n]) return;  // (a grid sized for a larger table)
  const int j = find_job(start, n, blockIdx.x);
  const int s0 = start[j];
  topr_gather_body<OUTF>(jobs[j], (int)blockIdx.x - s0, start[j + 1] - s0);
}
__global__ __launch_bounds__(kTThreads) void topr_rank_grouped(const TopRArgs *__restrict__ jobs) {
  topr_rank_body(jobs[blockIdx.x]);
}

__global__ void zero_bytes(unsigned int *p, size_t nwords) {
  for (size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x; q < nwords;
       q += size_t(gridDim.x) * blockDim.x)
    p[q] = 0u;
}

}  // namespace

int gemm_nmajor(const GemmArgs &g) {
  // n panels outer when B is the larger operand (and there are several m panels)
  return g.mbits > 6 && g.nbits > g.mbits ? 1 : 0;
}

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
template <int PREC, bool FOLD, bool OUTF, int REG>
int resident_groups() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (!cached[dev]) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gemm<PREC, FOLD, OUTF, REG>, kThreads, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 2;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    cached[dev] = per_cu * cus;
  }
  return cached[dev];
}

// Calls L::run<PREC, FOLD, OUTF, REG>() for the specialisation `sp`.
template <int PREC, bool FOLD, bool OUTF, class L>
int dispatch_r(const GemmSpec &sp, const L &l) {
  if (sp.reg == 4) return l.template run<PREC, FOLD, OUTF, 4>();
  if (sp.reg == 3) return l.template run<PREC, FOLD, OUTF, 3>();
  if (sp.reg == 2) return l.template run<PREC, FOLD, OUTF, 2>();
  if (sp.reg == 1) return l.template run<PREC, FOLD, OUTF, 1>();
  return l.template run<PREC, FOLD, OUTF, 0>();
}
template <int PREC, bool FOLD, class L>
int dispatch_o(const GemmSpec &sp, const L &l) {
  return sp.outf ? dispatch_r<PREC, FOLD, true>(sp, l) : dispatch_r<PREC, FOLD, false>(sp, l);
}
template <class L>
int dispatch(const GemmSpec &sp, const L &l) {
  if (sp.prec == SQC_F64) return dispatch_o<SQC_F64, false>(sp, l);
  if (sp.prec == SQC_F32) return sp.fold ? dispatch_o<SQC_F32, true>(sp, l) : dispatch_o<SQC_F32, false>(sp, l);
  return sp.fold ? dispatch_o<SQC_BF16X3, true>(sp, l) : dispatch_o<SQC_BF16X3, false>(sp, l);
}

struct GroupsQuery {
  int64_t tiles;
  template <int PREC, bool FOLD, bool OUTF, int REG>
  int run() const {
    int64_t cap = resident_groups<PREC, FOLD, OUTF, REG>();
    if (cap > kMaxGemmGroups) cap = kMaxGemmGroups;
    return (int)(tiles < cap ? tiles : cap);
  }
};

struct DirectLaunch {
  const GemmArgs &g;
  int groups;
  hipStream_t s;
  hipEvent_t start, stop;
  template <int PREC, bool FOLD, bool OUTF, int REG>
  int run() const {
    if (start)  // events recorded by the dispatch itself: the kernel's own span
      hipExtLaunchKernelGGL((gemm<PREC, FOLD, OUTF, REG>), dim3((unsigned)groups), dim3(kThreads), 0, s, start,
                            stop, 0, g);
    else
      hipLaunchKernelGGL((gemm<PREC, FOLD, OUTF, REG>), dim3((unsigned)groups), dim3(kThreads), 0, s, g);
    return groups;
  }
};

struct GroupedLaunch {
  const GemmArgs *jobs;
  const int *start;
  int n, total;
  hipStream_t s;
  template <int PREC, bool FOLD, bool OUTF, int REG>
  int run() const {
    hipLaunchKernelGGL((gemm_grouped<PREC, FOLD, OUTF, REG>), dim3((unsigned)total), dim3(kThreads), 0, s,
                       jobs, start, n);
    return total;
  }
};

GemmSpec prepare_gemm(GemmArgs &g, int prec) {
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
  GemmSpec sp;
  sp.prec = prec;
  // fold FP32 chunks into FP64 only when the final K spans several chunks;
  // a chunk is one K stage
  sp.fold = prec != SQC_F64 && g.final_step && g.kbits > 6;
  sp.outf = g.out_f32 != 0;
  const bool regular = g.mbits >= 6 && g.nbits >= 6 && g.kbits >= 6 && g.k.nruns >= 1 && g.k.bits[0] >= 4;
  const bool simple = g.m.nruns == 1 && g.n.nruns == 1 && g.k.nruns == 1;
  sp.reg = g.acc_mode ? 3 : regular ? (simple ? 2 : 1) : 0;
  return sp;
}

bool gemm_narrow_ok(const GemmArgs &g, const GemmSpec &sp) {
  return g.kbits <= 4 && sp.reg == 0 && !sp.fold && !g.acc_mode;
}

GemmSpec gemm_default_spec(const GemmArgs &g, const GemmSpec &sp) {
  GemmSpec d = sp;
  if (gemm_narrow_ok(g, sp)) d.reg = 4;
  return d;
}

int gemm_spec_id(const GemmSpec &sp) {
  return ((sp.prec * 2 + (sp.fold ? 1 : 0)) * 2 + (sp.outf ? 1 : 0)) * 5 + sp.reg;
}

int gemm_groups(const GemmArgs &g, const GemmSpec &sp) { return dispatch(sp, GroupsQuery{gemm_tiles(g)}); }

int gemm_resident_cap(const GemmSpec &sp) { return dispatch(sp, GroupsQuery{int64_t(kMaxGemmGroups)}); }

// ---- launch choices found by the tuner, per GEMM shape ----
namespace {
std::mutex tune_mu;
std::unordered_map<uint64_t, GemmTuning> tune_table;
uint64_t tune_epoch = 0;  // changes whenever the table does

void mix(uint64_t &h, int64_t v) {
  h ^= (uint64_t)v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
}
void mix_map(uint64_t &h, const IndexMap &m) {
  mix(h, m.nruns);
  for (int r = 0; r < m.nruns; ++r) {
    mix(h, m.bits[r]);
    mix(h, m.sx[r]);
    mix(h, m.sy[r]);
    mix(h, m.lx[r]);
    mix(h, m.ly[r]);
  }
}
}  // namespace

uint64_t gemm_tune_key(const GemmArgs &g, const GemmSpec &sp) {
  uint64_t h = 0x2207009330000001ull;
  mix(h, gemm_spec_id(sp));
  mix(h, g.mbits);
  mix(h, g.nbits);
  mix(h, g.kbits);
  mix(h, g.out_f32);
  mix(h, g.final_step);
  mix(h, g.stats);
  mix_map(h, g.m);
  mix_map(h, g.n);
  mix_map(h, g.k);
  return h;
}

bool gemm_tuned(const GemmArgs &g, const GemmSpec &sp, GemmTuning &out) {
  const uint64_t k = gemm_tune_key(g, sp);
  std::lock_guard<std::mutex> lk(tune_mu);
  auto it = tune_table.find(k);
  if (it == tune_table.end()) return false;
  out = it->second;
  return true;
}

void gemm_tune_store(const GemmArgs &g, const GemmSpec &sp, const GemmTuning &t) {
  const uint64_t k = gemm_tune_key(g, sp);
  std::lock_guard<std::mutex> lk(tune_mu);
  tune_table[k] = t;
  ++tune_epoch;
}

void gemm_tune_reset() {
  std::lock_guard<std::mutex> lk(tune_mu);
  tune_table.clear();
  ++tune_epoch;
}

size_t gemm_tune_size() {
  std::lock_guard<std::mutex> lk(tune_mu);
  return tune_table.size();
}

uint64_t gemm_tune_version() {
  std::lock_guard<std::mutex> lk(tune_mu);
  return tune_epoch;
}

void launch_gemm_spec(const GemmArgs &g, const GemmSpec &sp, int groups, hipStream_t s, hipEvent_t start,
                      hipEvent_t stop) {
  dispatch(sp, DirectLaunch{g, groups, s, start, stop});
}

void launch_gemm_grouped(const GemmSpec &sp, const GemmArgs *jobs, const int *start, int n, int total,
                         hipStream_t s) {
  dispatch(sp, GroupedLaunch{jobs, start, n, total, s});
}

int launch_gemm(const GemmArgs &g_in, int prec, hipStream_t s) {
  GemmArgs g = g_in;
  const GemmSpec sp = gemm_default_spec(g, prepare_gemm(g, prec));
  const int groups = gemm_groups(g, sp);
  launch_gemm_spec(g, sp, groups, s);
  return groups;
}

void launch_topr(const TopRArgs &t, hipStream_t s) {
  if (t.out_f32) hipLaunchKernelGGL(topr_gather<true>, dim3((unsigned)t.gather_groups), dim3(kTThreads), 0, s, t);
  else hipLaunchKernelGGL(topr_gather<false>, dim3((unsigned)t.gather_groups), dim3(kTThreads), 0, s, t);
  hipLaunchKernelGGL(topr_rank, dim3(1), dim3(kTThreads), 0, s, t);
}

int topr_gather_groups(int64_t nsub) {
  const int64_t g = (nsub + 63) / 64;
  return (int)(g < 1 ? 1 : (g > kTopRSlots ? kTopRSlots : g));
}

void launch_topr_grouped(const TopRArgs *jobs, const int *start, int n, int total, int out_f32, hipStream_t s) {
  if (out_f32)
    hipLaunchKernelGGL(topr_gather_grouped<true>, dim3((unsigned)total), dim3(kTThreads), 0, s, jobs, start, n);
  else
    hipLaunchKernelGGL(topr_gather_grouped<false>, dim3((unsigned)total), dim3(kTThreads), 0, s, jobs, start, n);
  hipLaunchKernelGGL(topr_rank_grouped, dim3((unsigned)n), dim3(kTThreads), 0, s, jobs);
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
