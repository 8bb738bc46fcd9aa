// Pairwise contraction of compute-graph tensors (Sec. 6.1: contracting two
// subcircuit tensors over their shared cut indices is the matrix product
// C = A B) as a strided-tensor GEMM on MFMA:
//
//   C[offC_m(m) + offC_n(n)] = sum_k A[offA_m(m) + offA_k(k)] * B[offB_n(n) + offB_k(k)]
//
// m runs over A's free axes, n over B's free axes, k over the shared cut
// labels; every dimension is a power of two and each offset is a sum of
// per-run strides (IndexMap), so operands are read in place, whatever the axis
// order the previous step left them in.
//
// Precisions: F64 (v_mfma_f64_16x16x4f64, FP64 tensors), F32
// (v_mfma_f32_16x16x4f32) and BF16X3 (each FP32 operand split into bf16
// hi + lo when staged into LDS; hi*hi + hi*lo + lo*hi on
// v_mfma_f32_16x16x32_bf16, FP32 accumulation).  The last step of a
// contraction (the sum over the final cut labels) folds the FP32 accumulator
// into FP64 every 2^chunk_bits labels with Neumaier compensation and writes
// per-work-group FP64 sums and maxima; the last work-group to finish reduces
// them in a fixed order (total sum, top-R threshold).
//
// Tiles: 64 x 64 per work-group of 4 waves (2 x 2, each 32 x 32 = 2 x 2 MFMA
// 16x16 tiles).  Work-groups are dispatched round-robin over the 8 XCDs; the
// tile order puts the n-tiles that share an A row-panel on one XCD so the
// panel is fetched into that XCD's L2 once.
#include "common.hpp"

namespace sqc {

namespace {

constexpr int kThreads = 256;
constexpr int BM = 64;
constexpr int BN = 64;

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short v8u16 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int64_t map_x(const IndexMap &m, int64_t idx) {
  int64_t off = 0;
  int sh = 0;
  for (int r = 0; r < m.nruns; ++r) {
    off += ((idx >> sh) & ((int64_t(1) << m.bits[r]) - 1)) * m.sx[r];
    sh += m.bits[r];
  }
  return off;
}

__device__ __forceinline__ int64_t map_y(const IndexMap &m, int64_t idx) {
  int64_t off = 0;
  int sh = 0;
  for (int r = 0; r < m.nruns; ++r) {
    off += ((idx >> sh) & ((int64_t(1) << m.bits[r]) - 1)) * m.sy[r];
    sh += m.bits[r];
  }
  return off;
}

// Tile coordinates of a work-group, XCD-aware (see file comment).
__device__ __forceinline__ void tile_of(int mbits, int nbits, int64_t &m0, int64_t &n0) {
  const int64_t nt = (nbits > 6) ? (int64_t(1) << (nbits - 6)) : 1;
  const int64_t nb = gridDim.x;
  const int64_t b = blockIdx.x;
  int64_t t = b;
  if ((nb & 7) == 0) t = (b & 7) * (nb >> 3) + (b >> 3);
  m0 = (t / nt) * BM;
  n0 = (t % nt) * BN;
}

// round-to-nearest-even float -> bf16 bits (finite inputs)
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
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

// Block-wide argmax (all threads get the result).  `sv`/`si` are 4-entry LDS.
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

template <int PREC>
struct Tr;
template <>
struct Tr<SQC_F64> {
  typedef double T;
  typedef v4d Acc;
  static constexpr int BK = 16;
};
template <>
struct Tr<SQC_F32> {
  typedef float T;
  typedef v4f Acc;
  static constexpr int BK = 16;
};
template <>
struct Tr<SQC_BF16X3> {
  typedef float T;
  typedef v4f Acc;
  static constexpr int BK = 32;
};

template <int PREC>
__global__ __launch_bounds__(kThreads) void gemm(GemmArgs g) {
  typedef typename Tr<PREC>::T T;
  typedef typename Tr<PREC>::Acc Acc;
  constexpr int BK = Tr<PREC>::BK;
  constexpr bool SPLIT = PREC == SQC_BF16X3;
  constexpr int PAD = 8;  // bf16 row padding
  // F32/F64: As[k][m]; BF16: Ah/Al[m][k]
  __shared__ __attribute__((aligned(16))) unsigned char lds[SPLIT ? (4 * BM * (BK + PAD) * 2)
                                                                  : (2 * BK * BM * sizeof(T))];
  __shared__ double red_v[4];
  __shared__ uint64_t red_i[4];
  __shared__ int last_flag;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t M = int64_t(1) << g.mbits;
  const int64_t N = int64_t(1) << g.nbits;
  const int64_t K = int64_t(1) << g.kbits;
  int64_t m0, n0;
  tile_of(g.mbits, g.nbits, m0, n0);

  const T *A = static_cast<const T *>(g.A);
  const T *B = static_cast<const T *>(g.B);

  // global -> LDS assignment: column = tid % 64 (m or n), rows tid / 64 + 4 j
  const int lcol = tid & 63;
  const int lrow = tid >> 6;
  const bool am_ok = m0 + lcol < M;
  const bool bn_ok = n0 + lcol < N;
  const int64_t a_moff = am_ok ? map_x(g.m, m0 + lcol) : 0;
  const int64_t b_noff = bn_ok ? map_x(g.n, n0 + lcol) : 0;

  Acc acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;
  double S[2][2][4], Cc[2][2][4];
  if (g.final_step) {
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int r = 0; r < 4; ++r) S[i][j][r] = Cc[i][j][r] = 0.0;
  }
  const int64_t chunk = int64_t(1) << g.chunk_bits;

  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    // ---- stage A and B tiles ----
    if constexpr (!SPLIT) {
      T *As = reinterpret_cast<T *>(lds);
      T *Bs = As + BK * BM;
      for (int j = 0; j < BK / 4; ++j) {
        int kr = lrow + 4 * j;
        int64_t k = k0 + kr;
        T av = 0, bv = 0;
        if (k < K) {
          if (am_ok) av = A[a_moff + map_x(g.k, k)];
          if (bn_ok) bv = B[b_noff + map_y(g.k, k)];
        }
        As[kr * BM + lcol] = av;
        Bs[kr * BN + lcol] = bv;
      }
    } else {
      unsigned short *Ah = reinterpret_cast<unsigned short *>(lds);
      unsigned short *Al = Ah + BM * (BK + PAD);
      unsigned short *Bh = Al + BM * (BK + PAD);
      unsigned short *Bl = Bh + BN * (BK + PAD);
      for (int j = 0; j < BK / 4; ++j) {
        int kr = lrow + 4 * j;
        int64_t k = k0 + kr;
        float av = 0.f, bv = 0.f;
        if (k < K) {
          if (am_ok) av = A[a_moff + map_x(g.k, k)];
          if (bn_ok) bv = B[b_noff + map_y(g.k, k)];
        }
        unsigned short ah = bf16_bits(av), bh = bf16_bits(bv);
        Ah[lcol * (BK + PAD) + kr] = ah;
        Al[lcol * (BK + PAD) + kr] = bf16_bits(av - bf16_float(ah));
        Bh[lcol * (BK + PAD) + kr] = bh;
        Bl[lcol * (BK + PAD) + kr] = bf16_bits(bv - bf16_float(bh));
      }
    }
    __syncthreads();
    // ---- MFMA ----
    if constexpr (!SPLIT) {
      const T *As = reinterpret_cast<const T *>(lds);
      const T *Bs = As + BK * BM;
      for (int kk = 0; kk < BK / 4; ++kk) {
        const int kr = kk * 4 + (lane >> 4);
        T a[2], b[2];
        for (int i = 0; i < 2; ++i) a[i] = As[kr * BM + wm * 32 + i * 16 + (lane & 15)];
        for (int j = 0; j < 2; ++j) b[j] = Bs[kr * BN + wn * 32 + j * 16 + (lane & 15)];
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) {
            if constexpr (PREC == SQC_F64)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
          }
      }
    } else {
      const unsigned short *Ah = reinterpret_cast<const unsigned short *>(lds);
      const unsigned short *Al = Ah + BM * (BK + PAD);
      const unsigned short *Bh = Al + BM * (BK + PAD);
      const unsigned short *Bl = Bh + BN * (BK + PAD);
      const int kc = 8 * (lane >> 4);
      v8bf ah[2], al[2], bh[2], bl[2];
      for (int i = 0; i < 2; ++i) {
        int row = wm * 32 + i * 16 + (lane & 15);
        ah[i] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v8u16 *>(Ah + row * (BK + PAD) + kc));
        al[i] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v8u16 *>(Al + row * (BK + PAD) + kc));
      }
      for (int j = 0; j < 2; ++j) {
        int col = wn * 32 + j * 16 + (lane & 15);
        bh[j] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v8u16 *>(Bh + col * (BK + PAD) + kc));
        bl[j] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v8u16 *>(Bl + col * (BK + PAD) + kc));
      }
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
    // ---- compensated FP64 fold of the FP32 chunk ----
    if constexpr (PREC != SQC_F64) {
      if (g.final_step && (((k0 + BK) & (chunk - 1)) == 0 || k0 + BK >= K)) {
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
              neumaier(S[i][j][r], Cc[i][j][r], (double)acc[i][j][r]);
              acc[i][j][r] = 0.f;
            }
      }
    }
  }

  // ---- epilogue: store, block statistics ----
  // MFMA result layout: lane holds column lane % 16 of each 16 x 16 tile and
  // four rows: 4 * (lane / 16) + r for the FP32 instructions, lane / 16 + 4 r
  // for v_mfma_f64_16x16x4f64.
  const int64_t row_base = m0 + wm * 32 + (PREC == SQC_F64 ? (lane >> 4) : 4 * (lane >> 4));
  const int row_step = PREC == SQC_F64 ? 4 : 1;
  const int64_t col_base = n0 + wn * 32 + (lane & 15);
  double lsum = 0.0, lmax = -INFINITY;
  for (int j = 0; j < 2; ++j) {
    const int64_t n = col_base + j * 16;
    if (n >= N) continue;
    const int64_t noff = map_y(g.n, n);
    for (int i = 0; i < 2; ++i)
      for (int r = 0; r < 4; ++r) {
        const int64_t m = row_base + i * 16 + r * row_step;
        if (m >= M) continue;
        double v;
        if (PREC == SQC_F64 || !g.final_step) v = (double)acc[i][j][r];
        else v = S[i][j][r] + Cc[i][j][r];
        const int64_t o = map_y(g.m, m) + noff;
        double stored;
        if (g.out_f32) {
          float f = (float)v;
          static_cast<float *>(g.C)[o] = f;
          stored = (double)f;
        } else {
          static_cast<double *>(g.C)[o] = v;
          stored = v;
        }
        if (g.stats) {
          lsum += v;
          lmax = stored > lmax ? stored : lmax;
        }
      }
  }
  if (!g.stats) return;

  // block sum (fixed order) and max
  for (int off = 32; off >= 1; off >>= 1) {
    lsum += __shfl_xor(lsum, off);
    double om = __shfl_xor(lmax, off);
    lmax = om > lmax ? om : lmax;
  }
  __syncthreads();
  if (lane == 0) {
    red_v[wave] = lsum;
    reinterpret_cast<double *>(red_i)[wave] = lmax;
  }
  __syncthreads();
  if (tid == 0) {
    double s = red_v[0], mx = reinterpret_cast<double *>(red_i)[0];
    for (int q = 1; q < 4; ++q) {
      s += red_v[q];
      double o = reinterpret_cast<double *>(red_i)[q];
      mx = o > mx ? o : mx;
    }
    g.blk_sum[blockIdx.x] = s;
    g.blk_max[blockIdx.x] = mx;
    __threadfence();
    unsigned int prev = atomicAdd(g.counter, 1u);
    last_flag = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!last_flag) return;
  __threadfence();
  // last work-group: total sum (Neumaier over work-group sums, fixed order)
  // and the top-R threshold tau = R-th largest work-group maximum
  const int nblk = gridDim.x;
  {
    double s = 0.0, c = 0.0;
    for (int q = tid; q < nblk; q += kThreads) neumaier(s, c, __builtin_nontemporal_load(&g.blk_sum[q]));
    __shared__ double ps[kThreads], pc[kThreads];
    ps[tid] = s;
    pc[tid] = c;
    __syncthreads();
    if (tid == 0) {
      double ts = 0.0, tc = 0.0;
      for (int q = 0; q < kThreads; ++q) {
        neumaier(ts, tc, ps[q]);
        tc += pc[q];
      }
      g.tau_sum[1] = ts + tc;
    }
  }
  const int R = g.top_r < nblk ? g.top_r : nblk;
  double pv = INFINITY;
  uint64_t pi = 0;
  bool first = true;
  for (int r = 0; r < R; ++r) {
    double bv = -INFINITY;
    uint64_t bi = ~uint64_t(0);
    for (int q = tid; q < nblk; q += kThreads) {
      double v = __builtin_nontemporal_load(&g.blk_max[q]);
      if (v != v) continue;
      bool below = first || better(pv, pi, v, (uint64_t)q);
      if (below && better(v, q, bv, bi)) {
        bv = v;
        bi = q;
      }
    }
    block_argmax(bv, bi, red_v, red_i);
    pv = bv;
    pi = bi;
    first = false;
  }
  if (tid == 0) {
    // with fewer work-groups than R every value is a candidate
    g.tau_sum[0] = g.top_r <= nblk ? pv : -INFINITY;
    *g.counter = 0u;
  }
}

// Top-R over the final bins: work-groups whose maximum reaches the threshold
// append their values >= tau (or, when they hold more than R of them, their own
// top R) to a candidate list; the last work-group ranks the list.
__global__ __launch_bounds__(kThreads) void topr(TopRArgs t) {
  __shared__ double red_v[4];
  __shared__ uint64_t red_i[4];
  __shared__ int s_cnt[4];
  __shared__ unsigned int s_base;
  __shared__ int last_flag;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const double tau = t.tau_sum[0];
  const int R = t.top_r;
  unsigned int *done = t.counter;
  unsigned int *appended = t.counter + 1;

  if (t.blk_max[blockIdx.x] >= tau) {
    // the same tile as the GEMM work-group of this index
    const int64_t M = int64_t(1) << t.mbits;
    const int64_t N = int64_t(1) << t.nbits;
    int64_t m0, n0;
    tile_of(t.mbits, t.nbits, m0, n0);
    double v[16];
    uint64_t ix[16];
    unsigned int cand = 0;  // bit q: entry q is a real bin with value >= tau
    int cnt = 0;
    for (int q = 0; q < 16; ++q) {
      const int e = tid + kThreads * q;  // 4096 entries of the 64 x 64 tile
      const int64_t m = m0 + (e & 63), n = n0 + (e >> 6);
      v[q] = -INFINITY;
      ix[q] = ~uint64_t(0);
      if (m < M && n < N) {
        const int64_t o = map_y(t.m, m) + map_y(t.n, n);
        double x = t.out_f32 ? (double)static_cast<const float *>(t.C)[o]
                             : static_cast<const double *>(t.C)[o];
        if (x == x) {
          v[q] = x;
          ix[q] = (uint64_t)o;
          if (x >= tau) {
            cand |= 1u << q;
            ++cnt;
          }
        }
      }
    }
    int wc = cnt;
    for (int off = 32; off >= 1; off >>= 1) wc += __shfl_xor(wc, off);
    if (lane == 0) s_cnt[wave] = wc;
    __syncthreads();
    const int total = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
    if (total <= R) {
      // append every value >= tau
      if (tid == 0) s_base = atomicAdd(appended, (unsigned int)total);
      // exclusive prefix of cnt over the block
      int incl = cnt;
      for (int off = 1; off < 64; off <<= 1) {
        int o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
      }
      __syncthreads();
      int woff = 0;
      for (int q = 0; q < wave; ++q) woff += s_cnt[q];
      unsigned int pos = s_base + woff + incl - cnt;
      for (int q = 0; q < 16; ++q)
        if ((cand >> q) & 1u) {
          t.cand_val[pos] = v[q];
          t.cand_idx[pos] = ix[q];
          ++pos;
        }
    } else {
      // R rounds of block argmax
      if (tid == 0) s_base = atomicAdd(appended, (unsigned int)R);
      __syncthreads();
      const unsigned int base = s_base;
      double pv = INFINITY;
      uint64_t pi = 0;
      for (int r = 0; r < R; ++r) {
        double bv = -INFINITY;
        uint64_t bi = ~uint64_t(0);
        for (int q = 0; q < 16; ++q) {
          if (!((cand >> q) & 1u)) continue;
          bool below = r == 0 || better(pv, pi, v[q], ix[q]);
          if (below && better(v[q], ix[q], bv, bi)) {
            bv = v[q];
            bi = ix[q];
          }
        }
        block_argmax(bv, bi, red_v, red_i);
        if (tid == 0) {
          t.cand_val[base + r] = bv;
          t.cand_idx[base + r] = bi;
        }
        pv = bv;
        pi = bi;
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    unsigned int prev = atomicAdd(done, 1u);
    last_flag = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!last_flag) return;
  __threadfence();
  // rank the candidates: R rounds of block argmax
  const unsigned int n = __hip_atomic_load(appended, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  double pv = INFINITY;
  uint64_t pi = 0;
  for (int r = 0; r < R; ++r) {
    double bv = -INFINITY;
    uint64_t bi = ~uint64_t(0);
    for (unsigned int q = tid; q < n; q += kThreads) {
      double v = __builtin_nontemporal_load(&t.cand_val[q]);
      uint64_t i = __builtin_nontemporal_load(&t.cand_idx[q]);
      bool below = r == 0 || better(pv, pi, v, i);
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
  if (tid == 0) {
    *t.sum_out = t.tau_sum[1];
    *done = 0u;
    *appended = 0u;
  }
}

__global__ void zero_bytes(unsigned int *p, size_t nwords) {
  for (size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x; q < nwords;
       q += size_t(gridDim.x) * blockDim.x)
    p[q] = 0u;
}

}  // namespace

int gemm_blocks(const GemmArgs &g, int prec) {
  (void)prec;
  int64_t mt = g.mbits > 6 ? (int64_t(1) << (g.mbits - 6)) : 1;
  int64_t nt = g.nbits > 6 ? (int64_t(1) << (g.nbits - 6)) : 1;
  return (int)(mt * nt);
}

void launch_gemm(const GemmArgs &g, int prec, hipStream_t s) {
  dim3 grid((unsigned)gemm_blocks(g, prec));
  switch (prec) {
    case SQC_F64: hipLaunchKernelGGL(gemm<SQC_F64>, grid, dim3(kThreads), 0, s, g); break;
    case SQC_F32: hipLaunchKernelGGL(gemm<SQC_F32>, grid, dim3(kThreads), 0, s, g); break;
    default: hipLaunchKernelGGL(gemm<SQC_BF16X3>, grid, dim3(kThreads), 0, s, g); break;
  }
}

void launch_topr(const TopRArgs &t, hipStream_t s) {
  hipLaunchKernelGGL(topr, dim3((unsigned)t.nblk), dim3(kThreads), 0, s, t);
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
