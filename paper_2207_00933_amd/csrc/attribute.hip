// Cut-basis attribution (Sec. 2.1, Eq. 1, Fig. 1): variant probabilities of
// one subcircuit -> entries T[x][sigma] for every I/X/Y/Z label assignment
// sigma of its cuts, with the factor 1/2 per out-cut folded in.  FP64.
//
// Structure: the map from (preparation s, basis beta, outcome b) to sigma is a
// tensor product of one small map per cut.  A work item is one combination of
// measurement bases beta (a label Z, X or Y per out-cut) and a tile of XT
// consecutive data states.  Its entries p[(s, beta)][x, b] for all
// preparations s and out-cut outcomes b are loaded, the maps of the first
// three out-cuts are applied in registers, the rest are staged in LDS and the
// other maps applied in place (one pass per out-cut, one per two in-cuts),
// and every label assignment
// compatible with beta is written (beta(I) = beta(Z) = Z, so a Z basis serves
// I and Z).  Loops over cuts have fixed bounds so that the parameters they
// read are fetched together rather than one dependent read per iteration.
//
//   in-cut  (digit of s -> digit of sigma):  I = p0 + p1,  Z = p0 - p1,
//            X = 2 p+ - p0 - p1,  Y = 2 p+i - p0 - p1
//   out-cut (bit b -> digit of sigma):       I = q0 + q1 (Z basis),
//            Z|X|Y = q0 - q1 (in that basis)
#include "common.hpp"

#include <algorithm>
#include <type_traits>

namespace sqc {

namespace {

constexpr int kThreads = 256;
constexpr int kLdsElems = 2048;   // doubles staged per work-group
constexpr int kPer = kLdsElems / kThreads;
constexpr int kMaxNS = 1024;
constexpr int kMaxNB = 1024;
constexpr int kMaxIn = 5;         // 4^n_in <= kMaxNS
constexpr int kMaxOut = 11;       // 4^n_in 2^n_out <= kLdsElems
constexpr int kMaxXt = 11;        // x-tile bits: 2^xt_bits <= kLdsElems
constexpr int kEBits = 11;        // bits of a staged element index (E <= 2^11)

__device__ __forceinline__ double load_prob(const void *p, int64_t i, int f32) {
  return f32 ? (double)static_cast<const float *>(p)[i] : static_cast<const double *>(p)[i];
}

// One subcircuit's parameters for the staged kernel, flattened by the host so
// that a work-group reads each one directly (no table lookups in chains).
// Entries past n_in, n_out and d are zero, so loops run to the fixed bounds
// without guards and their reads are issued together.
struct AttrJob {
  const void *var;
  void *out;
  double scale;
  int in_f32, out_f32;
  int w, d, c, n_in, n_out, xt_bits;
  int vec8;                 // a thread's 8 entries are consecutive in memory
  int out_merged;           // output [4^c][2^d] (see AttrArgs)
  int in_lab[kMaxIn];       // label bit position in sigma of in-cut j
  int out_place[kMaxOut];   // variant place value of out-cut j's basis
  int out_lab[kMaxOut];     // label bit position in sigma of out-cut j
  // variant offset added by bit i of a staged element index e: an outcome
  // bit, a tile bit or a bit of a preparation digit (with its place value)
  int64_t edelta[kEBits];
  uint32_t tile_nib[8][16]; // state bits of x-tile index bits 4q..4q+3
};
static_assert(sizeof(AttrJob) * kAttrJobs + 64 <= 4096, "attribution batch exceeds the kernel argument space");

// Padded LDS position of staged element e (one pad per 32): the passes over
// consecutive elements and the output reads at a stride of 32 elements then
// fall on distinct banks.
__device__ __forceinline__ int phys(int e) { return e + (e >> 5); }

// Bytes of dynamic LDS a work-group uses.
size_t attribute_lds_bytes(int xt_bits, int n_in, int n_out) {
  const size_t E = (size_t(1) << (2 * n_in)) << (n_out + xt_bits);
  const size_t NS = size_t(1) << (2 * n_in), NB = size_t(1) << n_out;
  return (E + (E >> 5)) * 8 + NS * 4 + 2 * NB * 4;
}

// One work-group = (basis combination beta, tile of XT consecutive data
// states); staged element e = (s XT + xt) NB + b.  Thread t owns elements
// [8t, 8t + 8): it computes their variant offsets directly and issues the
// loads first, builds the label tables while they are in flight, applies the
// maps of out-cuts 0..2 (bits 0..2 of e) in registers, and stages the result;
// the remaining out-cuts and the in-cuts take one LDS pass each.  LDS is sized
// to the subcircuit (dynamic), so small stages leave room for many
// work-groups per CU.
template <bool IN_F32, bool OUT_F32, bool VEC8>
__device__ __forceinline__ void attribute_lds_body(const AttrJob &a, int blk, unsigned char *dyn) {
  const int tid = threadIdx.x;
  const int XT = 1 << a.xt_bits;
  const int NB = 1 << a.n_out;
  const int NS = 1 << (2 * a.n_in);
  const int E = NS * XT * NB;
  double *buf = reinterpret_cast<double *>(dyn);                      // [phys(E)]
  uint32_t *sinl = reinterpret_cast<uint32_t *>(buf + E + (E >> 5));  // [NS] label bits of s
  uint32_t *sout = sinl + NS;                                         // [NV] label bits of slot v
  uint32_t *slot = sout + NB;                                         // [NV] its outcome bits
  const int lnxt = a.d - a.xt_bits;
  const int bidx = blk >> lnxt;
  // tile of data states: in the merged layout a label's tiles are adjacent
  // in memory, so the tiles of eight consecutive work-groups (the eight XCDs
  // take work-groups in turn) are spread: XCD k writes tiles k n/8 .. (k + 1)
  // n/8 - 1 of each label, and its partial lines meet in its own L2
  int xtile = blk & ((1 << lnxt) - 1);
  if (a.out_merged && lnxt >= 3) xtile = ((xtile & 7) << (lnxt - 3)) | (xtile >> 3);
  const int64_t x0 = int64_t(xtile) << a.xt_bits;

  // basis digits of this work-group: out-cut j measured in basis dig[j]
  // (Z = 0, X = 1, Y = 2)
  int dig[kMaxOut];  // 0 past n_out (bidx < 3^n_out)
  int zmask = 0, vbeta = 0;
  {
    // digits past the fourth only when there are more out-cuts (a uniform
    // branch: most subcircuits have few)
    int rem = bidx;
#pragma unroll
    for (int j = 0; j < kMaxOut; ++j) dig[j] = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      dig[j] = rem % 3;
      rem /= 3;
    }
    if (a.n_out > 4) {
#pragma unroll
      for (int j = 4; j < kMaxOut; ++j) {
        dig[j] = rem % 3;
        rem /= 3;
      }
    }
#pragma unroll
    for (int j = 0; j < kMaxOut; ++j) {
      vbeta += dig[j] * a.out_place[j];
      zmask |= (dig[j] == 0 ? 1 : 0) << j;
    }
    zmask &= (1 << a.n_out) - 1;
  }
  uint32_t base = 0;  // state bits of the tile's fixed data bits
  {
    const uint32_t xi = (uint32_t)(x0 >> a.xt_bits);
#pragma unroll
    for (int q = 0; q < 8; ++q) base |= a.tile_nib[q][(xi >> (4 * q)) & 15];
  }

  // the thread's variant entries, loads in flight together
  const int e0 = tid * kPer;
  const bool mine = e0 < E;
  typename std::conditional<IN_F32, float, double>::type raw[kPer];
  {
    int64_t off0 = ((int64_t)vbeta << a.w) + base;
#pragma unroll
    for (int i = 3; i < kEBits; ++i)
      if ((e0 >> i) & 1) off0 += a.edelta[i];
    // (converted where first used, so that the loads stay in flight while
    // the label tables are built)
    typedef typename std::conditional<IN_F32, float, double>::type I;
    const I *in = static_cast<const I *>(a.var);
    if constexpr (VEC8) {
      // 16-byte loads (the entries of outcome bits 0..2 are adjacent)
      typedef typename std::conditional<IN_F32, float4, double2>::type V;
      constexpr int per = sizeof(V) / sizeof(I);
      const V *pv = reinterpret_cast<const V *>(in + (mine ? off0 : 0));
      V x[kPer / per];
#pragma unroll
      for (int u = 0; u < kPer / per; ++u) x[u] = pv[u];
#pragma unroll
      for (int u = 0; u < kPer / per; ++u) {
        if constexpr (IN_F32) {
          raw[4 * u] = x[u].x;
          raw[4 * u + 1] = x[u].y;
          raw[4 * u + 2] = x[u].z;
          raw[4 * u + 3] = x[u].w;
        } else {
          raw[2 * u] = x[u].x;
          raw[2 * u + 1] = x[u].y;
        }
      }
    } else {
      int64_t off[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k)
        off[k] = (mine && e0 + k < E)
                     ? off0 + ((k & 1) ? a.edelta[0] : 0) + ((k & 2) ? a.edelta[1] : 0) + ((k & 4) ? a.edelta[2] : 0)
                     : 0;
#pragma unroll
      for (int k = 0; k < kPer; ++k) raw[k] = in[off[k]];
    }
  }

  // label tables for the output
  for (int t = tid; t < NS; t += kThreads) {
    uint32_t sg = 0;
#pragma unroll
    for (int j = 0; j < kMaxIn; ++j) sg |= uint32_t((t >> (2 * j)) & 3) << a.in_lab[j];
    sinl[t] = sg;
  }
  const int nz = __builtin_popcount(zmask);
  const int NV = 1 << nz;  // a Z-basis cut carries both I and Z
  for (int t = tid; t < NV; t += kThreads) {
    uint32_t sg = 0, sl = 0;
    int zb = 0;
    // (past n_out: digit 0 and bit (t >> zb) & 1 = 0 as t < 2^nz, so
    // nothing is added)
#pragma unroll
    for (int j = 0; j < kMaxOut; ++j) {
      int lab = dig[j];  // X = 1, Y = 2 coincide with the basis digits
      if (lab == 0) {
        const int bit = (t >> zb) & 1;
        ++zb;
        lab = bit ? 3 : 0;  // slot bit 0 holds I, bit 1 holds Z
        sl |= uint32_t(bit) << j;
      }
      sg |= uint32_t(lab) << a.out_lab[j];
    }
    sout[t] = sg;
    slot[t] = sl;
  }

  // out-cuts 0..2 in registers: pair (b_j = 0, b_j = 1) -> slot 0 / 1
  if (mine) {
    double v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) v[k] = (double)raw[k];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (i < a.n_out) {
        if ((zmask >> i) & 1) {
#pragma unroll
          for (int k = 0; k < kPer; ++k)
            if (!((k >> i) & 1)) {
              const double q0 = v[k], q1 = v[k | (1 << i)];
              v[k] = q0 + q1;
              v[k | (1 << i)] = q0 - q1;
            }
        } else {
#pragma unroll
          for (int k = 0; k < kPer; ++k)
            if (!((k >> i) & 1)) {
              v[k] -= v[k | (1 << i)];
              v[k | (1 << i)] = 0.0;
            }
        }
      }
    }
    const int p0 = phys(e0);  // the thread's 8 elements share one pad
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if (e0 + k < E) buf[p0 + k] = v[k];
  }
  __syncthreads();

  // out-cuts 3.. : one LDS pass each; a thread's pairs of one pass are read
  // together, then written
  for (int j = 3; j < a.n_out; ++j) {
    const bool zb = (zmask >> j) & 1;
    for (int p0 = 0; p0 < E / 2; p0 += 4 * kThreads) {
      double q0[4], q1[4];
      int e1[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p = p0 + u * kThreads + tid;
        e1[u] = p < E / 2 ? ((p >> j) << (j + 1)) | (p & ((1 << j) - 1)) : -1;
        q0[u] = e1[u] >= 0 ? buf[phys(e1[u])] : 0.0;
        q1[u] = e1[u] >= 0 ? buf[phys(e1[u] | (1 << j))] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e1[u] >= 0) {
          buf[phys(e1[u])] = zb ? q0[u] + q1[u] : q0[u] - q1[u];
          buf[phys(e1[u] | (1 << j))] = zb ? q0[u] - q1[u] : 0.0;
        }
    }
    __syncthreads();
  }
  // in-cut maps: digit j of s, 4 entries -> labels I, X, Y, Z.  Two digits
  // per LDS pass while two are left (a thread maps the 16 entries of one
  // block of digits j and j + 1 in registers).
  auto map4 = [](double &p0, double &p1, double &p2, double &p3) {
    const double s01 = p0 + p1;
    const double z = p0 - p1;
    p0 = s01;
    p1 = 2.0 * p2 - s01;
    p2 = 2.0 * p3 - s01;
    p3 = z;
  };
  int jd = 0;
  for (; jd + 1 < a.n_in; jd += 2) {
    const int sh = 2 * jd + a.xt_bits + a.n_out;
    const int st = 1 << sh;  // digit jd at stride st, digit jd + 1 at 4 st
    for (int p = tid; p < E / 16; p += kThreads) {
      const int e1 = ((p >> sh) << (sh + 4)) | (p & (st - 1));
      double q[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) q[r] = buf[phys(e1 + (r & 3) * st + (r >> 2) * 4 * st)];
#pragma unroll
      for (int r1 = 0; r1 < 4; ++r1) map4(q[4 * r1], q[4 * r1 + 1], q[4 * r1 + 2], q[4 * r1 + 3]);
#pragma unroll
      for (int r0 = 0; r0 < 4; ++r0) map4(q[r0], q[r0 + 4], q[r0 + 8], q[r0 + 12]);
#pragma unroll
      for (int r = 0; r < 16; ++r) buf[phys(e1 + (r & 3) * st + (r >> 2) * 4 * st)] = q[r];
    }
    __syncthreads();
  }
  // an odd last digit is applied by the output loop, which reads the two or
  // three entries each label needs (one LDS pass fewer)
  const bool lazy = jd < a.n_in;
  const int lsh = 2 * jd;
  const int lst = 1 << (2 * jd + a.xt_bits + a.n_out);

  // every label assignment compatible with beta: q = (xt, v, s), s fastest
  // ([2^d][4^c]: consecutive threads write consecutive labels), or
  // q = (v, s, xt), xt fastest, in the merged layout
  const int lNS = 2 * a.n_in;
  const int64_t L = int64_t(1) << (2 * a.c);
  const int nq = (XT * NV) << lNS;
  for (int q = tid; q < nq; q += kThreads) {
    int sdx, vv, xt;
    if (a.out_merged) {
      xt = q & (XT - 1);
      const int rest = q >> a.xt_bits;
      sdx = rest & (NS - 1);
      vv = rest >> lNS;
    } else {
      sdx = q & (NS - 1);
      const int rest = q >> lNS;
      vv = rest & (NV - 1);
      xt = rest >> nz;
    }
    const int eo = (sdx * XT + xt) * NB + slot[vv];
    double val;
    if (lazy) {
      const int dl = (sdx >> lsh) & 3;  // label digit of the last in-cut
      const int eb = eo - dl * lst;
      const double p0 = buf[phys(eb)], p1 = buf[phys(eb + lst)];
      const double pk = buf[phys(eb + (dl == 2 ? 3 : 2) * lst)];  // |+> for X, |+i> for Y
      const double s01 = p0 + p1;
      val = dl == 0 ? s01 : (dl == 3 ? p0 - p1 : 2.0 * pk - s01);
    } else {
      val = buf[phys(eo)];
    }
    val *= a.scale;
    const int64_t lab = (int64_t)(sinl[sdx] | sout[vv]);
    const int64_t o = a.out_merged ? (lab << a.d) + (x0 + xt) : (x0 + xt) * L + lab;
    // the merged layout's runs per work-group are short (XT states), so its
    // stores go through L2, where neighbouring work-groups' runs meet
    if constexpr (OUT_F32) {
      if (a.out_merged) static_cast<float *>(a.out)[o] = (float)val;
      else __builtin_nontemporal_store((float)val, static_cast<float *>(a.out) + o);
    } else {
      static_cast<double *>(a.out)[o] = val;
    }
  }
}

// Several subcircuits in one launch: work-group w belongs to the job j with
// start[j] <= w < start[j + 1]; dynamic LDS is the largest job's.
struct AttrBatch {
  int n;
  int start[kAttrJobs + 1];
  AttrJob job[kAttrJobs];
};

// Input and output precisions and the load form are template parameters (one
// combination per launch): no branch between a load and its use.
template <bool IN_F32, bool OUT_F32, bool VEC8>
__global__ __launch_bounds__(kThreads) void attribute_lds(AttrBatch b) {
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
  int j = 0;
#pragma unroll
  for (int q = 1; q < kAttrJobs; ++q) j += (q < b.n && (int)blockIdx.x >= b.start[q]) ? 1 : 0;
  attribute_lds_body<IN_F32, OUT_F32, VEC8>(b.job[j], (int)blockIdx.x - b.start[j], dyn);
}

// The vector-load form serves a batch whose jobs all allow it; the other form
// serves any job.
template <bool IN_F32, bool OUT_F32>
void launch_lds(const AttrBatch &b, size_t lds, hipStream_t s) {
  const dim3 grid((unsigned)b.start[b.n]), block(kThreads);
  bool vec8 = true;
  for (int j = 0; j < b.n; ++j) vec8 = vec8 && b.job[j].vec8;
  if (vec8) hipLaunchKernelGGL((attribute_lds<IN_F32, OUT_F32, true>), grid, block, lds, s, b);
  else hipLaunchKernelGGL((attribute_lds<IN_F32, OUT_F32, false>), grid, block, lds, s, b);
}

// The staged kernel's flattened parameters of a subcircuit.
AttrJob attr_job(const AttrArgs &a) {
  AttrJob J{};
  J.var = a.var;
  J.out = a.out;
  J.scale = a.scale;
  J.in_f32 = a.in_f32;
  J.out_f32 = a.out_f32;
  J.out_merged = a.out_merged;
  J.w = a.w;
  J.d = a.d;
  J.c = a.c;
  J.n_in = a.n_in;
  J.n_out = a.n_out;
  J.xt_bits = a.xt_bits;
  for (int j = 0; j < a.n_in; ++j) J.in_lab[j] = 2 * a.in_pos[j];
  for (int j = 0; j < a.n_out; ++j) {
    J.out_place[j] = (int)a.place[a.out_pos[j]];
    J.out_lab[j] = 2 * a.out_pos[j];
  }
  // e = (s XT + xt) NB + b: bit i of e is outcome bit i, then tile bit
  // i - n_out, then bit i' of s (digit i' / 2, weight 1 or 2)
  for (int i = 0; i < kEBits; ++i) {
    if (i < a.n_out) {
      J.edelta[i] = int64_t(1) << a.out_wire[i];
    } else if (i < a.n_out + a.xt_bits) {
      J.edelta[i] = int64_t(1) << a.data_wire[i - a.n_out];
    } else {
      const int sb = i - a.n_out - a.xt_bits;
      J.edelta[i] = sb < 2 * a.n_in ? (a.place[a.in_pos[sb >> 1]] * ((sb & 1) + 1)) << a.w : 0;
    }
  }
  J.vec8 = J.edelta[0] == 1 && J.edelta[1] == 2 && J.edelta[2] == 4 &&
           reinterpret_cast<uintptr_t>(a.var) % 16 == 0;
  // data bits xt_bits + 4q + r of the tile index, nibble by nibble
  for (int q = 0; q < 8; ++q)
    for (int v = 0; v < 16; ++v) {
      uint32_t o = 0;
      for (int r = 0; r < 4; ++r) {
        const int j = a.xt_bits + 4 * q + r;
        if (((v >> r) & 1) && j < a.d) o |= 1u << a.data_wire[j];
      }
      J.tile_nib[q][v] = o;
    }
  return J;
}

// Direct evaluation for subcircuits whose per-state slice does not fit the LDS
// stage: one thread per output element, reading the variants from memory.
__global__ __launch_bounds__(kThreads) void attribute_direct(AttrArgs a) {
  const int64_t L = int64_t(1) << (2 * a.c);
  const int64_t total = (int64_t(1) << a.d) * L;
  const int64_t row = int64_t(1) << a.w;
  const double C[4][4] = {{1, 1, 0, 0}, {-1, -1, 2, 0}, {-1, -1, 0, 2}, {1, -1, 0, 0}};
  for (int64_t o = int64_t(blockIdx.x) * kThreads + threadIdx.x; o < total;
       o += int64_t(gridDim.x) * kThreads) {
    // o runs over the output layout: [2^d][4^c], or [4^c][2^d] when merged
    const int64_t x = a.out_merged ? o & ((int64_t(1) << a.d) - 1) : o >> (2 * a.c);
    const int64_t sigma = a.out_merged ? o >> a.d : o & (L - 1);
    int64_t xo = 0;
    for (int j = 0; j < a.d; ++j)
      if ((x >> j) & 1) xo |= int64_t(1) << a.data_wire[j];
    int64_t vb = 0;
    int labo[kMaxIncident], labi[kMaxIncident];
    for (int j = 0; j < a.n_out; ++j) {
      int lab = (sigma >> (2 * a.out_pos[j])) & 3;
      labo[j] = lab;
      int basis = lab == 3 ? 0 : lab;
      vb += int64_t(basis) * a.place[a.out_pos[j]];
    }
    for (int j = 0; j < a.n_in; ++j) labi[j] = (sigma >> (2 * a.in_pos[j])) & 3;
    double acc = 0.0;
    const int NSm = 1 << (2 * a.n_in);
    for (int s = 0; s < NSm; ++s) {
      double cf = 1.0;
      int64_t v = vb;
      for (int j = 0; j < a.n_in && cf != 0.0; ++j) {
        int sj = (s >> (2 * j)) & 3;
        cf *= C[labi[j]][sj];
        v += int64_t(sj) * a.place[a.in_pos[j]];
      }
      if (cf == 0.0) continue;
      for (int b = 0; b < (1 << a.n_out); ++b) {
        int64_t oo = xo;
        double g = 1.0;
        for (int j = 0; j < a.n_out; ++j) {
          int bj = (b >> j) & 1;
          if (bj) oo |= int64_t(1) << a.out_wire[j];
          if (bj && labo[j] != 0) g = -g;
        }
        acc += cf * g * load_prob(a.var, v * row + oo, a.in_f32);
      }
    }
    double v = acc * a.scale;
    if (a.out_f32) static_cast<float *>(a.out)[o] = (float)v;
    else static_cast<double *>(a.out)[o] = v;
  }
}

}  // namespace

void launch_attributes(const AttrArgs *jobs, int n, hipStream_t s) {
  AttrBatch b{};
  size_t lds = 0;
  auto flush = [&]() {
    if (!b.n) return;
    const int fi = b.job[0].in_f32, fo = b.job[0].out_f32;
    if (fi && fo) launch_lds<true, true>(b, lds, s);
    else if (fi) launch_lds<true, false>(b, lds, s);
    else if (fo) launch_lds<false, true>(b, lds, s);
    else launch_lds<false, false>(b, lds, s);
    b = AttrBatch{};
    lds = 0;
  };
  for (int i = 0; i < n; ++i) {
    AttrArgs a = jobs[i];
    const int64_t per_x = (int64_t(1) << (2 * a.n_in)) << a.n_out;
    const int64_t ns = int64_t(1) << (2 * a.n_in);
    if (per_x <= kLdsElems && ns <= kMaxNS && (int64_t(1) << a.n_out) <= kMaxNB) {
      // x-tile: as many data states as fill the stage, then halved while that
      // gives too few work-groups to fill the device and keeps >= 256 entries
      int xb = 0;
      while ((per_x << (xb + 1)) <= kLdsElems && xb + 1 <= a.d) ++xb;
      int64_t nbeta = 1;
      for (int j = 0; j < a.n_out; ++j) nbeta *= 3;
      // (not below the 8 entries a thread takes when they are outcome and
      // tile bits, so that they stay adjacent in memory)
      const int xb_min = std::min(std::max(0, 3 - a.n_out), xb);
      while (xb > xb_min && (nbeta << (a.d - xb)) < 1024 && (per_x << (xb - 1)) >= 256) --xb;
      a.xt_bits = xb;
      const int64_t blocks = nbeta << (a.d - xb);
      // one launch holds jobs of one input and one output precision
      const AttrJob J = attr_job(a);
      if (b.n == kAttrJobs || b.start[b.n] + blocks > (int64_t(1) << 31) - 1 ||
          (b.n && (b.job[0].in_f32 != J.in_f32 || b.job[0].out_f32 != J.out_f32)))
        flush();
      b.job[b.n] = J;
      b.start[b.n + 1] = (int)(b.start[b.n] + blocks);
      ++b.n;
      lds = std::max(lds, attribute_lds_bytes(xb, a.n_in, a.n_out));
    } else {
      int64_t total = (int64_t(1) << a.d) << (2 * a.c);
      int64_t blocks = (total + kThreads - 1) / kThreads;
      if (blocks > 65536) blocks = 65536;
      hipLaunchKernelGGL(attribute_direct, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
    }
  }
  flush();
}

}  // namespace sqc
