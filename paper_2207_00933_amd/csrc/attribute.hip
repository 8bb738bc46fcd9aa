// Cut-basis attribution (Sec. 2.1, Eq. 1, Fig. 1): variant probabilities of
// one subcircuit -> entries T[x][sigma] for every I/X/Y/Z label assignment
// sigma of its cuts, with the factor 1/2 per out-cut folded in.  FP64.
//
// Structure: the map from (preparation s, basis beta, outcome b) to sigma is a
// tensor product of one small map per cut.  A work item is one combination of
// measurement bases beta (a label Z, X or Y per out-cut) and a tile of XT
// consecutive data states.  Its entries p[(s, beta)][x, b] for all
// preparations s and out-cut outcomes b are staged in LDS, the per-cut maps
// are applied in place, one pass per cut, and every label assignment
// compatible with beta is written (beta(I) = beta(Z) = Z, so a Z basis serves
// I and Z).  The code is kept in loops: a kernel's first pass over
// straight-line code is bound by instruction fetch.
//
//   in-cut  (digit of s -> digit of sigma):  I = p0 + p1,  Z = p0 - p1,
//            X = 2 p+ - p0 - p1,  Y = 2 p+i - p0 - p1
//   out-cut (bit b -> digit of sigma):       I = q0 + q1 (Z basis),
//            Z|X|Y = q0 - q1 (in that basis)
#include "common.hpp"

#include <algorithm>

namespace sqc {

namespace {

constexpr int kThreads = 256;
constexpr int kLdsElems = 2048;   // doubles staged per work-group
constexpr int kPer = kLdsElems / kThreads;
constexpr int kMaxNS = 1024;
constexpr int kMaxNB = 1024;

__device__ __forceinline__ double load_prob(const void *p, int64_t i, int f32) {
  return f32 ? (double)static_cast<const float *>(p)[i] : static_cast<const double *>(p)[i];
}

// Bytes of dynamic LDS a work-group uses.
size_t attribute_lds_bytes(int xt_bits, int n_in, int n_out) {
  const size_t E = (size_t(1) << (2 * n_in)) << (n_out + xt_bits);
  const size_t NS = size_t(1) << (2 * n_in), NB = size_t(1) << n_out, XT = size_t(1) << xt_bits;
  return E * 8 + NS * 8 + NS * 4 + 3 * NB * 4 + XT * 4;
}

// One work-group = (basis combination beta, tile of XT consecutive data
// states).  The threads first tabulate the offsets and label bits of the
// preparations, outcome bits and tile states (one entry each), then issue all
// variant loads at once.  LDS is sized to the subcircuit (dynamic), so small
// stages leave room for many work-groups per CU.
__device__ __forceinline__ void attribute_lds_body(const AttrArgs &a, int blk, unsigned char *dyn) {
  const int tid = threadIdx.x;
  const int XT = 1 << a.xt_bits;
  const int NB = 1 << a.n_out;
  const int NS = 1 << (2 * a.n_in);
  const int E = NS * XT * NB;
  double *buf = reinterpret_cast<double *>(dyn);            // [E]
  int64_t *vin = reinterpret_cast<int64_t *>(buf + E);      // [NS] variant index of the in-cut digits of s
  uint32_t *sinl = reinterpret_cast<uint32_t *>(vin + NS);  // [NS] their label bits
  uint32_t *boff = sinl + NS;                               // [NB] wire offset of outcome bits b
  uint32_t *sout = boff + NB;                               // [NV] label bits of valid out-cut slot v
  uint32_t *slot = sout + NB;                               // [NV] its outcome bits
  uint32_t *xoff = slot + NB;                               // [XT] wire offset of tile state xt
  const int lnxt = a.d - a.xt_bits;
  const int bidx = blk >> lnxt;
  const int64_t x0 = int64_t(blk & ((1 << lnxt) - 1)) << a.xt_bits;

  // basis digits of this work-group
  int zmask = 0;  // bit j: out-cut j measured in the Z basis
  int64_t vbeta = 0;
  {
    int rem = bidx;
    for (int j = 0; j < a.n_out; ++j) {
      const int bj = rem % 3;
      rem /= 3;
      vbeta += int64_t(bj) * a.place[a.out_pos[j]];
      zmask |= (bj == 0 ? 1 : 0) << j;
    }
  }
  const int nz = __builtin_popcount(zmask);
  const int NV = 1 << nz;  // a Z-basis cut carries both I and Z
  int64_t base = 0;
  for (int j = a.xt_bits; j < a.d; ++j)
    if ((x0 >> j) & 1) base |= int64_t(1) << a.data_wire[j];
  for (int t = tid; t < NS; t += kThreads) {
    int64_t vr = 0;
    uint32_t sg = 0;
    for (int j = 0; j < a.n_in; ++j) {
      const int dgt = (t >> (2 * j)) & 3;
      vr += int64_t(dgt) * a.place[a.in_pos[j]];
      sg |= uint32_t(dgt) << (2 * a.in_pos[j]);
    }
    vin[t] = vr;
    sinl[t] = sg;
  }
  for (int t = tid; t < NB; t += kThreads) {
    uint32_t o = 0;
    for (int j = 0; j < a.n_out; ++j)
      if ((t >> j) & 1) o |= uint32_t(1) << a.out_wire[j];
    boff[t] = o;
  }
  for (int t = tid; t < XT; t += kThreads) {
    uint32_t o = 0;
    for (int j = 0; j < a.xt_bits; ++j)
      if ((t >> j) & 1) o |= uint32_t(1) << a.data_wire[j];
    xoff[t] = o;
  }
  for (int t = tid; t < NV; t += kThreads) {
    uint32_t sg = 0, sl = 0;
    int zb = 0, rem = bidx;
    for (int j = 0; j < a.n_out; ++j) {
      const int bj = rem % 3;  // basis digit j
      rem /= 3;
      int lab = bj;            // X = 1, Y = 2 coincide with the basis digits
      if (bj == 0) {
        const int bit = (t >> zb) & 1;
        ++zb;
        lab = bit ? 3 : 0;  // slot bit 0 holds I, bit 1 holds Z
        sl |= uint32_t(bit) << j;
      }
      sg |= uint32_t(lab) << (2 * a.out_pos[j]);
    }
    sout[t] = sg;
    slot[t] = sl;
  }
  __syncthreads();

  // stage: element e = (s XT + xt) NB + b; all loads in flight together
  {
    int64_t off[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = tid + k * kThreads;
      const int b = e & (NB - 1);
      const int xt = (e >> a.n_out) & (XT - 1);
      const int sdx = (e >> (a.n_out + a.xt_bits)) & (NS - 1);
      off[k] = e < E ? ((vbeta + vin[sdx]) << a.w) + base + (int64_t)(xoff[xt] | boff[b]) : 0;
    }
    double v[kPer];
    if (a.in_f32) {
      const float *in = static_cast<const float *>(a.var);
#pragma unroll
      for (int k = 0; k < kPer; ++k) v[k] = (double)in[off[k]];
    } else {
      const double *in = static_cast<const double *>(a.var);
#pragma unroll
      for (int k = 0; k < kPer; ++k) v[k] = in[off[k]];
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if (tid + k * kThreads < E) buf[tid + k * kThreads] = v[k];
  }
  __syncthreads();

  // out-cut maps: pair (b_j = 0, b_j = 1) -> slot 0 / 1.  A thread's pairs
  // of one pass are read together, then written (one LDS round trip).
  for (int j = 0; j < a.n_out; ++j) {
    const bool zb = (zmask >> j) & 1;
    for (int p0 = 0; p0 < E / 2; p0 += 4 * kThreads) {
      double q0[4], q1[4];
      int e0[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p = p0 + u * kThreads + tid;
        e0[u] = p < E / 2 ? ((p >> j) << (j + 1)) | (p & ((1 << j) - 1)) : -1;
        q0[u] = e0[u] >= 0 ? buf[e0[u]] : 0.0;
        q1[u] = e0[u] >= 0 ? buf[e0[u] | (1 << j)] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0[u] >= 0) {
          buf[e0[u]] = zb ? q0[u] + q1[u] : q0[u] - q1[u];
          buf[e0[u] | (1 << j)] = zb ? q0[u] - q1[u] : 0.0;
        }
    }
    __syncthreads();
  }
  // in-cut maps: digit j of s, 4 entries -> labels I, X, Y, Z
  for (int j = 0; j < a.n_in; ++j) {
    const int sh = 2 * j + a.xt_bits + a.n_out;
    const int st = 1 << sh;
    for (int p0 = 0; p0 < E / 4; p0 += 2 * kThreads) {
      double q[2][4];
      int e0[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int p = p0 + u * kThreads + tid;
        e0[u] = p < E / 4 ? ((p >> sh) << (sh + 2)) | (p & (st - 1)) : -1;
#pragma unroll
        for (int r = 0; r < 4; ++r) q[u][r] = e0[u] >= 0 ? buf[e0[u] + r * st] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
        if (e0[u] >= 0) {
          const double s01 = q[u][0] + q[u][1];
          buf[e0[u]] = s01;
          buf[e0[u] + st] = 2.0 * q[u][2] - s01;
          buf[e0[u] + 2 * st] = 2.0 * q[u][3] - s01;
          buf[e0[u] + 3 * st] = q[u][0] - q[u][1];
        }
    }
    __syncthreads();
  }

  // every label assignment compatible with beta: q = (xt, v, s), s fastest
  const int lNS = 2 * a.n_in;
  const int64_t L = int64_t(1) << (2 * a.c);
  const int nq = (XT * NV) << lNS;
  for (int q = tid; q < nq; q += kThreads) {
    const int sdx = q & (NS - 1);
    const int rest = q >> lNS;
    const int vv = rest & (NV - 1);
    const int xt = rest >> nz;
    const double val = buf[(sdx * XT + xt) * NB + slot[vv]] * a.scale;
    const int64_t o = (x0 + xt) * L + (sinl[sdx] | sout[vv]);
    if (a.out_f32) static_cast<float *>(a.out)[o] = (float)val;
    else static_cast<double *>(a.out)[o] = val;
  }
}

// Several subcircuits in one launch: work-group w belongs to the job j with
// start[j] <= w < start[j + 1]; dynamic LDS is the largest job's.
struct AttrBatch {
  int n;
  int start[kAttrJobs + 1];
  AttrArgs job[kAttrJobs];
};

__global__ __launch_bounds__(kThreads) void attribute_lds(AttrBatch b) {
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
  int j = 0;
  while (j + 1 < b.n && (int)blockIdx.x >= b.start[j + 1]) ++j;
  attribute_lds_body(b.job[j], (int)blockIdx.x - b.start[j], dyn);
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
    int64_t x = o >> (2 * a.c);
    int64_t sigma = o & (L - 1);
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
    hipLaunchKernelGGL(attribute_lds, dim3((unsigned)b.start[b.n]), dim3(kThreads), lds, s, b);
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
      while (xb > 0 && (nbeta << (a.d - xb)) < 1024 && (per_x << (xb - 1)) >= 256) --xb;
      a.xt_bits = xb;
      const int64_t blocks = nbeta << (a.d - xb);
      if (b.n == kAttrJobs || b.start[b.n] + blocks > (int64_t(1) << 31) - 1) flush();
      b.job[b.n] = a;
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
