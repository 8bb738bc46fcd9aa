// Cut-basis attribution (Sec. 2.1, Eq. 1, Fig. 1): variant probabilities of
// one subcircuit -> entries T[x][sigma] for every I/X/Y/Z label assignment
// sigma of its cuts, with the factor 1/2 per out-cut folded in.  FP64.
//
// Structure: the map from (preparation s, basis beta, outcome b) to sigma is a
// tensor product of one small map per cut.  A work-group owns one combination
// of measurement bases beta (a label Z, X or Y per out-cut) and a tile of XT
// consecutive data states.  It stages p[(s, beta)][x, b] for all
// preparations s and out-cut outcomes b of its tile in LDS, applies the
// per-cut maps in place, one pass per cut, and writes every label assignment
// compatible with beta (beta(I) = beta(Z) = Z, so a Z basis serves I and Z).
//
//   in-cut  (digit of s -> digit of sigma):  I = p0 + p1,  Z = p0 - p1,
//            X = 2 p+ - p0 - p1,  Y = 2 p+i - p0 - p1
//   out-cut (bit b -> digit of sigma):       I = q0 + q1 (Z basis),
//            Z|X|Y = q0 - q1 (in that basis)
#include "common.hpp"

namespace sqc {

namespace {

constexpr int kThreads = 256;
constexpr int kLdsElems = 2048;  // doubles staged per work-group
constexpr int kMaxNS = 1024;     // preparation patterns a work-group tabulates
constexpr int kMaxNB = 1024;     // out-cut outcome patterns

__device__ __forceinline__ double load_prob(const void *p, int64_t i, int f32) {
  return f32 ? (double)static_cast<const float *>(p)[i] : static_cast<const double *>(p)[i];
}

__global__ __launch_bounds__(kThreads) void attribute_lds(AttrArgs a) {
  __shared__ double buf[kLdsElems];
  // per work-group tables (NS * XT * NB <= kLdsElems, NS <= kMaxNS, NB <= kMaxNB):
  //   vtab[s]   variant row offset of preparation index s (with this beta)
  //   xoff[xt]  outcome offset of tile entry xt;  boff[b] of out-cut bits b
  //   sin[s]    label index contributed by the in-cut digits of s
  //   sout[v]   label index of valid out-cut slot v;  slot[v] its bit pattern
  __shared__ uint32_t tab[kLdsElems + 2 * kMaxNB + 64];
  __shared__ int64_t vtab[kMaxNS];
  const int tid = threadIdx.x;
  const int XT = 1 << a.xt_bits;
  const int NB = 1 << a.n_out;
  const int NS = 1 << (2 * a.n_in);
  const int E = NS * XT * NB;
  const int64_t x0 = int64_t(blockIdx.x) << a.xt_bits;

  // basis digits of this work-group and the fixed part of the variant index
  int beta[kMaxIncident];
  int64_t vbeta = 0;
  int nz = 0;
  {
    int rem = blockIdx.y;
    for (int j = 0; j < a.n_out; ++j) {
      beta[j] = rem % 3;
      rem /= 3;
      vbeta += int64_t(beta[j]) * a.place[a.out_pos[j]];
      nz += beta[j] == 0 ? 1 : 0;
    }
  }
  const int NV = 1 << nz;  // valid out-cut slots: a Z-basis cut carries I and Z
  uint32_t *xoff = tab;
  uint32_t *boff = xoff + XT;
  uint32_t *sin = boff + NB;
  uint32_t *sout = sin + NS;
  uint32_t *slot = sout + NV;
  int64_t base = 0;
  for (int j = 0; j < a.d; ++j)
    if ((x0 >> j) & 1) base |= int64_t(1) << a.data_wire[j];
  for (int t = tid; t < XT; t += kThreads) {
    uint32_t o = 0;
    for (int j = 0; j < a.xt_bits; ++j)
      if ((t >> j) & 1) o |= uint32_t(1) << a.data_wire[j];
    xoff[t] = o;
  }
  for (int t = tid; t < NB; t += kThreads) {
    uint32_t o = 0;
    for (int j = 0; j < a.n_out; ++j)
      if ((t >> j) & 1) o |= uint32_t(1) << a.out_wire[j];
    boff[t] = o;
  }
  for (int t = tid; t < NS; t += kThreads) {
    int64_t v = vbeta;
    uint32_t sg = 0;
    for (int j = 0; j < a.n_in; ++j) {
      const int dgt = (t >> (2 * j)) & 3;
      v += int64_t(dgt) * a.place[a.in_pos[j]];
      sg |= uint32_t(dgt) << (2 * a.in_pos[j]);
    }
    vtab[t] = (v << a.w) + base;
    sin[t] = sg;
  }
  for (int t = tid; t < NV; t += kThreads) {
    uint32_t sg = 0, sl = 0;
    int zb = 0;
    for (int j = 0; j < a.n_out; ++j) {
      int lab;
      if (beta[j] == 0) {
        const int bit = (t >> zb) & 1;
        ++zb;
        lab = bit ? 3 : 0;  // slot bit 0 holds I, bit 1 holds Z
        sl |= uint32_t(bit) << j;
      } else {
        lab = beta[j];  // X = 1, Y = 2 coincide with the basis digits
      }
      sg |= uint32_t(lab) << (2 * a.out_pos[j]);
    }
    sout[t] = sg;
    slot[t] = sl;
  }
  __syncthreads();

  // stage: element e = (s * XT + xt) * NB + b; all of a thread's loads are
  // issued before the first is used (clamped offsets, no branches)
  {
    constexpr int kPer = kLdsElems / kThreads;
    int64_t off[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = tid + k * kThreads;
      const int b = e & (NB - 1);
      const int xt = (e >> a.n_out) & (XT - 1);
      const int s = (e >> (a.n_out + a.xt_bits)) & (NS - 1);
      off[k] = e < E ? vtab[s] + (int64_t)(xoff[xt] | boff[b]) : 0;
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

  // out-cut maps: pair (b_j = 0, b_j = 1) -> slot 0 / 1
  for (int j = 0; j < a.n_out; ++j) {
    const bool zb = beta[j] == 0;
    for (int p = tid; p < E / 2; p += kThreads) {
      int e0 = ((p >> j) << (j + 1)) | (p & ((1 << j) - 1));
      int e1 = e0 | (1 << j);
      double q0 = buf[e0], q1 = buf[e1];
      buf[e0] = zb ? q0 + q1 : q0 - q1;
      buf[e1] = zb ? q0 - q1 : 0.0;
    }
    __syncthreads();
  }
  // in-cut maps: digit j of s, 4 entries -> labels I, X, Y, Z
  for (int j = 0; j < a.n_in; ++j) {
    const int sh = 2 * j + a.xt_bits + a.n_out;
    for (int p = tid; p < E / 4; p += kThreads) {
      int lo = p & ((1 << sh) - 1);
      int e0 = ((p >> sh) << (sh + 2)) | lo;
      int st = 1 << sh;
      double p0 = buf[e0], p1 = buf[e0 + st], pp = buf[e0 + 2 * st], pi = buf[e0 + 3 * st];
      double s01 = p0 + p1;
      buf[e0] = s01;
      buf[e0 + st] = 2.0 * pp - s01;
      buf[e0 + 2 * st] = 2.0 * pi - s01;
      buf[e0 + 3 * st] = p0 - p1;
    }
    __syncthreads();
  }

  // write every label assignment compatible with beta: q = (xt, v, s), s fastest
  const int lNS = 2 * a.n_in;
  const int nq = (XT * NV) << lNS;
  const int64_t L = int64_t(1) << (2 * a.c);
  for (int q = tid; q < nq; q += kThreads) {
    const int s = q & (NS - 1);
    const int rest = q >> lNS;
    const int v = rest & (NV - 1);
    const int xt = rest >> nz;
    const double val = buf[(s * XT + xt) * NB + slot[v]] * a.scale;
    const int64_t o = (x0 + xt) * L + (sin[s] | sout[v]);
    if (a.out_f32) static_cast<float *>(a.out)[o] = (float)val;
    else static_cast<double *>(a.out)[o] = val;
  }
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

void launch_attribute(const AttrArgs &a0, hipStream_t s) {
  AttrArgs a = a0;
  const int64_t per_x = (int64_t(1) << (2 * a.n_in)) << a.n_out;
  const int64_t ns = int64_t(1) << (2 * a.n_in), nb = int64_t(1) << a.n_out;
  if (per_x <= kLdsElems && ns <= kMaxNS && nb <= kMaxNB && a.n_out <= 10) {  // grid.y = 3^n_out
    int xb = 0;
    while ((per_x << (xb + 1)) <= kLdsElems && xb + 1 <= a.d) ++xb;
    int64_t nbeta = 1;
    for (int j = 0; j < a.n_out; ++j) nbeta *= 3;
    // shrink the tile while that gives more work-groups and keeps >= 1024 entries
    while (xb > 0 && (((int64_t(1) << a.d) >> xb) * nbeta) < 1024 && (per_x << (xb - 1)) >= 1024)
      --xb;
    a.xt_bits = xb;
    dim3 grid((unsigned)((int64_t(1) << a.d) >> xb), (unsigned)nbeta);
    hipLaunchKernelGGL(attribute_lds, grid, dim3(kThreads), 0, s, a);
  } else {
    int64_t total = (int64_t(1) << a.d) << (2 * a.c);
    int64_t blocks = (total + kThreads - 1) / kThreads;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(attribute_direct, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
  }
}

}  // namespace sqc
