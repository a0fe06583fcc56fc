// gfx950 kernels for general netlists (Sec. III): the same backward-Euler step and
// correction sweeps as the mesh kernels, on an arbitrary node graph.
//
// The nodes are stored colour by colour (no branch joins two nodes of one colour), so all
// nodes of a colour update independently: one launch per colour, in colour order, is one
// Gauss-Seidel/SOR sweep of eqs. 16-17 in that node order (Theorem 1), done in place.
// Neighbours come from a compact sliced-ELL table with 64-slot slices: lane j of a wavefront
// owns slot 64 s + j, and the slice stores entry k of the rows that have one contiguously, so
// the lanes of a wave read each entry level as one unit-stride run with no padding, and only
// the neighbour values are gathered (from L2 for graphs whose node numbering keeps neighbours
// close).
#include "pgrid_internal.h"

namespace pgrid {

namespace {

constexpr int kGraphGroup = 8;  // table entry levels whose loads a lane issues together

// Walks the compact neighbour table (see GridDesc) for the slot of this lane; all 64 lanes of
// the wave (one slice) take part.  For entry level k the ballot of the lanes whose rows have
// more than k entries gives each of them its rank (the set bits below its own) and the count
// that the next level starts after.
struct RowWalk {
  int P;    // first table entry of the current level (uniform over the wave)
  int len;  // this lane's row length
  __device__ __forceinline__ RowWalk(const GridDesc& G, int i) {
    P = ld1(G.sl_off, __builtin_amdgcn_readfirstlane(i >> 6));
    len = ld1(G.sl_len, i);
  }
  // some lane of the wave has entry k (uniform)
  __device__ __forceinline__ bool any(int k) const { return __ballot(k < len) != 0; }
  // table position of this lane's entry k (meaningful for k < len); moves past level k
  __device__ __forceinline__ int next(int k) {
    const unsigned long long m = __ballot(k < len);
    const int e = P + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
    P += __popcll(m);
    return e;
  }
};

// b = (C/h) v + G0 v_s + (h/L) v_s - inductor history, with C/h's off-diagonal coupling terms.
__global__ __launch_bounds__(kChunk) void k_graph_rhs(const GraphChunk* __restrict__ chunks, int n,
                                                     const GridDesc* __restrict__ grids, Ctl c, int save_prev) {
  if (*c.stall) return;  // a stalled step opening
  const int ci = xcd_tile(n);
  if (ci < 0) return;
  const GraphChunk ch = chunks[ci];
  if ((int)threadIdx.x >= ch.count) return;
  const GridDesc& G = grids[ch.grid];
  const int64_t off = (int64_t)ch.scen * G.nstore;
  const int i = ch.slot0 + (int)threadIdx.x;
  const double* __restrict__ v = G.v[c.vidx[ch.item]] + off;
  double bb = G.ch64[i] * v[i] + G.bconst64[i];
  if (G.cap_off) {
    const int base = G.cap_off[i >> 6] + (i & 63), w = (G.cap_off[(i >> 6) + 1] - G.cap_off[i >> 6]) >> 6;
    for (int k = 0; k < w; ++k) bb -= G.cap_val[base + (k << 6)] * v[G.cap_col[base + (k << 6)]];
  }
  if (G.n_ind) {
    const double* __restrict__ il = G.ind_i + (int64_t)ch.scen * G.n_ind;
    for (int j = G.inc_off[i]; j < G.inc_off[i + 1]; ++j) {
      const int e = G.inc_ind[j];
      const int kk = (e > 0 ? e : -e) - 1;
      const double term = G.ind_alpha[kk] * il[kk];
      bb += (e > 0) ? -term : term;
    }
  }
  G.b[off + i] = bb;
  if (save_prev) G.vprev[(c.step[0] + 1) & 1][off + i] = v[i];
}

// Three-level right-hand side (eq. 11 / eq. 14) without the sources:
//   b = (C/h)(2 v(t) - v(t-h)) + G v(t) + (h/L) v_s,
// G being the resistor part of M (diagonal incl. resistors to supplies and ground); v(t) is
// kept as the next step's v(t-h) in the other vprev buffer.
__global__ __launch_bounds__(kChunk) void k_graph_rhs3(const GraphChunk* __restrict__ chunks, int n,
                                                      const GridDesc* __restrict__ grids, Ctl c) {
  if (*c.stall) return;
  const int ci = xcd_tile(n);
  if (ci < 0) return;
  const GraphChunk ch = chunks[ci];
  if ((int)threadIdx.x >= ch.count) return;
  const GridDesc& G = grids[ch.grid];
  const int64_t off = (int64_t)ch.scen * G.nstore;
  const int i = ch.slot0 + (int)threadIdx.x;
  const double* __restrict__ v = G.v[c.vidx[ch.item]] + off;
  const long long k0 = c.step[0];
  const double* __restrict__ vp = G.vprev[k0 & 1] + off;
  const double vi = v[i];
  double bb = G.ch64[i] * (2.0 * vi - vp[i]) + G.g3diag[i] * vi + G.bl64[i];
  {
    RowWalk t(G, i);
    for (int k = 0; t.any(k); ++k) {
      const int e = t.next(k);
      if (k < t.len) bb -= G.sl_g64[e] * v[G.sl_col[e]];
    }
  }
  if (G.cap_off) {
    const int base = G.cap_off[i >> 6] + (i & 63), w = (G.cap_off[(i >> 6) + 1] - G.cap_off[i >> 6]) >> 6;
    for (int k = 0; k < w; ++k) {
      const int j = G.cap_col[base + (k << 6)];
      bb -= G.cap_val[base + (k << 6)] * (2.0 * v[j] - vp[j]);
    }
  }
  G.b[off + i] = bb;
  G.vprev[(k0 + 1) & 1][off + i] = vi;
}

// Kirchhoff's current law at the current time with backward-Euler capacitor currents and the
// tracked inductor currents, without the sources (added next by the source kernel):
//   b = (C/h)(v - v(t-h)) + G v - G0 v_s + A_l^T i.
__global__ __launch_bounds__(kChunk) void k_graph_kcl(const GraphChunk* __restrict__ chunks, int n,
                                                     const GridDesc* __restrict__ grids, Ctl c) {
  const int ci = xcd_tile(n);
  if (ci < 0) return;
  const GraphChunk ch = chunks[ci];
  if ((int)threadIdx.x >= ch.count) return;
  const GridDesc& G = grids[ch.grid];
  const int64_t off = (int64_t)ch.scen * G.nstore;
  const int i = ch.slot0 + (int)threadIdx.x;
  const double* __restrict__ v = G.v[c.vidx[ch.item]] + off;
  const double* __restrict__ vp = G.vprev[c.step[0] & 1] + off;
  double res = G.ch64[i] * (v[i] - vp[i]) + G.g3diag[i] * v[i] - G.bres64[i];
  {
    RowWalk t(G, i);
    for (int k = 0; t.any(k); ++k) {
      const int e = t.next(k);
      if (k < t.len) res -= G.sl_g64[e] * v[G.sl_col[e]];
    }
  }
  if (G.cap_off) {
    const int base = G.cap_off[i >> 6] + (i & 63), w = (G.cap_off[(i >> 6) + 1] - G.cap_off[i >> 6]) >> 6;
    for (int k = 0; k < w; ++k) {
      const int j = G.cap_col[base + (k << 6)];
      res -= G.cap_val[base + (k << 6)] * (v[j] - vp[j]);
    }
  }
  if (G.n_ind) {
    const double* __restrict__ il = G.ind_i + (int64_t)ch.scen * G.n_ind;
    for (int j = G.inc_off[i]; j < G.inc_off[i + 1]; ++j) {
      const int e = G.inc_ind[j];
      const int kk = (e > 0 ? e : -e) - 1;
      res += (e > 0) ? il[kk] : -il[kk];  // current leaving through the near end
    }
  }
  G.b[off + i] = res;
}

// max_i |b_i| / M_ii of each chunk's item into c.norm_bits[item].
__global__ __launch_bounds__(kChunk) void k_graph_absmax_b(const GraphChunk* __restrict__ chunks, int n,
                                                          const GridDesc* __restrict__ grids, Ctl c) {
  __shared__ double wmax[kChunk / 64];
  const int ci = xcd_tile(n);
  if (ci < 0) return;
  const GraphChunk ch = chunks[ci];
  const GridDesc& G = grids[ch.grid];
  double m = 0.0;
  if ((int)threadIdx.x < ch.count) {
    const int i = ch.slot0 + (int)threadIdx.x;
    const double D = G.D64[i];
    if (D > 0.0) m = fabs(G.b[(int64_t)ch.scen * G.nstore + i]) / D;
  }
  for (int o = 32; o > 0; o >>= 1) m = nan_max(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double bm = wmax[0];
    for (int k = 1; k < kChunk / 64; ++k) bm = nan_max(bm, wmax[k]);
    raise_max(&c.norm_bits[ch.item], bm);
  }
}

// One colour of a sweep on M d = r: d_i <- d_i + omega ((r_i + sum_j w_ij d_j) / M_ii - d_i).
// zero_in: the sweep starts a refinement cycle from d = 0, so the old d_i and every neighbour
// not yet updated in this sweep (slot >= lim) count as zero.
template <typename T>
__global__ __launch_bounds__(kChunk) void k_graph_sweep(const GraphChunk* __restrict__ chunks, int n,
                                                       const GridDesc* __restrict__ grids, Ctl c, int zero_in,
                                                       T omega) {
  const int ci = xcd_tile(n);
  if (ci < 0) return;
  const GraphChunk ch = chunks[ci];
  if (!c.active[ch.item] || (int)threadIdx.x >= ch.count) return;
  const GridDesc& G = grids[ch.grid];
  const int64_t off = (int64_t)ch.scen * G.nstore;
  const int i = ch.slot0 + (int)threadIdx.x;
  T* __restrict__ d = static_cast<T*>(G.d[0]) + off;
  const T* __restrict__ r = static_cast<const T*>(G.r) + off;
  const T* __restrict__ wv = static_cast<const T*>(G.sl_ws);
  // chunks start on 64-slot slices and cover whole ones, so a wave is one slice
  RowWalk t(G, i);
  // zero_in: only neighbours already updated in this sweep (slot < lim) carry a value
  const int lim = zero_in ? ch.lim : 0x7fffffff;
  T acc = ld1(r, i);
  const T inv = ld1(static_cast<const T*>(G.invDs), i);
  const T old = zero_in ? T(0) : ld1(d, i);
  // kGraphGroup entry levels, then their gathers, in flight together
  for (int k = 0; t.any(k); k += kGraphGroup) {
    int j[kGraphGroup];
    T g[kGraphGroup], dj[kGraphGroup];
#pragma unroll
    for (int q = 0; q < kGraphGroup; ++q) {
      const int e = t.next(k + q);
      const bool has = k + q < t.len;
      j[q] = has ? ld1(G.sl_col, e) : lim;
      g[q] = has ? ld1(wv, e) : T(0);
    }
#pragma unroll
    for (int q = 0; q < kGraphGroup; ++q) dj[q] = j[q] < lim ? ld1(d, j[q]) : T(0);
#pragma unroll
    for (int q = 0; q < kGraphGroup; ++q)
      if (k + q < t.len) acc += g[q] * dj[q];
  }
  st1(d, i, old + omega * (inv * acc - old));
}

// FP64 residual r = b - M v' with v' = v + d[0] (has_d) written to the other voltage buffer, r in
// the sweep precision, and the Jacobi-scaled norm max |r_i| / M_ii of the chunk's item.
template <typename T>
__global__ __launch_bounds__(kChunk) void k_graph_resid(const GraphChunk* __restrict__ chunks, int n,
                                                       const GridDesc* __restrict__ grids, Ctl c, int has_d,
                                                       int norm) {
  __shared__ double wmax[kChunk / 64];
  if (*c.stall) return;
  const int ci = xcd_tile(n);
  if (ci < 0) return;
  const GraphChunk ch = chunks[ci];
  if (!c.active[ch.item]) return;  // uniform over the block
  const GridDesc& G = grids[ch.grid];
  const int64_t off = (int64_t)ch.scen * G.nstore;
  const int vi = c.vidx[ch.item];
  const double* __restrict__ v = G.v[vi] + off;
  const T* __restrict__ d = static_cast<const T*>(G.d[0]) + off;
  double m = 0.0;
  if ((int)threadIdx.x < ch.count) {
    const int i = ch.slot0 + (int)threadIdx.x;
    const double D = ld1(G.D64, i);
    const double own = has_d ? ld1(v, i) + (double)ld1(d, i) : ld1(v, i);
    double acc = ld1(G.b, off + i) - D * own;
    RowWalk t(G, i);  // a wave is one slice (see k_graph_sweep)
    for (int k = 0; t.any(k); k += kGraphGroup) {  // kGraphGroup levels, then their gathers, in flight
      int j[kGraphGroup];
      double g[kGraphGroup], x[kGraphGroup];
#pragma unroll
      for (int q = 0; q < kGraphGroup; ++q) {
        const int e = t.next(k + q);
        const bool has = k + q < t.len;
        j[q] = has ? ld1(G.sl_col, e) : -1;
        g[q] = has ? ld1(G.sl_w64, e) : 0.0;
      }
#pragma unroll
      for (int q = 0; q < kGraphGroup; ++q)
        x[q] = j[q] < 0 ? 0.0 : has_d ? ld1(v, j[q]) + (double)ld1(d, j[q]) : ld1(v, j[q]);
#pragma unroll
      for (int q = 0; q < kGraphGroup; ++q)
        if (k + q < t.len) acc += g[q] * x[q];
    }
    if (has_d) st1(G.v[vi ^ 1], off + i, own);
    st1(static_cast<T*>(G.r), off + i, (T)acc);
    if (D > 0.0) m = fabs(acc) / D;  // padding slots (D = 0) carry r = 0
  }
  if (!norm) return;  // uniform over the grid
  for (int o = 32; o > 0; o >>= 1) m = nan_max(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double bm = wmax[0];
    for (int k = 1; k < kChunk / 64; ++k) bm = nan_max(bm, wmax[k]);
    raise_max(&c.norm_bits[ch.item], bm);
  }
}

// The opening probe of a general netlist: a step predicted to converge at once, with the sources
// all zero and v' = v.  The C/h terms of b and of M v' cancel exactly (the coupling capacitors'
// with their off-diagonal entries), and with e = v - vref
//   r_i = q_i - history_i - gsup_i e_i + sum_j wG_ij (e_j - e_i),
// wG the conductance part of M's off-diagonal (resistors and inductor companions), gsup_i the
// conductance from node i to supplies and ground, q_i = (G0 v_s + (h/L) v_s)_i - gsup_i vref.
// The conductance terms are evaluated in FP32 on e_i and on the neighbour differences
// v_j - v_i (formed in FP64, exact for voltages within a factor of two of each other, then
// rounded); every rounding in them (of e_i, of the differences, of wG and gsup, of the products
// and of the sum of k + 1 terms) is a relative error of at most u = 2^-24 on a term of
// S_i = gsup_i |e_i| + sum_j wG_ij |v_j - v_i|, so (k + 8) 2^-23 S_i, k the row's length,
// bounds their total error; the scale 1/M_ii is widened by its rounding.  The result bounds the
// FP64 norm from above.
template <typename T>
__global__ __launch_bounds__(kChunk) void k_graph_probe(const GraphChunk* __restrict__ chunks, int n,
                                                       const GridDesc* __restrict__ grids, Ctl c) {
  constexpr double kWiden = sizeof(T) == 4 ? 1.0 + 0x1p-22 : 1.0 + 0x1p-51;
  __shared__ double wmax[kChunk / 64];
  if (*c.stall) return;
  const int ci = xcd_tile(n);
  if (ci < 0) return;
  const GraphChunk ch = chunks[ci];
  if (!c.active[ch.item]) return;  // uniform over the block
  const GridDesc& G = grids[ch.grid];
  const int64_t off = (int64_t)ch.scen * G.nstore;
  const double* __restrict__ v = G.v[c.vidx[ch.item]] + off;
  const double vref = G.vdd;
  double m = 0.0;
  if ((int)threadIdx.x < ch.count) {
    const int i = ch.slot0 + (int)threadIdx.x;
    const T inv = ld1(static_cast<const T*>(G.invDs), i);
    const double q0 = ld1(G.gq64, i);
    const float gs = ld1(G.gsup32, i);
    const double vi = ld1(v, i);
    const float ei = (float)(vi - vref);
    RowWalk t(G, i);  // a wave is one slice (see k_graph_sweep)
    float r = -gs * ei, s = gs * fabsf(ei);
    for (int k = 0; t.any(k); k += kGraphGroup) {  // kGraphGroup levels, then their gathers, in flight
      int j[kGraphGroup];
      float g[kGraphGroup], dj[kGraphGroup];
#pragma unroll
      for (int q = 0; q < kGraphGroup; ++q) {
        const int e = t.next(k + q);
        const bool has = k + q < t.len;
        j[q] = has ? ld1(G.sl_col, e) : -1;
        g[q] = has ? ld1(G.gw32, e) : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < kGraphGroup; ++q) dj[q] = j[q] < 0 ? 0.0f : (float)(ld1(v, j[q]) - vi);
#pragma unroll
      for (int q = 0; q < kGraphGroup; ++q)
        if (k + q < t.len) {
          r += g[q] * dj[q];
          s += g[q] * fabsf(dj[q]);
        }
    }
    double hist = 0.0;  // b's history: -alpha_k i_k for each branch k leaving node i (+ entering)
    if (G.n_ind) {
      const double* __restrict__ il = G.ind_i + (int64_t)ch.scen * G.n_ind;
      for (int t = G.inc_off[i]; t < G.inc_off[i + 1]; ++t) {
        const int e = G.inc_ind[t];
        const int kk = (e > 0 ? e : -e) - 1;
        const double term = G.ind_alpha[kk] * il[kk];
        hist += (e > 0) ? -term : term;
      }
    }
    const double bound = fabs(q0 + hist + (double)r) + (double)((float)(t.len + 8) * 0x1p-23f * s);
    m = bound * ((double)inv * kWiden);  // padding slots: inv = 0
  }
  for (int o = 32; o > 0; o >>= 1) m = nan_max(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double bm = wmax[0];
    for (int k = 1; k < kChunk / 64; ++k) bm = nan_max(bm, wmax[k]);
    raise_max(&c.norm_bits[ch.item], bm);
  }
}

__global__ void k_gather(const double* __restrict__ src, const int32_t* __restrict__ slot,
                         double* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[slot[i]];
}

}  // namespace

hipError_t launch_graph_rhs(const GraphChunk* ch, int n, const GridDesc* grids, const Ctl& c, int save_prev,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_graph_rhs, dim3(xcd_blocks(n)), dim3(kChunk), 0, s, ch, n, grids, c, save_prev);
  return hipGetLastError();
}

hipError_t launch_graph_rhs3(const GraphChunk* ch, int n, const GridDesc* grids, const Ctl& c, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_graph_rhs3, dim3(xcd_blocks(n)), dim3(kChunk), 0, s, ch, n, grids, c);
  return hipGetLastError();
}

hipError_t launch_graph_kcl(const GraphChunk* ch, int n, const GridDesc* grids, const Ctl& c, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_graph_kcl, dim3(xcd_blocks(n)), dim3(kChunk), 0, s, ch, n, grids, c);
  return hipGetLastError();
}

hipError_t launch_graph_absmax_b(const GraphChunk* ch, int n, const GridDesc* grids, const Ctl& c, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_graph_absmax_b, dim3(xcd_blocks(n)), dim3(kChunk), 0, s, ch, n, grids, c);
  return hipGetLastError();
}

hipError_t launch_graph_sweep(bool fp32, const GraphChunk* ch, int n, const GridDesc* grids, const Ctl& c,
                              int zero_in, double omega, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_graph_sweep<float>, dim3(xcd_blocks(n)), dim3(kChunk), 0, s, ch, n, grids, c, zero_in,
                       (float)omega);
  else
    hipLaunchKernelGGL(k_graph_sweep<double>, dim3(xcd_blocks(n)), dim3(kChunk), 0, s, ch, n, grids, c, zero_in,
                       omega);
  return hipGetLastError();
}

hipError_t launch_graph_probe(bool fp32, const GraphChunk* ch, int n, const GridDesc* grids, const Ctl& c,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_graph_probe<float>, dim3(xcd_blocks(n)), dim3(kChunk), 0, s, ch, n, grids, c);
  else
    hipLaunchKernelGGL(k_graph_probe<double>, dim3(xcd_blocks(n)), dim3(kChunk), 0, s, ch, n, grids, c);
  return hipGetLastError();
}

hipError_t launch_graph_resid(bool fp32, const GraphChunk* ch, int n, const GridDesc* grids, const Ctl& c,
                              int has_d, hipStream_t s, int norm) {
  if (n <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_graph_resid<float>, dim3(xcd_blocks(n)), dim3(kChunk), 0, s, ch, n, grids, c, has_d, norm);
  else
    hipLaunchKernelGGL(k_graph_resid<double>, dim3(xcd_blocks(n)), dim3(kChunk), 0, s, ch, n, grids, c, has_d, norm);
  return hipGetLastError();
}

hipError_t launch_gather(const double* src, const int32_t* slot, double* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, slot, dst, n);
  return hipGetLastError();
}

}  // namespace pgrid
