// gfx950 kernel for small layered meshes: one workgroup owns one item (a scenario of a mesh of
// at most kResMaxNodes nodes) and advances it through whole backward-Euler steps (eq. 2; eq. 10
// with the series R-L branch currents kept as state) without returning to the host: the
// right-hand side, the current sources, the red-black SOR sweeps of eqs. 16-17 and the stopping
// test of Algorithm 1 (the FP64 Jacobi-scaled residual, checked every check_every sweeps) all run
// inside the workgroup, separated by workgroup barriers only.  The node voltages and the
// right-hand side live in LDS; each thread keeps the coefficients of its nodes in registers.
//
// Thread t owns the node pairs p = t + k T (k < K) of the compact node numbering
// i = (l ny + y) nx + x, i.e. the nodes 2p and 2p + 1.  Consecutive compact nodes always have
// different colours (x + y + l parity: along a row x changes by one; a pair that wraps to the
// next row only exists when nx is odd, and then the parity flips as well), so each half-sweep
// updates exactly one node of every pair.  Sweeps run on the voltages directly,
//   v_i <- v_i + omega ((b_i + sum_j g_ij v_j) / M_ii - v_i),
// which has the iterates of the correction form used by the multi-launch path (a stationary
// iteration is affine), in FP64; the stopping test takes max_i |(b_i + sum_j g_ij v_j) / M_ii - v_i|,
// which is the Jacobi-scaled residual max_i |r_i| / M_ii.
#include "pgrid_internal.h"

namespace pgrid {

namespace {

template <int T>
__device__ __forceinline__ double block_max(double m, double* red) {
  for (int o = 32; o > 0; o >>= 1) m = nan_max(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int k = 1; k < T / 64; ++k) r = nan_max(r, red[k]);
  __syncthreads();  // red is reused by the next reduction
  return r;
}

// Piecewise-linear current of source k at time t (held constant outside its breakpoints).
__device__ __forceinline__ double pwl_current(const ResidentArgs& a, int k, double t) {
  const int lo0 = ld1(a.src_off, (int64_t)k), hi0 = ld1(a.src_off, (int64_t)k + 1) - 1;
  const double* __restrict__ ts = a.src_t;
  const double* __restrict__ is = a.src_i;
  if (t <= ts[lo0]) return is[lo0];
  if (t >= ts[hi0]) return is[hi0];
  int lo = lo0, hi = hi0;  // ts[lo] < t < ts[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ts[mid] <= t) lo = mid; else hi = mid;
  }
  return is[lo] + (is[hi] - is[lo]) * ((t - ts[lo]) / (ts[hi] - ts[lo]));
}

// Storage slot (row pitch X, layer stride PS) of compact node i of an nx x ny x nl mesh; the
// resident path's meshes are small, so 32-bit arithmetic suffices.
__device__ __forceinline__ int res_slot(int i, int nx, int P, int X, int PS) {
  const int l = i / P, rem = i - l * P, y = rem / nx, x = rem - y * nx;
  return l * PS + y * X + x;
}

// Compact node of storage slot s.
__device__ __forceinline__ int res_node(int s, int nx, int ny, int X, int PS) {
  const int l = s / PS, rem = s - l * PS, y = rem / X, x = rem - y * X;
  return (l * ny + y) * nx + x;
}

template <int K, int T, bool ML>
__global__ __launch_bounds__(T) void k_resident(ResidentArgs a) {
  constexpr int NPT = 2 * K;  // nodes per thread
  __shared__ double sv[kResMaxNodes];
  __shared__ double sb[kResMaxNodes];
  __shared__ double sil[kResMaxInd];
  __shared__ double red[T / 64];
  const int item = blockIdx.x;
  if (item >= a.n_items) return;
  const GridDesc& G = a.grids[a.item_grid[item]];
  const int scen = item - G.item0;
  const int nx = G.nx, ny = G.ny, X = G.X;
  const int P = nx * ny, n = P * G.nl;
  const int PS = X * ny;
  const int64_t off = (int64_t)scen * G.nstore;
  double* __restrict__ vg = G.v[a.vidx[item]] + off;
  const int n_ind = G.n_ind;
  double* __restrict__ ilg = G.ind_i + (int64_t)scen * n_ind;

  // this thread's nodes (compact index, -1 beyond the mesh), their colours (bit j) and the
  // conductances to the six neighbours (zero where absent) and 1/M_ii, in registers
  int idx[NPT];
  unsigned colour = 0u;
  double cE[NPT], cW[NPT], cN[NPT], cS[NPT], cU[NPT], cD[NPT], inv[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int i = 2 * ((int)threadIdx.x + (j >> 1) * T) + (j & 1);
    idx[j] = i < n ? i : -1;
    cE[j] = cW[j] = cN[j] = cS[j] = cU[j] = cD[j] = inv[j] = 0.0;
    if (i >= n) continue;
    const int l = i / P, rem = i - l * P, y = rem / nx, x = rem - y * nx;
    const int s = l * PS + y * X + x;
    colour |= (unsigned)((x + y + l) & 1) << j;
    cE[j] = ld1(G.gE64, s);
    cW[j] = x > 0 ? ld1(G.gE64, s - 1) : 0.0;
    cN[j] = ld1(G.gN64, s);
    cS[j] = y > 0 ? ld1(G.gN64, s - X) : 0.0;
    if (ML) {
      cU[j] = ld1(G.gU64, s);
      cD[j] = l > 0 ? ld1(G.gU64, s - PS) : 0.0;
    }
    inv[j] = 1.0 / ld1(G.D64, s);
    sv[i] = ld1((const double*)vg, s);
  }
  // b_i + sum_j g_ij v_j of node j from the voltages in LDS; an absent neighbour has g = 0 and
  // its index is clamped to the node itself, so every read stays in bounds
  auto nsum = [&](int j, double bj) {
    const int i = idx[j];
    double acc = bj;
    acc += cE[j] * sv[cE[j] != 0.0 ? i + 1 : i];
    acc += cW[j] * sv[cW[j] != 0.0 ? i - 1 : i];
    acc += cN[j] * sv[cN[j] != 0.0 ? i + nx : i];
    acc += cS[j] * sv[cS[j] != 0.0 ? i - nx : i];
    if (ML) {  // single-layer launches keep no via terms
      acc += cU[j] * sv[cU[j] != 0.0 ? i + P : i];
      acc += cD[j] * sv[cD[j] != 0.0 ? i - P : i];
    }
    return acc;
  };
  for (int k = threadIdx.x; k < n_ind; k += T) sil[k] = ld1((const double*)ilg, (int64_t)k);
  const int src0 = a.item_src_off[item], src1 = a.item_src_off[item + 1];
  // steps completed before this launch: the device clock, which k_resident_clock advances once
  // every workgroup of the launch has finished (so a replayed launch continues the transient)
  const long long k0 = __hip_atomic_load(a.step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  long long tot_sweeps = 0, tot_checks = 0;
  int max_sw = 0, last_sw = 0, failed = 0;
  double last_res = 0.0, max_res = 0.0;
  __syncthreads();

  for (int step = 0; step < a.nsteps; ++step) {
    const double t = (double)(k0 + step + 1) * a.h;
    // right-hand side: (C/h) v + G0 Vdd - the companion history of the series R-L branches
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      if (idx[j] < 0) continue;
      const int s = res_slot(idx[j], nx, P, X, PS);
      double bb = ld1(G.ch64, s) * sv[idx[j]] + ld1(G.bconst64, s);
      if (n_ind) {
        for (int q = ld1(G.inc_off, s); q < ld1(G.inc_off, s + 1); ++q) {
          const int e = ld1(G.inc_ind, (int64_t)q);
          const int kk = (e > 0 ? e : -e) - 1;
          const double term = ld1(G.ind_alpha, (int64_t)kk) * sil[kk];
          bb += (e > 0) ? -term : term;
        }
      }
      sb[idx[j]] = bb;
    }
    __syncthreads();
    // the loads at t (backward Euler samples the sources at the end of the step)
    for (int q = src0 + (int)threadIdx.x; q < src1; q += T) {
      const int k = ld1(a.item_src, (int64_t)q);
      const int node = res_node((int)((int64_t)ld1(a.src_index, (int64_t)k) - off), nx, ny, X, PS);
      atomicAdd(&sb[node], -pwl_current(a, k, t));
    }
    __syncthreads();
    double b[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) b[j] = idx[j] >= 0 ? sb[idx[j]] : 0.0;
    // Algorithm 1: from the previous step's solution, sweep until the scaled residual
    // max_i |r_i| / M_ii = max_i |(b + sum_j g_ij v_j) / M_ii - v_i| is <= tol
    int sw = 0;
    double res;
    while (true) {
      double m = 0.0;
#pragma unroll
      for (int j = 0; j < NPT; ++j)
        if (idx[j] >= 0) m = nan_max(m, fabs(nsum(j, b[j]) * inv[j] - sv[idx[j]]));
      res = block_max<T>(m, red);
      ++tot_checks;
      if (res <= a.tol) break;
      if (sw >= a.max_sweeps) {
        failed = 1;
        break;
      }
      for (int k = 0; k < a.check_every; ++k) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
#pragma unroll
          for (int j = 0; j < NPT; ++j) {
            if (idx[j] < 0 || (int)((colour >> j) & 1u) != half) continue;
            const double old = sv[idx[j]];
            sv[idx[j]] = old + a.omega * (nsum(j, b[j]) * inv[j] - old);
          }
          __syncthreads();
        }
      }
      sw += a.check_every;
    }
    // the branch currents at t: i = alpha i + g_eq (v_a - v_b)
    for (int k = threadIdx.x; k < n_ind; k += T) {
      const int sa = ld1(G.ind_a, (int64_t)k), sbs = ld1(G.ind_b, (int64_t)k);
      const double va = sv[res_node(sa, nx, ny, X, PS)];
      const double vb = sbs >= 0 ? sv[res_node(sbs, nx, ny, X, PS)] : (G.ind_vfar ? ld1(G.ind_vfar, (int64_t)k) : G.vdd);
      sil[k] = ld1(G.ind_alpha, (int64_t)k) * sil[k] + ld1(G.ind_geq, (int64_t)k) * (va - vb);
    }
    __syncthreads();
    tot_sweeps += sw;
    max_sw = max(max_sw, sw);
    last_sw = sw;
    last_res = res;
    max_res = nan_max(max_res, res);
  }

  // write the state back and fold this item's statistics into the context's
#pragma unroll
  for (int j = 0; j < NPT; ++j)
    if (idx[j] >= 0) st1(vg, res_slot(idx[j], nx, P, X, PS), sv[idx[j]]);
  for (int k = threadIdx.x; k < n_ind; k += T) st1(ilg, (int64_t)k, sil[k]);
  if (threadIdx.x == 0) {
    atomicAdd((unsigned long long*)a.stat_sweeps, (unsigned long long)tot_sweeps);
    atomicAdd((unsigned long long*)a.stat_updates, (unsigned long long)(tot_sweeps * (long long)n));
    atomicAdd((unsigned long long*)a.stat_checks, (unsigned long long)tot_checks);
    atomicMax(a.stat_max_sweeps, max_sw);
    atomicMax(a.stat_last_sweeps, last_sw);
    atomicMax((unsigned long long*)a.stat_last_res, (unsigned long long)__double_as_longlong(last_res));
    atomicMax((unsigned long long*)a.stat_max_res, (unsigned long long)__double_as_longlong(max_res));
    if (failed) atomicOr(a.stat_failed, 1);
  }
}

// Before a resident launch: the per-launch statistics that the items raise with atomics.
__global__ void k_resident_prep(int32_t* last_sweeps, double* last_res) {
  last_sweeps[0] = 0;
  last_res[0] = 0.0;
}

// After a resident launch of nsteps: advance the device clock (steps completed).
__global__ void k_resident_clock(long long* step, int nsteps) { step[0] += nsteps; }

}  // namespace

template <bool ML>
static void launch_resident_nl(const ResidentArgs& a, int max_nodes, hipStream_t s) {
  if (max_nodes <= 2 * 512)
    hipLaunchKernelGGL((k_resident<1, 512, ML>), dim3(a.n_items), dim3(512), 0, s, a);
  else if (max_nodes <= 2 * 1024)
    hipLaunchKernelGGL((k_resident<1, 1024, ML>), dim3(a.n_items), dim3(1024), 0, s, a);
  else
    hipLaunchKernelGGL((k_resident<2, 1024, ML>), dim3(a.n_items), dim3(1024), 0, s, a);
}

hipError_t launch_resident(const ResidentArgs& a, int max_nodes, bool multi_layer, hipStream_t s) {
  if (a.n_items <= 0 || a.nsteps <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_resident_prep, dim3(1), dim3(1), 0, s, a.stat_last_sweeps, a.stat_last_res);
  if (multi_layer)
    launch_resident_nl<true>(a, max_nodes, s);
  else
    launch_resident_nl<false>(a, max_nodes, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_resident_clock, dim3(1), dim3(1), 0, s, a.step, a.nsteps);
  return hipGetLastError();
}

}  // namespace pgrid
