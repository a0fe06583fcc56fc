// gfx950 kernels of the backward-Euler relaxation step.
//
// One backward-Euler step (eq. 2 for RC grids, eq. 10 with the inductor current kept as
// state for RLC grids) solves M v = b with
//   b_i = (C_i/h) v_i(t) + G0_i Vdd - I_i(t+h) - sum_branches(+-alpha i_l)      (rhs + sources)
// by repeated relaxation sweeps on the correction equation M d = r, r = b - M v, followed by
// v <- v + d and a new FP64 residual (iterative refinement when the sweeps run in FP32).
// A sweep is the red-black form of eqs. 16-17:
//   d_i <- d_i + omega * ( (r_i + sum_j g_ij d_j) / M_ii - d_i ),
// red nodes (x+y+layer even) first from the old black values, then black nodes from the new
// red values.  Because the sweep is an affine stationary iteration, sweeping the correction
// from d = 0 produces exactly the iterates of sweeping v itself (in exact arithmetic).
//
// Memory layout: every per-node array is padded to n = nl*ny*nx entries in natural order
// (x fastest), so a 64-lane wavefront reads 64 consecutive nodes of one row.  A workgroup
// owns a 64 x TY tile through all layers and stages the correction in LDS with a two-cell
// halo; the red half-sweep is recomputed on a one-cell ring around the tile so the black
// half-sweep sees exactly the red values a global red-black sweep would produce, which lets
// one launch perform a whole sweep with ping-pong buffers and no grid-wide barrier.
#include "pgrid_internal.h"

#include <cfloat>

namespace pgrid {

namespace {

// Tiles are numbered row-major over each grid.  Workgroups are dealt to the 8 XCDs round
// robin, so block b runs on XCD b % 8; give each XCD a contiguous run of tiles so vertically
// adjacent tiles (which re-read each other's halo rows) share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int ntiles) {
  const int per = (int)(gridDim.x / 8u);
  const int b = (int)blockIdx.x;
  const int t = (b % 8) * per + b / 8;
  return t < ntiles ? t : -1;
}

__device__ __forceinline__ double nan_max(double m, double x) {
  return (x > m || x != x) ? x : m;
}

}  // namespace

// ------------------------------------------------------------------------------------
// Step bookkeeping
// ------------------------------------------------------------------------------------
__global__ void k_step_begin(Ctl c, int G) {
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    c.active[g] = 1;
    c.step_sweeps[g] = 0;
    c.failed[g] = 0;
    c.norm_bits[g] = 0ull;
  }
}

__global__ void k_decide(Ctl c, int G, double tol, int has_d, int nchk, int max_sweeps) {
  __shared__ int any;
  __shared__ int worked;
  if (threadIdx.x == 0) { any = 0; worked = 0; }
  __syncthreads();
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    if (c.active[g]) {
      atomicOr(&worked, 1);
      if (has_d) {
        c.vidx[g] ^= 1;
        c.step_sweeps[g] += nchk;
      }
      const double nm = __longlong_as_double((long long)c.norm_bits[g]);
      c.last_norm[g] = nm;
      const bool conv = nm <= tol;                 // false for NaN
      const bool spent = c.step_sweeps[g] >= max_sweeps;
      const int act = (!conv && !spent) ? 1 : 0;
      c.active[g] = act;
      if (!conv && spent) c.failed[g] = 1;
      if (act) atomicOr(&any, 1);
    }
    c.norm_bits[g] = 0ull;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    c.any_active[0] = any;
    if (worked) c.stat_checks[0] += 1;
  }
}

__global__ void k_step_end(Ctl c, int G) {
  if (threadIdx.x != 0) return;
  long long sw = 0, upd = 0;
  int mx = 0, fail = 0;
  double res = 0.0;
  for (int g = 0; g < G; ++g) {
    const int s = c.step_sweeps[g];
    sw += s;
    upd += (long long)s * c.nodes[g];
    mx = s > mx ? s : mx;
    res = nan_max(res, c.last_norm[g]);
    fail |= c.failed[g];
  }
  c.stat_sweeps[0] += sw;
  c.stat_updates[0] += upd;
  c.stat_last_sweeps[0] = mx;
  if (mx > c.stat_max_sweeps[0]) c.stat_max_sweeps[0] = mx;
  c.stat_last_res[0] = res;
  c.stat_max_res[0] = nan_max(c.stat_max_res[0], res);
  c.stat_failed[0] |= fail;
}

// ------------------------------------------------------------------------------------
// Right-hand side of the step (eq. 2 / eq. 10): b = (C/h) v + G0 Vdd - inductor history.
// Sources are subtracted afterwards by k_sources.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_rhs(const Tile* __restrict__ tiles, int ntiles,
                                                 const GridDesc* __restrict__ grids, Ctl c, int TY) {
  const int ti = xcd_tile(ntiles);
  if (ti < 0) return;
  const Tile tl = tiles[ti];
  const GridDesc& G = grids[tl.grid];
  const int nx = G.nx, ny = G.ny, S = G.S;
  const int64_t P = (int64_t)nx * ny;
  const double* __restrict__ v = G.v[c.vidx[tl.grid]];
  const int per_layer = kTileX * TY * S;
  const int total = per_layer * G.nl;
  for (int k = threadIdx.x; k < total; k += kThreads) {
    const int l = k / per_layer;
    const int rem = k - l * per_layer;
    const int node_in = rem / S;
    const int s = rem - node_in * S;
    const int yy = node_in / kTileX, xx = node_in - yy * kTileX;
    const int x = tl.x0 + xx, y = tl.y0 + yy;
    if (x >= nx || y >= ny) continue;
    const int64_t i = l * P + (int64_t)y * nx + x;
    const int64_t idx = i * S + s;
    double bb = G.ch64[i] * v[idx] + G.bconst64[i];
    if (G.n_ind) {
      for (int j = G.inc_off[i]; j < G.inc_off[i + 1]; ++j) {
        const int e = G.inc_ind[j];
        const int kk = (e > 0 ? e : -e) - 1;
        const double term = G.ind_alpha[kk] * G.ind_i[(int64_t)kk * S + s];
        bb += (e > 0) ? -term : term;
      }
    }
    G.b[idx] = bb;
  }
}

// Piecewise-linear current sources at time t, subtracted from b (one thread per source).
__global__ void k_sources(SourceTable src, const GridDesc* __restrict__ grids, double t) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= src.count) return;
  const int a = src.off[k], e = src.off[k + 1];
  const double* __restrict__ ts = src.t;
  const double* __restrict__ is = src.i;
  double I;
  if (t <= ts[a]) {
    I = is[a];
  } else if (t >= ts[e - 1]) {
    I = is[e - 1];
  } else {
    int lo = a, hi = e - 1;  // ts[lo] < t < ts[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (ts[mid] <= t) lo = mid; else hi = mid;
    }
    I = is[lo] + (is[hi] - is[lo]) * ((t - ts[lo]) / (ts[hi] - ts[lo]));
  }
  const GridDesc& G = grids[src.grid[k]];
  G.b[src.index[k]] -= I;
}

// ------------------------------------------------------------------------------------
// FP64 residual r = b - M v' with v' = v + d, and the Jacobi-scaled norm max |r_i| / M_ii.
// Writes v' into the other voltage buffer (the decision kernel flips the index), and r in
// the sweep precision as the right-hand side of the next correction sweeps.
// ------------------------------------------------------------------------------------
template <typename T, int NL, int TY>
__global__ __launch_bounds__(kThreads) void k_resid(const Tile* __restrict__ tiles, int ntiles,
                                                   const GridDesc* __restrict__ grids, Ctl c,
                                                   int has_d, int din) {
  constexpr int TX = kTileX, HX = TX + 2, HY = TY + 2;
  __shared__ double sv[NL][HY][HX];
  __shared__ double wmax[kThreads / 64];
  const int ti = xcd_tile(ntiles);
  if (ti < 0) return;
  const Tile tl = tiles[ti];
  const int g = tl.grid;
  if (!c.active[g]) return;
  const GridDesc& G = grids[g];
  const int nx = G.nx, ny = G.ny;
  const int64_t P = (int64_t)nx * ny;
  const int vi = c.vidx[g];
  const double* __restrict__ v = G.v[vi];
  const T* __restrict__ d = static_cast<const T*>(G.d[din]);
  const int x0 = tl.x0, y0 = tl.y0;

  for (int k = threadIdx.x; k < NL * HY * HX; k += kThreads) {
    const int l = k / (HY * HX);
    const int rem = k - l * (HY * HX);
    const int yy = rem / HX, xx = rem - yy * HX;
    const int x = x0 - 1 + xx, y = y0 - 1 + yy;
    double val = 0.0;
    if (x >= 0 && x < nx && y >= 0 && y < ny) {
      const int64_t i = l * P + (int64_t)y * nx + x;
      val = v[i];
      if (has_d) val += (double)d[i];
    }
    sv[l][yy][xx] = val;
  }
  __syncthreads();

  const double* __restrict__ gE = G.gE64;
  const double* __restrict__ gN = G.gN64;
  const double* __restrict__ gU = G.gU64;
  const double* __restrict__ D = G.D64;
  const double* __restrict__ b = G.b;
  double* __restrict__ vout = G.v[vi ^ 1];
  T* __restrict__ r = static_cast<T*>(G.r);
  double m = 0.0;
  for (int k = threadIdx.x; k < NL * TY * TX; k += kThreads) {
    const int l = k / (TY * TX);
    const int rem = k - l * (TY * TX);
    const int yy = rem / TX, xx = rem - yy * TX;
    const int x = x0 + xx, y = y0 + yy;
    if (x >= nx || y >= ny) continue;
    const int64_t i = l * P + (int64_t)y * nx + x;
    const int sx = xx + 1, sy = yy + 1;
    const double vc = sv[l][sy][sx];
    double acc = b[i] - D[i] * vc;
    acc += gE[i] * sv[l][sy][sx + 1];
    acc += gN[i] * sv[l][sy + 1][sx];
    if (x > 0) acc += gE[i - 1] * sv[l][sy][sx - 1];
    if (y > 0) acc += gN[i - nx] * sv[l][sy - 1][sx];
    if (NL > 1) {
      if (l < NL - 1) acc += gU[i] * sv[l + 1][sy][sx];
      if (l > 0) acc += gU[i - P] * sv[l - 1][sy][sx];
    }
    if (has_d) vout[i] = vc;
    r[i] = (T)acc;
    m = nan_max(m, fabs(acc) / D[i]);
  }
  // wavefront max, then across the block, then one atomic per block
  for (int off = 32; off > 0; off >>= 1) m = nan_max(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double bm = wmax[0];
    for (int w = 1; w < kThreads / 64; ++w) bm = nan_max(bm, wmax[w]);
    atomicMax(&c.norm_bits[g], (unsigned long long)__double_as_longlong(bm));
  }
}

// ------------------------------------------------------------------------------------
// One red-black SOR sweep on M d = r (eqs. 16-17), whole sweep per launch.
// ------------------------------------------------------------------------------------
template <typename T, int NL, int TY>
__global__ __launch_bounds__(kThreads) void k_sweep_rb(const Tile* __restrict__ tiles, int ntiles,
                                                      const GridDesc* __restrict__ grids, Ctl c,
                                                      int din, int zero_in, T omega) {
  constexpr int TX = kTileX, HX = TX + 4, HY = TY + 4;   // two-cell halo
  constexpr int RX = TX + 2, RY = TY + 2;                // red region: tile + one-cell ring
  __shared__ T sd[NL][HY][HX];
  const int ti = xcd_tile(ntiles);
  if (ti < 0) return;
  const Tile tl = tiles[ti];
  const int g = tl.grid;
  if (!c.active[g]) return;
  const GridDesc& G = grids[g];
  const int nx = G.nx, ny = G.ny;
  const int64_t P = (int64_t)nx * ny;
  const int x0 = tl.x0, y0 = tl.y0;
  const T* __restrict__ dold = static_cast<const T*>(G.d[din]);
  T* __restrict__ dnew = static_cast<T*>(G.d[din ^ 1]);
  const T* __restrict__ gE = static_cast<const T*>(G.gEs);
  const T* __restrict__ gN = static_cast<const T*>(G.gNs);
  const T* __restrict__ gU = static_cast<const T*>(G.gUs);
  const T* __restrict__ invD = static_cast<const T*>(G.invDs);
  const T* __restrict__ r = static_cast<const T*>(G.r);

  // stage the old correction with a two-cell halo (zero outside the grid)
  for (int k = threadIdx.x; k < NL * HY * HX; k += kThreads) {
    const int l = k / (HY * HX);
    const int rem = k - l * (HY * HX);
    const int yy = rem / HX, xx = rem - yy * HX;
    const int x = x0 - 2 + xx, y = y0 - 2 + yy;
    T val = T(0);
    if (!zero_in && x >= 0 && x < nx && y >= 0 && y < ny) val = dold[l * P + (int64_t)y * nx + x];
    sd[l][yy][xx] = val;
  }
  __syncthreads();

  // red half-sweep on the tile and its one-cell ring, from old black values
  for (int k = threadIdx.x; k < NL * RY * RX; k += kThreads) {
    const int l = k / (RY * RX);
    const int rem = k - l * (RY * RX);
    const int yy = rem / RX, xx = rem - yy * RX;
    const int x = x0 - 1 + xx, y = y0 - 1 + yy;
    if (((x + y + l) & 1) != 0) continue;
    if (x < 0 || x >= nx || y < 0 || y >= ny) continue;
    const int64_t i = l * P + (int64_t)y * nx + x;
    const int sx = xx + 1, sy = yy + 1;
    T acc = r[i];
    acc += gE[i] * sd[l][sy][sx + 1];
    acc += gN[i] * sd[l][sy + 1][sx];
    if (x > 0) acc += gE[i - 1] * sd[l][sy][sx - 1];
    if (y > 0) acc += gN[i - nx] * sd[l][sy - 1][sx];
    if (NL > 1) {
      if (l < NL - 1) acc += gU[i] * sd[l + 1][sy][sx];
      if (l > 0) acc += gU[i - P] * sd[l - 1][sy][sx];
    }
    const T old = sd[l][sy][sx];
    sd[l][sy][sx] = old + omega * (invD[i] * acc - old);
  }
  __syncthreads();

  // black half-sweep on the tile from the new red values; write the whole tile
  for (int k = threadIdx.x; k < NL * TY * TX; k += kThreads) {
    const int l = k / (TY * TX);
    const int rem = k - l * (TY * TX);
    const int yy = rem / TX, xx = rem - yy * TX;
    const int x = x0 + xx, y = y0 + yy;
    if (x >= nx || y >= ny) continue;
    const int64_t i = l * P + (int64_t)y * nx + x;
    const int sx = xx + 2, sy = yy + 2;
    T val = sd[l][sy][sx];
    if ((x + y + l) & 1) {
      T acc = r[i];
      acc += gE[i] * sd[l][sy][sx + 1];
      acc += gN[i] * sd[l][sy + 1][sx];
      if (x > 0) acc += gE[i - 1] * sd[l][sy][sx - 1];
      if (y > 0) acc += gN[i - nx] * sd[l][sy - 1][sx];
      if (NL > 1) {
        if (l < NL - 1) acc += gU[i] * sd[l + 1][sy][sx];
        if (l > 0) acc += gU[i - P] * sd[l - 1][sy][sx];
      }
      val = val + omega * (invD[i] * acc - val);
    }
    dnew[i] = val;
  }
}

// Weighted Jacobi sweep: every node from the previous sweep's values.
template <typename T, int NL, int TY>
__global__ __launch_bounds__(kThreads) void k_sweep_jacobi(const Tile* __restrict__ tiles, int ntiles,
                                                          const GridDesc* __restrict__ grids, Ctl c,
                                                          int din, int zero_in, T omega) {
  constexpr int TX = kTileX, HX = TX + 2, HY = TY + 2;
  __shared__ T sd[NL][HY][HX];
  const int ti = xcd_tile(ntiles);
  if (ti < 0) return;
  const Tile tl = tiles[ti];
  const int g = tl.grid;
  if (!c.active[g]) return;
  const GridDesc& G = grids[g];
  const int nx = G.nx, ny = G.ny;
  const int64_t P = (int64_t)nx * ny;
  const int x0 = tl.x0, y0 = tl.y0;
  const T* __restrict__ dold = static_cast<const T*>(G.d[din]);
  T* __restrict__ dnew = static_cast<T*>(G.d[din ^ 1]);
  const T* __restrict__ gE = static_cast<const T*>(G.gEs);
  const T* __restrict__ gN = static_cast<const T*>(G.gNs);
  const T* __restrict__ gU = static_cast<const T*>(G.gUs);
  const T* __restrict__ invD = static_cast<const T*>(G.invDs);
  const T* __restrict__ r = static_cast<const T*>(G.r);
  for (int k = threadIdx.x; k < NL * HY * HX; k += kThreads) {
    const int l = k / (HY * HX);
    const int rem = k - l * (HY * HX);
    const int yy = rem / HX, xx = rem - yy * HX;
    const int x = x0 - 1 + xx, y = y0 - 1 + yy;
    T val = T(0);
    if (!zero_in && x >= 0 && x < nx && y >= 0 && y < ny) val = dold[l * P + (int64_t)y * nx + x];
    sd[l][yy][xx] = val;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NL * TY * TX; k += kThreads) {
    const int l = k / (TY * TX);
    const int rem = k - l * (TY * TX);
    const int yy = rem / TX, xx = rem - yy * TX;
    const int x = x0 + xx, y = y0 + yy;
    if (x >= nx || y >= ny) continue;
    const int64_t i = l * P + (int64_t)y * nx + x;
    const int sx = xx + 1, sy = yy + 1;
    T acc = r[i];
    acc += gE[i] * sd[l][sy][sx + 1];
    acc += gN[i] * sd[l][sy + 1][sx];
    if (x > 0) acc += gE[i - 1] * sd[l][sy][sx - 1];
    if (y > 0) acc += gN[i - nx] * sd[l][sy - 1][sx];
    if (NL > 1) {
      if (l < NL - 1) acc += gU[i] * sd[l + 1][sy][sx];
      if (l > 0) acc += gU[i - P] * sd[l - 1][sy][sx];
    }
    const T old = sd[l][sy][sx];
    dnew[i] = old + omega * (invD[i] * acc - old);
  }
}

// ------------------------------------------------------------------------------------
// Inductor branch currents after the node solve (second line of eq. 10, companion form):
//   i(t+h) = alpha i(t) + g_eq (v_a - v_b)(t+h),  v_b = Vdd for a pad branch.
// ------------------------------------------------------------------------------------
__global__ void k_inductors(const GridDesc* __restrict__ grids, const int32_t* __restrict__ ind_grid,
                            const int32_t* __restrict__ ind_local, int n_total, Ctl c) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_total) return;
  const int g = ind_grid[j];
  const GridDesc& G = grids[g];
  const int k = ind_local[j];
  const int S = G.S;
  const double* __restrict__ v = G.v[c.vidx[g]];
  const int a = G.ind_a[k], bnode = G.ind_b[k];
  const double geq = G.ind_geq[k], al = G.ind_alpha[k];
  for (int s = 0; s < S; ++s) {
    const double vb = bnode >= 0 ? v[(int64_t)bnode * S + s] : G.vdd;
    const int64_t q = (int64_t)k * S + s;
    G.ind_i[q] = al * G.ind_i[q] + geq * (v[(int64_t)a * S + s] - vb);
  }
}

// ------------------------------------------------------------------------------------
// Launch wrappers
// ------------------------------------------------------------------------------------
static inline unsigned xcd_blocks(int ntiles) { return 8u * (unsigned)((ntiles + 7) / 8); }

hipError_t launch_step_begin(const Ctl& c, int G, hipStream_t s) {
  hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(256), 0, s, c, G);
  return hipGetLastError();
}

hipError_t launch_decide(const Ctl& c, int G, double tol, int has_d, int nchk, int max_sweeps,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(256), 0, s, c, G, tol, has_d, nchk, max_sweeps);
  return hipGetLastError();
}

hipError_t launch_step_end(const Ctl& c, int G, hipStream_t s) {
  hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, s, c, G);
  return hipGetLastError();
}

hipError_t launch_rhs(const Tile* tiles, int ntiles, int tile_rows, const GridDesc* grids,
                      const Ctl& c, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rhs, dim3(xcd_blocks(ntiles)), dim3(kThreads), 0, s, tiles, ntiles,
                     grids, c, tile_rows);
  return hipGetLastError();
}

hipError_t launch_sources(const SourceTable& src, const GridDesc* grids, double t, hipStream_t s) {
  if (src.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sources, dim3((src.count + 255) / 256), dim3(256), 0, s, src, grids, t);
  return hipGetLastError();
}

hipError_t launch_inductors(const GridDesc* grids, const int32_t* ind_grid, const int32_t* ind_local,
                            int n_total, const Ctl& c, hipStream_t s) {
  if (n_total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_inductors, dim3((n_total + 255) / 256), dim3(256), 0, s, grids, ind_grid,
                     ind_local, n_total, c);
  return hipGetLastError();
}

template <typename T, int NL, int TY>
static void resid_t(const Tile* tiles, int ntiles, const GridDesc* grids, const Ctl& c, int has_d,
                    int din, hipStream_t s) {
  hipLaunchKernelGGL((k_resid<T, NL, TY>), dim3(xcd_blocks(ntiles)), dim3(kThreads), 0, s, tiles,
                     ntiles, grids, c, has_d, din);
}

template <typename T, int NL, int TY>
static void sweep_t(int ordering, const Tile* tiles, int ntiles, const GridDesc* grids, const Ctl& c,
                    int din, int zero_in, double omega, hipStream_t s) {
  if (ordering == 1)
    hipLaunchKernelGGL((k_sweep_jacobi<T, NL, TY>), dim3(xcd_blocks(ntiles)), dim3(kThreads), 0, s,
                       tiles, ntiles, grids, c, din, zero_in, (T)omega);
  else
    hipLaunchKernelGGL((k_sweep_rb<T, NL, TY>), dim3(xcd_blocks(ntiles)), dim3(kThreads), 0, s,
                       tiles, ntiles, grids, c, din, zero_in, (T)omega);
}

#define PG_DISPATCH_NL_TY(FN, T, ...)                                   \
  switch (nl * 100 + tile_rows) {                                       \
    case 108: FN<T, 1, 8>(__VA_ARGS__); break;                          \
    case 116: FN<T, 1, 16>(__VA_ARGS__); break;                         \
    case 132: FN<T, 1, 32>(__VA_ARGS__); break;                         \
    case 208: FN<T, 2, 8>(__VA_ARGS__); break;                          \
    case 216: FN<T, 2, 16>(__VA_ARGS__); break;                         \
    case 232: FN<T, 2, 32>(__VA_ARGS__); break;                         \
    case 308: FN<T, 3, 8>(__VA_ARGS__); break;                          \
    case 316: FN<T, 3, 16>(__VA_ARGS__); break;                         \
    case 332: FN<T, 3, 32>(__VA_ARGS__); break;                         \
    case 408: FN<T, 4, 8>(__VA_ARGS__); break;                          \
    case 416: FN<T, 4, 16>(__VA_ARGS__); break;                         \
    case 432: FN<T, 4, 32>(__VA_ARGS__); break;                         \
    default: return hipErrorInvalidValue;                               \
  }

hipError_t launch_resid(bool fp32, int nl, int tile_rows, const Tile* tiles, int ntiles,
                        const GridDesc* grids, const Ctl& c, int has_d, int din, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (fp32) {
    PG_DISPATCH_NL_TY(resid_t, float, tiles, ntiles, grids, c, has_d, din, s)
  } else {
    PG_DISPATCH_NL_TY(resid_t, double, tiles, ntiles, grids, c, has_d, din, s)
  }
  return hipGetLastError();
}

hipError_t launch_sweep(bool fp32, int ordering, int nl, int tile_rows, const Tile* tiles, int ntiles,
                        const GridDesc* grids, const Ctl& c, int din, int zero_in, double omega,
                        hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (fp32) {
    PG_DISPATCH_NL_TY(sweep_t, float, ordering, tiles, ntiles, grids, c, din, zero_in, omega, s)
  } else {
    PG_DISPATCH_NL_TY(sweep_t, double, ordering, tiles, ntiles, grids, c, din, zero_in, omega, s)
  }
  return hipGetLastError();
}

}  // namespace pgrid
