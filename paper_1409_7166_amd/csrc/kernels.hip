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
// Memory layout: per-node arrays in natural order with an aligned row pitch.  A workgroup
// owns a 128 x TY tile through all layers; lane j of row-wave w owns the node pair
// (x0 + 2j, x0 + 2j + 1) of tile row w.  Because x0 is even, exactly one node of every pair is
// red, so both half-sweeps keep every lane busy, and all global traffic is 8- or 16-byte pair
// accesses.  The old correction is staged in LDS with a two-node, two-row halo; the red
// half-sweep is also evaluated on a one-node ring around the tile so the black half-sweep sees
// exactly the red values a global red-black sweep produces.  One launch therefore performs a
// whole sweep (ping-pong buffers, no grid-wide barrier), and the black node's coefficients,
// loaded with its red partner's, stay in registers between the two halves.
#include <algorithm>
#include <cfloat>

#include "mesh_tile.h"

namespace pgrid {

// ------------------------------------------------------------------------------------
// Step bookkeeping
// ------------------------------------------------------------------------------------
// First index i in [0, n] with a[i] >= key (a[i] > key if strict) of the ascending array a,
// found by the whole block: every round probes blockDim.x evenly spaced entries of the remaining
// range, so a search takes log_blockDim(n) rounds of one load each.  Called by every thread.
__device__ int block_lower_bound(const double* __restrict__ a, int n, double key, bool strict) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int step = (hi - lo + (int)blockDim.x - 1) / (int)blockDim.x;
    const int p = lo + (int)threadIdx.x * step;
    int below = 0;
    if (p < hi) below = strict ? (a[p] <= key) : (a[p] < key);
    const int k = __syncthreads_count(below);  // probes 0..k-1 lie below the answer
    const int nlo = k == 0 ? lo : lo + (k - 1) * step + 1;
    hi = min(hi, lo + k * step);
    lo = nlo;
  }
  return lo;
}

// Open a step on the device (the whole block): activate every item (only_item < 0) or one item,
// reset its per-step control, set t = (step + 1) h and the window of sources that can be
// non-zero at t.  win_a >= 0: the window's bounds [win_a, win_b) in the windowed sources, found
// by the host for the step it knows will be opened; else searched here.
__device__ void step_begin_block(const Ctl& c, int I, int only_item, double h, const SourceTable& src,
                                 int win_a, int win_b, long long step = -1) {
  for (int g = threadIdx.x; g < I; g += blockDim.x) {
    c.active[g] = (only_item < 0 || g == only_item) ? 1 : 0;
    c.step_sweeps[g] = 0;
    c.failed[g] = 0;
    c.norm_bits[g] = 0ull;
  }
  const double t = (double)((step >= 0 ? step : c.step[0]) + 1) * h;
  // windowed sources whose first breakpoint lies in [t - widest window, t]
  const int a = win_a >= 0 ? win_a : block_lower_bound(src.win_t0, src.n_window, t - src.win_maxw, false);
  const int b = win_a >= 0 ? win_b : block_lower_bound(src.win_t0, src.n_window, t, true);
  if (threadIdx.x == 0) {
    c.t_now[0] = t;
    c.src_window[0] = src.n_always + a;
    c.src_window[1] = b - a;
  }
}

__global__ void k_step_begin(Ctl c, int I, int only_item, double h, SourceTable src, int win_a, int win_b) {
  if (*c.stall) return;
  step_begin_block(c, I, only_item, h, src, win_a, win_b);
}

// Sum / max over the 64 lanes of a wavefront (every lane gets the result).
__device__ __forceinline__ long long wave_sum(long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// The decision after a residual pass (one block): per item,
// converged when its scaled residual is <= tol, failed when its sweep budget is spent; writes
// the accounting words and the tagged flag of this decision to host-visible memory.
__device__ void decide_block(const Ctl& c, const DecideArgs& da) {
  const int I = da.I, G = da.G, has_d = da.has_d, nchk = da.nchk, max_sweeps = da.max_sweeps;
  const int nslots = da.nslots;
  const double tol = da.tol;
  const GridDesc* __restrict__ grids = da.grids;
  __shared__ int any;
  __shared__ int worked;
  __shared__ unsigned long long act_nodes, act_coef, act_rcoef;
  if (*c.stall) {  // a stalled opening: keep the sequence, report the decision as skipped
    if (threadIdx.x == 0) {
      const uint32_t seq = c.flag_seq[0];
      const uint32_t slot = seq & (uint32_t)(nslots - 1);
      c.flag_seq[0] = seq + 1u;
      const long long tag = (long long)(((unsigned long long)seq & 0xffffffull) << 40);
      c.acct[3 * slot] = tag;
      c.acct[3 * slot + 1] = tag;
      c.acct[3 * slot + 2] = tag;
      c.any_active[slot] = (int32_t)((seq & 0x1fffffffu) << 2 | 2u);
    }
    return;
  }
  // every load the decision needs is issued up front, so the block waits for memory about once:
  // the item's state, its mesh nodes and grid, each grid's coefficient words, the flag sequence
  constexpr int kMaxGridWords = 1024;
  __shared__ unsigned int gbits[kMaxGridWords];
  __shared__ uint32_t seq_s;
  const bool bitmap = G <= 32 * kMaxGridWords;
  const int nwords = bitmap ? (G + 31) / 32 : 0;
  long long coef_mine = 0, rcoef_mine = 0;  // coefficient words of grid threadIdx.x (the common case G <= blockDim)
  if (bitmap && (int)threadIdx.x < G) {
    coef_mine = grids[threadIdx.x].coef_words;
    rcoef_mine = grids[threadIdx.x].resid_words;
  }
  if (threadIdx.x == 0) {
    any = 0; worked = 0; act_nodes = 0ull; act_coef = 0ull; act_rcoef = 0ull;
    seq_s = c.flag_seq[0];
  }
  for (int w = threadIdx.x; w < nwords; w += blockDim.x) gbits[w] = 0u;
  __syncthreads();
  long long mine = 0;
  for (int g = threadIdx.x; g < I; g += blockDim.x) {
    const int was = c.active[g];
    const long long nodes = c.nodes[g];
    const int gi = c.item_grid[g];
    const int swept = c.step_sweeps[g];
    // the other workgroups' atomicMax results, read at device scope (not from a stale L1 line)
    const double nm = __longlong_as_double(
        (long long)__hip_atomic_load(&c.norm_bits[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (was) {
      atomicOr(&worked, 1);
      const int sw = has_d ? swept + nchk : swept;
      if (has_d) {
        c.vidx[g] ^= 1;
        c.step_sweeps[g] = sw;
      }
      c.last_norm[g] = nm;
      const bool conv = nm <= tol;                 // false for NaN
      const bool spent = sw >= max_sweeps;
      const int act = (!conv && !spent) ? 1 : 0;
      c.active[g] = act;
      if (!conv && spent) c.failed[g] = 1;
      if (act) {
        atomicOr(&any, 1);
        // the work the next sweeps will do: active scenarios, and the coefficients of the grids
        // with an active scenario (marked in a bitmap of grids)
        mine += nodes;
        if (bitmap) atomicOr(&gbits[gi >> 5], 1u << (gi & 31));
      }
    }
    c.norm_bits[g] = 0ull;
  }
  mine = wave_sum(mine);
  if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&act_nodes, (unsigned long long)mine);
  __syncthreads();
  for (int gi = threadIdx.x; gi < G; gi += blockDim.x) {
    bool any_in_grid = false;
    long long words, rwords;
    if (bitmap) {
      any_in_grid = (gbits[gi >> 5] >> (gi & 31)) & 1u;
      words = gi == (int)threadIdx.x ? coef_mine : grids[gi].coef_words;
      rwords = gi == (int)threadIdx.x ? rcoef_mine : grids[gi].resid_words;
    } else {
      const GridDesc& D = grids[gi];
      for (int sc = 0; sc < D.S && !any_in_grid; ++sc) any_in_grid = c.active[D.item0 + sc] != 0;
      words = D.coef_words;
      rwords = D.resid_words;
    }
    if (any_in_grid) {
      atomicAdd(&act_coef, (unsigned long long)words);
      atomicAdd(&act_rcoef, (unsigned long long)rwords);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t seq = seq_s;
    const uint32_t slot = seq & (uint32_t)(nslots - 1);
    const long long checks = worked ? c.stat_checks[0] : 0;
    c.flag_seq[0] = seq + 1u;
    // each accounting word carries the low 24 bits of the sequence above its 40-bit value, so the
    // host sees when it has arrived and no fence is needed before the flag
    const unsigned long long tag = ((unsigned long long)seq & 0xffffffull) << 40;
    constexpr unsigned long long kValue = (1ull << 40) - 1;
    c.acct[3 * slot] = (long long)(tag | (act_nodes & kValue));
    c.acct[3 * slot + 1] = (long long)(tag | (act_coef & kValue));
    c.acct[3 * slot + 2] = (long long)(tag | (act_rcoef & kValue));
    c.any_active[slot] = (int32_t)((seq & 0x1fffffffu) << 2 | (uint32_t)any);
    if (worked) c.stat_checks[0] = checks + 1;
  }
}



// Close a step: count_step 1 adds the step's statistics and advances the clock, 2 only advances
// the clock, 0 does neither; the failure flag is always gathered.  Items still iterating mean the
// close was queued ahead of the step's last decision: set the stall flag and do nothing.  With
// begin_next the same block then opens the next step (step_begin_block for every item).
__device__ void close_block(const Ctl& c, int I, int count_step, int begin_next, double h, const SourceTable& src,
                            int win_a, int win_b) {
  __shared__ long long s_sw[4], s_upd[4];
  __shared__ int s_mx[4], s_fail[4], s_act[4];
  __shared__ double s_res[4];
  if (*c.stall) return;
  long long sw = 0, upd = 0;
  int mx = 0, fail = 0, act = 0;
  double res = 0.0;
  for (int g = threadIdx.x; g < I; g += blockDim.x) {
    const int s = c.step_sweeps[g];
    sw += s;
    upd += (long long)s * c.nodes[g];
    mx = s > mx ? s : mx;
    res = nan_max(res, c.last_norm[g]);
    fail |= c.failed[g];
    act |= c.active[g];
  }
  // reduce within each wavefront, then over the block's wavefronts
  act = wave_max(act);
  sw = wave_sum(sw);
  upd = wave_sum(upd);
  mx = wave_max(mx);
  fail = wave_max(fail);
  for (int o = 32; o > 0; o >>= 1) res = nan_max(res, __shfl_xor(res, o, 64));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_sw[w] = sw; s_upd[w] = upd; s_mx[w] = mx; s_fail[w] = fail; s_res[w] = res; s_act[w] = act;
  }
  __syncthreads();
  // thread 0 completes the statistics from the other wavefronts' partial results; the
  // still-iterating test must be the same for every thread, since the block either returns
  // as a whole or goes on to the barriers of the next step's opening
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
    sw += s_sw[k]; upd += s_upd[k]; mx = max(mx, s_mx[k]); fail |= s_fail[k]; res = nan_max(res, s_res[k]);
  }
  int any_active = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) any_active |= s_act[k];
  if (any_active) {  // the step is still iterating: this close (and what was queued after it) must wait
    if (threadIdx.x == 0) c.stall[0] = 1;
    return;
  }
  __shared__ long long new_step;
  if (threadIdx.x == 0) {
    // every statistic is read before any is written, so the loads go out together
    const int f0 = c.stat_failed[0], mx0 = c.stat_max_sweeps[0];
    const long long sw0 = c.stat_sweeps[0], up0 = c.stat_updates[0], st0 = c.step[0];
    const double mr0 = c.stat_max_res[0];
    c.stat_failed[0] = f0 | fail;
    if (count_step == 1) {
      c.stat_sweeps[0] = sw0 + sw;
      c.stat_updates[0] = up0 + upd;
      c.stat_last_sweeps[0] = mx;
      c.stat_max_sweeps[0] = mx > mx0 ? mx : mx0;
      c.stat_last_res[0] = res;
      c.stat_max_res[0] = nan_max(mr0, res);
    }
    new_step = count_step ? st0 + 1 : st0;
    if (count_step) c.step[0] = new_step;
  }
  if (!begin_next) return;
  __syncthreads();  // the new step index is known to the block
  step_begin_block(c, I, -1, h, src, win_a, win_b, new_step);
}

__global__ void k_step_end(Ctl c, int I, int count_step, int begin_next, double h, SourceTable src,
                           int win_a, int win_b) {
  close_block(c, I, count_step, begin_next, h, src, win_a, win_b);
}

// A decision, optionally followed in the same block by the step's close (the opening of a step
// expected to converge at once carries its close, one launch fewer per such step).  Every value
// the close reads from the control block was written by the same thread in the decision.
__global__ void k_decide(Ctl c, DecideArgs da, CloseArgs ca) {
  decide_block(c, da);
  if (!ca.on) return;
  __syncthreads();
  close_block(c, da.I, ca.count_step, ca.begin_next, ca.h, ca.src, ca.win_a, ca.win_b);
}

// ------------------------------------------------------------------------------------
// Right-hand side of the step (eq. 2 / eq. 10): b = (C/h) v + G0 Vdd - inductor history.
// Sources are subtracted afterwards by k_sources.  predict = 1: also keep v(t) in vhist;
// predict = 2: also replace v by the step's first iterate 2 v(t) - v(t-h) (v(t-h) read from
// vhist) and keep v(t) in vhist; predict = 3: start from 3 v(t) - 3 v(t-h) + v(t-2h) (v(t-2h)
// read from vhist2).  With vhist2 present, the old vhist moves there.  A tile may be a block of
// Tile.pad consecutive scenarios of one
// grid: the shared C/h and G0 Vdd of a node pair are loaded once for all of them.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_rhs(const Tile* __restrict__ tiles, int ntiles,
                                             const GridDesc* __restrict__ grids, Ctl c, int predict) {
  if (*c.stall) return;  // a stalled step opening
  const int ti = xcd_tile(ntiles);
  if (ti < 0) return;
  const Tile tl = tiles[ti];
  const GridDesc& G = grids[tl.grid];
  const int X = G.X, ny = G.ny;
  // 64 x TY threads: thread (row w, lane j) owns the node pair (x0 + 2j, x0 + 2j + 1) of row
  // y0 + w in every layer, as in the sweeps (the pitch X is even, so a pair never straddles rows)
  const int x = tl.x0 + 2 * (int)(threadIdx.x & 63), y = tl.y0 + (int)(threadIdx.x >> 6);
  if (x >= X || y >= ny) return;
  const int64_t P = (int64_t)X * ny;
  for (int l = 0; l < G.nl; ++l) {
    const int64_t i = l * P + (int64_t)y * X + x;
    // layers with no capacitance (or no constant injection) contribute exact zeros
    const bool has_ch = (G.ch_layers >> l) & 1u;
    const double2 bcv = ((G.bc_layers >> l) & 1u) ? ld2(G.bconst64, i) : make_double2(0.0, 0.0);
    const double2 ch = has_ch ? ld2(G.ch64, i) : make_double2(0.0, 0.0);
    for (int s = 0; s < tl.pad; ++s) {
      const int64_t off = (int64_t)(tl.scen + s) * G.nstore;
      double* __restrict__ v = G.v[c.vidx[tl.item + s]] + off;
      const double2 vt = ld2(v, i);
      double2 bb = bcv;
      if (has_ch) {
        bb.x = ch.x * vt.x + bcv.x;
        bb.y = ch.y * vt.y + bcv.y;
      }
      if (G.n_ind) {
        const double* __restrict__ il = G.ind_i + (int64_t)(tl.scen + s) * G.n_ind;
        for (int q = 0; q < 2; ++q) {
          double h = q ? bb.y : bb.x;
          for (int j = G.inc_off[i + q]; j < G.inc_off[i + q + 1]; ++j) {
            const int e = G.inc_ind[j];
            const int kk = (e > 0 ? e : -e) - 1;
            const double term = G.ind_alpha[kk] * il[kk];
            h += (e > 0) ? -term : term;
          }
          if (q) bb.y = h; else bb.x = h;
        }
      }
      st2(G.b + off, i, bb);
      if (predict) {
        double* __restrict__ vh = G.vhist + off;
        double* __restrict__ vh2 = G.vhist2 ? G.vhist2 + off : nullptr;
        if (predict >= 2) {
          const double2 p1 = ld2(vh, i);
          if (predict == 3) {
            const double2 p2 = ld2(vh2, i);
            st2(v, i, make_double2(3.0 * (vt.x - p1.x) + p2.x, 3.0 * (vt.y - p1.y) + p2.y));
          } else {
            st2(v, i, make_double2(2.0 * vt.x - p1.x, 2.0 * vt.y - p1.y));
          }
          if (vh2) st2(vh2, i, p1);
        }
        st2(vh, i, vt);
      }
    }
  }
}

// Piecewise-linear current sources: b -= sign * I(t) at t = t_now + shift (sign 1, shift 0: the
// step's loads; the three-level recurrence also adds back the previous step's, shift -h and
// sign -1, which the window still covers because it is widened by a bucket of 8 steps).
// Grid-stride over the always-on sources and the window chosen by k_step_begin.
__global__ void k_sources(SourceTable src, const GridDesc* __restrict__ grids, Ctl c, double shift, double sign) {
  if (*c.stall) return;
  const double t = c.t_now[0] + shift;
  const int wbeg = c.src_window[0], wcnt = c.src_window[1];
  const int n = src.n_always + wcnt;
  const double* __restrict__ ts = src.t;
  const double* __restrict__ is = src.i;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const int k = q < src.n_always ? q : wbeg + (q - src.n_always);
    const int a = src.off[k], e = src.off[k + 1];
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
    G.b[src.index[k]] -= sign * I;
  }
}

// ------------------------------------------------------------------------------------
// FP64 residual r = b - M v' with v' = v + d, and the Jacobi-scaled norm max |r_i| / M_ii.
// Writes v' into the other voltage buffer (the decision kernel flips the index), and r in
// the sweep precision as the right-hand side of the next correction sweeps.
// Block: 64 x TY threads, lane j of row w owns the pair (x0 + 2j, x0 + 2j + 1) of row y0 + w.
// ------------------------------------------------------------------------------------
template <typename T, int NL, int TY>
__device__ void resid_tile(const Tile* __restrict__ tiles, int ti, const GridDesc* __restrict__ grids,
                           const Ctl& c, int has_d, int din, int fuse) {
  // fuse (the first pass of a step whose sources are all zero, has_d = 0): kFuseRhs forms b here;
  // kFuseProbe stores neither b nor r (only the norm counts); kFuseNoNorm stores b and r and
  // leaves the norm alone.  These passes form M_ii from the conductances they load and the pad
  // conductance G0 = (G0 Vdd) / Vdd, instead of reading it.
  const int fuse_rhs = fuse & kFuseRhs;
  const bool store = !(fuse & kFuseProbe), norm = !(fuse & kFuseNoNorm);
  constexpr int NP = kTileX / 2, HP = NP + 2, HY = TY + 2;
  constexpr int NT = 64 * TY;
  __shared__ double2 sv[NL][HY][HP];
  __shared__ double wmax[NT / 64];
  const Tile tl = tiles[ti];
  const int item = tl.item;
  if (!c.active[item]) return;
  const GridDesc& G = grids[tl.grid];
  const int nx = G.nx, ny = G.ny, X = G.X;
  const int64_t P = (int64_t)X * ny;
  const int64_t off = (int64_t)tl.scen * G.nstore;
  const int vi = c.vidx[item];
  const double* __restrict__ v = G.v[vi] + off;
  const T* __restrict__ d = static_cast<const T*>(G.d[din]) + off;
  const double* __restrict__ bvec = G.b + off;
  const int x0 = tl.x0, y0 = tl.y0;

  // stage v + d on the tile with a one-pair, one-row halo (zero outside the storage); each
  // thread issues all its loads before it writes any of them
  constexpr int NS = NL * HY * HP, SPT = (NS + NT - 1) / NT;
  double2 sval[SPT];
  V2<T> dval[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int k = threadIdx.x + q * NT;
    const int l = k / (HY * HP);
    const int rem = k - l * (HY * HP);
    const int hy = rem / HP, hp = rem - hy * HP;
    const int x = x0 - 2 + 2 * hp, y = y0 - 1 + hy;
    sval[q] = make_double2(0.0, 0.0);
    dval[q] = zero2<T>();
    if (k < NS && x >= 0 && x < X && y >= 0 && y < ny) {
      const int64_t i = l * P + (int64_t)y * X + x;
      sval[q] = ld2(v, i);
      if (has_d) dval[q] = ld2(d, i);
    }
  }
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int k = threadIdx.x + q * NT;
    if (k < NS) {
      double2 val = sval[q];
      val.x += (double)dval[q].x;
      val.y += (double)dval[q].y;
      (&sv[0][0][0])[k] = val;
    }
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int x = x0 + 2 * lane, y = y0 + row;
  const int hp = lane + 1, hy = row + 1;
  const bool dfly = fuse_rhs && G.vdd != 0.0;
  const double inv_vdd = dfly ? 1.0 / G.vdd : 0.0;
  double m = 0.0;
  if (x < X && y < ny) {
    double* __restrict__ vout = G.v[vi ^ 1] + off;
    T* __restrict__ r = static_cast<T*>(G.r) + off;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int64_t i = l * P + (int64_t)y * X + x;
      const double2 own = sv[l][hy][hp];
      double2 b2, ch2 = make_double2(0.0, 0.0), bc2 = make_double2(0.0, 0.0);
      if (fuse_rhs) {
        // the step's right-hand side formed here: b = (C/h) v + G0 Vdd - inductor history,
        // exactly as k_rhs forms it
        if ((G.ch_layers >> l) & 1u) ch2 = ld2(G.ch64, i);
        if ((G.bc_layers >> l) & 1u) bc2 = ld2(G.bconst64, i);
        b2.x = ch2.x * own.x + bc2.x;
        b2.y = ch2.y * own.y + bc2.y;
        if (G.n_ind) {
          const double* __restrict__ il = G.ind_i + (int64_t)tl.scen * G.n_ind;
          for (int q = 0; q < 2; ++q) {
            double bb = q ? b2.y : b2.x;
            for (int j = G.inc_off[i + q]; j < G.inc_off[i + q + 1]; ++j) {
              const int e = G.inc_ind[j];
              const int kk = (e > 0 ? e : -e) - 1;
              const double term = G.ind_alpha[kk] * il[kk];
              bb += (e > 0) ? -term : term;
            }
            if (q) b2.y = bb; else b2.x = bb;
          }
        }
        if (store) st2(G.b + off, i, b2);
      } else {
        b2 = ld2(bvec, i);
      }
      const double2 ge = ld2(G.gE64, i), gn = ld2(G.gN64, i);
      const double2 gs = y > 0 ? ld2(G.gN64, i - X) : make_double2(0.0, 0.0);
      const double gw = x > 0 ? ld1(G.gE64, i - 1) : 0.0;
      double2 gu = make_double2(0.0, 0.0), gd = make_double2(0.0, 0.0);
      if (NL > 1) {
        if (l < NL - 1) gu = ld2(G.gU64, i);
        if (l > 0) gd = ld2(G.gU64, i - P);
      }
      double2 D2;
      if (dfly) {  // node x: east ge.x, west gw; node x + 1: east ge.y, west ge.x
        D2.x = mesh_diag(ch2.x, ge.x, gw, gn.x, gs.x, gu.x, gd.x, bc2.x * inv_vdd);
        D2.y = mesh_diag(ch2.y, ge.y, ge.x, gn.y, gs.y, gu.y, gd.y, bc2.y * inv_vdd);
      } else {
        D2 = ld2(G.D64, i);
      }
      const double2 eastp = sv[l][hy][hp + 1], westp = sv[l][hy][hp - 1];
      const double2 nth = sv[l][hy + 1][hp], sth = sv[l][hy - 1][hp];
      double2 up = make_double2(0.0, 0.0), dn = make_double2(0.0, 0.0);
      if (NL > 1) {
        if (l < NL - 1) up = sv[l + 1][hy][hp];
        if (l > 0) dn = sv[l - 1][hy][hp];
      }
      double r0 = b2.x - D2.x * own.x + ge.x * own.y + gw * westp.y + gn.x * nth.x + gs.x * sth.x +
                  gu.x * up.x + gd.x * dn.x;
      double r1 = b2.y - D2.y * own.y + ge.y * eastp.x + ge.x * own.x + gn.y * nth.y + gs.y * sth.y +
                  gu.y * up.y + gd.y * dn.y;
      if (x >= nx) r0 = 0.0;
      if (x + 1 >= nx) r1 = 0.0;
      if (has_d) st2(vout, i, own);
      if (store) {
        V2<T> rr;
        rr.x = (T)r0;
        rr.y = (T)r1;
        st2(r, i, rr);
      }
      if (x < nx) m = nan_max(m, fabs(r0) / D2.x);
      if (x + 1 < nx) m = nan_max(m, fabs(r1) / D2.y);
    }
  }
  if (!norm) return;  // uniform over the block
  // wavefront max, then across the block, then one atomic per block
  for (int off = 32; off > 0; off >>= 1) m = nan_max(m, __shfl_xor(m, off, 64));
  if (lane == 0) wmax[row] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double bm = wmax[0];
    for (int w = 1; w < NT / 64; ++w) bm = nan_max(bm, wmax[w]);
    atomicMax(&c.norm_bits[item], (unsigned long long)__double_as_longlong(bm));
  }
}

template <typename T, int NL, int TY>
__global__ __launch_bounds__(64 * TY) void k_resid(const Tile* __restrict__ tiles, int ntiles,
                                                  const GridDesc* __restrict__ grids, Ctl c,
                                                  int has_d, int din, int fuse) {
  const int ti = xcd_tile(ntiles);
  if (!*c.stall && ti >= 0) resid_tile<T, NL, TY>(tiles, ti, grids, c, has_d, din, fuse);
}

// ------------------------------------------------------------------------------------
// The opening probe of a step predicted to converge at once (sources all zero, v' = v, a
// non-zero supply on every mesh): only the norm of r = b - M v is wanted, and only to learn
// whether it is below the tolerance.  The C/h terms of b and of M v cancel exactly there, and
// with the deviations e_i = v_i - Vdd
//   r_i = -G0_i e_i - history_i + sum_j g_ij (e_j - e_i),   G0_i = (G0 Vdd)_i / Vdd.
// The probe stages e in FP32 and forms the conductance terms in FP32 from the sweeps' copies of
// the conductances and of 1/M_ii.  Every rounding in that (of e, of g and G0 to FP32, of the
// differences, products and the sum of at most eight terms) is a relative error of at most
// u = 2^-24 on a term of S_i = G0_i |e_i| + sum_j g_ij (|e_i| + |e_j|), about 11 u S_i in all, so
// |r_i| <= |r~_i| + 2^-19 S~_i with the computed S~_i; the scale 1/M_ii is widened by its own
// rounding.  The probe's norm therefore bounds the FP64 residual norm from above: a step it
// passes has converged, and one it fails gets the FP64 passes (the bound only costs work when
// the tolerance is close to 2^-19 S_i / M_ii).
// ------------------------------------------------------------------------------------
template <typename T, int NL, int TY, bool IND>
__device__ void probe_tile(const Tile* __restrict__ tiles, int ti, const GridDesc* __restrict__ grids,
                           const Ctl& c) {
  constexpr int NP = kTileX / 2, HP = NP + 2, HY = TY + 2;
  constexpr int NT = 64 * TY;
  constexpr float kBound = 0x1p-19f;
  constexpr double kWiden = sizeof(T) == 4 ? 1.0 + 0x1p-22 : 1.0 + 0x1p-51;
  __shared__ float2 se[NL][HY][HP];
  __shared__ double wmax[NT / 64];
  const Tile tl = tiles[ti];
  const int item = tl.item;
  if (!c.active[item]) return;
  const GridDesc& G = grids[tl.grid];
  const int nx = G.nx, ny = G.ny, X = G.X;
  const int64_t P = (int64_t)X * ny;
  const int64_t off = (int64_t)tl.scen * G.nstore;
  const double vdd = G.vdd;
  const double* __restrict__ v = G.v[c.vidx[item]] + off;
  const T* __restrict__ sE = static_cast<const T*>(G.gEs);
  const T* __restrict__ sN = static_cast<const T*>(G.gNs);
  const T* __restrict__ sU = static_cast<const T*>(G.gUs);
  const T* __restrict__ sI = static_cast<const T*>(G.invDs);
  const int x0 = tl.x0, y0 = tl.y0;

  // stage e = v - Vdd on the tile with a one-pair, one-row halo (zero outside the storage, where
  // every conductance to the tile is zero)
  constexpr int NS = NL * HY * HP, SPT = (NS + NT - 1) / NT;
  double2 sval[SPT];
  bool sin[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int k = threadIdx.x + q * NT;
    const int l = k / (HY * HP);
    const int rem = k - l * (HY * HP);
    const int hy = rem / HP, hp = rem - hy * HP;
    const int gx = x0 - 2 + 2 * hp, gy = y0 - 1 + hy;
    sin[q] = k < NS && gx >= 0 && gx < X && gy >= 0 && gy < ny;
    sval[q] = make_double2(vdd, vdd);
    if (sin[q]) sval[q] = ld2(v, l * P + (int64_t)gy * X + gx);
  }
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int k = threadIdx.x + q * NT;
    if (k < NS) (&se[0][0][0])[k] = make_float2((float)(sval[q].x - vdd), (float)(sval[q].y - vdd));
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int x = x0 + 2 * lane, y = y0 + row;
  const int hp = lane + 1, hy = row + 1;
  const double inv_vdd = 1.0 / vdd;
  double m = 0.0;
  if (x < X && y < ny) {
    // one layer's words; the next layer's loads are issued before this layer is evaluated
    struct Words {
      NV2<T> ge, gn, gs, gu, gd, iv;
      T gw;
      NV2<double> bc;
    };
    auto load = [&](int l, Words& w) {
      const int64_t i = l * P + (int64_t)y * X + x;
      const NV2<T> z = {T(0), T(0)};
      w.ge = ld2n(sE, i);
      w.gn = ld2n(sN, i);
      w.iv = ld2n(sI, i);
      w.gs = y > 0 ? ld2n(sN, i - X) : z;
      w.gw = x > 0 ? ld1(sE, i - 1) : T(0);
      w.gu = z;
      w.gd = z;
      if (NL > 1) {
        if (l < NL - 1) w.gu = ld2n(sU, i);
        if (l > 0) w.gd = ld2n(sU, i - P);
      }
      w.bc = NV2<double>{0.0, 0.0};
      if ((G.bc_layers >> l) & 1u) w.bc = ld2n(G.bconst64, i);
    };
    // (with inductors the history loop needs the registers: each layer loads as it starts)
    Words cur, nxt;
    load(0, cur);
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      if (IND) {
        if (l > 0) load(l, cur);
      } else if (l + 1 < NL) {
        load(l + 1, nxt);
      }
      const int64_t i = l * P + (int64_t)y * X + x;
      const NV2<T> ge = cur.ge, gn = cur.gn, gs = cur.gs, gu = cur.gu, gd = cur.gd, iv = cur.iv;
      const T gw = cur.gw;
      const float2 pad = make_float2((float)(cur.bc.x * inv_vdd), (float)(cur.bc.y * inv_vdd));
      double2 hist = make_double2(0.0, 0.0);
      if (IND && G.n_ind) {  // history_i: alpha_k i_k summed over branches k leaving node i, minus entering
        const double* __restrict__ il = G.ind_i + (int64_t)tl.scen * G.n_ind;
        for (int q = 0; q < 2; ++q) {
          double hh = 0.0;
          for (int j = G.inc_off[i + q]; j < G.inc_off[i + q + 1]; ++j) {
            const int e = G.inc_ind[j];
            const int kk = (e > 0 ? e : -e) - 1;
            const double term = G.ind_alpha[kk] * il[kk];
            hh += (e > 0) ? term : -term;
          }
          if (q) hist.y = hh; else hist.x = hh;
        }
      }
      const float2 own = se[l][hy][hp], eastp = se[l][hy][hp + 1], westp = se[l][hy][hp - 1];
      const float2 nth = se[l][hy + 1][hp], sth = se[l][hy - 1][hp];
      float2 up = make_float2(0.0f, 0.0f), dn = make_float2(0.0f, 0.0f);
      if (NL > 1) {
        if (l < NL - 1) up = se[l + 1][hy][hp];
        if (l > 0) dn = se[l - 1][hy][hp];
      }
      // node x: east is node x + 1 (ge.x), west gw; node x + 1: east ge.y, west node x (ge.x)
      const float e0 = own.x, e1 = own.y, a0 = fabsf(e0), a1 = fabsf(e1);
      const float n0[6] = {e1, westp.y, nth.x, sth.x, up.x, dn.x};
      const float n1[6] = {eastp.x, e0, nth.y, sth.y, up.y, dn.y};
      const float g0[6] = {(float)ge.x, (float)gw, (float)gn.x, (float)gs.x, (float)gu.x, (float)gd.x};
      const float g1[6] = {(float)ge.y, (float)ge.x, (float)gn.y, (float)gs.y, (float)gu.y, (float)gd.y};
      float r0 = -pad.x * e0, r1 = -pad.y * e1, s0 = pad.x * a0, s1 = pad.y * a1;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        r0 += g0[k] * (n0[k] - e0);
        r1 += g1[k] * (n1[k] - e1);
        s0 += g0[k] * (a0 + fabsf(n0[k]));
        s1 += g1[k] * (a1 + fabsf(n1[k]));
      }
      const double q0 = fabs((double)r0 - hist.x) + (double)(kBound * s0);
      const double q1 = fabs((double)r1 - hist.y) + (double)(kBound * s1);
      if (x < nx) m = nan_max(m, q0 * ((double)iv.x * kWiden));
      if (x + 1 < nx) m = nan_max(m, q1 * ((double)iv.y * kWiden));
      if (!IND && l + 1 < NL) cur = nxt;
    }
  }
  for (int o = 32; o > 0; o >>= 1) m = nan_max(m, __shfl_xor(m, o, 64));
  if (lane == 0) wmax[row] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double bm = wmax[0];
    for (int w = 1; w < NT / 64; ++w) bm = nan_max(bm, wmax[w]);
    atomicMax(&c.norm_bits[item], (unsigned long long)__double_as_longlong(bm));
  }
}

// IND: some grid carries inductors (their history enters b); without them the probe has no
// data-dependent branch between its loads.
template <typename T, int NL, int TY, bool IND>
__global__ __launch_bounds__(64 * TY) void k_probe(const Tile* __restrict__ tiles, int ntiles,
                                                   const GridDesc* __restrict__ grids, Ctl c) {
  const int ti = xcd_tile(ntiles);
  if (!*c.stall && ti >= 0) probe_tile<T, NL, TY, IND>(tiles, ti, grids, c);
}

// ------------------------------------------------------------------------------------
// One red-black SOR sweep on M d = r (eqs. 16-17), a whole sweep per launch.
// ------------------------------------------------------------------------------------
template <typename T, int NL, int TY>
__global__ __launch_bounds__(64 * TY) void k_sweep_rb(const Tile* __restrict__ tiles, int ntiles,
                                                     const GridDesc* __restrict__ grids, Ctl c,
                                                     int din, int zero_in, T omega) {
  constexpr int NP = kTileX / 2;      // pairs per tile row
  constexpr int HP = NP + 2;          // staged pairs per row (one halo pair each side)
  constexpr int HY = TY + 4;          // staged rows (two halo rows each side)
  constexpr int NT = 64 * TY;
  __shared__ V2<T> sd[NL][HY][HP];
  const int ti = xcd_tile(ntiles);
  if (ti < 0) return;
  const Tile tl = tiles[ti];
  if (!c.active[tl.item]) return;
  const GridDesc& G = grids[tl.grid];
  const int ny = G.ny, X = G.X;
  const int64_t P = (int64_t)X * ny;
  const int64_t off = (int64_t)tl.scen * G.nstore;
  const int x0 = tl.x0, y0 = tl.y0;
  const T* __restrict__ dold = static_cast<const T*>(G.d[din]) + off;
  T* __restrict__ dnew = static_cast<T*>(G.d[din ^ 1]) + off;
  const T* __restrict__ gE = static_cast<const T*>(G.gEs);
  const T* __restrict__ gN = static_cast<const T*>(G.gNs);
  const T* __restrict__ gU = static_cast<const T*>(G.gUs);
  const T* __restrict__ invD = static_cast<const T*>(G.invDs);
  const T* __restrict__ r = static_cast<const T*>(G.r) + off;

  // stage the old correction (zero outside the storage, and everywhere on a cold start); each
  // thread issues all its loads before it writes any of them
  constexpr int NS = NL * HY * HP, SPT = (NS + NT - 1) / NT;
  V2<T> sval[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int k = threadIdx.x + q * NT;
    const int l = k / (HY * HP);
    const int rem = k - l * (HY * HP);
    const int hy = rem / HP, hp = rem - hy * HP;
    const int x = x0 - 2 + 2 * hp, y = y0 - 2 + hy;
    sval[q] = zero2<T>();
    if (!zero_in && k < NS && x >= 0 && x < X && y >= 0 && y < ny) sval[q] = ld2(dold, l * P + (int64_t)y * X + x);
  }
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int k = threadIdx.x + q * NT;
    if (k < NS) (&sd[0][0][0])[k] = sval[q];
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int x = x0 + 2 * lane, y = y0 + row;
  const int hp = lane + 1, hy = row + 2;
  const bool mine = x < X && y < ny;

  // red half-sweep on the owned pairs; keep the black partner's coefficients.  Each layer's
  // update runs while the next layer's loads are in flight.
  NodeCoef<T> keep[NL];
  if (mine) {
    PairRaw<T> cur, nxt;
    load_pair_raw<T, NL>(G, gE, gN, gU, invD, r, 0, y, x, cur);
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      if (l + 1 < NL) load_pair_raw<T, NL>(G, gE, gN, gU, invD, r, l + 1, y, x, nxt);
      const int er = (y + l) & 1;  // x is even: the pair's red node is x + er
      keep[l] = node_of(cur, 1 - er);
      const T nv = relax<T, NL, HY, HP>(sd, l, hy, hp, er, node_of(cur, er), omega);
      put(sd[l][hy][hp], er, nv);
      if (l + 1 < NL) cur = nxt;
    }
  }
  // red half-sweep on the one-node ring: rows y0-1 and y0+TY (tile columns), and the
  // columns x0-1 and x0+TX (tile rows).  Only the ring node of each edge pair is updated, so
  // only its words are loaded.
  constexpr int NRING = 2 * NP + 2 * TY;
  for (int k = threadIdx.x; k < NL * NRING; k += NT) {
    const int l = k / NRING;
    const int q = k - l * NRING;
    int rhy, rhp, want;  // staged row, staged pair, element that must be red (-1: either)
    if (q < 2 * NP) {
      rhy = q < NP ? 1 : TY + 2;
      rhp = 1 + (q < NP ? q : q - NP);
      want = -1;
    } else {
      const int q2 = q - 2 * NP;
      rhy = 2 + (q2 < TY ? q2 : q2 - TY);
      rhp = q2 < TY ? 0 : NP + 1;
      want = q2 < TY ? 1 : 0;
    }
    const int gx = x0 - 2 + 2 * rhp, gy = y0 - 2 + rhy;
    if (gx < 0 || gx >= X || gy < 0 || gy >= ny) continue;
    const int er = (gy + l) & 1;
    if (want >= 0 && er != want) continue;
    const NodeCoef<T> kr = load_node<T, NL>(G, gE, gN, gU, invD, r, l, gy, gx + er);
    const T nv = relax<T, NL, HY, HP>(sd, l, rhy, rhp, er, kr, omega);
    put(sd[l][rhy][rhp], er, nv);
  }
  __syncthreads();

  // black half-sweep on the owned pairs from the new red values; write both nodes
  if (mine) {
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int eb = 1 - ((y + l) & 1);
      V2<T> out = sd[l][hy][hp];
      const T nv = relax<T, NL, HY, HP>(sd, l, hy, hp, eb, keep[l], omega);
      put(out, eb, nv);
      st2(dnew, l * P + (int64_t)y * X + x, out);
    }
  }
}

// ------------------------------------------------------------------------------------
// Scenario blocks: the tiles of a grid that carries several current scenarios cover
// tl.pad consecutive scenarios.  The workgroup loads the tile's coefficients (shared by the
// scenarios) once and then, scenario by scenario, streams only that scenario's r and d (and,
// in the residual, v and b), so coefficient traffic is divided by the block size.
// ------------------------------------------------------------------------------------
template <typename T, int NL, int TY>
__global__ __launch_bounds__(64 * TY) void k_sweep_rb_multi(const Tile* __restrict__ tiles, int ntiles,
                                                           const GridDesc* __restrict__ grids, Ctl c,
                                                           int din, int zero_in, T omega) {
  constexpr int NP = kTileX / 2, HP = NP + 2, HY = TY + 4, NT = 64 * TY;
  constexpr int NRING = 2 * NP + 2 * TY;
  constexpr int RT = (NL * NRING + NT - 1) / NT;  // ring tasks per thread
  __shared__ V2<T> sd[NL][HY][HP];
  const int ti = xcd_tile(ntiles);
  if (ti < 0) return;
  const Tile tl = tiles[ti];
  const GridDesc& G = grids[tl.grid];
  const int ny = G.ny, X = G.X;
  const int64_t P = (int64_t)X * ny;
  const int x0 = tl.x0, y0 = tl.y0;
  const T* __restrict__ gE = static_cast<const T*>(G.gEs);
  const T* __restrict__ gN = static_cast<const T*>(G.gNs);
  const T* __restrict__ gU = static_cast<const T*>(G.gUs);
  const T* __restrict__ invD = static_cast<const T*>(G.invDs);
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int x = x0 + 2 * lane, y = y0 + row;
  const int hp = lane + 1, hy = row + 2;
  const bool mine = x < X && y < ny;

  // the owned pair on every layer (red node and black partner)
  NodeCoef<T> kr[NL], kb[NL];
  if (mine) {
#pragma unroll
    for (int l = 0; l < NL; ++l) load_pair_coef<T, NL>(G, gE, gN, gU, invD, l, y, x, (y + l) & 1, kr[l], kb[l]);
  }
  // this thread's ring tasks (red ring nodes around the tile)
  NodeCoef<T> kring[RT];
  int ring_l[RT], ring_hy[RT], ring_hp[RT], ring_e[RT];
  int64_t ring_i[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    ring_e[t] = -1;
    const int k = threadIdx.x + t * NT;
    if (k >= NL * NRING) continue;
    const int l = k / NRING;
    const int q = k - l * NRING;
    int rhy, rhp, want;
    if (q < 2 * NP) {
      rhy = q < NP ? 1 : TY + 2;
      rhp = 1 + (q < NP ? q : q - NP);
      want = -1;
    } else {
      const int q2 = q - 2 * NP;
      rhy = 2 + (q2 < TY ? q2 : q2 - TY);
      rhp = q2 < TY ? 0 : NP + 1;
      want = q2 < TY ? 1 : 0;
    }
    const int gx = x0 - 2 + 2 * rhp, gy = y0 - 2 + rhy;
    if (gx < 0 || gx >= X || gy < 0 || gy >= ny) continue;
    const int er = (gy + l) & 1;
    if (want >= 0 && er != want) continue;
    NodeCoef<T> unused;
    load_pair_coef<T, NL>(G, gE, gN, gU, invD, l, gy, gx, er, kring[t], unused);
    ring_l[t] = l;
    ring_hy[t] = rhy;
    ring_hp[t] = rhp;
    ring_e[t] = er;
    ring_i[t] = l * P + (int64_t)gy * X + gx + er;
  }

  // The scenario loop.  Single-layer FP32 blocks first collect the block's still-iterating
  // scenarios (at most 16) and keep one scenario of loads in flight ahead: while scenario s is
  // swept, the next active one's old correction and right-hand side are already being read.
  // Elsewhere the second set of registers would cost occupancy or spills, so each scenario loads
  // as it starts.
  constexpr bool kAhead = NL == 1 && sizeof(T) == 4;
  if constexpr (kAhead) {
    unsigned amask = 0u;
    for (int sc = 0; sc < tl.pad; ++sc) amask |= (c.active[tl.item + sc] ? 1u : 0u) << sc;
    constexpr int NS = NL * HY * HP, SPT = (NS + NT - 1) / NT;
    struct Loads {
      V2<T> stage[SPT];
      V2<T> rr[NL];
      T rring[RT];
    };
    auto issue = [&](int sc, Loads& L) {
      const int64_t off = (int64_t)(tl.scen + sc) * G.nstore;
      const T* __restrict__ dold = static_cast<const T*>(G.d[din]) + off;
      const T* __restrict__ r = static_cast<const T*>(G.r) + off;
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        const int k = threadIdx.x + q * NT;
        const int l = k / (HY * HP);
        const int rem = k - l * (HY * HP);
        const int shy = rem / HP, shp = rem - shy * HP;
        const int sx = x0 - 2 + 2 * shp, sy = y0 - 2 + shy;
        L.stage[q] = zero2<T>();
        if (!zero_in && k < NS && sx >= 0 && sx < X && sy >= 0 && sy < ny) L.stage[q] = ld2(dold, l * P + (int64_t)sy * X + sx);
      }
#pragma unroll
      for (int l = 0; l < NL; ++l) L.rr[l] = mine ? ld2(r, l * P + (int64_t)y * X + x) : zero2<T>();
#pragma unroll
      for (int t = 0; t < RT; ++t) L.rring[t] = ring_e[t] >= 0 ? ld1(r, ring_i[t]) : T(0);
    };
    Loads cur, nxt;
    int sc = amask ? __builtin_ctz(amask) : -1;
    if (sc >= 0) issue(sc, cur);
    while (sc >= 0) {
      const unsigned rest = amask & ~((2u << sc) - 1u);  // active scenarios after sc
      const int sn = rest ? __builtin_ctz(rest) : -1;
      if (sn >= 0) issue(sn, nxt);
      const int64_t off = (int64_t)(tl.scen + sc) * G.nstore;
      T* __restrict__ dnew = static_cast<T*>(G.d[din ^ 1]) + off;
      __syncthreads();  // the previous scenario's readers are done with sd
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        const int k = threadIdx.x + q * NT;
        if (k < NS) (&sd[0][0][0])[k] = cur.stage[q];
      }
      __syncthreads();
      if (mine) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          const int er = (y + l) & 1;
          kr[l].r = pick(cur.rr[l], er);
          kb[l].r = pick(cur.rr[l], 1 - er);
          const T nv = relax<T, NL, HY, HP>(sd, l, hy, hp, er, kr[l], omega);
          put(sd[l][hy][hp], er, nv);
        }
      }
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        if (ring_e[t] < 0) continue;
        kring[t].r = cur.rring[t];
        const T nv = relax<T, NL, HY, HP>(sd, ring_l[t], ring_hy[t], ring_hp[t], ring_e[t], kring[t], omega);
        put(sd[ring_l[t]][ring_hy[t]][ring_hp[t]], ring_e[t], nv);
      }
      __syncthreads();
      if (mine) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          const int eb = 1 - ((y + l) & 1);
          V2<T> out = sd[l][hy][hp];
          const T nv = relax<T, NL, HY, HP>(sd, l, hy, hp, eb, kb[l], omega);
          put(out, eb, nv);
          st2(dnew, l * P + (int64_t)y * X + x, out);
        }
      }
      sc = sn;
      if (sn >= 0) cur = nxt;
    }
  } else {
    for (int sc = 0; sc < tl.pad; ++sc) {
      if (!c.active[tl.item + sc]) continue;  // uniform across the block
      const int64_t off = (int64_t)(tl.scen + sc) * G.nstore;
      const T* __restrict__ dold = static_cast<const T*>(G.d[din]) + off;
      T* __restrict__ dnew = static_cast<T*>(G.d[din ^ 1]) + off;
      const T* __restrict__ r = static_cast<const T*>(G.r) + off;
      __syncthreads();  // the previous scenario's readers are done with sd
      for (int k = threadIdx.x; k < NL * HY * HP; k += NT) {
        const int l = k / (HY * HP);
        const int rem = k - l * (HY * HP);
        const int shy = rem / HP, shp = rem - shy * HP;
        const int sx = x0 - 2 + 2 * shp, sy = y0 - 2 + shy;
        V2<T> val = zero2<T>();
        if (!zero_in && sx >= 0 && sx < X && sy >= 0 && sy < ny) val = ld2(dold, l * P + (int64_t)sy * X + sx);
        sd[l][shy][shp] = val;
      }
      __syncthreads();
      if (mine) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          const int er = (y + l) & 1;
          const V2<T> rr = ld2(r, l * P + (int64_t)y * X + x);
          kr[l].r = pick(rr, er);
          kb[l].r = pick(rr, 1 - er);
          const T nv = relax<T, NL, HY, HP>(sd, l, hy, hp, er, kr[l], omega);
          put(sd[l][hy][hp], er, nv);
        }
      }
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        if (ring_e[t] < 0) continue;
        kring[t].r = r[ring_i[t]];
        const T nv = relax<T, NL, HY, HP>(sd, ring_l[t], ring_hy[t], ring_hp[t], ring_e[t], kring[t], omega);
        put(sd[ring_l[t]][ring_hy[t]][ring_hp[t]], ring_e[t], nv);
      }
      __syncthreads();
      if (mine) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          const int eb = 1 - ((y + l) & 1);
          V2<T> out = sd[l][hy][hp];
          const T nv = relax<T, NL, HY, HP>(sd, l, hy, hp, eb, kb[l], omega);
          put(out, eb, nv);
          st2(dnew, l * P + (int64_t)y * X + x, out);
        }
      }
    }
  }
}

// FP64 residual over a scenario block (see k_resid): coefficients once, v, d, b per scenario.
template <typename T, int NL, int TY>
__device__ void resid_multi_tile(const Tile* __restrict__ tiles, int ti, const GridDesc* __restrict__ grids,
                                 const Ctl& c, int has_d, int din) {
  constexpr int NP = kTileX / 2, HP = NP + 2, HY = TY + 2, NT = 64 * TY;
  __shared__ double2 sv[NL][HY][HP];
  __shared__ double wmax[NT / 64];
  const Tile tl = tiles[ti];
  const GridDesc& G = grids[tl.grid];
  const int nx = G.nx, ny = G.ny, X = G.X;
  const int64_t P = (int64_t)X * ny;
  const int x0 = tl.x0, y0 = tl.y0;
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int x = x0 + 2 * lane, y = y0 + row;
  const int hp = lane + 1, hy = row + 1;
  const bool mine = x < X && y < ny;
  double2 D2[NL], ge[NL], gn[NL], gs[NL], gu[NL], gd[NL];
  double gw[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    D2[l] = ge[l] = gn[l] = gs[l] = gu[l] = gd[l] = make_double2(0.0, 0.0);
    gw[l] = 0.0;
    if (!mine) continue;
    const int64_t i = l * P + (int64_t)y * X + x;
    D2[l] = ld2(G.D64, i);
    ge[l] = ld2(G.gE64, i);
    gn[l] = ld2(G.gN64, i);
    if (y > 0) gs[l] = ld2(G.gN64, i - X);
    if (x > 0) gw[l] = G.gE64[i - 1];
    if (NL > 1) {
      if (l < NL - 1) gu[l] = ld2(G.gU64, i);
      if (l > 0) gd[l] = ld2(G.gU64, i - P);
    }
  }
  for (int sc = 0; sc < tl.pad; ++sc) {
    const int item = tl.item + sc;
    if (!c.active[item]) continue;  // uniform across the block
    const int64_t off = (int64_t)(tl.scen + sc) * G.nstore;
    const int vi = c.vidx[item];
    const double* __restrict__ v = G.v[vi] + off;
    const T* __restrict__ d = static_cast<const T*>(G.d[din]) + off;
    __syncthreads();
    for (int k = threadIdx.x; k < NL * HY * HP; k += NT) {
      const int l = k / (HY * HP);
      const int rem = k - l * (HY * HP);
      const int shy = rem / HP, shp = rem - shy * HP;
      const int sx = x0 - 2 + 2 * shp, sy = y0 - 1 + shy;
      double2 val = make_double2(0.0, 0.0);
      if (sx >= 0 && sx < X && sy >= 0 && sy < ny) {
        const int64_t i = l * P + (int64_t)sy * X + sx;
        val = ld2(v, i);
        if (has_d) {
          const V2<T> dd = ld2(d, i);
          val.x += (double)dd.x;
          val.y += (double)dd.y;
        }
      }
      sv[l][shy][shp] = val;
    }
    __syncthreads();
    double m = 0.0;
    if (mine) {
      double* __restrict__ vout = G.v[vi ^ 1] + off;
      T* __restrict__ r = static_cast<T*>(G.r) + off;
      const double* __restrict__ bvec = G.b + off;
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        const int64_t i = l * P + (int64_t)y * X + x;
        const double2 b2 = ld2(bvec, i);
        const double2 own = sv[l][hy][hp], eastp = sv[l][hy][hp + 1], westp = sv[l][hy][hp - 1];
        const double2 nth = sv[l][hy + 1][hp], sth = sv[l][hy - 1][hp];
        double2 up = make_double2(0.0, 0.0), dn = make_double2(0.0, 0.0);
        if (NL > 1) {
          if (l < NL - 1) up = sv[l + 1][hy][hp];
          if (l > 0) dn = sv[l - 1][hy][hp];
        }
        double r0 = b2.x - D2[l].x * own.x + ge[l].x * own.y + gw[l] * westp.y + gn[l].x * nth.x +
                    gs[l].x * sth.x + gu[l].x * up.x + gd[l].x * dn.x;
        double r1 = b2.y - D2[l].y * own.y + ge[l].y * eastp.x + ge[l].x * own.x + gn[l].y * nth.y +
                    gs[l].y * sth.y + gu[l].y * up.y + gd[l].y * dn.y;
        if (x >= nx) r0 = 0.0;
        if (x + 1 >= nx) r1 = 0.0;
        if (has_d) st2(vout, i, own);
        V2<T> rr;
        rr.x = (T)r0;
        rr.y = (T)r1;
        st2(r, i, rr);
        if (x < nx) m = nan_max(m, fabs(r0) / D2[l].x);
        if (x + 1 < nx) m = nan_max(m, fabs(r1) / D2[l].y);
      }
    }
    for (int o = 32; o > 0; o >>= 1) m = nan_max(m, __shfl_xor(m, o, 64));
    if (lane == 0) wmax[row] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double bm = wmax[0];
      for (int w = 1; w < NT / 64; ++w) bm = nan_max(bm, wmax[w]);
      atomicMax(&c.norm_bits[item], (unsigned long long)__double_as_longlong(bm));
    }
  }
}

template <typename T, int NL, int TY>
__global__ __launch_bounds__(64 * TY) void k_resid_multi(const Tile* __restrict__ tiles, int ntiles,
                                                        const GridDesc* __restrict__ grids, Ctl c,
                                                        int has_d, int din) {
  const int ti = xcd_tile(ntiles);
  if (!*c.stall && ti >= 0) resid_multi_tile<T, NL, TY>(tiles, ti, grids, c, has_d, din);
}

// ------------------------------------------------------------------------------------
// Two red-black SOR sweeps per launch (overlapped temporal blocking).  The old correction is
// staged with a four-node halo; the first red half-sweep is also computed on a three-node
// ring around the tile, the first black half-sweep on a two-node ring and the second red one
// on a one-node ring, so the second black half-sweep of the owned nodes reads exactly the
// values two separate sweeps would give.  A launch reads and writes the bytes of one sweep.
// Tiles may be scenario blocks (Tile.pad scenarios sharing the coefficients, kept in
// registers for the owned pairs).
// ------------------------------------------------------------------------------------

// One half-sweep of `colour` on the ring of width k around the tile (all layers); the ring's
// coefficients and right-hand side come from global memory (mostly L2: they belong to the
// neighbouring tiles).  Top and bottom bands visit only cells of the colour; the narrow side
// bands visit every cell and skip the other colour.
template <typename T, int NL, int TY, int HY, int HP>
__device__ __forceinline__ void ring_half(V2<T> (*sd)[HY][HP], const GridDesc& G, const T* __restrict__ gE,
                                          const T* __restrict__ gN, const T* __restrict__ gU,
                                          const T* __restrict__ invD, const T* __restrict__ r, int x0,
                                          int y0, int k, int colour, T omega) {
  constexpr int NT = 64 * TY, HALO = 4;
  const int W = kTileX + 2 * k;
  const int band = k * (W / 2);  // cells of the colour in the top (or bottom) band of a layer
  const int side = k * TY;       // cells in the left (or right) band of a layer
  const int per_layer = 2 * band + 2 * side;
  const int X = G.X, ny = G.ny;
  const int64_t P = (int64_t)X * ny;
  for (int q = threadIdx.x; q < NL * per_layer; q += NT) {
    const int l = q / per_layer;
    int rem = q - l * per_layer;
    int gx, gy;
    if (rem < 2 * band) {
      const int b = rem >= band;  // 0: top band, 1: bottom band
      rem -= b * band;
      const int rr = rem / (W / 2), j = rem - rr * (W / 2);
      gy = b ? y0 + TY + rr : y0 - k + rr;
      const int xs = x0 - k;
      gx = xs + ((colour + gy + l + xs) & 1) + 2 * j;
    } else {
      rem -= 2 * band;
      const int b = rem >= side;  // 0: left band, 1: right band
      rem -= b * side;
      const int rr = rem / k, cc = rem - rr * k;
      gy = y0 + rr;
      gx = b ? x0 + kTileX + cc : x0 - k + cc;
      if (((gx + gy + l) & 1) != colour) continue;
    }
    if (gx < 0 || gx >= X || gy < 0 || gy >= ny) continue;
    const int e = gx & 1, px = gx - e;
    NodeCoef<T> mine, other;
    load_pair_coef<T, NL>(G, gE, gN, gU, invD, l, gy, px, e, mine, other);
    mine.r = r[l * P + (int64_t)gy * X + gx];
    const int hy = gy - y0 + HALO, hp = (px - x0 + HALO) >> 1;
    const T nv = relax<T, NL, HY, HP>(sd, l, hy, hp, e, mine, omega);
    put(sd[l][hy][hp], e, nv);
  }
}

template <typename T, int NL, int TY>
__global__ __launch_bounds__(64 * TY) void k_sweep_rb2(const Tile* __restrict__ tiles, int ntiles,
                                                      const GridDesc* __restrict__ grids, Ctl c,
                                                      int din, int zero_in, T omega) {
  constexpr int HALO = 4;                       // staged nodes beyond the tile on every side
  constexpr int NP = kTileX / 2, HP = NP + HALO, HY = TY + 2 * HALO, NT = 64 * TY;
  __shared__ V2<T> sd[NL][HY][HP];
  const int ti = xcd_tile(ntiles);
  if (ti < 0) return;
  const Tile tl = tiles[ti];
  const GridDesc& G = grids[tl.grid];
  const int ny = G.ny, X = G.X;
  const int64_t P = (int64_t)X * ny;
  const int x0 = tl.x0, y0 = tl.y0;
  const T* __restrict__ gE = static_cast<const T*>(G.gEs);
  const T* __restrict__ gN = static_cast<const T*>(G.gNs);
  const T* __restrict__ gU = static_cast<const T*>(G.gUs);
  const T* __restrict__ invD = static_cast<const T*>(G.invDs);
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int x = x0 + 2 * lane, y = y0 + row;
  const int hp = lane + HALO / 2, hy = row + HALO;
  const bool mine = x < X && y < ny;

  NodeCoef<T> kr[NL], kb[NL];  // the owned pair on every layer: red node and black partner
  if (mine) {
#pragma unroll
    for (int l = 0; l < NL; ++l) load_pair_coef<T, NL>(G, gE, gN, gU, invD, l, y, x, (y + l) & 1, kr[l], kb[l]);
  }
  for (int sc = 0; sc < tl.pad; ++sc) {
    if (!c.active[tl.item + sc]) continue;  // uniform across the block
    const int64_t off = (int64_t)(tl.scen + sc) * G.nstore;
    const T* __restrict__ dold = static_cast<const T*>(G.d[din]) + off;
    T* __restrict__ dnew = static_cast<T*>(G.d[din ^ 1]) + off;
    const T* __restrict__ r = static_cast<const T*>(G.r) + off;
    __syncthreads();  // the previous scenario is done with sd
    for (int k = threadIdx.x; k < NL * HY * HP; k += NT) {
      const int l = k / (HY * HP);
      const int rem = k - l * (HY * HP);
      const int shy = rem / HP, shp = rem - shy * HP;
      const int sx = x0 - HALO + 2 * shp, sy = y0 - HALO + shy;
      V2<T> val = zero2<T>();
      if (!zero_in && sx >= 0 && sx < X && sy >= 0 && sy < ny) val = ld2(dold, l * P + (int64_t)sy * X + sx);
      sd[l][shy][shp] = val;
    }
    if (mine) {
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        const int er = (y + l) & 1;
        const V2<T> rr = ld2(r, l * P + (int64_t)y * X + x);
        kr[l].r = pick(rr, er);
        kb[l].r = pick(rr, 1 - er);
      }
    }
    __syncthreads();
#pragma unroll
    for (int half = 0; half < 4; ++half) {  // red, black, red, black
      const int colour = half & 1;
      if (mine) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          const int ec = ((y + l) & 1) ^ colour;  // element of the pair with this colour
          const T nv = relax<T, NL, HY, HP>(sd, l, hy, hp, ec, colour ? kb[l] : kr[l], omega);
          if (half < 3) {
            put(sd[l][hy][hp], ec, nv);
          } else {
            V2<T> out = sd[l][hy][hp];
            put(out, ec, nv);
            st2(dnew, l * P + (int64_t)y * X + x, out);
          }
        }
      }
      if (half < 3) {
        ring_half<T, NL, TY, HY, HP>(sd, G, gE, gN, gU, invD, r, x0, y0, 3 - half, colour, omega);
        __syncthreads();
      }
    }
  }
}

// Weighted Jacobi sweep: every node from the previous sweep's values (element-wise).
template <typename T, int NL>
__global__ __launch_bounds__(kThreads) void k_sweep_jacobi(const Tile* __restrict__ tiles, int ntiles,
                                                          int TY, const GridDesc* __restrict__ grids,
                                                          Ctl c, int din, int zero_in, T omega) {
  const int ti = xcd_tile(ntiles);
  if (ti < 0) return;
  const Tile tl = tiles[ti];
  const GridDesc& G = grids[tl.grid];
  const int ny = G.ny, X = G.X;
  const int64_t P = (int64_t)X * ny;
  const T* __restrict__ gE = static_cast<const T*>(G.gEs);
  const T* __restrict__ gN = static_cast<const T*>(G.gNs);
  const T* __restrict__ gU = static_cast<const T*>(G.gUs);
  const T* __restrict__ invD = static_cast<const T*>(G.invDs);
  for (int sc = 0; sc < tl.pad; ++sc) {  // the scenarios of a scenario block
    if (!c.active[tl.item + sc]) continue;
    const int64_t off = (int64_t)(tl.scen + sc) * G.nstore;
    const T* __restrict__ dold = static_cast<const T*>(G.d[din]) + off;
    T* __restrict__ dnew = static_cast<T*>(G.d[din ^ 1]) + off;
    const T* __restrict__ r = static_cast<const T*>(G.r) + off;
    for (int k = threadIdx.x; k < NL * TY * kTileX; k += kThreads) {
      const int l = k / (TY * kTileX);
      const int rem = k - l * (TY * kTileX);
      const int yy = rem / kTileX, xx = rem - yy * kTileX;
      const int x = tl.x0 + xx, y = tl.y0 + yy;
      if (x >= X || y >= ny) continue;
      const int64_t i = l * P + (int64_t)y * X + x;
      T acc = r[i];
      if (!zero_in) {
        if (x + 1 < X) acc += gE[i] * dold[i + 1];
        if (x > 0) acc += gE[i - 1] * dold[i - 1];
        if (y + 1 < ny) acc += gN[i] * dold[i + X];
        if (y > 0) acc += gN[i - X] * dold[i - X];
        if (NL > 1) {
          if (l < NL - 1) acc += gU[i] * dold[i + P];
          if (l > 0) acc += gU[i - P] * dold[i - P];
        }
      }
      const T old = zero_in ? T(0) : dold[i];
      dnew[i] = old + omega * (invD[i] * acc - old);
    }
  }
}

// ------------------------------------------------------------------------------------
// Inductor branch currents after the node solve (second line of eq. 10, companion form):
//   i(t+h) = alpha i(t) + g_eq (v_a - v_b)(t+h),  v_b = Vdd for a pad branch.
// ------------------------------------------------------------------------------------
__global__ void k_inductors(const GridDesc* __restrict__ grids, const int32_t* __restrict__ ind_grid,
                            const int32_t* __restrict__ ind_local, int n_total, Ctl c) {
  if (*c.stall) return;  // the step's close is waiting for more sweeps
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_total) return;
  const GridDesc& G = grids[ind_grid[j]];
  const int k = ind_local[j];
  const int a = G.ind_a[k], bslot = G.ind_b[k];
  const double geq = G.ind_geq[k], al = G.ind_alpha[k];
  for (int s = 0; s < G.S; ++s) {
    const double* __restrict__ v = G.v[c.vidx[G.item0 + s]] + (int64_t)s * G.nstore;
    const double vb = bslot >= 0 ? v[bslot] : (G.ind_vfar ? G.ind_vfar[k] : G.vdd);
    double* q = G.ind_i + (int64_t)s * G.n_ind + k;
    *q = al * *q + geq * (v[a] - vb);
  }
}

// ------------------------------------------------------------------------------------
// Reverse-time adjoint of the softplus voltage-drop loss over a BE transient (RC grids):
//   J = sum_k sum_i softplus(Vdd - v_k,i - margin)^2,
//   M lambda_k = dJ/dv_k + (C/h) lambda_{k+1}   (M is symmetric, Lemma 1),
//   dJ/dC_i += lambda_k,i (v_k-1,i - v_k,i) / h,  dJ/dg_e -= (lambda_a - lambda_b)(v_a - v_b).
// All three kernels walk the tiles of one item; sums are per block in a fixed order.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ double softplus(double u) { return fmax(u, 0.0) + log1p(exp(-fabs(u))); }
__device__ __forceinline__ double sigmoid(double u) { return 1.0 / (1.0 + exp(-u)); }

// Block b writes the loss of its tile's nodes at the item's current state to part[b].
__global__ __launch_bounds__(kThreads) void k_loss(const Tile* __restrict__ tiles, int ntiles, int TY,
                                                  const GridDesc* __restrict__ grids, Ctl c, double margin,
                                                  double* __restrict__ part) {
  __shared__ double red[kThreads / 64];
  const int ti = blockIdx.x;
  if (ti >= ntiles) return;
  const Tile tl = tiles[ti];
  const GridDesc& G = grids[tl.grid];
  const int nx = G.nx, ny = G.ny, X = G.X;
  const int64_t P = (int64_t)X * ny;
  const double* __restrict__ v = G.v[c.vidx[tl.item]] + (int64_t)tl.scen * G.nstore;
  double acc = 0.0;
  const int per_layer = kTileX * TY;
  for (int k = threadIdx.x; k < per_layer * G.nl; k += kThreads) {
    const int l = k / per_layer, rem = k - l * per_layer;
    const int yy = rem / kTileX, xx = rem - yy * kTileX;
    const int x = tl.x0 + xx, y = tl.y0 + yy;
    if (x >= nx || y >= ny) continue;
    const double sp = softplus(G.vdd - v[l * P + (int64_t)y * X + x] - margin);
    acc += sp * sp;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) s += red[w];
    part[ti] = s;
  }
}

// total[0] += sum of part[0..n) in a fixed order (one block).
__global__ void k_sum_into(const double* __restrict__ part, int n, double* __restrict__ total) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) total[0] += red[0];
}

// Adjoint right-hand side dJ/dv_k + (C/h) lambda_{k+1} into `rhs` (one scenario slice).
// Adjoint right-hand side dJ/dv_k + (C/h) lambda_{k+1} into b.  Runs on the adjoint view of the
// grid, whose current state buffer holds lambda_{k+1}.
__global__ __launch_bounds__(kThreads) void k_adj_rhs(const Tile* __restrict__ tiles, int ntiles, int TY,
                                                     const GridDesc* __restrict__ grids, Ctl c,
                                                     const double* __restrict__ vk, double margin,
                                                     const double* __restrict__ mu, int nind) {
  const int ti = blockIdx.x;
  if (ti >= ntiles) return;
  const Tile tl = tiles[ti];
  const GridDesc& G = grids[tl.grid];
  const int nx = G.nx, ny = G.ny, X = G.X;
  const int64_t P = (int64_t)X * ny;
  const int64_t off = (int64_t)tl.scen * G.nstore;
  const double* __restrict__ lam_next = G.v[c.vidx[tl.item]] + off;
  double* __restrict__ rhs = G.b + off;
  const int per_layer = kTileX * TY;
  for (int k = threadIdx.x; k < per_layer * G.nl; k += kThreads) {
    const int l = k / per_layer, rem = k - l * per_layer;
    const int yy = rem / kTileX, xx = rem - yy * kTileX;
    const int x = tl.x0 + xx, y = tl.y0 + yy;
    if (x >= X || y >= ny) continue;
    const int64_t i = l * P + (int64_t)y * X + x;
    double val = 0.0;
    if (x < nx) {
      const double u = G.vdd - vk[i] - margin;
      val = -2.0 * softplus(u) * sigmoid(u) + G.ch64[i] * lam_next[i];
      // inductive branches: + g_eq A^T mu_k (near end +, far end -)
      for (int j = nind ? G.inc_off[i] : 0, je = nind ? G.inc_off[i + 1] : 0; j < je; ++j) {
        const int e = G.inc_ind[j];
        const int kk = (e > 0 ? e : -e) - 1;
        const double t = G.ind_geq[kk] * mu[kk];
        val += (e > 0) ? t : -t;
      }
    }
    rhs[i] = val;
  }
}

// Gradient accumulation for step k (FP64); each segment gradient belongs to its lower node.
// Gradient accumulation for step k (FP64), on the adjoint view (current state = lambda_k).
// Each segment's gradient belongs to its lower node.
__global__ __launch_bounds__(kThreads) void k_adj_grad(const Tile* __restrict__ tiles, int ntiles, int TY,
                                                      const GridDesc* __restrict__ grids, Ctl c,
                                                      const double* __restrict__ vk,
                                                      const double* __restrict__ vprev, double inv_h,
                                                      double* __restrict__ dC, double* __restrict__ dgE,
                                                      double* __restrict__ dgN) {
  const int ti = blockIdx.x;
  if (ti >= ntiles) return;
  const Tile tl = tiles[ti];
  const GridDesc& G = grids[tl.grid];
  const int nx = G.nx, ny = G.ny, X = G.X;
  const int64_t P = (int64_t)X * ny;
  const double* __restrict__ lam = G.v[c.vidx[tl.item]] + (int64_t)tl.scen * G.nstore;
  const int per_layer = kTileX * TY;
  for (int k = threadIdx.x; k < per_layer * G.nl; k += kThreads) {
    const int l = k / per_layer, rem = k - l * per_layer;
    const int yy = rem / kTileX, xx = rem - yy * kTileX;
    const int x = tl.x0 + xx, y = tl.y0 + yy;
    if (x >= nx || y >= ny) continue;
    const int64_t i = l * P + (int64_t)y * X + x;
    const double li = lam[i], vi = vk[i];
    dC[i] += li * (vprev[i] - vi) * inv_h;
    if (x + 1 < nx) dgE[i] -= (li - lam[i + 1]) * (vi - vk[i + 1]);
    if (y + 1 < ny) dgN[i] -= (li - lam[i + X]) * (vi - vk[i + X]);
  }
}

// The adjoint of the inductor-current recurrence i_k = alpha i_{k-1} + g_eq (A v_k - v_far):
// mu_k = alpha (mu_{k+1} - A lambda_{k+1}), with lambda_{k+1} the item's current adjoint state.
// One thread per inductive branch of the grid.
__global__ void k_adj_mu(const GridDesc* __restrict__ grids, int grid, int item, int scen, Ctl c,
                         double* __restrict__ mu, int nind) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nind) return;
  const GridDesc& G = grids[grid];
  const double* __restrict__ lam = G.v[c.vidx[item]] + (int64_t)scen * G.nstore;
  const int a = G.ind_a[k], b = G.ind_b[k];
  const double el = lam[a] - (b >= 0 ? lam[b] : 0.0);
  mu[k] = G.ind_alpha[k] * (mu[k] - el);
}

// Gradients with respect to the conductance g and the series inductance L of every via and pad
// at one reverse step (branches: vias, then pads).  With e the branch's incidence (a via joins
// slots a and a + P; a pad joins slot a to the supply), g_eq = h g / (g L + h) and
// alpha = g L / (g L + h) (a plain resistor: g_eq = g, alpha = 0, mu = 0):
//   dJ/dtheta += (mu_k - e.lambda_k) (dg_eq/dtheta (e.v_k - v_far) + dalpha/dtheta i_{k-1}).
// For a resistor this is -(e.lambda_k)(e.v_k - v_far).  One thread per branch.
__global__ void k_adj_branch_grad(const GridDesc* __restrict__ grids, int grid, int item, int scen, Ctl c,
                                  const double* __restrict__ vk, const int32_t* __restrict__ br_slot,
                                  const int32_t* __restrict__ br_ind, const double* __restrict__ br_g,
                                  const double* __restrict__ br_L, int n_vias, int n_br, int64_t P, double h,
                                  const double* __restrict__ mu, const double* __restrict__ iprev,
                                  double* __restrict__ dg, double* __restrict__ dL) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_br) return;
  const GridDesc& G = grids[grid];
  const double* __restrict__ lam = G.v[c.vidx[item]] + (int64_t)scen * G.nstore;
  const int64_t a = br_slot[j];
  const bool via = j < n_vias;
  const double el = lam[a] - (via ? lam[a + P] : 0.0);
  const double ev = vk[a] - (via ? vk[a + P] : G.vdd);
  const int k = br_ind[j];
  if (k < 0) {
    dg[j] -= el * ev;
    return;
  }
  const double g = br_g[j], L = br_L[j], den = g * L + h, den2 = den * den;
  const double m = mu[k] - el, ip = iprev[k];
  dg[j] += m * (h * h / den2 * ev + h * L / den2 * ip);
  dL[j] += m * (-h * g * g / den2 * ev + g * h / den2 * ip);
}

// The inductor update of one scenario of one grid (the other items stand still while a segment
// of the adjoint's forward pass is recomputed).
__global__ void k_ind_update_item(const GridDesc* __restrict__ grids, int grid, int item, int scen, Ctl c, int nind) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nind) return;
  const GridDesc& G = grids[grid];
  const double* __restrict__ v = G.v[c.vidx[item]] + (int64_t)scen * G.nstore;
  const int a = G.ind_a[k], b = G.ind_b[k];
  const double vb = b >= 0 ? v[b] : (G.ind_vfar ? G.ind_vfar[k] : G.vdd);
  double* q = G.ind_i + (int64_t)scen * G.n_ind + k;
  *q = G.ind_alpha[k] * *q + G.ind_geq[k] * (v[a] - vb);
}

// ------------------------------------------------------------------------------------
// Launch wrappers
// ------------------------------------------------------------------------------------

hipError_t launch_step_begin(const Ctl& c, int I, int only_item, double h, const SourceTable& src, int win_a,
                             int win_b, hipStream_t s) {
  hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(256), 0, s, c, I, only_item, h, src, win_a, win_b);
  return hipGetLastError();
}

hipError_t launch_step_end(const Ctl& c, int I, int count_step, int begin_next, double h, const SourceTable& src,
                           int win_a, int win_b, hipStream_t s) {
  hipLaunchKernelGGL(k_step_end, dim3(1), dim3(256), 0, s, c, I, count_step, begin_next, h, src, win_a, win_b);
  return hipGetLastError();
}

hipError_t launch_rhs(const Tile* tiles, int ntiles, int tile_rows, const GridDesc* grids,
                      const Ctl& c, hipStream_t s, int predict) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rhs, dim3(xcd_blocks(ntiles)), dim3(64 * tile_rows), 0, s, tiles, ntiles, grids, c,
                     predict);
  return hipGetLastError();
}

hipError_t launch_sources(const SourceTable& src, const GridDesc* grids, const Ctl& c, double shift, double sign,
                          hipStream_t s) {
  if (src.count <= 0) return hipSuccess;
  const int blocks = (src.count + 255) / 256 < 2048 ? (src.count + 255) / 256 : 2048;
  hipLaunchKernelGGL(k_sources, dim3(blocks), dim3(256), 0, s, src, grids, c, shift, sign);
  return hipGetLastError();
}

hipError_t launch_inductors(const GridDesc* grids, const int32_t* ind_grid, const int32_t* ind_local,
                            int n_total, const Ctl& c, hipStream_t s) {
  if (n_total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_inductors, dim3((n_total + 255) / 256), dim3(256), 0, s, grids, ind_grid,
                     ind_local, n_total, c);
  return hipGetLastError();
}

// Copy the current voltages of each tile's item to / from a plain per-scenario buffer.
__global__ __launch_bounds__(kThreads) void k_state_copy(const Tile* __restrict__ tiles, int ntiles, int TY,
                                                        const GridDesc* __restrict__ grids, Ctl c,
                                                        double* __restrict__ buf, int to_buf) {
  const int ti = blockIdx.x;
  if (ti >= ntiles) return;
  const Tile tl = tiles[ti];
  const GridDesc& G = grids[tl.grid];
  const int X = G.X, ny = G.ny;
  const int64_t P = (int64_t)X * ny;
  double* __restrict__ v = G.v[c.vidx[tl.item]] + (int64_t)tl.scen * G.nstore;
  const int per_layer = kTileX * TY;
  for (int k = threadIdx.x; k < per_layer * G.nl; k += kThreads) {
    const int l = k / per_layer, rem = k - l * per_layer;
    const int yy = rem / kTileX, xx = rem - yy * kTileX;
    const int x = tl.x0 + xx, y = tl.y0 + yy;
    if (x >= X || y >= ny) continue;
    const int64_t i = l * P + (int64_t)y * X + x;
    if (to_buf == 1) buf[i] = v[i]; else if (to_buf == 0) v[i] = buf[i]; else v[i] = 2.0 * v[i] - buf[i];
  }
}

// Exchange the buffer index of one item with a saved value (switching between two state views).
// Vector utilities on one item's tiles (one workgroup per tile): op 0 sets d[which] to 1 on the
// mesh nodes (0 in the padding) and r to 0; op 1 takes max |d[which]| and op 4 max |v| over
// the mesh nodes into norm_bits[item]; op 2 scales d[which] by s; op 3 sets v = 0 and b = M_ii.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_item_vec(const Tile* __restrict__ tiles, int ntiles, int TY,
                                                      const GridDesc* __restrict__ grids, Ctl c, int op,
                                                      int which, double s) {
  __shared__ double wmax[kThreads / 64];
  const int ti = blockIdx.x;
  if (ti >= ntiles) return;
  const Tile tl = tiles[ti];
  const GridDesc& G = grids[tl.grid];
  const int nx = G.nx, X = G.X, ny = G.ny;
  const int64_t P = (int64_t)X * ny;
  const int64_t off = (int64_t)tl.scen * G.nstore;
  T* __restrict__ d = static_cast<T*>(G.d[which]) + off;
  T* __restrict__ r = static_cast<T*>(G.r) + off;
  double* __restrict__ v = G.v[c.vidx[tl.item]] + off;
  double* __restrict__ b = G.b + off;
  const int per_layer = kTileX * TY;
  double m = 0.0;
  for (int k = threadIdx.x; k < per_layer * G.nl; k += kThreads) {
    const int l = k / per_layer, rem = k - l * per_layer;
    const int yy = rem / kTileX, xx = rem - yy * kTileX;
    const int x = tl.x0 + xx, y = tl.y0 + yy;
    if (x >= X || y >= ny) continue;
    const int64_t i = l * P + (int64_t)y * X + x;
    const bool real = x < nx;
    switch (op) {
      case 0: d[i] = real ? T(1) : T(0); r[i] = T(0); break;
      case 1: if (real) m = fmax(m, fabs((double)d[i])); break;
      case 2: d[i] = (T)((double)d[i] * s); break;
      case 3: v[i] = 0.0; b[i] = real ? G.D64[i] : 0.0; break;
      default: if (real) m = fmax(m, fabs(v[i])); break;
    }
  }
  if (op != 1 && op != 4) return;
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double bm = wmax[0];
    for (int w = 1; w < kThreads / 64; ++w) bm = fmax(bm, wmax[w]);
    atomicMax(&c.norm_bits[tl.item], (unsigned long long)__double_as_longlong(bm));
  }
}

__global__ void k_swap_vidx(Ctl c, int item, int32_t* saved) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int32_t t = c.vidx[item];
    c.vidx[item] = saved[0];
    saved[0] = t;
  }
}

hipError_t launch_state_copy(const Tile* tiles, int ntiles, int tile_rows, const GridDesc* grids, const Ctl& c,
                             double* buf, int to_buf, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_state_copy, dim3(ntiles), dim3(kThreads), 0, s, tiles, ntiles, tile_rows, grids, c, buf,
                     to_buf);
  return hipGetLastError();
}

hipError_t launch_item_vec(bool fp32, const Tile* tiles, int ntiles, int tile_rows, const GridDesc* grids,
                           const Ctl& c, int op, int which, double s, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_item_vec<float>, dim3(ntiles), dim3(kThreads), 0, st, tiles, ntiles, tile_rows, grids, c,
                       op, which, s);
  else
    hipLaunchKernelGGL(k_item_vec<double>, dim3(ntiles), dim3(kThreads), 0, st, tiles, ntiles, tile_rows, grids, c,
                       op, which, s);
  return hipGetLastError();
}

__global__ void k_resume(Ctl c) {
  if (threadIdx.x == 0) c.stall[0] = 0;
}

hipError_t launch_decide(const Ctl& c, const DecideArgs& da, const CloseArgs& ca, hipStream_t s) {
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(256), 0, s, c, da, ca);
  return hipGetLastError();
}

hipError_t launch_resume(const Ctl& c, hipStream_t s) {
  hipLaunchKernelGGL(k_resume, dim3(1), dim3(64), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_swap_vidx(const Ctl& c, int item, int32_t* saved, hipStream_t s) {
  hipLaunchKernelGGL(k_swap_vidx, dim3(1), dim3(64), 0, s, c, item, saved);
  return hipGetLastError();
}

hipError_t launch_loss(const Tile* tiles, int ntiles, int tile_rows, const GridDesc* grids, const Ctl& c,
                       double margin, double* part, double* total, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_loss, dim3(ntiles), dim3(kThreads), 0, s, tiles, ntiles, tile_rows, grids, c, margin, part);
  hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(256), 0, s, part, ntiles, total);
  return hipGetLastError();
}

hipError_t launch_adj_rhs(const Tile* tiles, int ntiles, int tile_rows, const GridDesc* grids, const Ctl& c,
                          const double* vk, double margin, const double* mu, int nind, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_rhs, dim3(ntiles), dim3(kThreads), 0, s, tiles, ntiles, tile_rows, grids, c, vk, margin,
                     mu, nind);
  return hipGetLastError();
}

hipError_t launch_adj_mu(const GridDesc* grids, int grid, int item, int scen, const Ctl& c, double* mu, int nind,
                         hipStream_t s) {
  if (nind <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_mu, dim3((nind + 255) / 256), dim3(256), 0, s, grids, grid, item, scen, c, mu, nind);
  return hipGetLastError();
}

hipError_t launch_adj_branch_grad(const GridDesc* grids, int grid, int item, int scen, const Ctl& c, const double* vk,
                                  const int32_t* br_slot, const int32_t* br_ind, const double* br_g,
                                  const double* br_L, int n_vias, int n_br, int64_t P, double h, const double* mu,
                                  const double* iprev, double* dg, double* dL, hipStream_t s) {
  if (n_br <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_branch_grad, dim3((n_br + 255) / 256), dim3(256), 0, s, grids, grid, item, scen, c, vk,
                     br_slot, br_ind, br_g, br_L, n_vias, n_br, P, h, mu, iprev, dg, dL);
  return hipGetLastError();
}

hipError_t launch_ind_update_item(const GridDesc* grids, int grid, int item, int scen, const Ctl& c, int nind,
                                  hipStream_t s) {
  if (nind <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ind_update_item, dim3((nind + 255) / 256), dim3(256), 0, s, grids, grid, item, scen, c, nind);
  return hipGetLastError();
}

hipError_t launch_adj_grad(const Tile* tiles, int ntiles, int tile_rows, const GridDesc* grids, const Ctl& c,
                           const double* vk, const double* vprev, double inv_h, double* dC, double* dgE,
                           double* dgN, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_grad, dim3(ntiles), dim3(kThreads), 0, s, tiles, ntiles, tile_rows, grids, c, vk, vprev,
                     inv_h, dC, dgE, dgN);
  return hipGetLastError();
}

template <typename T, int NL, int TY>
static void resid_t(bool multi, const Tile* tiles, int ntiles, const GridDesc* grids, const Ctl& c, int has_d,
                    int din, int fuse, hipStream_t s) {
  if (multi)
    hipLaunchKernelGGL((k_resid_multi<T, NL, TY>), dim3(xcd_blocks(ntiles)), dim3(64 * TY), 0, s, tiles,
                       ntiles, grids, c, has_d, din);
  else if ((fuse & kFuseProbe) && (fuse & kFuseCancelled) && (fuse & kFuseInd))
    hipLaunchKernelGGL((k_probe<T, NL, TY, true>), dim3(xcd_blocks(ntiles)), dim3(64 * TY), 0, s, tiles,
                       ntiles, grids, c);
  else if ((fuse & kFuseProbe) && (fuse & kFuseCancelled))
    hipLaunchKernelGGL((k_probe<T, NL, TY, false>), dim3(xcd_blocks(ntiles)), dim3(64 * TY), 0, s, tiles,
                       ntiles, grids, c);
  else
    hipLaunchKernelGGL((k_resid<T, NL, TY>), dim3(xcd_blocks(ntiles)), dim3(64 * TY), 0, s, tiles,
                       ntiles, grids, c, has_d, din, fuse);
}

template <typename T, int NL, int TY>
static void sweep_t(bool multi, int ordering, const Tile* tiles, int ntiles, const GridDesc* grids, const Ctl& c,
                    int din, int zero_in, double omega, hipStream_t s) {
  if (ordering == 1)  // element-wise; loops over the scenarios of a block itself
    hipLaunchKernelGGL((k_sweep_jacobi<T, NL>), dim3(xcd_blocks(ntiles)), dim3(kThreads), 0, s,
                       tiles, ntiles, TY, grids, c, din, zero_in, (T)omega);
  else if (multi)
    hipLaunchKernelGGL((k_sweep_rb_multi<T, NL, TY>), dim3(xcd_blocks(ntiles)), dim3(64 * TY), 0, s,
                       tiles, ntiles, grids, c, din, zero_in, (T)omega);
  else
    hipLaunchKernelGGL((k_sweep_rb<T, NL, TY>), dim3(xcd_blocks(ntiles)), dim3(64 * TY), 0, s,
                       tiles, ntiles, grids, c, din, zero_in, (T)omega);
}

template <typename T, int NL, int TY>
static void sweep2_t(const Tile* tiles, int ntiles, const GridDesc* grids, const Ctl& c, int din, int zero_in,
                     double omega, hipStream_t s) {
  hipLaunchKernelGGL((k_sweep_rb2<T, NL, TY>), dim3(xcd_blocks(ntiles)), dim3(64 * TY), 0, s, tiles, ntiles,
                     grids, c, din, zero_in, (T)omega);
}

#define PG_DISPATCH_NL_TY(FN, T, ...)                                   \
  switch (nl * 100 + tile_rows) {                                       \
    case 104: FN<T, 1, 4>(__VA_ARGS__); break;                          \
    case 108: FN<T, 1, 8>(__VA_ARGS__); break;                          \
    case 116: FN<T, 1, 16>(__VA_ARGS__); break;                         \
    case 204: FN<T, 2, 4>(__VA_ARGS__); break;                          \
    case 208: FN<T, 2, 8>(__VA_ARGS__); break;                          \
    case 216: FN<T, 2, 16>(__VA_ARGS__); break;                         \
    case 304: FN<T, 3, 4>(__VA_ARGS__); break;                          \
    case 308: FN<T, 3, 8>(__VA_ARGS__); break;                          \
    case 316: FN<T, 3, 16>(__VA_ARGS__); break;                         \
    case 404: FN<T, 4, 4>(__VA_ARGS__); break;                          \
    case 408: FN<T, 4, 8>(__VA_ARGS__); break;                          \
    case 416: FN<T, 4, 16>(__VA_ARGS__); break;                         \
    default: return hipErrorInvalidValue;                               \
  }

hipError_t launch_resid(bool fp32, bool multi, int nl, int tile_rows, const Tile* tiles, int ntiles,
                        const GridDesc* grids, const Ctl& c, int has_d, int din, int fuse, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (fp32) {
    PG_DISPATCH_NL_TY(resid_t, float, multi, tiles, ntiles, grids, c, has_d, din, fuse, s)
  } else {
    PG_DISPATCH_NL_TY(resid_t, double, multi, tiles, ntiles, grids, c, has_d, din, fuse, s)
  }
  return hipGetLastError();
}

hipError_t launch_sweep(bool fp32, bool multi, int ordering, int nl, int tile_rows, const Tile* tiles,
                        int ntiles, const GridDesc* grids, const Ctl& c, int din, int zero_in, double omega,
                        hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (fp32) {
    PG_DISPATCH_NL_TY(sweep_t, float, multi, ordering, tiles, ntiles, grids, c, din, zero_in, omega, s)
  } else {
    PG_DISPATCH_NL_TY(sweep_t, double, multi, ordering, tiles, ntiles, grids, c, din, zero_in, omega, s)
  }
  return hipGetLastError();
}

hipError_t launch_sweep2(bool fp32, int nl, int tile_rows, const Tile* tiles, int ntiles, const GridDesc* grids,
                         const Ctl& c, int din, int zero_in, double omega, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (fp32) {
    PG_DISPATCH_NL_TY(sweep2_t, float, tiles, ntiles, grids, c, din, zero_in, omega, s)
  } else {
    PG_DISPATCH_NL_TY(sweep2_t, double, tiles, ntiles, grids, c, din, zero_in, omega, s)
  }
  return hipGetLastError();
}

// ---- device rebuild of mesh coefficients (pg_update_mesh_values_dev) -----------------------

__global__ __launch_bounds__(kThreads) void k_mesh_check(const double* __restrict__ gE, const double* __restrict__ gN,
                                                         const double* __restrict__ C, int nx, int ny, int nl, double h,
                                                         unsigned long long* bad, unsigned int* ch_mask) {
  const int64_t nE = (int64_t)nl * ny * (nx - 1), nN = (int64_t)nl * (ny - 1) * nx, nC = (int64_t)nl * ny * nx;
  const int64_t P = (int64_t)nx * ny;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long mine = ~0ull;
  unsigned int mask = 0u;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nC; k += stride) {
    if (gE && k < nE) {
      const double g = ld1(gE, k);
      if (!(g >= 0.0 && g <= DBL_MAX)) mine = min(mine, (unsigned long long)k);
    }
    if (gN && k < nN) {
      const double g = ld1(gN, k);
      if (!(g >= 0.0 && g <= DBL_MAX)) mine = min(mine, (1ull << 40) | (unsigned long long)k);
    }
    if (C) {
      const double c = ld1(C, k);
      if (!(c >= 0.0 && c <= DBL_MAX)) mine = min(mine, (2ull << 40) | (unsigned long long)k);
      else if (c / h != 0.0) mask |= 1u << (int)(k / P);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    mine = min(mine, (unsigned long long)__shfl_xor((long long)mine, o, 64));
    mask |= (unsigned int)__shfl_xor((int)mask, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (mine != ~0ull) atomicMin(bad, mine);
    if (mask) atomicOr(ch_mask, mask);
  }
}

template <typename S>
__global__ __launch_bounds__(kThreads) void k_mesh_coef(MeshCoefArgs a) {
  const int nx = a.nx, ny = a.ny, X = a.X;
  const int64_t PS = (int64_t)X * ny, ns = PS * a.nl;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const int l = (int)(i / PS);
  const int64_t rem = i - (int64_t)l * PS;
  const int y = (int)(rem / X), x = (int)(rem - (int64_t)y * X);
  double e = 0.0, n = 0.0, ch = 0.0, D = 0.0, inv = 0.0;
  if (x < nx) {
    const int64_t rowE = ((int64_t)l * ny + y) * (nx - 1);
    const double w = x > 0 ? ld1(a.gE_raw, rowE + x - 1) : 0.0;
    if (x + 1 < nx) e = ld1(a.gE_raw, rowE + x);
    const double s = y > 0 ? ld1(a.gN_raw, ((int64_t)l * (ny - 1) + y - 1) * nx + x) : 0.0;
    if (y + 1 < ny) n = ld1(a.gN_raw, ((int64_t)l * (ny - 1) + y) * nx + x);
    ch = ld1(a.C_raw, ((int64_t)l * ny + y) * nx + x) / a.h;
    const double u = ld1(a.gU64, i), d = l > 0 ? ld1(a.gU64, i - PS) : 0.0;
    D = mesh_diag(ch, e, w, n, s, u, d, 0.0);
    inv = 1.0 / D;
  }
  st1(a.gE64, i, e);
  st1(a.gN64, i, n);
  st1(a.ch64, i, ch);
  st1(a.D64, i, D);
  st1((S*)a.invDs, i, (S)inv);
  if (a.fp32) {
    st1((float*)a.gEs, i, (float)e);
    st1((float*)a.gNs, i, (float)n);
  }
}

template <typename S>
__global__ __launch_bounds__(kThreads) void k_mesh_pads(int n, const int32_t* __restrict__ slot,
                                                        const double* __restrict__ val, double* D64, void* invDs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t a = ld1(slot, k);
  const double D = ld1((const double*)D64, a) + ld1(val, k);
  st1(D64, a, D);
  st1((S*)invDs, a, (S)(1.0 / D));
}

hipError_t launch_mesh_check(const double* gE, const double* gN, const double* C, int nx, int ny, int nl, double h,
                             unsigned long long* bad, unsigned int* ch_mask, hipStream_t s) {
  const int64_t n = (int64_t)nl * ny * nx;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 4096);
  hipLaunchKernelGGL(k_mesh_check, dim3(blocks), dim3(kThreads), 0, s, gE, gN, C, nx, ny, nl, h, bad, ch_mask);
  return hipGetLastError();
}

hipError_t launch_mesh_coef(const MeshCoefArgs& a, hipStream_t s) {
  const int64_t ns = (int64_t)a.X * a.ny * a.nl;
  const unsigned blocks = (unsigned)((ns + kThreads - 1) / kThreads);
  if (a.fp32)
    hipLaunchKernelGGL(k_mesh_coef<float>, dim3(blocks), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_mesh_coef<double>, dim3(blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mesh_pads(int n, const int32_t* pad_slot, const double* pad_val, double* D64, void* invDs, int fp32,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
  if (fp32)
    hipLaunchKernelGGL(k_mesh_pads<float>, dim3(blocks), dim3(kThreads), 0, s, n, pad_slot, pad_val, D64, invDs);
  else
    hipLaunchKernelGGL(k_mesh_pads<double>, dim3(blocks), dim3(kThreads), 0, s, n, pad_slot, pad_val, D64, invDs);
  return hipGetLastError();
}

}  // namespace pgrid
