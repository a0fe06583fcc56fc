// gfx950 kernel that runs K red-black SOR sweeps (eqs. 16-17) of a layered mesh per launch, for
// meshes whose tiles are too few to hide a launch (a few hundred tiles: about one per CU).
//
// Overlapped temporal blocking.  A workgroup stages its 128 x TY tile (all layers) with a halo
// of H = 2K nodes on every side once: the old correction in LDS, the right-hand side and the
// coefficients of every staged pair in registers.  Half-sweep i (i = 1 .. 2K, red first) updates
// the nodes of its colour that lie within H - i nodes of the tile (the tile's box grown by
// H - i in x and in y, clipped to the mesh).  A node's update reads its four in-plane neighbours
// (one step in x or in y) and the nodes above and below it, all of which lie in the box of the
// previous half-sweep, so every value read is the one a mesh-wide half-sweep would have
// produced; after the last (black) half-sweep the tile's own nodes hold exactly the result of K
// separate sweeps, and only they are written.  Each node update is the same expression, on the
// same operands, as in the one-sweep kernel, so the results are bit-identical.
//
// A launch reads the arrays of one sweep for its tile plus the halo (the halo mostly from L2:
// it belongs to the neighbouring tiles of the same XCD) and does K sweeps of work.
#include "mesh_tile.h"

namespace pgrid {

namespace {

constexpr int kTbThreads = 1024;

// load_pair_raw without the right-hand side (which each scenario of a block has its own of).
template <typename T, int NL>
__device__ __forceinline__ void load_pair_coefs(const GridDesc& G, const T* __restrict__ gE,
                                                const T* __restrict__ gN, const T* __restrict__ gU,
                                                const T* __restrict__ invD, int l, int y, int x, PairRaw<T>& p) {
  const int64_t P = (int64_t)G.X * G.ny;
  const int64_t i = l * P + (int64_t)y * G.X + x;
  const NV2<T> z = {T(0), T(0)};
  p.ge = ld2n(gE, i);
  p.gn = ld2n(gN, i);
  p.iv = ld2n(invD, i);
  p.gs = y > 0 ? ld2n(gN, i - G.X) : z;
  p.gw = x > 0 ? ld1(gE, i - 1) : T(0);
  p.gu = z;
  p.gd = z;
  if (NL > 1) {
    if (l < NL - 1) p.gu = ld2n(gU, i);
    if (l > 0) p.gd = ld2n(gU, i - P);
  }
}

template <typename T, int NL, int TY, int K, bool MULTI>
__global__ __launch_bounds__(kTbThreads) void k_sweep_tb(const Tile* __restrict__ tiles, int ntiles,
                                                        const GridDesc* __restrict__ grids, Ctl c, int din,
                                                        int zero_in, T omega) {
  constexpr int H = 2 * K;               // staged nodes beyond the tile on every side
  constexpr int HP = kTileX / 2 + H;     // staged pairs per row
  constexpr int HY = TY + 2 * H;         // staged rows
  constexpr int NQ = NL * HY * HP;       // staged pairs
  constexpr int J = (NQ + kTbThreads - 1) / kTbThreads;
  constexpr int kOut = 0xff;             // distance of a node outside the mesh (never updated)
  static_assert(H < kOut, "distances are stored in 8 bits");
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

  // Staged pair q = (l HY + hy) HP + hp of this thread: q = threadIdx.x + j * kTbThreads.  For
  // each, the pair's coefficients (shared by the scenarios of a block) and its scenario's r, its
  // packed position (l, hy, hp), and the distance from the tile of its red node (bits 0-7) and
  // of its black node (bits 8-15).
  PairRaw<T> pr[J];
  int at[J], dist[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int q = threadIdx.x + j * kTbThreads;
    const int l = q / (HY * HP), rem = q - l * (HY * HP), hy = rem / HP, hp = rem - hy * HP;
    const int gx = x0 - H + 2 * hp, gy = y0 - H + hy;
    at[j] = (l << 16) | (hy << 8) | hp;
    dist[j] = kOut | (kOut << 8);
    if (q < NQ && gx >= 0 && gx < X && gy >= 0 && gy < ny) {
      load_pair_coefs<T, NL>(G, gE, gN, gU, invD, l, gy, gx, pr[j]);
      const int er = (gy + l) & 1;  // gx is even: the pair's red node is gx + er
      const int dy = max(max(y0 - gy, gy - (y0 + TY - 1)), 0);
      const int xr = gx + er, xb = gx + 1 - er;
      const int dr = max(max(max(x0 - xr, xr - (x0 + kTileX - 1)), 0), dy);
      const int db = max(max(max(x0 - xb, xb - (x0 + kTileX - 1)), 0), dy);
      dist[j] = dr | (db << 8);
    }
  }

  // The tile's scenarios (one, or with MULTI a scenario block's tl.pad) in turn: stage the old
  // correction and r, sweep K times on chip, write the tile.
  bool first = true;
  const int nsc = MULTI ? tl.pad : 1;
  for (int sc = 0; sc < nsc; ++sc) {
    if (!c.active[tl.item + sc]) continue;  // uniform across the block
    const int64_t off = (int64_t)(tl.scen + sc) * G.nstore;
    const T* __restrict__ dold = static_cast<const T*>(G.d[din]) + off;
    T* __restrict__ dnew = static_cast<T*>(G.d[din ^ 1]) + off;
    const T* __restrict__ r = static_cast<const T*>(G.r) + off;
    if (!first) __syncthreads();  // the previous scenario is done with sd
    first = false;
    {
      V2<T> dv[J];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        dv[j] = zero2<T>();
        if ((dist[j] & 0xff) != kOut) {  // inside the mesh
          const int l = at[j] >> 16, hy = (at[j] >> 8) & 0xff, hp = at[j] & 0xff;
          const int64_t i = l * P + (int64_t)(y0 - H + hy) * X + (x0 - H + 2 * hp);
          if (!zero_in) dv[j] = ld2(dold, i);
          pr[j].rr = ld2n(r, i);
        }
      }
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int q = threadIdx.x + j * kTbThreads;
        if (q < NQ) (&sd[0][0][0])[q] = dv[j];
      }
    }
    __syncthreads();

    // Each pair update first issues all its LDS reads, then computes and writes; a pair outside
    // the half-sweep's box reads its own word in place of every neighbour and writes nothing, so
    // the reads carry no branch and the compiler can run them ahead of the previous pair's update.
    // Within a half-sweep the words written (this colour) are read only by the thread that owns
    // them.  The update is relax()'s expression, term for term.
    const T* __restrict__ fs = reinterpret_cast<const T*>(&sd[0][0][0]);  // element k of pair q at 2q + k
    T* __restrict__ fw = reinterpret_cast<T*>(&sd[0][0][0]);
#pragma unroll
    for (int i = 1; i <= 2 * K; ++i) {
      const int colour = (i - 1) & 1;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int dc = colour ? (dist[j] >> 8) : (dist[j] & 0xff);
        const bool ok = dc <= H - i;  // inside this half-sweep's box (never for nodes outside the mesh)
        const int l = at[j] >> 16, hy = (at[j] >> 8) & 0xff, hp = at[j] & 0xff;
        const int q = (l * HY + hy) * HP + hp;
        const int e = ((y0 - H + hy + l) & 1) ^ colour;  // element of the pair with this colour
        const int me = 2 * q + e;
        const V2<T> own = sd[l][hy][hp];
        // the one in-plane x neighbour in another pair: the east pair's element 0 for e = 1, the
        // west pair's element 1 for e = 0
        const T side = fs[ok ? (e ? 2 * q + 2 : 2 * q - 1) : me];
        const T nn = fs[ok ? me + 2 * HP : me];
        const T ss = fs[ok ? me - 2 * HP : me];
        T uu = T(0), dd = T(0);
        if (NL > 1) {
          uu = fs[ok && l < NL - 1 ? me + 2 * HY * HP : me];
          dd = fs[ok && l > 0 ? me - 2 * HY * HP : me];
        }
        if (!ok) continue;
        const NodeCoef<T> k = node_of(pr[j], e);
        const T old = pick(own, e);
        const T east = e ? side : own.y;
        const T west = e ? own.x : side;
        T acc = k.r + k.e * east + k.w * west + k.n * nn + k.s * ss;
        if (NL > 1) {
          if (l < NL - 1) acc += k.u * uu;
          if (l > 0) acc += k.d * dd;
        }
        const T nv = old + omega * (k.inv * acc - old);
        if (i < 2 * K) {
          fw[me] = nv;
        } else {  // the tile's black nodes: write the pair with its red partner's final value
          V2<T> out = own;
          put(out, e, nv);
          st2(dnew, l * P + (int64_t)(y0 - H + hy) * X + (x0 - H + 2 * hp), out);
        }
      }
      if (i < 2 * K) __syncthreads();
    }
  }
}

template <typename T, int K, int NL, int TY, bool MULTI>
void tb_t(const Tile* tiles, int ntiles, const GridDesc* grids, const Ctl& c, int din, int zero_in, double omega,
          hipStream_t s) {
  hipLaunchKernelGGL((k_sweep_tb<T, NL, TY, K, MULTI>), dim3(xcd_blocks(ntiles)), dim3(kTbThreads), 0, s, tiles,
                     ntiles, grids, c, din, zero_in, (T)omega);
}

// The shapes instantiated below, those whose staged pairs' registers fit without spilling, as
// k * 1000 + layers * 100 + tile rows: FP32 single-scenario tiles and scenario blocks (whose
// scenario loop keeps more registers live), FP64 (twice the registers per staged pair) likewise.
constexpr int kTbShapes32[] = {4104, 4108, 4116, 4204, 4208,
                               2104, 2108, 2116, 2204, 2208, 2216, 2304, 2308, 2316, 2404, 2408};
constexpr int kTbMulti32[] = {4104, 4108, 4116, 4204, 2104, 2108, 2116, 2204, 2208, 2304};
constexpr int kTbShapes64[] = {4104, 4108, 4116, 2104, 2108, 2116, 2204};
constexpr int kTbMulti64[] = {2104, 2108, 2116};

template <size_t N>
bool in_list(const int (&a)[N], int key) {
  for (int v : a)
    if (v == key) return true;
  return false;
}

}  // namespace

bool sweep_tb_supported(bool fp32, bool multi, int ordering, int nl, int tile_rows, int k) {
  if (ordering != 0) return false;  // red-black sweeps
  const int key = k * 1000 + nl * 100 + tile_rows;
  if (fp32) return multi ? in_list(kTbMulti32, key) : in_list(kTbShapes32, key);
  return multi ? in_list(kTbMulti64, key) : in_list(kTbShapes64, key);
}

hipError_t launch_sweep_tb(bool fp32, int k, bool multi, int nl, int tile_rows, const Tile* tiles, int ntiles,
                           const GridDesc* grids, const Ctl& c, int din, int zero_in, double omega, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (!sweep_tb_supported(fp32, multi, 0, nl, tile_rows, k)) return hipErrorInvalidValue;
  const int key = k * 1000 + nl * 100 + tile_rows;
#define PG_TB(T, K, NL, TY)                                                   \
  case K * 1000 + NL * 100 + TY:                                              \
    tb_t<T, K, NL, TY, false>(tiles, ntiles, grids, c, din, zero_in, omega, s); \
    break;
#define PG_TB_BOTH(T, K, NL, TY)                                              \
  case K * 1000 + NL * 100 + TY:                                              \
    if (multi)                                                                \
      tb_t<T, K, NL, TY, true>(tiles, ntiles, grids, c, din, zero_in, omega, s); \
    else                                                                      \
      tb_t<T, K, NL, TY, false>(tiles, ntiles, grids, c, din, zero_in, omega, s); \
    break;
  if (fp32) {
    switch (key) {
      PG_TB_BOTH(float, 4, 1, 4) PG_TB_BOTH(float, 4, 1, 8) PG_TB_BOTH(float, 4, 1, 16)
      PG_TB_BOTH(float, 4, 2, 4) PG_TB(float, 4, 2, 8)
      PG_TB_BOTH(float, 2, 1, 4) PG_TB_BOTH(float, 2, 1, 8) PG_TB_BOTH(float, 2, 1, 16)
      PG_TB_BOTH(float, 2, 2, 4) PG_TB_BOTH(float, 2, 2, 8) PG_TB(float, 2, 2, 16)
      PG_TB_BOTH(float, 2, 3, 4) PG_TB(float, 2, 3, 8) PG_TB(float, 2, 3, 16)
      PG_TB(float, 2, 4, 4) PG_TB(float, 2, 4, 8)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (key) {
      PG_TB(double, 4, 1, 4) PG_TB(double, 4, 1, 8) PG_TB(double, 4, 1, 16)
      PG_TB_BOTH(double, 2, 1, 4) PG_TB_BOTH(double, 2, 1, 8) PG_TB_BOTH(double, 2, 1, 16)
      PG_TB(double, 2, 2, 4)
      default: return hipErrorInvalidValue;
    }
  }
#undef PG_TB
#undef PG_TB_BOTH
  return hipGetLastError();
}

}  // namespace pgrid
