// Device helpers shared by the layered-mesh kernels (kernels.hip, kernels_tb.hip): node pairs
// as two-element vectors in the global segment, a pair's coefficients as they come from memory,
// and the SOR update of one staged node (eqs. 16-17).
#pragma once

#include "pgrid_internal.h"

namespace pgrid {

namespace {

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };
template <typename T> using V2 = typename Vec2<T>::type;

// Pairs move through the global segment (ld1 in pgrid_internal.h says why) as native
// two-element vectors: the HIP vector classes copy through generic references, which would turn
// the access back into a flat one.
template <typename T> using NV2 = T __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ V2<T> ld2(const T* __restrict__ p, int64_t i) {
  const NV2<T> w = *((const PG_GLOBAL NV2<T>*)(p + i));
  V2<T> v;
  v.x = w.x;
  v.y = w.y;
  return v;
}
template <typename T>
__device__ __forceinline__ void st2(T* __restrict__ p, int64_t i, V2<T> v) {
  NV2<T> w;
  w.x = v.x;
  w.y = v.y;
  *((PG_GLOBAL NV2<T>*)(p + i)) = w;
}
template <typename V>
__device__ __forceinline__ auto pick(const V& v, int e) -> decltype(v.x) { return e ? v.y : v.x; }
template <typename T>
__device__ __forceinline__ V2<T> zero2() { V2<T> z; z.x = T(0); z.y = T(0); return z; }


// Coefficients of one node of a pair: the conductances to its six neighbours, 1/M_ii, r_i.
template <typename T>
struct NodeCoef {
  T e, w, n, s, u, d, inv, r;
};

// Load the pair's coefficients without the right-hand side and return those of element `e`
// (0: even node, 1: odd node); `other` receives the partner's.  Conductances beyond the mesh
// are stored as zero, so only the array bounds are guarded.
template <typename T, int NL>
__device__ __forceinline__ void load_pair_coef(const GridDesc& G, const T* __restrict__ gE,
                                               const T* __restrict__ gN, const T* __restrict__ gU,
                                               const T* __restrict__ invD, int l, int y, int x, int e,
                                               NodeCoef<T>& mine, NodeCoef<T>& other) {
  const int64_t P = (int64_t)G.X * G.ny;
  const int64_t i = l * P + (int64_t)y * G.X + x;
  const V2<T> ge = ld2(gE, i), gn = ld2(gN, i), iv = ld2(invD, i);
  const V2<T> gs = y > 0 ? ld2(gN, i - G.X) : zero2<T>();
  const T gw = x > 0 ? ld1(gE, i - 1) : T(0);
  V2<T> gu = zero2<T>(), gd = zero2<T>();
  if (NL > 1) {
    if (l < NL - 1) gu = ld2(gU, i);
    if (l > 0) gd = ld2(gU, i - P);
  }
  // element 0: west edge is gE[x-1]; element 1: west edge is element 0's east edge
  NodeCoef<T> c0{ge.x, gw, gn.x, gs.x, gu.x, gd.x, iv.x, T(0)};
  NodeCoef<T> c1{ge.y, ge.x, gn.y, gs.y, gu.y, gd.y, iv.y, T(0)};
  mine = e ? c1 : c0;
  other = e ? c0 : c1;
}

// load_pair_coef plus the pair's right-hand side r.
template <typename T, int NL>
__device__ __forceinline__ void load_pair(const GridDesc& G, const T* __restrict__ gE,
                                          const T* __restrict__ gN, const T* __restrict__ gU,
                                          const T* __restrict__ invD, const T* __restrict__ r,
                                          int l, int y, int x, int e, NodeCoef<T>& mine,
                                          NodeCoef<T>& other) {
  load_pair_coef<T, NL>(G, gE, gN, gU, invD, l, y, x, e, mine, other);
  const V2<T> rr = ld2(r, l * (int64_t)G.X * G.ny + (int64_t)y * G.X + x);
  mine.r = pick(rr, e);
  other.r = pick(rr, 1 - e);
}

// A pair's coefficients and right-hand side as they come from memory (both nodes, as native
// vectors), so a kernel can issue the loads of one layer while it computes another, and pick a
// node's values only where it uses them.
template <typename T>
struct PairRaw {
  NV2<T> ge, gn, gs, gu, gd, iv, rr;
  T gw;
};

template <typename T>
__device__ __forceinline__ NV2<T> ld2n(const T* __restrict__ p, int64_t i) {
  return *((const PG_GLOBAL NV2<T>*)(p + i));
}

template <typename T, int NL>
__device__ __forceinline__ void load_pair_raw(const GridDesc& G, const T* __restrict__ gE, const T* __restrict__ gN,
                                              const T* __restrict__ gU, const T* __restrict__ invD,
                                              const T* __restrict__ r, int l, int y, int x, PairRaw<T>& p) {
  const int64_t P = (int64_t)G.X * G.ny;
  const int64_t i = l * P + (int64_t)y * G.X + x;
  const NV2<T> z = {T(0), T(0)};
  p.ge = ld2n(gE, i);
  p.gn = ld2n(gN, i);
  p.iv = ld2n(invD, i);
  p.rr = ld2n(r, i);
  p.gs = y > 0 ? ld2n(gN, i - G.X) : z;
  p.gw = x > 0 ? ld1(gE, i - 1) : T(0);
  p.gu = z;
  p.gd = z;
  if (NL > 1) {
    if (l < NL - 1) p.gu = ld2n(gU, i);
    if (l > 0) p.gd = ld2n(gU, i - P);
  }
}

// Element e of a raw pair (element 1's west edge is element 0's east edge).
template <typename T>
__device__ __forceinline__ NodeCoef<T> node_of(const PairRaw<T>& p, int e) {
  const NV2<T> ge = p.ge, gn = p.gn, gs = p.gs, gu = p.gu, gd = p.gd, iv = p.iv, rr = p.rr;
  NodeCoef<T> k;
  k.e = e ? ge.y : ge.x;
  k.w = e ? ge.x : p.gw;
  k.n = e ? gn.y : gn.x;
  k.s = e ? gs.y : gs.x;
  k.u = e ? gu.y : gu.x;
  k.d = e ? gd.y : gd.x;
  k.inv = e ? iv.y : iv.x;
  k.r = e ? rr.y : rr.x;
  return k;
}

// One node's coefficients and right-hand side, word by word (node xn of row y, layer l): the
// words load_pair_raw reads for that node.
template <typename T, int NL>
__device__ __forceinline__ NodeCoef<T> load_node(const GridDesc& G, const T* __restrict__ gE,
                                                 const T* __restrict__ gN, const T* __restrict__ gU,
                                                 const T* __restrict__ invD, const T* __restrict__ r, int l, int y,
                                                 int xn) {
  const int64_t P = (int64_t)G.X * G.ny;
  const int64_t i = l * P + (int64_t)y * G.X + xn;
  NodeCoef<T> k;
  k.e = ld1(gE, i);
  k.w = xn > 0 ? ld1(gE, i - 1) : T(0);
  k.n = ld1(gN, i);
  k.s = y > 0 ? ld1(gN, i - G.X) : T(0);
  k.u = T(0);
  k.d = T(0);
  if (NL > 1) {
    if (l < NL - 1) k.u = ld1(gU, i);
    if (l > 0) k.d = ld1(gU, i - P);
  }
  k.inv = ld1(invD, i);
  k.r = ld1(r, i);
  return k;
}

// SOR update of element e of the staged pair (l, hy, hp) from its staged neighbours.
template <typename T, int NL, int HY, int HP>
__device__ __forceinline__ T relax(const V2<T> (*sd)[HY][HP], int l, int hy, int hp, int e,
                                   const NodeCoef<T>& k, T omega) {
  const V2<T> own = sd[l][hy][hp];
  const T old = pick(own, e);
  const T east = e ? sd[l][hy][hp + 1].x : own.y;
  const T west = e ? own.x : sd[l][hy][hp - 1].y;
  T acc = k.r + k.e * east + k.w * west + k.n * pick(sd[l][hy + 1][hp], e) +
          k.s * pick(sd[l][hy - 1][hp], e);
  if (NL > 1) {
    if (l < NL - 1) acc += k.u * pick(sd[l + 1][hy][hp], e);
    if (l > 0) acc += k.d * pick(sd[l - 1][hy][hp], e);
  }
  return old + omega * (k.inv * acc - old);
}

template <typename V, typename T>
__device__ __forceinline__ void put(V& v, int e, T val) {
  if (e) v.y = val; else v.x = val;
}

}  // namespace

}  // namespace pgrid
