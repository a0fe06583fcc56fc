// General netlists (Sec. III, eqs. 4-9) in the form the gather-based sweep kernels use: the
// trivial nodes are coloured so that no branch joins two nodes of one colour, then stored
// colour by colour, so one colour is a set of independent Gauss-Seidel updates (eq. 16) and a
// sweep visits the colours in order (Theorem 1: any order converges).  Host code.

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <set>
#include <utility>
#include <vector>

#include "graph_form.h"

namespace pgrid {

namespace {

pg_status gfail(pg_status st, char* msg, size_t len, const char* fmt, ...) {
  if (msg && len) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(msg, len, fmt, ap);
    va_end(ap);
  }
  return st;
}

// DSATUR: repeatedly colour the uncoloured node whose neighbours already show the most distinct
// colours (ties: smallest node id) with the smallest colour none of them holds.  Returns the
// number of colours, or 0 if a node would need a colour beyond 63 (the caller then falls back).
int dsatur(int32_t n, const std::vector<int64_t>& off, const std::vector<int32_t>& adj, std::vector<int32_t>& color) {
  color.assign(n, -1);
  std::vector<uint64_t> seen(n, 0);  // colours held by coloured neighbours
  std::vector<int> sat(n, 0);
  std::vector<std::set<int32_t>> bucket(1);
  for (int32_t i = 0; i < n; ++i) bucket[0].insert(bucket[0].end(), i);
  int top = 0, nc = 0;
  for (int32_t done = 0; done < n; ++done) {
    while (bucket[top].empty()) --top;
    const int32_t u = *bucket[top].begin();
    bucket[top].erase(bucket[top].begin());
    if (~seen[u] == 0) return 0;
    const int c = __builtin_ctzll(~seen[u]);
    color[u] = c;
    nc = std::max(nc, c + 1);
    const uint64_t bit = 1ull << c;
    for (int64_t k = off[u]; k < off[u + 1]; ++k) {
      const int32_t w = adj[k];
      if (color[w] >= 0 || (seen[w] & bit)) continue;
      seen[w] |= bit;
      bucket[sat[w]].erase(w);
      ++sat[w];
      if ((int)bucket.size() <= sat[w]) bucket.resize(sat[w] + 1);
      bucket[sat[w]].insert(w);
      top = std::max(top, sat[w]);
    }
  }
  return nc;
}

// Two colours when the node graph is bipartite (breadth-first parity per connected part),
// else DSATUR (or, should that run past 64 colours, the greedy colouring in node order: each
// node takes the smallest colour none of its earlier neighbours holds).
int colour_nodes(int32_t n, const std::vector<int64_t>& off, const std::vector<int32_t>& adj,
                 std::vector<int32_t>& color) {
  color.assign(n, -1);
  bool bip = true;
  std::deque<int32_t> q;
  for (int32_t s = 0; s < n && bip; ++s) {
    if (color[s] >= 0) continue;
    color[s] = 0;
    q.assign(1, s);
    while (!q.empty() && bip) {
      const int32_t u = q.front();
      q.pop_front();
      for (int64_t k = off[u]; k < off[u + 1]; ++k) {
        const int32_t w = adj[k];
        if (color[w] < 0) {
          color[w] = color[u] ^ 1;
          q.push_back(w);
        } else if (color[w] == color[u]) {
          bip = false;
          break;
        }
      }
    }
  }
  if (bip) {
    int nc = 0;
    for (int32_t i = 0; i < n; ++i) nc = std::max(nc, color[i] + 1);
    return nc;
  }
  int nd = dsatur(n, off, adj, color);
  if (nd > 0) {
    // iterated greedy (Culberson): recolour greedily, taking the colour classes as blocks in
    // reverse order (nodes in id order inside a class); this never adds a colour and often
    // empties the last, smallest classes
    std::vector<int32_t> order(n), mark;
    for (int pass = 0; pass < 16 && nd > 2; ++pass) {
      std::vector<int64_t> cnt(nd + 1, 0);
      for (int32_t i = 0; i < n; ++i) cnt[nd - 1 - color[i] + 1]++;
      for (int c = 0; c < nd; ++c) cnt[c + 1] += cnt[c];
      for (int32_t i = 0; i < n; ++i) order[cnt[nd - 1 - color[i]]++] = i;
      std::vector<int32_t> nc2(n, -1);
      mark.assign(nd + 1, -1);
      int used = 0;
      for (int32_t u : order) {
        for (int64_t k = off[u]; k < off[u + 1]; ++k)
          if (nc2[adj[k]] >= 0) mark[nc2[adj[k]]] = u;
        int cu = 0;
        while (mark[cu] == u) ++cu;
        nc2[u] = cu;
        used = std::max(used, cu + 1);
      }
      const bool better = used < nd;
      color.swap(nc2);
      nd = used;
      if (!better && pass >= 3) break;
    }
    return nd;
  }
  color.assign(n, -1);
  int nc = 0;
  std::vector<int32_t> mark;  // mark[c] == u + 1: colour c is taken by a neighbour of u
  for (int32_t u = 0; u < n; ++u) {
    for (int64_t k = off[u]; k < off[u + 1]; ++k) {
      const int32_t cw = color[adj[k]];
      if (cw >= 0) {
        if ((int)mark.size() <= cw) mark.resize(cw + 1, 0);
        mark[cw] = u + 1;
      }
    }
    int cu = 0;
    while (cu < (int)mark.size() && mark[cu] == u + 1) ++cu;
    color[u] = cu;
    nc = std::max(nc, cu + 1);
  }
  return nc;
}

// Cuthill-McKee order: breadth first from a pseudo-peripheral node of each connected part (the
// parts in the order of their smallest node), the unvisited neighbours of a node taken by
// increasing degree (ties: node id).  A node's neighbours then lie in the breadth-first levels
// next to its own, so on mesh-like graphs they sit about one level width apart in this order
// whatever the numbering (the layers of a layered grid interleave, vias joining nearby slots).
std::vector<int32_t> cm_order(int32_t n, const std::vector<int64_t>& off, const std::vector<int32_t>& adj) {
  std::vector<int32_t> order, q, level(n, 0), stamp(n, -1), nb;
  std::vector<char> placed(n, 0);
  order.reserve(n);
  auto deg = [&](int32_t u) { return off[u + 1] - off[u]; };
  auto before = [&](int32_t a, int32_t b) { return deg(a) != deg(b) ? deg(a) < deg(b) : a < b; };
  int32_t pass = 0;
  for (int32_t s0 = 0; s0 < n; ++s0) {
    if (placed[s0]) continue;
    // pseudo-peripheral root: from s0, move to a least-degree node of the deepest level while
    // the depth grows
    int32_t root = s0, depth = -1;
    for (int it = 0; it < 8; ++it) {
      ++pass;
      q.assign(1, root);
      stamp[root] = pass;
      level[root] = 0;
      for (size_t h = 0; h < q.size(); ++h) {
        const int32_t u = q[h];
        for (int64_t k = off[u]; k < off[u + 1]; ++k)
          if (stamp[adj[k]] != pass) {
            stamp[adj[k]] = pass;
            level[adj[k]] = level[u] + 1;
            q.push_back(adj[k]);
          }
      }
      const int32_t d = level[q.back()];
      if (d <= depth) break;
      depth = d;
      int32_t best = q.back();
      for (size_t t = q.size(); t-- > 0 && level[q[t]] == d;)
        if (before(q[t], best)) best = q[t];
      root = best;
    }
    q.assign(1, root);
    placed[root] = 1;
    for (size_t h = 0; h < q.size(); ++h) {
      const int32_t u = q[h];
      order.push_back(u);
      nb.clear();
      for (int64_t k = off[u]; k < off[u + 1]; ++k)
        if (!placed[adj[k]]) {
          placed[adj[k]] = 1;
          nb.push_back(adj[k]);
        }
      std::sort(nb.begin(), nb.end(), before);
      q.insert(q.end(), nb.begin(), nb.end());
    }
  }
  return order;
}

}  // namespace

pg_status build_graph_form(int32_t n, int32_t p, const double* source_v, int32_t m, const int32_t* from,
                           const int32_t* to, const uint8_t* kind, const double* value, GraphForm& f,
                           char* msg, size_t len) {
  pg_status st = pg_validate_netlist(n, p, m, from, to, kind, value, msg, len);
  if (st != PG_OK) return st;
  if (p > 0 && !source_v) return gfail(PG_ERR_INVALID_ARG, msg, len, "source voltages are NULL");
  for (int j = 0; j < p; ++j)
    if (!std::isfinite(source_v[j])) return gfail(PG_ERR_INVALID_ARG, msg, len, "source %d: voltage not finite", j);
  f = GraphForm{};
  f.n = n;
  f.c_diag.assign(n, 0.0);
  f.g_diag.assign(n, 0.0);
  f.b_res.assign(n, 0.0);
  auto triv = [&](int32_t a) { return a >= 0 && a < n; };
  auto fixed_v = [&](int32_t a) { return a < 0 ? 0.0 : source_v[a - n]; };  // ground or a supply
  // node pairs joined by R, L or C (one record per branch, merged below)
  struct PairVal { int32_t a, b; double g, il, c; };
  std::vector<PairVal> pv;
  for (int e = 0; e < m; ++e) {
    const int32_t a = from[e], b = to[e];
    const uint8_t k = kind[e];
    const double v = value[e];
    if (k == 'I') continue;  // positions of current sources; waveforms are set per scenario
    const bool ta = triv(a), tb = triv(b);
    if (k == 'L') {
      // the branch current flows from -> to; near is a trivial end
      const int32_t near = ta ? a : b, far = ta ? b : a;
      f.ind_near.push_back(near);
      f.ind_far.push_back(triv(far) ? far : -1);
      f.ind_inv_l.push_back(1.0 / v);
      f.ind_far_v.push_back(triv(far) ? 0.0 : fixed_v(far));
      f.ind_sign.push_back(ta ? 1 : -1);
    }
    if (ta && tb) {
      pv.push_back(PairVal{std::min(a, b), std::max(a, b), k == 'R' ? v : 0.0, k == 'L' ? 1.0 / v : 0.0,
                           k == 'C' ? v : 0.0});
      if (k == 'C') f.has_coupling = true;
    }
    for (int32_t end : {a, b}) {
      if (!triv(end)) continue;
      if (k == 'C') f.c_diag[end] += v;
      if (k == 'R') f.g_diag[end] += v;
    }
    if (k == 'R' && (ta != tb)) {
      const int32_t t = ta ? a : b, o = ta ? b : a;
      f.b_res[t] += v * fixed_v(o);
    }
  }
  std::sort(pv.begin(), pv.end(), [](const PairVal& x, const PairVal& y) {
    return x.a != y.a ? x.a < y.a : x.b < y.b;
  });
  std::vector<PairVal> pairs;
  for (const PairVal& q : pv) {
    if (!pairs.empty() && pairs.back().a == q.a && pairs.back().b == q.b) {
      pairs.back().g += q.g; pairs.back().il += q.il; pairs.back().c += q.c;
    } else {
      pairs.push_back(q);
    }
  }
  // adjacency (both directions), neighbours in node order
  std::vector<int64_t> off(n + 1, 0);
  for (const PairVal& q : pairs) { off[q.a + 1]++; off[q.b + 1]++; }
  for (int32_t i = 0; i < n; ++i) off[i + 1] += off[i];
  std::vector<int32_t> adj(off[n]);
  std::vector<int32_t> pid(off[n]);
  {
    std::vector<int64_t> fill(off.begin(), off.end() - 1);
    for (size_t k = 0; k < pairs.size(); ++k) {
      adj[fill[pairs[k].a]] = pairs[k].b; pid[fill[pairs[k].a]++] = (int32_t)k;
      adj[fill[pairs[k].b]] = pairs[k].a; pid[fill[pairs[k].b]++] = (int32_t)k;
    }
  }
  f.nnz = off[n];
  {
    std::vector<int32_t> parent(n);
    for (int32_t i = 0; i < n; ++i) parent[i] = i;
    auto find = [&](int32_t i) {
      while (parent[i] != i) i = parent[i] = parent[parent[i]];
      return i;
    };
    std::vector<char> rfix(n, 0);
    for (const PairVal& q : pairs)
      if (q.g > 0) parent[find(q.a)] = find(q.b);
    for (int e = 0; e < m; ++e)
      if (kind[e] == 'R' && (triv(from[e]) != triv(to[e]))) rfix[triv(from[e]) ? from[e] : to[e]] = 1;
    std::vector<char> ok(n, 0);
    for (int32_t i = 0; i < n; ++i)
      if (rfix[i]) ok[find(i)] = 1;
    f.dc_anchored = true;
    for (int32_t i = 0; i < n && f.dc_anchored; ++i) f.dc_anchored = ok[find(i)] != 0;
  }
  f.ncolors = colour_nodes(n, off, adj, f.color);
  if (f.ncolors > 255)
    return gfail(PG_ERR_UNSUPPORTED, msg, len, "the node graph needs %d colours (at most 255)", f.ncolors);
  // slots: colour by colour, Cuthill-McKee order inside a colour (so the neighbours a wavefront
  // gathers lie close together in each colour, at about the same relative position as the
  // wavefront's own slots in theirs), each colour padded to whole slices
  std::vector<int64_t> count(f.ncolors, 0);
  for (int32_t i = 0; i < n; ++i) count[f.color[i]]++;
  f.cstart.assign(f.ncolors + 1, 0);
  for (int c = 0; c < f.ncolors; ++c)
    f.cstart[c + 1] = f.cstart[c] + (count[c] + kSlice - 1) / kSlice * kSlice;
  f.nslots = f.cstart[f.ncolors];
  if (f.nslots > (int64_t)INT32_MAX / 2) return gfail(PG_ERR_UNSUPPORTED, msg, len, "too many nodes");
  f.slot.assign(n, 0);
  std::vector<int32_t> node_at(f.nslots, -1);
  {
    std::vector<int64_t> next(f.cstart.begin(), f.cstart.end() - 1);
    for (const int32_t i : cm_order(n, off, adj)) {
      const int64_t s = next[f.color[i]]++;
      f.slot[i] = (int32_t)s;
      node_at[s] = i;
    }
  }
  // compact sliced ELL (see GraphForm): row lengths, slice extents, then entry k of each row
  // that has one, k = 0, 1, ...
  const int64_t nsl = f.nslots / kSlice;
  f.rlen.assign(f.nslots, 0);
  for (int64_t s = 0; s < f.nslots; ++s) {
    const int32_t i = node_at[s];
    if (i < 0) continue;
    const int64_t deg = off[i + 1] - off[i];
    if (deg > kMaxRowLen)
      return gfail(PG_ERR_UNSUPPORTED, msg, len, "node %d has %lld neighbours (at most %d)", i, (long long)deg,
                   kMaxRowLen);
    f.rlen[s] = (uint16_t)deg;
  }
  f.soff.assign(nsl + 1, 0);
  int64_t total = 0;
  for (int64_t s = 0; s < nsl; ++s) {
    for (int j = 0; j < kSlice; ++j) total += f.rlen[s * kSlice + j];
    if (total > (int64_t)INT32_MAX)
      return gfail(PG_ERR_UNSUPPORTED, msg, len, "the neighbour table exceeds 2^31 entries");
    f.soff[s + 1] = (int32_t)total;
  }
  f.col.assign(total, 0);
  f.g.assign(total, 0.0);
  f.inv_l.assign(total, 0.0);
  f.cc.assign(total, 0.0);
  std::vector<std::vector<std::pair<int32_t, int32_t>>> rows(kSlice);  // (neighbour slot, pair)
  for (int64_t s = 0; s < nsl; ++s) {
    size_t w = 0;
    for (int j = 0; j < kSlice; ++j) {
      const int32_t i = node_at[s * kSlice + j];
      rows[j].clear();
      if (i >= 0)
        for (int64_t k = off[i]; k < off[i + 1]; ++k) rows[j].emplace_back(f.slot[adj[k]], pid[k]);
      std::sort(rows[j].begin(), rows[j].end());
      w = std::max(w, rows[j].size());
    }
    int64_t e = f.soff[s];
    for (size_t k = 0; k < w; ++k)
      for (int j = 0; j < kSlice; ++j) {
        if (k >= rows[j].size()) continue;
        const PairVal& q = pairs[rows[j][k].second];
        f.col[e] = rows[j][k].first;
        f.g[e] = q.g;
        f.inv_l[e] = q.il;
        f.cc[e] = q.c;
        ++e;
      }
  }
  // coupling-capacitor table (padded sliced ELL)
  f.csoff.assign(nsl + 1, 0);
  int64_t ctotal = 0;
  std::vector<std::vector<std::pair<int32_t, double>>> crow(kSlice);
  for (int64_t s = 0; s < nsl; ++s) {
    int64_t w = 0;
    for (int j = 0; j < kSlice; ++j) {
      const int32_t i = node_at[s * kSlice + j];
      crow[j].clear();
      if (i >= 0)
        for (int64_t k = off[i]; k < off[i + 1]; ++k)
          if (pairs[pid[k]].c > 0) crow[j].emplace_back(f.slot[adj[k]], pairs[pid[k]].c);
      std::sort(crow[j].begin(), crow[j].end());
      w = std::max<int64_t>(w, (int64_t)crow[j].size());
    }
    for (int64_t k = 0; k < w; ++k)
      for (int j = 0; j < kSlice; ++j) {
        const bool has = k < (int64_t)crow[j].size();
        f.ccol.push_back(has ? crow[j][k].first : (int32_t)(s * kSlice + j));
        f.cval.push_back(has ? crow[j][k].second : 0.0);
      }
    ctotal += w * kSlice;
    if (ctotal > (int64_t)INT32_MAX)
      return gfail(PG_ERR_UNSUPPORTED, msg, len, "the padded capacitor table exceeds 2^31 entries");
    f.csoff[s + 1] = (int32_t)ctotal;
  }
  return PG_OK;
}

}  // namespace pgrid

extern "C" {

pg_status pg_netlist_coloring(int32_t n, int32_t p, const double* source_v, int32_t m, const int32_t* from,
                              const int32_t* to, const uint8_t* kind, const double* value, int32_t* color,
                              int32_t* slot, int32_t* n_colors, int64_t* n_slots, char* msg, size_t msg_len) {
  pgrid::GraphForm f;
  pg_status st = pgrid::build_graph_form(n, p, source_v, m, from, to, kind, value, f, msg, msg_len);
  if (st != PG_OK) return st;
  if (color) std::copy(f.color.begin(), f.color.end(), color);
  if (slot) std::copy(f.slot.begin(), f.slot.end(), slot);
  if (n_colors) *n_colors = f.ncolors;
  if (n_slots) *n_slots = f.nslots;
  return PG_OK;
}

}  // extern "C"
