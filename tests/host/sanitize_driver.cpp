// Host-only driver for the library's validation, netlist-mapping and colouring code
// (validate.cpp, netlist.cpp, graph.cpp), built with AddressSanitizer and UndefinedBehavior-
// Sanitizer by tests/test_host_sanitizers.py.  These are the functions that enforce the
// topological assumptions of Sec. III-B and map a branch list (Sec. III, eqs. 4-6) onto the
// layered mesh or the colour-ordered graph form.  The driver feeds them seeded random meshes,
// their branch lists (R segments, R or series R-L vias and pads, C and I to ground, in random
// order and orientation), corrupted copies of both, and arbitrary branch lists, and checks:
//   * a mesh's branch list maps back onto exactly the mesh (pg_netlist_to_mesh round trip);
//   * the colouring joins no two nodes of one colour by an R, L or C branch, and the slots
//     are a permutation that follows the colours, each colour padded to a multiple of 64;
//   * walking the compact neighbour table level by level, as a wavefront does (the rows with
//     more than k entries take entry k in slot order), gives every node exactly its
//     neighbours, in increasing slot order, with the summed R, 1/L and C of the branches
//     joining each pair, and each slice's walk ends at the next slice's first entry;
//   * every corrupted input is refused with PG_ERR_INVALID_ARG;
//   * every status is one of pg_status, and messages are terminated within their buffers.
// The sanitizers report any out-of-bounds access, use after free, leak or undefined behaviour.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <vector>

#include "../../include/pgrid.h"
#include "../../paper_1409_7166_amd/csrc/graph_form.h"

// The device side is not linked: these runtime entry points are never reached from the
// host-only functions exercised here.
extern "C" pg_status pg_upload_mesh(pg_ctx*, const pg_mesh*, int32_t, int32_t*) { return PG_ERR_UNSUPPORTED; }
namespace pgrid {
pg_status report_error(pg_ctx*, pg_status st, const char*) { return st; }
pg_status upload_graph(pg_ctx*, GraphForm&, double, int32_t, int32_t*) { return PG_ERR_UNSUPPORTED; }
}  // namespace pgrid

namespace {

struct Rng {  // splitmix64
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  int below(int n) { return (int)(next() % (uint64_t)n); }
  double unit() { return (double)(next() >> 11) * 0x1.0p-53; }
  double range(double a, double b) { return a + (b - a) * unit(); }
};

int failures = 0;
int round_trips = 0, colourings = 0, accepted_arbitrary = 0, graphs_ok = 0;
#define CHECK(cond, ...)                                           \
  do {                                                             \
    if (!(cond)) {                                                 \
      std::fprintf(stderr, "check failed at line %d: ", __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                           \
      std::fprintf(stderr, "\n");                                  \
      ++failures;                                                  \
    }                                                              \
  } while (0)

bool known_status(pg_status s) { return s <= 0 && s >= PG_ERR_UNSUPPORTED; }

struct MeshData {
  int nx, ny, nl;
  std::vector<double> gE, gN, C, via_g, via_L, pad_g, pad_L;
  std::vector<int32_t> via_node, pad_node;
  double vdd;
  pg_mesh view() const {
    pg_mesh m{};
    m.nx = nx; m.ny = ny; m.nl = nl;
    m.gE = gE.data(); m.gN = gN.data(); m.C = C.data();
    m.n_vias = (int32_t)via_node.size(); m.via_node = via_node.data(); m.via_g = via_g.data(); m.via_L = via_L.data();
    m.n_pads = (int32_t)pad_node.size(); m.pad_node = pad_node.data(); m.pad_g = pad_g.data(); m.pad_L = pad_L.data();
    m.vdd = vdd;
    return m;
  }
};

MeshData random_mesh(Rng& r) {
  MeshData m;
  m.nx = 2 + r.below(9); m.ny = 2 + r.below(9); m.nl = 1 + r.below(4);
  const int P = m.nx * m.ny, n = P * m.nl;
  m.gE.resize((size_t)m.nl * m.ny * (m.nx - 1)); m.gN.resize((size_t)m.nl * (m.ny - 1) * m.nx); m.C.resize(n);
  for (auto& g : m.gE) g = r.range(0.5, 2.0);
  for (auto& g : m.gN) g = r.range(0.5, 2.0);
  for (auto& c : m.C) c = r.below(3) == 0 ? 0.0 : r.range(0.1e-12, 5e-12);
  std::vector<char> used(n, 0);
  for (int a = 0; a < P * (m.nl - 1); ++a)
    if (r.below(3) == 0) {  // at most one via per lower node, so the mapping cannot merge two
      m.via_node.push_back(a); m.via_g.push_back(r.range(1.0, 6.0));
      m.via_L.push_back(r.below(2) ? 0.0 : r.range(1e-12, 1e-11));
    }
  for (int a = 0; a < n; ++a)
    if (r.below(5) == 0) {
      m.pad_node.push_back(a); m.pad_g.push_back(r.range(5.0, 10.0));
      m.pad_L.push_back(r.below(2) ? 0.0 : r.range(1e-12, 1e-11));
    }
  m.vdd = r.below(4) == 0 ? 0.0 : r.range(0.7, 1.2);
  return m;
}

struct Netlist {
  int32_t n = 0, p = 1;
  std::vector<double> source_v;
  std::vector<int32_t> from, to;
  std::vector<uint8_t> kind;
  std::vector<double> value;
  void add(Rng& r, int a, int b, char k, double v, bool may_flip = true) {
    if (may_flip && r.below(2)) std::swap(a, b);
    from.push_back(a); to.push_back(b); kind.push_back((uint8_t)k); value.push_back(v);
  }
};

// The mesh's branch list: node (l, y, x) is (l*ny + y)*nx + x, the supply is node n, internal
// nodes of series R-L branches follow the mesh nodes.
Netlist mesh_netlist(Rng& r, const MeshData& m) {
  Netlist nl;
  const int P = m.nx * m.ny, nmesh = P * m.nl;
  int n_int = 0;
  for (double L : m.via_L) n_int += L > 0;
  for (double L : m.pad_L) n_int += L > 0;
  nl.n = nmesh + n_int;
  const int src = nl.n;
  nl.source_v = {m.vdd};
  int next_int = nmesh;
  for (int l = 0; l < m.nl; ++l)
    for (int y = 0; y < m.ny; ++y)
      for (int x = 0; x < m.nx; ++x) {
        const int i = (l * m.ny + y) * m.nx + x;
        if (x + 1 < m.nx) nl.add(r, i, i + 1, 'R', m.gE[((size_t)l * m.ny + y) * (m.nx - 1) + x]);
        if (y + 1 < m.ny) nl.add(r, i, i + m.nx, 'R', m.gN[((size_t)l * (m.ny - 1) + y) * m.nx + x]);
        if (m.C[i] > 0) nl.add(r, i, -1, 'C', m.C[i]);
        if (r.below(4) == 0) nl.add(r, i, -1, 'I', 0.0, false);
      }
  for (size_t k = 0; k < m.via_node.size(); ++k) {
    const int a = m.via_node[k], b = a + P;
    if (m.via_L[k] > 0) {
      const int q = next_int++;
      if (r.below(2)) { nl.add(r, a, q, 'R', m.via_g[k]); nl.add(r, q, b, 'L', m.via_L[k]); }
      else { nl.add(r, a, q, 'L', m.via_L[k]); nl.add(r, q, b, 'R', m.via_g[k]); }
    } else {
      nl.add(r, a, b, 'R', m.via_g[k]);
    }
  }
  for (size_t k = 0; k < m.pad_node.size(); ++k) {
    const int a = m.pad_node[k];
    if (m.pad_L[k] > 0) {
      const int q = next_int++;
      nl.add(r, a, q, 'R', m.pad_g[k]);
      nl.add(r, q, src, 'L', m.pad_L[k]);
    } else {
      nl.add(r, a, src, 'R', m.pad_g[k]);
    }
  }
  // shuffle the branch order
  for (int e = (int)nl.kind.size() - 1; e > 0; --e) {
    const int f = r.below(e + 1);
    std::swap(nl.from[e], nl.from[f]); std::swap(nl.to[e], nl.to[f]);
    std::swap(nl.kind[e], nl.kind[f]); std::swap(nl.value[e], nl.value[f]);
  }
  return nl;
}

void check_msg(const char* msg, size_t len) {
  if (len) CHECK(std::memchr(msg, 0, len) != nullptr, "message not terminated within %zu bytes", len);
}

void round_trip(Rng& r, const MeshData& m) {
  const pg_mesh mv = m.view();
  char msg[256];
  const pg_status vs = pg_validate_mesh(&mv, msg, sizeof msg);
  CHECK(vs == PG_OK || vs == PG_ERR_NOT_SPD, "pg_validate_mesh: %d (%s)", vs, msg);
  Netlist nl = mesh_netlist(r, m);
  const int32_t dims[3] = {m.nx, m.ny, m.nl};
  const int32_t mm = (int32_t)nl.kind.size();
  int32_t nv = -1, np = -1;
  pg_status s = pg_netlist_mesh_counts(nl.n, nl.p, nl.source_v.data(), mm, nl.from.data(), nl.to.data(),
                                       nl.kind.data(), nl.value.data(), dims, &nv, &np, msg, sizeof msg);
  if (vs == PG_ERR_NOT_SPD) {
    CHECK(s == PG_ERR_NOT_SPD, "an unanchored mesh's branch list gave %d", s);
    return;
  }
  CHECK(s == PG_OK, "pg_netlist_mesh_counts: %d (%s)", s, msg);
  if (s != PG_OK) return;
  CHECK(nv == (int)m.via_node.size() && np == (int)m.pad_node.size(), "counts %d %d", nv, np);
  std::vector<double> gE(m.gE.size()), gN(m.gN.size()), C(m.C.size()), vg(nv), vL(nv), pgv(np), pL(np);
  std::vector<int32_t> vn(nv), pn(np);
  double vdd = -1;
  s = pg_netlist_to_mesh(nl.n, nl.p, nl.source_v.data(), mm, nl.from.data(), nl.to.data(), nl.kind.data(),
                         nl.value.data(), dims, gE.data(), gN.data(), C.data(), vn.data(), vg.data(), vL.data(),
                         pn.data(), pgv.data(), pL.data(), &vdd, msg, sizeof msg);
  CHECK(s == PG_OK, "pg_netlist_to_mesh: %d (%s)", s, msg);
  CHECK(gE == m.gE && gN == m.gN && C == m.C, "segment or capacitance arrays differ after the round trip");
  CHECK(vn == m.via_node && vg == m.via_g && vL == m.via_L, "vias differ after the round trip");
  CHECK(pn == m.pad_node && pgv == m.pad_g && pL == m.pad_L, "pads differ after the round trip");
  CHECK(vdd == m.vdd, "vdd differs");
  ++round_trips;
  // the colour-ordered graph form of the same branch list
  std::vector<int32_t> color(nl.n, -1), slot(nl.n, -1);
  int32_t ncol = 0;
  int64_t nslots = 0;
  s = pg_netlist_coloring(nl.n, nl.p, nl.source_v.data(), mm, nl.from.data(), nl.to.data(), nl.kind.data(),
                          nl.value.data(), color.data(), slot.data(), &ncol, &nslots, msg, sizeof msg);
  CHECK(s == PG_OK, "pg_netlist_coloring: %d (%s)", s, msg);
  if (s != PG_OK) return;
  CHECK(ncol >= 1 && nslots % 64 == 0 && nslots >= nl.n, "colours %d slots %lld", ncol, (long long)nslots);
  for (int e = 0; e < mm; ++e) {
    const int a = nl.from[e], b = nl.to[e];
    if (nl.kind[e] == 'I' || a < 0 || b < 0 || a >= nl.n || b >= nl.n) continue;
    CHECK(color[a] != color[b], "branch %d joins two nodes of colour %d", e, color[a]);
  }
  std::vector<char> seen(nslots, 0);
  std::vector<int64_t> lo(ncol, INT64_MAX), hi(ncol, -1);
  for (int i = 0; i < nl.n; ++i) {
    CHECK(color[i] >= 0 && color[i] < ncol && slot[i] >= 0 && slot[i] < nslots, "node %d: colour/slot", i);
    if (!(slot[i] >= 0 && slot[i] < nslots && color[i] >= 0 && color[i] < ncol)) return;
    CHECK(!seen[slot[i]], "slot %d used twice", slot[i]);
    seen[slot[i]] = 1;
    lo[color[i]] = std::min<int64_t>(lo[color[i]], slot[i]);
    hi[color[i]] = std::max<int64_t>(hi[color[i]], slot[i]);
  }
  for (int c = 0; c + 1 < ncol; ++c)
    if (hi[c] >= 0 && lo[c + 1] != INT64_MAX) CHECK(hi[c] < lo[c + 1], "colour %d slots overlap colour %d", c, c + 1);
  for (int c = 0; c < ncol; ++c)
    if (lo[c] != INT64_MAX) CHECK(lo[c] % 64 == 0, "colour %d starts at slot %lld", c, (long long)lo[c]);
  ++colourings;
}

void corrupted_meshes(Rng& r, const MeshData& m0) {
  char msg[64];
  for (int t = 0; t < 8; ++t) {
    MeshData m = m0;
    switch (t) {
      case 0: m.gE[r.below((int)m.gE.size())] = NAN; break;
      case 1: m.gN[r.below((int)m.gN.size())] = -1.0; break;
      case 2: m.C[r.below((int)m.C.size())] = INFINITY; break;
      case 3: m.via_node.push_back(m.nx * m.ny * (m.nl - 1) + r.below(m.nx * m.ny));
              m.via_g.push_back(1.0); m.via_L.push_back(0.0); break;
      case 4: m.pad_node.push_back(-1 - r.below(5)); m.pad_g.push_back(1.0); m.pad_L.push_back(0.0); break;
      case 5: m.pad_node.push_back(m.nx * m.ny * m.nl + r.below(5)); m.pad_g.push_back(1.0); m.pad_L.push_back(0.0); break;
      case 6: m.pad_node.push_back(0); m.pad_g.push_back(0.0); m.pad_L.push_back(0.0); break;
      case 7: m.vdd = NAN; break;
    }
    const pg_mesh mv = m.view();
    const size_t len = (size_t)r.below(65);
    const pg_status s = pg_validate_mesh(&mv, len ? msg : nullptr, len);
    CHECK(s == PG_ERR_INVALID_ARG, "corruption %d of a mesh gave %d", t, s);
    if (len) check_msg(msg, len);
  }
}

void arbitrary_netlists(Rng& r) {
  const int n = 1 + r.below(40), p = r.below(3), m = r.below(120);
  std::vector<double> sv(p);
  for (auto& v : sv) v = r.below(6) == 0 ? NAN : r.range(0.5, 1.5);
  std::vector<int32_t> from(m), to(m);
  std::vector<uint8_t> kind(m);
  std::vector<double> value(m);
  const char kinds[] = {'R', 'R', 'R', 'C', 'L', 'I', 'X'};
  for (int e = 0; e < m; ++e) {
    from[e] = r.below(n + p + 3) - 2;
    to[e] = r.below(n + p + 3) - 2;
    kind[e] = (uint8_t)kinds[r.below(r.below(20) == 0 ? 7 : 6)];
    value[e] = r.below(30) == 0 ? -1.0 : (r.below(30) == 0 ? NAN : r.range(1e-3, 10.0));
  }
  char msg[128];
  const size_t len = (size_t)r.below(129);
  char* mp = len ? msg : nullptr;
  pg_status s = pg_validate_netlist(n, p, m, from.data(), to.data(), kind.data(), value.data(), mp, len);
  CHECK(known_status(s), "validate status %d", s);
  if (len) check_msg(msg, len);
  accepted_arbitrary += s == PG_OK;
  int32_t dims[3] = {2 + r.below(4), 2 + r.below(4), 1 + r.below(3)};
  int32_t nv = 0, np = 0;
  s = pg_netlist_mesh_counts(n, p, p ? sv.data() : nullptr, m, from.data(), to.data(), kind.data(), value.data(),
                             dims, &nv, &np, mp, len);
  CHECK(known_status(s), "counts status %d", s);
  if (s == PG_OK) {
    const int P = dims[0] * dims[1];
    std::vector<double> gE((size_t)dims[2] * dims[1] * (dims[0] - 1)), gN((size_t)dims[2] * (dims[1] - 1) * dims[0]),
        C((size_t)P * dims[2]), vg(nv), vL(nv), pgv(np), pL(np);
    std::vector<int32_t> vn(nv), pn(np);
    double vdd = 0;
    s = pg_netlist_to_mesh(n, p, sv.data(), m, from.data(), to.data(), kind.data(), value.data(), dims, gE.data(),
                           gN.data(), C.data(), vn.data(), vg.data(), vL.data(), pn.data(), pgv.data(), pL.data(),
                           &vdd, mp, len);
    CHECK(s == PG_OK, "to_mesh after counts: %d", s);
  }
  std::vector<int32_t> color(n), slot(n);
  int32_t nc = 0;
  int64_t ns = 0;
  s = pg_netlist_coloring(n, p, p ? sv.data() : nullptr, m, from.data(), to.data(), kind.data(), value.data(),
                          r.below(2) ? color.data() : nullptr, r.below(2) ? slot.data() : nullptr, &nc, &ns, mp, len);
  CHECK(known_status(s), "colouring status %d", s);
}

// The compact neighbour table of the graph form against the branch list: the walk a wavefront
// makes over each 64-slot slice (entry level k holds entry k of every row longer than k, in
// slot order) must give each node's neighbours with their summed values.
bool table_matches(const Netlist& nl, const std::vector<int32_t>& slot) {
  pgrid::GraphForm f;
  char msg[128];
  pg_status s = pgrid::build_graph_form(nl.n, nl.p, nl.source_v.data(), (int32_t)nl.kind.size(), nl.from.data(),
                                        nl.to.data(), nl.kind.data(), nl.value.data(), f, msg, sizeof msg);
  CHECK(s == PG_OK, "graph form of a valid random graph: %d (%s)", s, msg);
  if (s != PG_OK) return false;
  struct Val { double g = 0, il = 0, c = 0; };
  std::vector<std::vector<std::pair<int32_t, Val>>> want(f.nslots);  // by slot: (neighbour slot, values)
  {
    std::vector<std::pair<std::pair<int32_t, int32_t>, Val>> pairs;
    for (size_t e = 0; e < nl.kind.size(); ++e) {
      const int a = nl.from[e], b = nl.to[e];
      const char k = (char)nl.kind[e];
      if (k == 'I' || a < 0 || b < 0 || a >= nl.n || b >= nl.n) continue;
      Val v;
      if (k == 'R') v.g = nl.value[e];
      if (k == 'L') v.il = 1.0 / nl.value[e];
      if (k == 'C') v.c = nl.value[e];
      pairs.push_back({{std::min(a, b), std::max(a, b)}, v});
    }
    std::sort(pairs.begin(), pairs.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    for (size_t q = 0; q < pairs.size();) {
      Val sum;
      size_t t = q;
      for (; t < pairs.size() && pairs[t].first == pairs[q].first; ++t) {
        sum.g += pairs[t].second.g; sum.il += pairs[t].second.il; sum.c += pairs[t].second.c;
      }
      const int a = pairs[q].first.first, b = pairs[q].first.second;
      want[slot[a]].push_back({slot[b], sum});
      want[slot[b]].push_back({slot[a], sum});
      q = t;
    }
    for (auto& w : want) std::sort(w.begin(), w.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
  }
  const int64_t nsl = f.nslots / pgrid::kSlice;
  bool ok = (int64_t)f.soff.size() == nsl + 1 && (int64_t)f.rlen.size() == f.nslots && f.soff[0] == 0 &&
            (int64_t)f.col.size() == f.soff[nsl] && f.soff[nsl] == f.nnz;
  CHECK(ok, "graph table extents: %zu offsets, %zu lengths, %zu entries, nnz %lld", f.soff.size(), f.rlen.size(),
        f.col.size(), (long long)f.nnz);
  if (!ok) return false;
  auto close = [](double x, double y) { return std::fabs(x - y) <= 1e-12 * std::max(std::fabs(x), std::fabs(y)); };
  for (int64_t sl = 0; sl < nsl; ++sl) {
    std::vector<std::vector<int64_t>> got(pgrid::kSlice);
    int64_t P = f.soff[sl];
    for (int k = 0;; ++k) {
      int rank = 0;
      for (int j = 0; j < pgrid::kSlice; ++j)
        if (k < f.rlen[sl * pgrid::kSlice + j]) got[j].push_back(P + rank++);
      if (rank == 0) break;
      P += rank;
    }
    CHECK(P == f.soff[sl + 1], "slice %lld: the walk ends at %lld, the next slice starts at %d", (long long)sl,
          (long long)P, f.soff[sl + 1]);
    if (P != f.soff[sl + 1]) return false;
    for (int j = 0; j < pgrid::kSlice; ++j) {
      const int64_t own = sl * pgrid::kSlice + j;
      const auto& w = want[own];
      bool row_ok = got[j].size() == w.size();
      for (size_t q = 0; row_ok && q < w.size(); ++q) {
        const int64_t e = got[j][q];
        row_ok = f.col[e] == w[q].first && close(f.g[e], w[q].second.g) && close(f.inv_l[e], w[q].second.il) &&
                 close(f.cc[e], w[q].second.c);
      }
      CHECK(row_ok, "slot %lld: its table row (%zu entries) is not its %zu neighbours", (long long)own,
            got[j].size(), w.size());
      if (!row_ok) return false;
    }
  }
  return true;
}

// A random valid general netlist: a random tree of resistors over n trivial nodes, extra R, L and
// coupling-C branches between random pairs, capacitors and current sources to ground, and
// resistors to the supplies; the colouring must separate every coupled pair.
void random_graph(Rng& r) {
  Netlist nl;
  nl.n = 1 + r.below(200);
  nl.p = 1 + r.below(2);
  nl.source_v.assign(nl.p, 1.0);
  for (int i = 1; i < nl.n; ++i) nl.add(r, i, r.below(i), 'R', r.range(0.5, 2.0));
  const int extra = r.below(2 * nl.n + 1);
  for (int e = 0; e < extra; ++e) {
    const int a = r.below(nl.n), b = r.below(nl.n);
    if (a == b) continue;
    const char k = "RRLC"[r.below(4)];
    nl.add(r, a, b, k, k == 'R' ? r.range(0.5, 2.0) : (k == 'L' ? r.range(1e-12, 1e-11) : r.range(1e-13, 1e-12)));
  }
  for (int i = 0; i < nl.n; ++i) {
    if (r.below(2)) nl.add(r, i, -1, 'C', r.range(1e-13, 5e-12));
    if (r.below(3) == 0) nl.add(r, i, -1, 'I', 0.0, false);
    if (r.below(8) == 0 || i == 0) nl.add(r, i, nl.n + r.below(nl.p), 'R', r.range(5.0, 10.0));
  }
  char msg[128];
  const int32_t m = (int32_t)nl.kind.size();
  pg_status s = pg_validate_netlist(nl.n, nl.p, m, nl.from.data(), nl.to.data(), nl.kind.data(), nl.value.data(),
                                    msg, sizeof msg);
  CHECK(s == PG_OK, "a valid random graph was refused: %d (%s)", s, msg);
  if (s != PG_OK) return;
  std::vector<int32_t> color(nl.n, -1), slot(nl.n, -1);
  int32_t ncol = 0;
  int64_t nslots = 0;
  s = pg_netlist_coloring(nl.n, nl.p, nl.source_v.data(), m, nl.from.data(), nl.to.data(), nl.kind.data(),
                          nl.value.data(), color.data(), slot.data(), &ncol, &nslots, msg, sizeof msg);
  CHECK(s == PG_OK, "colouring of a valid random graph: %d (%s)", s, msg);
  if (s != PG_OK) return;
  for (int e = 0; e < m; ++e) {
    const int a = nl.from[e], b = nl.to[e];
    if (nl.kind[e] == 'I' || a < 0 || b < 0 || a >= nl.n || b >= nl.n) continue;
    CHECK(color[a] != color[b], "graph branch %d joins two nodes of colour %d", e, color[a]);
  }
  std::vector<char> seen(nslots, 0);
  for (int i = 0; i < nl.n; ++i) {
    const bool ok = slot[i] >= 0 && slot[i] < nslots && !seen[slot[i]] && color[i] >= 0 && color[i] < ncol;
    CHECK(ok, "graph node %d: slot %d colour %d", i, slot[i], color[i]);
    if (!ok) return;
    seen[slot[i]] = 1;
  }
  if (!table_matches(nl, slot)) return;
  ++graphs_ok;
}

void options(Rng& r) {
  pg_options o;
  CHECK(pg_default_options(&o) == PG_OK, "defaults");
  char msg[32];
  CHECK(pg_validate_options(&o, msg, sizeof msg) == PG_OK, "defaults invalid: %s", msg);
  for (int t = 0; t < 6; ++t) {
    pg_options b = o;
    switch (t) {
      case 0: b.h = -1.0; break;
      case 1: b.tol = NAN; break;
      case 2: b.omega = 2.0 + r.unit(); break;
      case 3: b.max_sweeps = 0; break;
      case 4: b.tile_rows = 5; break;
      case 5: b.predictor = 3; break;
    }
    const pg_status s = pg_validate_options(&b, msg, (size_t)r.below(33));
    CHECK(s == PG_ERR_INVALID_ARG, "option corruption %d gave %d", t, s);
  }
  CHECK(pg_validate_mesh(nullptr, nullptr, 0) == PG_ERR_INVALID_ARG, "null mesh");
  for (int s = 1; s >= -9; --s) CHECK(pg_status_name(s) != nullptr, "status name");
}

}  // namespace

int main(int argc, char** argv) {
  const int cases = argc > 1 ? std::atoi(argv[1]) : 300;
  Rng r{0x1409716600ull};
  options(r);
  for (int c = 0; c < cases; ++c) {
    const MeshData m = random_mesh(r);
    round_trip(r, m);
    corrupted_meshes(r, m);
    arbitrary_netlists(r);
    random_graph(r);
  }
  std::printf("host driver: %d cases, %d round trips, %d colourings, %d valid random graphs coloured, "
              "%d arbitrary lists accepted, %d failed checks\n",
              cases, round_trips, colourings, graphs_ok, accepted_arbitrary, failures);
  return failures ? 1 : 0;
}
