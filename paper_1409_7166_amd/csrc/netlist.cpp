// Mapping of a branch-form netlist (Sec. III, eqs. 4-6) onto the layered-mesh form the sweep
// kernels use (host code, no device needed).
//
// Trivial nodes 0 .. nx*ny*nl-1 are mesh nodes, id = (layer*ny + y)*nx + x; trivial nodes above
// that range may only be the internal node of a series R-L branch (one R and one L incident).
// Branch values: R as a conductance (S), C in F, L in H; 'I' branches only mark where current
// sources sit (their waveforms are set per scenario).

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <utility>
#include <vector>

#include "../../include/pgrid.h"
#include "graph_form.h"

namespace pgrid {
// Records a message as the context's last error (runtime.hip).
pg_status report_error(pg_ctx* c, pg_status st, const char* msg);
}  // namespace pgrid

namespace {

pg_status nfail(pg_status st, char* msg, size_t len, const char* fmt, ...) {
  if (msg && len) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(msg, len, fmt, ap);
    va_end(ap);
  }
  return st;
}

struct MeshForm {
  int nx = 0, ny = 0, nl = 0;
  std::vector<double> gE, gN, C;
  std::map<int32_t, std::pair<double, double>> via, pad;  // lower / pad node -> (g, L)
  double vdd = 0.0;
};

// Every check of pg_netlist_to_mesh; fills `out` on success.
pg_status map_netlist(int32_t n, int32_t p, const double* source_v, int32_t m, const int32_t* from,
                      const int32_t* to, const uint8_t* kind, const double* value, const int32_t* dims,
                      MeshForm& out, char* msg, size_t len) {
  pg_status st = pg_validate_netlist(n, p, m, from, to, kind, value, msg, len);
  if (st != PG_OK) return st;
  if (!dims) return nfail(PG_ERR_INVALID_ARG, msg, len, "mesh dimensions are NULL");
  const int nx = dims[0], ny = dims[1], nl = dims[2];
  if (nx < 2 || ny < 2 || nl < 1 || nl > 4)
    return nfail(PG_ERR_INVALID_ARG, msg, len, "mesh dimensions need nx, ny >= 2 and 1 <= nl <= 4");
  const int64_t plane = (int64_t)nx * ny, nmesh = plane * nl;
  if (nmesh > n) return nfail(PG_ERR_INVALID_ARG, msg, len, "the netlist has fewer trivial nodes than the mesh");
  if (p > 0 && !source_v) return nfail(PG_ERR_INVALID_ARG, msg, len, "source voltages are NULL");
  for (int j = 0; j < p; ++j) {
    if (!std::isfinite(source_v[j])) return nfail(PG_ERR_INVALID_ARG, msg, len, "source %d: voltage not finite", j);
    if (source_v[j] != source_v[0])
      return nfail(PG_ERR_UNSUPPORTED, msg, len, "the mesh form has one supply voltage; source %d differs", j);
  }
  out.nx = nx; out.ny = ny; out.nl = nl;
  out.gE.assign((size_t)nl * ny * (nx - 1), 0.0);
  out.gN.assign((size_t)nl * (ny - 1) * nx, 0.0);
  out.C.assign((size_t)nmesh, 0.0);
  out.vdd = p > 0 ? source_v[0] : 0.0;
  auto is_mesh = [&](int32_t a) { return a >= 0 && a < nmesh; };
  auto is_internal = [&](int32_t a) { return a >= nmesh && a < n; };
  auto is_source = [&](int32_t a) { return a >= n && a < n + p; };
  // incident R / L branches of every internal node
  std::vector<int> int_r(n - nmesh, -1), int_l(n - nmesh, -1), int_deg(n - nmesh, 0);
  for (int e = 0; e < m; ++e) {
    for (int32_t end : {from[e], to[e]}) {
      if (!is_internal(end)) continue;
      const int q = (int)(end - nmesh);
      ++int_deg[q];
      if (kind[e] == 'R') int_r[q] = e;
      else if (kind[e] == 'L') int_l[q] = e;
    }
  }
  for (int q = 0; q < n - nmesh; ++q)
    if (int_deg[q] != 2 || int_r[q] < 0 || int_l[q] < 0)
      return nfail(PG_ERR_UNSUPPORTED, msg, len,
                   "node %d lies outside the mesh and is not the middle of one series R-L branch", (int)(nmesh + q));
  // a branch (resistive, or series R-L with inductance L) between mesh node a and b (a mesh
  // node or a source node)
  auto place = [&](int e, int32_t a, int32_t b, double g, double L, bool series) -> pg_status {
    if (is_mesh(b) && b < a) std::swap(a, b);
    if (!is_mesh(a)) return nfail(PG_ERR_UNSUPPORTED, msg, len, "branch %d: no mesh-node end", e);
    if (is_source(b)) {
      auto it = out.pad.find(a);
      if (it == out.pad.end()) { out.pad[a] = {g, L}; return PG_OK; }
      if (series || it->second.second > 0)
        return nfail(PG_ERR_UNSUPPORTED, msg, len, "branch %d: an inductive pad in parallel with another pad", e);
      it->second.first += g;
      return PG_OK;
    }
    if (!is_mesh(b)) return nfail(PG_ERR_UNSUPPORTED, msg, len, "branch %d: a resistor to ground is not a mesh element", e);
    const int64_t la = a / plane, ya = (a % plane) / nx, xa = a % nx;
    const int64_t lb = b / plane, yb = (b % plane) / nx, xb = b % nx;
    if (lb == la + 1 && yb == ya && xb == xa) {
      auto it = out.via.find(a);
      if (it == out.via.end()) { out.via[a] = {g, L}; return PG_OK; }
      if (series || it->second.second > 0)
        return nfail(PG_ERR_UNSUPPORTED, msg, len, "branch %d: an inductive via in parallel with another via", e);
      it->second.first += g;
      return PG_OK;
    }
    if (series) return nfail(PG_ERR_UNSUPPORTED, msg, len, "branch %d: a series R-L branch inside a layer", e);
    if (lb == la && yb == ya && xb == xa + 1) {
      out.gE[(size_t)(la * ny + ya) * (nx - 1) + xa] += g;
      return PG_OK;
    }
    if (lb == la && yb == ya + 1 && xb == xa) {
      out.gN[(size_t)(la * (ny - 1) + ya) * nx + xa] += g;
      return PG_OK;
    }
    return nfail(PG_ERR_UNSUPPORTED, msg, len, "branch %d joins nodes %d and %d, which are not mesh neighbours", e,
                 (int)a, (int)b);
  };
  for (int e = 0; e < m; ++e) {
    const int32_t a = from[e], b = to[e];
    const uint8_t k = kind[e];
    if (is_internal(a) || is_internal(b)) continue;  // series R-L, placed below
    if (k == 'I' || k == 'C') {
      const int32_t node = a == -1 ? b : a, other = a == -1 ? a : b;
      if (!is_mesh(node) || other != -1)
        return nfail(PG_ERR_UNSUPPORTED, msg, len, "branch %d: a %s must join a mesh node and ground", e,
                     k == 'C' ? "capacitor" : "current source");
      if (k == 'C') out.C[node] += value[e];
      continue;
    }
    if (k == 'L')
      return nfail(PG_ERR_UNSUPPORTED, msg, len,
                   "branch %d: an inductor needs a series resistor through an internal node", e);
    pg_status s2 = place(e, a, b, value[e], 0.0, false);
    if (s2 != PG_OK) return s2;
  }
  for (int q = 0; q < n - nmesh; ++q) {
    const int er = int_r[q], el = int_l[q];
    const int32_t mid = (int32_t)(nmesh + q);
    const int32_t xr = from[er] == mid ? to[er] : from[er];
    const int32_t xl = from[el] == mid ? to[el] : from[el];
    pg_status s2 = place(er, xr, xl, value[er], value[el], true);
    if (s2 != PG_OK) return s2;
  }
  return PG_OK;
}

}  // namespace

extern "C" {

pg_status pg_netlist_mesh_counts(int32_t n, int32_t p, const double* source_v, int32_t m, const int32_t* from,
                                 const int32_t* to, const uint8_t* kind, const double* value,
                                 const int32_t* mesh_dims, int32_t* n_vias, int32_t* n_pads, char* msg,
                                 size_t msg_len) {
  MeshForm f;
  pg_status st = map_netlist(n, p, source_v, m, from, to, kind, value, mesh_dims, f, msg, msg_len);
  if (st != PG_OK) return st;
  if (n_vias) *n_vias = (int32_t)f.via.size();
  if (n_pads) *n_pads = (int32_t)f.pad.size();
  return PG_OK;
}

pg_status pg_netlist_to_mesh(int32_t n, int32_t p, const double* source_v, int32_t m, const int32_t* from,
                             const int32_t* to, const uint8_t* kind, const double* value,
                             const int32_t* mesh_dims, double* gE, double* gN, double* C, int32_t* via_node,
                             double* via_g, double* via_L, int32_t* pad_node, double* pad_g, double* pad_L,
                             double* vdd, char* msg, size_t msg_len) {
  MeshForm f;
  pg_status st = map_netlist(n, p, source_v, m, from, to, kind, value, mesh_dims, f, msg, msg_len);
  if (st != PG_OK) return st;
  if (!gE || !gN || !C || !vdd || (!f.via.empty() && (!via_node || !via_g || !via_L)) ||
      (!f.pad.empty() && (!pad_node || !pad_g || !pad_L)))
    return nfail(PG_ERR_INVALID_ARG, msg, msg_len, "output arrays are NULL");
  std::copy(f.gE.begin(), f.gE.end(), gE);
  std::copy(f.gN.begin(), f.gN.end(), gN);
  std::copy(f.C.begin(), f.C.end(), C);
  size_t k = 0;
  for (auto& kv : f.via) { via_node[k] = kv.first; via_g[k] = kv.second.first; via_L[k] = kv.second.second; ++k; }
  k = 0;
  for (auto& kv : f.pad) { pad_node[k] = kv.first; pad_g[k] = kv.second.first; pad_L[k] = kv.second.second; ++k; }
  *vdd = f.vdd;
  return PG_OK;
}

pg_status pg_upload_netlist(pg_ctx* ctx, int32_t n, int32_t p, const double* source_v, int32_t m,
                            const int32_t* from, const int32_t* to, const uint8_t* kind, const double* value,
                            const int32_t* mesh_dims, int32_t n_scen, int32_t* grid_id) {
  if (!ctx) return PG_ERR_INVALID_ARG;
  char msg[256] = {0};
  if (!mesh_dims) {  // a general netlist: colour-ordered graph form
    pgrid::GraphForm g;
    pg_status st = pgrid::build_graph_form(n, p, source_v, m, from, to, kind, value, g, msg, sizeof msg);
    if (st != PG_OK) return pgrid::report_error(ctx, st, msg);
    return pgrid::upload_graph(ctx, g, p > 0 ? source_v[0] : 0.0, n_scen, grid_id);
  }
  MeshForm f;
  pg_status st = map_netlist(n, p, source_v, m, from, to, kind, value, mesh_dims, f, msg, sizeof msg);
  if (st != PG_OK) return pgrid::report_error(ctx, st, msg);
  std::vector<int32_t> vn, pn;
  std::vector<double> vg, vl, pgv, pl;
  for (auto& kv : f.via) { vn.push_back(kv.first); vg.push_back(kv.second.first); vl.push_back(kv.second.second); }
  for (auto& kv : f.pad) { pn.push_back(kv.first); pgv.push_back(kv.second.first); pl.push_back(kv.second.second); }
  pg_mesh mesh{};
  mesh.nx = f.nx; mesh.ny = f.ny; mesh.nl = f.nl;
  mesh.gE = f.gE.data(); mesh.gN = f.gN.data(); mesh.C = f.C.data();
  mesh.n_vias = (int32_t)vn.size();
  mesh.via_node = vn.data(); mesh.via_g = vg.data(); mesh.via_L = vl.data();
  mesh.n_pads = (int32_t)pn.size();
  mesh.pad_node = pn.data(); mesh.pad_g = pgv.data(); mesh.pad_L = pl.data();
  mesh.vdd = f.vdd;
  return pg_upload_mesh(ctx, &mesh, n_scen, grid_id);
}

}  // extern "C"
