// Host-only argument and topology checks of the C ABI (no HIP calls, no device needed).
//
// The topological assumptions are those of Sec. III-B: supplies have grounded negative
// terminals (implied by the encoding), every trivial node reaches another non-ground node
// through a branch that is not a current source (assumption 2), and each group of trivial
// nodes connected through trivial nodes (assumption 3; Fig. 1 splits a circuit that breaks
// it into independent sub-circuits) must make the system matrix definite.  Lemma 1 gives
// weak diagonal dominance and irreducibility; definiteness additionally needs one strictly
// dominant row per sub-circuit, i.e. a capacitor, a branch to a supply or a branch to ground.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/pgrid.h"

namespace {

pg_status fail(pg_status st, char* msg, size_t len, const char* fmt, ...) {
  if (msg && len) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(msg, len, fmt, ap);
    va_end(ap);
  }
  return st;
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

struct DSU {
  std::vector<int64_t> p;
  explicit DSU(int64_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
  int64_t find(int64_t a) {
    while (p[a] != a) { p[a] = p[p[a]]; a = p[a]; }
    return a;
  }
  void unite(int64_t a, int64_t b) {
    a = find(a); b = find(b);
    if (a != b) p[a < b ? b : a] = a < b ? a : b;
  }
};

}  // namespace

extern "C" {

int32_t pg_abi_version(void) { return PG_ABI_VERSION; }

const char* pg_status_name(int32_t s) {
  switch (s) {
    case PG_OK: return "PG_OK";
    case PG_ERR_INVALID_ARG: return "PG_ERR_INVALID_ARG";
    case PG_ERR_TOPOLOGY: return "PG_ERR_TOPOLOGY";
    case PG_ERR_NOT_SPD: return "PG_ERR_NOT_SPD";
    case PG_ERR_NO_CONVERGENCE: return "PG_ERR_NO_CONVERGENCE";
    case PG_ERR_DEVICE: return "PG_ERR_DEVICE";
    case PG_ERR_OOM: return "PG_ERR_OOM";
    case PG_ERR_STATE: return "PG_ERR_STATE";
    case PG_ERR_UNSUPPORTED: return "PG_ERR_UNSUPPORTED";
    default: return "PG_ERR_UNKNOWN";
  }
}

pg_status pg_default_options(pg_options* o) {
  if (!o) return PG_ERR_INVALID_ARG;
  std::memset(o, 0, sizeof(*o));
  o->h = 10e-12;
  o->tol = 1e-6;
  o->omega = 1.0;
  o->max_sweeps = 10000;
  o->check_every = 8;
  o->precision = PG_PREC_FP64;
  o->ordering = PG_ORDER_RED_BLACK;
  o->tile_rows = 8;
  o->lookahead = 1;
  return PG_OK;
}

pg_status pg_validate_options(const pg_options* o, char* msg, size_t len) {
  if (!o) return fail(PG_ERR_INVALID_ARG, msg, len, "options pointer is NULL");
  if (!(std::isfinite(o->h) && o->h > 0)) return fail(PG_ERR_INVALID_ARG, msg, len, "h must be finite and > 0 (got %g)", o->h);
  if (!(std::isfinite(o->tol) && o->tol > 0)) return fail(PG_ERR_INVALID_ARG, msg, len, "tol must be finite and > 0 (got %g)", o->tol);
  if (!(o->omega > 0.0 && o->omega < 2.0)) return fail(PG_ERR_INVALID_ARG, msg, len, "omega must lie in (0, 2) (got %g)", o->omega);
  if (o->max_sweeps < 1) return fail(PG_ERR_INVALID_ARG, msg, len, "max_sweeps must be >= 1");
  if (o->check_every < 1) return fail(PG_ERR_INVALID_ARG, msg, len, "check_every must be >= 1");
  if (o->precision != PG_PREC_FP64 && o->precision != PG_PREC_FP32_REFINE)
    return fail(PG_ERR_INVALID_ARG, msg, len, "unknown precision %d", o->precision);
  if (o->ordering != PG_ORDER_RED_BLACK && o->ordering != PG_ORDER_JACOBI)
    return fail(PG_ERR_INVALID_ARG, msg, len, "unknown ordering %d", o->ordering);
  if (o->tile_rows != 0 && o->tile_rows != 4 && o->tile_rows != 8 && o->tile_rows != 16)
    return fail(PG_ERR_INVALID_ARG, msg, len, "tile_rows must be 0, 4, 8 or 16 (got %d)", o->tile_rows);
  if (o->lookahead < 0 || o->lookahead > 4) return fail(PG_ERR_INVALID_ARG, msg, len, "lookahead must be in 0..4");
  if (o->graphs != 0 && o->graphs != 1) return fail(PG_ERR_INVALID_ARG, msg, len, "graphs must be 0 or 1");
  if (o->scen_block < 0 || o->scen_block > 16)
    return fail(PG_ERR_INVALID_ARG, msg, len, "scen_block must be 0 (default) or 1..16");
  if (o->sweeps_per_launch < 0 || o->sweeps_per_launch > 4 || o->sweeps_per_launch == 3)
    return fail(PG_ERR_INVALID_ARG, msg, len, "sweeps_per_launch must be 0 (default), 1, 2 or 4");
  if (o->recurrence != PG_REC_TWO_LEVEL && o->recurrence != PG_REC_THREE_LEVEL)
    return fail(PG_ERR_INVALID_ARG, msg, len, "unknown recurrence %d", o->recurrence);
  if (o->recurrence == PG_REC_THREE_LEVEL && o->graphs)
    return fail(PG_ERR_UNSUPPORTED, msg, len, "the three-level recurrence runs with plain launches (graphs = 0)");
  if (o->resident != 0 && o->resident != 1)
    return fail(PG_ERR_INVALID_ARG, msg, len, "resident must be 0 or 1 (got %d)", o->resident);
  if (o->predictor < 0 || o->predictor > 2)
    return fail(PG_ERR_INVALID_ARG, msg, len, "predictor must be 0, 1 or 2 (got %d)", o->predictor);
  if (o->predictor && o->graphs)
    return fail(PG_ERR_UNSUPPORTED, msg, len, "the predictor runs with plain launches (graphs = 0)");
  return PG_OK;
}

pg_status pg_validate_mesh(const pg_mesh* m, char* msg, size_t len) {
  if (!m) return fail(PG_ERR_INVALID_ARG, msg, len, "mesh pointer is NULL");
  if (m->nx < 2 || m->ny < 2) return fail(PG_ERR_INVALID_ARG, msg, len, "nx and ny must be >= 2");
  if (m->nl < 1 || m->nl > 4) return fail(PG_ERR_UNSUPPORTED, msg, len, "nl must be in 1..4 (got %d)", m->nl);
  const int64_t P = (int64_t)m->nx * m->ny, n = P * m->nl;
  if (n > (int64_t)INT32_MAX / 2) return fail(PG_ERR_UNSUPPORTED, msg, len, "mesh too large for int32 node ids");
  if (!m->gE || !m->gN || !m->C) return fail(PG_ERR_INVALID_ARG, msg, len, "gE, gN and C must be non-NULL");
  if (!std::isfinite(m->vdd)) return fail(PG_ERR_INVALID_ARG, msg, len, "vdd must be finite");
  const int64_t nE = (int64_t)m->nl * m->ny * (m->nx - 1), nN = (int64_t)m->nl * (m->ny - 1) * m->nx;
  for (int64_t k = 0; k < nE; ++k)
    if (!finite_nonneg(m->gE[k])) return fail(PG_ERR_INVALID_ARG, msg, len, "gE[%lld] = %g is not finite and >= 0", (long long)k, m->gE[k]);
  for (int64_t k = 0; k < nN; ++k)
    if (!finite_nonneg(m->gN[k])) return fail(PG_ERR_INVALID_ARG, msg, len, "gN[%lld] = %g is not finite and >= 0", (long long)k, m->gN[k]);
  for (int64_t k = 0; k < n; ++k)
    if (!finite_nonneg(m->C[k])) return fail(PG_ERR_INVALID_ARG, msg, len, "C[%lld] = %g is not finite and >= 0", (long long)k, m->C[k]);
  if (m->n_vias < 0 || m->n_pads < 0) return fail(PG_ERR_INVALID_ARG, msg, len, "negative via or pad count");
  if (m->n_vias > 0 && (!m->via_node || !m->via_g)) return fail(PG_ERR_INVALID_ARG, msg, len, "via arrays are NULL");
  if (m->n_pads > 0 && (!m->pad_node || !m->pad_g)) return fail(PG_ERR_INVALID_ARG, msg, len, "pad arrays are NULL");
  for (int k = 0; k < m->n_vias; ++k) {
    const int64_t a = m->via_node[k];
    if (a < 0 || a >= P * (m->nl - 1)) return fail(PG_ERR_INVALID_ARG, msg, len, "via %d: lower node %lld not below the top layer", k, (long long)a);
    if (!(std::isfinite(m->via_g[k]) && m->via_g[k] > 0)) return fail(PG_ERR_INVALID_ARG, msg, len, "via %d: conductance must be finite and > 0", k);
    if (m->via_L && !finite_nonneg(m->via_L[k])) return fail(PG_ERR_INVALID_ARG, msg, len, "via %d: inductance must be finite and >= 0", k);
  }
  for (int k = 0; k < m->n_pads; ++k) {
    const int64_t a = m->pad_node[k];
    if (a < 0 || a >= n) return fail(PG_ERR_INVALID_ARG, msg, len, "pad %d: node %lld out of range", k, (long long)a);
    if (!(std::isfinite(m->pad_g[k]) && m->pad_g[k] > 0)) return fail(PG_ERR_INVALID_ARG, msg, len, "pad %d: conductance must be finite and > 0", k);
    if (m->pad_L && !finite_nonneg(m->pad_L[k])) return fail(PG_ERR_INVALID_ARG, msg, len, "pad %d: inductance must be finite and >= 0", k);
  }
  // every connected component of the conductance graph needs a pad or a capacitor
  DSU dsu(n);
  for (int l = 0; l < m->nl; ++l)
    for (int y = 0; y < m->ny; ++y)
      for (int x = 0; x < m->nx; ++x) {
        const int64_t i = (int64_t)l * P + (int64_t)y * m->nx + x;
        if (x + 1 < m->nx && m->gE[((int64_t)l * m->ny + y) * (m->nx - 1) + x] > 0) dsu.unite(i, i + 1);
        if (y + 1 < m->ny && m->gN[((int64_t)l * (m->ny - 1) + y) * m->nx + x] > 0) dsu.unite(i, i + m->nx);
      }
  for (int k = 0; k < m->n_vias; ++k) dsu.unite(m->via_node[k], m->via_node[k] + P);
  std::vector<char> anchored(n, 0);
  for (int64_t k = 0; k < n; ++k)
    if (m->C[k] > 0) anchored[dsu.find(k)] = 1;
  for (int k = 0; k < m->n_pads; ++k) anchored[dsu.find(m->pad_node[k])] = 1;
  for (int64_t k = 0; k < n; ++k)
    if (!anchored[dsu.find(k)])
      return fail(PG_ERR_NOT_SPD, msg, len,
                  "node %lld lies in a connected component with no pad and no capacitor (singular system)",
                  (long long)k);
  return PG_OK;
}

pg_status pg_validate_netlist(int32_t n, int32_t p, int32_t m, const int32_t* from, const int32_t* to,
                              const uint8_t* kind, const double* value, char* msg, size_t len) {
  if (n < 1 || p < 0 || m < 0) return fail(PG_ERR_INVALID_ARG, msg, len, "need n >= 1, p >= 0, m >= 0");
  if (m > 0 && (!from || !to || !kind || !value)) return fail(PG_ERR_INVALID_ARG, msg, len, "branch arrays are NULL");
  const int32_t top = n + p;
  std::vector<int> useful(n, 0);      // assumption 2: a non-source branch to a non-ground node
  std::vector<char> anchor(n, 0);     // a diagonal-dominance anchor: C, or R/L to a supply or ground
  DSU dsu(n);
  for (int e = 0; e < m; ++e) {
    const int32_t a = from[e], b = to[e];
    const uint8_t k = kind[e];
    if (a < -1 || a >= top || b < -1 || b >= top)
      return fail(PG_ERR_INVALID_ARG, msg, len, "branch %d: endpoint out of range", e);
    if (a == b) return fail(PG_ERR_INVALID_ARG, msg, len, "branch %d: both ends on the same node", e);
    if (k != 'R' && k != 'C' && k != 'L' && k != 'I')
      return fail(PG_ERR_INVALID_ARG, msg, len, "branch %d: unknown kind '%c'", e, (char)k);
    const double v = value[e];
    if (k != 'I' && !(std::isfinite(v) && v > 0))
      return fail(PG_ERR_INVALID_ARG, msg, len, "branch %d: value must be finite and > 0", e);
    const bool a_triv = a >= 0 && a < n, b_triv = b >= 0 && b < n;
    if (!a_triv && !b_triv && k != 'I')
      return fail(PG_ERR_TOPOLOGY, msg, len, "branch %d joins no trivial node", e);
    if (k == 'I') continue;
    if (a_triv && b != -1) useful[a] = 1;
    if (b_triv && a != -1) useful[b] = 1;
    if (a_triv && b_triv) {
      dsu.unite(a, b);
    } else {  // one end on a supply or on ground: a strictly dominant row of M
      if (a_triv) anchor[a] = 1;
      if (b_triv) anchor[b] = 1;
    }
  }
  for (int i = 0; i < n; ++i)
    if (!useful[i])
      return fail(PG_ERR_TOPOLOGY, msg, len,
                  "trivial node %d reaches no other non-ground node except through current sources", i);
  std::vector<char> comp(n, 0);
  for (int i = 0; i < n; ++i)
    if (anchor[i]) comp[dsu.find(i)] = 1;
  for (int i = 0; i < n; ++i)
    if (!comp[dsu.find(i)])
      return fail(PG_ERR_NOT_SPD, msg, len,
                  "trivial node %d belongs to a sub-circuit with no capacitor and no branch to a supply or ground", i);
  return PG_OK;
}

}  // extern "C"
