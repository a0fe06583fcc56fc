// Host runtime of the C ABI: context, coefficient layout, device memory and the
// per-step schedule of Algorithm 1 (warm start from the previous step, sweep until the
// scaled residual is below tol), with the convergence decision taken on the device.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <string>
#include <mutex>
#include <vector>

#include "../../include/pgrid.h"
#include "graph_form.h"
#include "pgrid_internal.h"

using namespace pgrid;

namespace {

constexpr int kFlagSlots = 32;  // host-visible decision flags (at most 31 decisions in flight)
static_assert((kFlagSlots & (kFlagSlots - 1)) == 0, "decision slots are selected by masking");
constexpr uint32_t kTagMask = 0x1fffffffu;  // a decision's tag: its sequence number, masked

// Device scratch of the allocation-free entry point (pg_error_bound_factor_noalloc): 32 MiB that
// every GPU the library runs on holds in its copy of this code object until the process ends.
// Host code never uses the array's name as an address: pg_create resolves each device's copy
// once, with that device current, and contexts keep the resolved pointer.
constexpr size_t kScratchDoubles = size_t(1) << 22;
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_dev;  // per device ordinal; null until resolved

// The device address of `scratch` on `device`, which must be current.
hipError_t scratch_address(int device, double** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize(device + 1, nullptr);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = (double*)p;
  }
  *out = g_scratch_dev[device];
  return hipSuccess;
}

struct Src {
  std::vector<int32_t> node, off;
  std::vector<double> t, i;
};

// Device allocation owned by a context.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct GridHost {
  int kind = 0;                                  // 0 layered mesh, 1 general graph (form below)
  int32_t nx = 0, ny = 0, nl = 0, S = 1;
  int32_t X = 0;                                 // storage row pitch (>= nx, multiple of kPitchAlign)
  int32_t item0 = 0;                             // control-block item of scenario 0
  int64_t n = 0, P = 0;                          // mesh nodes, nodes per layer
  int64_t nstore = 0;                            // storage slots per scenario, nl*ny*X
  int64_t storage(int64_t node) const {          // node id -> storage slot
    if (kind) return form.slot[node];
    const int64_t l = node / P, rem = node - l * P, y = rem / nx, x = rem - y * nx;
    return (l * ny + y) * X + x;
  }
  double vdd = 1.0;
  std::vector<double> gE, gN, C;                 // as uploaded (unpadded)
  std::vector<int32_t> via_node, pad_node;
  std::vector<double> via_g, via_L, pad_g, pad_L;
  std::vector<Src> src;                          // per scenario
  GraphForm form;                                // general graph: colouring, slots, neighbour table
  // inductive branches in via-then-pad order (mesh) or netlist order (graph); ind_branch[k] =
  // index into that order; ind_sign[k] turns the stored near -> far current into the branch's
  std::vector<int32_t> ind_a, ind_b, ind_branch;
  std::vector<double> ind_sign;
  int64_t coef_words = 0, resid_words = 0;       // coefficient words of one sweep / residual (accounting)
  uint32_t ch_layers = 0, bc_layers = 0;         // layers with non-zero C/h, constant injection
  // device buffers
  DBuf gE64, gN64, gU64, D64, ch64, bconst64, gEs, gNs, gUs, invDs;
  DBuf v0, v1, b, r, d0, d1;
  DBuf vh, vh2;                                  // v(t-h), v(t-2h) per scenario (meshes, predictor on)
  DBuf ind_a_d, ind_b_d, ind_geq_d, ind_alpha_d, ind_i_d, inc_off_d, inc_ind_d, ind_vfar_d;
  DBuf slot_d, sl_off_d, sl_len_d, sl_col_d, sl_w64_d, sl_ws_d, cap_off_d, cap_col_d, cap_val_d;
  DBuf vprev0, vprev1, g3diag_d, sl_g64_d, bres_d, bl_d;  // three-level recurrence
  DBuf gq64_d, gsup32_d, gw32_d;                          // opening probe (general graph)
  int sweep_fp32 = -1;                           // precision the sweep buffers were built for
  // Library copies of the unpadded gE, gN, C on the device (pg_update_mesh_values_dev): while
  // raw_valid they equal the grid's current values; while host_stale they, not the host
  // vectors gE, gN, C, hold them (the host vectors are refreshed before any host rebuild).
  DBuf gE_raw, gN_raw, C_raw, chk_d;
  bool raw_valid = false, host_stale = false;
  // every storage slot with a pad, and the pad term mesh_diag adds to its diagonal
  DBuf padt_slot_d, padt_val_d;
  int32_t n_padt = 0;
};

struct ProfEvent {
  hipEvent_t a, b;
  int kind;          // 0 sweep, 1 resid, 2 rhs, 3 other, -1 idle (queued after convergence)
  int chunk;         // refinement cycle of the step the launch belongs to (0: before any sweep)
  int64_t units;     // node-updates (sweep) or nodes (resid)
  double bytes;      // algorithmic bytes of the launches
  int launches;      // kernel launches between the two events
};

}  // namespace

struct pg_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  pg_options opt{};
  std::string err;
  std::vector<GridHost> grids;
  bool dirty = true;
  bool dc_mode = false;                          // coefficients of the DC matrix (C open, L shorted)
  int64_t step = 0;
  double seconds = 0.0;
  double* scratch_dev = nullptr;                 // this device's copy of the allocation-free scratch
  bool clock_on_device = false;                  // pg_step_enqueue has run: the device clock is authoritative
  // device tables
  DBuf grid_desc, tiles_all, tiles_sweep, src_grid, src_index, src_off, src_t, src_i, ind_grid, ind_local;
  // nodes: mesh nodes x scenarios of the group's grids; mesh_nodes: mesh nodes (coefficients
  // are shared by the scenarios of a grid)
  // multi: the group's tiles are scenario blocks (Tile.pad consecutive scenarios of a grid)
  struct Group { int nl, off, count; int64_t nodes, mesh_nodes; bool multi; };
  // Algorithmic bytes (see pgrid.h) for `an` active mesh nodes x scenarios whose grids hold
  // `coef` coefficient words: a cycle of nchk sweeps, charged sweep by sweep as one-sweep
  // launches move them (the first starts from d = 0 and reads no old correction; a launch that
  // fuses several sweeps is charged each of them), and one residual pass.
  double cycle_bytes(int64_t an, int64_t coef, int nchk) const {
    const double e = opt.precision == PG_PREC_FP32_REFINE ? 4.0 : 8.0;
    return e * ((2.0 + 3.0 * (nchk - 1)) * an + (double)nchk * coef);
  }
  // `coef` sweep-precision coefficient words (the probe reads those), `rcoef` FP64 words.
  double resid_bytes(int64_t an, int64_t coef, int64_t rcoef, bool has_d, int fuse = 0) const {
    const double e = opt.precision == PG_PREC_FP32_REFINE ? 4.0 : 8.0;
    if ((fuse & kFuseProbe) && (fuse & kFuseCancelled)) {
      // the cancelled-form probe: v and G0 Vdd on the layers that have it (probe_read bytes per
      // node on average), and the sweeps' coefficient words (1/M_ii included) in their precision
      return probe_read * an + e * (double)coef;
    }
    if (fuse & kFuseRhs) {
      // forms b and M_ii: v, C/h and G0 Vdd on the layers that have them (fuse_read bytes per
      // node on average), b and r unless a probe; coefficients without M_ii (one word per node)
      const double st = (fuse & kFuseProbe) ? 0.0 : 8.0 + e;
      return (fuse_read + st) * an + 8.0 * (double)std::max<int64_t>(0, rcoef - an);
    }
    return (16.0 + e + (has_d ? e + 8.0 : 0.0)) * an + 8.0 * rcoef;
  }
  std::vector<Group> tile_groups;                 // sweep/residual tiles by (layers, block): [off, off+count) of tiles_sweep
  int ntiles_all = 0;
  int tile_rows = 16;
  double fuse_read = 24.0;                       // bytes per node a right-hand-side-forming pass reads
  double probe_read = 16.0;                      // bytes per node a cancelled-form probe reads besides coefficients
  bool probe_cancelled = true;                   // every mesh grid has a non-zero supply (cancelled-form probes)
  bool tb_ok = false;                            // every mesh tile group has the four-sweep kernel
  // general-graph chunks: all slots (right-hand side, residual) and, per colour index, the
  // chunks of that colour over every graph grid ([off, off+count) of g_chunks_sweep)
  DBuf g_chunks_all, g_chunks_sweep;
  int n_gchunks_all = 0;
  std::vector<std::pair<int, int>> gcolor;
  std::vector<int> item_gchunk_off, item_gchunk_cnt;
  int n_src = 0, n_ind_total = 0;
  SourceTable src_table{};                       // device source tables (see pgrid_internal.h)
  DBuf res_src_off, res_src;                     // resident path: each item's source-table entries (CSR)
  int res_max_nodes = 0;                         // resident path: the largest grid's node count
  bool res_multi_layer = false;                  // resident path: some grid has more than one layer
  DBuf src_win_t0;
  long long step_host = 0;                       // staging for the device step counter
  DBuf c_clock;                                  // step (int64), t_now (double), window (2 x int32)
  std::vector<int> item_tile_off, item_tile_cnt; // each item's tiles in tiles_all (one scenario per tile)
  std::vector<GridDesc> desc_host;               // descriptors as uploaded (forward view)
  // recorded forward pass of the softplus-loss adjoint
  struct Adj {
    bool recorded = false;
    int grid = -1, scen = 0, item = -1, K = 0, ckpt = 1, nseg = 0;
    double margin = 0.0;
    int64_t k0 = 0;
    GridDesc view{};                             // the grid's descriptor with lambda as its state
    DBuf ckpts, vend, seg, lam0, lam1, arhs, dC, dgE, dgN, part, J, saved_vidx;
    DBuf lamp, lamq;  // the adjoint states of the last two solves (predictor on)
    // vias then pads: storage slot, index among the inductive branches (-1: resistive), g, L,
    // and the gradients with respect to g and L
    DBuf br_slot, br_ind, br_g, br_L, dbr_g, dbr_L;
    int n_pads = 0, n_vias = 0, n_ind = 0;
    // inductor currents of the item at the checkpoints, per step of a segment, at the end, and
    // the adjoint mu of the current recurrence
    DBuf ickpts, iseg, iend, mu;
    bool branch_ready = false;                   // dbr_g / dbr_L hold the last backward pass
  } adj;
  // control block
  DBuf c_norm, c_last, c_active, c_vidx, c_sweeps, c_failed, c_any, c_stats64, c_stats32, c_statsd, c_nodes, c_item_grid;
  Ctl ctl{};
  int32_t* host_flags = nullptr;                 // pinned, written by the decision kernel
  uint64_t flag_seq_host = 0;                    // decisions queued so far (mirrors the device counter)
  hipStream_t cap_stream = nullptr;              // private stream for graph capture
  hipGraphExec_t g_prologue = nullptr, g_sweeps = nullptr, g_check = nullptr, g_epilogue = nullptr;
  bool graphs_ready = false;
  int64_t all_nodes = 0;                         // mesh nodes x scenarios over all grids
  int64_t all_coef = 0, all_rcoef = 0;           // coefficient words over all grids (sweep, residual)
  int64_t graph_nodes = 0, graph_coef = 0, graph_rcoef = 0, graph_entries = 0;  // the general graphs' share
  int64_t begin_nodes = 0, begin_coef = 0, begin_rcoef = 0;  // work of the step's first residual (items begun)
  long long* host_acct = nullptr;                // pinned [slots][3]: active work after each decision
  long long* dev_acct = nullptr;
  int32_t* dev_flags = nullptr;                  // device address of host_flags
  // profiling
  int profile_every = 0;
  int64_t prof_count[4] = {0, 0, 0, 0};          // intervals seen per kind (sampling)
  int cur_chunk = 0;                             // refinement cycle being queued
  int pred_chunks = 1;                           // cycles the previous step needed
  bool opening_queued = false;                   // the next step's opening is already queued
  int opening_tag = 0;                           // ... and the tag of its first decision
  bool maybe_stalled = false;                    // a speculative close may have stalled the device
  bool begun_next = false;                       // the last close also began the next step
  bool prev_valid = false;                       // v(t-h) is kept: graph grids' vprev (three-level)
  int pred_hist = 0;                             // earlier states the predictor holds (meshes' vh, vh2)
  int fuse_next = 0;                             // kFuse* mode of the next residual pass (mesh RHS)
  bool gprobe_next = false;                      // the next residual pass probes the general graphs
  bool gstore_next = false;                      // the next residual pass forms and stores their b, r
  bool opening_probe = false;                    // the last queued opening only took the norm
  bool opening_gprobe = false;                   // ... on the general graphs
  bool opening_closes = false;                   // ... and its decision carries the step's close
  bool capturing = false;                        // launches are being captured into a graph
  std::vector<double> win_t0_host;               // bucket starts of the windowed sources (host copy)
  std::vector<ProfEvent> prof_live;
  std::vector<hipEvent_t> prof_pool;
  pg_kernel_times prof_acc{};
};

namespace {

void drop_graphs(pg_ctx* c);

pg_status set_err(pg_ctx* c, pg_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

}  // namespace

namespace pgrid {
// Records a message as the context's last error (used by the host-side netlist mapping).
__attribute__((visibility("hidden"))) pg_status report_error(pg_ctx* c, pg_status st, const char* msg) {
  return set_err(c, st, "%s", msg);
}
}  // namespace pgrid

namespace {

#define HIP_TRY(ctx, expr)                                                                \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return set_err((ctx), e_ == hipErrorOutOfMemory ? PG_ERR_OOM : PG_ERR_DEVICE,       \
                     "%s failed: %s", #expr, hipGetErrorString(e_));                      \
  } while (0)

#define PG_TRY(expr)                        \
  do {                                      \
    pg_status s_ = (expr);                  \
    if (s_ != PG_OK) return s_;             \
  } while (0)

pg_status dalloc(pg_ctx* c, DBuf& b, size_t bytes) {
  if (b.p && b.bytes == bytes) return PG_OK;
  if (b.p) { (void)hipFree(b.p); b.p = nullptr; b.bytes = 0; }
  if (bytes == 0) return PG_OK;
  HIP_TRY(c, hipMalloc(&b.p, bytes));
  b.bytes = bytes;
  return PG_OK;
}

void dfree(DBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

// Set-up copies are synchronous: the host vectors are temporaries.
template <typename T>
pg_status upload(pg_ctx* c, DBuf& b, const std::vector<T>& h) {
  PG_TRY(dalloc(c, b, h.size() * sizeof(T)));
  if (!h.empty()) {
    HIP_TRY(c, hipMemcpyAsync(b.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return PG_OK;
}

bool fp32_mode(const pg_ctx* c) { return c->opt.precision == PG_PREC_FP32_REFINE; }

// ---- profiling helpers ---------------------------------------------------------------
hipEvent_t prof_get(pg_ctx* c) {
  if (!c->prof_pool.empty()) {
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

struct ProfScope {
  pg_ctx* c;
  ProfEvent ev{};
  bool on = false;
  ProfScope(pg_ctx* ctx, int kind, int64_t units, double bytes = 0.0, int launches = 1) : c(ctx) {
    if (c->profile_every <= 0) return;
    if ((c->prof_count[kind]++ % c->profile_every) != 0) return;  // every k-th interval of each kind
    on = true;
    ev.a = prof_get(c);
    ev.b = prof_get(c);
    ev.kind = kind;
    ev.chunk = c->cur_chunk;
    ev.units = units;
    ev.bytes = bytes;
    ev.launches = launches;
    (void)hipEventRecord(ev.a, c->stream);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(ev.b, c->stream);
    c->prof_live.push_back(ev);
  }
};

void prof_drain(pg_ctx* c) {
  if (c->prof_live.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& e : c->prof_live) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e.a, e.b);
    auto& A = c->prof_acc;
    switch (e.kind) {
      case -1: break;
      case 0: A.sweep_launches += e.launches; A.sweep_ms += ms; A.sweep_node_updates += e.units; A.sweep_bytes += e.bytes; break;
      case 1: A.resid_launches += e.launches; A.resid_ms += ms; A.resid_nodes += e.units; A.resid_bytes += e.bytes; break;
      case 2: A.rhs_launches++; A.rhs_ms += ms; break;
      default: A.other_launches++; A.other_ms += ms; break;
    }
    c->prof_pool.push_back(e.a);
    c->prof_pool.push_back(e.b);
  }
  c->prof_live.clear();
}

int n_items(const pg_ctx* c) {
  int I = 0;
  for (auto& H : c->grids) I += H.S;
  return I;
}

// ---- coefficient layout ------------------------------------------------------------
// Builds the padded FP64 coefficient arrays and the companion model of every inductive
// branch for step h (series R-L: g_eq = h/(L + hR), alpha = L/(L + hR); eq. 10 with the
// inductor current kept as state), then the sweep-precision copies.
// Bring the host vectors gE, gN, C of a mesh up to the values a device update left in the
// library's device copies.
pg_status ensure_host_values(pg_ctx* c, GridHost& G) {
  if (!G.host_stale) return PG_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(G.gE.data(), G.gE_raw.p, G.gE.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(G.gN.data(), G.gN_raw.p, G.gN.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(G.C.data(), G.C_raw.p, G.C.size() * sizeof(double), hipMemcpyDeviceToHost));
  G.host_stale = false;
  return PG_OK;
}

// Residual and correction buffers in the sweep precision (zero, so padding slots read as zero).
pg_status alloc_sweep_bufs(pg_ctx* c, GridHost& G, bool f32) {
  const size_t es = f32 ? sizeof(float) : sizeof(double);
  const size_t nss = (size_t)G.nstore * G.S;
  if (G.sweep_fp32 != (int)f32) {
    PG_TRY(dalloc(c, G.r, nss * es)); PG_TRY(dalloc(c, G.d0, nss * es)); PG_TRY(dalloc(c, G.d1, nss * es));
    HIP_TRY(c, hipMemsetAsync(G.r.p, 0, nss * es, c->stream));
    HIP_TRY(c, hipMemsetAsync(G.d0.p, 0, nss * es, c->stream));
    HIP_TRY(c, hipMemsetAsync(G.d1.p, 0, nss * es, c->stream));
    G.sweep_fp32 = (int)f32;
  }
  return PG_OK;
}

// Inductive branches (G.ind_a / ind_b filled): companion values, per-branch far voltages
// (vfar, or null for the grid's vdd), the branch currents (kept when the branch set is
// unchanged) and the slot -> branch incidence in CSR form.
pg_status upload_inductors(pg_ctx* c, GridHost& G, const std::vector<double>& geq,
                           const std::vector<double>& alpha, const std::vector<double>* vfar) {
  const int64_t ns = G.nstore;
  const int ni = (int)G.ind_a.size();
  PG_TRY(upload(c, G.ind_a_d, G.ind_a)); PG_TRY(upload(c, G.ind_b_d, G.ind_b));
  PG_TRY(upload(c, G.ind_geq_d, geq)); PG_TRY(upload(c, G.ind_alpha_d, alpha));
  if (vfar) PG_TRY(upload(c, G.ind_vfar_d, *vfar)); else dfree(G.ind_vfar_d);
  if (G.ind_i_d.bytes != (size_t)ni * G.S * sizeof(double)) {
    PG_TRY(dalloc(c, G.ind_i_d, (size_t)ni * G.S * sizeof(double)));
    if (ni) HIP_TRY(c, hipMemsetAsync(G.ind_i_d.p, 0, (size_t)ni * G.S * sizeof(double), c->stream));
  }
  if (ni) {
    std::vector<int32_t> cnt(ns + 1, 0);
    for (int k = 0; k < ni; ++k) { cnt[G.ind_a[k] + 1]++; if (G.ind_b[k] >= 0) cnt[G.ind_b[k] + 1]++; }
    for (int64_t i = 0; i < ns; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> inc(cnt[ns]), fillp(cnt.begin(), cnt.end() - 1);
    for (int k = 0; k < ni; ++k) {
      inc[fillp[G.ind_a[k]]++] = k + 1;
      if (G.ind_b[k] >= 0) inc[fillp[G.ind_b[k]]++] = -(k + 1);
    }
    PG_TRY(upload(c, G.inc_off_d, cnt)); PG_TRY(upload(c, G.inc_ind_d, inc));
  } else {
    dfree(G.inc_off_d); dfree(G.inc_ind_d);
  }
  return PG_OK;
}

pg_status build_mesh_grid(pg_ctx* c, int gi) {
  GridHost& G = c->grids[gi];
  PG_TRY(ensure_host_values(c, G));
  const double h = c->opt.h;
  // DC matrix (the limit h -> infinity): no C/h, and a series R-L branch is its resistor
  // (g_eq -> 1/R, alpha -> 0), so the branch update gives the DC current g (v_a - v_b)
  const bool dc = c->dc_mode;
  const int nx = G.nx, ny = G.ny, nl = G.nl, X = G.X;
  const int64_t ns = G.nstore, PS = (int64_t)X * ny;  // storage slots, storage layer stride
  auto sidx = [&](int64_t node) { return G.storage(node); };
  std::vector<double> gE(ns, 0.0), gN(ns, 0.0), gU(ns, 0.0), D(ns, 0.0), ch(ns, 0.0), bc(ns, 0.0);
  for (int l = 0; l < nl; ++l)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int64_t i = (int64_t)l * PS + (int64_t)y * X + x;
        if (x + 1 < nx) gE[i] = G.gE[((int64_t)l * ny + y) * (nx - 1) + x];
        if (y + 1 < ny) gN[i] = G.gN[((int64_t)l * (ny - 1) + y) * nx + x];
        ch[i] = dc ? 0.0 : G.C[((int64_t)l * ny + y) * nx + x] / h;
      }
  G.ind_a.clear(); G.ind_b.clear(); G.ind_branch.clear();
  std::vector<double> geq, alpha;
  const int nv = (int)G.via_node.size(), np = (int)G.pad_node.size();
  for (int k = 0; k < nv; ++k) {
    const int64_t a = sidx(G.via_node[k]);
    const double L = G.via_L.empty() ? 0.0 : G.via_L[k];
    if (L > 0) {
      const double R = 1.0 / G.via_g[k];
      const double g = dc ? G.via_g[k] : h / (L + h * R);
      gU[a] += g;
      G.ind_a.push_back((int32_t)a); G.ind_b.push_back((int32_t)(a + PS)); G.ind_branch.push_back(k);
      geq.push_back(g); alpha.push_back(dc ? 0.0 : L / (L + h * R));
    } else {
      gU[a] += G.via_g[k];
    }
  }
  for (int k = 0; k < np; ++k) {
    const int64_t a = sidx(G.pad_node[k]);
    const double L = G.pad_L.empty() ? 0.0 : G.pad_L[k];
    double g = G.pad_g[k];
    if (L > 0) {
      const double R = 1.0 / G.pad_g[k];
      if (!dc) g = h / (L + h * R);
      G.ind_a.push_back((int32_t)a); G.ind_b.push_back(-1); G.ind_branch.push_back(nv + k);
      geq.push_back(g); alpha.push_back(dc ? 0.0 : L / (L + h * R));
    }
    D[a] += g;
    bc[a] += g * G.vdd;
  }
  // diagonal of M and its inverse; padding slots keep D = 0 and invD = 0.  With a non-zero
  // supply voltage the pad conductance enters as (G0 Vdd) (1/Vdd), the form the first residual
  // pass of a step recovers it in (mesh_diag); D already holds the pads otherwise.
  std::vector<double> inv(ns, 0.0);
  const double inv_vdd = G.vdd != 0.0 ? 1.0 / G.vdd : 0.0;
  std::vector<int32_t> padt_slot;  // slots with a pad term, for a device rebuild of D
  std::vector<double> padt_val;
  for (int l = 0; l < nl; ++l)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int64_t i = (int64_t)l * PS + (int64_t)y * X + x;
        const double w = x > 0 ? gE[i - 1] : 0.0, s = y > 0 ? gN[i - X] : 0.0, d = l > 0 ? gU[i - PS] : 0.0;
        const double pad = G.vdd != 0.0 ? bc[i] * inv_vdd : D[i];
        if (pad != 0.0) { padt_slot.push_back((int32_t)i); padt_val.push_back(pad); }
        D[i] = mesh_diag(ch[i], gE[i], w, gN[i], s, gU[i], d, pad);
        inv[i] = 1.0 / D[i];
      }
  PG_TRY(upload(c, G.padt_slot_d, padt_slot)); PG_TRY(upload(c, G.padt_val_d, padt_val));
  G.n_padt = (int32_t)padt_slot.size();
  G.ch_layers = G.bc_layers = 0;
  for (int l = 0; l < nl; ++l)
    for (int64_t i = (int64_t)l * PS; i < (int64_t)(l + 1) * PS; ++i) {
      if (ch[i] != 0.0) G.ch_layers |= 1u << l;
      if (bc[i] != 0.0) G.bc_layers |= 1u << l;
    }
  PG_TRY(upload(c, G.gE64, gE)); PG_TRY(upload(c, G.gN64, gN)); PG_TRY(upload(c, G.gU64, gU));
  PG_TRY(upload(c, G.D64, D)); PG_TRY(upload(c, G.ch64, ch)); PG_TRY(upload(c, G.bconst64, bc));
  const bool f32 = fp32_mode(c);
  if (f32) {
    std::vector<float> a(ns), b(ns), u(ns), q(ns);
    for (int64_t i = 0; i < ns; ++i) {
      a[i] = (float)gE[i]; b[i] = (float)gN[i]; u[i] = (float)gU[i]; q[i] = (float)inv[i];
    }
    PG_TRY(upload(c, G.gEs, a)); PG_TRY(upload(c, G.gNs, b)); PG_TRY(upload(c, G.gUs, u));
    PG_TRY(upload(c, G.invDs, q));
  } else {
    dfree(G.gEs); dfree(G.gNs); dfree(G.gUs);
    PG_TRY(upload(c, G.invDs, inv));
  }
  PG_TRY(alloc_sweep_bufs(c, G, f32));
  G.ind_sign.assign(G.ind_a.size(), 1.0);
  PG_TRY(upload_inductors(c, G, geq, alpha, nullptr));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PG_OK;
}

// General graph: the same quantities from the graph form.  Diagonal D_i = C_i/h + the
// conductances at i + h/L of every inductor at i; off-diagonal w_ij = g_ij + h/L_ij + C_ij/h
// (eq. 11, M = C/h + G + hL, with the inductor current kept as state: alpha = 1, g_eq = h/L).
pg_status build_graph_grid(pg_ctx* c, int gi) {
  GridHost& G = c->grids[gi];
  const GraphForm& F = G.form;
  const double h = c->opt.h;
  const bool dc = c->dc_mode;
  if (dc && !F.ind_near.empty())
    return set_err(c, PG_ERR_UNSUPPORTED,
                   "grid %d: an inductor is a short circuit at DC; the DC point of a general netlist with "
                   "inductors is not built", gi);
  const int64_t ns = G.nstore;
  std::vector<double> D(ns, 0.0), ch(ns, 0.0), bc(ns, 0.0), inv(ns, 0.0);
  for (int32_t i = 0; i < F.n; ++i) {
    const int32_t s = F.slot[i];
    ch[s] = dc ? 0.0 : F.c_diag[i] / h;
    D[s] = ch[s] + F.g_diag[i];
    bc[s] = F.b_res[i];
  }
  G.ind_a.clear(); G.ind_b.clear(); G.ind_branch.clear(); G.ind_sign.clear();
  std::vector<double> geq, alpha, vfar;
  for (size_t k = 0; k < F.ind_near.size(); ++k) {
    const double g = h * F.ind_inv_l[k];
    const int32_t a = F.slot[F.ind_near[k]];
    D[a] += g;
    if (F.ind_far[k] >= 0) D[F.slot[F.ind_far[k]]] += g;
    else bc[a] += g * F.ind_far_v[k];
    G.ind_a.push_back(a);
    G.ind_b.push_back(F.ind_far[k] >= 0 ? F.slot[F.ind_far[k]] : -1);
    G.ind_branch.push_back((int32_t)k);
    G.ind_sign.push_back((double)F.ind_sign[k]);
    geq.push_back(g); alpha.push_back(1.0); vfar.push_back(F.ind_far_v[k]);
  }
  for (int64_t s = 0; s < ns; ++s) inv[s] = D[s] > 0.0 ? 1.0 / D[s] : 0.0;
  const size_t ne = F.col.size();
  std::vector<double> w(ne), cap;
  for (size_t e = 0; e < ne; ++e) w[e] = F.g[e] + h * F.inv_l[e] + (dc ? 0.0 : F.cc[e] / h);
  // the opening probe's quantities: with e = v - vref, at v' = v and zero sources the residual is
  // q_i - history_i - gsup_i e_i + sum_j wG_ij (e_j - e_i), wG = the conductance part of w,
  // gsup_i = D_i - C_i/h - sum_j wG_ij (the conductance to supplies and ground), and
  // q_i = (G0 v_s + (h/L) v_s)_i - gsup_i vref
  {
    std::vector<double> gsum(ns, 0.0);
    std::vector<float> wg32(ne);
    for_each_entry(F, [&](int64_t e, int64_t s) {
      const double wg = F.g[e] + h * F.inv_l[e];
      gsum[s] += wg;
      wg32[e] = (float)wg;
    });
    std::vector<double> q(ns, 0.0);
    std::vector<float> gsup(ns, 0.0f);
    for (int64_t s = 0; s < ns; ++s) {
      const double gs = (D[s] - ch[s]) - gsum[s];
      gsup[s] = (float)gs;
      q[s] = bc[s] - gs * G.vdd;
    }
    PG_TRY(upload(c, G.gq64_d, q)); PG_TRY(upload(c, G.gsup32_d, gsup)); PG_TRY(upload(c, G.gw32_d, wg32));
  }
  if (F.has_coupling) {  // same size at DC (zeros: capacitors open), so the buffer stays put
    cap.assign(F.cval.size(), 0.0);
    if (!dc)
      for (size_t e = 0; e < cap.size(); ++e) cap[e] = F.cval[e] / h;
  }
  PG_TRY(upload(c, G.D64, D)); PG_TRY(upload(c, G.ch64, ch)); PG_TRY(upload(c, G.bconst64, bc));
  PG_TRY(upload(c, G.sl_off_d, F.soff)); PG_TRY(upload(c, G.sl_col_d, F.col)); PG_TRY(upload(c, G.sl_w64_d, w));
  PG_TRY(upload(c, G.sl_len_d, F.rlen));
  PG_TRY(upload(c, G.slot_d, F.slot));
  if (!F.has_coupling) {
    dfree(G.cap_off_d); dfree(G.cap_col_d); dfree(G.cap_val_d);
  } else {
    PG_TRY(upload(c, G.cap_off_d, F.csoff)); PG_TRY(upload(c, G.cap_col_d, F.ccol)); PG_TRY(upload(c, G.cap_val_d, cap));
  }
  const bool f32 = fp32_mode(c);
  if (f32) {
    std::vector<float> wf(ne), qf(ns);
    for (size_t e = 0; e < ne; ++e) wf[e] = (float)w[e];
    for (int64_t i = 0; i < ns; ++i) qf[i] = (float)inv[i];
    PG_TRY(upload(c, G.sl_ws_d, wf)); PG_TRY(upload(c, G.invDs, qf));
  } else {
    dfree(G.sl_ws_d);
    PG_TRY(upload(c, G.invDs, inv));
  }
  PG_TRY(alloc_sweep_bufs(c, G, f32));
  PG_TRY(upload_inductors(c, G, geq, alpha, &vfar));
  if (c->opt.recurrence == PG_REC_THREE_LEVEL) {
    // the conductance part of M and the two constant injections, for the three-level recurrence
    std::vector<double> gd(ns, 0.0), br(ns, 0.0), bl(ns, 0.0);
    for (int32_t i = 0; i < F.n; ++i) { gd[F.slot[i]] = F.g_diag[i]; br[F.slot[i]] = F.b_res[i]; }
    for (size_t k = 0; k < F.ind_near.size(); ++k)
      if (F.ind_far[k] < 0) bl[F.slot[F.ind_near[k]]] += h * F.ind_inv_l[k] * F.ind_far_v[k];
    PG_TRY(upload(c, G.g3diag_d, gd)); PG_TRY(upload(c, G.bres_d, br)); PG_TRY(upload(c, G.bl_d, bl));
    PG_TRY(upload(c, G.sl_g64_d, F.g));
    PG_TRY(dalloc(c, G.vprev0, (size_t)ns * G.S * sizeof(double)));
    PG_TRY(dalloc(c, G.vprev1, (size_t)ns * G.S * sizeof(double)));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PG_OK;
}

pg_status sync_desc(pg_ctx* c, int gi);

pg_status build_grid(pg_ctx* c, int gi) {
  PG_TRY(c->grids[gi].kind ? build_graph_grid(c, gi) : build_mesh_grid(c, gi));
  GridHost& H = c->grids[gi];
  // the predictor's history, filled by the openings that follow (pred_hist is 0 then)
  if (!H.kind && c->opt.predictor) {
    if (!H.vh.p) PG_TRY(dalloc(c, H.vh, (size_t)H.nstore * H.S * sizeof(double)));
  } else {
    dfree(H.vh);
  }
  if (!H.kind && c->opt.predictor == 2) {
    if (!H.vh2.p) PG_TRY(dalloc(c, H.vh2, (size_t)H.nstore * H.S * sizeof(double)));
  } else {
    dfree(H.vh2);
  }
  return sync_desc(c, gi);
}

// The device descriptor of a grid (pointers to its current buffers).
GridDesc make_desc(pg_ctx* c, GridHost& H) {
  GridDesc D;
  std::memset(&D, 0, sizeof D);
  D.kind = H.kind;
  D.nx = H.nx; D.ny = H.ny; D.nl = H.nl; D.S = H.S; D.X = H.X; D.item0 = H.item0; D.nstore = H.nstore;
  D.gE64 = (const double*)H.gE64.p; D.gN64 = (const double*)H.gN64.p; D.gU64 = (const double*)H.gU64.p;
  D.D64 = (const double*)H.D64.p; D.ch64 = (const double*)H.ch64.p; D.bconst64 = (const double*)H.bconst64.p;
  if (fp32_mode(c)) { D.gEs = H.gEs.p; D.gNs = H.gNs.p; D.gUs = H.gUs.p; }
  else { D.gEs = H.gE64.p; D.gNs = H.gN64.p; D.gUs = H.gU64.p; }
  D.invDs = H.invDs.p;
  D.v[0] = (double*)H.v0.p; D.v[1] = (double*)H.v1.p; D.b = (double*)H.b.p;
  D.vhist = (double*)H.vh.p;
  D.vhist2 = (double*)H.vh2.p;
  D.r = H.r.p; D.d[0] = H.d0.p; D.d[1] = H.d1.p;
  D.n_ind = (int32_t)H.ind_a.size();
  D.ind_a = (const int32_t*)H.ind_a_d.p; D.ind_b = (const int32_t*)H.ind_b_d.p;
  D.ind_geq = (const double*)H.ind_geq_d.p; D.ind_alpha = (const double*)H.ind_alpha_d.p;
  D.ind_i = (double*)H.ind_i_d.p;
  D.inc_off = (const int32_t*)H.inc_off_d.p; D.inc_ind = (const int32_t*)H.inc_ind_d.p;
  D.ind_vfar = (const double*)H.ind_vfar_d.p;
  D.vdd = H.vdd;
  if (H.kind) {
    D.sl_off = (const int32_t*)H.sl_off_d.p; D.sl_len = (const uint16_t*)H.sl_len_d.p;
    D.sl_col = (const int32_t*)H.sl_col_d.p;
    D.sl_w64 = (const double*)H.sl_w64_d.p;
    D.sl_ws = fp32_mode(c) ? H.sl_ws_d.p : H.sl_w64_d.p;
    D.cap_off = (const int32_t*)H.cap_off_d.p; D.cap_col = (const int32_t*)H.cap_col_d.p;
    D.cap_val = (const double*)H.cap_val_d.p;
    D.vprev[0] = (double*)H.vprev0.p; D.vprev[1] = (double*)H.vprev1.p;
    D.g3diag = (const double*)H.g3diag_d.p; D.sl_g64 = (const double*)H.sl_g64_d.p;
    D.bres64 = (const double*)H.bres_d.p; D.bl64 = (const double*)H.bl_d.p;
    D.gq64 = (const double*)H.gq64_d.p; D.gsup32 = (const float*)H.gsup32_d.p; D.gw32 = (const float*)H.gw32_d.p;
    // sweep: 1/M_ii and w in the sweep precision, a 2-byte row length per slot and a 4-byte
    // column index per table entry; residual: M_ii and w in FP64, the row length (a quarter of
    // an FP64 word) and the column index (half a word); nstore is a multiple of 64
    H.coef_words = fp32_mode(c) ? H.nstore + H.nstore / 2 + 2 * H.form.nnz
                                : H.nstore + H.nstore / 4 + (3 * H.form.nnz) / 2;
    H.resid_words = H.nstore + H.nstore / 4 + (3 * H.form.nnz) / 2;
  } else {
    H.coef_words = 3 * H.n + (int64_t)H.nx * H.ny * (H.nl - 1);
    H.resid_words = H.coef_words;
  }
  D.coef_words = H.coef_words;
  D.resid_words = H.resid_words;
  D.ch_layers = H.ch_layers;
  D.bc_layers = H.bc_layers;
  return D;
}

// After a rebuild outside prepare (the DC matrix and back), re-upload the grid's descriptor
// if any of its buffers moved, so no launch reads through a stale pointer.
pg_status sync_desc(pg_ctx* c, int gi) {
  if (c->dirty || gi >= (int)c->desc_host.size() || !c->grid_desc.p) return PG_OK;
  const GridDesc D = make_desc(c, c->grids[gi]);
  if (std::memcmp(&D, &c->desc_host[gi], sizeof D) == 0) return PG_OK;
  c->desc_host[gi] = D;
  HIP_TRY(c, hipMemcpyAsync((GridDesc*)c->grid_desc.p + gi, &c->desc_host[gi], sizeof D, hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PG_OK;
}

pg_status prepare(pg_ctx* c) {
  if (c->grids.empty()) return set_err(c, PG_ERR_STATE, "no grid uploaded");
  for (int g = 0; g < (int)c->grids.size(); ++g) {
    if (c->grids[g].kind && c->opt.ordering != PG_ORDER_RED_BLACK)
      return set_err(c, PG_ERR_UNSUPPORTED, "grid %d: general netlists are swept in colour order; the Jacobi "
                     "ordering is built for meshes only", g);
    if (!c->grids[g].kind && c->opt.recurrence == PG_REC_THREE_LEVEL)
      return set_err(c, PG_ERR_UNSUPPORTED, "grid %d: the three-level recurrence is built for general netlists", g);
  }
  if (!c->dirty) return PG_OK;
  c->prev_valid = false;
  c->pred_hist = 0;
  drop_graphs(c);
  const int G = (int)c->grids.size();
  c->tile_rows = c->opt.tile_rows ? c->opt.tile_rows : 8;
  for (int g = 0; g < G; ++g) PG_TRY(build_grid(c, g));
  // grid descriptors
  std::vector<GridDesc> desc(G);
  std::vector<long long> nodes;
  for (int g = 0; g < G; ++g) {
    GridHost& H = c->grids[g];
    desc[g] = make_desc(c, H);
    for (int sc = 0; sc < H.S; ++sc) nodes.push_back((long long)H.n);
  }
  PG_TRY(upload(c, c->grid_desc, desc));
  c->desc_host = desc;
  c->adj.recorded = false;
  PG_TRY(upload(c, c->c_nodes, nodes));
  c->ctl.nodes = (const long long*)c->c_nodes.p;
  std::vector<int32_t> item_grid;
  for (int g = 0; g < G; ++g)
    for (int sc = 0; sc < c->grids[g].S; ++sc) item_grid.push_back(g);
  PG_TRY(upload(c, c->c_item_grid, item_grid));
  c->ctl.item_grid = (const int32_t*)c->c_item_grid.p;
  // tiles_all: one tile per (scenario, tile) grouped by layer count, for the right-hand side,
  // the state copies and the loss kernels.  tiles_sweep: the sweep and residual tiles; a grid
  // with several scenarios is covered by scenario blocks of up to scen_block scenarios, whose
  // workgroups load the shared coefficients once per block.
  const int TY = c->tile_rows;
  const int SB = c->opt.scen_block ? c->opt.scen_block : kScenBlock;
  std::vector<Tile> tiles, sweep;
  c->tile_groups.clear();
  c->item_tile_off.assign(n_items(c), 0);
  c->item_tile_cnt.assign(n_items(c), 0);
  for (int nl = 1; nl <= 4; ++nl) {
    for (int g = 0; g < G; ++g) {
      const GridHost& H = c->grids[g];
      if (H.nl != nl || H.kind) continue;
      for (int sc = 0; sc < H.S; ++sc) {
        c->item_tile_off[H.item0 + sc] = (int)tiles.size();
        for (int y0 = 0; y0 < H.ny; y0 += TY)
          for (int x0 = 0; x0 < H.nx; x0 += kTileX) tiles.push_back(Tile{g, H.item0 + sc, sc, x0, y0, 1});
        c->item_tile_cnt[H.item0 + sc] = (int)tiles.size() - c->item_tile_off[H.item0 + sc];
      }
    }
    for (int multi = 0; multi <= 1; ++multi) {
      const int start = (int)sweep.size();
      int64_t nodes_g = 0, mesh_g = 0;
      for (int g = 0; g < G; ++g) {
        const GridHost& H = c->grids[g];
        if (H.nl != nl || H.kind || (H.S > 1) != (multi == 1)) continue;
        nodes_g += H.n * H.S;
        mesh_g += H.n;
        for (int s0 = 0; s0 < H.S; s0 += SB) {
          const int nb = std::min(SB, H.S - s0);
          for (int y0 = 0; y0 < H.ny; y0 += TY)
            for (int x0 = 0; x0 < H.nx; x0 += kTileX) sweep.push_back(Tile{g, H.item0 + s0, s0, x0, y0, nb});
        }
      }
      if ((int)sweep.size() > start)
        c->tile_groups.push_back({nl, start, (int)sweep.size() - start, nodes_g, mesh_g, multi == 1});
    }
  }
  c->ntiles_all = (int)tiles.size();
  c->tb_ok = true;
  for (auto& grp : c->tile_groups)
    c->tb_ok = c->tb_ok && sweep_tb_supported(fp32_mode(c), grp.multi, c->opt.ordering, grp.nl, TY, kTbSweeps);
  c->all_nodes = 0;
  c->all_coef = c->all_rcoef = 0;
  c->graph_nodes = c->graph_coef = c->graph_rcoef = c->graph_entries = 0;
  for (auto& grp : c->tile_groups) c->all_nodes += grp.nodes;
  double fr = 0.0, fp = 0.0, fn = 0.0;
  c->probe_cancelled = true;
  for (auto& H : c->grids) {
    c->all_coef += H.coef_words;
    c->all_rcoef += H.resid_words;
    if (H.kind) {
      c->all_nodes += H.n * H.S;
      c->graph_nodes += H.n * H.S;
      c->graph_coef += H.coef_words;
      c->graph_rcoef += H.resid_words;
      c->graph_entries += H.form.nnz * H.S;  // table entries (the table stores no padding)
    } else {
      const double w = (double)H.n * H.S;
      fr += w * (8.0 + 8.0 * (__builtin_popcount(H.ch_layers) + __builtin_popcount(H.bc_layers)) / H.nl);
      fp += w * (8.0 + 8.0 * __builtin_popcount(H.bc_layers) / H.nl);
      fn += w;
      if (H.vdd == 0.0) c->probe_cancelled = false;
    }
  }
  c->fuse_read = fn > 0 ? fr / fn : 24.0;
  c->probe_read = fn > 0 ? fp / fn : 16.0;
  // general-graph chunks: every slot of every scenario (right-hand side, residual), and the
  // sweep chunks colour by colour.  In the first list each scenario's chunks interleave the
  // colours by position inside their colour: a node's neighbours lie at about the same relative
  // position of the other colours, so the run of chunks one XCD takes (xcd_tile) finds most of
  // its neighbour values in chunks of its own, in its own L2.
  std::vector<GraphChunk> gall, gsweep;
  c->gcolor.clear();
  c->item_gchunk_off.assign(n_items(c), 0);
  c->item_gchunk_cnt.assign(n_items(c), 0);
  int maxc = 0;
  for (int g = 0; g < G; ++g) {
    const GridHost& H = c->grids[g];
    if (!H.kind) continue;
    maxc = std::max(maxc, H.form.ncolors);
    for (int sc = 0; sc < H.S; ++sc) {
      c->item_gchunk_off[H.item0 + sc] = (int)gall.size();
      std::vector<std::pair<double, GraphChunk>> keyed;
      for (int k = 0; k < H.form.ncolors; ++k) {
        const int64_t a = H.form.cstart[k], b = H.form.cstart[k + 1];
        for (int64_t s0 = a; s0 < b; s0 += kChunk)
          keyed.emplace_back((double)(s0 - a) / (double)(b - a),
                             GraphChunk{g, H.item0 + sc, sc, (int32_t)s0, (int32_t)std::min<int64_t>(kChunk, b - s0), 0});
      }
      std::stable_sort(keyed.begin(), keyed.end(),
                       [](const std::pair<double, GraphChunk>& x, const std::pair<double, GraphChunk>& y) {
                         return x.first < y.first;
                       });
      for (const auto& kc : keyed) gall.push_back(kc.second);
      c->item_gchunk_cnt[H.item0 + sc] = (int)gall.size() - c->item_gchunk_off[H.item0 + sc];
    }
  }
  for (int k = 0; k < maxc; ++k) {
    const int start = (int)gsweep.size();
    for (int g = 0; g < G; ++g) {
      const GridHost& H = c->grids[g];
      if (!H.kind || H.form.ncolors <= k) continue;
      const int64_t a = H.form.cstart[k], b = H.form.cstart[k + 1];
      for (int sc = 0; sc < H.S; ++sc)
        for (int64_t s0 = a; s0 < b; s0 += kChunk)
          gsweep.push_back(GraphChunk{g, H.item0 + sc, sc, (int32_t)s0, (int32_t)std::min<int64_t>(kChunk, b - s0),
                                      (int32_t)a});
    }
    c->gcolor.emplace_back(start, (int)gsweep.size() - start);
  }
  c->n_gchunks_all = (int)gall.size();
  PG_TRY(upload(c, c->g_chunks_all, gall));
  PG_TRY(upload(c, c->g_chunks_sweep, gsweep));
  PG_TRY(upload(c, c->tiles_sweep, sweep));
  PG_TRY(upload(c, c->tiles_all, tiles));
  // sources: first those that are non-zero outside their breakpoints ("always"), then the
  // windowed ones (zero before the first and after the last breakpoint, like every triangle),
  // so a step only visits the windows that can contain t.  Windowed sources are grouped in
  // buckets of their first breakpoint, 8 steps wide, and ordered by target slot inside a
  // bucket (and the "always" ones by slot), so the scattered updates of b touch memory in
  // order; the window test uses the bucket start and is widened by one bucket (the extra
  // sources add zero).
  struct SrcRef { double t0, t1, bucket; int g, s; size_t k; int64_t slot; };
  std::vector<SrcRef> always, windowed;
  const double bw = 8.0 * c->opt.h;
  for (int g = 0; g < G; ++g) {
    const GridHost& H = c->grids[g];
    for (int sc = 0; sc < H.S; ++sc) {
      const Src& S = H.src[sc];
      for (size_t k = 0; k < S.node.size(); ++k) {
        const int a = S.off[k], b = S.off[k + 1];
        SrcRef ref{S.t[a], S.t[b - 1], std::floor(S.t[a] / bw), g, sc, k,
                   (int64_t)sc * H.nstore + H.storage(S.node[k])};
        if (S.i[a] == 0.0 && S.i[b - 1] == 0.0) windowed.push_back(ref); else always.push_back(ref);
      }
    }
  }
  auto by_slot = [](const SrcRef& x, const SrcRef& y) { return x.g != y.g ? x.g < y.g : x.slot < y.slot; };
  std::sort(always.begin(), always.end(), by_slot);
  std::sort(windowed.begin(), windowed.end(), [&](const SrcRef& x, const SrcRef& y) {
    return x.bucket != y.bucket ? x.bucket < y.bucket : by_slot(x, y);
  });
  std::vector<double> win_t0;
  double win_maxw = 0.0;
  for (auto& w : windowed) { win_t0.push_back(w.bucket * bw); win_maxw = std::max(win_maxw, w.t1 - w.t0); }
  if (!windowed.empty()) win_maxw += bw;
  std::vector<int32_t> sg, si, so{0};
  std::vector<double> st, sv;
  for (const auto* list : {&always, &windowed})
    for (const SrcRef& ref : *list) {
      const GridHost& H = c->grids[ref.g];
      const Src& S = H.src[ref.s];
      sg.push_back(ref.g);
      si.push_back((int32_t)ref.slot);
      for (int j = S.off[ref.k]; j < S.off[ref.k + 1]; ++j) { st.push_back(S.t[j]); sv.push_back(S.i[j]); }
      so.push_back((int32_t)st.size());
    }
  c->n_src = (int)sg.size();
  PG_TRY(upload(c, c->src_grid, sg)); PG_TRY(upload(c, c->src_index, si)); PG_TRY(upload(c, c->src_off, so));
  PG_TRY(upload(c, c->src_t, st)); PG_TRY(upload(c, c->src_i, sv)); PG_TRY(upload(c, c->src_win_t0, win_t0));
  c->win_t0_host = win_t0;
  c->src_table = SourceTable{c->n_src, (const int32_t*)c->src_grid.p, (const int32_t*)c->src_index.p,
                             (const int32_t*)c->src_off.p, (const double*)c->src_t.p, (const double*)c->src_i.p,
                             (int32_t)always.size(), (int32_t)windowed.size(), (const double*)c->src_win_t0.p,
                             win_maxw};
  if (c->opt.resident) {
    // resident path: every grid must fit one workgroup; each item's sources, grouped by item
    c->res_max_nodes = 0;
    c->res_multi_layer = false;
    for (int g = 0; g < G; ++g) {
      const GridHost& H = c->grids[g];
      if (H.kind || H.n > kResMaxNodes || (int64_t)H.ind_a.size() > kResMaxInd)
        return set_err(c, PG_ERR_UNSUPPORTED, "resident: grid %d is %s; the resident path takes layered meshes of "
                       "at most %d nodes and %d series R-L branches", g,
                       H.kind ? "a general netlist" : "too large", kResMaxNodes, kResMaxInd);
      c->res_max_nodes = std::max<int>(c->res_max_nodes, (int)H.n);
      c->res_multi_layer = c->res_multi_layer || H.nl > 1;
    }
    if (c->opt.ordering != PG_ORDER_RED_BLACK)
      return set_err(c, PG_ERR_UNSUPPORTED, "resident: the resident path sweeps in red-black order");
    const int I = n_items(c);
    std::vector<int32_t> cnt(I + 1, 0), ids(sg.size());
    auto item_of = [&](size_t k) { const GridHost& H = c->grids[sg[k]]; return H.item0 + (int)(si[k] / H.nstore); };
    for (size_t k = 0; k < sg.size(); ++k) cnt[item_of(k) + 1]++;
    for (int q = 0; q < I; ++q) cnt[q + 1] += cnt[q];
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (size_t k = 0; k < sg.size(); ++k) ids[fill[item_of(k)]++] = (int32_t)k;
    PG_TRY(upload(c, c->res_src_off, cnt)); PG_TRY(upload(c, c->res_src, ids));
  }
  // flattened inductor list
  std::vector<int32_t> ig, il;
  for (int g = 0; g < G; ++g)
    for (size_t k = 0; k < c->grids[g].ind_a.size(); ++k) { ig.push_back(g); il.push_back((int32_t)k); }
  c->n_ind_total = (int)ig.size();
  PG_TRY(upload(c, c->ind_grid, ig)); PG_TRY(upload(c, c->ind_local, il));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->dirty = false;
  return PG_OK;
}

pg_status alloc_ctl(pg_ctx* c) {
  // grow the per-item control arrays, preserving vidx (which buffer holds each item's state)
  const int I = n_items(c);
  const int I_old = (int)(c->c_vidx.bytes / sizeof(int32_t));
  std::vector<int32_t> vidx(I, 0);
  if (c->c_vidx.p && I_old > 0)
    HIP_TRY(c, hipMemcpy(vidx.data(), c->c_vidx.p, std::min(I_old, I) * sizeof(int32_t), hipMemcpyDeviceToHost));
  PG_TRY(dalloc(c, c->c_norm, I * sizeof(unsigned long long)));
  PG_TRY(dalloc(c, c->c_last, I * sizeof(double)));
  PG_TRY(dalloc(c, c->c_active, I * sizeof(int32_t)));
  PG_TRY(dalloc(c, c->c_vidx, I * sizeof(int32_t)));
  PG_TRY(dalloc(c, c->c_sweeps, I * sizeof(int32_t)));
  PG_TRY(dalloc(c, c->c_failed, I * sizeof(int32_t)));
  HIP_TRY(c, hipMemcpy(c->c_vidx.p, vidx.data(), I * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemset(c->c_norm.p, 0, I * sizeof(unsigned long long)));
  HIP_TRY(c, hipMemset(c->c_last.p, 0, I * sizeof(double)));
  HIP_TRY(c, hipMemset(c->c_active.p, 0, I * sizeof(int32_t)));
  HIP_TRY(c, hipMemset(c->c_sweeps.p, 0, I * sizeof(int32_t)));
  HIP_TRY(c, hipMemset(c->c_failed.p, 0, I * sizeof(int32_t)));
  Ctl& k = c->ctl;
  k.norm_bits = (unsigned long long*)c->c_norm.p;
  k.last_norm = (double*)c->c_last.p;
  k.active = (int32_t*)c->c_active.p;
  k.vidx = (int32_t*)c->c_vidx.p;
  k.step_sweeps = (int32_t*)c->c_sweeps.p;
  k.failed = (int32_t*)c->c_failed.p;
  return PG_OK;
}

pg_status reset_stats_dev(pg_ctx* c) {
  HIP_TRY(c, hipMemsetAsync(c->c_stats64.p, 0, c->c_stats64.bytes, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->c_stats32.p, 0, c->c_stats32.bytes, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->c_statsd.p, 0, c->c_statsd.bytes, c->stream));
  c->seconds = 0.0;
  return PG_OK;
}

int32_t cur_vidx(pg_ctx* c, int item) {
  int32_t v = 0;
  (void)hipStreamSynchronize(c->stream);
  (void)hipMemcpy(&v, (const int32_t*)c->c_vidx.p + item, sizeof v, hipMemcpyDeviceToHost);
  return v;
}

pg_status check_gs(pg_ctx* c, int grid, int scen) {
  if (!c) return PG_ERR_INVALID_ARG;
  if (grid < 0 || grid >= (int)c->grids.size()) return set_err(c, PG_ERR_INVALID_ARG, "grid %d out of range", grid);
  if (scen < 0 || scen >= c->grids[grid].S) return set_err(c, PG_ERR_INVALID_ARG, "scenario %d out of range", scen);
  return PG_OK;
}

// Entry points built for layered meshes only.
pg_status mesh_only(pg_ctx* c, int grid, const char* what) {
  if (c->grids[grid].kind)
    return set_err(c, PG_ERR_UNSUPPORTED, "grid %d is a general netlist; %s is built for layered meshes", grid, what);
  return PG_OK;
}

// Inductive branches reported by pg_read_inductor_currents.
int64_t n_branches(const GridHost& H) {
  if (H.kind) return (int64_t)H.form.ind_near.size();
  return (int64_t)H.via_node.size() + (int64_t)H.pad_node.size();
}

// ---- one backward-Euler step -----------------------------------------------------------
// Profiled as one block: the work is charged once the active items are known (cycle_loop).
// Reserve the next decision: returns its tag; its flag slot is tag % kFlagSlots.  The device
// numbers its decisions with its own counter, which this host counter mirrors.
int next_tag(pg_ctx* c) { return (int)(c->flag_seq_host++ & kTagMask); }

// One residual pass over every tile group; with `tag`, followed by its decision (see
// pgrid_internal.h), whose tag is returned.
pg_status launch_resid_all(pg_ctx* c, int has_d, int din, double tol = 0.0, int* tag = nullptr,
                           const CloseArgs* close = nullptr, bool meshes = true) {
  const Tile* T = (const Tile*)c->tiles_sweep.p;
  int fuse = has_d ? 0 : c->fuse_next;
  if ((fuse & kFuseProbe) && c->probe_cancelled) fuse |= kFuseCancelled | (c->n_ind_total ? kFuseInd : 0);
  c->fuse_next = 0;
  const bool gprobe = !has_d && c->gprobe_next, gstore = !has_d && c->gstore_next;
  c->gprobe_next = c->gstore_next = false;
  double bytes = c->resid_bytes(c->begin_nodes, c->begin_coef, c->begin_rcoef, has_d != 0, fuse);
  if (gprobe || gstore) {  // whole steps only: the meshes' share, then the graphs' by their pass
    const double e = c->opt.precision == PG_PREC_FP32_REFINE ? 4.0 : 8.0;
    const double gn = (double)c->graph_nodes;
    bytes = meshes ? c->resid_bytes(c->all_nodes - c->graph_nodes, c->all_coef - c->graph_coef,
                                    c->all_rcoef - c->graph_rcoef, false, fuse) : 0.0;
    if (gprobe)  // v, 1/M_ii, q, gsup, row length per slot; column and FP32 conductance per entry
      bytes += (22.0 + e) * gn + 8.0 * (double)c->graph_entries;
    else  // b formed (C/h, constant, v, b), then r and v stored
      bytes += 32.0 * gn + (16.0 + e) * gn + 8.0 * (double)c->graph_rcoef;
  }
  ProfScope ps(c, 1, c->begin_nodes, bytes, (int)c->tile_groups.size() + (c->n_gchunks_all ? 1 : 0) + (tag ? 1 : 0));
  for (auto& grp : c->tile_groups) {
    if (!meshes) break;
    hipError_t e = launch_resid(fp32_mode(c), grp.multi, grp.nl, c->tile_rows, T + grp.off, grp.count,
                                (const GridDesc*)c->grid_desc.p, c->ctl, has_d, din, fuse, c->stream);
    if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "residual launch: %s", hipGetErrorString(e));
  }
  if (c->n_gchunks_all) {
    const GraphChunk* GC = (const GraphChunk*)c->g_chunks_all.p;
    const GridDesc* GD = (const GridDesc*)c->grid_desc.p;
    hipError_t e = hipSuccess;
    if (gprobe) {  // the opening probe
      e = launch_graph_probe(fp32_mode(c), GC, c->n_gchunks_all, GD, c->ctl, c->stream);
    } else if (gstore) {  // after a probe that found work: b, then r and v without the norm
      e = launch_graph_rhs(GC, c->n_gchunks_all, GD, c->ctl, 0, c->stream);
      if (e == hipSuccess) e = launch_graph_resid(fp32_mode(c), GC, c->n_gchunks_all, GD, c->ctl, 0, c->stream, 0);
    } else if (!(fuse & kFuseNoNorm)) {  // a mesh-only storing pass leaves the graphs alone
      e = launch_graph_resid(fp32_mode(c), GC, c->n_gchunks_all, GD, c->ctl, has_d, c->stream);
    }
    if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "residual launch: %s", hipGetErrorString(e));
  }
  if (!tag) return PG_OK;
  const DecideArgs da{1, n_items(c), (int)c->grids.size(), has_d, c->opt.check_every, c->opt.max_sweeps,
                      kFlagSlots, tol, (const GridDesc*)c->grid_desc.p};
  CloseArgs none{};
  hipError_t e = launch_decide(c->ctl, da, close ? *close : none, c->stream);
  if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "decision launch: %s", hipGetErrorString(e));
  *tag = next_tag(c);
  return PG_OK;
}

// Sweeps fused per launch (1 or 2); Jacobi sweeps are always launched one by one.
// Sweeps per launch of every mesh tile group: 4 only where every group has the four-sweep
// kernel (else the groups' launch counts, and so the buffer holding a cycle's result, would differ).
int sweeps_per_launch(const pg_ctx* c) {
  if (c->opt.ordering != PG_ORDER_RED_BLACK) return 1;
  const int spl = c->opt.sweeps_per_launch ? c->opt.sweeps_per_launch : 1;
  return spl == kTbSweeps && !c->tb_ok ? 1 : spl;
}

// Kernel launches per tile group in a cycle of nchk sweeps (fused launches, then one-sweep
// launches for the remainder); the cycle's result is in d[launches & 1].  (General graphs sweep
// in place in d[0], one launch per colour.)
int cycle_launches(const pg_ctx* c, int nchk) {
  const int spl = sweeps_per_launch(c);
  return nchk / spl + nchk % spl;
}

// All kernel launches of a cycle of nchk sweeps.
int cycle_launches_all(const pg_ctx* c, int nchk) {
  return cycle_launches(c, nchk) * (int)c->tile_groups.size() + nchk * (int)c->gcolor.size();
}

// The nchk sweeps of a cycle are timed as one block of back-to-back launches (one event pair
// per block, so event overhead does not inflate the per-launch average); every
// profile_every-th block is timed.  Its work is charged in cycle_loop from the active items.
pg_status launch_sweeps(pg_ctx* c, int nchk) {
  const Tile* T = (const Tile*)c->tiles_sweep.p;
  const int spl = sweeps_per_launch(c);
  ProfScope ps(c, 0, 0, 0.0, cycle_launches_all(c, nchk));
  for (auto& grp : c->tile_groups) {
    for (int s = 0, j = 0; s < nchk; ++j) {
      const int zero_in = s == 0 ? 1 : 0;
      hipError_t e;
      if (spl == kTbSweeps && nchk - s >= kTbSweeps) {
        e = launch_sweep_tb(fp32_mode(c), kTbSweeps, grp.multi, grp.nl, c->tile_rows, T + grp.off, grp.count,
                            (const GridDesc*)c->grid_desc.p, c->ctl, j & 1, zero_in, c->opt.omega, c->stream);
        s += kTbSweeps;
      } else if (spl == 2 && nchk - s >= 2) {  // staged once where the group has the kernel, else rings
        if (sweep_tb_supported(fp32_mode(c), grp.multi, c->opt.ordering, grp.nl, c->tile_rows, 2))
          e = launch_sweep_tb(fp32_mode(c), 2, grp.multi, grp.nl, c->tile_rows, T + grp.off, grp.count,
                              (const GridDesc*)c->grid_desc.p,
                              c->ctl, j & 1, zero_in, c->opt.omega, c->stream);
        else
          e = launch_sweep2(fp32_mode(c), grp.nl, c->tile_rows, T + grp.off, grp.count,
                            (const GridDesc*)c->grid_desc.p, c->ctl, j & 1, zero_in, c->opt.omega, c->stream);
        s += 2;
      } else {
        e = launch_sweep(fp32_mode(c), grp.multi, c->opt.ordering, grp.nl, c->tile_rows, T + grp.off, grp.count,
                         (const GridDesc*)c->grid_desc.p, c->ctl, j & 1, zero_in, c->opt.omega, c->stream);
        s += 1;
      }
      if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "sweep launch: %s", hipGetErrorString(e));
    }
  }
  // general graphs: one launch per colour and sweep, colours in order
  const GraphChunk* GC = (const GraphChunk*)c->g_chunks_sweep.p;
  for (int s = 0; s < nchk && !c->gcolor.empty(); ++s)
    for (auto& cr : c->gcolor) {
      hipError_t e = launch_graph_sweep(fp32_mode(c), GC + cr.first, cr.second, (const GridDesc*)c->grid_desc.p,
                                        c->ctl, s == 0 ? 1 : 0, c->opt.omega, c->stream);
      if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "sweep launch: %s", hipGetErrorString(e));
    }
  return PG_OK;
}

// Set the step clock (host mirror and device counter).
pg_status set_step(pg_ctx* c, int64_t k) {
  c->step = k;
  c->prev_valid = false;     // the three-level recurrence restarts with a two-level step
  c->pred_hist = 0;          // and the predictor from v(t)
  c->begun_next = false;     // a clock change voids any step opened ahead
  c->opening_queued = false;
  c->step_host = (long long)k;
  HIP_TRY(c, hipMemcpyAsync(c->ctl.step, &c->step_host, sizeof(long long), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PG_OK;
}

// Once pg_step_enqueue has run, a captured graph may replay it at any time without the host's
// knowledge, so from then on the step count is taken from the device clock, once the context's
// stream has drained.
pg_status sync_clock(pg_ctx* c) {
  if (!c->clock_on_device) return PG_OK;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  long long k = 0;
  HIP_TRY(c, hipMemcpy(&k, c->ctl.step, sizeof k, hipMemcpyDeviceToHost));
  c->step = k;
  return PG_OK;
}

// Whether any source can be non-zero at the time of step index `dev_step` (t = (dev_step + 1) h),
// judged from the host copy of the window table with one step of slack on either side.
bool sources_may_act(const pg_ctx* c, int64_t dev_step) {
  if (c->src_table.n_always > 0) return true;
  if (c->win_t0_host.empty()) return false;
  const double h = c->opt.h, t = (double)(dev_step + 1) * h;
  const auto lo = std::lower_bound(c->win_t0_host.begin(), c->win_t0_host.end(), t - c->src_table.win_maxw - h);
  const auto hi = std::upper_bound(c->win_t0_host.begin(), c->win_t0_host.end(), t + h);
  return lo < hi;
}

// The window of windowed sources for step index dev_step (t = (dev_step + 1) h), as the device
// search computes it: [first t0 >= t - widest window, first t0 > t).  -1 when dev_step < 0.
void host_window(const pg_ctx* c, int64_t dev_step, int* a, int* b) {
  *a = *b = -1;
  if (dev_step < 0) return;
  const double t = (double)(dev_step + 1) * c->opt.h;
  const auto& w = c->win_t0_host;
  *a = (int)(std::lower_bound(w.begin(), w.end(), t - c->src_table.win_maxw) - w.begin());
  *b = (int)(std::upper_bound(w.begin(), w.end(), t) - w.begin());
}

// Begin a step at time (step + 1) h: activate every item (only_item < 0) or one item, form the
// right-hand side on the active tiles, subtract the sources.  `begun`: the previous close has
// already opened the clock and the items.  dev_step >= 0 (the device step index the opening
// will see) lets the source launch be left out when no source can be non-zero.
pg_status begin_step(pg_ctx* c, int only_item, bool begun = false, int64_t dev_step = -1) {
  const int G = n_items(c);
  c->begin_nodes = c->all_nodes;
  c->begin_coef = c->all_coef;
  c->begin_rcoef = c->all_rcoef;
  if (only_item >= 0) {
    for (auto& H : c->grids)
      if (only_item >= H.item0 && only_item < H.item0 + H.S) {
        c->begin_nodes = H.n;
        c->begin_coef = H.coef_words;
        c->begin_rcoef = H.resid_words;
      }
  }
  Ctl k = c->ctl;
  hipError_t e;
  const bool three = c->opt.recurrence == PG_REC_THREE_LEVEL && c->n_gchunks_all > 0;
  if (!begun) {
    ProfScope ps(c, 3, 0);
    int wa = -1, wb = -1;
    host_window(c, dev_step, &wa, &wb);
    e = launch_step_begin(k, G, only_item, c->opt.h, c->src_table, wa, wb, c->stream);
    if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "step launch: %s", hipGetErrorString(e));
  }
  // A step opened from the host's clock (dev_step >= 0) with no source that can be non-zero
  // needs no separate right-hand-side pass on single-scenario meshes: the step's first residual
  // pass forms b itself (launch_resid_all picks up fuse_rhs_next).
  const bool loads = dev_step < 0 || sources_may_act(c, dev_step);
  // the predictor moves v to the step's first iterate after the right-hand side has read v(t):
  // 1 keeps v(t) only, 2 starts from 2 v(t) - v(t-h), 3 from 3 v(t) - 3 v(t-h) + v(t-2h)
  // so the right-hand side keeps its own pass
  const int predict = c->opt.predictor && only_item < 0 ? 1 + std::min(c->pred_hist, c->opt.predictor) : 0;
  bool fuse = only_item < 0 && !loads && c->ntiles_all > 0 && !predict;
  for (auto& grp : c->tile_groups) fuse = fuse && !grp.multi;
  // a step predicted to converge at once (the previous one did) only needs the norm: if it has
  // work after all, cycle_loop stores b and r before the first sweep
  c->fuse_next = fuse ? (kFuseRhs | (c->pred_chunks == 0 ? kFuseProbe : 0)) : 0;
  c->opening_probe = (c->fuse_next & kFuseProbe) != 0;
  // general graphs likewise: a step predicted to converge at once (two-level) opens with
  // k_graph_probe instead of the right-hand side and residual passes
  const bool gprobe = only_item < 0 && !loads && c->n_gchunks_all > 0 && !three && c->pred_chunks == 0;
  c->gprobe_next = gprobe;
  c->opening_gprobe = gprobe;
  // every item: the sweeps' tiles, whose scenario blocks load the shared C/h and G0 Vdd once;
  // one item: its own single-scenario tiles
  const Tile* T = (const Tile*)c->tiles_sweep.p;
  int off = 0, cnt = 0;
  if (!fuse)
    for (auto& grp : c->tile_groups) cnt = std::max(cnt, grp.off + grp.count);
  if (only_item >= 0) {
    T = (const Tile*)c->tiles_all.p;
    off = c->item_tile_off[only_item];
    cnt = c->item_tile_cnt[only_item];
  }
  const GraphChunk* GC = (const GraphChunk*)c->g_chunks_all.p;
  int goff = 0, gcnt = gprobe ? 0 : c->n_gchunks_all;
  if (only_item >= 0) { goff = c->item_gchunk_off[only_item]; gcnt = c->item_gchunk_cnt[only_item]; }
  if (cnt > 0 || gcnt > 0) {
    ProfScope ps(c, 2, 0, 0.0, (cnt > 0 ? 1 : 0) + (gcnt > 0 ? 1 : 0));
    e = launch_rhs(T + off, cnt, c->tile_rows, (const GridDesc*)c->grid_desc.p, k, c->stream, predict);
    if (e == hipSuccess) {
      if (three && c->prev_valid)
        e = launch_graph_rhs3(GC + goff, gcnt, (const GridDesc*)c->grid_desc.p, k, c->stream);
      else
        e = launch_graph_rhs(GC + goff, gcnt, (const GridDesc*)c->grid_desc.p, k, three ? 1 : 0, c->stream);
    }
    if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "rhs launch: %s", hipGetErrorString(e));
  }
  if (loads) {
    ProfScope ps(c, 2, 0);
    e = launch_sources(c->src_table, (const GridDesc*)c->grid_desc.p, k, 0.0, 1.0, c->stream);
    // the three-level right-hand side takes the change of the loads: add back I(t - h)
    if (e == hipSuccess && three && c->prev_valid)
      e = launch_sources(c->src_table, (const GridDesc*)c->grid_desc.p, k, -c->opt.h, -1.0, c->stream);
    if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "source launch: %s", hipGetErrorString(e));
  }
  if (three) c->prev_valid = true;
  if (predict) c->pred_hist = std::min(c->pred_hist + 1, c->opt.predictor);
  return PG_OK;
}


// Wait for the decision `tag`: spin on its host-visible flag, which the decision sets to
// (tag << 2) | (skipped << 1) | any after writing its accounting words; every so often ask
// whether the stream still has work, so a flag that can no longer arrive is reported, not
// awaited.
// The active work a decision found (scenario nodes, sweep and residual coefficient words).
// k_decide stores these three words just before its flag without a fence; each carries the low
// 24 bits of the decision's sequence above a 40-bit value, so once the flag is seen the host
// waits until all three match.
struct Acct { long long nodes, coef, rcoef; };
pg_status read_acct(pg_ctx* c, int tag, Acct* out) {
  const int slot = (int)((uint32_t)tag & (kFlagSlots - 1));
  const unsigned long long want = (uint32_t)tag & 0xffffffu, value = (1ull << 40) - 1;
  for (long spin = 1;; ++spin) {
    unsigned long long w[3];
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
      w[k] = (unsigned long long)__atomic_load_n(c->host_acct + 3 * slot + k, __ATOMIC_ACQUIRE);
      ok = ok && (w[k] >> 40) == want;
    }
    if (ok) {
      out->nodes = (long long)(w[0] & value);
      out->coef = (long long)(w[1] & value);
      out->rcoef = (long long)(w[2] & value);
      return PG_OK;
    }
    if ((spin & 1023) == 0 && hipStreamQuery(c->stream) == hipSuccess && spin > (1L << 20))
      return set_err(c, PG_ERR_STATE, "decision %d: accounting words out of sequence", tag);
  }
}

pg_status wait_decision(pg_ctx* c, int tag, int* any, int* skipped = nullptr) {
  const int slot = (int)((uint32_t)tag & (kFlagSlots - 1));
  const uint32_t want = (uint32_t)tag;
  auto take = [&](uint32_t f) {
    *any = (int)(f & 1u);
    if (skipped) *skipped = (int)((f >> 1) & 1u);
  };
  for (long spin = 1;; ++spin) {
    const uint32_t f = (uint32_t)__atomic_load_n(c->host_flags + slot, __ATOMIC_ACQUIRE);
    if ((f >> 2) == want) {
      take(f);
      return PG_OK;
    }
    if ((spin & 1023) == 0) {
      const hipError_t q = hipStreamQuery(c->stream);  // idle stream: the flag can no longer arrive
      if (q == hipSuccess) {
        const uint32_t g = (uint32_t)__atomic_load_n(c->host_flags + slot, __ATOMIC_ACQUIRE);
        if ((g >> 2) == want) {
          take(g);
          return PG_OK;
        }
        return set_err(c, PG_ERR_STATE, "decision %d: flag out of sequence", tag);
      }
      if (q != hipErrorNotReady) return set_err(c, PG_ERR_DEVICE, "decision wait: %s", hipGetErrorString(q));
    }
    __builtin_ia32_pause();
  }
}

// One refinement cycle: check_every sweeps, the FP64 residual with v <- v + d, the decision.
pg_status issue_cycle(pg_ctx* c, double tol, bool graphs, int* tag) {
  const int nchk = c->opt.check_every;
  if (graphs) {
    {
      ProfScope ps(c, 0, 0, 0.0, cycle_launches_all(c, nchk));
      HIP_TRY(c, hipGraphLaunch(c->g_sweeps, c->stream));
    }
    {
      ProfScope ps(c, 1, 0, 0.0, (int)c->tile_groups.size() + (c->n_gchunks_all ? 1 : 0));  // residual pass and its decision
      HIP_TRY(c, hipGraphLaunch(c->g_check, c->stream));
    }
    *tag = next_tag(c);
    return PG_OK;
  }
  PG_TRY(launch_sweeps(c, nchk));
  return launch_resid_all(c, 1, cycle_launches(c, nchk) & 1, tol, tag);
}

// Algorithm 1's inner loop for every active item, after the initial check (its decision tag in
// `first`) has been queued: refinement cycles until each item's scaled residual is <= tol.
// The host queues as many cycles as the previous step needed before waiting; past that
// prediction it keeps `lookahead` cycles queued beyond the one whose decision it waits for.
// Cycles queued after convergence find every item inactive and exit at once.
pg_status queue_opening(pg_ctx* c, int* first, int ahead, bool close_after = false);
pg_status queue_close(pg_ctx* c, bool open_next);

pg_status resume(pg_ctx* c) {
  hipError_t e = launch_resume(c->ctl, c->stream);
  if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "resume launch: %s", hipGetErrorString(e));
  c->maybe_stalled = false;
  return PG_OK;
}

pg_status cycle_loop(pg_ctx* c, double tol, bool graphs, int first, bool speculate = false,
                     int* next_first = nullptr, bool speculate_after = false) {
  const int nchk = c->opt.check_every;
  const int L = c->opt.lookahead;
  std::deque<int> pending{first};
  const size_t prof_base = c->prof_live.size();
  const int max_chunks = (c->opt.max_sweeps + nchk - 1) / nchk;
  int issued = 0, consumed = 0, last = -1;
  std::vector<Acct> work;  // active work after decision j (0: the initial check)
  // Speculation: after the predicted cycles, queue this step's close and the next step's opening
  // before waiting.  If a decision queued before them converges, the step is done and the next
  // opening is already on its way; if none does, the close stalls the device, the opening does
  // nothing, and the host resumes and queues more cycles.
  bool spec_tried = false, spec_live = false;
  int spec_tag = -1;
  size_t spec_b = 0, spec_e = 0;
  if (next_first) *next_first = -1;
  // the step's opening only took the norm (a probe): its b and r are stored before the first
  // sweep, by a pass that leaves the decided norm alone
  bool need_store = c->opening_probe;
  bool need_gstore = c->opening_gprobe;
  c->opening_probe = c->opening_gprobe = false;
  const bool closed_ahead = c->opening_closes;  // the opening's decision carries this step's close
  c->opening_closes = false;
  while (true) {
    if (!spec_live) {
      int want = consumed <= c->pred_chunks ? c->pred_chunks : consumed + L;
      want = std::min(want, consumed + kFlagSlots - 2);  // never reuse a slot still awaited
      while (issued < max_chunks && issued < want) {
        if (need_store || need_gstore) {
          c->fuse_next = kFuseRhs | kFuseNoNorm;
          c->gstore_next = need_gstore;
          // meshes whose opening was not a probe have stored their b and r already
          PG_TRY(launch_resid_all(c, 0, 0, 0.0, nullptr, nullptr, need_store));
          need_store = need_gstore = false;
        }
        c->cur_chunk = ++issued;
        int tag = 0;
        PG_TRY(issue_cycle(c, tol, graphs, &tag));
        pending.push_back(tag);
      }
    }
    if (speculate && !spec_tried) {
      spec_tried = true;
      const int saved_chunk = c->cur_chunk;
      spec_b = c->prof_live.size();
      c->maybe_stalled = true;
      if (!closed_ahead) PG_TRY(queue_close(c, true));
      PG_TRY(queue_opening(c, &spec_tag, 1, speculate_after && c->pred_chunks == 0 && !graphs));
      spec_e = c->prof_live.size();
      c->cur_chunk = saved_chunk;
      spec_live = true;
    }
    if (pending.empty()) break;
    const int t0 = pending.front();
    pending.pop_front();
    int any = 0;
    PG_TRY(wait_decision(c, t0, &any));
    ++consumed;
    Acct a{};
    PG_TRY(read_acct(c, t0, &a));
    work.push_back(a);
    if (!any) {
      last = consumed - 1;
      break;
    }
    if (spec_live && pending.empty()) {
      // the speculative close found the step still iterating: wait until the stalled opening's
      // decision has reported itself skipped, then let the device go on
      int a2 = 0, skipped = 0;
      PG_TRY(wait_decision(c, spec_tag, &a2, &skipped));
      if (!skipped) return set_err(c, PG_ERR_STATE, "a step was closed before it converged");
      PG_TRY(resume(c));
      spec_live = false;
      for (size_t q = spec_b; q < spec_e; ++q) c->prof_live[q].kind = -1;
    }
  }
  if (spec_live) {
    c->maybe_stalled = false;
    if (next_first) *next_first = spec_tag;
  }
  if (last < 0) last = issued;
  c->pred_chunks = last;
  c->cur_chunk = 0;
  // charge cycle k's sweeps and residual with the items the decision before it left active;
  // launches queued after convergence did no work
  for (size_t q = prof_base; q < c->prof_live.size(); ++q) {
    if (q >= spec_b && q < spec_e) continue;  // the close and the next opening
    ProfEvent& ev = c->prof_live[q];
    if (ev.chunk > last) { ev.kind = -1; continue; }
    if (ev.chunk < 1 || (ev.kind != 0 && ev.kind != 1)) continue;
    const Acct& wk = work[ev.chunk - 1];
    if (ev.kind == 0) {
      ev.units = wk.nodes * nchk;
      ev.bytes = c->cycle_bytes(wk.nodes, wk.coef, nchk);
    } else {
      ev.units = wk.nodes;
      ev.bytes = c->resid_bytes(wk.nodes, wk.coef, wk.rcoef, true);
    }
  }
  return PG_OK;
}

pg_status solve_active(pg_ctx* c, double tol) {
  c->cur_chunk = 0;
  int first = 0;
  PG_TRY(launch_resid_all(c, 0, 0, tol, &first));
  return cycle_loop(c, tol, false, first);
}

// Close a step: advance the device clock, statistics (count_step = 1) and the inductor branch
// currents.
pg_status end_step(pg_ctx* c, int count_step = 1, int begin_next = 0) {
  Ctl k = c->ctl;
  hipError_t e;
  {
    ProfScope ps(c, 3, 0);
    int wa = -1, wb = -1;
    if (begin_next && !c->capturing) host_window(c, c->step + 1, &wa, &wb);
    e = launch_step_end(k, n_items(c), count_step, begin_next, c->opt.h, c->src_table, wa, wb, c->stream);
    if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "step-end launch: %s", hipGetErrorString(e));
  }
  if (c->n_ind_total) {
    ProfScope ps(c, 3, 0);
    e = launch_inductors((const GridDesc*)c->grid_desc.p, (const int32_t*)c->ind_grid.p,
                         (const int32_t*)c->ind_local.p, c->n_ind_total, k, c->stream);
    if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "inductor launch: %s", hipGetErrorString(e));
  }
  return PG_OK;
}

// Capture the launches queued by `body` on a private stream into an executable graph.
template <typename F>
pg_status capture(pg_ctx* c, hipGraphExec_t* out, F body) {
  hipStream_t saved = c->stream;
  const int saved_prof = c->profile_every;
  c->stream = c->cap_stream;
  c->profile_every = 0;
  c->capturing = true;
  hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  pg_status st = e == hipSuccess ? body() : PG_ERR_DEVICE;
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
  c->capturing = false;
  c->stream = saved;
  c->profile_every = saved_prof;
  if (e != hipSuccess || e2 != hipSuccess)
    return set_err(c, PG_ERR_DEVICE, "graph capture failed: %s",
                   hipGetErrorString(e != hipSuccess ? e : e2));
  if (st != PG_OK) { (void)hipGraphDestroy(g); return st; }
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
  return PG_OK;
}

void drop_graphs(pg_ctx* c) {
  for (hipGraphExec_t* g : {&c->g_prologue, &c->g_sweeps, &c->g_check, &c->g_epilogue})
    if (*g) { (void)hipGraphExecDestroy(*g); *g = nullptr; }
  c->graphs_ready = false;
}

// The four graphs of a step: prologue (begin, RHS, sources, first residual and decision), the
// sweeps of a refinement cycle, its residual and decision, the epilogue.  Their launches have
// fixed arguments because the step clock and the flag slot advance on the device.
pg_status build_graphs(pg_ctx* c) {
  drop_graphs(c);
  const double tol = c->opt.tol;
  int dummy = 0;
  const uint64_t seq = c->flag_seq_host;
  PG_TRY(capture(c, &c->g_prologue, [&]() -> pg_status {
    PG_TRY(begin_step(c, -1));
    return launch_resid_all(c, 0, 0, tol, &dummy);
  }));
  PG_TRY(capture(c, &c->g_sweeps, [&]() { return launch_sweeps(c, c->opt.check_every); }));
  PG_TRY(capture(c, &c->g_check, [&]() -> pg_status {
    return launch_resid_all(c, 1, cycle_launches(c, c->opt.check_every) & 1, tol, &dummy);
  }));
  PG_TRY(capture(c, &c->g_epilogue, [&]() { return end_step(c, 1); }));
  (void)dummy;
  c->flag_seq_host = seq;  // capture queued nothing on the device
  c->graphs_ready = true;
  return PG_OK;
}

// Queue the opening of a step: clock and activation, right-hand side, sources, first residual
// and its decision (tag in *first).
pg_status queue_opening(pg_ctx* c, int* first, int ahead, bool close_after) {
  c->cur_chunk = 0;
  c->opening_closes = false;
  if (c->opt.graphs) {
    if (!c->graphs_ready) PG_TRY(build_graphs(c));
    c->opening_probe = false;
    {
      ProfScope ps(c, 3, 0);
      HIP_TRY(c, hipGraphLaunch(c->g_prologue, c->stream));
    }
    *first = next_tag(c);
    return PG_OK;
  }
  const bool begun = c->begun_next;  // the previous close already opened the clock and the items
  c->begun_next = false;
  PG_TRY(begin_step(c, -1, begun, c->step + ahead));
  if (!close_after) return launch_resid_all(c, 0, 0, c->opt.tol, first);
  // a step expected to converge at once (the previous one did) and followed by another: its
  // opening's decision also closes it and opens the next step; if it finds work, the close
  // stalls the device and cycle_loop goes on as after any stalled close
  CloseArgs ca{1, 1, 1, -1, -1, c->opt.h, c->src_table};
  host_window(c, c->step + ahead + 1, &ca.win_a, &ca.win_b);
  c->maybe_stalled = true;
  PG_TRY(launch_resid_all(c, 0, 0, c->opt.tol, first, &ca));
  if (c->n_ind_total) {
    ProfScope ps(c, 3, 0);
    hipError_t e = launch_inductors((const GridDesc*)c->grid_desc.p, (const int32_t*)c->ind_grid.p,
                                    (const int32_t*)c->ind_local.p, c->n_ind_total, c->ctl, c->stream);
    if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "inductor launch: %s", hipGetErrorString(e));
  }
  c->opening_closes = true;
  c->begun_next = true;
  return PG_OK;
}

// Queue the close of a step: statistics and clock, inductor branch currents; with open_next
// (plain launches) the same kernel also opens the next step's clock and items.
pg_status queue_close(pg_ctx* c, bool open_next) {
  if (c->opt.graphs) {
    HIP_TRY(c, hipGraphLaunch(c->g_epilogue, c->stream));
    return PG_OK;
  }
  PG_TRY(end_step(c, 1, open_next ? 1 : 0));
  c->begun_next = open_next;
  return PG_OK;
}

// One BE step of every item.  With `speculate`, the next step's opening is queued ahead (see
// cycle_loop) and picked up by the next call.
// The arguments of a resident launch of nsteps steps.
ResidentArgs resident_args(pg_ctx* c, int nsteps) {
  ResidentArgs a{};
  const Ctl& k = c->ctl;
  a.grids = (const GridDesc*)c->grid_desc.p;
  a.item_grid = (const int32_t*)c->c_item_grid.p;
  a.vidx = k.vidx;
  a.item_src_off = (const int32_t*)c->res_src_off.p;
  a.item_src = (const int32_t*)c->res_src.p;
  a.src_index = c->src_table.index;
  a.src_off = c->src_table.off;
  a.src_t = c->src_table.t;
  a.src_i = c->src_table.i;
  a.stat_sweeps = k.stat_sweeps; a.stat_updates = k.stat_updates; a.stat_checks = k.stat_checks;
  a.stat_max_sweeps = k.stat_max_sweeps; a.stat_last_sweeps = k.stat_last_sweeps; a.stat_failed = k.stat_failed;
  a.stat_last_res = k.stat_last_res; a.stat_max_res = k.stat_max_res;
  a.step = k.step;
  a.n_items = n_items(c);
  a.nsteps = nsteps;
  a.check_every = c->opt.check_every;
  a.max_sweeps = c->opt.max_sweeps;
  a.h = c->opt.h;
  a.tol = c->opt.tol;
  a.omega = c->opt.omega;
  return a;
}

// nsteps whole steps of every item in one launch (the resident path).
pg_status resident_steps(pg_ctx* c, int nsteps) {
  const ResidentArgs a = resident_args(c, nsteps);
  hipError_t e;
  {
    ProfScope ps(c, 3, 0);
    e = launch_resident(a, c->res_max_nodes, c->res_multi_layer, c->stream);
  }
  if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "resident launch: %s", hipGetErrorString(e));
  c->step += nsteps;
  return PG_OK;
}

pg_status one_step(pg_ctx* c, bool speculate = false, bool speculate_after = false) {
  int first = 0;
  if (c->opening_queued) {
    first = c->opening_tag;
    c->opening_queued = false;
  } else {
    if (c->maybe_stalled) PG_TRY(resume(c));  // an earlier call stopped on an error mid-speculation
    PG_TRY(queue_opening(c, &first, 0, speculate && c->pred_chunks == 0 && !c->opt.graphs));
  }
  int next = -1;
  PG_TRY(cycle_loop(c, c->opt.tol, c->opt.graphs != 0, first, speculate, &next, speculate_after));
  if (next >= 0) {
    c->opening_queued = true;
    c->opening_tag = next;
  } else {
    PG_TRY(queue_close(c, speculate));
  }
  c->step++;
  return PG_OK;
}

// ---- adjoint helpers ----------------------------------------------------------------
// to_buf 1: buf <- v; 0: v <- buf; 2: v <- 2 v - buf (the extrapolated first iterate)
pg_status state_copy(pg_ctx* c, int item, double* buf, int to_buf) {
  const Tile* T = (const Tile*)c->tiles_all.p + c->item_tile_off[item];
  hipError_t e = launch_state_copy(T, c->item_tile_cnt[item], c->tile_rows, (const GridDesc*)c->grid_desc.p,
                                   c->ctl, buf, to_buf, c->stream);
  if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "state copy: %s", hipGetErrorString(e));
  return PG_OK;
}

// Switch grid adj.grid between its forward view (state = voltages) and its adjoint view
// (state = lambda, right-hand side = adjoint right-hand side); the item's buffer index is
// exchanged with the one saved for the other view.
pg_status use_view(pg_ctx* c, bool adjoint) {
  auto& A = c->adj;
  const GridDesc* src = adjoint ? &A.view : &c->desc_host[A.grid];
  HIP_TRY(c, hipMemcpyAsync((GridDesc*)c->grid_desc.p + A.grid, src, sizeof(GridDesc), hipMemcpyHostToDevice,
                            c->stream));
  hipError_t e = launch_swap_vidx(c->ctl, A.item, (int32_t*)A.saved_vidx.p, c->stream);
  if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "view switch: %s", hipGetErrorString(e));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PG_OK;
}

// Copy an item-slice array in storage layout to the caller's [nl][rows][cols] layout.
pg_status unpad(pg_ctx* c, const GridHost& H, const double* src, double* dst, int cols, int rows, bool to_device) {
  const hipMemcpyKind kind = to_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  for (int l = 0; l < H.nl; ++l)
    HIP_TRY(c, hipMemcpy2DAsync(dst + (size_t)l * rows * cols, cols * sizeof(double),
                                src + (size_t)l * H.ny * H.X, H.X * sizeof(double), cols * sizeof(double), rows,
                                kind, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PG_OK;
}

pg_status loss_backward(pg_ctx* c, double tol_adj, double* dC, double* dgE, double* dgN, bool on_device) {
  if (!c) return PG_ERR_INVALID_ARG;
  auto& A = c->adj;
  if (!A.recorded) return set_err(c, PG_ERR_STATE, "pg_loss_backward needs a recorded pg_loss_forward");
  if (!(std::isfinite(tol_adj) && tol_adj > 0)) return set_err(c, PG_ERR_INVALID_ARG, "tol_adj must be > 0");
  if (!dC || !dgE || !dgN) return set_err(c, PG_ERR_INVALID_ARG, "gradient outputs are NULL");
  HIP_TRY(c, hipSetDevice(c->device));
  GridHost& H = c->grids[A.grid];
  const size_t ns = (size_t)H.nstore;
  HIP_TRY(c, hipMemsetAsync(A.lam0.p, 0, A.lam0.bytes, c->stream));
  HIP_TRY(c, hipMemsetAsync(A.lam1.p, 0, A.lam1.bytes, c->stream));
  HIP_TRY(c, hipMemsetAsync(A.dC.p, 0, A.dC.bytes, c->stream));
  HIP_TRY(c, hipMemsetAsync(A.dgE.p, 0, A.dgE.bytes, c->stream));
  HIP_TRY(c, hipMemsetAsync(A.dgN.p, 0, A.dgN.bytes, c->stream));
  if (A.dbr_g.bytes) HIP_TRY(c, hipMemsetAsync(A.dbr_g.p, 0, A.dbr_g.bytes, c->stream));
  if (A.dbr_L.bytes) HIP_TRY(c, hipMemsetAsync(A.dbr_L.p, 0, A.dbr_L.bytes, c->stream));
  if (A.mu.bytes) HIP_TRY(c, hipMemsetAsync(A.mu.p, 0, A.mu.bytes, c->stream));
  A.branch_ready = false;
  const int ni = A.n_ind;
  double* icur = (double*)H.ind_i_d.p + (size_t)A.scen * ni;  // the item's inductor currents
  double* isg = (double*)A.iseg.p;
  HIP_TRY(c, hipMemsetAsync(A.saved_vidx.p, 0, sizeof(int32_t), c->stream));
  double* ck = (double*)A.ckpts.p;
  double* seg = (double*)A.seg.p;
  const Tile* T = (const Tile*)c->tiles_all.p + c->item_tile_off[A.item];
  const int nt = c->item_tile_cnt[A.item];
  const GridDesc* gd = (const GridDesc*)c->grid_desc.p;
  // with the predictor: the adjoint states of the last two solves (lam_keep[lam_cur] the older)
  double* lam_keep[2] = {(double*)A.lamp.p, (double*)A.lamq.p};
  int lam_cur = 0;
  bool lam_prev = false;
  for (int j = A.nseg - 1; j >= 0; --j) {
    const int kb = j * A.ckpt, ke = std::min(A.K, kb + A.ckpt), len = ke - kb;
    // recompute the forward states of the segment from its checkpoint (only this item steps)
    PG_TRY(state_copy(c, A.item, ck + (size_t)j * ns, 0));
    HIP_TRY(c, hipMemcpyAsync(seg, ck + (size_t)j * ns, ns * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (ni) {
      HIP_TRY(c, hipMemcpyAsync(icur, (const double*)A.ickpts.p + (size_t)j * ni, ni * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream));
      HIP_TRY(c, hipMemcpyAsync(isg, icur, ni * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    }
    PG_TRY(set_step(c, A.k0 + kb));
    for (int q = 1; q <= len; ++q) {
      PG_TRY(begin_step(c, A.item));
      // with the predictor, from the segment's second step on: start from 2 v(q-1) - v(q-2)
      if (c->opt.predictor && q >= 2) PG_TRY(state_copy(c, A.item, seg + (size_t)(q - 2) * ns, 2));
      PG_TRY(solve_active(c, c->opt.tol));
      hipError_t e2 = launch_step_end(c->ctl, n_items(c), 2, 0, c->opt.h, c->src_table, -1, -1, c->stream);
      if (e2 == hipSuccess) e2 = launch_ind_update_item(gd, A.grid, A.item, A.scen, c->ctl, ni, c->stream);
      if (e2 != hipSuccess) return set_err(c, PG_ERR_DEVICE, "step-end launch: %s", hipGetErrorString(e2));
      c->step++;
      PG_TRY(state_copy(c, A.item, seg + (size_t)q * ns, 1));
      if (ni)
        HIP_TRY(c, hipMemcpyAsync(isg + (size_t)q * ni, icur, ni * sizeof(double), hipMemcpyDeviceToDevice,
                                  c->stream));
    }
    // reverse sweep over the segment on the adjoint view
    PG_TRY(use_view(c, true));
    for (int q = len; q >= 1; --q) {
      // mu_k from mu_{k+1} and lambda_{k+1} (the adjoint state before this step's solve)
      hipError_t e = launch_adj_mu(gd, A.grid, A.item, A.scen, c->ctl, (double*)A.mu.p, ni, c->stream);
      if (e == hipSuccess)
        e = launch_adj_rhs(T, nt, c->tile_rows, gd, c->ctl, seg + (size_t)q * ns, A.margin, (const double*)A.mu.p,
                           ni, c->stream);
      if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "adjoint rhs: %s", hipGetErrorString(e));
      e = launch_step_begin(c->ctl, n_items(c), A.item, c->opt.h, c->src_table, -1, -1, c->stream);
      if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "adjoint step: %s", hipGetErrorString(e));
      if (c->opt.predictor && A.lamp.p) {  // keep lambda_{q+1}; start from 2 lambda_{q+1} - lambda_{q+2}
        PG_TRY(state_copy(c, A.item, lam_keep[1 - lam_cur], 1));
        if (lam_prev) PG_TRY(state_copy(c, A.item, lam_keep[lam_cur], 2));
        lam_cur = 1 - lam_cur;
        lam_prev = true;
      }
      PG_TRY(solve_active(c, tol_adj));
      e = launch_adj_grad(T, nt, c->tile_rows, gd, c->ctl, seg + (size_t)q * ns, seg + (size_t)(q - 1) * ns,
                          1.0 / c->opt.h, (double*)A.dC.p, (double*)A.dgE.p, (double*)A.dgN.p, c->stream);
      if (e == hipSuccess)
        e = launch_adj_branch_grad(gd, A.grid, A.item, A.scen, c->ctl, seg + (size_t)q * ns,
                                   (const int32_t*)A.br_slot.p, (const int32_t*)A.br_ind.p, (const double*)A.br_g.p,
                                   (const double*)A.br_L.p, A.n_vias, A.n_vias + A.n_pads, (int64_t)H.X * H.ny,
                                   c->opt.h, (const double*)A.mu.p, isg + (size_t)(q - 1) * ni,
                                   (double*)A.dbr_g.p, (double*)A.dbr_L.p, c->stream);
      if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "adjoint gradient: %s", hipGetErrorString(e));
    }
    PG_TRY(use_view(c, false));
  }
  // back to the state the forward pass ended in
  PG_TRY(state_copy(c, A.item, (double*)A.vend.p, 0));
  if (ni) HIP_TRY(c, hipMemcpyAsync(icur, A.iend.p, ni * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  PG_TRY(set_step(c, A.k0 + A.K));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int32_t failed = 0;
  HIP_TRY(c, hipMemcpy(&failed, c->ctl.stat_failed, sizeof failed, hipMemcpyDeviceToHost));
  PG_TRY(unpad(c, H, (const double*)A.dC.p, dC, H.nx, H.ny, on_device));
  PG_TRY(unpad(c, H, (const double*)A.dgE.p, dgE, H.nx - 1, H.ny, on_device));
  PG_TRY(unpad(c, H, (const double*)A.dgN.p, dgN, H.nx, H.ny - 1, on_device));
  if (failed) {
    HIP_TRY(c, hipMemset(c->ctl.stat_failed, 0, sizeof(int32_t)));
    return set_err(c, PG_ERR_NO_CONVERGENCE, "an adjoint or recomputed step reached max_sweeps");
  }
  A.branch_ready = true;
  return PG_OK;
}

pg_status fill_v(pg_ctx* c, GridHost& H, const double* v, int scen, int32_t vidx) {
  c->prev_valid = false;
  c->pred_hist = 0;
  // write the voltages of one scenario into its slice of the current buffer
  std::vector<double> buf((size_t)H.nstore, H.vdd);
  for (int64_t i = 0; i < H.n; ++i) buf[(size_t)H.storage(i)] = v ? v[i] : H.vdd;
  double* dst = (double*)(vidx ? H.v1.p : H.v0.p) + (size_t)scen * H.nstore;
  HIP_TRY(c, hipMemcpy(dst, buf.data(), buf.size() * sizeof(double), hipMemcpyHostToDevice));
  return PG_OK;
}

}  // namespace

namespace pgrid {

pg_status upload_graph(pg_ctx* c, GraphForm& form, double vdd, int32_t n_scen, int32_t* grid_id) {
  if (n_scen < 1) return set_err(c, PG_ERR_INVALID_ARG, "n_scen must be >= 1");
  HIP_TRY(c, hipSetDevice(c->device));
  c->grids.emplace_back();
  GridHost& H = c->grids.back();
  H.kind = 1;
  H.nx = form.n; H.ny = 1; H.nl = 1; H.S = n_scen; H.item0 = n_items(c) - n_scen;
  H.P = form.n; H.n = form.n; H.vdd = vdd;
  H.X = (int32_t)form.nslots;
  H.nstore = form.nslots;
  H.form = std::move(form);
  H.src.assign(n_scen, Src{});
  for (auto& s : H.src) s.off = {0};
  const size_t ns = (size_t)H.nstore * H.S;
  pg_status ps;
  if ((ps = dalloc(c, H.v0, ns * sizeof(double))) != PG_OK || (ps = dalloc(c, H.v1, ns * sizeof(double))) != PG_OK ||
      (ps = dalloc(c, H.b, ns * sizeof(double))) != PG_OK) {
    c->grids.pop_back();
    return ps;
  }
  std::vector<double> vinit(ns, H.vdd);
  HIP_TRY(c, hipMemcpy(H.v0.p, vinit.data(), ns * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(H.v1.p, vinit.data(), ns * sizeof(double), hipMemcpyHostToDevice));
  PG_TRY(alloc_ctl(c));
  c->dirty = true;
  if (grid_id) *grid_id = (int32_t)c->grids.size() - 1;
  return PG_OK;
}

}  // namespace pgrid

extern "C" {

pg_status pg_create(pg_ctx** out, int32_t device, void* stream) {
  if (!out) return PG_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return PG_ERR_DEVICE;
  if (device < 0 || device >= count) return PG_ERR_INVALID_ARG;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return PG_ERR_DEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PG_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return PG_ERR_DEVICE;
  double* scr = nullptr;
  if (scratch_address(device, &scr) != hipSuccess) return PG_ERR_DEVICE;
  pg_ctx* c = new pg_ctx();
  c->device = device;
  c->scratch_dev = scr;
  pg_default_options(&c->opt);
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) { delete c; return PG_ERR_DEVICE; }
    c->own_stream = true;
  }
  const int nslots = kFlagSlots;
  if (hipHostMalloc((void**)&c->host_flags, nslots * sizeof(int32_t), hipHostMallocMapped | hipHostMallocCoherent) !=
          hipSuccess ||
      hipHostGetDevicePointer((void**)&c->dev_flags, c->host_flags, 0) != hipSuccess) {
    pg_destroy(c);
    return PG_ERR_DEVICE;
  }
  std::memset(c->host_flags, 0xff, nslots * sizeof(int32_t));  // no tag matches before a decision runs
  if (hipHostMalloc((void**)&c->host_acct, 3 * nslots * sizeof(long long), hipHostMallocMapped | hipHostMallocCoherent) !=
          hipSuccess ||
      hipHostGetDevicePointer((void**)&c->dev_acct, c->host_acct, 0) != hipSuccess) {
    pg_destroy(c);
    return PG_ERR_DEVICE;
  }
  // slot s only ever receives decisions whose sequence is s modulo nslots; its initial words carry
  // the tag s + 1 (not congruent to s), so no decision's tag matches them before it has written
  for (int s = 0; s < nslots; ++s)
    for (int k = 0; k < 3; ++k) c->host_acct[3 * s + k] = (long long)((unsigned long long)(s + 1) << 40);

  if (dalloc(c, c->c_stats64, 3 * sizeof(long long)) != PG_OK || dalloc(c, c->c_stats32, 4 * sizeof(int32_t)) != PG_OK ||
      dalloc(c, c->c_statsd, 2 * sizeof(double)) != PG_OK) {
    pg_destroy(c);
    return PG_ERR_OOM;
  }
  if (dalloc(c, c->c_clock, 64) != PG_OK || hipMemset(c->c_clock.p, 0, 64) != hipSuccess) {
    pg_destroy(c);
    return PG_ERR_OOM;
  }
  Ctl& k = c->ctl;
  k.step = (long long*)c->c_clock.p;
  k.t_now = (double*)((char*)c->c_clock.p + 8);
  k.src_window = (int32_t*)((char*)c->c_clock.p + 16);
  k.flag_seq = (uint32_t*)((char*)c->c_clock.p + 24);
  k.stall = (int32_t*)((char*)c->c_clock.p + 28);
  k.any_active = c->dev_flags;
  k.acct = c->dev_acct;
  if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    pg_destroy(c);
    return PG_ERR_DEVICE;
  }
  k.stat_sweeps = (long long*)c->c_stats64.p;
  k.stat_updates = k.stat_sweeps + 1;
  k.stat_checks = k.stat_sweeps + 2;
  k.stat_last_sweeps = (int32_t*)c->c_stats32.p;
  k.stat_max_sweeps = k.stat_last_sweeps + 1;
  k.stat_failed = k.stat_last_sweeps + 2;
  k.stat_last_res = (double*)c->c_statsd.p;
  k.stat_max_res = k.stat_last_res + 1;
  if (reset_stats_dev(c) != PG_OK || hipStreamSynchronize(c->stream) != hipSuccess) { pg_destroy(c); return PG_ERR_DEVICE; }
  *out = c;
  return PG_OK;
}

void pg_destroy(pg_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto& H : c->grids) {
    DBuf* bufs[] = {&H.gE64, &H.gN64, &H.gU64, &H.D64, &H.ch64, &H.bconst64, &H.gEs, &H.gNs, &H.gUs, &H.invDs,
                    &H.v0, &H.v1, &H.b, &H.r, &H.d0, &H.d1, &H.vh, &H.vh2, &H.ind_a_d, &H.ind_b_d, &H.ind_geq_d,
                    &H.ind_alpha_d, &H.ind_i_d, &H.inc_off_d, &H.inc_ind_d, &H.ind_vfar_d,
                    &H.slot_d, &H.sl_off_d, &H.sl_len_d, &H.sl_col_d, &H.sl_w64_d, &H.sl_ws_d, &H.cap_off_d, &H.cap_col_d,
                    &H.cap_val_d, &H.vprev0, &H.vprev1, &H.g3diag_d, &H.sl_g64_d, &H.bres_d, &H.bl_d,
                    &H.gq64_d, &H.gsup32_d, &H.gw32_d, &H.gE_raw, &H.gN_raw, &H.C_raw, &H.chk_d,
                    &H.padt_slot_d, &H.padt_val_d};
    for (DBuf* b : bufs) dfree(*b);
  }
  DBuf* bufs[] = {&c->grid_desc, &c->tiles_all, &c->tiles_sweep, &c->src_grid, &c->src_index, &c->src_off, &c->src_t, &c->src_i,
                  &c->g_chunks_all, &c->g_chunks_sweep,
                  &c->ind_grid, &c->ind_local, &c->c_norm, &c->c_last, &c->c_active, &c->c_vidx, &c->c_sweeps,
                  &c->c_failed, &c->c_any, &c->c_stats64, &c->c_stats32, &c->c_statsd, &c->c_nodes, &c->c_item_grid,
                  &c->c_clock, &c->src_win_t0, &c->res_src_off, &c->res_src};
  for (DBuf* b : bufs) dfree(*b);
  DBuf* abufs[] = {&c->adj.ckpts, &c->adj.vend, &c->adj.seg, &c->adj.lam0, &c->adj.lam1, &c->adj.arhs,
                   &c->adj.dC, &c->adj.dgE, &c->adj.dgN, &c->adj.part, &c->adj.J, &c->adj.saved_vidx,
                   &c->adj.br_slot, &c->adj.br_ind, &c->adj.br_g, &c->adj.br_L, &c->adj.dbr_g, &c->adj.dbr_L,
                   &c->adj.ickpts, &c->adj.iseg, &c->adj.iend, &c->adj.mu};
  for (DBuf* b : abufs) dfree(*b);
  for (auto& e : c->prof_live) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
  for (auto e : c->prof_pool) (void)hipEventDestroy(e);
  if (c->host_flags) (void)hipHostFree(c->host_flags);
  if (c->host_acct) (void)hipHostFree(c->host_acct);
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* pg_last_error(const pg_ctx* c) { return c ? c->err.c_str() : "null context"; }

pg_status pg_set_options(pg_ctx* c, const pg_options* o) {
  if (!c) return PG_ERR_INVALID_ARG;
  char msg[256] = {0};
  pg_status st = pg_validate_options(o, msg, sizeof msg);
  if (st != PG_OK) return set_err(c, st, "%s", msg);
  // h and precision change the coefficients, tile_rows and scen_block the tiles, the recurrence
  // the buffers of general netlists: rebuild; anything else only invalidates the captured graphs
  if (o->h != c->opt.h || o->precision != c->opt.precision || o->tile_rows != c->opt.tile_rows ||
      o->scen_block != c->opt.scen_block || o->recurrence != c->opt.recurrence || o->resident != c->opt.resident ||
      o->predictor != c->opt.predictor)
    c->dirty = true;
  drop_graphs(c);
  c->opt = *o;
  return PG_OK;
}

pg_status pg_get_options(const pg_ctx* c, pg_options* out) {
  if (!c || !out) return PG_ERR_INVALID_ARG;
  *out = c->opt;
  return PG_OK;
}

pg_status pg_upload_mesh(pg_ctx* c, const pg_mesh* m, int32_t n_scen, int32_t* grid_id) {
  if (!c) return PG_ERR_INVALID_ARG;
  char msg[256] = {0};
  pg_status st = pg_validate_mesh(m, msg, sizeof msg);
  if (st != PG_OK) return set_err(c, st, "%s", msg);
  if (n_scen < 1) return set_err(c, PG_ERR_INVALID_ARG, "n_scen must be >= 1");
  HIP_TRY(c, hipSetDevice(c->device));
  c->grids.emplace_back();
  GridHost& H = c->grids.back();
  H.nx = m->nx; H.ny = m->ny; H.nl = m->nl; H.S = n_scen; H.item0 = n_items(c) - n_scen;
  H.P = (int64_t)m->nx * m->ny; H.n = H.P * m->nl; H.vdd = m->vdd;
  H.X = (m->nx + kPitchAlign - 1) / kPitchAlign * kPitchAlign;
  H.nstore = (int64_t)H.X * m->ny * m->nl;
  H.gE.assign(m->gE, m->gE + (size_t)m->nl * m->ny * (m->nx - 1));
  H.gN.assign(m->gN, m->gN + (size_t)m->nl * (m->ny - 1) * m->nx);
  H.C.assign(m->C, m->C + H.n);
  H.via_node.assign(m->via_node, m->via_node + m->n_vias);
  H.via_g.assign(m->via_g, m->via_g + m->n_vias);
  if (m->via_L) H.via_L.assign(m->via_L, m->via_L + m->n_vias);
  H.pad_node.assign(m->pad_node, m->pad_node + m->n_pads);
  H.pad_g.assign(m->pad_g, m->pad_g + m->n_pads);
  if (m->pad_L) H.pad_L.assign(m->pad_L, m->pad_L + m->n_pads);
  H.src.assign(n_scen, Src{});
  for (auto& s : H.src) s.off = {0};
  const size_t ns = (size_t)H.nstore * H.S;
  pg_status ps;
  if ((ps = dalloc(c, H.v0, ns * sizeof(double))) != PG_OK || (ps = dalloc(c, H.v1, ns * sizeof(double))) != PG_OK ||
      (ps = dalloc(c, H.b, ns * sizeof(double))) != PG_OK) {
    c->grids.pop_back();
    return ps;
  }
  std::vector<double> vinit(ns, H.vdd);
  HIP_TRY(c, hipMemcpy(H.v0.p, vinit.data(), ns * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(H.v1.p, vinit.data(), ns * sizeof(double), hipMemcpyHostToDevice));
  PG_TRY(alloc_ctl(c));
  c->dirty = true;
  if (grid_id) *grid_id = (int32_t)c->grids.size() - 1;
  return PG_OK;
}

pg_status pg_sweep_launch_info(pg_ctx* c, int32_t* sweeps_per_launch_out, int32_t* staged) {
  if (!c) return PG_ERR_INVALID_ARG;
  if (!sweeps_per_launch_out || !staged) return set_err(c, PG_ERR_INVALID_ARG, "output pointers are NULL");
  HIP_TRY(c, hipSetDevice(c->device));
  PG_TRY(prepare(c));
  const int spl = sweeps_per_launch(c);
  bool all = spl > 1 && !c->tile_groups.empty();
  for (auto& grp : c->tile_groups)
    all = all && sweep_tb_supported(fp32_mode(c), grp.multi, c->opt.ordering, grp.nl, c->tile_rows, spl);
  *sweeps_per_launch_out = spl;
  *staged = all ? 1 : 0;
  return PG_OK;
}

pg_status pg_graph_info(const pg_ctx* c, int32_t grid, int32_t* n_nodes, int32_t* n_colors, int64_t* n_slots,
                        int64_t* nnz, int32_t* n_inductors) {
  if (!c || grid < 0 || grid >= (int)c->grids.size()) return PG_ERR_INVALID_ARG;
  const GridHost& H = c->grids[grid];
  if (!H.kind) return PG_ERR_INVALID_ARG;
  if (n_nodes) *n_nodes = (int32_t)H.n;
  if (n_colors) *n_colors = H.form.ncolors;
  if (n_slots) *n_slots = H.form.nslots;
  if (nnz) *nnz = H.form.nnz;
  if (n_inductors) *n_inductors = (int32_t)H.form.ind_near.size();
  return PG_OK;
}

pg_status pg_recurrence_drift(pg_ctx* c, int32_t grid, int32_t scen, double* drift) {
  PG_TRY(check_gs(c, grid, scen));
  if (!drift) return set_err(c, PG_ERR_INVALID_ARG, "drift output is NULL");
  GridHost& H = c->grids[grid];
  if (!H.kind || c->opt.recurrence != PG_REC_THREE_LEVEL || !c->prev_valid || c->opening_queued || c->dirty)
    return set_err(c, PG_ERR_STATE, "pg_recurrence_drift needs a general netlist stepped under the three-level "
                   "recurrence");
  HIP_TRY(c, hipSetDevice(c->device));
  const int item = H.item0 + scen;
  const GraphChunk* GC = (const GraphChunk*)c->g_chunks_all.p + c->item_gchunk_off[item];
  const int n = c->item_gchunk_cnt[item];
  const GridDesc* gd = (const GridDesc*)c->grid_desc.p;
  unsigned long long* nb = (unsigned long long*)c->c_norm.p + item;
  // the right-hand sides are rebuilt at the next step, so b serves as scratch here
  HIP_TRY(c, hipMemsetAsync(nb, 0, sizeof *nb, c->stream));
  hipError_t e = launch_graph_kcl(GC, n, gd, c->ctl, c->stream);
  if (e == hipSuccess) e = launch_sources(c->src_table, gd, c->ctl, 0.0, -1.0, c->stream);
  if (e == hipSuccess) e = launch_graph_absmax_b(GC, n, gd, c->ctl, c->stream);
  if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "drift launch: %s", hipGetErrorString(e));
  unsigned long long bits = 0;
  HIP_TRY(c, hipMemcpyAsync(&bits, nb, sizeof bits, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemsetAsync(nb, 0, sizeof *nb, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::memcpy(drift, &bits, sizeof bits);
  return PG_OK;
}

pg_status pg_set_pwl(pg_ctx* c, int32_t grid, int32_t scen, int32_t n_src, const int32_t* node,
                     const int32_t* offsets, const double* t, const double* i) {
  PG_TRY(check_gs(c, grid, scen));
  GridHost& H = c->grids[grid];
  if (n_src < 0 || (n_src > 0 && (!node || !offsets || !t || !i)))
    return set_err(c, PG_ERR_INVALID_ARG, "bad source arrays");
  if (n_src > 0 && offsets[0] != 0) return set_err(c, PG_ERR_INVALID_ARG, "offsets[0] must be 0");
  std::vector<char> seen(H.n, 0);
  for (int k = 0; k < n_src; ++k) {
    if (node[k] < 0 || node[k] >= H.n) return set_err(c, PG_ERR_INVALID_ARG, "source %d: node out of range", k);
    if (seen[node[k]]) return set_err(c, PG_ERR_INVALID_ARG, "source %d: node %d already has a source", k, node[k]);
    seen[node[k]] = 1;
    if (offsets[k + 1] <= offsets[k]) return set_err(c, PG_ERR_INVALID_ARG, "source %d: no breakpoints", k);
    for (int j = offsets[k]; j < offsets[k + 1]; ++j) {
      if (!std::isfinite(t[j]) || !std::isfinite(i[j])) return set_err(c, PG_ERR_INVALID_ARG, "source %d: non-finite breakpoint", k);
      if (j > offsets[k] && !(t[j] > t[j - 1])) return set_err(c, PG_ERR_INVALID_ARG, "source %d: times not increasing", k);
    }
  }
  Src S;
  S.node.assign(node, node + n_src);
  S.off.assign(offsets, offsets + n_src + 1);
  if (n_src == 0) S.off = {0};
  const int nb = n_src ? offsets[n_src] : 0;
  S.t.assign(t ? t : nullptr, t ? t + nb : nullptr);
  S.i.assign(i ? i : nullptr, i ? i + nb : nullptr);
  H.src[scen] = std::move(S);
  c->dirty = true;
  return PG_OK;
}

pg_status pg_set_pulses(pg_ctx* c, int32_t grid, int32_t scen, int32_t n_src, const int32_t* node,
                        const double* peak, const double* start, const double* width) {
  PG_TRY(check_gs(c, grid, scen));
  if (n_src < 0 || (n_src > 0 && (!node || !peak || !start || !width)))
    return set_err(c, PG_ERR_INVALID_ARG, "bad pulse arrays");
  std::vector<int32_t> off(n_src + 1);
  std::vector<double> t(3 * (size_t)n_src), i(3 * (size_t)n_src);
  for (int k = 0; k < n_src; ++k) {
    if (!(std::isfinite(width[k]) && width[k] > 0) || !std::isfinite(start[k]) || !std::isfinite(peak[k]))
      return set_err(c, PG_ERR_INVALID_ARG, "pulse %d: width must be > 0 and values finite", k);
    off[k] = 3 * k;
    const double half = 0.5 * width[k];
    t[3 * k] = start[k]; t[3 * k + 1] = start[k] + half; t[3 * k + 2] = start[k] + width[k];
    i[3 * k] = 0.0; i[3 * k + 1] = peak[k]; i[3 * k + 2] = 0.0;
  }
  off[n_src] = 3 * n_src;
  return pg_set_pwl(c, grid, scen, n_src, node, off.data(), t.data(), i.data());
}

pg_status pg_set_state(pg_ctx* c, int32_t grid, int32_t scen, const double* v, const double* i_l) {
  PG_TRY(check_gs(c, grid, scen));
  HIP_TRY(c, hipSetDevice(c->device));
  GridHost& H = c->grids[grid];
  if (v)
    for (int64_t k = 0; k < H.n; ++k)
      if (!std::isfinite(v[k])) return set_err(c, PG_ERR_INVALID_ARG, "v[%lld] is not finite", (long long)k);
  PG_TRY(prepare(c));
  PG_TRY(fill_v(c, H, v, scen, cur_vidx(c, H.item0 + scen)));
  const int ni = (int)H.ind_a.size();
  if (ni) {
    std::vector<double> buf(ni);
    for (int k = 0; k < ni; ++k) buf[k] = i_l ? H.ind_sign[k] * i_l[H.ind_branch[k]] : 0.0;
    HIP_TRY(c, hipMemcpy((double*)H.ind_i_d.p + (size_t)scen * ni, buf.data(), ni * sizeof(double),
                         hipMemcpyHostToDevice));
  }
  return PG_OK;
}

pg_status pg_reset(pg_ctx* c) {
  if (!c) return PG_ERR_INVALID_ARG;
  HIP_TRY(c, hipSetDevice(c->device));
  PG_TRY(prepare(c));
  for (int g = 0; g < (int)c->grids.size(); ++g)
    for (int s = 0; s < c->grids[g].S; ++s) PG_TRY(pg_set_state(c, g, s, nullptr, nullptr));
  PG_TRY(set_step(c, 0));
  PG_TRY(reset_stats_dev(c));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PG_OK;
}

namespace {

// With capacitors open, every connected part of a grid's conductance graph must reach a pad,
// or the DC matrix is singular.
bool dc_anchored(const GridHost& G) {
  if (G.kind) return G.form.dc_anchored;
  const int64_t n = G.n, plane = (int64_t)G.nx * G.ny;
  std::vector<int64_t> parent(n);
  for (int64_t i = 0; i < n; ++i) parent[i] = i;
  auto find = [&](int64_t i) {
    while (parent[i] != i) i = parent[i] = parent[parent[i]];
    return i;
  };
  auto unite = [&](int64_t a, int64_t b) { parent[find(a)] = find(b); };
  for (int l = 0; l < G.nl; ++l)
    for (int y = 0; y < G.ny; ++y)
      for (int x = 0; x < G.nx; ++x) {
        const int64_t i = (int64_t)l * plane + (int64_t)y * G.nx + x;
        if (x + 1 < G.nx && G.gE[((int64_t)l * G.ny + y) * (G.nx - 1) + x] > 0) unite(i, i + 1);
        if (y + 1 < G.ny && G.gN[((int64_t)l * (G.ny - 1) + y) * G.nx + x] > 0) unite(i, i + G.nx);
      }
  for (int32_t v : G.via_node) unite(v, v + plane);
  std::vector<char> ok(n, 0);
  for (int32_t p : G.pad_node) ok[find(p)] = 1;
  for (int64_t i = 0; i < n; ++i)
    if (!ok[find(i)]) return false;
  return true;
}

}  // namespace

pg_status pg_dc_operating_point(pg_ctx* c, int64_t k, double omega, double tol, int32_t max_sweeps) {
  if (!c) return PG_ERR_INVALID_ARG;
  if (k < 0 || !(std::isfinite(tol) && tol > 0) || max_sweeps < 1 || !(omega >= 0 && omega < 2))
    return set_err(c, PG_ERR_INVALID_ARG, "need k >= 0, tol > 0, max_sweeps >= 1 and 0 <= omega < 2");
  HIP_TRY(c, hipSetDevice(c->device));
  PG_TRY(sync_clock(c));
  PG_TRY(prepare(c));
  for (int g = 0; g < (int)c->grids.size(); ++g) {
    PG_TRY(ensure_host_values(c, c->grids[g]));
    if (!dc_anchored(c->grids[g]))
      return set_err(c, PG_ERR_NOT_SPD, "grid %d: a connected part reaches no pad, so the DC matrix is singular", g);
  }
  const pg_options saved = c->opt;
  const int64_t saved_step = c->step;
  const int saved_pred = c->pred_chunks;
  drop_graphs(c);
  c->dc_mode = true;
  pg_status st = PG_OK;
  for (int g = 0; g < (int)c->grids.size() && st == PG_OK; ++g) st = build_grid(c, g);
  if (omega > 0) c->opt.omega = omega;
  c->opt.tol = tol;
  c->opt.max_sweeps = max_sweeps;
  c->pred_chunks = 1;
  // the sources at t = k h: the step clock's next time is (step + 1) h
  if (st == PG_OK) st = set_step(c, k - 1);
  if (st == PG_OK) st = begin_step(c, -1);
  if (st == PG_OK) st = solve_active(c, tol);
  if (st == PG_OK) st = end_step(c, 0);  // branch currents g (v_a - v_b); no step, no statistics
  // back to the transient matrix, even after a failure
  c->dc_mode = false;
  c->opt = saved;
  c->pred_chunks = saved_pred;
  for (int g = 0; g < (int)c->grids.size(); ++g) {
    const pg_status s2 = build_grid(c, g);
    if (st == PG_OK) st = s2;
  }
  PG_TRY(st);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int32_t failed = 0;
  HIP_TRY(c, hipMemcpy(&failed, c->ctl.stat_failed, sizeof failed, hipMemcpyDeviceToHost));
  if (failed) {
    HIP_TRY(c, hipMemset(c->ctl.stat_failed, 0, sizeof(int32_t)));
    PG_TRY(set_step(c, saved_step));
    return set_err(c, PG_ERR_NO_CONVERGENCE, "the DC solve reached max_sweeps = %d with the residual above tol = %g",
                   max_sweeps, tol);
  }
  return set_step(c, k);
}

namespace {

// One item's vector utility (k_item_vec) on its own tiles.
pg_status item_vec(pg_ctx* c, int item, int op, int which, double scale) {
  const Tile* T = (const Tile*)c->tiles_all.p + c->item_tile_off[item];
  hipError_t e = launch_item_vec(fp32_mode(c), T, c->item_tile_cnt[item], c->tile_rows,
                                 (const GridDesc*)c->grid_desc.p, c->ctl, op, which, scale, c->stream);
  return e == hipSuccess ? PG_OK : set_err(c, PG_ERR_DEVICE, "vector kernel: %s", hipGetErrorString(e));
}

// max |d[which]| (op 1) or max |v| (op 4) over the item's mesh nodes.
pg_status item_absmax(pg_ctx* c, int item, int op, int which, double* out) {
  HIP_TRY(c, hipMemsetAsync((unsigned long long*)c->c_norm.p + item, 0, sizeof(unsigned long long), c->stream));
  PG_TRY(item_vec(c, item, op, which, 0.0));
  unsigned long long bits = 0;
  HIP_TRY(c, hipMemcpyAsync(&bits, (unsigned long long*)c->c_norm.p + item, sizeof bits, hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::memcpy(out, &bits, sizeof bits);
  return PG_OK;
}

// Activate one item (the others exit at once) without forming a right-hand side.
pg_status activate_only(pg_ctx* c, int item) {
  hipError_t e = launch_step_begin(c->ctl, n_items(c), item, c->opt.h, c->src_table, -1, -1, c->stream);
  return e == hipSuccess ? PG_OK : set_err(c, PG_ERR_DEVICE, "activation: %s", hipGetErrorString(e));
}

// kappa = ||M^-1 D||_inf of grid `grid` (coefficients built): x = M^-1 D 1 from x = 0 with
// b = diag(M); every entry of x is >= 1 and its maximum is the norm (M is an M-matrix, so
// M^-1 >= 0 entrywise).  The grid's first scenario's voltages are saved in `keep` (nstore
// device doubles) and restored; the stream is synchronised before returning.
pg_status bound_factor(pg_ctx* c, int grid, double rel_tol, double* kappa, double* keep) {
  GridHost& H = c->grids[grid];
  const int item = H.item0;
  PG_TRY(state_copy(c, item, keep, 1));
  const int saved_pred = c->pred_chunks;
  c->pred_chunks = 1;
  pg_status st = activate_only(c, item);
  if (st == PG_OK) st = item_vec(c, item, 3, 0, 0.0);
  if (st == PG_OK) st = solve_active(c, rel_tol);
  double k = 0.0;
  if (st == PG_OK) st = item_absmax(c, item, 4, 0, &k);
  c->pred_chunks = saved_pred;
  const pg_status s2 = state_copy(c, item, keep, 0);
  if (st == PG_OK) st = s2;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  PG_TRY(st);
  int32_t item_failed = 0;
  HIP_TRY(c, hipMemcpy(&item_failed, (int32_t*)c->c_failed.p + item, sizeof item_failed, hipMemcpyDeviceToHost));
  if (item_failed)
    return set_err(c, PG_ERR_NO_CONVERGENCE, "the solve for M^-1 D 1 reached max_sweeps = %d", c->opt.max_sweeps);
  *kappa = k;
  return PG_OK;
}

}  // namespace

pg_status pg_estimate_omega(pg_ctx* c, int32_t grid, int32_t dc, int32_t iters, double* rho, double* omega_opt) {
  PG_TRY(check_gs(c, grid, 0));
  PG_TRY(mesh_only(c, grid, "pg_estimate_omega"));
  if (iters < 32 || (dc != 0 && dc != 1) || !rho || !omega_opt)
    return set_err(c, PG_ERR_INVALID_ARG, "need iters >= 32, dc in {0, 1} and output pointers");
  HIP_TRY(c, hipSetDevice(c->device));
  PG_TRY(prepare(c));
  if (dc) PG_TRY(ensure_host_values(c, c->grids[grid]));
  if (dc && !dc_anchored(c->grids[grid]))
    return set_err(c, PG_ERR_NOT_SPD, "grid %d: a connected part reaches no pad, so the DC matrix is singular", grid);
  const int item = c->grids[grid].item0;
  drop_graphs(c);
  c->dc_mode = dc != 0;
  pg_status st = PG_OK;
  if (dc)
    for (int g = 0; g < (int)c->grids.size() && st == PG_OK; ++g) st = build_grid(c, g);
  // power iteration with the Jacobi operator J = D^-1 (D - M) (a weighted Jacobi sweep with
  // omega = 1 on M d = 0), renormalised every 16 applications; J^16 has the eigenvalues
  // lambda^16 >= 0, so the growth over a block estimates rho(J)^16 without the sign flips of
  // the +-lambda pairs of a bipartite graph
  const Tile* T = (const Tile*)c->tiles_sweep.p;
  double est = 0.0;
  if (st == PG_OK) st = activate_only(c, item);
  if (st == PG_OK) st = item_vec(c, item, 0, 0, 0.0);
  const int blocks = (iters + 15) / 16;
  for (int blk = 0; blk < blocks && st == PG_OK; ++blk) {
    for (int k = 0; k < 16 && st == PG_OK; ++k)
      for (auto& grp : c->tile_groups) {
        hipError_t e = launch_sweep(fp32_mode(c), grp.multi, PG_ORDER_JACOBI, grp.nl, c->tile_rows, T + grp.off,
                                    grp.count, (const GridDesc*)c->grid_desc.p, c->ctl, k & 1, 0, 1.0, c->stream);
        if (e != hipSuccess) st = set_err(c, PG_ERR_DEVICE, "Jacobi launch: %s", hipGetErrorString(e));
      }
    double nrm = 0.0;
    if (st == PG_OK) st = item_absmax(c, item, 1, 0, &nrm);  // 16 applications end in d[0]
    if (st != PG_OK) break;
    if (!(nrm > 0) || !std::isfinite(nrm)) { est = 0.0; break; }
    est = std::pow(nrm, 1.0 / 16.0);
    st = item_vec(c, item, 2, 0, 1.0 / nrm);
  }
  if (c->dc_mode) {
    c->dc_mode = false;
    for (int g = 0; g < (int)c->grids.size(); ++g) {
      const pg_status s2 = build_grid(c, g);
      if (st == PG_OK) st = s2;
    }
  }
  PG_TRY(st);
  *rho = est;
  *omega_opt = est < 1.0 ? 2.0 / (1.0 + std::sqrt(1.0 - est * est)) : 1.99;
  return PG_OK;
}

pg_status pg_error_bound_factor(pg_ctx* c, int32_t grid, double rel_tol, double* kappa) {
  PG_TRY(check_gs(c, grid, 0));
  PG_TRY(mesh_only(c, grid, "pg_error_bound_factor"));
  if (!(std::isfinite(rel_tol) && rel_tol > 0) || !kappa)
    return set_err(c, PG_ERR_INVALID_ARG, "need rel_tol > 0 and an output pointer");
  HIP_TRY(c, hipSetDevice(c->device));
  PG_TRY(prepare(c));
  DBuf keep;
  PG_TRY(dalloc(c, keep, (size_t)c->grids[grid].nstore * sizeof(double)));
  const pg_status st = bound_factor(c, grid, rel_tol, kappa, (double*)keep.p);
  dfree(keep);
  return st;
}

pg_status pg_error_bound_factor_noalloc(pg_ctx* c, int32_t grid, double rel_tol, double* kappa) {
  PG_TRY(check_gs(c, grid, 0));
  PG_TRY(mesh_only(c, grid, "pg_error_bound_factor_noalloc"));
  if (!(std::isfinite(rel_tol) && rel_tol > 0) || !kappa)
    return set_err(c, PG_ERR_INVALID_ARG, "need rel_tol > 0 and an output pointer");
  if ((size_t)c->grids[grid].nstore > kScratchDoubles)
    return set_err(c, PG_ERR_INVALID_ARG, "grid %d stores %lld node slots; the allocation-free variant holds at "
                   "most %zu (its device scratch is %zu MiB)", grid, (long long)c->grids[grid].nstore,
                   kScratchDoubles, kScratchDoubles * sizeof(double) >> 20);
  if (c->dirty)
    return set_err(c, PG_ERR_STATE, "the coefficients are not built yet: pg_step, pg_error_bound_factor or "
                   "pg_estimate_omega builds them (and allocates) first");
  if (!c->scratch_dev) return set_err(c, PG_ERR_DEVICE, "device scratch address was not resolved");
  HIP_TRY(c, hipSetDevice(c->device));
  // event timing would create events: off for the call
  const int saved_profile = c->profile_every;
  c->profile_every = 0;
  const pg_status st = bound_factor(c, grid, rel_tol, kappa, c->scratch_dev);
  c->profile_every = saved_profile;
  return st;
}

pg_status pg_step(pg_ctx* c, int32_t nsteps) { return pg_run_transient(c, nsteps, 1, 0, 0, nullptr); }

pg_status pg_run_transient(pg_ctx* c, int32_t nsteps, int32_t record_every, int32_t grid, int32_t scen,
                           double* out) {
  if (!c) return PG_ERR_INVALID_ARG;
  if (nsteps < 0 || record_every < 1) return set_err(c, PG_ERR_INVALID_ARG, "nsteps >= 0 and record_every >= 1 required");
  HIP_TRY(c, hipSetDevice(c->device));
  PG_TRY(sync_clock(c));
  PG_TRY(prepare(c));
  if (out) PG_TRY(check_gs(c, grid, scen));
  const auto t0 = std::chrono::steady_clock::now();
  int rec = 0;
  if (c->opt.resident) {  // one launch per call, or per recorded interval
    const int chunk = out ? record_every : std::max(1, nsteps);
    for (int k = 0; k < nsteps; k += chunk) {
      const int m = std::min(chunk, nsteps - k);
      PG_TRY(resident_steps(c, m));
      if (out && m == record_every) {
        PG_TRY(pg_read_voltages(c, grid, scen, out + (size_t)rec * c->grids[grid].n, c->grids[grid].n));
        ++rec;
      }
    }
  } else {
    // With the predictor the next step's opening overwrites v with its first iterate, so a step
    // whose voltages are recorded does not queue that opening ahead of the record's copy.
    auto ahead = [&](int k) {
      return k + 1 < nsteps && !(out && c->opt.predictor && (k + 1) % record_every == 0);
    };
    for (int k = 0; k < nsteps; ++k) {
      PG_TRY(one_step(c, ahead(k), ahead(k + 1)));
      if (out && ((k + 1) % record_every) == 0) {
        PG_TRY(pg_read_voltages(c, grid, scen, out + (size_t)rec * c->grids[grid].n, c->grids[grid].n));
        ++rec;
      }
    }
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int32_t failed = 0;
  HIP_TRY(c, hipMemcpy(&failed, c->ctl.stat_failed, sizeof failed, hipMemcpyDeviceToHost));
  if (failed) {
    HIP_TRY(c, hipMemsetAsync(c->ctl.stat_failed, 0, sizeof(int32_t), c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return set_err(c, PG_ERR_NO_CONVERGENCE, "a step reached max_sweeps = %d with the residual above tol = %g",
                   c->opt.max_sweeps, c->opt.tol);
  }
  return PG_OK;
}

pg_status pg_get_time(const pg_ctx* cc, int64_t* step) {
  if (!cc || !step) return PG_ERR_INVALID_ARG;
  pg_ctx* c = const_cast<pg_ctx*>(cc);
  PG_TRY(sync_clock(c));
  *step = c->step;
  return PG_OK;
}

pg_status pg_step_enqueue(pg_ctx* c, int32_t nsteps) {
  if (!c) return PG_ERR_INVALID_ARG;
  if (nsteps < 0) return set_err(c, PG_ERR_INVALID_ARG, "nsteps >= 0 required");
  if (!c->opt.resident)
    return set_err(c, PG_ERR_UNSUPPORTED, "pg_step_enqueue runs the resident path (pg_options.resident = 1)");
  if (c->dirty || c->grids.empty())
    return set_err(c, PG_ERR_STATE, "the coefficients are not built: one pg_step (or pg_run_transient) first");
  if (nsteps == 0) return PG_OK;
  int cur = -1;  // launches go to the context's device (setting the device is no stream operation)
  HIP_TRY(c, hipGetDevice(&cur));
  if (cur != c->device) HIP_TRY(c, hipSetDevice(c->device));
  ResidentArgs a = resident_args(c, nsteps);
  const hipError_t e = launch_resident(a, c->res_max_nodes, c->res_multi_layer, c->stream);
  if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "resident launch: %s", hipGetErrorString(e));
  c->clock_on_device = true;
  return PG_OK;
}

pg_status pg_set_time(pg_ctx* c, int64_t step) {
  if (!c || step < 0) return PG_ERR_INVALID_ARG;
  HIP_TRY(c, hipSetDevice(c->device));
  return set_step(c, step);
}

pg_status pg_num_grids(const pg_ctx* c, int32_t* count) {
  if (!c || !count) return PG_ERR_INVALID_ARG;
  *count = (int32_t)c->grids.size();
  return PG_OK;
}

pg_status pg_grid_info(const pg_ctx* c, int32_t grid, int32_t* nx, int32_t* ny, int32_t* nl, int32_t* n_scen,
                       int32_t* n_vias, int32_t* n_pads) {
  if (!c || grid < 0 || grid >= (int)c->grids.size()) return PG_ERR_INVALID_ARG;
  const GridHost& H = c->grids[grid];
  if (nx) *nx = H.nx;
  if (ny) *ny = H.ny;
  if (nl) *nl = H.nl;
  if (n_scen) *n_scen = H.S;
  if (n_vias) *n_vias = (int32_t)H.via_node.size();
  if (n_pads) *n_pads = (int32_t)H.pad_node.size();
  return PG_OK;
}

pg_status pg_read_voltages(pg_ctx* c, int32_t grid, int32_t scen, double* out, int64_t n) {
  PG_TRY(check_gs(c, grid, scen));
  GridHost& H = c->grids[grid];
  if (!out || n < H.n) return set_err(c, PG_ERR_INVALID_ARG, "output buffer too small (need %lld)", (long long)H.n);
  HIP_TRY(c, hipSetDevice(c->device));
  const int32_t vi = cur_vidx(c, H.item0 + scen);
  const double* src = (const double*)(vi ? H.v1.p : H.v0.p) + (size_t)scen * H.nstore;
  if (!H.kind && H.X == H.nx) {
    HIP_TRY(c, hipMemcpy(out, src, H.n * sizeof(double), hipMemcpyDeviceToHost));
    return PG_OK;
  }
  std::vector<double> buf((size_t)H.nstore);
  HIP_TRY(c, hipMemcpy(buf.data(), src, buf.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < H.n; ++i) out[i] = buf[(size_t)H.storage(i)];
  return PG_OK;
}

pg_status pg_read_voltages_dev(pg_ctx* c, int32_t grid, int32_t scen, double* dev_out, int64_t n) {
  PG_TRY(check_gs(c, grid, scen));
  GridHost& H = c->grids[grid];
  if (!dev_out || n < H.n) return set_err(c, PG_ERR_INVALID_ARG, "output buffer too small");
  if (!H.kind && H.X != H.nx)
    return set_err(c, PG_ERR_UNSUPPORTED, "device read needs nx to be a multiple of %d", kPitchAlign);
  HIP_TRY(c, hipSetDevice(c->device));
  PG_TRY(prepare(c));
  const int32_t vi = cur_vidx(c, H.item0 + scen);
  const double* src = (const double*)(vi ? H.v1.p : H.v0.p) + (size_t)scen * H.nstore;
  if (H.kind) {
    hipError_t e = launch_gather(src, (const int32_t*)H.slot_d.p, dev_out, H.n, c->stream);
    if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "gather launch: %s", hipGetErrorString(e));
    return PG_OK;
  }
  HIP_TRY(c, hipMemcpyAsync(dev_out, src, H.n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return PG_OK;
}

pg_status pg_read_inductor_currents(pg_ctx* c, int32_t grid, int32_t scen, double* out, int64_t n) {
  PG_TRY(check_gs(c, grid, scen));
  GridHost& H = c->grids[grid];
  const int64_t nb = n_branches(H);
  if ((!out && nb > 0) || n < nb) return set_err(c, PG_ERR_INVALID_ARG, "output buffer too small (need %lld)", (long long)nb);
  HIP_TRY(c, hipSetDevice(c->device));
  PG_TRY(prepare(c));
  std::fill(out, out + nb, 0.0);
  const int ni = (int)H.ind_a.size();
  if (!ni) return PG_OK;
  std::vector<double> buf(ni);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(buf.data(), (const double*)H.ind_i_d.p + (size_t)scen * ni, ni * sizeof(double),
                       hipMemcpyDeviceToHost));
  for (int k = 0; k < ni; ++k) out[H.ind_branch[k]] = H.ind_sign[k] * buf[k];
  return PG_OK;
}

pg_status pg_get_stats(const pg_ctx* cc, pg_stats* out) {
  if (!cc || !out) return PG_ERR_INVALID_ARG;
  pg_ctx* c = const_cast<pg_ctx*>(cc);
  HIP_TRY(c, hipSetDevice(c->device));
  PG_TRY(sync_clock(c));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  long long s64[3];
  int32_t s32[4];
  double sd[2];
  HIP_TRY(c, hipMemcpy(s64, c->c_stats64.p, sizeof s64, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(s32, c->c_stats32.p, sizeof(int32_t) * 3, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(sd, c->c_statsd.p, sizeof sd, hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof *out);
  out->steps = c->step;
  out->sweeps = s64[0];
  out->node_updates = s64[1];
  out->checks = s64[2];
  out->last_step_sweeps = s32[0];
  out->max_step_sweeps = s32[1];
  out->last_residual = sd[0];
  out->max_final_residual = sd[1];
  out->seconds = c->seconds;
  return PG_OK;
}

pg_status pg_reset_stats(pg_ctx* c) {
  if (!c) return PG_ERR_INVALID_ARG;
  HIP_TRY(c, hipSetDevice(c->device));
  PG_TRY(reset_stats_dev(c));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PG_OK;
}

pg_status pg_profile(pg_ctx* c, int32_t enable) {
  if (!c || enable < 0) return PG_ERR_INVALID_ARG;
  c->profile_every = enable;
  for (auto& n : c->prof_count) n = 0;
  return PG_OK;
}

pg_status pg_read_kernel_times(pg_ctx* c, pg_kernel_times* out) {
  if (!c || !out) return PG_ERR_INVALID_ARG;
  HIP_TRY(c, hipSetDevice(c->device));
  prof_drain(c);
  *out = c->prof_acc;
  std::memset(&c->prof_acc, 0, sizeof c->prof_acc);
  return PG_OK;
}

pg_status pg_loss_forward(pg_ctx* c, int32_t grid, int32_t scen, int32_t nsteps, int32_t ckpt_every,
                          double margin, double* J) {
  PG_TRY(check_gs(c, grid, scen));
  PG_TRY(mesh_only(c, grid, "the loss adjoint"));
  if (nsteps < 1 || ckpt_every < 1 || !std::isfinite(margin))
    return set_err(c, PG_ERR_INVALID_ARG, "need nsteps >= 1, ckpt_every >= 1 and a finite margin");
  HIP_TRY(c, hipSetDevice(c->device));
  PG_TRY(sync_clock(c));
  PG_TRY(prepare(c));
  GridHost& H = c->grids[grid];
  auto& A = c->adj;
  A.recorded = false;
  A.grid = grid; A.scen = scen; A.item = H.item0 + scen; A.K = nsteps; A.ckpt = std::min(ckpt_every, nsteps);
  A.nseg = (nsteps + A.ckpt - 1) / A.ckpt; A.margin = margin; A.k0 = c->step;
  const size_t ns = (size_t)H.nstore, nfull = ns * H.S;
  PG_TRY(dalloc(c, A.ckpts, (size_t)A.nseg * ns * sizeof(double)));
  PG_TRY(dalloc(c, A.vend, ns * sizeof(double)));
  PG_TRY(dalloc(c, A.seg, (size_t)(A.ckpt + 1) * ns * sizeof(double)));
  if (c->opt.predictor) {
    PG_TRY(dalloc(c, A.lamp, ns * sizeof(double)));
    PG_TRY(dalloc(c, A.lamq, ns * sizeof(double)));
  }
  PG_TRY(dalloc(c, A.lam0, nfull * sizeof(double)));
  PG_TRY(dalloc(c, A.lam1, nfull * sizeof(double)));
  PG_TRY(dalloc(c, A.arhs, nfull * sizeof(double)));
  PG_TRY(dalloc(c, A.dC, ns * sizeof(double)));
  PG_TRY(dalloc(c, A.dgE, ns * sizeof(double)));
  PG_TRY(dalloc(c, A.dgN, ns * sizeof(double)));
  {
    // branches: vias then pads (the order of the inductive-branch index ind_branch)
    const int nv = (int)H.via_node.size(), np = (int)H.pad_node.size();
    std::vector<int32_t> slot, ind(nv + np, -1);
    std::vector<double> g, L;
    for (int k = 0; k < nv; ++k) {
      slot.push_back((int32_t)H.storage(H.via_node[k])); g.push_back(H.via_g[k]);
      L.push_back(H.via_L.empty() ? 0.0 : H.via_L[k]);
    }
    for (int k = 0; k < np; ++k) {
      slot.push_back((int32_t)H.storage(H.pad_node[k])); g.push_back(H.pad_g[k]);
      L.push_back(H.pad_L.empty() ? 0.0 : H.pad_L[k]);
    }
    for (size_t k = 0; k < H.ind_branch.size(); ++k) ind[H.ind_branch[k]] = (int32_t)k;
    A.n_vias = nv;
    A.n_pads = np;
    A.n_ind = (int)H.ind_a.size();
    PG_TRY(upload(c, A.br_slot, slot)); PG_TRY(upload(c, A.br_ind, ind));
    PG_TRY(upload(c, A.br_g, g)); PG_TRY(upload(c, A.br_L, L));
    PG_TRY(dalloc(c, A.dbr_g, (size_t)(nv + np) * sizeof(double)));
    PG_TRY(dalloc(c, A.dbr_L, (size_t)(nv + np) * sizeof(double)));
    PG_TRY(dalloc(c, A.ickpts, (size_t)A.nseg * A.n_ind * sizeof(double)));
    PG_TRY(dalloc(c, A.iseg, (size_t)(A.ckpt + 1) * A.n_ind * sizeof(double)));
    PG_TRY(dalloc(c, A.iend, (size_t)A.n_ind * sizeof(double)));
    PG_TRY(dalloc(c, A.mu, (size_t)A.n_ind * sizeof(double)));
    A.branch_ready = false;
  }
  PG_TRY(dalloc(c, A.part, (size_t)std::max(1, c->item_tile_cnt[A.item]) * sizeof(double)));
  PG_TRY(dalloc(c, A.J, sizeof(double)));
  PG_TRY(dalloc(c, A.saved_vidx, sizeof(int32_t)));
  A.view = c->desc_host[grid];
  A.view.v[0] = (double*)A.lam0.p;
  A.view.v[1] = (double*)A.lam1.p;
  A.view.b = (double*)A.arhs.p;
  A.view.n_ind = 0;
  HIP_TRY(c, hipMemsetAsync(A.J.p, 0, sizeof(double), c->stream));
  const Tile* T = (const Tile*)c->tiles_all.p + c->item_tile_off[A.item];
  const int nt = c->item_tile_cnt[A.item];
  double* ck = (double*)A.ckpts.p;
  // the item's inductor currents travel with its voltages at every checkpoint
  const int ni = A.n_ind;
  const double* icur = (const double*)H.ind_i_d.p + (size_t)scen * ni;
  auto save_i = [&](void* dst) -> pg_status {
    if (ni) HIP_TRY(c, hipMemcpyAsync(dst, icur, ni * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return PG_OK;
  };
  PG_TRY(state_copy(c, A.item, ck, 1));
  PG_TRY(save_i(A.ickpts.p));
  const auto t0 = std::chrono::steady_clock::now();
  for (int k = 1; k <= nsteps; ++k) {
    PG_TRY(one_step(c));
    hipError_t e = launch_loss(T, nt, c->tile_rows, (const GridDesc*)c->grid_desc.p, c->ctl, margin,
                               (double*)A.part.p, (double*)A.J.p, c->stream);
    if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "loss launch: %s", hipGetErrorString(e));
    if (k % A.ckpt == 0 && k / A.ckpt < A.nseg) {
      PG_TRY(state_copy(c, A.item, ck + (size_t)(k / A.ckpt) * ns, 1));
      PG_TRY(save_i((double*)A.ickpts.p + (size_t)(k / A.ckpt) * ni));
    }
  }
  PG_TRY(state_copy(c, A.item, (double*)A.vend.p, 1));
  PG_TRY(save_i(A.iend.p));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (J) HIP_TRY(c, hipMemcpy(J, A.J.p, sizeof(double), hipMemcpyDeviceToHost));
  int32_t failed = 0;
  HIP_TRY(c, hipMemcpy(&failed, c->ctl.stat_failed, sizeof failed, hipMemcpyDeviceToHost));
  if (failed) {
    HIP_TRY(c, hipMemset(c->ctl.stat_failed, 0, sizeof(int32_t)));
    return set_err(c, PG_ERR_NO_CONVERGENCE, "a forward step reached max_sweeps");
  }
  A.recorded = true;
  return PG_OK;
}

pg_status pg_loss_backward(pg_ctx* c, double tol_adj, double* dJ_dC, double* dJ_dgE, double* dJ_dgN) {
  return loss_backward(c, tol_adj, dJ_dC, dJ_dgE, dJ_dgN, false);
}

pg_status pg_loss_backward_dev(pg_ctx* c, double tol_adj, double* dJ_dC, double* dJ_dgE, double* dJ_dgN) {
  return loss_backward(c, tol_adj, dJ_dC, dJ_dgE, dJ_dgN, true);
}

static pg_status loss_branch_outputs(pg_ctx* c, const DBuf& src, double* dvia, double* dpad, const char* what) {
  if (!c) return PG_ERR_INVALID_ARG;
  auto& A = c->adj;
  if (!A.recorded || !A.branch_ready) return set_err(c, PG_ERR_STATE, "%s needs a completed pg_loss_backward", what);
  if ((A.n_vias && !dvia) || (A.n_pads && !dpad)) return set_err(c, PG_ERR_INVALID_ARG, "gradient outputs are NULL");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (A.n_vias) HIP_TRY(c, hipMemcpy(dvia, src.p, A.n_vias * sizeof(double), hipMemcpyDeviceToHost));
  if (A.n_pads)
    HIP_TRY(c, hipMemcpy(dpad, (const double*)src.p + A.n_vias, A.n_pads * sizeof(double), hipMemcpyDeviceToHost));
  return PG_OK;
}

pg_status pg_loss_branch_gradients(pg_ctx* c, double* dJ_dvia_g, double* dJ_dpad_g) {
  return loss_branch_outputs(c, c ? c->adj.dbr_g : DBuf{}, dJ_dvia_g, dJ_dpad_g, "pg_loss_branch_gradients");
}

pg_status pg_loss_inductance_gradients(pg_ctx* c, double* dJ_dvia_L, double* dJ_dpad_L) {
  return loss_branch_outputs(c, c ? c->adj.dbr_L : DBuf{}, dJ_dvia_L, dJ_dpad_L, "pg_loss_inductance_gradients");
}

pg_status pg_update_mesh_values(pg_ctx* c, int32_t grid, const double* gE, const double* gN, const double* C) {
  PG_TRY(check_gs(c, grid, 0));
  PG_TRY(mesh_only(c, grid, "pg_update_mesh_values"));
  GridHost& H = c->grids[grid];
  const size_t nE = (size_t)H.nl * H.ny * (H.nx - 1), nN = (size_t)H.nl * (H.ny - 1) * H.nx, nC = (size_t)H.n;
  for (size_t k = 0; gE && k < nE; ++k)
    if (!(std::isfinite(gE[k]) && gE[k] >= 0)) return set_err(c, PG_ERR_INVALID_ARG, "gE[%zu] invalid", k);
  for (size_t k = 0; gN && k < nN; ++k)
    if (!(std::isfinite(gN[k]) && gN[k] >= 0)) return set_err(c, PG_ERR_INVALID_ARG, "gN[%zu] invalid", k);
  for (size_t k = 0; C && k < nC; ++k)
    if (!(std::isfinite(C[k]) && C[k] >= 0)) return set_err(c, PG_ERR_INVALID_ARG, "C[%zu] invalid", k);
  PG_TRY(ensure_host_values(c, H));  // arrays left out keep the values of an earlier device update
  if (gE) H.gE.assign(gE, gE + nE);
  if (gN) H.gN.assign(gN, gN + nN);
  if (C) H.C.assign(C, C + nC);
  H.raw_valid = false;
  c->dirty = true;
  c->adj.recorded = false;
  return PG_OK;
}

pg_status pg_update_mesh_values_dev(pg_ctx* c, int32_t grid, const double* gE, const double* gN, const double* C) {
  PG_TRY(check_gs(c, grid, 0));
  PG_TRY(mesh_only(c, grid, "pg_update_mesh_values_dev"));
  HIP_TRY(c, hipSetDevice(c->device));
  GridHost& H = c->grids[grid];
  const size_t nE = H.gE.size(), nN = H.gN.size(), nC = H.C.size();
  if (!H.raw_valid) {  // the device copies start from the current values
    PG_TRY(ensure_host_values(c, H));
    PG_TRY(upload(c, H.gE_raw, H.gE)); PG_TRY(upload(c, H.gN_raw, H.gN)); PG_TRY(upload(c, H.C_raw, H.C));
    H.raw_valid = true;
  }
  // check the new values where the caller left them, before anything is replaced
  PG_TRY(dalloc(c, H.chk_d, 16));
  struct { unsigned long long bad; unsigned int mask, pad; } chk{~0ull, 0u, 0u};
  HIP_TRY(c, hipMemcpyAsync(H.chk_d.p, &chk, sizeof chk, hipMemcpyHostToDevice, c->stream));
  unsigned long long* bad_d = (unsigned long long*)H.chk_d.p;
  unsigned int* mask_d = (unsigned int*)(bad_d + 1);
  hipError_t e = launch_mesh_check(gE, gN, C, H.nx, H.ny, H.nl, c->opt.h, bad_d, mask_d, c->stream);
  if (e == hipSuccess && !C)  // the layers with capacitance, from the values that stay
    e = launch_mesh_check(nullptr, nullptr, (const double*)H.C_raw.p, H.nx, H.ny, H.nl, c->opt.h, bad_d, mask_d,
                          c->stream);
  if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "value check: %s", hipGetErrorString(e));
  HIP_TRY(c, hipMemcpyAsync(&chk, H.chk_d.p, sizeof chk, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (chk.bad != ~0ull) {
    static const char* names[3] = {"gE", "gN", "C"};
    return set_err(c, PG_ERR_INVALID_ARG, "%s[%llu] is not finite and >= 0", names[std::min<unsigned>(2u, (unsigned)(chk.bad >> 40))],
                   chk.bad & ((1ull << 40) - 1));
  }
  if (gE) HIP_TRY(c, hipMemcpyAsync(H.gE_raw.p, gE, nE * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (gN) HIP_TRY(c, hipMemcpyAsync(H.gN_raw.p, gN, nN * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (C) HIP_TRY(c, hipMemcpyAsync(H.C_raw.p, C, nC * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));  // the caller may free or overwrite its arrays on return
  H.host_stale = true;
  c->adj.recorded = false;
  if (c->dirty || chk.mask != H.ch_layers) {
    // a rebuild is pending anyway, or the layers that carry C/h (which the kernels are told) change:
    // rebuild on the host from the new values at the next step
    PG_TRY(ensure_host_values(c, H));
    c->dirty = true;
    return PG_OK;
  }
  const bool f32 = fp32_mode(c);
  MeshCoefArgs a{};
  a.gE_raw = (const double*)H.gE_raw.p; a.gN_raw = (const double*)H.gN_raw.p; a.C_raw = (const double*)H.C_raw.p;
  a.gE64 = (double*)H.gE64.p; a.gN64 = (double*)H.gN64.p; a.ch64 = (double*)H.ch64.p; a.D64 = (double*)H.D64.p;
  a.gU64 = (const double*)H.gU64.p;
  a.gEs = H.gEs.p; a.gNs = H.gNs.p; a.invDs = H.invDs.p;
  a.fp32 = f32 ? 1 : 0;
  a.nx = H.nx; a.ny = H.ny; a.nl = H.nl; a.X = H.X;
  a.h = c->opt.h;
  e = launch_mesh_coef(a, c->stream);
  if (e == hipSuccess)
    e = launch_mesh_pads(H.n_padt, (const int32_t*)H.padt_slot_d.p, (const double*)H.padt_val_d.p, (double*)H.D64.p,
                         H.invDs.p, a.fp32, c->stream);
  if (e != hipSuccess) return set_err(c, PG_ERR_DEVICE, "coefficient rebuild: %s", hipGetErrorString(e));
  return PG_OK;
}

}  // extern "C"

// ---- autotuner ------------------------------------------------------------------------------
namespace {

struct Snapshot {
  std::vector<std::vector<double>> v, il;
  int64_t step = 0;
};

pg_status take_snapshot(pg_ctx* c, Snapshot& sn) {
  sn.v.clear();
  sn.il.clear();
  for (int g = 0; g < (int)c->grids.size(); ++g) {
    const GridHost& H = c->grids[g];
    const int64_t nb = n_branches(H);
    for (int s = 0; s < H.S; ++s) {
      sn.v.emplace_back(H.n);
      sn.il.emplace_back(std::max<int64_t>(nb, 1));
      PG_TRY(pg_read_voltages(c, g, s, sn.v.back().data(), H.n));
      PG_TRY(pg_read_inductor_currents(c, g, s, sn.il.back().data(), nb));
    }
  }
  sn.step = c->step;
  return PG_OK;
}

pg_status restore_snapshot(pg_ctx* c, const Snapshot& sn) {
  size_t k = 0;
  for (int g = 0; g < (int)c->grids.size(); ++g)
    for (int s = 0; s < c->grids[g].S; ++s, ++k) PG_TRY(pg_set_state(c, g, s, sn.v[k].data(), sn.il[k].data()));
  PG_TRY(set_step(c, sn.step));
  PG_TRY(reset_stats_dev(c));
  return PG_OK;
}

std::string tune_key(pg_ctx* c) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) arch = std::string(prop.gcnArchName).substr(0, 6);
  char buf[256];
  std::string key;
  for (auto& H : c->grids) {
    if (H.kind)
      std::snprintf(buf, sizeof buf, "graph%lldn%lldc%d*%d;", (long long)H.n, (long long)H.form.nnz, H.form.ncolors, H.S);
    else
      std::snprintf(buf, sizeof buf, "%dx%dx%d*%d;", H.nx, H.ny, H.nl, H.S);
    key += buf;
  }
  std::snprintf(buf, sizeof buf, "prec%d;h%.6g;tol%.3g;%s", c->opt.precision, c->opt.h, c->opt.tol, arch.c_str());
  return key + buf;
}

// The cache is a flat JSON object {"key": {"omega": w, "check_every": n, "tile_rows": r,
// "graphs": g, "sweeps_per_launch": f, "scen_block": b, "seconds": t}, ...} written and read
// only by this library.
bool cache_lookup(const char* path, const std::string& key, pg_options* o) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  std::string text;
  char buf[4096];
  size_t nread;
  while ((nread = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, nread);
  std::fclose(f);
  const std::string needle = "\"" + key + "\"";
  const size_t at = text.find(needle);
  if (at == std::string::npos) return false;
  const size_t end = text.find('}', at);
  const std::string entry = text.substr(at, end - at);
  auto num = [&](const char* name, double* out) {
    const size_t p = entry.find(std::string("\"") + name + "\"");
    if (p == std::string::npos) return false;
    const size_t colon = entry.find(':', p);
    *out = std::strtod(entry.c_str() + colon + 1, nullptr);
    return true;
  };
  double w, ce, tr, gr;
  if (!num("omega", &w) || !num("check_every", &ce) || !num("tile_rows", &tr) || !num("graphs", &gr)) return false;
  o->omega = w;
  o->check_every = (int32_t)ce;
  o->tile_rows = (int32_t)tr;
  o->graphs = (int32_t)gr;
  double spl = 0.0, blk = 0.0;
  o->sweeps_per_launch = num("sweeps_per_launch", &spl) ? (int32_t)spl : 0;
  o->scen_block = num("scen_block", &blk) ? (int32_t)blk : 0;
  return true;
}

void cache_store(const char* path, const std::string& key, const pg_options& o, double seconds) {
  if (!path) return;
  std::string text;
  if (FILE* f = std::fopen(path, "r")) {
    char buf[4096];
    size_t nread;
    while ((nread = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, nread);
    std::fclose(f);
  }
  char entry[512];
  std::snprintf(entry, sizeof entry,
                "\"%s\": {\"omega\": %.4f, \"check_every\": %d, \"tile_rows\": %d, \"graphs\": %d, "
                "\"sweeps_per_launch\": %d, \"scen_block\": %d, \"seconds\": %.6f}",
                key.c_str(), o.omega, o.check_every, o.tile_rows, o.graphs, o.sweeps_per_launch, o.scen_block,
                seconds);
  const std::string needle = "\"" + key + "\"";
  const size_t at = text.find(needle);
  if (at != std::string::npos) {
    const size_t end = text.find('}', at);
    text.replace(at, end + 1 - at, entry);
  } else {
    const size_t close = text.rfind('}');
    if (close == std::string::npos || text.find('{') == std::string::npos) {
      text = std::string("{\n  ") + entry + "\n}\n";
    } else {
      const bool empty = text.find('"') == std::string::npos;
      text.insert(close, std::string(empty ? "  " : ",\n  ") + entry + "\n");
    }
  }
  if (FILE* f = std::fopen(path, "w")) {
    std::fwrite(text.data(), 1, text.size(), f);
    std::fclose(f);
  }
}

}  // namespace

extern "C" pg_status pg_autotune(pg_ctx* c, int32_t nsteps, const char* cache_path, pg_options* chosen) {
  if (!c || nsteps < 1) return PG_ERR_INVALID_ARG;
  HIP_TRY(c, hipSetDevice(c->device));
  PG_TRY(prepare(c));
  const std::string key = tune_key(c);
  pg_options best = c->opt;
  if (cache_lookup(cache_path, key, &best)) {
    PG_TRY(pg_set_options(c, &best));
    if (chosen) *chosen = best;
    return PG_OK;
  }
  // report what runs: 0 sweeps per launch means the default, one
  if (best.sweeps_per_launch == 0) best.sweeps_per_launch = 1;
  Snapshot sn;
  PG_TRY(take_snapshot(c, sn));
  auto trial = [&](const pg_options& o, double* secs) -> pg_status {
    PG_TRY(pg_set_options(c, &o));
    PG_TRY(prepare(c));
    PG_TRY(restore_snapshot(c, sn));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const auto t0 = std::chrono::steady_clock::now();
    pg_status st = PG_OK;
    for (int k = 0; k < nsteps && st == PG_OK; ++k) st = one_step(c, k + 1 < nsteps, k + 2 < nsteps);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int32_t failed = 0;
    HIP_TRY(c, hipMemcpy(&failed, c->ctl.stat_failed, sizeof failed, hipMemcpyDeviceToHost));
    if (failed) HIP_TRY(c, hipMemset(c->ctl.stat_failed, 0, sizeof(int32_t)));
    if (st != PG_OK && st != PG_ERR_NO_CONVERGENCE) return st;
    *secs = (st == PG_OK && !failed) ? std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count()
                                     : 1e30;
    return PG_OK;
  };
  double best_t = 0.0;
  PG_TRY(trial(best, &best_t));
  const double omegas[] = {1.0, 1.2, 1.4, 1.5, 1.6, 1.7, 1.8, 1.85, 1.9, 1.95};
  const int checks[] = {4, 8, 12, 16, 24};
  const int rows[] = {4, 8, 16};
  for (double w : omegas) {
    pg_options o = best;
    o.omega = w;
    double t;
    PG_TRY(trial(o, &t));
    if (t < best_t) { best_t = t; best = o; }
  }
  for (int ce : checks) {
    pg_options o = best;
    o.check_every = ce;
    double t;
    PG_TRY(trial(o, &t));
    if (t < best_t) { best_t = t; best = o; }
  }
  for (int r : rows) {
    pg_options o = best;
    o.tile_rows = r;
    double t;
    PG_TRY(trial(o, &t));
    if (t < best_t) { best_t = t; best = o; }
  }
  for (int f : {1, 2, kTbSweeps}) {
    if (f == best.sweeps_per_launch || best.ordering != PG_ORDER_RED_BLACK) continue;
    pg_options o = best;
    o.sweeps_per_launch = f;
    double t;
    PG_TRY(trial(o, &t));
    if (t < best_t) { best_t = t; best = o; }
  }
  bool batched = false;
  for (auto& H : c->grids) batched = batched || H.S > 1;
  for (int b : {4, 8, 16}) {
    if (!batched) break;
    pg_options o = best;
    o.scen_block = b;
    double t;
    PG_TRY(trial(o, &t));
    if (t < best_t) { best_t = t; best = o; }
  }
  for (int g = 0; g <= 1; ++g) {
    pg_options o = best;
    o.graphs = g;
    double t;
    PG_TRY(trial(o, &t));
    if (t < best_t) { best_t = t; best = o; }
  }
  PG_TRY(pg_set_options(c, &best));
  PG_TRY(prepare(c));
  PG_TRY(restore_snapshot(c, sn));
  if (best_t < 1e29) cache_store(cache_path, key, best, best_t);
  if (chosen) *chosen = best;
  return best_t < 1e29 ? PG_OK : set_err(c, PG_ERR_NO_CONVERGENCE, "no candidate converged");
}
