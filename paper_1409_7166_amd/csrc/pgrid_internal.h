// Internal declarations shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace pgrid {

constexpr int kTileX = 128;       // nodes per tile row: 64 lanes x one node pair
constexpr int kThreads = 256;     // threads per workgroup of the element-wise kernels
constexpr int kScenBlock = 8;     // scenarios per sweep/residual workgroup on multi-scenario grids
constexpr int kPitchAlign = 4;    // row pitch multiple (keeps pair and quad accesses aligned)

// Work items (tiles, chunks) are numbered in storage order.  Workgroups are dealt to the 8 XCDs
// round robin, so block b runs on XCD b % 8; give each XCD a contiguous run of work items so
// neighbouring ones (which re-read each other's halo or neighbour values) share that XCD's L2.
// Launch xcd_blocks(n) blocks.
__device__ __forceinline__ int xcd_tile(int ntiles) {
  const int per = (int)(gridDim.x / 8u);
  const int b = (int)blockIdx.x;
  const int t = (b % 8) * per + b / 8;
  return t < ntiles ? t : -1;
}
inline unsigned xcd_blocks(int ntiles) { return 8u * (unsigned)((ntiles + 7) / 8); }

// Device buffers reach the kernels as generic pointers (through the grid descriptors), and a
// load through a generic pointer is a flat load, which also counts against the scalar/LDS wait
// counter: every wait for a descriptor field or an LDS value would then drain the vector loads
// in flight as well.  These helpers address the global segment directly (every buffer they
// touch is device or host-mapped global memory), so the two counters stay apart.
#define PG_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T ld1(const T* __restrict__ p, int64_t i) {
  return ((const PG_GLOBAL T*)p)[i];
}
template <typename T>
__device__ __forceinline__ void st1(T* __restrict__ p, int64_t i, T v) {
  ((PG_GLOBAL T*)p)[i] = v;
}

// max that keeps a NaN (a diverged residual must never read as converged)
__device__ __forceinline__ double nan_max(double m, double x) {
  return (x > m || x != x) ? x : m;
}

// Raise a running maximum stored as the bits of a double >= 0 (NaN above +inf) to x >= 0.  The
// stored value only grows while a pass runs, so a workgroup whose x does not exceed what it reads
// skips the atomic: thousands of workgroups of one item would otherwise serialize on one word.
__device__ __forceinline__ void raise_max(unsigned long long* p, double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  if (b > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(p, b);
}

// Diagonal of M at a mesh node from the terms the residual pass has at hand: C/h, the six
// neighbour conductances (east, west, north, south, up, down; zero where absent) and the pad
// conductance, summed in this order without contraction, so the host (which stores M_ii) and the
// device (which forms it in the first pass of a step) get the same bits.
__host__ __device__ inline double mesh_diag(double ch, double e, double w, double n, double s, double u, double d,
                                            double pad) {
#pragma clang fp contract(off)
  return ((((((ch + e) + w) + n) + s) + u) + d) + pad;
}

// Per-grid device descriptor.  A layered mesh (kind 0) stores every per-node array with a row
// pitch X >= nx (a multiple of kPitchAlign): slot (l*ny + y)*X + x.  Coefficients are zero in
// the padding columns, at x = nx-1 (gE), y = ny-1 (gN), on the top layer (gU) and wherever no
// via exists; invD is zero in the padding, so padding corrections stay zero.  A general graph
// (kind 1, nx = nodes, ny = nl = 1) stores its nodes colour by colour, each colour padded to
// whole 64-slot slices, and M's off-diagonal part (w = -M_ij > 0) as a compact sliced-ELL
// neighbour table: slice s (64 slots, one wavefront) stores from sl_off[s] on entry 0 of each of
// its rows that has one, in slot order, then entry 1 of each row with more than one, and so on;
// sl_len holds the row lengths.  Its padding slots have D = invD = 0 and no entries.  A grid carries S current scenarios that
// share its coefficients; state arrays are scenario-major (scenario s occupies slots
// [s*nstore, (s+1)*nstore)), so one scenario is an ordinary contiguous field.
struct GridDesc {
  int32_t kind;                    // 0 layered mesh, 1 general graph
  int32_t nx, ny, nl, S;
  int32_t X;                       // row pitch
  int32_t item0;                   // control-block item of scenario 0 (item = item0 + s)
  int64_t nstore;                  // nl*ny*X storage slots per scenario
  // FP64 masters: conductances, diagonal of M, C/h, constant injection (pads x Vdd)
  const double* gE64;
  const double* gN64;
  const double* gU64;
  const double* D64;
  const double* ch64;
  const double* bconst64;
  // coefficient copies in the sweep precision (float or double)
  const void* gEs;
  const void* gNs;
  const void* gUs;
  const void* invDs;
  // state, S * nstore entries each
  double* v[2];                    // ping-pong FP64 voltages; ctl.vidx[item] selects the current one
  double* b;                       // right-hand side of the current step
  void* r;                         // residual b - M v at the last check (sweep precision)
  void* d[2];                      // correction ping-pong (sweep precision)
  // inductive branches (companion model); node-to-branch incidence in CSR form
  int32_t n_ind;
  const int32_t* ind_a;            // near slot
  const int32_t* ind_b;            // far slot, or -1 for the supply
  const double* ind_geq;
  const double* ind_alpha;
  double* ind_i;                   // [S][n_ind] branch currents
  const int32_t* inc_off;          // [nstore+1] (null when n_ind == 0)
  const int32_t* inc_ind;          // signed: k+1 if the slot is ind_a[k], -(k+1) if ind_b[k]
  const double* ind_vfar;          // far-end voltage of a branch with ind_b = -1 (null: vdd)
  double vdd;
  // layered mesh under pg_options.predictor: v(t-h) per scenario (same layout as v), else null;
  // v(t-2h) likewise under the quadratic predictor
  double* vhist;
  double* vhist2;
  // general graph: neighbour table (see above), and the table of the pairs joined by
  // capacitors, padded (entry k of slot i at cap_off[i/64] + 64 k + i%64, rows shorter than
  // their slice's widest padded with their own slot and zero), values C_ij / h; cap_off null
  // when there are none
  const int32_t* sl_off;
  const uint16_t* sl_len;
  const int32_t* sl_col;
  const double* sl_w64;
  const void* sl_ws;               // w in the sweep precision
  const int32_t* cap_off;
  const int32_t* cap_col;
  const double* cap_val;
  // three-level recurrence (general graphs): v(t-h) per scenario in vprev[k & 1] while step
  // k + 1 is opened (k = steps completed; the opening writes v(t) into vprev[(k + 1) & 1]), the
  // conductance part of M (diagonal incl. resistors to supplies and ground, and w's resistor
  // part per entry), and the constant injections of resistors (G0 v_s) and of inductors
  // (h/L v_s) to supplies
  double* vprev[2];
  const double* g3diag;
  const double* sl_g64;
  const double* bres64;
  const double* bl64;
  // general graph, the opening probe (k_graph_probe): per slot the constant q_i (FP64) and the
  // conductance gsup_i from the node to supplies and ground (FP32), per table entry the
  // conductance part of w (resistors and inductor companions, no capacitors; FP32)
  const double* gq64;
  const float* gsup32;
  const float* gw32;
  // coefficient words one sweep reads, in the sweep precision, and FP64 words one residual pass
  // reads (for the activity accounting of the decision)
  int64_t coef_words, resid_words;
  // layered mesh: bit l set if layer l has a non-zero C/h (ch_layers) or a non-zero constant
  // injection (bc_layers); layers without are neither read nor written as anything but zero
  uint32_t ch_layers, bc_layers;
};

// 256 consecutive slots of one scenario of a general-graph grid, all of one colour in the sweep
// lists; lim is the first slot of that colour (slots at or above it have not been updated yet
// in the current sweep).
struct GraphChunk {
  int32_t grid, item, scen, slot0, count, lim;
};
constexpr int kChunk = 256;

// One 128 x rows tile of one grid (all layers) for scenario `scen`, or, in the scenario-block
// lists used by the sweeps and residuals of multi-scenario grids, for scenarios
// scen .. scen + pad - 1 (items item .. item + pad - 1).
struct Tile {
  int32_t grid;
  int32_t item;                    // control-block item (grid, scenario)
  int32_t scen;
  int32_t x0;
  int32_t y0;
  int32_t pad;                     // scenarios in the block (1 outside scenario-block lists)
};

// Flattened current sources of every grid and scenario: first the n_always sources that are
// non-zero outside their breakpoints, then the windowed ones (zero before the first and after the
// last breakpoint) sorted by first breakpoint; win_t0 holds those first breakpoints and win_maxw
// the widest window, so a step only visits windowed sources with t0 in [t - win_maxw, t].
struct SourceTable {
  int32_t count;
  const int32_t* grid;
  const int32_t* index;            // scenario*nstore + slot within the grid's state arrays
  const int32_t* off;              // [count+1] into t / i
  const double* t;
  const double* i;
  int32_t n_always;
  int32_t n_window;
  const double* win_t0;            // [n_window]
  double win_maxw;
};

// Device-side control block.  An item is one scenario of one grid; every item converges on
// its own (per-item masks), and the decision is taken on the device so the host never has to
// read a residual before queueing the next refinement cycle.
struct Ctl {
  unsigned long long* norm_bits;   // [I] running max of the scaled residual (bits of a double >= 0)
  double* last_norm;               // [I]
  int32_t* active;                 // [I]
  int32_t* vidx;                   // [I]
  int32_t* step_sweeps;            // [I]
  int32_t* failed;                 // [I]
  int32_t* any_active;             // [nslots] host-visible flags, one per outstanding decision
  // [nslots][2] host-visible, beside each flag: the items left active by the decision, as
  // mesh nodes x scenarios (state words per sweep) and as the coefficient words of the grids
  // with at least one active item (each read once per sweep)
  long long* acct;
  // running statistics, updated once per step on the device
  long long* stat_sweeps;          // [1]
  long long* stat_updates;         // [1]
  long long* stat_checks;          // [1]
  int32_t* stat_last_sweeps;       // [1]
  int32_t* stat_max_sweeps;        // [1]
  double* stat_last_res;           // [1]
  double* stat_max_res;            // [1]
  int32_t* stat_failed;            // [1]
  const long long* nodes;          // [I] mesh nodes of the item's grid
  const int32_t* item_grid;        // [I] grid of the item
  // step clock: the step being solved advances on the device, so every launch of a step has
  // fixed arguments (and the step's launches can be replayed from a captured graph)
  long long* step;                 // [1] steps completed
  double* t_now;                   // [1] time of the step being solved, (step + 1) h
  int32_t* src_window;             // [2] first windowed source visited, number visited
  uint32_t* flag_seq;              // [1] decisions taken so far, modulo 2^32 (selects the flag slot)
  // [1] set by k_step_end when it finds items still iterating (the host queued the close of a
  // step, and the next step's opening, ahead of the step's last decision); every kernel of a
  // step's close and opening does nothing while it is set, until k_resume clears it
  int32_t* stall;
};

// Arguments of the decision after a residual pass.
struct DecideArgs {
  int on;
  int I;                           // items
  int G;                           // grids
  int has_d;                       // the pass added a correction (a refinement cycle ended)
  int nchk;                        // sweeps in the cycle
  int max_sweeps;
  int nslots;                      // host-visible flag slots
  double tol;
  const GridDesc* grids;
};

// ---- launch wrappers (kernels.hip) ----
// win_a >= 0: the source window [win_a, win_b) of the step being opened, found by the host;
// -1: searched on the device (launches replayed from graphs, or steps the host does not track)
hipError_t launch_step_begin(const Ctl& c, int G, int only_item, double h, const SourceTable& src, int win_a,
                             int win_b, hipStream_t s);
// predict: 0 none, 1 keep v in vhist, 2 also start the step from 2 v - vhist, 3 from
// 3 v - 3 vhist + vhist2 (k_rhs; vhist2, where present, takes the old vhist)
hipError_t launch_rhs(const Tile* tiles, int ntiles, int tile_rows, const GridDesc* grids,
                      const Ctl& c, hipStream_t s, int predict = 0);
// b -= sign * I(t_now + shift) at every source in the window of the step being opened
hipError_t launch_sources(const SourceTable& src, const GridDesc* grids, const Ctl& c, double shift, double sign,
                          hipStream_t s);
// multi: the tiles are scenario blocks (Tile.pad consecutive scenarios of one grid).
// fuse (single-scenario tiles, has_d = 0; the first pass of a step whose sources are all zero, so
// no k_rhs or k_sources launch precedes it): kFuseRhs forms the step's right-hand side as k_rhs
// would and stores it; with kFuseProbe it stores neither b nor r (a step expected to converge
// at once only needs the norm); with kFuseNoNorm it stores both and leaves the norm alone (the
// pass that follows a probe that found work).  kFuseCancelled with kFuseProbe (every mesh grid
// has a non-zero supply) takes the probe kernel, whose norm bounds the FP64 one from above;
// kFuseInd tells it that some grid carries inductors.
constexpr int kFuseRhs = 1, kFuseProbe = 2, kFuseNoNorm = 4, kFuseCancelled = 8, kFuseInd = 16;
hipError_t launch_resid(bool fp32, bool multi, int nl, int tile_rows, const Tile* tiles, int ntiles,
                        const GridDesc* grids, const Ctl& c, int has_d, int din, int fuse, hipStream_t s);
// The decision after a residual pass, with sequence number q = (*flag_seq)++, writes
// ((q & 0x1fffffff) << 2) | (skipped << 1) | (any item still active) to slot q & (nslots - 1) of
// c.any_active (host-visible memory; nslots is a power of two), after the slot's accounting
// words; `skipped` marks a
// decision that found the stall flag set and took no action.
// A step's close carried by a decision (on = 1): as launch_step_end's arguments.
struct CloseArgs {
  int on, count_step, begin_next, win_a, win_b;
  double h;
  SourceTable src;
};
hipError_t launch_decide(const Ctl& c, const DecideArgs& da, const CloseArgs& ca, hipStream_t s);
// Two red-black sweeps in one launch (tiles may be scenario blocks); reads d[din], writes d[din ^ 1].
hipError_t launch_sweep2(bool fp32, int nl, int tile_rows, const Tile* tiles, int ntiles, const GridDesc* grids,
                         const Ctl& c, int din, int zero_in, double omega, hipStream_t s);
hipError_t launch_sweep(bool fp32, bool multi, int ordering, int nl, int tile_rows, const Tile* tiles,
                        int ntiles, const GridDesc* grids, const Ctl& c, int din, int zero_in,
                        double omega, hipStream_t s);
// k = 2 or kTbSweeps red-black sweeps in one launch by temporal blocking (kernels_tb.hip), for
// the tile groups sweep_tb_supported accepts (ordering: 0 red-black); reads d[din], writes
// d[din ^ 1].
constexpr int kTbSweeps = 4;
bool sweep_tb_supported(bool fp32, bool multi, int ordering, int nl, int tile_rows, int k);
hipError_t launch_sweep_tb(bool fp32, int k, bool multi, int nl, int tile_rows, const Tile* tiles, int ntiles,
                           const GridDesc* grids, const Ctl& c, int din, int zero_in, double omega, hipStream_t s);
// count_step: 1 statistics and clock, 2 clock only, 0 neither; begin_next opens the next step.
hipError_t launch_step_end(const Ctl& c, int G, int count_step, int begin_next, double h, const SourceTable& src,
                           int win_a, int win_b, hipStream_t s);
// adjoint of the softplus loss (tiles of one item; vk, vprev and grads are plain slices)
hipError_t launch_loss(const Tile* tiles, int ntiles, int tile_rows, const GridDesc* grids, const Ctl& c,
                       double margin, double* part, double* total, hipStream_t s);
// adjoint right-hand side dJ/dv_k + (C/h) lambda_{k+1} (+ g_eq A^T mu_k over the nind inductive
// branches of the grid when nind > 0)
hipError_t launch_adj_rhs(const Tile* tiles, int ntiles, int tile_rows, const GridDesc* grids, const Ctl& c,
                          const double* vk, double margin, const double* mu, int nind, hipStream_t s);
// mu_k = alpha (mu_{k+1} - A lambda_{k+1}) for the grid's inductive branches
hipError_t launch_adj_mu(const GridDesc* grids, int grid, int item, int scen, const Ctl& c, double* mu, int nind,
                         hipStream_t s);
// the inductor update of one scenario of one grid
hipError_t launch_ind_update_item(const GridDesc* grids, int grid, int item, int scen, const Ctl& c, int nind,
                                  hipStream_t s);
hipError_t launch_adj_grad(const Tile* tiles, int ntiles, int tile_rows, const GridDesc* grids, const Ctl& c,
                           const double* vk, const double* vprev, double inv_h, double* dC, double* dgE,
                           double* dgN, hipStream_t s);
// conductance and inductance gradients of every via and pad at one reverse step (branches: vias
// then pads; br_ind: index among the grid's inductive branches or -1; P = layer stride)
hipError_t launch_adj_branch_grad(const GridDesc* grids, int grid, int item, int scen, const Ctl& c, const double* vk,
                                  const int32_t* br_slot, const int32_t* br_ind, const double* br_g,
                                  const double* br_L, int n_vias, int n_br, int64_t P, double h, const double* mu,
                                  const double* iprev, double* dg, double* dL, hipStream_t s);
hipError_t launch_state_copy(const Tile* tiles, int ntiles, int tile_rows, const GridDesc* grids, const Ctl& c,
                             double* buf, int to_buf, hipStream_t s);
// One item's vector utilities (op codes at k_item_vec); tiles are the item's tiles.
hipError_t launch_item_vec(bool fp32, const Tile* tiles, int ntiles, int tile_rows, const GridDesc* grids,
                           const Ctl& c, int op, int which, double s, hipStream_t st);
// Device rebuild of a layered mesh's coefficients from new unpadded values (row-major
// gE [nl][ny][nx-1], gN [nl][ny-1][nx], C [nl][ny][nx], device memory):
//  launch_mesh_check: every given array (null: skipped) must be finite and >= 0; the smallest
//    offending position (array 0, 1 or 2 above bit 40) lowers *bad (start it at ~0), and the
//    layers where C_raw / h is non-zero are OR-ed into *ch_mask (start it at 0).
//  launch_mesh_coef: from the three arrays and the grid's via conductances gU64, writes gE64,
//    gN64, ch64 = C/h, D64 = the diagonal without the pad term and 1/D64 (in invDs), and the
//    sweep-precision copies (gEs, gNs when fp32); padding columns are zero.
//  launch_mesh_pads: adds the pad term pad_val[k] to D64 at slot pad_slot[k] (distinct slots)
//    and rewrites its inverse, so D64 gets the bits of mesh_diag with that pad term.
struct MeshCoefArgs {
  const double* gE_raw;
  const double* gN_raw;
  const double* C_raw;
  double* gE64;
  double* gN64;
  double* ch64;
  double* D64;
  const double* gU64;
  void* gEs;
  void* gNs;
  void* invDs;
  int fp32;
  int nx, ny, nl, X;
  double h;
};
hipError_t launch_mesh_check(const double* gE, const double* gN, const double* C, int nx, int ny, int nl, double h,
                             unsigned long long* bad, unsigned int* ch_mask, hipStream_t s);
hipError_t launch_mesh_coef(const MeshCoefArgs& a, hipStream_t s);
hipError_t launch_mesh_pads(int n, const int32_t* pad_slot, const double* pad_val, double* D64, void* invDs, int fp32,
                            hipStream_t s);
// Resident path (pg_options.resident): one workgroup per item advances every item of the
// context (layered meshes of at most kResMaxNodes nodes and kResMaxInd series R-L branches)
// through nsteps whole backward-Euler steps in one launch, from the device clock's step, then
// advances the clock by nsteps (kernels only, no host interaction: the launch can be captured in
// a HIP graph and replayed).  item_src_off / item_src: the source-table entries of each item (CSR).  The
// statistics are folded into the control block (stat_last_* are reset first).
constexpr int kResMaxNodes = 4096;
constexpr int kResMaxInd = 2048;
struct ResidentArgs {
  const GridDesc* grids;
  const int32_t* item_grid;        // [I]
  const int32_t* vidx;             // [I] current voltage buffer of each item
  const int32_t* item_src_off;     // [I+1]
  const int32_t* item_src;
  const int32_t* src_index;        // the source table's target, offset and breakpoint arrays
  const int32_t* src_off;
  const double* src_t;
  const double* src_i;
  long long* stat_sweeps;          // the control block's statistics
  long long* stat_updates;
  long long* stat_checks;
  int32_t* stat_max_sweeps;
  int32_t* stat_last_sweeps;
  int32_t* stat_failed;
  double* stat_last_res;
  double* stat_max_res;
  long long* step;                 // the device clock (steps completed; read at the start)
  int n_items, nsteps, check_every, max_sweeps;
  double h, tol, omega;
};
hipError_t launch_resident(const ResidentArgs& a, int max_nodes, bool multi_layer, hipStream_t s);
// Clear the stall flag (after the host has re-queued a stalled step's remaining work).
hipError_t launch_resume(const Ctl& c, hipStream_t s);
// general graphs: right-hand side, one colour of a sweep (in place on d[0]), FP64 residual
// with v <- v + d[0] and its scaled norm, and the gather of one scenario's voltages into node order
// save_prev: also copy v into vprev (the first step of the three-level recurrence)
hipError_t launch_graph_rhs(const GraphChunk* ch, int n, const GridDesc* grids, const Ctl& c, int save_prev,
                            hipStream_t s);
// three-level right-hand side (eq. 11 / 14, sources added separately); then vprev <- v
hipError_t launch_graph_rhs3(const GraphChunk* ch, int n, const GridDesc* grids, const Ctl& c, hipStream_t s);
// b <- KCL residual at t_now without the sources (see pg_recurrence_drift); sources are added
// by launch_sources(shift 0, sign -1); then max |b_i| / M_ii into c.norm_bits[item]
hipError_t launch_graph_kcl(const GraphChunk* ch, int n, const GridDesc* grids, const Ctl& c, hipStream_t s);
hipError_t launch_graph_absmax_b(const GraphChunk* ch, int n, const GridDesc* grids, const Ctl& c, hipStream_t s);
hipError_t launch_graph_sweep(bool fp32, const GraphChunk* ch, int n, const GridDesc* grids, const Ctl& c,
                              int zero_in, double omega, hipStream_t s);
// norm = 0: the residual and v are stored but the norm is left alone (the pass that stores b and r
// after an opening probe found work, whose decision has already taken the norm)
hipError_t launch_graph_resid(bool fp32, const GraphChunk* ch, int n, const GridDesc* grids, const Ctl& c,
                              int has_d, hipStream_t s, int norm = 1);
// the opening probe of a step predicted to converge at once (sources all zero, two-level step):
// an upper bound of the FP64 scaled residual norm into c.norm_bits[item]; stores nothing
hipError_t launch_graph_probe(bool fp32, const GraphChunk* ch, int n, const GridDesc* grids, const Ctl& c,
                              hipStream_t s);
hipError_t launch_gather(const double* src, const int32_t* slot, double* dst, int64_t n, hipStream_t s);
hipError_t launch_swap_vidx(const Ctl& c, int item, int32_t* saved, hipStream_t s);
hipError_t launch_inductors(const GridDesc* grids, const int32_t* ind_grid,
                            const int32_t* ind_local, int n_total, const Ctl& c, hipStream_t s);

}  // namespace pgrid
