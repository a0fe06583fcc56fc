// Internal declarations shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace pgrid {

constexpr int kTileX = 128;       // nodes per tile row: 64 lanes x one node pair
constexpr int kThreads = 256;     // threads per workgroup of the element-wise kernels
constexpr int kPitchAlign = 4;    // row pitch multiple (keeps pair and quad accesses aligned)

// Per-grid device descriptor.  Every per-node array is stored with a row pitch X >= nx
// (a multiple of kPitchAlign): storage index (l*ny + y)*X + x.  Coefficients are zero in the
// padding columns, at x = nx-1 (gE), y = ny-1 (gN), on the top layer (gU) and wherever no via
// exists; invD is zero in the padding, so padding corrections stay zero.  State arrays hold
// nstore*S entries, scenario-minor (index storage*S + s).
struct GridDesc {
  int32_t nx, ny, nl, S;
  int32_t X;                       // row pitch
  int32_t pad_;
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
  // state
  double* v[2];                    // ping-pong FP64 voltages; ctl.vidx selects the current one
  double* b;                       // right-hand side of the current step
  void* r;                         // residual b - M v at the last check (sweep precision)
  void* d[2];                      // correction ping-pong (sweep precision)
  // inductive branches (companion model); node-to-branch incidence in CSR form
  int32_t n_ind;
  const int32_t* ind_a;            // near node
  const int32_t* ind_b;            // far node, or -1 for the supply
  const double* ind_geq;
  const double* ind_alpha;
  double* ind_i;                   // [n_ind][S] branch currents
  const int32_t* inc_off;          // [n+1] (null when n_ind == 0)
  const int32_t* inc_ind;          // signed: k+1 if the node is ind_a[k], -(k+1) if ind_b[k]
  double vdd;
};

// One 64 x rows tile of one grid (all layers, all scenarios).
struct Tile {
  int32_t grid;
  int32_t x0;
  int32_t y0;
  int32_t pad;
};

// Flattened current sources of every grid and scenario.
struct SourceTable {
  int32_t count;
  const int32_t* grid;
  const int32_t* index;            // node*S + scenario within the grid's state arrays
  const int32_t* off;              // [count+1] into t / i
  const double* t;
  const double* i;
};

// Device-side control block: per-grid convergence state, decided on the device so the
// host never has to read a residual before queueing the next refinement cycle.
struct Ctl {
  unsigned long long* norm_bits;   // [G] running max of the scaled residual (bits of a double >= 0)
  double* last_norm;               // [G]
  int32_t* active;                 // [G]
  int32_t* vidx;                   // [G]
  int32_t* step_sweeps;            // [G]
  int32_t* failed;                 // [G]
  int32_t* any_active;             // [1]
  // running statistics, updated once per step on the device
  long long* stat_sweeps;          // [1]
  long long* stat_updates;         // [1]
  long long* stat_checks;          // [1]
  int32_t* stat_last_sweeps;       // [1]
  int32_t* stat_max_sweeps;        // [1]
  double* stat_last_res;           // [1]
  double* stat_max_res;            // [1]
  int32_t* stat_failed;            // [1]
  const long long* nodes;          // [G] n*S
};

// ---- launch wrappers (kernels.hip) ----
hipError_t launch_step_begin(const Ctl& c, int G, hipStream_t s);
hipError_t launch_rhs(const Tile* tiles, int ntiles, int tile_rows, const GridDesc* grids,
                      const Ctl& c, hipStream_t s);
hipError_t launch_sources(const SourceTable& src, const GridDesc* grids, double t, hipStream_t s);
hipError_t launch_resid(bool fp32, int nl, int tile_rows, const Tile* tiles, int ntiles,
                        const GridDesc* grids, const Ctl& c, int has_d, int din, hipStream_t s);
hipError_t launch_decide(const Ctl& c, int G, double tol, int has_d, int nchk, int max_sweeps,
                         hipStream_t s);
hipError_t launch_sweep(bool fp32, int ordering, int nl, int tile_rows, const Tile* tiles,
                        int ntiles, const GridDesc* grids, const Ctl& c, int din, int zero_in,
                        double omega, hipStream_t s);
hipError_t launch_step_end(const Ctl& c, int G, hipStream_t s);
hipError_t launch_inductors(const GridDesc* grids, const int32_t* ind_grid,
                            const int32_t* ind_local, int n_total, const Ctl& c, hipStream_t s);

}  // namespace pgrid
