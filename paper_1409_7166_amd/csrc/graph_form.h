// Host form of a general netlist (Sec. III, eqs. 4-9) for the gather-based sweep kernels:
// a colouring of the node graph, the node -> slot permutation and the sparsity pattern of M's
// off-diagonal part in sliced-ELL form (slices of 64 slots, one wavefront each).  Values stay
// per element kind, because M depends on the step h (C/h, inductor companions h/L).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/pgrid.h"

namespace pgrid {

constexpr int kSlice = 64;  // slots per sliced-ELL slice (one wavefront)

struct GraphForm {
  int32_t n = 0;                     // trivial nodes
  int32_t ncolors = 0;
  std::vector<int32_t> color;        // [n] colour of each trivial node
  std::vector<int64_t> cstart;       // [ncolors + 1] first slot of each colour (multiples of kSlice)
  std::vector<int32_t> slot;         // [n] node -> slot; slots inside a colour follow node order
  int64_t nslots = 0;                // cstart[ncolors]
  // sliced ELL over slots: the entries of slice s are [soff[s], soff[s+1]), column-major in the
  // slice (entry k of the slice's row j at soff[s] + k * kSlice + j); rows shorter than the
  // slice's widest row are padded with col = own slot and zero values
  std::vector<int32_t> soff;         // [nslots / kSlice + 1]
  std::vector<int32_t> col;          // neighbour slot
  std::vector<double> g;             // sum of the resistor conductances joining the pair, S
  std::vector<double> inv_l;         // sum of 1 / L over the inductors joining the pair, 1/H
  std::vector<double> cc;            // sum of the capacitors joining the pair, F
  int64_t nnz = 0;                   // off-diagonal pattern entries (both directions, no padding)
  // the pairs joined by a capacitor alone, as a second sliced-ELL table of the same layout
  // (most slices are empty), for the off-diagonal part of (C/h) v in the right-hand side
  std::vector<int32_t> csoff, ccol;
  std::vector<double> cval;          // F
  // per trivial node (node order)
  std::vector<double> c_diag;        // every capacitor at the node (to ground, a supply or a node), F
  std::vector<double> g_diag;        // every resistor at the node, S
  std::vector<double> b_res;         // sum of g * v_s over resistors to supplies, A
  // every inductor, for its branch current: near node, far node (-1: fixed at far_v), 1/L, and
  // the sign that turns the near -> far current into the netlist direction (from -> to)
  std::vector<int32_t> ind_near, ind_far;
  std::vector<double> ind_inv_l, ind_far_v;
  std::vector<int8_t> ind_sign;
  bool has_coupling = false;         // some capacitor joins two trivial nodes
  // with capacitors open, every group of nodes joined by resistors reaches a supply or ground
  // through a resistor (else the DC matrix is singular)
  bool dc_anchored = false;
};

// Validates (pg_validate_netlist) and builds the form; on failure writes a message.
__attribute__((visibility("hidden"))) pg_status build_graph_form(int32_t n, int32_t p, const double* source_v, int32_t m, const int32_t* from,
                           const int32_t* to, const uint8_t* kind, const double* value, GraphForm& out,
                           char* msg, size_t len);

// Adds a general-graph grid to the context (runtime); takes the form over.
__attribute__((visibility("hidden"))) pg_status upload_graph(pg_ctx* c, GraphForm& form, double vdd, int32_t n_scen, int32_t* grid_id);

}  // namespace pgrid
