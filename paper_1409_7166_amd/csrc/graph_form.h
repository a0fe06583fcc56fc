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
  std::vector<int32_t> slot;         // [n] node -> slot; slots inside a colour follow the
                                     // Cuthill-McKee order of the node graph
  int64_t nslots = 0;                // cstart[ncolors]
  // compact sliced ELL over slots: the entries of slice s are [soff[s], soff[s+1]), stored
  // entry by entry: first entry 0 of every row of the slice that has one, in slot order, then
  // entry 1 of every row that has more than one, and so on (a row's entries follow its
  // neighbour slots in increasing order).  No padding is stored: entry k of a row sits at
  // soff[s] + (the slice's entries before k) + (the number of rows before it in the slice with
  // more than k entries); rlen holds each slot's row length (0 for padding slots)
  std::vector<int32_t> soff;         // [nslots / kSlice + 1]
  std::vector<uint16_t> rlen;        // [nslots]
  std::vector<int32_t> col;          // neighbour slot
  std::vector<double> g;             // sum of the resistor conductances joining the pair, S
  std::vector<double> inv_l;         // sum of 1 / L over the inductors joining the pair, 1/H
  std::vector<double> cc;            // sum of the capacitors joining the pair, F
  int64_t nnz = 0;                   // off-diagonal pattern entries (both directions, no padding)
  // the pairs joined by a capacitor, as a second sliced-ELL table (most slices are empty), for
  // the off-diagonal part of (C/h) v in the right-hand side; this one is padded: entry k of the
  // slice's row j at csoff[s] + k * kSlice + j, rows shorter than the slice's widest padded with
  // col = own slot and zero values
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

constexpr int kMaxRowLen = 65535;  // neighbours of one node (rlen is 16-bit)

// Calls fn(entry, slot) for every entry of the compact neighbour table, in storage order.
template <typename Fn>
void for_each_entry(const GraphForm& f, Fn fn) {
  const int64_t nsl = (int64_t)f.soff.size() - 1;
  for (int64_t s = 0; s < nsl; ++s) {
    int64_t e = f.soff[s];
    for (int k = 0; e < f.soff[s + 1]; ++k)
      for (int j = 0; j < kSlice; ++j)
        if (k < f.rlen[s * kSlice + j]) fn(e++, s * kSlice + j);
  }
}

// Validates (pg_validate_netlist) and builds the form; on failure writes a message.
__attribute__((visibility("hidden"))) pg_status build_graph_form(int32_t n, int32_t p, const double* source_v, int32_t m, const int32_t* from,
                           const int32_t* to, const uint8_t* kind, const double* value, GraphForm& out,
                           char* msg, size_t len);

// Adds a general-graph grid to the context (runtime); takes the form over.
__attribute__((visibility("hidden"))) pg_status upload_graph(pg_ctx* c, GraphForm& form, double vdd, int32_t n_scen, int32_t* grid_id);

}  // namespace pgrid
