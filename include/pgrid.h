/*
 * pgrid.h - C ABI of the MI355X (gfx950) power-grid transient relaxation library.
 *
 * The library advances the backward-Euler transient of an on-chip power mesh
 * (Sec. II-A eqs. 1-3 for RC grids, Sec. III eqs. 9-10 for series R-L vias and
 * pads).  Every time step solves the symmetric positive definite nodal system
 * (Lemma 1)
 *     M v(t+h) = (C/h) v(t) + G0 Vdd - i(t+h) + [inductor history terms],
 *     M = C/h + G + G0 + [inductor companion conductances],
 * by topology-based relaxation sweeps (eqs. 15-17, Algorithm 1 with the SOR
 * blend of eq. 17), without assembling M.  The nodes are swept in red-black
 * order (colour = parity of x + y + layer); by Theorem 1 any sweep order of a
 * Gauss-Seidel/SOR iteration on an SPD matrix converges to the same solution.
 *
 * Conventions for every entry point:
 *  - Units are SI (S, F, H, s, A, V) and every value crossing the ABI is a
 *    double, whatever precision the sweeps use internally.
 *  - Host arrays are owned by the caller; the library copies what it keeps.
 *    Device pointers (the *_dev entry points) are also owned by the caller and
 *    must stay valid until the work queued on the context's stream completes.
 *  - Mesh node id = (layer * ny + y) * nx + x.  A grid may carry n_scen
 *    independent current scenarios that share its coefficients.
 *  - No exception crosses the ABI.  A negative return value is an error;
 *    pg_last_error() gives a message.  A context is used by one host thread
 *    at a time.
 *  - On PG_ERR_NO_CONVERGENCE the state holds the last iterate and the
 *    statistics are filled in.
 */
#ifndef PGRID_H
#define PGRID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PG_ABI_VERSION 1

typedef struct pg_ctx pg_ctx;

typedef enum pg_status {
  PG_OK = 0,
  PG_ERR_INVALID_ARG = -1,      /* bad pointer, size, NaN/negative value, option out of range */
  PG_ERR_TOPOLOGY = -2,         /* violates the topological assumptions 1-3 of Sec. III-B */
  PG_ERR_NOT_SPD = -3,          /* a connected component has neither a pad nor a capacitor, so M is singular */
  PG_ERR_NO_CONVERGENCE = -4,   /* a step reached max_sweeps with the residual above tol */
  PG_ERR_DEVICE = -5,           /* HIP runtime error or no usable gfx950 device */
  PG_ERR_OOM = -6,              /* device allocation failed */
  PG_ERR_STATE = -7,            /* call out of order (e.g. stepping before any grid was uploaded) */
  PG_ERR_UNSUPPORTED = -8       /* valid input this build does not handle */
} pg_status;

typedef enum pg_precision {
  PG_PREC_FP64 = 0,             /* sweeps, residual and state in FP64 */
  PG_PREC_FP32_REFINE = 1       /* FP32 correction sweeps, FP64 residual, state and refinement */
} pg_precision;

typedef enum pg_ordering {
  PG_ORDER_RED_BLACK = 0,       /* SOR in red-black order (eqs. 16-17) */
  PG_ORDER_JACOBI = 1           /* weighted Jacobi: every node from the previous sweep's values */
} pg_ordering;

typedef enum pg_recurrence {
  /* backward Euler with every inductor current kept as state (eq. 10, companion form) */
  PG_REC_TWO_LEVEL = 0,
  /* the three-level recurrence of eq. 11 / eq. 14 with the inductor currents eliminated:
   *   (C/h + G + hL) v(t+h) = (2C/h + G) v(t) - (C/h) v(t-h) - h L_s v_d - (I(t+h) - I(t)),
   * same matrix, so the same sweeps.  The first step after the state is set (upload, reset,
   * pg_set_state, pg_dc_operating_point, pg_set_time) is a two-level step, which supplies
   * v(t-h).  The recurrence has a root at 1 for solver error (each step's residual is carried
   * forward, not damped); pg_recurrence_drift measures what it has accumulated.  The inductor
   * currents are still updated (i(t+h) = i(t) + (h/L)(v_a - v_b)(t+h)) so they can be read.
   * General-netlist grids only, plain launches only (graphs = 0); PG_ERR_UNSUPPORTED
   * otherwise. */
  PG_REC_THREE_LEVEL = 1
} pg_recurrence;

/* Solver options (Algorithm 1 inputs h and tol; omega of eq. 17). */
typedef struct pg_options {
  double h;             /* backward-Euler step in seconds, > 0 */
  double tol;           /* stop a step when max_i |(b - M v)_i| / M_ii <= tol (volts), > 0 */
  double omega;         /* relaxation factor of eq. 17, 0 < omega < 2 */
  int32_t max_sweeps;   /* sweep budget per step per grid, >= 1 */
  int32_t check_every;  /* sweeps between FP64 residual checks (one refinement cycle), >= 1 */
  int32_t precision;    /* pg_precision */
  int32_t ordering;     /* pg_ordering */
  int32_t tile_rows;    /* rows per 128-node-wide sweep tile: 4, 8 or 16 (0 = library default, 8) */
  int32_t lookahead;    /* refinement cycles queued ahead of the host's convergence check, 0..4 */
  int32_t graphs;       /* 1: replay each step's launches from captured HIP graphs; 0: launch one by one */
  int32_t scen_block;   /* scenarios per sweep/residual workgroup on grids that carry several
                           scenarios (coefficients are loaded once per block): 1..16 (0 = 8) */
  int32_t sweeps_per_launch; /* red-black sweeps fused into one kernel launch: 1, 2 or 4 (0 = 1).
                           Fused sweeps stage the tile with a halo of 2 nodes per sweep and its
                           coefficients once and run the sweeps on chip (the scenarios of a
                           scenario block in turn), where the tile shape has the kernel: four
                           needs every tile group to have it (FP32: 1 layer with 4, 8 or 16 tile
                           rows, 2 layers with 4, or 8 without scenario blocks; FP64: 1 layer
                           without scenario blocks), else one sweep per launch; two (FP32: 1-4
                           layers, FP64: 1 layer or 2 with 4 rows) falls back per tile group to
                           recomputing the halo's rings from memory.  pg_sweep_launch_info tells
                           which runs.  A staged launch moves the bytes of about one sweep.
                           Results are identical.  Jacobi ordering always uses 1 */
  int32_t recurrence;   /* PG_REC_TWO_LEVEL (default) or PG_REC_THREE_LEVEL (general netlists only) */
  int32_t resident;     /* 1: pg_step / pg_run_transient advance every item in one launch per call
                           (per recorded interval), one workgroup per item carrying whole steps
                           (right-hand side, sources, sweeps, the stopping test of Algorithm 1 and
                           the branch currents) with the voltages in LDS, in FP64 whatever the
                           precision option; every grid must be a layered mesh of at most 4096
                           nodes and 2048 series R-L branches, with red-black ordering and the
                           two-level recurrence (PG_ERR_UNSUPPORTED otherwise, at the next step).
                           A step that reaches max_sweeps keeps its last iterate and the remaining
                           steps still run; the call then returns PG_ERR_NO_CONVERGENCE.
                           0 (default): one launch per sweep, decisions on the device. */
  int32_t predictor;    /* 0 (default): each step's iteration starts from the previous step's
                           voltages (Algorithm 1's V(s-1)); 1: layered meshes start it from the
                           linear extrapolation 2 V(s-1) - V(s-2) (from V(s-1) on the first step
                           after the state or the clock was set), which leaves the stopping test
                           and the converged solution unchanged and, on smooth stretches of a
                           transient, needs fewer sweeps; 2: from the quadratic extrapolation
                           3 V(s-1) - 3 V(s-2) + V(s-3) (the linear one on the second step after
                           a restart, V(s-1) on the first).  It keeps one (two for 2) more FP64
                           voltage arrays per scenario and forms every step's right-hand side in
                           its own pass (no opening probe).  Ignored by the resident path and by general
                           netlists.  In the adjoint's backward pass (pg_loss_backward*) the
                           recomputed steps of a segment start, from its second step on, from
                           the extrapolation of the two states before, and each adjoint solve
                           from 2 lambda(k+1) - lambda(k+2) (two more state arrays of the item,
                           allocated by pg_loss_forward when the option is on).  0, 1 or 2;
                           1 and 2 need graphs = 0 (else PG_ERR_UNSUPPORTED). */
} pg_options;

/* A layered RC/RLC mesh (the representative node of Fig. 2 repeated on a grid).
 * Array shapes are C-ordered.  Every conductance and capacitance must be finite and >= 0. */
typedef struct pg_mesh {
  int32_t nx, ny, nl;         /* nodes per row, rows per layer, layers; nx, ny >= 2, 1 <= nl <= 4 */
  const double* gE;           /* [nl][ny][nx-1] segment (l,y,x)-(l,y,x+1), S */
  const double* gN;           /* [nl][ny-1][nx] segment (l,y,x)-(l,y+1,x), S */
  const double* C;            /* [nl][ny][nx] node-to-ground capacitance, F */
  int32_t n_vias;
  const int32_t* via_node;    /* lower node (layer l < nl-1); the upper node is via_node + nx*ny */
  const double* via_g;        /* via conductance, S, > 0 */
  const double* via_L;        /* series inductance, H (NULL or 0: resistive via) */
  int32_t n_pads;
  const int32_t* pad_node;    /* node joined to the ideal supply */
  const double* pad_g;        /* pad conductance, S, > 0 */
  const double* pad_L;        /* series inductance, H (NULL or 0: resistive pad) */
  double vdd;                 /* supply voltage, V */
} pg_mesh;

typedef struct pg_stats {
  int64_t steps;              /* backward-Euler steps completed */
  int64_t sweeps;             /* sweeps summed over grids */
  int64_t node_updates;       /* sum over sweeps of active nodes x scenarios */
  int64_t checks;             /* residual passes (each followed by a decision) */
  int32_t last_step_sweeps;   /* max over grids, last step */
  int32_t max_step_sweeps;    /* max over steps and grids */
  /* The final scaled residual max_i |(b - M v)_i| / M_ii of a step, V.  For a step that
   * converged at its opening (no sweep), on a mesh with a non-zero supply or on a general
   * netlist (two-level recurrence), it is the opening probe's value: an upper bound of the
   * FP64 norm that exceeds it by at most its rounding term (single-precision arithmetic on
   * v - Vdd for meshes, on v_i minus the first supply and on neighbour differences for
   * netlists). */
  double last_residual;       /* max over grids, last step */
  double max_final_residual;  /* max over steps */
  double seconds;             /* wall time inside pg_step / pg_run_transient */
} pg_stats;

/* Kernel timing gathered with HIP events on the context stream while profiling is on
 * (pg_profile(ctx, k): the back-to-back sweep launches of a refinement cycle form one interval,
 * a residual pass over all tile groups another, and other launches one each; every k-th
 * interval of each kind is timed).  Launches queued after a step had converged (which exit at
 * once) are left out.
 * *_bytes are algorithmic bytes of the timed launches, charged for the (grid, scenario) items
 * that were still iterating (the rest exit at once): every array the kernel needs read once
 * and every array it produces written once, with e = 4 (FP32 sweeps) or 8 (FP64) bytes; sweeps
 * are charged one by one, so a launch that fuses k sweeps (sweeps_per_launch) is charged the
 * bytes of k one-sweep launches, although it moves about those of one.  Per
 * active node and scenario: sweep e * (r + d_new [+ d_old unless it starts from zero]),
 * residual 8 * (v + b) + e * r [+ e * d + 8 * v_out]; per mesh node of a grid with an active
 * scenario (coefficients are shared by the scenarios of a grid): sweep e * (gE + gN + invD)
 * + e * (nl-1)/nl (vias exist below the top layer only), residual 8 * (D + gE + gN)
 * + 8 * (nl-1)/nl; per storage slot of a general netlist with an active scenario, sweep e * invD
 * + 2 (its row length) and residual 8 * D + 2, and per off-diagonal entry of M (the table stores
 * no padding), sweep e * w + 4 (its column index) and residual 8 * w + 4. */
typedef struct pg_kernel_times {
  int64_t sweep_launches;  double sweep_ms;      int64_t sweep_node_updates;  double sweep_bytes;
  int64_t resid_launches;  double resid_ms;      int64_t resid_nodes;         double resid_bytes;
  int64_t rhs_launches;    double rhs_ms;
  int64_t other_launches;  double other_ms;
} pg_kernel_times;

int32_t pg_abi_version(void);
const char* pg_status_name(int32_t status);

/* Fill *out with the defaults: h = 10 ps, tol = 1e-6 V, omega = 1, max_sweeps = 10000,
 * check_every = 8, FP64, red-black, tile_rows = 8, lookahead = 1, graphs = 0, scen_block = 8,
 * sweeps_per_launch = 1. */
pg_status pg_default_options(pg_options* out);

/* Host-only checks (no device needed).  msg (may be NULL) receives a description of the
 * first problem found, truncated to msg_len bytes. */
pg_status pg_validate_options(const pg_options* opt, char* msg, size_t msg_len);

/* Checks array sizes and values, the via/pad indices, and Lemma 1's requirement that
 * every connected component of the mesh graph reaches a pad or holds a node with C > 0
 * (PG_ERR_NOT_SPD otherwise). */
pg_status pg_validate_mesh(const pg_mesh* mesh, char* msg, size_t msg_len);

/* General netlist check against the assumptions of Sec. III-B.  Nodes 0..n-1 are trivial
 * nodes, n..n+p-1 source nodes (supplies with grounded negative terminals), -1 is ground.
 * kind[e] is 'R' (value = conductance), 'C', 'L' or 'I'.  Returns PG_ERR_TOPOLOGY if a
 * trivial node has no non-source branch (assumption 2) or is linked to other nodes only
 * through current sources, PG_ERR_NOT_SPD if a group of trivial nodes connected through
 * trivial nodes (a sub-circuit in the sense of Fig. 1) has no capacitor, no branch to a
 * source node and no branch to ground, and PG_ERR_INVALID_ARG on bad indices or values. */
pg_status pg_validate_netlist(int32_t n, int32_t p, int32_t m, const int32_t* from,
                              const int32_t* to, const uint8_t* kind, const double* value,
                              char* msg, size_t msg_len);

/* The layered-mesh form of a netlist given as in pg_validate_netlist (Sec. III, eqs. 4-6; R values
 * are conductances).  mesh_dims = {nx, ny, nl}: trivial node (layer*ny + y)*nx + x is the mesh
 * node (x, y, layer) for the first nx*ny*nl trivial nodes; any further trivial node must be the
 * internal node of one series R-L branch (exactly one R and one L incident).  The mapping:
 *   R between in-layer neighbours          -> gE / gN segment (parallel resistors add),
 *   R between (x, y, l) and (x, y, l+1)     -> via (parallel resistors add),
 *   R from a mesh node to a source node     -> pad (parallel resistors add),
 *   R - internal node - L (either order) between vertical neighbours, or from a mesh node to a
 *   source node                             -> via / pad with series inductance,
 *   C from a mesh node to ground            -> node capacitance (parallel capacitors add),
 *   I from a mesh node to ground            -> marks a current-source position (waveforms come
 *                                              from pg_set_pwl / pg_set_pulses).
 * Vias come out sorted by lower node, pads by node; vdd is the common source voltage (0 when
 * p = 0).  Anything else (a resistor to ground or between non-neighbours, a capacitor between
 * two nodes, an inductor without its series resistor, sources at different voltages, an
 * inductive branch in parallel with another) is PG_ERR_UNSUPPORTED; the checks of
 * pg_validate_netlist come first.  Host-only.  pg_netlist_mesh_counts gives the via and pad
 * counts; pg_netlist_to_mesh fills caller arrays shaped as in pg_mesh. */
pg_status pg_netlist_mesh_counts(int32_t n, int32_t p, const double* source_v, int32_t m, const int32_t* from,
                                 const int32_t* to, const uint8_t* kind, const double* value,
                                 const int32_t* mesh_dims, int32_t* n_vias, int32_t* n_pads, char* msg,
                                 size_t msg_len);
pg_status pg_netlist_to_mesh(int32_t n, int32_t p, const double* source_v, int32_t m, const int32_t* from,
                             const int32_t* to, const uint8_t* kind, const double* value,
                             const int32_t* mesh_dims, double* gE, double* gN, double* C, int32_t* via_node,
                             double* via_g, double* via_L, int32_t* pad_node, double* pad_g, double* pad_L,
                             double* vdd, char* msg, size_t msg_len);

/* The colouring used for a general netlist (host only, no device): color[i] in 0..n_colors-1
 * for trivial node i, with no R, L or C branch joining two nodes of one colour (two colours when
 * the node graph is bipartite, else DSATUR refined by iterated greedy passes; should DSATUR need
 * more than 64 colours, the greedy colouring in node order), and the storage slot of
 * each node: colours in order, inside a colour the Cuthill-McKee order of the node graph
 * (breadth first from a pseudo-peripheral node of each connected part, the parts in the order
 * of their smallest node, a node's unvisited neighbours by increasing degree, ties by node),
 * each colour padded to a multiple of 64 slots (n_slots in all).  color and slot are caller arrays of n entries or NULL. */
pg_status pg_netlist_coloring(int32_t n, int32_t p, const double* source_v, int32_t m, const int32_t* from,
                              const int32_t* to, const uint8_t* kind, const double* value, int32_t* color,
                              int32_t* slot, int32_t* n_colors, int64_t* n_slots, char* msg, size_t msg_len);

/* Create a context on HIP device `device` (must be gfx950).  `stream` is a hipStream_t
 * (for instance torch.cuda.current_stream().cuda_stream) or NULL for a stream owned by
 * the context.  Every kernel and copy of the context runs on that stream. */
pg_status pg_create(pg_ctx** out, int32_t device, void* stream);
void pg_destroy(pg_ctx* ctx);
const char* pg_last_error(const pg_ctx* ctx);

pg_status pg_set_options(pg_ctx* ctx, const pg_options* opt);
pg_status pg_get_options(const pg_ctx* ctx, pg_options* out);

/* Upload a mesh (validated as by pg_validate_mesh) with n_scen >= 1 current scenarios.
 * Must precede the first step; options (h, precision) must be set before upload.
 * The state starts at v = vdd on every node and zero inductor current.  Returns the grid
 * id (0, 1, ...) in *grid_id.  All grids of a context advance together in time. */
pg_status pg_upload_mesh(pg_ctx* ctx, const pg_mesh* mesh, int32_t n_scen, int32_t* grid_id);

/* Upload a netlist (Sec. III branch form, as in pg_validate_netlist).
 * mesh_dims != NULL: through its layered-mesh form (pg_netlist_to_mesh), then as pg_upload_mesh;
 * errors as in pg_netlist_to_mesh.
 * mesh_dims == NULL: as a general graph (any topology the checks of pg_validate_netlist accept),
 * swept by the colour-ordered kernels: the trivial nodes are coloured (pg_netlist_coloring) and
 * one sweep updates the colours in order (eqs. 16-17; Theorem 1 covers any order).  Element
 * rules (eqs. 8-11, inductor current kept as state): R to a supply or ground and C to a supply or
 * ground act on the diagonal (a supply's voltage enters the right-hand side); C between two
 * trivial nodes is a coupling capacitor (an off-diagonal term of C/h in M and in the right-hand
 * side); every L is a pure inductor with companion g = h/L, alpha = 1 (a series R-L branch is
 * its R and L through an internal trivial node); I branches only mark positions, the waveforms
 * come from pg_set_pwl / pg_set_pulses with node = trivial node (current drawn to ground).  The
 * state starts at v = source_v[0] (0 if p = 0).  Inductor currents (pg_read_inductor_currents,
 * pg_set_state) are per L branch in netlist order, positive from `from` to `to`.  Built for
 * such grids: stepping, pg_run_transient, reads, pg_set_state, graphs and scenarios, and
 * pg_dc_operating_point when the grid has no inductor; pg_estimate_omega,
 * pg_error_bound_factor, the loss adjoint and pg_update_mesh_values return
 * PG_ERR_UNSUPPORTED, as does the Jacobi ordering.
 * Errors are reported with the message in pg_last_error. */
pg_status pg_upload_netlist(pg_ctx* ctx, int32_t n, int32_t p, const double* source_v, int32_t m,
                            const int32_t* from, const int32_t* to, const uint8_t* kind, const double* value,
                            const int32_t* mesh_dims, int32_t n_scen, int32_t* grid_id);

/* Replace the current sources of one scenario by triangular pulses (one per node, nodes
 * unique): i(t) = peak * max(0, 1 - |t - (start + width/2)| / (width/2)), width > 0. */
pg_status pg_set_pulses(pg_ctx* ctx, int32_t grid, int32_t scen, int32_t n_src,
                        const int32_t* node, const double* peak, const double* start,
                        const double* width);

/* Replace the current sources of one scenario by piecewise-linear waveforms (Sec. II-A):
 * source k draws, at node[k], the current interpolated through the breakpoints
 * (t[j], i[j]) for j in offsets[k] .. offsets[k+1]-1 (t strictly increasing, at least one
 * breakpoint), held constant before the first and after the last breakpoint. */
pg_status pg_set_pwl(pg_ctx* ctx, int32_t grid, int32_t scen, int32_t n_src,
                     const int32_t* node, const int32_t* offsets, const double* t,
                     const double* i);

/* Set the state of one scenario: v (n doubles; NULL = vdd everywhere) and the inductor
 * currents (n_vias + n_pads doubles in via-then-pad order, entries of resistive branches
 * ignored; NULL = 0).  Does not change the time index. */
pg_status pg_set_state(pg_ctx* ctx, int32_t grid, int32_t scen, const double* v, const double* i_l);

/* Back to t = 0: every state to v = vdd, zero inductor currents; statistics cleared. */
pg_status pg_reset(pg_ctx* ctx);

/* DC operating point with the sources at time index k (t = k h; Sec. II-A eq. 3 with the
 * capacitors open, and each series R-L branch reduced to its resistor since an inductor is a
 * short at DC), solved for every grid and scenario by the same relaxation sweeps from the
 * current state, with the given omega (0: the context's; the DC matrix is worse conditioned
 * than a step's, so its best omega is larger), tol and max_sweeps.  Sets every state to the DC
 * voltages and branch currents i = g (v_a - v_b), and the time index to k, so that pg_step
 * continues the transient from that operating point (the initial-condition recipe with
 * non-zero loads at the start).  PG_ERR_NOT_SPD if a connected part of a grid reaches no pad
 * (the DC matrix is singular); PG_ERR_NO_CONVERGENCE leaves the last iterate as the state and
 * the time index unchanged. */
pg_status pg_dc_operating_point(pg_ctx* ctx, int64_t k, double omega, double tol, int32_t max_sweeps);

/* Spectral radius rho of the Jacobi iteration matrix I - D^-1 M of grid `grid`'s step matrix
 * (dc = 1: of its DC matrix), by `iters` (>= 32, rounded up to a multiple of 16) power
 * iterations of a Jacobi sweep on the device, and Young's optimal relaxation factor for the
 * red-black ordering, omega_opt = 2 / (1 + sqrt(1 - rho^2)) (eq. 17's omega; the mesh graph
 * is bipartite, so the red-black ordered matrix is consistently ordered).  The estimate is the
 * growth of the max-norm over the last 16 applications; its error falls like the ratio of the
 * two largest eigenvalue magnitudes to the power of the iteration count.  The grid's correction
 * buffers are overwritten (the state is not).  PG_ERR_NOT_SPD for dc = 1 as in
 * pg_dc_operating_point. */
pg_status pg_estimate_omega(pg_ctx* ctx, int32_t grid, int32_t dc, int32_t iters, double* rho,
                            double* omega_opt);

/* Error-bound factor kappa = ||M^-1 D||_inf of grid `grid`'s step matrix (D its diagonal),
 * computed as max_i x_i of the solution of M x = D 1 (M is an M-matrix, so M^-1 >= 0) by the
 * relaxation sweeps to a scaled residual of rel_tol (so kappa carries a relative error of
 * about rel_tol * kappa).  A step stopped at a scaled residual max_i |r_i| / M_ii <= tol is
 * within kappa * tol volts of the exact backward-Euler solution, so tol = err / kappa asks for
 * a voltage error err (the adaptive tolerance).  The state of the grid is restored. */
pg_status pg_error_bound_factor(pg_ctx* ctx, int32_t grid, double rel_tol, double* kappa);

/* pg_error_bound_factor for callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): same arguments, kernels and result, but the grid's state is
 * saved in a fixed device scratch array of 2^22 doubles (32 MiB) that the library holds on every
 * GPU it runs on until the process ends, instead of a buffer allocated per call; the call makes no
 * hipMalloc/hipFree and creates no events (kernel timing is suspended for it).  Errors:
 * PG_ERR_INVALID_ARG when the grid stores more than 2^22 node slots (nl * ny * nx rounded up to
 * the row pitch), PG_ERR_STATE when the coefficients still have to be built (after upload or a
 * change of options or values: pg_step, pg_error_bound_factor or pg_estimate_omega builds them),
 * otherwise as pg_error_bound_factor.  All contexts on one GPU share its scratch array: calls on
 * one GPU that overlap in time (contexts driven from different host threads) race, and must be
 * serialised by the caller.  The call synchronises the context's stream. */
pg_status pg_error_bound_factor_noalloc(pg_ctx* ctx, int32_t grid, double rel_tol, double* kappa);

/* Advance every grid and scenario by nsteps backward-Euler steps (Algorithm 1 loop:
 * warm start from the previous step, sweep until the scaled residual is <= tol). */
pg_status pg_step(pg_ctx* ctx, int32_t nsteps);

/* Queue nsteps backward-Euler steps of every grid and scenario on the context's stream and return
 * at once (the resident path, pg_options.resident = 1): three kernel launches, no host wait, no
 * allocation and no host-visible memory, so a caller can capture the call in a HIP graph (stream
 * capture on the context's stream, e.g. torch.cuda.graph) and replay it.  Each launch starts
 * from the step count on the device and advances it, so every replay continues the transient
 * (the sources are evaluated at the device's time).  The host's step count is refreshed from
 * the device, after waiting for the context's stream, by the next pg_step, pg_run_transient,
 * pg_get_time, pg_get_stats, pg_loss_forward or pg_dc_operating_point (replays on another stream
 * must be synchronised by the caller first); a step of an enqueued launch that reached
 * max_sweeps is reported by the next pg_step or pg_run_transient as PG_ERR_NO_CONVERGENCE.
 * PG_ERR_UNSUPPORTED unless resident = 1; PG_ERR_STATE while the coefficients still have to be
 * built (after upload or a change of options: one pg_step builds them). */
pg_status pg_step_enqueue(pg_ctx* ctx, int32_t nsteps);

/* pg_step(nsteps) that also copies the voltages of (grid, scen) to out after every
 * record_every-th step: out holds floor(nsteps / record_every) * n doubles (may be NULL). */
pg_status pg_run_transient(pg_ctx* ctx, int32_t nsteps, int32_t record_every, int32_t grid,
                           int32_t scen, double* out);

/* Current step index k (time t = k h); pg_set_time moves the clock without touching the state. */
pg_status pg_get_time(const pg_ctx* ctx, int64_t* step);
pg_status pg_set_time(pg_ctx* ctx, int64_t step);

/* Number of uploaded grids, and the sizes of one (any output pointer may be NULL). */
pg_status pg_num_grids(const pg_ctx* ctx, int32_t* count);
pg_status pg_grid_info(const pg_ctx* ctx, int32_t grid, int32_t* nx, int32_t* ny, int32_t* nl, int32_t* n_scen,
                       int32_t* n_vias, int32_t* n_pads);

/* Autotuner: times `nsteps` steps from the current state for candidate settings (omega, sweeps
 * per residual check, tile rows, sweeps per launch, scenario block size when a grid carries
 * several scenarios, graph replay), by coordinate descent from the current options,
 * restoring the state and clock after every trial, and sets the fastest.  The winner is cached in
 * the JSON file `cache_path` (may be NULL: no cache) under a key built from the grid shapes,
 * scenario counts, precision, h, tolerance and the GPU architecture; a cached entry is applied
 * without timing.  *chosen (may be NULL) receives the options set. */
pg_status pg_autotune(pg_ctx* ctx, int32_t nsteps, const char* cache_path, pg_options* chosen);

/* How the mesh sweeps run under the current options (the context's device data are built first if
 * the grids or options changed, as pg_step does): *sweeps_per_launch receives the sweeps each
 * mesh sweep launch performs (1, 2 or 4: four only where every tile group has the four-sweep
 * kernel, else one), *staged 1 if every fused launch stages its tiles once and sweeps on chip,
 * 0 if some recompute halo rings from memory or the sweeps run one per launch. */
pg_status pg_sweep_launch_info(pg_ctx* ctx, int32_t* sweeps_per_launch, int32_t* staged);

/* Size of a general-netlist grid: trivial nodes, colours, storage slots, off-diagonal entries
 * of M (both directions) and L branches.  PG_ERR_INVALID_ARG for a mesh grid. */
pg_status pg_graph_info(const pg_ctx* ctx, int32_t grid, int32_t* n_nodes, int32_t* n_colors, int64_t* n_slots,
                        int64_t* nnz, int32_t* n_inductors);

/* Copy the node voltages (n doubles) or inductor currents of one scenario to host memory
 * (blocking) or to device memory (queued on the context stream).  Inductor currents of a mesh:
 * n_vias + n_pads doubles, via then pad order, zero for resistive branches; of a general
 * netlist: one per L branch in netlist order. */
/* Under PG_REC_THREE_LEVEL, after at least one step: the Jacobi-scaled residual of Kirchhoff's
 * current law at the current time t_k with the backward-Euler capacitor currents and the
 * inductor currents the library keeps updating,
 *   max_i |C (v_k - v_{k-1})/h + G v_k + G_s v_d + A_l^T i_k + A_i^T I(t_k)|_i / M_ii   (volts),
 * for (grid, scen).  Under the two-level recurrence this would be the step's own residual (at most
 * tol); under the three-level one it also holds the solver error the recurrence has carried
 * forward.  Queued on the context stream and waited for; PG_ERR_STATE before a three-level step
 * or under the two-level recurrence. */
pg_status pg_recurrence_drift(pg_ctx* ctx, int32_t grid, int32_t scen, double* drift);
pg_status pg_read_voltages(pg_ctx* ctx, int32_t grid, int32_t scen, double* out, int64_t n);
pg_status pg_read_voltages_dev(pg_ctx* ctx, int32_t grid, int32_t scen, double* dev_out, int64_t n);
pg_status pg_read_inductor_currents(pg_ctx* ctx, int32_t grid, int32_t scen, double* out, int64_t n);

/* Replace the conductances and capacitances of an uploaded grid (same shapes as in pg_mesh;
 * a NULL array is left unchanged).  Topology, pads, vias, sources and state are kept; the
 * coefficients are rebuilt before the next step. */
pg_status pg_update_mesh_values(pg_ctx* ctx, int32_t grid, const double* gE, const double* gN,
                                const double* C);

/* pg_update_mesh_values with the new values in device memory (for instance the data of torch
 * tensors that an optimiser updates): gE, gN, C are device pointers laid out as in pg_mesh, read
 * on the context's stream (any may be NULL: unchanged) and copied before the call returns; the
 * caller keeps ownership.  The values are checked on the device (finite and >= 0, as in
 * pg_validate_mesh; the anchoring of Lemma 1 is not checked again) and, once the coefficients of
 * the grid are built, its FP64 and sweep-precision coefficient arrays (M's diagonal with the
 * unchanged vias and pads included) are rebuilt by kernels, with the bits the host build gives;
 * nothing crosses PCIe except a status word.  If a rebuild is pending anyway, or the set of layers
 * with non-zero C changes, the values are copied to the host and the next step rebuilds there.
 * Errors: PG_ERR_INVALID_ARG naming the first offending entry (nothing is changed). */
pg_status pg_update_mesh_values_dev(pg_ctx* ctx, int32_t grid, const double* gE, const double* gN, const double* C);

/* Voltage-drop loss of a backward-Euler transient and its gradient by the reverse-time adjoint
 * (mesh grids, RC or with series R-L vias and pads; PG_ERR_UNSUPPORTED for general netlists).
 * From the current state at step k0, pg_loss_forward advances the whole context by nsteps
 * steps (as pg_step) and returns
 *     J = sum_{k=1..nsteps} sum_i softplus(Vdd - v_i(t_{k0+k}) - margin)^2,
 * keeping the state of (grid, scen) (voltages and inductor currents) every ckpt_every steps
 * (FP64, on the device).  pg_loss_backward then solves, for k = nsteps .. 1, the adjoint of the
 * BE recurrence of eq. 2 / eq. 10 (companion form: i_k = alpha i_{k-1} + g_eq (A v_k - v_far)),
 *     mu_k = alpha (mu_{k+1} - A lambda_{k+1}),
 *     M lambda_k = dJ/dv_k + (C/h) lambda_{k+1} + g_eq A^T mu_k,  lambda_{nsteps+1} = mu_{nsteps+1} = 0,
 * with the same relaxation sweeps (M is symmetric, Lemma 1) until max |residual|/M_ii <= tol_adj
 * (in lambda's units), recomputing the forward states of each checkpoint segment, and writes
 *     dJ/dC_i  = sum_k lambda_k,i (v_{k-1,i} - v_k,i) / h             [nl][ny][nx]
 *     dJ/dgE_e = -sum_k (lambda_a - lambda_b)(v_a - v_b) over east segments   [nl][ny][nx-1]
 *     dJ/dgN_e = the same over north segments                                 [nl][ny-1][nx]
 * to host memory (pg_loss_backward) or device memory (pg_loss_backward_dev).  Sources are held
 * fixed.  The context is left at step k0 + nsteps with the forward end state.
 * The same reverse pass accumulates, for every via and pad (g in series with L, g_eq =
 * h g / (g L + h), alpha = g L / (g L + h); a resistive branch has L = 0), the gradients with
 * respect to g and L:
 *     dJ/dtheta = sum_k (mu_k - A lambda_k) (dg_eq/dtheta (A v_k - v_far) + dalpha/dtheta i_{k-1}),
 * which for a resistive branch is -sum_k (A lambda_k)(A v_k - v_far) (a via joins two layers like
 * a segment, a pad joins its node to Vdd).  pg_loss_branch_gradients (g) and
 * pg_loss_inductance_gradients (L; zero for resistive branches) copy them to host arrays in the
 * mesh's via and pad order (n_vias and n_pads doubles).  PG_ERR_STATE before a completed
 * pg_loss_backward(_dev). */
pg_status pg_loss_forward(pg_ctx* ctx, int32_t grid, int32_t scen, int32_t nsteps, int32_t ckpt_every,
                          double margin, double* J);
pg_status pg_loss_backward(pg_ctx* ctx, double tol_adj, double* dJ_dC, double* dJ_dgE, double* dJ_dgN);
pg_status pg_loss_backward_dev(pg_ctx* ctx, double tol_adj, double* dJ_dC, double* dJ_dgE, double* dJ_dgN);
pg_status pg_loss_branch_gradients(pg_ctx* ctx, double* dJ_dvia_g, double* dJ_dpad_g);
pg_status pg_loss_inductance_gradients(pg_ctx* ctx, double* dJ_dvia_L, double* dJ_dpad_L);

pg_status pg_get_stats(const pg_ctx* ctx, pg_stats* out);
pg_status pg_reset_stats(pg_ctx* ctx);

/* Kernel timing with HIP events on the context stream: enable = k > 0 times every k-th interval
 * of each kind (see pg_kernel_times), 0 turns it off.  Each timed interval adds two event records
 * to the stream.  pg_read_kernel_times synchronises the stream. */
pg_status pg_profile(pg_ctx* ctx, int32_t enable);
pg_status pg_read_kernel_times(pg_ctx* ctx, pg_kernel_times* out);

#ifdef __cplusplus
}
#endif

#endif /* PGRID_H */
