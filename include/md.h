/*
 * md.h -- C ABI of the MI355X EAM timestep library (libmdeam.so).
 *
 * The library advances Embedded Atom Method molecular dynamics on one GPU:
 * cell binning, a Verlet neighbour list with skin, the density pass
 * rho_i = sum_j rho(r_ij), the embedding derivative F'(rho_i), the force pass
 * and leap-frog / velocity-Verlet integration.  Paper: "Breaking the Molecular
 * Dynamics Timescale Barrier Using a Wafer-Scale System" (arXiv 2405.07898):
 *   - per-atom state is identity, position and velocity          (Sec. III-A)
 *   - rho, F and phi are polynomial splines with a hard cutoff    (Sec. II-A)
 *   - U = 1/2 sum_{i!=j} phi(r_ij) + sum_i F(rho_i)               (Eq. potential)
 *   - force = -dU/dx_i                                             (Eq. EAMforce)
 *   - second-order leap-frog time stepping                         (Eq. leapfrog)
 *   - only the MD loop is timed; setup sits outside md_step        (Sec. IV-B)
 *
 * Conventions
 *   - Units: Angstrom, fs, eV, amu.  ftm2v converts (eV/A)/amu to A/fs^2.
 *   - Every state array crossing the boundary is a DEVICE pointer to float64
 *     AoS [n_atoms][3] in the caller's original atom order (replicas
 *     concatenated in replica order).  Spline tables and per-replica sizes
 *     are HOST pointers, copied during md_create.
 *   - The caller owns all device memory.  md_create borrows a workspace of
 *     md_workspace_size() bytes (256-byte aligned) until md_destroy; the
 *     library allocates no device memory of its own apart from what the HIP
 *     runtime needs to instantiate graphs.
 *   - A context is bound to one HIP stream (hipStream_t passed as void*);
 *     every call enqueues on it.  Calls that return host values (md_energy,
 *     md_stats, md_step's status) synchronise that stream.  A context is not
 *     thread-safe.
 *   - Device-side conditions are latched in a status word read at the end of
 *     md_step / md_build_neighbors.  After an error every kernel of the
 *     context becomes a no-op; md_step rolls the state back to the last clean
 *     chunk start and clears the error, md_set_state clears it too.
 */
#ifndef MDEAM_MD_H
#define MDEAM_MD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t md_status;

/* Status codes: 0 ok, < 0 error, > 0 warning (sticky bits). */
#define MD_OK 0
#define MD_E_ARG (-1)           /* invalid argument */
#define MD_E_BOX (-2)           /* periodic edge < 2 (r_cut + skin) or < 3 cells; edge 0 */
#define MD_E_TABLE (-3)         /* malformed spline table */
#define MD_E_NBR_OVERFLOW (-4)  /* some atom has more than nbr_capacity list entries */
#define MD_E_CELL_OVERFLOW (-5) /* some cell holds more than cell_capacity atoms */
#define MD_E_NONFINITE (-6)     /* non-finite position or force */
#define MD_E_HIP (-7)           /* HIP runtime error (see md_last_error) */
#define MD_E_ORDER (-8)         /* call out of order (e.g. md_step before md_build_neighbors) */
#define MD_E_LOST_ATOM (-9)     /* an atom moved more than one box length past a periodic edge */
#define MD_E_WORKSPACE (-10)    /* workspace too small or misaligned */
#define MD_E_STALL (-11)        /* a grid barrier of a persistent launch timed out, or a
                                   one-XCD launch found too few workgroups on that XCD */
#define MD_W_RHO_RANGE 1        /* some rho_i exceeded the F table's last knot; F continued
                                   along its end tangent there */

/* Precision of the pair passes. */
#define MD_FP64 0  /* everything in float64 */
#define MD_MIXED 1 /* pair terms, rho_i and force sums in float32 with compensated
                      (TwoSum) accumulation; positions, velocities, integration
                      and energy totals in float64.  The pair passes take the
                      separations from a 16-byte record per atom: the position
                      in 32-bit fixed point (2^32 quanta per periodic box
                      length, so integer wrap-around is the minimum image;
                      2^26 per A in an open dimension) and F' in float32 */

/* Neighbour-list form of the pair passes.
 * MD_LIST_FULL: every atom walks both directions of each pair and writes only
 *   itself (each pair term is evaluated twice).
 * MD_LIST_HALF: force symmetry (the paper's Sec. VI-A projection): each pair is
 *   evaluated once, by its lower-slot atom, into a pair slot; a second pass
 *   gathers every atom's pair slots in a fixed (sorted) order.  Deterministic
 *   (no float atomics; bitwise repeatable), float64 only (MD_FP64), one lane
 *   per atom (lanes_per_atom is ignored).  Takes 52 + 52 nbr_capacity extra
 *   bytes per atom of workspace. */
#define MD_LIST_FULL 0
#define MD_LIST_HALF 1

/* How md_step launches a chunk of chunk_steps steps.
 * MD_LAUNCH_GRAPH: a captured hipGraph of four kernels per step (binning and
 *   list build run only when flagged).  Small systems (the whole rebuild fits
 *   at most 64 co-resident workgroups; one atom type, full list, one lanes-
 *   per-atom value) fold binning, list build and density pass into one kernel
 *   with grid barriers, so a step without a rebuild is two kernels.
 * MD_LAUNCH_PERSISTENT: one cooperative launch runs the whole chunk, its
 *   workgroups meeting at grid barriers between the phases of each step (for
 *   small systems, where the graph's per-kernel launch cost dominates the
 *   step; the paper's case for time steps per second at small N, Sec. II-B).
 *   A system whose atom tiles fit one thread each on the workgroups of one
 *   XCD runs there with its per-atom state in registers; larger ones use
 *   every XCD.  Full list and one atom type only; results are bitwise those
 *   of the graph.  A barrier that waits too long ends the launch with
 *   MD_E_STALL. */
#define MD_LAUNCH_GRAPH 0
#define MD_LAUNCH_PERSISTENT 1

/* Most atom types of the multi-species form. */
#define MD_MAX_TYPES 4

/* A cubic spline on equally spaced knots x0 + k/inv_dx, k = 0..n_knots-1.
 * coef (host) holds (n_knots-1) rows of 4 float64: segment k evaluates
 * c0 + c1 t + c2 t^2 + c3 t^3 with t = (s - x0) inv_dx - k in [0,1); the
 * segment index is int((s - x0) inv_dx) clamped to [0, n_knots-2] (segment
 * arithmetic as in the paper's Table "flopmodel": x = alpha r, k = int(x),
 * dx = x - k).  Past the last knot a table continues along its end tangent:
 * value f(end) + f'(end) (s - s_end), slope f'(end).  The r tables end at or
 * past r_cut, so only the embedding F(rho) is ever evaluated there. */
typedef struct md_spline {
  int32_t n_knots;
  int32_t reserved;
  double x0;
  double inv_dx;
  const double* coef;
} md_spline;

/* Parameters shared by all replicas of a context.  The per-box quantities
 * (atom count, edge lengths, which dimensions are periodic) are not fields
 * here: they are passed per replica (rep_atoms, rep_box) to md_init,
 * md_init_batch, md_create and the workspace queries, a negative edge length
 * marking an open dimension.  The rebuild rule is fixed: the list is rebuilt
 * in the step after any atom of a replica moved more than skin/2 from its
 * position at the last build. */
typedef struct md_params {
  double mass;           /* amu */
  double dt;             /* fs */
  double r_cut;          /* interaction cutoff, A (pairs with r^2 < r_cut^2 interact) */
  double skin;           /* Verlet skin, A (list holds pairs with r^2 < (r_cut+skin)^2) */
  double ftm2v;          /* (eV/A)/amu -> A/fs^2 */
  double kboltz;         /* eV/K, for temperatures reported by md_stats */
  int32_t precision;     /* MD_FP64 or MD_MIXED */
  int32_t nbr_capacity;  /* max list entries per atom (<= 1024) */
  int32_t cell_capacity; /* max atoms per binning cell (<= 256) */
  int32_t chunk_steps;   /* steps per captured hipGraph (even, >= 2), e.g. 100 */
  int32_t lanes_per_atom;/* 0 = automatic, else 1, 2, 4 or 8 lanes per atom */
  int32_t sort_every;    /* re-sort atoms by cell every this many chunks (0 = never) */
  int32_t list_mode;     /* MD_LIST_FULL or MD_LIST_HALF */
  int32_t n_types;       /* atom types: 0 or 1 (one species, md_create), or
                            2..MD_MAX_TYPES (md_create_multi) */
  int32_t launch_mode;   /* MD_LAUNCH_GRAPH or MD_LAUNCH_PERSISTENT */
  int32_t reserved;      /* 0 */
} md_params;

typedef struct md_ctx md_ctx;

/* Counters and observables; md_stats fills it (synchronises). */
typedef struct md_stats_t {
  int64_t steps;        /* MD steps taken since md_build_neighbors */
  int64_t rebuilds;     /* neighbour-list rebuilds inside md_step */
  int64_t list_entries; /* total list entries at the last build (mean length = /n_atoms) */
  int32_t max_list;     /* longest list at the last build */
  int32_t max_cell;     /* fullest cell at the last binning */
  int32_t status_bits;  /* latched device status bits */
  int32_t reserved;
} md_stats_t;

/* Bytes of device workspace md_create needs for these sizes.
 * n_rep replicas; rep_atoms[r] atoms and orthorhombic box rep_box[3r..3r+2]
 * (A) for replica r (host arrays).
 *
 * Sizes: n_rep >= 1 and every replica holds at least one atom (an empty one
 * is MD_E_ARG).  All replicas together hold fewer than 2^26 atoms (the list
 * keeps a 26-bit atom index), and atoms x nbr_capacity x 4 bytes of list stay
 * below 2^32 (8,388,607 atoms at capacity 128); larger sizes are MD_E_ARG.
 *
 * Box convention: a positive length L makes that dimension periodic on
 * [0, L).  A negative length -E makes it open (free surfaces, as on the
 * lateral faces of the paper's slab, Sec. IV): no wrap and no image; E is the
 * extent of the cell grid along it, [0, E).  Atoms of an open dimension may
 * sit outside [0, E); they are binned into the edge cells, which stays exact
 * (a cell is at least r_cut + skin wide) but crowds those cells, so choose E
 * to cover the atoms. */
md_status md_workspace_size(const md_params* p, int32_t n_rep, const int64_t* rep_atoms,
                            const double* rep_box, size_t* bytes);

/* Same as md_workspace_size, returning the byte count (0 for invalid
 * parameters or sizes). */
size_t md_workspace_bytes(const md_params* p, int32_t n_rep, const int64_t* rep_atoms,
                          const double* rep_box);

/* Create a context for one box and upload its state in one call (md_create
 * followed by md_set_state; the paper's per-atom state is identity, position
 * and velocity, Sec. III-A, and set-up stays outside the timed MD loop,
 * Sec. IV-B).  box: 3 edge lengths (host; negative = open dimension).
 * x, v: device [n_atoms][3] float64, original order, on-step velocities.
 * workspace: device, at least md_workspace_bytes(p, 1, &n_atoms, box) bytes,
 * 256-byte aligned, borrowed until md_destroy.  On an error nothing is
 * created (*out = NULL).  md_build_neighbors must follow before md_step. */
md_status md_init(md_ctx** out, const md_params* p, int64_t n_atoms, const double* box,
                  const md_spline* phi, const md_spline* rho, const md_spline* emb,
                  const double* x, const double* v, void* workspace, size_t workspace_bytes,
                  void* stream);

/* md_init for n_rep independent boxes in one context (the batched form):
 * replica r holds rep_atoms[r] atoms in box rep_box[3r..3r+2]; x and v hold
 * all replicas concatenated in replica order.  Every pass runs all replicas
 * in one launch; each replica rebuilds its list on its own schedule. */
md_status md_init_batch(md_ctx** out, const md_params* p, int32_t n_rep,
                        const int64_t* rep_atoms, const double* rep_box, const md_spline* phi,
                        const md_spline* rho, const md_spline* emb, const double* x,
                        const double* v, void* workspace, size_t workspace_bytes,
                        void* stream);

/* Create a context.  phi(r), rho(r) tables must cover [0, r_cut]; emb(rho)
 * any range (values past its last knot raise MD_W_RHO_RANGE).  workspace is
 * a device pointer of at least md_workspace_size() bytes; stream is a
 * hipStream_t.  Returns MD_E_BOX if a periodic replica edge is below
 * 2 (r_cut + skin) or gives fewer than 3 cells, or an edge is 0 or not
 * finite. */
md_status md_create(md_ctx** out, const md_params* p, int32_t n_rep, const int64_t* rep_atoms,
                    const double* rep_box, const md_spline* phi, const md_spline* rho,
                    const md_spline* emb, void* workspace, size_t workspace_bytes, void* stream);

/* Multi-species EAM (paper Sec. II-A: the density, embedding and pair
 * functions depend on the atom types, after Eq. potential):
 *   rho_i = sum_j rho_{t_j}(r_ij), U = 1/2 sum phi_{t_i t_j} + sum_i F_{t_i}(rho_i),
 *   F_i = sum_j [F'_i rho'_{t_j} + F'_j rho'_{t_i} + phi'_{t_i t_j}] (x_j - x_i)/r.
 * p->n_types = T in 2..MD_MAX_TYPES; float64 (MD_FP64) and the full list only.
 * Host arrays: phi[a*T + b] (the table of pair types a, b; phi[b*T + a] must
 * hold the same coefficients), rho[t] (the density an atom of type t emits),
 * emb[t] (F of type t), masses[t] (amu; p->mass is not used).  Every rho and
 * phi table shares rho[0]'s knot grid (x0 = 0, reaching r_cut); every F table
 * shares emb[0]'s.  Returns MD_E_TABLE for mismatched grids or an asymmetric
 * phi, MD_E_ARG for a bad count or mass.  All atoms are type 0 until
 * md_set_types.  The workspace size comes from md_workspace_size with the
 * same p. */
md_status md_create_multi(md_ctx** out, const md_params* p, int32_t n_rep,
                          const int64_t* rep_atoms, const double* rep_box, const md_spline* phi,
                          const md_spline* rho, const md_spline* emb, const double* masses,
                          void* workspace, size_t workspace_bytes, void* stream);

/* Types of the atoms (device, [n] int32, original order, each in [0, T)) of a
 * context made by md_create_multi.  Returns MD_E_ARG if any type is out of
 * range (those atoms become type 0) or if the context has one species.
 * Forces belong to the old types afterwards:
 * md_build_neighbors must follow before md_step. */
md_status md_set_types(md_ctx* ctx, const int32_t* type);

/* Upload positions x and on-step velocities v (device, [n][3] float64,
 * original order).  Positions are wrapped into the box along periodic
 * dimensions (open ones are kept as given).  Clears the status
 * word; md_build_neighbors must follow before md_step. */
md_status md_set_state(md_ctx* ctx, const double* x, const double* v);

/* Sort atoms by cell, bin them, build the Verlet list (pairs with
 * r^2 < (r_cut+skin)^2 under the minimum image), and compute rho, F' and
 * forces at the current positions (paper Sec. III-A steps 1-3). */
md_status md_build_neighbors(md_ctx* ctx);

/* Advance n steps.  Each step: density pass, force pass fused with the
 * leap-frog kick and drift and the skin/2 displacement check; the list is
 * rebuilt on the device in the step after any atom moved more than skin/2.
 * Whole chunks run as one captured hipGraph; the steps left over (fewer than
 * chunk_steps) run as one shorter captured graph, kept for reuse (a few
 * lengths at a time).  With MD_LAUNCH_PERSISTENT the left-over steps are
 * launched kernel by kernel.  On an error the state rolls back to the start
 * of the graph (or chunk) in which it occurred and the list is rebuilt there
 * (the status is returned; md_stats().steps tells where).  Should that
 * rebuild fail as well, no list is valid: md_step, md_compute_forces and
 * md_get_state with forces return MD_E_ORDER until md_set_state and
 * md_build_neighbors start over.
 * n = 0 takes no step and returns the latched status; n < 0 is MD_E_ARG. */
md_status md_step(md_ctx* ctx, int64_t n);

/* Capture, without running them, the graphs that md_step(n) would launch
 * from the current state (the chunk graph and the shorter graphs of the
 * left-over steps), so that the next md_step(n) spends no time capturing.
 * Changes no state; graphs are dropped again by md_set_schedule.  Nothing to
 * do with MD_LAUNCH_PERSISTENT.  Requires md_build_neighbors. */
md_status md_prepare(md_ctx* ctx, int64_t n);

/* Potential and kinetic energy per replica (host arrays of n_rep doubles;
 * either may be NULL), with on-step velocities.  Fixed-order reductions:
 * bitwise reproducible. */
md_status md_energy(md_ctx* ctx, double* pe, double* ke);

/* Download state in original order (device pointers, [n][3] float64; any
 * may be NULL): wrapped positions, on-step velocities, forces. */
md_status md_get_state(md_ctx* ctx, double* x, double* v, double* f);

/* Recompute forces at the current positions (fresh list); same outputs as
 * md_get_state's f, also giving rho_i and F'_i (device [n] float64, NULL
 * allowed).  Used for force-error reports. */
md_status md_compute_forces(md_ctx* ctx, double* f, double* rho, double* fp);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the forces,
 * rho_i and F'_i that md_create + md_set_state + md_build_neighbors +
 * md_compute_forces give for one box, with no workspace and no device
 * allocation.  Every intermediate (spline rows, tile tables, sorted state,
 * bins, neighbour list, status words) lives in a fixed 16 MiB device array
 * that the library holds on each GPU it runs on until the process ends.
 * Limits: n_atoms <= MD_STATIC_MAX_ATOMS, at most MD_STATIC_MAX_CELLS
 * binning cells, tables of at most MD_STATIC_MAX_KNOTS knots,
 * p->nbr_capacity <= 128, p->cell_capacity <= 64, the full list and one atom
 * type; past them the call returns MD_E_ARG (MD_E_TABLE for tables) before
 * touching the device.  Unlike elsewhere, the three tables' coef fields are
 * DEVICE pointers here ((n_knots-1) x 4 float64 each).  x: device
 * [n_atoms][3] float64; f: device [n_atoms][3], rho and fp: device
 * [n_atoms] (any of the three may be NULL); all in the caller's order.
 * Synchronises the stream.  Calls on one GPU share the array: calls that
 * overlap in time on one GPU (other threads, other streams) race. */
#define MD_STATIC_MAX_ATOMS 16384
#define MD_STATIC_MAX_CELLS 4096
#define MD_STATIC_MAX_KNOTS 2048
md_status md_forces_static(const md_params* p, int64_t n_atoms, const double* box,
                           const md_spline* phi, const md_spline* rho, const md_spline* emb,
                           const double* x, double* f, double* rho_out, double* fp_out,
                           void* stream);

/* Counters (synchronises). */
md_status md_stats(md_ctx* ctx, md_stats_t* out);

/* Inspection of the last build, original order and original ids (device
 * pointers): cell id of each atom within its replica, list length and up
 * to cap_out list entries per atom (row-major [n][cap_out], unused -1). */
md_status md_get_cells(md_ctx* ctx, int32_t* cell);
md_status md_get_neighbors(md_ctx* ctx, int32_t* cnt, int32_t* nbr, int32_t cap_out);

/* Enqueue reps launches of one pass on the context stream, with no
 * synchronisation, for timing with events: 0 = density, 1 = force+integrate
 * (state restored from a snapshot afterwards), 2 = list build (after one
 * binning), 3 = binning (followed by one list build), 4 = force+integrate
 * alone: every launch reads the same positions and advances the velocities,
 * so the state is not usable afterwards until md_set_state. */
md_status md_launch_pass(md_ctx* ctx, int32_t pass, int32_t reps);

/* Pair-pass schedule: lanes per atom (1, 2, 4 or 8) cooperating on one
 * atom's neighbour list, with a fixed-order shuffle reduction.  Results are
 * identical up to that reduction order.  Drops the captured step graphs. */
md_status md_set_schedule(md_ctx* ctx, int32_t lanes_per_atom);

/* Per-replica schedule of a batched context (the batched form's multi-core
 * workers, Sec. VI-A): lanes[r] (host, n_rep values of 1, 2, 4 or 8) lanes
 * per atom for replica r, all in the same launch per pass.  The pair passes
 * then take work in pair tiles of 64 / lanes[r] atoms of one replica, one
 * wave per tile.  A replica's results depend only on its own value: bitwise
 * those of the replica alone with md_set_schedule(lanes[r]).  All values
 * equal: the same as md_set_schedule.  Full list, one atom type and graph
 * launches only (else MD_E_ARG).  Drops the captured step graphs. */
md_status md_set_replica_schedule(md_ctx* ctx, const int32_t* lanes);

/* Lanes per atom of each replica (host, n_rep values). */
md_status md_get_replica_schedule(md_ctx* ctx, int32_t* lanes);

/* Autotuner: times reps rounds of the step's density and force-plus-update
 * kernels at the current state for every lanes-per-atom choice (HIP events on
 * the context stream, two sweeps, the faster sweep of each choice kept),
 * keeps the fastest and reports it in microseconds per round (either pointer
 * may be NULL).  With several replicas (full list, one atom type, graph
 * launches) it then searches one value per replica size class (up to 2,048
 * atoms, up to 8,192, larger), class by class from the uniform choice in two
 * passes, and keeps that per-replica schedule if it is faster
 * (md_get_replica_schedule tells; *best_lanes_per_atom stays the best
 * uniform value, *best_us the time of the kept schedule).  Positions,
 * velocities and the step count come back from the rollback snapshot, which
 * then holds the current state.  Requires md_build_neighbors. */
md_status md_autotune(md_ctx* ctx, int32_t reps, int32_t* best_lanes_per_atom, float* best_us);

/* Last error text of this context (or of the library when ctx is NULL). */
const char* md_last_error(const md_ctx* ctx);
const char* md_status_string(md_status s);

void md_destroy(md_ctx* ctx);

/* ------------------------------------------------------------------ */
/* Force matching (gradient of a force-matching loss w.r.t. the spline
 * coefficients).  Configurations are static periodic boxes; the loss is
 * L = sum_c sum_i |F_i - Fref_i|^2 with forces from Eq. (EAMforce).
 * The gradient is taken with respect to the per-segment coefficients of
 * phi, rho and F (layouts as md_spline.coef). */
typedef struct md_fm_ctx md_fm_ctx;

/* Bytes of device workspace for n_cfg configs (host rep_atoms, rep_box) with
 * n_knots-knot tables for each of phi, rho, F.  Returns MD_E_TABLE when the
 * three tables have more than 2048 segments together (the coefficient
 * gradients are accumulated in one 64 KB LDS histogram per workgroup). */
md_status md_fm_workspace_size(int32_t n_cfg, const int64_t* cfg_atoms, const double* cfg_box,
                               double r_cut, int32_t nbr_capacity, const int32_t n_knots[3],
                               size_t* bytes);

/* x and fref: device [n][3] float64 (all configs concatenated).  The knot
 * grids (x0, inv_dx, n_knots) of the three tables are fixed here; their
 * coefficients are passed to each forward call.  The context keeps 16 bytes
 * of pinned host memory (hipHostMalloc) for the scalars the calls return,
 * freed by md_fm_destroy. */
md_status md_fm_create(md_fm_ctx** out, int32_t n_cfg, const int64_t* cfg_atoms,
                       const double* cfg_box, double r_cut, int32_t nbr_capacity,
                       const md_spline* grid_phi, const md_spline* grid_rho,
                       const md_spline* grid_emb, const double* x, const double* fref,
                       void* workspace, size_t workspace_bytes, void* stream);

/* Forward: coefficients (device, [(n_knots-1)*4] float64 each) -> loss (host
 * double) and, if f_out is not NULL, forces (device [n][3]). */
md_status md_fm_forward(md_fm_ctx* ctx, const double* coef_phi, const double* coef_rho,
                        const double* coef_emb, double* loss, double* f_out);

/* Backward for the last forward: dL/dcoef into device arrays of the same
 * layouts (overwritten), scaled by seed (dL_total/dL). Deterministic. */
md_status md_fm_backward(md_fm_ctx* ctx, double seed, double* g_phi, double* g_rho,
                         double* g_emb);

/* The same two calls without a host synchronisation, for loops that need
 * neither the loss nor the status on the host every evaluation (an optimiser
 * on the device).  forward_async writes the loss to loss_dev (device double);
 * backward_async reads its seed from seed_dev (device double).  Non-finite
 * values and fixed-point overflows stay latched on the device until
 * md_fm_check, which synchronises the context's stream, returns MD_OK or
 * MD_E_NONFINITE for every call since the last check, and clears the latch
 * (md_fm_forward also clears it first).  Launch order on the context's stream
 * is the only ordering: a gradient array must not be read before the stream
 * has run the backward call that writes it. */
md_status md_fm_forward_async(md_fm_ctx* ctx, const double* coef_phi, const double* coef_rho,
                              const double* coef_emb, double* loss_dev, double* f_out);
md_status md_fm_backward_async(md_fm_ctx* ctx, const double* seed_dev, double* g_phi,
                               double* g_rho, double* g_emb);
md_status md_fm_check(md_fm_ctx* ctx);

void md_fm_destroy(md_fm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* MDEAM_MD_H */
