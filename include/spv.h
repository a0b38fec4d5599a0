/*
 * spv.h -- C-ABI of the MI355X self-propelled Voronoi (SPV) step library
 * (libspv.so, HIP for gfx950).
 *
 * Model (Sussman, "cellGPU: massively parallel simulations of dynamic vertex
 * models", arXiv:1702.02939):
 *   cells are points r_i in a periodic box; their shapes are the Voronoi
 *   cells of the Delaunay triangulation of the points (Sec. II.A, Fig. 1);
 *   E = sum_i K_A (A_i - A0_i)^2 + K_P (P_i - P0_i)^2            (Eq. 1)
 *   F_i = -dE/dr_i, by the chain rule through the Voronoi vertices (App. B)
 *   dr_i/dt = mu F_i + v0 n_i, n_i = (cos theta_i, sin theta_i)     (Eq. 3)
 *   d theta_i/dt = eta_i, white noise of variance 2 Dr             (Sec. II.A)
 * One step = forces and update, then the empty-circumcircle test of every
 * cell's neighbour ring (Sec. II.C.3) and the local repair of failed rings
 * (Sec. II.C.4), entirely on the device.
 *
 * A handle holds one system or a batch of independent systems (each with its
 * own size, box, target shape, self-propulsion speed and seed) that are
 * stepped together; a single system is a batch of one.
 *
 * Conventions shared by every entry point:
 *   - every call returns spv_status; nothing throws across the ABI; on a
 *     non-OK status spv_last_error() returns a message (thread-local);
 *   - array arguments are plain pointers to host memory or to device memory
 *     of the current HIP device (hipMemcpyDefault semantics); the caller
 *     owns them; the library copies inputs and owns its device state;
 *   - per-cell arrays are in "tag order": system by system, and inside a
 *     system by input index (tag), whatever order the library keeps
 *     internally;
 *   - positions are kept on the dyadic grid 2^-q, q = 51 - ceil(log2
 *     max(Lx, Ly)) of their system; inputs are rounded to it (and the box
 *     sides too);
 *   - all work is ordered on the HIP stream given at creation; calls that
 *     return data synchronise that stream;
 *   - a handle is not thread-safe: one host thread per handle.
 */
#ifndef SPV_H
#define SPV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPV_OK = 0,
    SPV_EINVAL = -1,     /* bad argument: N < 3, NULL pointer, non-finite or out-of-box input, duplicate cells */
    SPV_ENOMEM = -2,     /* device or host allocation failed */
    SPV_EHIP = -3,       /* HIP runtime error */
    SPV_EPRECOND = -4,   /* a Delaunay circumradius reached min(Lx, Ly)/4 (box too small for the cells) */
    SPV_ECAPACITY = -5,  /* a ring longer than kcap, or too many repair candidates */
    SPV_ENONFINITE = -6, /* non-finite force or position */
    SPV_EREPAIR = -7     /* topology repair did not converge within repair_rounds */
} spv_status;

/* Arithmetic of the geometry and force kernels.  Positions, their update,
 * the topology predicates (exact) and the noise are FP64 in both. */
enum { SPV_FP64 = 0, SPV_MIXED = 1 /* FP32 Voronoi geometry, forces and energy coefficients */ };

typedef struct {
    double KA, KP;          /* area and perimeter moduli (Eq. 1) */
    double mu;              /* mobility (Eq. 3) */
    double v0;              /* self-propulsion speed (Eq. 3); per system in spv_batch_create */
    double Dr;              /* rotational diffusion constant (Sec. II.A) */
    double dt;              /* time step */
    uint64_t seed;          /* noise: Philox4x64-10, key (seed, 0), counter (step, tag, 0, 0) */
    int32_t precision;      /* SPV_FP64 or SPV_MIXED */
    int32_t resort_every;   /* steps between spatial re-sorts (Sec. II.B), rounded up to even (0: 32;
                               shortened while the cells' drift bound would pass a bin side within
                               it); -1: never re-sort -- the memory order stays that of creation and
                               every step's repairs search a cell list of the step's positions */
    int32_t kcap;           /* ring capacity = max Delaunay degree: 16 or 32 (0: 16, regrown
                               to 32 when a ring needs more, at creation or in a run) */
    int32_t repair_rounds;  /* max test/repair rounds per step, device and host together (0: 16, max 32) */
    int32_t device_rounds;  /* repair rounds run on the device inside each step: round 0 over the whole
                               grid, later ones in one block (0: 8) */
    int32_t no_graphs;      /* 0: replay whole re-sort periods as captured HIP graphs; 1: launch eagerly */
    int32_t repair_cells;   /* flagged cells per repair wavefront: the repair grid is N / repair_cells
                               blocks, clamped to [256, 4096] (0: 64) */
    int32_t autotune;       /* 0: use the scheduling knobs given here (resort_every, device_rounds,
                               repair_cells, tail_items, full_rounds, force_mode, bin_factor); 1: take them from the tuning cache for this
                               device and size class, else choose them by timed trial runs and cache
                               them; 2: always run the trials and refresh the cache.  The cache is the
                               JSON file named by the environment variable SPV_TUNE_CACHE, else held
                               in this process only.  The knobs never change results. */
    int32_t tail_items;     /* a later round with more flagged cells than this is handed to the host
                               (full-grid rounds) instead of the one-block tail (0: 64) */
    int32_t full_rounds;    /* repair rounds per step run over the whole grid before the tail takes
                               the rest (0: 1; at most 4) */
    int32_t bin_order;      /* memory order of the cell-list bins (Sec. II.B spatial sorting):
                               0 = Hilbert curve, 1 = row-major (for locality comparisons) */
    int32_t force_mode;     /* layout of the force kernel (Eq. 2, App. A-B) and of the all-cells
                               geometry and validity pass (Sec. II.C), bitwise the same results
                               either way: 1 = lanes per cell, 2 = one thread per (cell, ring
                               slot); 0 = 2 from 2^18 cells on, else 1 */
    double bin_factor;      /* cell-list bin side in mean cell spacings sqrt(Lx Ly / N) (0: 1; 0.5..8) */
    int32_t dense;          /* first repair rounds of a step (Sec. II.C.4) as dense rounds, which mark
                               flagged and touched cells in one byte per cell and scan them, instead of
                               appending them to worklists (suits steps in which a large share of the
                               cells fails): 0 = while cells move fast (after a random start), 1 =
                               never, 2 = every step.  Never changes results. */
    int32_t repair_mode;    /* where failed rings are rebuilt (Sec. II.C.3-4): 0 = on the device, inside
                               the step; 1 = hybrid comparison mode, the paper's own split: the device
                               tests every ring, the worklist and the positions go to the host each
                               step, the library's host code rebuilds the rings (exact gift-wrapping,
                               the device's tie-break) and uploads them, the device re-tests the touched
                               cells, round after round.  Same results; steps run eagerly, with no
                               graphs and no autotuning.  Single systems and batches. */
} spv_params;

/* Scheduling knobs a handle runs with (see spv_params). */
typedef struct {
    int32_t resort_every, device_rounds, repair_cells, tail_items, full_rounds;
    int32_t force_mode;  /* the force kernel in use: 1 or 2 (see spv_params) */
    int32_t source;      /* 0: given in spv_params, 1: tuning cache, 2: timed trials */
    double bin_factor;
    double ms_per_step;  /* trial time per step of the chosen knobs (0 when source = 0) */
} spv_tuning;

typedef struct spv_sys spv_sys; /* opaque handle: all device state of one system or batch */

/*
 * Create one system of N cells at positions (x[i], y[i]) in [0, Lx) x [0, Ly)
 * and build its periodic Delaunay triangulation on the device.
 *   A0, P0   per-cell preferred area / perimeter (Eq. 1); A0 == NULL means 1;
 *            P0 == NULL means P0_i = p0 * sqrt(A0_i)
 *   theta0   initial directors; NULL means theta_i = 2 pi u with u from
 *            Philox counter (2^64 - 1, tag, 0, 0)
 *   stream   hipStream_t to order all work on (NULL: the default stream)
 * Ownership: *out receives a new handle (free with spv_destroy).  All input
 * arrays are read during the call only.
 * Size limit: N * kcap < 2^30 (N < 2^26 cells at kcap 16, 2^25 at kcap 32;
 * ring rows are addressed with 32-bit offsets); larger N is SPV_EINVAL,
 * decided before any input is read or any memory allocated.
 * Errors: SPV_EINVAL (arguments), SPV_EPRECOND (box too small), SPV_ENOMEM,
 * SPV_EHIP; *out is then NULL.
 */
spv_status spv_create(spv_sys** out, int64_t N, const double* x, const double* y, double Lx, double Ly,
                      const double* A0, const double* P0, double p0, const double* theta0,
                      const spv_params* params, void* stream);

/*
 * Create a batch of S independent systems, stepped together by every
 * spv_step call (each with its own noise key, so a system in a batch follows
 * exactly the trajectory it follows alone).
 *   N_s[S], Lx_s[S], Ly_s[S]   cells and box of each system
 *   x, y                        positions, concatenated system by system (sum N_s entries)
 *   P0                          per-cell target perimeters, concatenated, or NULL:
 *                               P0 = p0_s[s] * sqrt(A0) with A0 = 1
 *   p0_s, v0_s, seed_s          per-system target shape index, speed, noise seed
 *                               (v0_s / seed_s NULL: params->v0 / params->seed)
 * Other model parameters (K_A, K_P, mu, Dr, dt, precision, ...) are shared.
 * Size limit: (sum of N_s) * kcap < 2^30, as spv_create.
 * Errors as spv_create.
 */
spv_status spv_batch_create(spv_sys** out, int32_t S, const int64_t* N_s, const double* Lx_s, const double* Ly_s,
                            const double* x, const double* y, const double* P0, const double* p0_s,
                            const double* v0_s, const uint64_t* seed_s, const spv_params* params, void* stream);

/*
 * Advance nsteps steps (Sec. II.C): forces and Eq. (3) update, then the
 * validity test and device-side repair of the triangulation.  The step index
 * used for the noise counter continues across calls.
 * Errors: SPV_EPRECOND, SPV_ECAPACITY, SPV_ENONFINITE, SPV_EREPAIR, SPV_EHIP.
 * After an error the handle holds the state reached when it was detected and
 * every later spv_step returns the same error.
 */
spv_status spv_step(spv_sys* s, int64_t nsteps);

/* Number of systems and total number of cells of the handle. */
spv_status spv_get_size(spv_sys* s, int32_t* S, int64_t* N);

/* Current ring capacity (16 or 32).  With kcap 0 the handle starts at 16 and
 * moves to 32 when a ring needs more: at creation, or during spv_step, where
 * the step whose repair overflowed is finished by rebuilding the topology of
 * its positions at capacity 32 (statistics then restart as after
 * spv_load_state; the handle pointer stays valid). */
spv_status spv_get_kcap(spv_sys* s, int32_t* kcap);

/* First cell (in tag order) and cell count of system sys. */
spv_status spv_get_system_range(spv_sys* s, int32_t sys, int64_t* first, int64_t* n);

/* Box sides of system 0 after rounding to the grid, and the grid exponent q. */
spv_status spv_get_box(spv_sys* s, double* Lx, double* Ly, int32_t* q);

/* Box of system sys (batches). */
spv_status spv_get_system_box(spv_sys* s, int32_t sys, double* Lx, double* Ly, int32_t* q);

/* Current positions / directors, tag order, total-N entries each. */
spv_status spv_get_positions(spv_sys* s, double* x, double* y);
spv_status spv_get_directors(spv_sys* s, double* theta);

/* Forces F = -dE/dr at the current positions and topology, tag order. */
spv_status spv_get_forces(spv_sys* s, double* fx, double* fy);

/* Voronoi area and perimeter of every cell, tag order. */
spv_status spv_get_geometry(spv_sys* s, double* A, double* P);

/*
 * Neighbour lists (Delaunay rings), CSR in tag order: the neighbours of cell
 * t are nbr[offsets[t] .. offsets[t+1]), counter-clockwise, starting at the
 * smallest tag; entries are tag-order indices (system first cell + tag).
 * offsets has total-N + 1 entries; nbr has room for cap entries.  *needed
 * receives the total (3 N_s per system on the torus).  Host pointers only.
 * Errors: SPV_ECAPACITY if cap < *needed (offsets are still written).
 */
spv_status spv_get_neighbors(spv_sys* s, int32_t* offsets, int32_t* nbr, int64_t cap, int64_t* needed);

/*
 * Fault injection for tests of the topology test and repair (Sec. II.C: every
 * ring is tested after each move and the failing ones are rebuilt).  Replaces
 * the ring of cell `cell` (tag-order index, as in spv_get_neighbors) with
 * the k entries of nbr (tag-order indices, host pointer), whatever the
 * geometry says, and records no opposite cell for any of its edges, so that
 * the next step's test of the cell fails and the repair rebuilds its ring
 * from the positions.  That step's forces still use the ring as written.
 * Errors: SPV_EINVAL for a cell out of range, k outside [3, kcap], or an
 * entry outside the cell's system, equal to the cell or repeated (the
 * handle unchanged).
 */
spv_status spv_debug_set_ring(spv_sys* s, int64_t cell, int32_t k, const int32_t* nbr);

/*
 * Observables of the current state summed over all systems: E (Eq. 1),
 * qbar = mean of P_i/sqrt(A_i), sumA = sum of A_i; counters[13] (host
 * pointer, may be NULL):
 *   [0] steps taken  [1] cells repaired  [2] repair rounds used  [3] exact-arithmetic fallbacks
 *   [4] max ring length written  [5] spatial re-sorts  [6] repair radius retries  [7] error word
 *   [8] re-sort periods replayed as captured graphs  [9] steps with dense first rounds
 *   [10] repair rounds run by host recovery  [11] steps finished by host recovery
 *   [12] candidate cells gathered by the repairs (summed over their radius attempts)
 * (statistics since creation or the last load)
 */
spv_status spv_get_observables(spv_sys* s, double* E, double* qbar, double* sumA, int64_t* counters);

/* Observables of one system of a batch. */
spv_status spv_get_system_observables(spv_sys* s, int32_t sys, double* E, double* qbar, double* sumA);

/*
 * Checkpoint and resume (the state of Eq. 3's dynamics: positions, directors,
 * per-cell targets A0/P0 of Eq. 1, the step index that drives the noise).
 * The triangulation is not stored: it is the unique Delaunay triangulation
 * of the positions (Sec. II.C.3, ties broken by tag), rebuilt on load, so a
 * loaded handle continues bitwise as the saved one would have.  Model
 * parameters (K_A, K_P, mu, Dr, dt, v0, seed) are the loading handle's own.
 *   spv_save_state  buf: host or device pointer to cap bytes (may be NULL to
 *                   query); *needed = size.  Layout, little-endian: header
 *                   {char magic[8] = "SPVSTAT\1"; int32 S, precision; int64 N;
 *                   uint64 step}, S records {int64 n; double Lx, Ly, v0;
 *                   uint64 seed}, then x, y, theta, A0, P0 as double[N] each
 *                   in tag order (systems concatenated).
 *   spv_load_state  buf of len bytes as written by spv_save_state into a
 *                   handle of the same layout (S, N_s, grid-rounded boxes,
 *                   precision).  Clears a sticky error on success; repair
 *                   statistics restart.
 * Errors: spv_save_state SPV_ECAPACITY (cap < *needed, nothing written),
 * SPV_EHIP; spv_load_state SPV_EINVAL (size, magic, layout, off-grid or
 * non-finite values; the handle is unchanged), repair errors while
 * rebuilding (the handle then reports that error until the next load).
 */
spv_status spv_save_state(spv_sys* s, void* buf, int64_t cap, int64_t* needed);
spv_status spv_load_state(spv_sys* s, const void* buf, int64_t len);

/*
 * Scheduling knobs of a handle.  With spv_params.autotune set, creation first
 * runs the tuner: a clone of the input is stepped 256 steps from the given
 * state, then clones of that state are timed over whole re-sort periods for
 * each candidate bin side, repair grid, device repair budget and re-sort
 * period (one knob at a time, each against a fresh time of the current best).
 * The handle itself starts from the caller's input, so its trajectory is
 * exactly that of an untuned handle.  A trial that fails leaves the given
 * knobs in place (source 0).
 * Errors: SPV_EINVAL (NULL argument).
 */
spv_status spv_get_tuning(spv_sys* s, spv_tuning* out);

/*
 * Kernel timing.  While enabled, steps are launched eagerly (not as captured
 * graphs; eager batches as otherwise) and every kernel launch carries a pair
 * of HIP events attached to its dispatch (start and end of its execution on
 * the handle's stream); spv_kernel_time returns the summed duration (ms) and
 * number of timed launches of one kernel class since enabling.
 *   which: 0 = force + update (Eq. 3, App. B), 1 = geometry + validity test
 *          of all cells (Sec. II.C), 2 = repair (Sec. II.C.4; every device
 *          round), 3 = re-test of the cells a repair touched, 4 = step tail
 *          (later rounds, step close), 5 = the step's cell list (fast-moving
 *          phase), 6 = flag compaction (dense rounds), 7 = spatial re-sort
 *          (Sec. II.B), 8 = host-driven recovery rounds
 */
spv_status spv_set_timing(spv_sys* s, int32_t enable);
spv_status spv_kernel_time(spv_sys* s, int32_t which, double* total_ms, int64_t* launches);

/*
 * Trajectory adjoint (single FP64 system).  Gradient of the time-averaged
 * mean shape index Q = (1/T) sum_{t=1..T} qbar(r_t), qbar = mean P_i/sqrt(A_i),
 * with respect to the per-cell target shape index p0_i (P0_i = p0_i sqrt(A0_i)).
 *
 * spv_traj_forward runs T steps from the current state (noise counter
 * continuing), checkpointing the full state every ckpt_every steps, and
 * returns Q.  spv_traj_backward(dQ) recomputes every segment from its
 * checkpoint (bit-reproducibly, with the same topology) and propagates the
 * adjoint backwards: lambda_{t-1} = lambda_t + dt mu dF(r_{t-1})[lambda_t]
 * (+ dQ/dr_{t-1}), dQ/dP0 += dt mu 2 K_P dP(r_{t-1})[lambda_t], where dF[v] =
 * -H v is the Hessian-vector product of Eq. 1 through the Voronoi geometry
 * with the recorded topology (App. A/B derivatives in forward-mode tangent
 * arithmetic).  The quantisation of positions is not differentiated.
 * dQ_dp0 receives dQ * dQ/dp0 (N entries, tag order, host or device).
 * The handle ends in the state reached by spv_traj_forward.  Any spv_step
 * between the two calls invalidates the record (SPV_EINVAL).
 */
spv_status spv_traj_forward(spv_sys* s, int64_t T, int64_t ckpt_every, double* Q);
spv_status spv_traj_backward(spv_sys* s, double dQ, double* dQ_dp0);

/*
 * Directional derivative of the forces along v at the current state with the
 * current topology: dF[v] = -H v (Hessian-vector product of Eq. 1), tag
 * order (v and the result: N entries per component).  FP64 handles.
 */
spv_status spv_force_tangent(spv_sys* s, const double* vx, const double* vy, double* fx, double* fy);

/*
 * spv_force_tangent for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and result, with their scratch (v and the result in memory order,
 * the tangents of A and P) in a static device array of the library instead
 * of handle buffers, and no host staging.  No hipMalloc, hipFree or host
 * synchronisation: the result is written on the handle's stream.
 *   vx, vy, fx, fy: device pointers (N entries each, tag order); host
 *   pointers are SPV_EINVAL.
 * Limit: N <= 65536 cells (3 MiB of scratch per device, held until the
 * process ends); larger handles are SPV_EINVAL.  Every call on one device
 * shares that scratch: calls that overlap on one GPU (different streams or
 * threads) race.  Single FP64 systems, as spv_force_tangent.
 */
spv_status spv_force_tangent_static(spv_sys* s, const double* vx, const double* vy, double* fx, double* fy);

/* Release all device state of the handle. */
spv_status spv_destroy(spv_sys* s);

/* ====================================================================== */
/*
 * Active vertex model (AVM; Sec. II.A Eq. 4, Sec. II.D, App. A).  The
 * degrees of freedom are the vertices h_v of a trivalent polygonal tiling of
 * the periodic box (every vertex in exactly three cells; Nv = 2 Nc on the
 * torus); the energy is Eq. 1 over the polygons' areas and perimeters, the
 * force F_v = -dE/dh_v (App. A, with dP/dh = t_in - t_out: incoming minus
 * outgoing unit edge vector), and the vertices move by Eq. 4:
 *   dh_v/dt = mu F_v + (v0 / 3) sum of n_c over the three cells at v,
 * the cell directors n_c = (cos theta_c, sin theta_c) rotating with white
 * noise of variance 2 Dr (Philox4x64-10, counter (step, cell label)).  After
 * every move, T1 transitions (Sec. II.D): an edge shorter than t1_length
 * is replaced by its perpendicular of length t1_new_length through the same
 * midpoint, so that the two cells that shared it lose a vertex and the two
 * cells at its ends become neighbours; an edge qualifies only when both
 * cells sharing it have more than three vertices and the end cells share no
 * vertex yet; at most one transition per cell in a round (an edge flips
 * when its key (smaller vertex label, larger vertex label) is the smallest
 * among the qualifying edges at its four cells); rounds repeat until no
 * edge qualifies.  Vertices are kept on the grid 2^-q of the box (as the
 * Voronoi model's cells) and the T1 test is dx*dx + dy*dy < t1_length^2 on
 * exact differences, evaluated without fused operations.  FP64.
 *
 * Labels are the indices the caller created vertices and cells with; every
 * read-out is in label order.  The library keeps vertices and cells in its
 * own memory order (Sec. II.B spatial sorting: bins of about one cell ranked
 * along a Hilbert curve, re-sorted every resort_every steps) and nothing a
 * result depends on is taken from that order, so results are bitwise the
 * same for every resort_every and bin_order.
 */
typedef struct {
    double KA, KP, mu, v0, Dr, dt;  /* as spv_params */
    uint64_t seed;                  /* noise key */
    double t1_length;               /* T1 threshold (> 0) */
    double t1_new_length;           /* length of the edge a T1 creates (0: 1.5 t1_length; must exceed it) */
    int32_t resort_every;           /* steps between spatial re-sorts (also one at creation);
                                       0: 1000; -1: never (memory order stays the caller's) */
    int32_t bin_order;              /* 0: bins along a Hilbert curve; 1: row by row */
} spv_avm_params;

typedef struct spv_avm spv_avm;

/*
 * Create from a polygon network: Nv vertices at (vx, vy) in [0,Lx) x [0,Ly),
 * Nc cells whose vertex lists are cell_vtx[cell_off[c] .. cell_off[c+1]),
 * counter-clockwise (3 to 16 vertices each; cell_off has Nc + 1 entries).
 * A0, P0, p0, theta0 as spv_create (theta0 NULL: 2 pi u with u from Philox
 * counter (2^64 - 1, c)).  Host or device pointers, read during the call.
 * Errors: SPV_EINVAL (not a trivalent, consistently oriented network; Nv !=
 * 2 Nc; bad parameters or positions; resort_every < -1; bin_order not 0 or
 * 1), SPV_ENOMEM, SPV_EHIP.
 */
spv_status spv_avm_create(spv_avm** out, int64_t Nc, int64_t Nv, const double* vx, const double* vy,
                          const int32_t* cell_off, const int32_t* cell_vtx, double Lx, double Ly, const double* A0,
                          const double* P0, double p0, const double* theta0, const spv_avm_params* params,
                          void* stream);
/* nsteps steps (three T1 rounds per step on the device, more from the host
 * when needed; batches of 8 steps replay a captured HIP graph); errors:
 * SPV_ENONFINITE, SPV_ECAPACITY (a T1 would give a cell more than 16
 * vertices), SPV_EREPAIR (T1 rounds did not settle within 64 rounds of a
 * step); the handle then keeps returning the error. */
spv_status spv_avm_step(spv_avm* h, int64_t nsteps);
spv_status spv_avm_get_vertices(spv_avm* h, double* vx, double* vy);       /* Nv each */
spv_status spv_avm_get_forces(spv_avm* h, double* fx, double* fy);         /* at the current state */
spv_status spv_avm_get_directors(spv_avm* h, double* theta);               /* Nc */
spv_status spv_avm_get_geometry(spv_avm* h, double* A, double* P);         /* Nc each */
/* current topology: cell_off (Nc + 1 entries) and the counter-clockwise
 * vertex lists (cap entries; *needed = 3 Nv); SPV_ECAPACITY if cap is
 * smaller (cell_off is still written).  Host pointers. */
spv_status spv_avm_get_cells(spv_avm* h, int32_t* cell_off, int32_t* cell_vtx, int64_t cap, int64_t* needed);
/* E (Eq. 1), qbar = mean P/sqrt(A); counters[6] (may be NULL): steps, T1
 * transitions, T1 rounds with transitions, rounds run from the host,
 * batches replayed from a captured graph, re-sorts */
spv_status spv_avm_get_observables(spv_avm* h, double* E, double* qbar, int64_t* counters);
spv_status spv_avm_destroy(spv_avm* h);

/*
 * The polygon network of a Voronoi system's current tessellation (its
 * Voronoi cells: one vertex per Delaunay triangle at its circumcentre), the
 * usual start of an active vertex model (single systems).  Vertices are
 * numbered by first appearance, cells visited in tag order and each ring
 * from its smallest-tag neighbour; a vertex's position is its circumcentre
 * in the frame of its smallest-tag cell, wrapped into the box and put on the
 * grid 2^-q.  Host arrays: vx, vy (2N), cell_off (N + 1), cell_vtx (6N).
 */
spv_status spv_voronoi_network(spv_sys* s, double* vx, double* vy, int32_t* cell_off, int32_t* cell_vtx);

/* Message for the last non-OK status returned on this thread. */
const char* spv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPV_H */
