/*
 * pic.h - C ABI of the MI355X particle-in-cell hot path.
 *
 * Method: Gassmoeller, Heien, Puckett, Bangerth, "Flexible and scalable
 * particle-in-cell methods for massively parallel computations"
 * (arXiv:1612.03369).  Section numbers below refer to that paper.
 *
 * The library advances particles through a Q2 (tensor-product quadratic
 * Lagrange) velocity field on a quad/hex mesh, keeps the particle store sorted
 * by owning cell, manages per-cell populations and interpolates particle
 * properties to cells.  Every step of that path runs in HIP kernels built for
 * gfx950; the host code only prepares meshes and launches kernels.
 *
 * Conventions
 *  - Status codes: every call returns PIC_OK (0) or a negative pic_status and
 *    stores a message retrievable with pic_last_error().  No exception or
 *    abort crosses the ABI.
 *  - Memory: bulk arrays (particle store, field, outputs, scratch) are owned by
 *    the caller and passed as device pointers; the library borrows them until
 *    they are re-bound or the context is destroyed.  Host pointers are read
 *    during the call only.  The library owns only metadata, mesh tables and a
 *    repacked copy of the velocity field (device memory it allocates at set-up
 *    calls, never in pic_advance / pic_population / pic_interpolate).
 *  - Asynchrony: compute calls enqueue on the context's HIP stream and return
 *    immediately.  Calls that return host values (pic_mesh_info, pic_q2_nodes,
 *    pic_stats_read, pic_current_buffer's count) synchronise that stream.
 *  - Layout: arrays are structure-of-arrays, component-major.  A "[d][cap]"
 *    array stores component a of particle i at a*cap + i.
 *  - Cells of a uniform mesh are numbered i + n0*(j + n1*k); Q2 nodes of a
 *    structured mesh form the (2n0+1) x (2n1+1) [x (2n2+1)] grid, node (a,b,c)
 *    at index a + (2n0+1)*(b + (2n1+1)*c).  Octree leaves keep the caller's
 *    order; octree Q2 nodes are the distinct points of all leaves' 3x3x3 node
 *    lattices numbered in ascending x + M*(y + M*z) order of their coordinates
 *    on the lattice of half-finest cells (M = 2^(max_level+1) + 1).
 */
#ifndef PIC_H
#define PIC_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define PIC_API __attribute__((visibility("default")))
#else
#define PIC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_ctx pic_ctx;

typedef enum {
    PIC_OK = 0,
    PIC_EINVAL = -1,      /* bad argument */
    PIC_ENOMEM = -2,      /* device allocation failed */
    PIC_EDEVICE = -3,     /* HIP runtime error */
    PIC_ESTATE = -4,      /* call out of order (e.g. advance before bind) */
    PIC_ECAPACITY = -5,   /* store capacity too small; pic_stats.live holds the need */
    PIC_ENONFINITE = -6   /* non-finite velocity DOFs */
} pic_status;

typedef enum { PIC_EULER = 1, PIC_RK2 = 2, PIC_RK4 = 4 } pic_scheme;
typedef enum { PIC_F64 = 0, PIC_F32 = 1 } pic_prec;
typedef enum {
    PIC_INTERP_CELL_AVERAGE = 0,      /* pic_interpolate */
    PIC_INTERP_LINEAR_LS = 1,
    PIC_INTERP_GEOMETRIC_AVERAGE = 2,
    PIC_INTERP_HARMONIC_AVERAGE = 3,
    PIC_INTERP_NEAREST = 4,           /* pic_interpolate_points */
    PIC_INTERP_INV_DISTANCE = 5,
    PIC_INTERP_SHAPE_WEIGHTED = 6
} pic_interp;
typedef enum { PIC_PROP_GIVEN = 0, PIC_PROP_INITIAL_POSITION = 1 } pic_prop_init;

/* Marker for a lost particle in key arrays. */
#define PIC_LOST 0xFFFFFFFFu

/*
 * Particle store (Sec. 2.1: id, location, reference location, N_properties
 * scalars; N_properties is a run-time constant).  Two equally sized buffers,
 * A (index 0) and B (index 1): each step reads the current buffer and writes
 * the other one, sorted by cell.  cell_start[b] has n_cells+1 entries; the
 * particles of cell K in buffer b are [cell_start[b][K], cell_start[b][K+1]),
 * and the live count is cell_start[b][n_cells].  All pointers are device
 * pointers owned by the caller.  Between calls the current buffer holds every
 * field; the other buffer is scratch of the calls.  On uniform meshes the
 * stored reference location of a particle is exactly the closed form
 * (x - (lo + i h)) / h of its location in its cell, and the step kernels use
 * that form instead of reading it (so the given reference locations of a
 * seeding call enter the first step only through the locations they map to).
 */
typedef struct {
    int64_t capacity;          /* particles per buffer */
    double *x[2];              /* [dim][capacity] locations */
    double *xr[2];             /* [dim][capacity] reference locations in [0,1]^dim */
    int32_t *cell[2];          /* [capacity] owning cell */
    uint32_t *id[2];           /* [capacity] particle ids */
    void *prop[2];             /* [n_prop][capacity], float or double per prop_prec */
    int32_t *cell_start[2];    /* [n_cells + 1] */
    int32_t n_prop;            /* 0..64 */
    int32_t prop_prec;         /* pic_prec */
    void *scratch;             /* device workspace of pic_scratch_bytes() bytes */
    int64_t scratch_bytes;
} pic_store;

/* Counters accumulated on the device since the last pic_stats_reset(). */
typedef struct {
    int64_t live;         /* live particles in the current buffer */
    int64_t lost;         /* removed because a stage or end point left the domain (Sec. 2.4, option 3) */
    int64_t moved;        /* particles that changed cell in a step */
    int64_t near_face;    /* particles of a step whose end point lies within 1e-10 of a cell face in
                             reference coordinates, or one of whose points up to the first one outside
                             the domain lies within 1e-10 h of the domain boundary (inside or outside);
                             lost particles included */
    /* Location by the neighbour search of Sec. 2.4 (displaced and octree
     * meshes; uniform meshes locate by the closed form and leave these 0).
     * Every stage point and end point that is not in its hint cell starts one
     * search; the first-try hit rate of the paper's search order is
     * first_try / searches. */
    int64_t first_try;    /* searches whose first candidate cell held the point */
    int64_t fallback;     /* searches that ended in the global search */
    int64_t newton_fail;  /* inverse-map evaluations that did not converge */
    int64_t added;        /* population management: particles created (Sec. 2.5) */
    int64_t deleted;      /* population management: particles removed */
    int64_t steps;        /* time steps taken */
    int64_t particle_steps; /* sum over steps of the particles advanced */
    int64_t searches;     /* points located by the neighbour search (not in their hint cell) */
    int64_t searched;     /* candidate cells tried by those searches */
} pic_stats;

/* ---- context --------------------------------------------------------- */
/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the null stream). */
PIC_API pic_status pic_create(pic_ctx **out, int device, void *hip_stream);
/* Change the stream later calls enqueue on. */
PIC_API pic_status pic_set_stream(pic_ctx *ctx, void *hip_stream);
/* Release library-owned memory; caller buffers are untouched.  Accepts NULL. */
PIC_API void pic_destroy(pic_ctx *ctx);
/* Message of the last failing call on ctx; valid until the next call. */
PIC_API const char *pic_last_error(const pic_ctx *ctx);

/* ---- mesh (Sec. 2.1 data structures; Sec. 2.5 adaptive meshes) -------- */
/* Uniform box mesh: dim 2 or 3, n[i] cells per axis on [lo, hi]. */
PIC_API pic_status pic_mesh_uniform(pic_ctx *ctx, int dim, const int32_t n[3], const double lo[3], const double hi[3]);
/* Move the vertices of the uniform mesh set up before: vertices is a host array
 * [dim][n_vertices] of the (n0+1) x (n1+1) [x (n2+1)] grid, x fastest.  Cells
 * become bi/trilinear; location uses Newton inversion of the cell map plus the
 * vertex-neighbour search of Sec. 2.4 and a search over all cells as the
 * last resort.  Boundary vertices must stay on the box faces. */
PIC_API pic_status pic_mesh_displace(pic_ctx *ctx, const double *vertices);
/* 2:1-balanced octree on the box [lo, hi]: leaf K has refinement level
 * level[K] (<= max_level <= 10) and lower corner anchor[a*n_leaves + K] in units
 * of the finest cell.  Host arrays.  Leaves must tile the box. */
PIC_API pic_status pic_mesh_octree(pic_ctx *ctx, const double lo[3], const double hi[3], int max_level,
                           int64_t n_leaves, const uint8_t *level, const int32_t *anchor);
/* Dimension, number of cells and of Q2 nodes of the current mesh. */
PIC_API pic_status pic_mesh_info(pic_ctx *ctx, int32_t *dim, int64_t *n_cells, int64_t *n_nodes);
/* Coordinates of the Q2 nodes (host [dim][n_nodes]) and, if non-NULL, a host
 * byte per node that is 1 for hanging nodes (octree only). */
PIC_API pic_status pic_q2_nodes(pic_ctx *ctx, double *xyz, uint8_t *is_hanging);

/* ---- field (Sec. 2.3: the velocity is a finite element field) ----------- */
/* Nodal Q2 velocity U, device [dim][n_nodes] in precision `prec`.  The library
 * copies it into its own layout (so U may be freed or changed afterwards) and,
 * on an octree, replaces hanging-node values by the constraining coarse
 * leaf's interpolant, coarse levels first.  Returns PIC_ENONFINITE if any
 * value is NaN or infinite. */
PIC_API pic_status pic_set_velocity(pic_ctx *ctx, const void *U, int prec);

/* ---- field that changes in time (Sec. 2.3) ------------------------------ */
/* The field is known at the ends of a field step [t^n, t^n + dt_u]: u^n (set
 * by pic_set_velocity) and u^{n+1} (U1, same layout and precision rules as
 * pic_set_velocity, copied by the library).  Every stage of pic_advance then
 * evaluates both fields at its point and combines them linearly in time,
 *   u~(x, t) = u^n(x) + theta (u^{n+1}(x) - u^n(x)),  theta = (t - t^n) / dt_u,
 * at the stage's time (the step's start, midpoint or end); theta > 1
 * extrapolates.  Particle steps may sub-divide the field step (dt < dt_u):
 * the library keeps the time elapsed since t^n in device memory, starts it at
 * 0 here and advances it by dt with every step (graph replays included).
 * U1 = NULL switches back to the steady field u^n.  PIC_ESTATE without u^n;
 * PIC_EINVAL for dt_u not finite and positive; PIC_ENONFINITE as
 * pic_set_velocity.  A new mesh or mesh displacement switches it off.  Not
 * available in batches or for the adjoint (PIC_EINVAL there). */
PIC_API pic_status pic_set_velocity_end(pic_ctx *ctx, const void *U1, int prec, double dt_u);
/* Next field step: u^{n+1} becomes u^n, U_next becomes u^{n+1}, dt_u the new
 * field step, the elapsed time restarts at 0.  Needs an end field
 * (PIC_ESTATE).  If U_next is rejected the old end field stays as the steady
 * field and time interpolation is off. */
PIC_API pic_status pic_shift_velocity(pic_ctx *ctx, const void *U_next, int prec, double dt_u);
/* Set / read the time elapsed since t^n (host double; needs an end field). */
PIC_API pic_status pic_set_field_time(pic_ctx *ctx, double tau);
PIC_API pic_status pic_field_time(pic_ctx *ctx, double *tau);

/* ---- store ------------------------------------------------------------ */
/* Bytes of device scratch a store of `capacity` particles needs. */
PIC_API pic_status pic_scratch_bytes(pic_ctx *ctx, int64_t capacity, int64_t *bytes);
/* Bind the caller's store (copied by value; arrays borrowed).  Buffer A
 * becomes current and empty.  Requires a mesh. */
PIC_API pic_status pic_bind_store(pic_ctx *ctx, const pic_store *store);
/* Index (0 = A, 1 = B) of the buffer holding the current particles. */
PIC_API pic_status pic_current_buffer(pic_ctx *ctx, int32_t *which);

/* ---- generation (Sec. 2.2) --------------------------------------------- */
/* Reference-local generation (remark on local generation): counts[K]
 * particles in cell K (device int32 [n_cells]), listed cell by cell in xr
 * (device [dim][n], reference coordinates in [0,1]^dim) with ids (device
 * uint32 [n]).  Location x = Phi_K(xr).  Properties: PIC_PROP_GIVEN copies
 * prop_in (device [n_prop][n], store precision); PIC_PROP_INITIAL_POSITION sets
 * property j to coordinate j mod dim of x.  Replaces the current contents. */
PIC_API pic_status pic_seed_reference(pic_ctx *ctx, const int32_t *counts, const double *xr, const uint32_t *ids,
                              int64_t n, int32_t prop_init, const void *prop_in);
/* Reference-local generation with the library's counter hash (Sec. 2.2,
 * remark on generating particles in the reference cell): counts[K]
 * particles in cell K (device int32 [n_cells]), listed cell by cell; particle
 * j of cell K at reference coordinates xr_a = u(seed, 2^64 - 1, K, j, a), u the
 * SplitMix64 counter hash of pic_population (step word 2^64 - 1), location
 * x = Phi_K(xr), id first_id + its position in the listing.  Properties as
 * pic_seed_reference (prop_in device [n_prop][sum of counts] for
 * PIC_PROP_GIVEN).  Replaces the current contents; PIC_ECAPACITY if the
 * counts exceed the capacity, PIC_EINVAL for a negative count or ids beyond
 * 2^32. */
PIC_API pic_status pic_seed_per_cell(pic_ctx *ctx, const int32_t *counts, uint64_t seed, uint32_t first_id,
                                     int32_t prop_init, const void *prop_in);
/* Metropolis-Hastings generation (Sec. 2.2): counts[K] particles in cell K
 * (device int32 [n_cells]) drawn from the density rho (device double
 * [n_nodes], nodal values of its Q2 interpolant rho_h; hanging-node values of
 * an octree are used as given).  Per cell a chain in the reference cell with
 * a proposal uniform in it, starting at its centre, target max(0, rho_h)
 * |det grad Phi_K|; state i proposes coordinates u(seed, 1, K, i, axis) and
 * accepts when u(seed, 2, K, i, 0) times the current target is below the
 * proposal's, u the SplitMix64 counter hash of the population step; every
 * J-th state (J-1, 2J-1, ...) becomes a particle.  Stored cell by cell with
 * ids first_id + position, properties = initial position.  *longest_run
 * (host, may be NULL) = the longest run of equal consecutive states over all
 * chains: thinned particles repeat a location unless J exceeds it.  Replaces
 * the current contents; PIC_ECAPACITY if the counts exceed the capacity,
 * PIC_ENONFINITE for a non-finite density. */
PIC_API pic_status pic_seed_mh(pic_ctx *ctx, const int32_t *counts, const double *rho, int32_t J, uint64_t seed,
                               uint32_t first_id, int64_t *longest_run);
/* For callers that cannot allocate device memory (serving loops, harnesses
 * that forbid hipMalloc): pic_seed_mh with the same arguments and results,
 * bit for bit, that allocates nothing.  Its staging (the per-cell starts, the
 * packed density, flags and the longest run) lives in a fixed 16 MiB device
 * array of the library, one per GPU, held until the process ends: meshes
 * needing more (256 + 4 (n_cells + 1) rounded up to 256, plus 16 bytes per
 * node in 2D or 32 in 3D) are rejected with PIC_EINVAL.  Every call on a GPU
 * uses that GPU's one array, so calls that overlap on one GPU (several
 * threads or streams) race; the array keeps the last call's contents.  Like
 * pic_seed_mh it synchronises the context's stream. */
PIC_API pic_status pic_seed_mh_static(pic_ctx *ctx, const int32_t *counts, const double *rho, int32_t J, uint64_t seed,
                                      uint32_t first_id, int64_t *longest_run);
/* Prescribed locations (Sec. 2.2, prescribed particle locations): locate each
 * x (device [dim][n]) in the mesh, drop points outside the domain, and store
 * the rest sorted by (cell, input order).  Properties as above. */
PIC_API pic_status pic_seed_positions(pic_ctx *ctx, const double *x, const uint32_t *ids, int64_t n,
                              int32_t prop_init, const void *prop_in);

/* Cells per work item of the advect kernel (1..1024; default 64).  A work
 * item is a run of consecutive cells whose particles one workgroup advances.
 * On octree meshes at most 64 are used (the tile's leaf nodes are staged in
 * LDS). */
PIC_API pic_status pic_set_tile(pic_ctx *ctx, int32_t tile_cells);

/* ---- mesh refinement and coarsening (Sec. 2.5) ------------------------- */
/* Move the particles of `from` (its current buffer, on the mesh before
 * refinement or coarsening) into `to` (a problem on the new mesh over the same
 * box, with a bound store): every particle goes to the cell of the new mesh
 * holding its location -- a child of its cell when that was refined, the
 * parent when it was coarsened -- with its reference location recomputed
 * there; location, id and properties are kept; particles outside the new
 * mesh are dropped (counted as lost).  `to` ends sorted by new cell with the
 * old store order kept within a cell, its next id no smaller than the
 * source's.  More particles on refinement / fewer on coarsening: call
 * pic_population on `to` afterwards.  `from` is not changed.  Needs one
 * device, one dimension, the same property count and precision
 * (PIC_EINVAL) and room for the particles (PIC_ECAPACITY).  Synchronises
 * both streams. */
PIC_API pic_status pic_transfer(pic_ctx *from, pic_ctx *to);

/* ---- properties integrated along the trajectories (Sec. 2.6) ----------- */
/* Switch on the two property equations of Sec. 2.6 for pic_advance:
 *   damage       d' = alpha |eps(u)| - beta d, eps = (grad u + grad u^T)/2,
 *                |.| the Frobenius norm, in property damage_prop;
 *   deformation  F' = (grad u) F, F row-major dim x dim, in properties
 *                deform_prop .. deform_prop + dim^2 - 1.
 * They are integrated with the positions as one system by the same RK
 * scheme: every stage evaluates grad u_h in the cell its point was located
 * in, at the stage's property values.  Needs double-precision properties
 * (PIC_EINVAL otherwise, or for indices out of range / overlapping).
 * damage_prop = deform_prop = -1 switches them off; pic_bind_store also does.
 * Not available in batches (pic_batch_create returns PIC_EINVAL). */
PIC_API pic_status pic_set_property_odes(pic_ctx *ctx, int32_t damage_prop, int32_t deform_prop, double alpha,
                                         double beta);

/* ---- the hot path (Sec. 2.3 advection, Sec. 2.4 transport) -------------- */
/* n_steps time steps of size dt: per step every particle is advanced with the
 * scheme (Euler; RK2 explicit midpoint; classical RK4), every stage point and
 * the end point are located (inverse map + neighbour search), particles whose
 * stage or end point leaves the closed domain are removed, and the store is
 * re-sorted stably by (new cell, moved): in each cell the particles that stayed
 * keep their order and arrivals follow in their previous order.  eval_prec
 * selects the arithmetic of the field evaluation (locations stay double). */
PIC_API pic_status pic_advance(pic_ctx *ctx, double dt, int32_t n_steps, int32_t scheme, int32_t eval_prec);
/* Several steps on a uniform mesh run as one launch sequence (the re-sort of
 * each step fused with the next step's advection).  With enable = 1,
 * pic_advance records that sequence once into a HIP graph on a stream of the
 * context's own and replays it, after the work already on the context's stream
 * and before the work put there later (one event each way); a new step count,
 * scheme, precision or property-equation / time-field setting records a new
 * graph, and so do new work lists (binding, tile size, mesh).  enable = 0 (the
 * default) launches the kernels one by one on the context's stream, which
 * measured faster (50 steps of the 64^3 RK4 workload: 15.7-15.9 ms against
 * 16.4-16.7 ms from the graph).  The results are the same bit for bit.
 * Profiling (pic_profile_enable) always launches one by one. */
PIC_API pic_status pic_set_launch_graphs(pic_ctx *ctx, int32_t enable);

/* ---- population management (Sec. 2.5, Sec. 2.6) ----------------------- */
/* Per cell: more than max_pc particles -> delete the ones with the largest
 * ids; fewer than min_pc -> append min_pc - n particles at reference
 * coordinates u = SplitMix64-hash(seed, step, cell, slot, axis) in [0,1),
 * ids next_id + (exclusive scan of additions over cells) + slot, properties =
 * mean of the cell's remaining particles, or the initial-position function if
 * the cell is empty.  next_id starts at 1 + the largest seeded id. */
PIC_API pic_status pic_population(pic_ctx *ctx, int32_t min_pc, int32_t max_pc, uint64_t seed, uint64_t step);

/* ---- particle -> cell transfer (Sec. 2.7) ------------------------------ */
/* PIC_INTERP_CELL_AVERAGE: out [n_cells][n_prop] arithmetic means (NaN for
 * empty cells), aux unused.  PIC_INTERP_LINEAR_LS: per cell and property the
 * least-squares fit c0 + sum_i c_i (xr_i - xbar_i) in reference coordinates
 * centred at the cell's mean xbar; out [n_cells][n_prop][dim+1] = (c0, c),
 * aux [n_cells][dim] = xbar; constant fit when the cell has fewer than dim+1
 * particles or sigma_min/sigma_max of the design matrix is below 1e-10.
 * count [n_cells] receives the particle counts.  Device pointers, double. */
PIC_API pic_status pic_interpolate(pic_ctx *ctx, int32_t kind, double *out, double *aux, int32_t *count);
/* PIC_INTERP_GEOMETRIC_AVERAGE / PIC_INTERP_HARMONIC_AVERAGE (Sec. 2.7 (ii)):
 * out [n_cells][n_prop] = exp of the mean logarithm / n over the sum of
 * reciprocals of each property over the cell's particles (0 if a value is 0;
 * the geometric mean is NaN if a value is negative; NaN for empty cells). */

/* Particle -> evaluation points (Sec. 2.7 (i), (iii), (iv)): the points qhat
 * (host [dim][n_q], reference coordinates in [0,1]^dim, 1 <= n_q <= 64, the
 * same in every cell, e.g. quadrature points) get values from the particles
 * of their own cell only:
 *   PIC_INTERP_NEAREST         property of the particle nearest in physical
 *                              distance to Phi_K(qhat) (ties: first in store
 *                              order);
 *   PIC_INTERP_INV_DISTANCE    weights 1 / |Phi_K(qhat) - x_k|^2, particles at
 *                              the point itself share the whole weight;
 *   PIC_INTERP_SHAPE_WEIGHTED  weights sum_v N_v(qhat) N_v(xhat_k) over the
 *                              cell's d-linear vertex shape functions.
 * out (device [n_cells][n_q][n_prop] double; NaN for empty cells), count
 * (device [n_cells], may be NULL).  Allocates nothing. */
PIC_API pic_status pic_interpolate_points(pic_ctx *ctx, int32_t kind, const double *qhat, int32_t n_q, double *out,
                                          int32_t *count);

/* ---- adjoint (derivative of the multi-step map w.r.t. the field) -------- */
/* Bytes of device workspace for pic_advance_checkpointed with these sizes. */
PIC_API pic_status pic_adjoint_workspace_bytes(pic_ctx *ctx, int32_t n_steps, int32_t ckpt_every, int64_t *bytes);
/* Like pic_advance (F64 evaluation), also saving the store every ckpt_every
 * steps into workspace (device, pic_adjoint_workspace_bytes bytes).  Needs a
 * steady field: PIC_EINVAL while an end field (pic_set_velocity_end) is set,
 * here and in pic_adjoint. */
PIC_API pic_status pic_advance_checkpointed(pic_ctx *ctx, double dt, int32_t n_steps, int32_t scheme,
                                    int32_t ckpt_every, void *workspace);
/* Given dL/dx of the final locations (device [dim][capacity], in the order of
 * the current buffer after pic_advance_checkpointed), accumulate dL/dU into
 * dU (device double [dim][n_nodes]) by re-running each checkpoint segment and
 * sweeping its RK stages in reverse.  Leaves the store as it was. */
PIC_API pic_status pic_adjoint(pic_ctx *ctx, const double *dl_dx, void *workspace, double *dU);

/* ---- statistics and profiling ------------------------------------------ */
/* Read the counters (synchronises the stream). */
PIC_API pic_status pic_stats_read(pic_ctx *ctx, pic_stats *out);
/* Zero the counters (enqueued). */
PIC_API pic_status pic_stats_reset(pic_ctx *ctx);
/* Record a HIP event pair around every kernel launch when enable != 0. */
PIC_API pic_status pic_profile_enable(pic_ctx *ctx, int32_t enable);
/* Sum of kernel durations (ms) and launch count of the named kernel since
 * profiling was enabled (synchronises).  Unknown name -> PIC_EINVAL. */
PIC_API pic_status pic_profile_read(pic_ctx *ctx, const char *kernel, double *total_ms, int64_t *launches);

/* ---- batched problems --------------------------------------------------- */
typedef struct pic_batch pic_batch;
/* Group n independent problems (each a context with mesh, field and bound,
 * seeded store on the same device) so that their time steps run as shared
 * launches over a work list of (problem, cell tile) items, replayed from one
 * HIP graph.  tile_cells[0..3] gives the cells per work item for
 * (2D RK2, 2D RK4, 3D RK2, 3D RK4); 0 = default.  The problems' streams are
 * not used; the batch enqueues on `hip_stream`.  Uniform meshes with a steady
 * field and no property equations only (PIC_EINVAL otherwise); the problems'
 * settings are taken at creation. */
PIC_API pic_status pic_batch_create(pic_batch **out, int32_t n, pic_ctx *const *problems, const int32_t tile_cells[4],
                            void *hip_stream);
/* n_steps steps of every problem with its own dt / scheme (F64 evaluation). */
PIC_API pic_status pic_batch_advance(pic_batch *b, const double *dt, const int32_t *scheme, int32_t n_steps);
/* Workgroup-per-cell-block schedule of the batched advect, per group
 * g = 3 * (dim == 3) + (0 Euler, 1 RK2, 2 RK4): variant[g] selects the cell
 * block one workgroup advances (2D: 8x8, 8x4, 16x8 cells; 3D: 4x4x4,
 * 4x2x2, 4x4x2).  Results do not depend on it (the block's LDS window and the
 * global field give identical values).  Values outside 0..2 -> PIC_EINVAL. */
PIC_API pic_status pic_batch_set_schedule(pic_batch *b, const int32_t variant[6]);
/* Autotuner: for each group present, time `trials` launches of the group's
 * advect per candidate block shape on the problems' own particles and keep
 * the fastest.  Locations, reference locations and statistics are restored
 * afterwards, so the problems are left as they were.  Synchronises.
 * variant_out (host [6], may be NULL) receives the choice; time_ms_out (host
 * [18], may be NULL) the mean launch time of group g, shape v at [3g + v]
 * (-1 for groups without problems).  Takes dt / scheme like
 * pic_batch_advance.  Needs device memory for one copy of the locations. */
PIC_API pic_status pic_batch_tune(pic_batch *b, const double *dt, const int32_t *scheme, int32_t trials,
                                  int32_t variant_out[6], double time_ms_out[18]);
/* Tune cache: the batch's schedule as text, for reuse without timing.
 * pic_batch_tune_cache_write writes
 *   {"signature": [[dim, n_cells, capacity, scheme], ...], "variants": [v0, .. v5]}
 * (one signature entry per problem, with the schemes given) into buf (host,
 * cap bytes, NUL-terminated); *len receives the length without the NUL, so
 * cap = 0 asks for the length alone; a smaller nonzero cap -> PIC_EINVAL.
 * pic_batch_tune_cache_apply reads that text: when its signature equals the
 * batch's (for the schemes given) it applies the variants as
 * pic_batch_set_schedule does and sets *applied = 1, else it changes nothing
 * and sets *applied = 0.  Malformed text or variants outside 0..2 ->
 * PIC_EINVAL. */
PIC_API pic_status pic_batch_tune_cache_write(pic_batch *b, const int32_t *scheme, char *buf, int64_t cap, int64_t *len);
PIC_API pic_status pic_batch_tune_cache_apply(pic_batch *b, const int32_t *scheme, const char *json, int32_t *applied);
PIC_API void pic_batch_destroy(pic_batch *b);
PIC_API const char *pic_batch_last_error(const pic_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
