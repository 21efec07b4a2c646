/*
 * mdlts.h -- C ABI of the MI355X (gfx950) library for the explicit SIPG-DG
 * monodomain step under synchronous local time stepping.
 *
 * Method: Ogiermann, Balzani, Perotti, "An Explicit Local Space-Time Adaptive
 * Framework for Monodomain Models in Cardiac Electrophysiology",
 * arXiv:2310.07607.  Problem statement: Sec. 2 (monodomain model with
 * homogeneous Neumann boundary, D = kappa/(chi C_m), I = I'/C_m); spatial
 * discretisation: Sec. 2.1; adaptivity: Sec. 2.2; synchronous LTS: Sec. 2.3
 * and Algorithm 1.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every function returns an mdlts_status; MDLTS_OK (0) on success.  No
 *    function aborts, prints, or retains a host pointer after it returns.
 *    No C++ exception leaves the library: a failed host allocation inside a
 *    call returns MDLTS_ENOMEM, any other host-side exception MDLTS_EDEVICE.
 *  - Host arrays are owned by the caller and copied during the call.
 *  - Device memory comes from the allocator given to mdlts_ctx_create and is
 *    used on the context's stream.  A caller without an allocator (plain C)
 *    passes NULL, and the library then calls hipMalloc/hipFree itself.
 *  - Mesh: an axis-aligned box [0,len0]x[0,len1](x[0,len2]) split into a root
 *    grid n0 x n1 (x n2) of boxes ("root elements", Sec. 2.2); each root is
 *    the root of a 2^d-tree.  Root id = rx + n0*(ry + n1*rz).  Child index =
 *    bx | by<<1 | bz<<2 (bit k set: upper half in dimension k).
 *  - Canonical leaf order: roots in id order, pre-order inside each tree.
 *  - Element nodes: tensor Gauss-Legendre nodes of degree `order`, node index
 *    ix + m*iy + m*m*iz with m = order+1 (x fastest).  State vectors are
 *    [leaf][node] in canonical leaf order, FP64 at this ABI.
 *  - Refine-bit stream: pre-order over every node of every tree, roots in id
 *    order, one byte per node: 1 = refined (its 2^d children follow in child
 *    index order), 0 = leaf.  Trees must be 2:1 balanced across faces.
 *  - Units: cm, ms; u (transmembrane potential) and v (gate) dimensionless.
 *  - Thread safety: one context per host thread; calls on one context are
 *    serialised by the caller.
 */
#ifndef MDLTS_H
#define MDLTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MDLTS_OK = 0,
    MDLTS_EINVAL = 1,     /* bad argument, size, or mesh */
    MDLTS_ENOMEM = 2,     /* device allocation failed */
    MDLTS_EDEVICE = 3,    /* a HIP call or kernel failed */
    MDLTS_EUNSTABLE = 4,  /* a leaf needs more LTS levels than configured, or non-finite state */
    MDLTS_ESTATE = 5,     /* call out of order (e.g. step before assign_levels) */
    MDLTS_EBUSY = 6       /* simulation belongs to a running batch */
} mdlts_status;

enum { MDLTS_FP64 = 0, MDLTS_FP32 = 1 };

typedef struct mdlts_ctx mdlts_ctx;
typedef struct mdlts_sim mdlts_sim;

/* Optional device allocator (e.g. a framework's caching allocator).  alloc
 * returns NULL on failure; both are called with the context's stream. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, void *stream, void *user);
    void *user;
} mdlts_allocator;

typedef struct {
    int dim;          /* 2 or 3 */
    int order;        /* polynomial degree p: 1, 2 or 3 */
    int n[3];         /* root grid (n[2] ignored for dim 2) */
    double len[3];    /* box edge lengths [cm] */
    int max_depth;    /* refinement depth cap, 0..8 */
    int n_levels;     /* LTS levels L, 1..8; level l takes 2^l substeps */
    int precision;    /* MDLTS_FP64 or MDLTS_FP32 (bulk arithmetic and storage) */
} mdlts_mesh_desc;

/* Aliev-Panfilov two-variable model: du/dt += -k u (u-a)(u-1) - u v;
 * dv/dt = (eps0 + mu1 v/(u+mu2)) (-v - k u (u-a-1)). */
typedef struct { double k, a, eps0, mu1, mu2; } mdlts_ap_params;

/* Stimulus: adds amp [1/ms] to du/dt at nodes with lo <= x <= hi for
 * t_on <= t < t_off (the -I_stim/C_m term of the model, Sec. 2). */
typedef struct { double lo[3], hi[3], t_on, t_off, amp; } mdlts_stim_box;

const char *mdlts_strerror(mdlts_status s);

/* ---- context ------------------------------------------------------------ */
/* device: HIP device ordinal; hip_stream: a hipStream_t (NULL = default
 * stream); alloc may be NULL.  Errors: EINVAL, EDEVICE. */
mdlts_status mdlts_ctx_create(int device, void *hip_stream, const mdlts_allocator *alloc, mdlts_ctx **out);
/* EBUSY while simulations created on the context are still alive. */
mdlts_status mdlts_ctx_destroy(mdlts_ctx *ctx);
/* Waits for the stream and reports asynchronous kernel failures (EDEVICE). */
mdlts_status mdlts_sync(mdlts_ctx *ctx);

/* ---- simulation: mesh and parameters (Sec. 2, Sec. 2.2) ------------------ */
/* Creates a simulation on the root mesh (all roots leaves, u = v = 0, t = 0,
 * D = 1e-3 I, gamma = 2 / 4 / 8 for degree 1 / 2 / 3, standard Aliev-Panfilov
 * constants, no stimulus). */
mdlts_status mdlts_sim_create(mdlts_ctx *ctx, const mdlts_mesh_desc *desc, mdlts_sim **out);
mdlts_status mdlts_sim_destroy(mdlts_sim *sim);
/* Replaces the forest (refine-bit stream, see above).  The state is reset to
 * zero.  EINVAL: malformed stream, depth above max_depth, or not 2:1 balanced. */
mdlts_status mdlts_set_tree(mdlts_sim *sim, const uint8_t *refine_bits, size_t n_bits);
/* Serialises the current forest; *n_bits receives the length (also when
 * bits is NULL or cap is too small, in which case nothing is written). */
mdlts_status mdlts_get_tree(mdlts_sim *sim, uint8_t *bits, size_t cap, size_t *n_bits);
mdlts_status mdlts_n_leaves(mdlts_sim *sim, size_t *n_leaves);
/* Diffusion tensor D (Sec. 2: D = kappa/(chi C_m)) as Dxx,Dyy,Dzz,Dxy,Dxz,Dyz
 * [cm^2/ms] and the SIPG penalty gamma (Sec. 2.1; sigma_F uses n.D n).  D
 * must be symmetric positive definite; off-diagonal entries (fibres not
 * along the axes) select kernels with the mixed-derivative volume terms and
 * the tangential parts of the face fluxes, and a CFL bound from the full own
 * element block.  In 2-D, Dzz is ignored and Dxz, Dyz must be 0.  EINVAL for
 * a tensor that is not accepted, or a gamma for which some element block
 * loses its negative diagonal. */
mdlts_status mdlts_set_conductivity(mdlts_sim *sim, const double D_sym[6], double gamma);
mdlts_status mdlts_set_ionic(mdlts_sim *sim, const mdlts_ap_params *p);
/* At most 8 boxes. */
mdlts_status mdlts_set_stimulus(mdlts_sim *sim, const mdlts_stim_box *boxes, int n_boxes);
/* u, v: [n_leaves * (order+1)^dim] FP64 in canonical order; n_dof must match.
 * Either pointer may be NULL (that field is left unchanged / not read). */
mdlts_status mdlts_set_state(mdlts_sim *sim, const double *u, const double *v, size_t n_dof);
mdlts_status mdlts_get_state(mdlts_sim *sim, double *u, double *v, size_t n_dof);
/* Simulated time of the next barrier; also resets the barrier counter. */
mdlts_status mdlts_set_time(mdlts_sim *sim, double t);

/* ---- LTS levels (Sec. 2.3: Gershgorin CFL, b^CFL, S_e = 2^b) ------------- */
/* Per leaf: CFL_e = 1 / max_i sum_j |(M_e^-1 K_ee)_ij| (own block, neighbours
 * frozen), level b_e = smallest b >= 0 with dt_barrier*2^-b <= CFL_e.  Leaves
 * are then grouped by level, finest first, stable in canonical order.  Runs on
 * the device.  level_hist (optional, [n_levels]) receives the counts per
 * level.  EUNSTABLE if some leaf needs b_e > n_levels-1 (levels are then
 * left unassigned).  ENOMEM if the two time slots of u would exceed 4 GiB
 * (2 * n_leaves * (p+1)^d * bytes per value; e.g. 19.8M Q2 hexahedra in
 * FP32), the limit of the substep kernels' 32-bit offsets; this also applies
 * to mdlts_assign_uniform. */
mdlts_status mdlts_assign_levels(mdlts_sim *sim, double dt_barrier, int32_t *level_hist);
/* Every leaf on the given level (0 <= level < n_levels): 2^level substeps of
 * dt_barrier / 2^level per barrier, without the CFL test.  level 0 is the
 * plain global forward-Euler step of Sec. 2.3 with step dt_barrier, whose
 * stability (dt * lambda_max < 2) is the caller's responsibility.  The CFL
 * values are still computed for mdlts_get_cfl. */
mdlts_status mdlts_assign_uniform(mdlts_sim *sim, double dt_barrier, int level, int32_t *level_hist);
/* The barrier step chosen from the current leaves (Sec. 2.3 leaves the
 * barrier step to the user): dt_barrier = 2^(n_levels-1) * min_e CFL_e *
 * (1 - 2^-20), the largest step that keeps every leaf within the configured
 * levels (off the power-of-two ties), then mdlts_assign_levels with it.
 * *dt_barrier receives the step.  With n_levels up to 8 this is the paper's
 * form: the coarsest leaves step near their own CFL limit instead of at the
 * finest level's.  Synchronises. */
mdlts_status mdlts_assign_levels_auto(mdlts_sim *sim, double *dt_barrier, int32_t *level_hist);

/* ---- RV-T temporal indicator and the cell criterion (Sec. 2.3) ------------ */
/* Saves the current state and time as the start t_a of the interval the RV-T
 * indicator will cover (device copy; valid until the leaves change). */
mdlts_status mdlts_rvt_snapshot(mdlts_sim *sim);
/* RV-T indicator per leaf over [t_a, t_now]: the L2 norms over the interval
 * and the element of the changes of the ionic current (stimulus included) and
 * of the gate rate since t_a, divided by t_now - t_a; the time integrals by
 * the midpoint rule at the state linear in time between the two end states.
 * FP64 on the device, kept there for mdlts_assign_levels_cell; eta_t
 * [n_leaves] (canonical order, may be NULL) and eta_t_max (may be NULL)
 * receive copies.  ESTATE without a snapshot on the current leaves or if no
 * time has passed since it.  Synchronises. */
mdlts_status mdlts_rvt_indicator(mdlts_sim *sim, double *eta_t, size_t n_leaves, double *eta_t_max);
/* mdlts_assign_levels with both criteria: b_e = max(b^CFL_e, b^cell_e), with
 * b^cell_e = ceil(log2(dt_barrier / dt_cell)) where the last RV-T indicator
 * exceeds tau_cell and 0 elsewhere (ceiling by exact scaling, ties
 * satisfied).  ESTATE if the indicator was not computed on the current
 * leaves; EUNSTABLE as mdlts_assign_levels. */
mdlts_status mdlts_assign_levels_cell(mdlts_sim *sim, double dt_barrier, double tau_cell, double dt_cell,
                                      int32_t *level_hist);
/* Copies the last assignment: level [n_leaves] (canonical order), perm
 * [n_leaves] (grouped position -> canonical leaf), cnt_ge [n_levels]
 * (number of leaves with level >= l).  Any pointer may be NULL. */
mdlts_status mdlts_get_levels(mdlts_sim *sim, int8_t *level, int32_t *perm, int32_t *cnt_ge, size_t n_leaves);
/* FP64 CFL_e per leaf in canonical order, as used by mdlts_assign_levels. */
mdlts_status mdlts_get_cfl(mdlts_sim *sim, double *cfl, size_t n_leaves);

/* ---- stepping (Sec. 2.3, Algorithm 1) ------------------------------------ */
/* Advances n_barriers barrier intervals.  In each, substep i = 0..2^lmax-1
 * updates every leaf of level >= lmax - v2(i) (all at i = 0) by one
 * forward-Euler step of the SIPG operator (element volume + interior-penalty
 * faces + inverse diagonal mass) with the Aliev-Panfilov reaction and the
 * stimulus, and one exponential step of the gate, with dt_e = dt_barrier /
 * 2^level; neighbours not updated at substep i are linearly interpolated in
 * time.  Asynchronous on the context stream.  ESTATE if levels are not
 * assigned for the current forest. */
mdlts_status mdlts_step(mdlts_sim *sim, int n_barriers);

/* ---- many simulations at once -------------------------------------------- */
/* Advances each simulation of the list (all created on ctx, levels assigned)
 * by n_barriers barrier intervals, like mdlts_step on each, with one launch
 * per substep index and element kind (dimension, order, precision) covering
 * all of them: every simulation runs its own 2^lmax substeps per interval
 * (Sec. 2.3; the elements of one sweep are independent) with its own
 * barrier step, parameters and time.  Each result is bitwise the same as
 * running the simulation alone.  The per-barrier launch sequence is cached
 * until a simulation of the list changes and, when it holds more than one
 * kernel variant, replayed as HIP graphs of eight barriers; the first
 * barriers of a new list time the candidate launch shapes (threads per
 * block, one block per tile) and keep the fastest for each kernel variant.
 * Asynchronous on the context stream.  EINVAL for a repeated or foreign
 * simulation, ESTATE if levels are not assigned. */
mdlts_status mdlts_batch_step(mdlts_ctx *ctx, mdlts_sim *const *sims, int n_sims, int n_barriers);
/* Error indicator, adaptation and level assignment of several simulations
 * (Algorithm 1's adaptation step at a barrier): for each simulation the same
 * work and results as mdlts_indicator (no readback), mdlts_adapt (with the
 * device indicator) and mdlts_assign_levels(dt_barrier[q]) in sequence, with
 * two host synchronisations for all simulations together instead of several
 * per simulation.  With two or more simulations each step of the sequence
 * is one launch per kernel variant over all of them (the per-simulation
 * arguments go to the device as tables, one copy per half), all on the
 * context stream.  sims as for mdlts_batch_step; dt_barrier [n_sims].
 * Returns the first error of any simulation (EUNSTABLE: non-finite
 * indicator or a leaf beyond the levels; that simulation's levels are then
 * invalid); the others are still processed. */
mdlts_status mdlts_batch_adapt(mdlts_ctx *ctx, mdlts_sim *const *sims, int n_sims, double tau_refine,
                               double tau_coarsen, const double *dt_barrier);
/* enable = 1 (default): batches whose substeps launch more than one kernel
 * variant replay graphs of eight barriers (each variant's launches form a
 * chain of their own through them, and the chains run concurrently; the
 * barriers of a call that do not fill a graph are launched directly);
 * single-variant plans (mdlts_step, or a batch of one variant) launch their
 * tile kernels directly or replay graphs of four barriers, whichever the
 * autotuner timed faster.  enable = 0: every launch goes directly to the stream, and
 * mdlts_step uses the per-element kernel without tile lists. */
mdlts_status mdlts_set_graphs(mdlts_ctx *ctx, int enable);
/* Event timing of the batched substep launches (launched directly while
 * enabled); read returns kernel ms, launches, DoF-updates since the last
 * read, and the launch shape in use (threads per block of the kernel variant
 * with the most device time; per_cu is always 0: one block per tile).
 * ESTATE before the first mdlts_batch_step. */
mdlts_status mdlts_batch_profile(mdlts_ctx *ctx, int enable);
mdlts_status mdlts_batch_profile_read(mdlts_ctx *ctx, double *substep_ms, uint64_t *n_launches,
                                      uint64_t *dof_updates, int *block, int *per_cu);

/* ---- error indicator and adaptivity (Sec. 2.2, Algorithm 1) -------------- */
/* Kelly-type indicator eta_e^2 = sum over interior face pieces F of e of
 * h_F/(2p) * W_F^2 * ||[[D grad u . n]]||^2_{L2(F)} at the barrier (FP64
 * accumulation on the device).  eta: [n_leaves] canonical order (may be
 * NULL); eta_max: max over leaves (may be NULL).  Synchronises the stream.
 * EUNSTABLE if the state holds a non-finite value. */
mdlts_status mdlts_indicator(mdlts_sim *sim, double *eta, size_t n_leaves, double *eta_max);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * indicator of mdlts_indicator with the same arguments, results and errors,
 * calling no hipMalloc, hipFree or allocator.  Its scratch memory (the
 * canonical copy of the state, eta on the device, the maximum and the
 * non-finite flag) is one fixed device array of 64 MiB per GPU, held from
 * the first context on that GPU until the process ends.  ENOMEM if a call
 * needs more: 256 + 8 E bytes, plus E (p+1)^d bytes-per-value while the
 * state is grouped by level (after a level assignment), each part rounded up
 * to 256 bytes; about 2.8M Q1 quadrilaterals or 0.58M Q2 hexahedra in FP32.
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (several host threads or
 * contexts) race, and the caller must serialise them.  Unlike
 * mdlts_indicator, the result is not kept for mdlts_adapt(eta = NULL).
 * Synchronises. */
mdlts_status mdlts_indicator_noalloc(mdlts_sim *sim, double *eta, size_t n_leaves, double *eta_max);
/* Refines leaves with eta >= tau_refine (below max_depth), closes the 2:1
 * balance by refining coarser face neighbours, coarsens parents whose
 * children all have eta <= tau_coarsen (when that keeps 2:1 balance), and
 * transfers u and v (prolongation by evaluation, restriction by L2
 * projection).  eta: [n_leaves] canonical order, or NULL to use the last
 * mdlts_indicator result (ESTATE if the state or forest changed since).
 * Runs on the device; the host reads back only the new leaf count.  Levels
 * must be assigned again afterwards. */
mdlts_status mdlts_adapt(mdlts_sim *sim, const double *eta, size_t n_leaves, double tau_refine,
                         double tau_coarsen, int64_t *n_refined, int64_t *n_coarsened);

/* DoF-updates performed so far (sum over substeps of active leaves times
 * nodes per leaf) and the simulated time of the next barrier. */
mdlts_status mdlts_counters(mdlts_sim *sim, uint64_t *dof_updates, double *t_sim);

/* ---- measurement ---------------------------------------------------------- */
/* enable != 0: bracket every substep kernel launch with a pair of HIP events
 * on the context stream (resets the accumulators). */
mdlts_status mdlts_profile(mdlts_sim *sim, int enable);
/* Waits for the recorded events and returns, since the last read or enable,
 * the summed substep kernel time [ms], the number of launches and the
 * DoF-updates they performed; then resets the accumulators. */
mdlts_status mdlts_profile_read(mdlts_sim *sim, double *substep_ms, uint64_t *n_launches, uint64_t *dof_updates);

/* ---- host-only planning utilities (no device work) ---------------------- */
/* Lower bound on CFL_e over the leaves of the given depth (worst face kinds
 * per direction that a 2:1-balanced forest allows, jointly over all faces
 * for a full tensor; attained on uniform meshes).  A barrier step of 2^(L-1) * bound(max_depth) keeps every leaf
 * within L levels. */
mdlts_status mdlts_cfl_bound(const mdlts_mesh_desc *desc, const double D_sym[6], double gamma, int depth,
                             double *cfl_min);
/* The adaptation decisions of mdlts_adapt on a given forest and indicator,
 * computed on the host: writes the new refine-bit stream (*n_out receives
 * its length; nothing is written if cap is too small). */
mdlts_status mdlts_plan_adapt(const mdlts_mesh_desc *desc, const uint8_t *bits, size_t n_bits, const double *eta,
                              size_t n_leaves, double tau_refine, double tau_coarsen, uint8_t *out_bits,
                              size_t cap, size_t *n_out);
/* Levels, grouping and CFL of mdlts_assign_levels computed on the host for a
 * given forest (any output pointer may be NULL). */
mdlts_status mdlts_plan_levels(const mdlts_mesh_desc *desc, const uint8_t *bits, size_t n_bits, const double D_sym[6],
                               double gamma, double dt_barrier, int8_t *level, int32_t *perm, int32_t *cnt_ge,
                               double *cfl, size_t n_leaves);
/* Upper bound, in bytes, of the device memory one simulation of this shape
 * holds while it never has more than max_leaves leaves: both state layouts,
 * the transfer and staging buffers, face, level and adaptation tables, and its
 * share of a batch plan, each with the 1/8 headroom a growing buffer is given
 * so that small changes of the leaf count do not reallocate.  A request loop that admits solves by device memory
 * (continuous batching of many simulations, as in the batched form of the
 * LTS step) reserves this for the worst-case leaf count of a request, i.e.
 * every root refined to max_depth.  Host only; no device call.
 * EINVAL: bad descriptor, max_leaves < 1 or >= 2^27, bytes NULL. */
mdlts_status mdlts_memory_bound(const mdlts_mesh_desc *desc, int64_t max_leaves, uint64_t *bytes);

#ifdef __cplusplus
}
#endif
#endif
