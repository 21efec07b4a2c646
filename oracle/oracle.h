/*
 * oracle.h -- plain FP64 CPU oracle for the explicit SIPG-DG monodomain
 * step under synchronous local time stepping (Ogiermann, Balzani, Perotti,
 * "An Explicit Local Space-Time Adaptive Framework for Monodomain Models in
 * Cardiac Electrophysiology", arXiv:2310.07607).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant with the GPU library; the two are written
 * independently and compared element by element.
 *
 * Everything here is deliberately slow and literal: a pointer forest for the
 * mesh, element and face matrices assembled by quadrature in physical
 * coordinates (as the paper's serial implementation pre-assembles K_e and
 * M_e^{-1}, Sec. 2.3), and the synchronous LTS barrier written from its
 * definitions in Sec. 2.3 (per-element update ticks, linear-in-time coarser
 * neighbours), checked bitwise against a level-bucket form.
 *
 * Index conventions (shared with the GPU library's ABI, not with its code):
 *   - root grid n[0] x n[1] (x n[2]); root id = rx + n0*(ry + n1*rz);
 *   - child index = bx | by<<1 | bz<<2 (bit k set = upper half in dim k);
 *   - canonical leaf order = roots in id order, pre-order inside each tree;
 *   - element nodes = tensor Gauss-Legendre nodes, x fastest;
 *   - state vectors are [leaf][node] in canonical leaf order.
 *   - refine-bit stream: pre-order over all nodes of every tree, roots in id
 *     order, one byte per node: 1 = refined (its 2^d children follow in child
 *     index order), 0 = leaf.
 */
#ifndef MDLTS_ORACLE_H
#define MDLTS_ORACLE_H
#include <stdint.h>

#define OR_OK 0
#define OR_EINVAL 1
#define OR_EUNSTABLE 4

typedef struct or_sim or_sim;

or_sim *or_create(int dim, int p, const int n[3], const double len[3], int max_depth);
void or_free(or_sim *S);

/* mesh */
int or_set_tree(or_sim *S, const uint8_t *bits, int64_t n_bits);
int64_t or_tree_bits(const or_sim *S, uint8_t *out, int64_t cap);
int64_t or_n_leaves(const or_sim *S);
int or_n_dof_per_leaf(const or_sim *S);
void or_leaf_info(const or_sim *S, int32_t *depth, int64_t *coords /* [E][3] */);
int or_leaf_nodes(const or_sim *S, double *xyz /* [E*np][3] */);

/* parameters: D is the full 3x3 diffusion tensor (row-major, symmetric) */
int or_set_params(or_sim *S, const double D[9], double gamma, const double ap[5]);
int or_set_stimulus(or_sim *S, const double *boxes /* [n][9]: lo3 hi3 t_on t_off amp */, int n);

/* state, [E*np] each, canonical order */
int or_set_state(or_sim *S, const double *u, const double *v);
int or_get_state(const or_sim *S, double *u, double *v);

/* operators */
int or_assemble(or_sim *S);
int or_dense_operators(or_sim *S, double *K /* N*N or NULL */, double *Mfull /* N*N or NULL */);
int or_apply_K(or_sim *S, const double *u, double *Ku);

/* time stepping */
int or_step_global(or_sim *S, double dt, double t0, int64_t n_steps);
int or_cfl(or_sim *S, double *cfl);
int or_levels(or_sim *S, double dt_barrier, int n_levels, int8_t *level);
/* RV-T temporal indicator of every leaf over [t_a, t_b]: the state at t_a
 * is given (u_a, v_a), the state at t_b is the current one. */
int or_rvt_indicator(or_sim *S, const double *u_a, const double *v_a, double t_a, double t_b, double *eta_t);
/* levels from max(b^CFL, b^cell): b^cell = ceil(log2(dt_barrier/dt_cell))
 * where eta_t > tau_cell, else 0 */
int or_levels_cell(or_sim *S, double dt_barrier, int n_levels, const double *eta_t, double tau_cell,
                   double dt_cell, int8_t *level);
void or_bucket(int64_t E, const int8_t *level, int n_levels, int32_t *perm, int32_t *cnt_ge);
/* mode 0: time-history form (an element of level l updates at the ticks that
 * are multiples of 2^(lmax-l); a coarser neighbour is linear in time between
 * its values at the ticks enclosing the substep); mode 1: two-slot
 * level-bucket form.
 * trace (optional, capacity trace_cap rows of 4 doubles): substep, element,
 * neighbour, theta for every neighbour read of every element update. */
int or_lts_barrier(or_sim *S, double dt_barrier, double t_n, const int8_t *level, int mode,
                   double *trace, int64_t trace_cap, int64_t *trace_len, int64_t *n_updates);

/* error indicator and adaptivity */
int or_indicator(or_sim *S, double *eta);
int or_adapt(or_sim *S, const double *eta, double tau_refine, double tau_coarsen,
             int64_t *n_refined, int64_t *n_coarsened);

/* evaluate the DG field u at physical points */
int or_eval_points(or_sim *S, const double *xyz, int64_t n_pts, double *out);

/* one element's update at one substep, with neighbour fields given as full
 * state vectors at the neighbour's interpolated time (for sampled checks) */
int or_element_update(or_sim *S, int64_t e, const double *u_at_t, double t, double dt,
                      double *u_new /* np */, double *v_new /* np */);

#endif
