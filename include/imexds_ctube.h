/*
 * imexds_ctube.h -- creation tubes: phase creation inside the mesh of the
 * isothermal two-phase scheme of imexds.h (May & Thein, arXiv 2211.00705:
 * appendix "Phase Creation", step (iv) and the sentence after the step lists
 * -- the next step has two phase boundaries treated as before; Sec. 4,
 * cavitation and nucleation tests).
 *
 * A tube has N regular cells of length h, all of one phase, on a fixed
 * mesh.  In every step, while the tube has no created cell, step (i) of the
 * appendix (single-phase Riemann problem, test p* < p_min for a liquid,
 * p* > p_tilde for a vapour, a missing root counting as creation; see
 * imexds_creation.h) runs on every inner face.  The first step with a
 * creating face j (between cells j-1 and j) is the creation step: step (ii)
 * solves the five-state problem there; cell j-1 takes the flux of the left
 * phase boundary on its right and the length h + w_l dt, cell j the flux of
 * the right boundary on its left and the length h - w_r dt; the new cell,
 * stored in slot N, gets the new phase's star state (rho_b, rho_b u_b) and
 * the length (w_r - w_l) dt; every other cell is updated explicitly (HLL).
 * In later steps the created cell is bounded by two phase boundaries at
 * x_j + dl and x_j + dr; Algorithm 1 treats every cell but "created cell
 * +- Z cells" explicitly, and Algorithm 2 (dual time stepping with Delta
 * tau_i = theta_i dt, theta_i = min(theta_nb, h_i^pred / h), the stop rule
 * of Sec. 4 with tol_tiny on the created cell) solves that zone: HLL on its
 * inner faces of the outer phase, the interface solver on the two phase
 * boundaries (their speeds move the lengths of the created cell and its two
 * neighbours), the zone's outer faces from U^n, Part 2 conservative.  CFL
 * step (eq. "cfl_cond:unif") over all cells including the created one.
 *
 * Not modelled (the tube is frozen with a status bit): a second creating
 * face in one step (IMEXDS_CT_ST_MULTI), a neighbour of the created cell
 * shorter than h/2 or a zone reaching past the domain (IMEXDS_CT_ST_MESH);
 * the created cell is never merged (its neighbours are of the other phase).
 *
 * Arithmetic: IEEE FP64, no fused multiply-add, the fixed-order logarithm
 * of imexds.h: results do not depend on the math library.  The material,
 * parameters and error codes are those of imexds.h; of imexds_params, cfl,
 * zone_half (1..3), theta_nb, tol_mode, tol_nb, tol_tiny, tol_rel, lmax,
 * bc_left, bc_right, newton_maxit, newton_rtol and t_end are used (the same
 * for every tube).
 */
#ifndef IMEXDS_CTUBE_H
#define IMEXDS_CTUBE_H

#include <stdint.h>

#include "imexds.h"

#ifdef __cplusplus
extern "C" {
#endif

/* status bits of a tube (frozen once nonzero; its cell values are then
 * unspecified) */
#define IMEXDS_CT_ST_NEWTON 1  /* a Riemann solve (creation or boundary) failed */
#define IMEXDS_CT_ST_NONPHYS 2 /* a nonphysical state (rho <= 0, not finite) */
#define IMEXDS_CT_ST_MESH 4    /* a neighbour of the created cell below h/2, the
                                  created cell collapsed, or its zone leaves the tube */
#define IMEXDS_CT_ST_MULTI 8   /* more than one creating face in one step */

/* per-step log flags */
#define IMEXDS_CT_FL_CREATED 1  /* this step created the cell */
#define IMEXDS_CT_FL_LMAX 2     /* dual time stepping stopped at lmax */
#define IMEXDS_CT_FL_INACTIVE 4 /* tube frozen or finished: nothing done */

typedef struct imexds_ct_ctx imexds_ct_ctx; /* opaque; owns its device buffers */

/* Tubes (host pointers, copied by imexds_ct_create): tube p has n_cells[p]
 * >= 4 regular cells of length h[p] > 0 and phase phase[p] (0 liquid,
 * 1 vapour), and owns n_cells[p] + 1 consecutive slots of the flat state
 * arrays, tubes in order; its last slot holds the created cell. */
typedef struct {
  int32_t n_problems;
  const int32_t *n_cells;
  const double *h;
  const int32_t *phase;
} imexds_ct_batch;

/* Creates a context on the current HIP device; work is ordered after
 * hip_stream (NULL: the null stream) on entry and before it on return.
 * p_min, p_tilde: the creation thresholds (0 Pa and 70388.660656 Pa at
 * 363.15 K, Sec. 4).  Returns IMEXDS_ERR_INVALID_ARG for invalid material,
 * parameters (zone_half outside 1..3, lmax < 1, ...) or tubes,
 * IMEXDS_ERR_OOM, IMEXDS_ERR_HIP. */
int imexds_ct_create(imexds_ct_ctx **out, const imexds_material *mat, const imexds_params *par,
                     double p_min, double p_tilde, const imexds_ct_batch *batch,
                     void *hip_stream);

/* Copies the initial state (device arrays of n_slots doubles: rho and
 * rho u; the created slots are ignored until used) and resets every tube:
 * t = 0, no created cell, status, steps and iteration counts zero, the
 * first CFL step. */
int imexds_ct_set_state(imexds_ct_ctx *ctx, const double *rho, const double *mom);

/* n_steps steps of every active tube (async; a finished or frozen tube does
 * nothing).  IMEXDS_ERR_NO_STATE before imexds_ct_set_state. */
int imexds_ct_step(imexds_ct_ctx *ctx, int32_t n_steps);

/* The same steps launched tube by tube (every kernel of a step once per tube,
 * in turn, on one stream; no log): the unbatched form, results bitwise those
 * of imexds_ct_step. */
int imexds_ct_step_per_problem(imexds_ct_ctx *ctx, int32_t n_steps);

/* Steps in chunks of check_every until no tube is active or max_steps are
 * done (synchronises between chunks); *steps_done gets the steps issued. */
int imexds_ct_run(imexds_ct_ctx *ctx, int32_t max_steps, int32_t check_every,
                  int32_t *steps_done);

/* Copies the current state to device arrays of n_slots doubles (async). */
int imexds_ct_get_state(imexds_ct_ctx *ctx, double *rho, double *mom);

/* Per-tube results to host arrays of n_problems entries (each may be NULL;
 * synchronises): time, status bits, steps done, dual time iterations, the
 * created cell's face (-1: none) and its boundaries' offsets from that face
 * (x_face + dl, x_face + dr). */
int imexds_ct_get_problems(imexds_ct_ctx *ctx, double *t, int32_t *status, int32_t *steps,
                           int64_t *iters, int32_t *face, double *dl, double *dr);

/* Per-step log of the next max_steps steps (0: off): dual time iterations
 * and IMEXDS_CT_FL_* flags per tube, rows of n_problems. */
int imexds_ct_enable_log(imexds_ct_ctx *ctx, int32_t max_steps);
int imexds_ct_get_log(imexds_ct_ctx *ctx, int32_t *count, int32_t *flags, int32_t *rows);

/* Launch shape of the zone kernel: zone_lanes 1 (one lane per tube, the two
 * boundaries in turn), 2 (one lane per boundary) or 4 (two lanes per
 * boundary, one per side of its Riemann problem); tubes per 64-lane wave
 * (zone_problems_per_wave * zone_lanes <= 64).  Default 4 lanes, 2 tubes
 * per wave.  Results do not depend on it. */
int imexds_ct_set_launch(imexds_ct_ctx *ctx, int32_t zone_lanes, int32_t zone_problems_per_wave);

/* The solver of the zone's implicit step.  IMEXDS_CT_SOLVER_DTS (default):
 * Algorithm 2 as described above.  IMEXDS_CT_SOLVER_NEWTON: Newton on the
 * same implicit step (the Newton-like solver of the paper's outlook), any
 * zone_half: unknowns the zone's 2 (2 zone_half + 1) values, residual
 *   R_c(W) = (h_c(W) / h_c^n) W_c - U_c^n + (dt / h_c^n)(F_{c+1/2}(W) - F_{c-1/2}(W))
 * (lengths from the boundary speeds at W, outer zone faces from U^n),
 * Jacobian by forward differences with step 1e-7 max(|W_j|, 1), the block
 * Thomas algorithm on its 2x2 blocks beside the diagonal (the created cell
 * couples its two neighbours only; no pivoting, a pivot block without a
 * finite inverse fails the tube with IMEXDS_CT_ST_NEWTON), full steps from
 * W = U^n; converged when every step component is below rtol max(|W_j|, 1) (e.g. 1e-10), at most
 * maxit steps (e.g. 30; then IMEXDS_CT_FL_LMAX); Part 2 as in Algorithm 2.
 * The log's count is the number of Newton steps. */
#define IMEXDS_CT_SOLVER_DTS 0
#define IMEXDS_CT_SOLVER_NEWTON 1
int imexds_ct_set_solver(imexds_ct_ctx *ctx, int32_t solver, int32_t maxit, double rtol);

int imexds_ct_get_sizes(imexds_ct_ctx *ctx, int32_t *n_problems, int64_t *n_slots);

/* HIP-event timing of the sweep, the zone kernel and the whole step, averaged
 * over the steps since the last imexds_ct_time_kernels(ctx, 1). */
int imexds_ct_time_kernels(imexds_ct_ctx *ctx, int32_t on);
int imexds_ct_last_timing(imexds_ct_ctx *ctx, double *bulk_ms, double *zone_ms, double *step_ms);

void imexds_ct_destroy(imexds_ct_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif
