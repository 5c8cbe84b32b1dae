/*
 * imexds.h -- C ABI of the MI355X (gfx950) implementation of the
 * explicit-implicit domain-splitting (IMEX-DS) time step of May & Thein,
 * "Explicit-Implicit Domain Splitting for Two Phase Flows with Phase
 * Transition" (arXiv 2211.00705), for the 1D isothermal Euler equations with
 * sharp liquid-vapour interfaces and a kinetic mass-transfer relation.
 *
 * The library advances a batch of independent 1D problems.  One physical
 * step of one problem is Algorithm 1 of the paper: every cell away from the
 * tiny cut cells is updated explicitly with HLL fluxes (Step 1, eq. "update
 * expl time"); the cells of each implicit zone (the tiny cut cell and Z
 * neighbours on each side) are updated by Algorithm 2, dual time stepping
 * with local pseudo steps (eq. "dual time tau diff") followed by a
 * conservative update from the accepted iterate (Part 2), with moving
 * interface-adjacent cells (Sec. 3.4, eq. "godunov_meth:nonunif").  The flux
 * across a phase boundary comes from the two-phase Riemann problem with the
 * kinetic relation z = tau p_V [[g + e_kin]] (Sec. 2.1, eq. "isoT:kin_rel1";
 * Appendix A, eqs. "2p_RP:ex_sys", "jacobian:ex_sys", "pb_flux:pt").  The
 * time step follows the CFL condition (eq. "cfl_cond:unif") per problem.
 *
 * Units: SI.  Arithmetic: IEEE FP64 throughout, no fused multiply-add.
 *
 * Conventions for every function returning int:
 *   0 on success, a negative IMEXDS_ERR_* code otherwise (imexds_strerror
 *   names it).  Nothing aborts; no C++ exception crosses the ABI.  A failure
 *   of one problem (Newton not converging, non-physical state, mesh failure,
 *   overlapping zones, a vanishing phase) does not fail the call: that problem is frozen and its
 *   IMEXDS_ST_* bits show in its status word (imexds_get_problems).
 * Pointers: "device" pointers are HIP device memory on the context's device
 *   (e.g. torch tensors on cuda), "host" pointers are ordinary memory.  The
 *   caller keeps them alive for the duration of the call; the library keeps no
 *   reference to caller memory after a call returns.
 * Streams: all device work is enqueued on the stream given to imexds_create
 *   (NULL = the null stream).  Functions marked "async" return before the
 *   work is done; functions that return host data synchronize the stream.
 */
#ifndef IMEXDS_H
#define IMEXDS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define IMEXDS_OK 0
#define IMEXDS_ERR_INVALID_ARG (-1)
#define IMEXDS_ERR_OOM (-2)
#define IMEXDS_ERR_HIP (-3)
#define IMEXDS_ERR_NO_STATE (-4)
#define IMEXDS_ERR_UNSUPPORTED (-5)
#define IMEXDS_ERR_TOO_LARGE (-6) /* size above an entry point's fixed maximum */

/* per-problem status bits (sticky; a problem with any bit set is frozen) */
#define IMEXDS_ST_NEWTON_FAIL 1  /* interface Newton-Armijo did not converge */
#define IMEXDS_ST_NONPHYSICAL 2  /* rho <= 0 or non-finite state */
#define IMEXDS_ST_MESH_FAIL 4    /* a cut piece collapsed / could not merge */
#define IMEXDS_ST_ZONE_OVERLAP 8 /* implicit zones overlap outside a pair (three in a row,
                                    or any overlap under IMEXDS_ZONE_NEWTON) */
#define IMEXDS_ST_PHASE_VANISH 16 /* a merge would leave the phase between two phase
                                     boundaries as one cell bounded by both */

/* per-step, per-interface log flags (imexds_get_log) */
#define IMEXDS_FL_TINY_RIGHT 1 /* the smaller cut piece is right of the interface */
#define IMEXDS_FL_MERGED 2     /* that piece was merged into its outer neighbour */
#define IMEXDS_FL_REDO 4       /* merge forced after a collapse inside the zone solve */
#define IMEXDS_FL_LMAX 8       /* dual time stepping stopped at lmax */
#define IMEXDS_FL_CROSS_L 16   /* interface moved into the left neighbour cell */
#define IMEXDS_FL_CROSS_R 32   /* interface moved into the right neighbour cell */
#define IMEXDS_FL_FAIL 64      /* the zone failed this step (status set) */
#define IMEXDS_FL_INACTIVE 128 /* problem frozen or finished: nothing done */
#define IMEXDS_FL_PAIR 256     /* solved in one zone with the neighbouring interface */

/* dual-time stopping rules (Algorithm 2, "Stopping criterium"):
 * IMEXDS_TOL_PAPER: the residual of Sec. 4 (Numerical results),
 *   res_i = |(1 + dtau_i/dt)(W_i^{l+1} - W_i^l)| / (dtau_i max(|W_i^l|, 1)),
 *   dtau_i = theta_i dt, largest over the two components, must be below
 *   tol_tiny on the tiny cell and below tol_nb on every other cell of the
 *   (2Z+1)-cell zone (the paper's k-1, k+1 for Z = 1; the zone's outer cells
 *   too for Z > 1);
 * IMEXDS_TOL_REL: max |W^{l+1}-W^l| / max(|W^l|,1) < tol_rel over the zone. */
#define IMEXDS_TOL_PAPER 0
#define IMEXDS_TOL_REL 1

#define IMEXDS_BC_WALL 0
#define IMEXDS_BC_TRANSMISSIVE 1

typedef struct imexds_ctx imexds_ctx; /* opaque; owns all of its device buffers */

/* Phase pressure laws (Sec. 4): vapour ideal gas p = a2_vap rho
 * (eq. "eos:isoT_idgas", a2_vap = k T0 / m); liquid linear Tait law
 * p = p_sat + a2_liq (rho - rho_liq_sat) (eq. "eos:isoT_lintait" with
 * a2_liq = K0 / rho0).  Gibbs energies g = a^2 ln(rho / rho_sat) per phase,
 * equal at saturation (Maxwell construction, Sec. 2.1).  tau is the kinetic
 * coefficient of eq. "isoT:kin_rel1". */
typedef struct {
  double a2_vap, a2_liq, p_sat, rho_liq_sat, tau;
} imexds_material;

typedef struct {
  double cfl;         /* C_CFL of eq. "cfl_cond:unif" */
  int32_t zone_half;  /* Z: an implicit zone is the tiny cut piece +- Z slots (1..3) */
  double theta_nb;    /* theta for full cells (0.9 in Sec. 4) */
  int32_t tol_mode;   /* IMEXDS_TOL_* */
  double tol_nb;      /* 1e-3 in Sec. 4 */
  double tol_tiny;    /* 1e-1 in Sec. 4 */
  double tol_rel;     /* for IMEXDS_TOL_REL */
  int32_t lmax;       /* maximal pseudo steps per zone and step (Algorithm 2) */
  double alpha_floor; /* cut pieces shorter than alpha_floor*h are merged */
  double merge_safety;/* factor on the predicted shrink in the merge test */
  int32_t bc_left, bc_right; /* IMEXDS_BC_* */
  int32_t newton_maxit;      /* per Newton-Armijo start */
  double newton_rtol;        /* Newton step below this (relative) is the last one: added to
                                the root and, to first order, to the outputs without a
                                further evaluation (e.g. 1e-10) */
  double t_end;              /* stop time per problem (INFINITY: step counts only) */
} imexds_params;

/* A batch of independent problems (host pointers, copied by imexds_create).
 * Problem p has n_cells[p] background cells of width h[p] starting at
 * x_left[p] and the interfaces iface_off[p] .. iface_off[p+1]-1, sorted left
 * to right.  Interface k lies in background cell home[k] (0-based) at offset
 * hl[k] in [0, h[p]] from its left face and splits it into two slots, so
 * problem p owns n_cells[p] + (iface_off[p+1]-iface_off[p]) consecutive
 * slots of the flat state arrays, problems in order.  phase_first[p] is the
 * phase of the problem's first slot (0 liquid, 1 vapour); phases alternate
 * across interfaces; home cells of one problem must increase strictly, at
 * most 64 interfaces per problem.  With Algorithm 2, two neighbouring
 * interfaces whose implicit zones overlap are solved in one zone holding both
 * phase boundaries (log flag IMEXDS_FL_PAIR); a merge there that would leave
 * the phase between them as a single cell freezes the problem with
 * IMEXDS_ST_PHASE_VANISH.  Any other overlap (three zones in a row, or the
 * Newton zone solver) freezes it with IMEXDS_ST_ZONE_OVERLAP.  Neither fails
 * the call. */
typedef struct {
  int32_t n_problems;
  const int32_t *n_cells;
  const double *h;
  const double *x_left;
  const int32_t *phase_first;
  const int32_t *iface_off; /* [n_problems + 1] */
  const int32_t *home;      /* [n_iface] */
  const double *hl;         /* [n_iface] */
} imexds_batch;

/* Counters since the last imexds_set_state (imexds_get_stats). */
typedef struct {
  int64_t steps;          /* physical steps completed, summed over problems */
  int64_t cell_updates;   /* sum over problems of slots x steps completed */
  int64_t pseudo_iters;   /* dual-time iterations (Algorithm 2, Part 1), summed over
                             zones and steps; Newton steps with IMEXDS_ZONE_NEWTON */
  int64_t merges;         /* merges of vanishing cut pieces (Sec. 3.4) */
  int64_t lmax_hits;      /* zone steps that stopped at lmax */
  int32_t n_failed;       /* problems with a nonzero status */
  int32_t n_active;       /* problems still advancing (status 0, t < t_end) */
  int64_t newton_iters;   /* evaluations of G (Appendix A, eq. "2p_RP:ex_sys") in the
                             interface Newton-Armijo solves: Newton steps and Armijo
                             trials (dual time zone solver; 0 with IMEXDS_ZONE_NEWTON) */
  int64_t iface_solves;   /* interface solves those evaluations belong to */
  int64_t events;         /* mesh events: merges, redone zone solves, interfaces
                             moved into a neighbouring background cell */
  double gpu_ms;          /* device time of the imexds_step / imexds_run /
                             imexds_step_per_problem calls (HIP events) */
  int64_t pair_zones;     /* zone steps solved as one zone holding the two phase
                             boundaries of neighbouring interfaces */
} imexds_stats;

/* Creates a context on the current HIP device for the problem statement of
 * Sec. 2 (Problem Formulation): the phase pressure laws and kinetic
 * coefficient of Sec. 4 (eqs. "eos:isoT_idgas", "eos:isoT_lintait",
 * "isoT:kin_rel1"), the grid-aligned interfaces of Sec. 2.3 and the
 * parameters of Algorithms 1 and 2.  Validates the inputs (IMEXDS_ERR_INVALID_ARG
 * on bad sizes, interfaces outside their problem or out of order, more than
 * 64 interfaces in a problem, parameters out of range), allocates the device
 * buffers
 * (about 4 doubles per slot plus small per-problem/-interface records), and
 * copies the layout to the device.  *out is NULL on failure.  An empty batch
 * (n_problems = 0) is valid and every step on it is a no-op. */
int imexds_create(imexds_ctx **out, const imexds_material *mat, const imexds_params *par,
                  const imexds_batch *batch, void *hip_stream);

/* Loads the cell averages U = (rho, rho u) of the isothermal Euler system
 * (Sec. 2.1) of every slot (device pointers, n_slots doubles each, flat
 * layout above; read before the call returns, not kept), resets t = 0,
 * statuses, step counts, interface positions (to the batch's home/hl),
 * Newton warm starts and statistics, and computes the first time step
 * dt = C h / max(|u| + a) over all slots (eq. "cfl_cond:unif"). */
int imexds_set_state(imexds_ctx *ctx, const double *rho, const double *mom);

/* Enqueues n_steps physical steps of every problem (async): each is
 * Algorithm 1 (explicit update of the bulk, eq. "update expl time") with
 * Algorithm 2 on every implicit zone (eq. "dual time tau diff", Part 2 with
 * the moving lengths of eq. "godunov_meth:nonunif"), then the next CFL time
 * step.  Problems that reached t_end or failed are left unchanged. */
int imexds_step(imexds_ctx *ctx, int32_t n_steps);

/* The steps of imexds_step (Algorithm 1) until every problem has t >= t_end
 * or is frozen, or max_steps steps were enqueued; checks progress every
 * check_every steps (synchronizes).
 * *steps_done (host, may be NULL) receives the number of steps enqueued. */
int imexds_run(imexds_ctx *ctx, int32_t max_steps, int32_t check_every, int32_t *steps_done);

/* Baseline launch form of the steps of imexds_step (Algorithm 1): the same
 * kernels, launched problem by problem on the context's stream (n_steps
 * steps of every problem, async).  Results are bit for bit those of
 * imexds_step. */
int imexds_step_per_problem(imexds_ctx *ctx, int32_t n_steps);

/* Copies the current cell averages U = (rho, rho u) (Sec. 2.1) to device
 * pointers (n_slots each, async). */
int imexds_get_state(imexds_ctx *ctx, double *rho, double *mom);

/* Host copies of the per-interface mesh state of the grid alignment
 * (Sec. 2.3) (n_iface each; any may be NULL): background cell, offset in
 * it, and position x_left + home*h + hl.
 * Synchronizes. */
int imexds_get_interfaces(imexds_ctx *ctx, int32_t *home, double *hl, double *x_iface);

/* Host copies of per-problem time (advanced by the CFL steps of eq.
 * "cfl_cond:unif"), status bits and completed steps (n_problems each; any
 * may be NULL).  Synchronizes. */
int imexds_get_problems(imexds_ctx *ctx, double *t, int32_t *status, int64_t *steps);

/* Enables per-step logging of the next max_steps steps (0 disables): the
 * dual time iteration count of Algorithm 2, the IMEXDS_FL_* flags (mesh
 * events of Sec. 3.4) and the first zone slot (local to the problem) of
 * every interface.  Logging restarts at row 0. */
int imexds_enable_log(imexds_ctx *ctx, int32_t max_steps);

/* Host copies of the logged rows, [rows][n_iface] each (any may be NULL);
 * *rows receives the number of rows written.  Synchronizes. */
int imexds_get_log(imexds_ctx *ctx, int32_t *count, int32_t *flags, int32_t *zlo, int32_t *rows);

/* Statistics since the last imexds_set_state (imexds_stats: counts of
 * Algorithm 2's iterations, the interface solves of Appendix A, the mesh
 * events of Sec. 3.4, device time).  Synchronizes. */
int imexds_get_stats(imexds_ctx *ctx, imexds_stats *out);

/* Launch configuration of the batched step (no counterpart in the paper,
 * which steps one problem at a time): bulk tile class (256, 512, 1024, 2048: R = class/256
 * rows of 62 cells per wave, four waves per tile), zone lanes per 64-lane
 * workgroup (1..64, with one lane per zone), number of zone workgroups (0 =
 * enough for all zones at once; otherwise that many workgroups whose zone
 * slots keep taking the next unsolved zone until none is left), physical
 * steps per captured HIP graph (0 = launch kernels directly, else an even
 * number up to 512) and lanes per zone (1: one lane runs a whole zone; 8: an
 * 8-lane group runs it, one lane per zone cell, the interface solve split
 * over the two lanes next to the phase boundary; zones_per_group then counts
 * the zone groups per 64-lane wave, clamped to 1..8).
 * Rebuilds the tile table and drops captured graphs.  Results do not depend
 * on it (bit for bit). */
int imexds_set_launch(imexds_ctx *ctx, int32_t tile_cells, int32_t zones_per_group,
                      int32_t zone_groups, int32_t graph_steps, int32_t zone_lanes);

/* The solver of the zones' implicit step.  IMEXDS_ZONE_DTS (default):
 * Algorithm 2, dual time stepping with the stop rule of the parameters.
 * IMEXDS_ZONE_NEWTON: Newton on the same implicit step (the Newton-like
 * solver of the paper's outlook), any zone_half (1..3): unknowns the
 * zone's values W,
 * residual R_i(W) = (h_i(W)/h_i^n) W_i - U_i^n + (dt/h_i^n)(F_{i+1/2}(W) -
 * F_{i-1/2}(W)) with h_i(W) = h_i^n + mov_i w(W) dt and the zone's outer
 * faces from U^n; from W = U^n a forward-difference Jacobian (step
 * 1e-7 max(|W_j|, 1)) of which the 2x2 blocks beside the diagonal are kept
 * (R_i depends on W_{i-1}, W_i and W_{i+1} only), the block Thomas
 * algorithm (no pivoting; a 2x2 pivot block without a finite inverse fails
 * the problem with IMEXDS_ST_NEWTON), full steps; converged when every step
 * component is below rtol max(|W_j|, 1)
 * (e.g. 1e-10), at most maxit steps (e.g. 30; then IMEXDS_FL_LMAX).  The
 * prediction, merges, redo, Part 2 and re-split are those of Algorithm 2's
 * path; the logs count Newton steps.  Launch: 1 + 4 zone_half + 2 lane
 * groups per zone, each of one lane (zone_lanes 1 in imexds_set_launch) or
 * of two (otherwise).  Not differentiated:
 * imexds_forward_ckpt returns IMEXDS_ERR_UNSUPPORTED while it is set.
 * Drops captured graphs; synchronizes. */
#define IMEXDS_ZONE_DTS 0
#define IMEXDS_ZONE_NEWTON 1
int imexds_set_zone_solver(imexds_ctx *ctx, int32_t solver, int32_t maxit, double rtol);

/* Launch autotuner (no counterpart in the paper): times launch
 * configurations on the current state for steps_per_trial
 * steps each (zone launch shapes first, then tile classes), restores the
 * state afterwards and keeps the fastest configuration.  Results (host, may
 * be NULL): chosen tile class, zone lanes per group, zone groups, lanes per
 * zone and the measured ms per step.  Synchronizes. */
int imexds_autotune(imexds_ctx *ctx, int32_t steps_per_trial, int32_t *tile_cells,
                    int32_t *zones_per_group, int32_t *zone_groups, int32_t *zone_lanes,
                    double *ms_per_step);

/* Sizes of the batch of imexds_create (host, any may be NULL). */
int imexds_get_sizes(imexds_ctx *ctx, int32_t *n_problems, int32_t *n_iface, int64_t *n_slots);

/* Device-time of the most recent imexds_step / imexds_step_per_problem /
 * imexds_forward_ckpt / imexds_adjoint call
 * measured with HIP events on the context's stream, and the average
 * duration of one bulk-sweep launch inside it (ms, host).  Synchronizes. */
int imexds_last_timing(imexds_ctx *ctx, double *total_ms, double *bulk_ms_per_launch);

/* Enables HIP-event timing of the bulk-sweep kernel (Algorithm 1, Step 1)
 * and the zone kernel (Algorithm 2) inside imexds_step: kernels are launched
 * directly (no graphs), each bulk launch and each zone launch is bracketed
 * by events on the main stream and runs alone (the zones follow the bulk
 * sweep on the same stream instead of overlapping it).  Results are
 * unchanged. */
int imexds_time_bulk(imexds_ctx *ctx, int32_t on);

/* Average device time of one bulk-sweep launch and of one zone launch in the
 * most recent imexds_step made with imexds_time_bulk on (ms, host; any may
 * be NULL), and the number of launches of each.  IMEXDS_ERR_NO_STATE if no
 * step was timed.  Synchronizes. */
int imexds_kernel_timing(imexds_ctx *ctx, double *bulk_ms, double *zone_ms, int32_t *launches);

/* Replaces the kinetic coefficient tau of the kinetic relation (Sec. 2.1,
 * eq. "isoT:kin_rel1") for later steps (tau >= 0, finite).  Synchronizes;
 * drops captured graphs and any recorded checkpointed forward. */
int imexds_set_tau(imexds_ctx *ctx, double tau);

/* ------------------------------------------------------------------------
 * Adjoint (reverse-mode derivative of n steps)
 * ------------------------------------------------------------------------
 * The differentiated map is the discrete one the steps execute: every
 * decision (pseudo-iteration count and stop, merges and crossings of cut
 * pieces, HLL branches, the cell that sets each CFL time step, a clipped
 * last step) is frozen as the forward took it.  Each interface solve is
 * differentiated at its root by the implicit function theorem on
 * G(p_l*, p_r*) = 0 with the Jacobian of Appendix A (eq. "jacobian:ex_sys");
 * the pseudo iterations of Algorithm 2 are reversed one by one from stored
 * iterates.
 *
 * imexds_forward_ckpt runs n_steps steps (async) from the current state like
 * imexds_step, keeping a full copy of the state every ckpt_every steps
 * (device memory owned by the context: about (n_steps / ckpt_every + 1) x
 * (16 B per slot + 40 B per interface + 32 B per problem)).
 *
 * imexds_adjoint then returns, for a scalar objective L of the end state,
 * the derivatives of L with respect to the state and tau at the start of
 * that forward.  Inputs (device, [n_slots] / [n_iface]): dL/drho, dL/d(rho u)
 * of the end state and dL/dhl of its interface offsets (gL_hl may be NULL:
 * zero).  Outputs (device): dL/drho and dL/d(rho u) of the start state
 * ([n_slots]), dL/dhl of the start offsets ([n_iface], may be NULL) and
 * dL/dtau (one double).  Each segment of ckpt_every steps is run again from
 * its checkpoint while its per-step states and zone iterates are kept in a
 * tape (about ckpt_every x (16 B per slot + 8 B x (2 Z + 2) x (l_max + 1)
 * per interface)), then reversed step by step.  With more than one segment
 * a second tape is allocated if device memory allows, and each segment is
 * run again while the one after it is reversed; without it the two
 * alternate.  Sums are taken in a fixed
 * order, so results are reproducible.  Async; the end state of the forward
 * is in place again afterwards, and the call may be repeated with other
 * end-state derivatives.  Returns IMEXDS_ERR_NO_STATE unless the last call
 * that changed the state was imexds_forward_ckpt. */
int imexds_forward_ckpt(imexds_ctx *ctx, int32_t n_steps, int32_t ckpt_every);
int imexds_adjoint(imexds_ctx *ctx, const double *gL_rho, const double *gL_mom,
                   const double *gL_hl, double *g_rho0, double *g_mom0, double *g_hl0,
                   double *g_tau);

/* Frees the context and every device buffer it owns (after synchronizing its
 * streams); NULL is ignored. */
void imexds_destroy(imexds_ctx *ctx);
/* Static text naming an IMEXDS_ERR_* code (the last HIP error's text for
 * IMEXDS_ERR_HIP, on the calling thread). */
const char *imexds_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* IMEXDS_H */
