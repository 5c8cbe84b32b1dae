/*
 * imexds_creation.h -- phase creation (cavitation and nucleation) for
 * batches of single-phase Riemann problems of the isothermal two-phase model
 * of imexds.h (May & Thein, arXiv 2211.00705, appendix section "Phase
 * Creation", steps (i)-(iii) and (v); eqs. "flux:cavitation",
 * "flux:nucleation").
 *
 * Problem j has two states of one phase (liquid or vapour).  Step (i): the
 * Riemann problem without phase transition, f_l(p*) + f_r(p*) + u_r - u_l
 * = 0 with the outer isothermal waves of the interface solver (shock
 * a (rho* - rho)/sqrt(rho rho*), rarefaction a ln(rho* / rho)), by Newton from
 * the mean pressure, stopped when a step falls below 1e-12 max(|p|, p_sat)
 * or below 1e-13 a^2 rho(p) (a relative density change of 1e-13).
 * A liquid problem with p* < p_min, a vapour problem with p* > p_tilde, or
 * one without a root with rho* > 0 creates a layer of the other phase.
 * Step (ii): the five-state problem -- outer wave, star state a, phase
 * boundary, new-phase state b, phase boundary, star state c, outer wave --
 * with the mass and momentum jump conditions and the kinetic relation
 * z = tau p_V [[g + e_kin]] (eq. "isoT:kin_rel1") at both boundaries, solved
 * by Newton-Armijo on (p_a, p_b, p_c) from all three at p_sat (analytic
 * Jacobian, Cramer's rule, Armijo halving at most 20 times on the merit
 * (E1 zref^-1)^2 + (E2 zref^-1)^2 + E3^2, convergence as the interface
 * solver's: a Newton step below rtol max(|p|, p_sat) is taken and ends the
 * solve).  Step (iii)/(v): velocities, mass fluxes and boundary speeds
 * w = u_b + z / rho_b, and the fluxes (-z, -z u_b + p_b) across both
 * boundaries.  The size of the created cell after a step dt is
 * (w_r - w_l) dt (step (iv)); the caller owns the mesh.
 *
 * Arithmetic: IEEE FP64, no fused multiply-add, the fixed-order logarithm
 * of imexds.h: results do not depend on the math library.
 */
#ifndef IMEXDS_CREATION_H
#define IMEXDS_CREATION_H

#include <stdint.h>

#include "imexds.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Fields of one problem's output record (20 doubles, in this order). */
#define IMEXDS_CR_KIND 0  /* 0 none, 1 cavitation (vapour created), 2 nucleation (liquid) */
#define IMEXDS_CR_P1 1    /* star pressure of step (i) (0 if it has no root) */
#define IMEXDS_CR_PA 2    /* star pressures: outer phase left, new phase, outer phase right */
#define IMEXDS_CR_PB 3
#define IMEXDS_CR_PC 4
#define IMEXDS_CR_RA 5    /* densities of the three star states */
#define IMEXDS_CR_RB 6
#define IMEXDS_CR_RC 7
#define IMEXDS_CR_UA 8    /* velocities */
#define IMEXDS_CR_UB 9
#define IMEXDS_CR_UC 10
#define IMEXDS_CR_ZL 11   /* mass fluxes through the left and right phase boundary */
#define IMEXDS_CR_ZR 12
#define IMEXDS_CR_WL 13   /* speeds of the two phase boundaries */
#define IMEXDS_CR_WR 14
#define IMEXDS_CR_FL0 15  /* flux (mass, momentum) across the left boundary */
#define IMEXDS_CR_FL1 16
#define IMEXDS_CR_FR0 17  /* and across the right one */
#define IMEXDS_CR_FR1 18
#define IMEXDS_CR_ITERS 19 /* Newton steps of step (ii) */
#define IMEXDS_CR_FIELDS 20

/* Solves n problems on the current HIP device, enqueued on hip_stream (NULL:
 * the null stream; async): a pass that queues the problems by phase, step
 * (i) over that queue, which queues the creating problems by phase, then
 * step (ii) over the second queue.  Scratch of 8 n + 16 bytes comes from the
 * stream-ordered allocator (hipMallocAsync) and is released on the stream
 * (IMEXDS_ERR_OOM if it cannot be had).
 *   phase          device [n]: 0 liquid, 1 vapour (both states of problem j)
 *   rho_l, mom_l   device [n]: left state (rho, rho u)
 *   rho_r, mom_r   device [n]: right state
 *   p_min, p_tilde the creation thresholds (0 Pa and 70388.660656 Pa at
 *                  363.15 K, Sec. 4)
 *   maxit, rtol    Newton-Armijo limits of step (ii) (e.g. 50, 1e-14)
 *   status         device [n] out: 0 no creation, 1 created, -1 invalid
 *                  input (rho <= 0, unknown phase) or step (ii) failed
 *   out            device [n * IMEXDS_CR_FIELDS] out: the records above
 *                  (all zero but KIND and P1 when nothing is created)
 * Returns IMEXDS_ERR_INVALID_ARG for n < 0, missing pointers, a material
 * that is not positive and finite, maxit < 1 or rtol <= 0; IMEXDS_ERR_HIP
 * if the launch fails.  n = 0 is a no-op. */
int imexds_creation_rp(const imexds_material *mat, int32_t n, const int32_t *phase,
                       const double *rho_l, const double *mom_l, const double *rho_r,
                       const double *mom_r, double p_min, double p_tilde, int32_t maxit,
                       double rtol, int32_t *status, double *out, void *hip_stream);

/* Largest n that imexds_creation_rp_noalloc accepts. */
#define IMEXDS_CR_NOALLOC_MAX (1 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same solve as
 * imexds_creation_rp, with the same arguments, outputs and error codes, but
 * its scratch (queue counters and queues, 8 n + 16 bytes) is a fixed array in
 * the library's device memory, 8 MiB + 16 B on each device the library runs
 * on, held until the process ends.  No allocation or release of any memory is
 * made.  n must be at most IMEXDS_CR_NOALLOC_MAX, else IMEXDS_ERR_TOO_LARGE.
 * The counters are cleared by a kernel at the start of every call.  Every
 * call on one device uses that device's one array: calls that overlap on one
 * device (on different streams, or from different host threads without
 * ordering) race and give wrong results; calls ordered on one stream are
 * safe.  IMEXDS_ERR_HIP if the array's device address cannot be obtained. */
int imexds_creation_rp_noalloc(const imexds_material *mat, int32_t n, const int32_t *phase,
                               const double *rho_l, const double *mom_l, const double *rho_r,
                               const double *mom_r, double p_min, double p_tilde, int32_t maxit,
                               double rtol, int32_t *status, double *out, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif
