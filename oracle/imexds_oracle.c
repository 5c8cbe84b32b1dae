/*
 * imexds_oracle.c -- plain, slow, FP64 CPU oracle of the explicit-implicit
 * domain-splitting (IMEX-DS) scheme of May & Thein (arXiv 2211.00705) for the
 * 1D isothermal Euler equations with sharp liquid-vapour interfaces and a
 * kinetic mass-transfer relation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent CPU reference that
 * the GPU path is checked against.  Only tests/, the package smoke check and
 * the bench's cpu_baseline leg may load it.  It shares no code, header or
 * constant with the HIP library; it is built on its own with
 *   gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC
 * so that no multiply-add is ever fused.
 *
 * What it computes, in the paper's order (section / equation names refer to
 * the paper):
 *   - phase pressure laws: ideal gas vapour (eq. eos:isoT_idgas) and linear
 *     Tait liquid (eq. eos:isoT_lintait, read as p0 + K0 (rho/rho0 - 1),
 *     written here as p0 + aL^2 (rho - rho0));
 *   - Gibbs energies g_K = a_K^2 ln(rho/rho_K0), equal at saturation by the
 *     Maxwell construction (Sec. 2.1);
 *   - the HLL flux for same-phase faces (Sec. 4, "HLL solver as in Toro"),
 *     Davis wave speeds;
 *   - the two-phase interface Riemann solve: Newton-Armijo on
 *     G(p_l*, p_r*) = 0 (Appendix A, eqs. 2p_RP:ex_sys and jacobian:ex_sys),
 *     kinetic relation z = tau p_V [[g + e_kin]] (eq. isoT:kin_rel1) with
 *     e_kin = z^2 v^2 / 2 relative to the interface, HLLC-type initial guess
 *     (eq. HLLC:2p_nopt) and phase-boundary flux F_PB (eq. pb_flux:pt);
 *   - Algorithm 1 (explicit bulk update, saved bounding fluxes) and
 *     Algorithm 2 (dual time stepping, Part 1 and Part 2) on a zone of
 *     2Z+1 cells around each tiny cut cell, with local pseudo steps
 *     (eq. dual time tau diff), the residual and stopping rule of Sec. 4 and
 *     moving cell lengths (Sec. 3.4, eq. godunov_meth:nonunif);
 *   - CFL time step (eq. cfl_cond:unif);
 *   - grid alignment with merging of vanishing cut pieces and re-splitting
 *     (Sec. 2.3), by the deterministic rule stated in the design notes.
 *
 * Tangent build.  Every quantity that depends on the state or on the kinetic
 * coefficient has the type `real`.  Compiled as C, `real` is double and this
 * is the oracle above.  Compiled as C++ with -DOR_TANGENT, `real` is a dual
 * number (value, derivative) from or_dual.h: the value parts go through
 * exactly the same IEEE operations in the same order (so every branch,
 * count and event is the same), and the derivative parts carry the exact
 * directional derivative of the executed discrete map (forward-mode
 * differentiation, decisions frozen).  That build is the reference the
 * hand-written reverse-mode GPU adjoint is checked against.
 *
 * Replay.  oracle_run can also be told the discrete decisions of a previous
 * run (pseudo-iteration counts, merges, crossings, CFL cell) and then
 * repeats them instead of testing; central finite differences of the loss
 * with decisions frozen use it.
 *
 * Plain-arithmetic build (-DOR_PLAIN, C only).  The default build fixes the
 * rounding of every operation: its own fixed-order logarithm, reciprocals
 * multiplied in, the stop test of Sec. 4 evaluated without its division, a
 * squared merit in the Armijo test and a shortcut after a small full Newton
 * step.  Compiled with OR_PLAIN the same source instead uses the C library's
 * log and writes every formula as the paper prints it: divisions by a^2,
 * rho_sat, det and h^{n,l+1}, the pressure-form shock wave
 * sqrt((p* - p_K)(1/rho_K - 1/rho*)), the rarefaction a ln(rho* / rho_K), the
 * update of Sec. 3.4 with its ratios h^n/h^{n,l+1} and dt/h^{n,l+1}, the
 * residual res_i with its division by dtau_i max(|U|,1), Kelley's Armijo test
 * on the unsquared merit, and Newton run until its step is below rtol.  It is
 * the check that the default build's rounding choices change nothing beyond
 * round-off (tests run both, the plain one with the default one's decisions
 * replayed).
 *
 * Trace.  oracle_run_trace records, for one interface of one problem at one
 * step, the zone's pseudo-step fractions and every dual time iterate W^l
 * with the phase-boundary speed used to advance it, so that tests can
 * evaluate the paper's residual on them independently.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef OR_TANGENT
#include "or_dual.h"
typedef or_dual real;
#define OR_API extern "C"
#else
typedef double real;
#define OR_API
#endif

#define OR_LIQ 0
#define OR_VAP 1

#define OR_ST_NEWTON 1
#define OR_ST_NONPHYS 2
#define OR_ST_MESH 4
#define OR_ST_OVERLAP 8
#define OR_ST_VANISH 16

#define OR_FL_TINY_RIGHT 1
#define OR_FL_MERGED 2
#define OR_FL_REDO 4
#define OR_FL_LMAX 8
#define OR_FL_CROSS_L 16
#define OR_FL_CROSS_R 32
#define OR_FL_FAIL 64
#define OR_FL_INACTIVE 128
#define OR_FL_PAIR 256

#define OR_MAXC 32

typedef struct {
  real a2v;   /* vapour: p = a2v rho,  a2v = k T0 / m  */
  real a2l;   /* liquid: p = p0 + a2l (rho - rhol0), a2l = K0 / rho0 */
  real p0;    /* saturation pressure */
  real rhol0; /* liquid saturation density */
  real tau;   /* kinetic coefficient */
} or_material;

typedef struct {
  double cfl;
  int zone_half;
  double theta_nb;
  int tol_mode; /* 0: paper residual (tol_nb, tol_tiny); 1: relative update (tol_rel) */
  double tol_nb, tol_tiny, tol_rel;
  int lmax;
  double alpha_floor;
  double merge_safety;
  int bc_left, bc_right; /* 0 wall, 1 transmissive */
  int newton_maxit;
  double newton_rtol;
  double t_end;
  int zone_solver; /* 0: Algorithm 2 (dual time stepping), 1: Newton on the implicit step */
  int zn_maxit;    /* Newton: at most this many steps */
  double zn_rtol;  /* Newton: relative step tolerance */
} or_params;

/* ------------------------------------------------------------------ */
/* phase laws                                                          */
/* ------------------------------------------------------------------ */
static real or_a2(const or_material *M, int ph) { return ph == OR_VAP ? M->a2v : M->a2l; }

static real or_pres(const or_material *M, int ph, real rho) {
  return ph == OR_VAP ? M->a2v * rho : M->p0 + M->a2l * (rho - M->rhol0);
}

/* inverse pressure law (used inside the interface solve), reciprocal form */
static real or_rho_of_p(const or_material *M, int ph, real p) {
#ifdef OR_PLAIN
  return ph == OR_VAP ? p / M->a2v : M->rhol0 + (p - M->p0) / M->a2l;
#else
  return ph == OR_VAP ? p * (1.0 / M->a2v) : M->rhol0 + (p - M->p0) * (1.0 / M->a2l);
#endif
}

/* Natural logarithm of a positive finite double.  Argument reduction
 * x = 2^e m with m in [sqrt(1/2), sqrt(2)], then ln m = 2 atanh(f) with
 * f = (m-1)/(m+1), the atanh series 2 f (1 + f^2/3 + f^4/5 + ... + f^24/25)
 * by Estrin's scheme, and e ln 2 with ln 2 split into a head with trailing
 * zero bits and a tail (as in fdlibm).  Written as plain IEEE double
 * operations in a fixed order, so every IEEE machine gives the same bits;
 * accurate to a few ulp (checked against the C library in the tests). */
OR_API double oracle_log(double x) {
  if (!(x > 0.0)) return x == 0.0 ? -INFINITY : NAN;
  if (!isfinite(x)) return x;
  uint64_t b;
  memcpy(&b, &x, 8);
  int ex = (int)((b >> 52) & 0x7ff);
  int e;
  if (ex == 0) { /* subnormal: scale by 2^54 first */
    double y = x * 18014398509481984.0;
    memcpy(&b, &y, 8);
    e = (int)((b >> 52) & 0x7ff) - 1023 - 54;
  } else {
    e = ex - 1023;
  }
  b = (b & 0x000fffffffffffffULL) | 0x3ff0000000000000ULL;
  double m;
  memcpy(&m, &b, 8);
  if (m > 1.4142135623730951) {
    m = 0.5 * m;
    e += 1;
  }
  double f = (m - 1.0) / (m + 1.0);
  double s = f * f;
  /* Estrin's scheme for sum_{k=0}^{12} s^k / (2k+1) */
  double s2 = s * s, s4 = s2 * s2, s8 = s4 * s4;
  double q0 = 1.0 + (1.0 / 3.0) * s, q1 = (1.0 / 5.0) + (1.0 / 7.0) * s;
  double q2 = (1.0 / 9.0) + (1.0 / 11.0) * s, q3 = (1.0 / 13.0) + (1.0 / 15.0) * s;
  double q4 = (1.0 / 17.0) + (1.0 / 19.0) * s, q5 = (1.0 / 21.0) + (1.0 / 23.0) * s;
  double r0 = q0 + q1 * s2, r1 = q2 + q3 * s2, r2 = q4 + q5 * s2;
  double t0 = r0 + r1 * s4, t1 = r2 + (1.0 / 25.0) * s4;
  double p = t0 + t1 * s8;
  double r = (2.0 * f) * p;
  double de = (double)e;
  return de * 0x1.62e42feep-1 + (de * 0x1.a39ef35793c76p-33 + r);
}

#if defined(OR_TANGENT)
static real or_log(real x) { return or_dual(oracle_log(x.v), x.d / x.v); }
#elif defined(OR_PLAIN)
static real or_log(real x) { return log(x); }
#else
static real or_log(real x) { return oracle_log(x); }
#endif

/* ------------------------------------------------------------------ */
/* HLL flux of the isothermal Euler system, same phase both sides      */
/* ------------------------------------------------------------------ */
static void or_hll(const or_material *M, int ph, real rl, real ml, real rr, real mr,
                real *F) {
  real a = sqrt(or_a2(M, ph));
  real ul = ml / rl, ur = mr / rr;
  real pl = or_pres(M, ph, rl), pr = or_pres(M, ph, rr);
  real sl = (ul < ur ? ul : ur) - a;
  real sr = (ul > ur ? ul : ur) + a;
  real fl0 = ml, fl1 = ml * ul + pl;
  real fr0 = mr, fr1 = mr * ur + pr;
  if (sl >= 0.0) {
    F[0] = fl0;
    F[1] = fl1;
    return;
  }
  if (sr <= 0.0) {
    F[0] = fr0;
    F[1] = fr1;
    return;
  }
  real d = sr - sl, ss = sl * sr;
  F[0] = ((sr * fl0 - sl * fr0) + ss * (rr - rl)) / d;
  F[1] = ((sr * fl1 - sl * fr1) + ss * (mr - ml)) / d;
}

#ifndef OR_TANGENT
void oracle_hll(const or_material *M, int ph, double rl, double ml, double rr, double mr,
                double *F) {
  or_hll(M, ph, rl, ml, rr, mr, F);
}
#endif

/* boundary flux: ghost state (rho, -m) for a wall, (rho, m) transmissive */
static void or_bflux(const or_material *M, int ph, int side_right, int bc, real r, real m,
                     real *F) {
  real mg = (bc == 0) ? -m : m;
  if (side_right)
    or_hll(M, ph, r, m, r, mg, F);
  else
    or_hll(M, ph, r, mg, r, m, F);
}

/* ------------------------------------------------------------------ */
/* interface Riemann problem with phase transition (Appendix A)        */
/* ------------------------------------------------------------------ */
typedef struct {
  real pl, pr; /* star pressures left / right of the phase boundary */
  real rl, rr; /* star densities */
  real ul, ur; /* star velocities */
  real z, w;   /* mass flux, phase-boundary speed */
  real F0, F1; /* flux across the moving phase boundary */
  int iters;
  int ok;
} or_iface;

/* One side of the interface problem: its state, phase constants and
 * L_K = ln(rho_K / rho_K,sat).  One logarithm per side and evaluation,
 * L* = ln(rho* / rho_K,sat), then gives both the Gibbs energy a^2 L* and the
 * rarefaction wave a ln(rho_star / rho_K) = a (L* - L_K). */
typedef struct {
  int ph;
  real r, u, p, LK;
  real a, a2, ia, ia2, hia, irs;
  real rsat; /* saturation density of the side's phase */
} or_side;

static void or_side_init(const or_material *M, int ph, real r, real m, or_side *S) {
  S->ph = ph;
  S->r = r;
  S->u = m / r;
  S->p = or_pres(M, ph, r);
  S->a2 = or_a2(M, ph);
  S->a = sqrt(S->a2);
  S->ia = 1.0 / S->a;
  S->ia2 = 1.0 / S->a2;
  S->hia = 0.5 * S->ia;
  S->rsat = ph == OR_VAP ? M->p0 / M->a2v : M->rhol0;
  S->irs = 1.0 / S->rsat;
#ifdef OR_PLAIN
  S->LK = or_log(r / S->rsat);
#else
  S->LK = or_log(r * S->irs);
#endif
}

typedef struct {
  real rs, v, g, f, df;
} or_seval;

/* Outer wave at star pressure ps (Appendix A): density, specific volume,
 * Gibbs energy, f_K and df_K/dp*.  Shock branch sqrt(-[[p]][[v]]) written
 * a (rho* - rho_K)/sqrt(rho_K rho*) (exact for pressure laws affine in rho);
 * rarefaction branch: the integral of v/a, a ln(rho_star / rho_K). */
static int or_wave(const or_material *M, const or_side *S, real ps, or_seval *E) {
  real r = or_rho_of_p(M, S->ph, ps);
  if (!(r > 0.0) || !isfinite(r)) return 0;
  real v = 1.0 / r;
#ifdef OR_PLAIN
  /* as printed: shock sqrt(-[[p]][[v]]) = sqrt((p_s - p_K)(v_K - v_s)), whose
   * derivative is ((v_K - v_s) + (p_s - p_K) v_s^2 / a^2) / (2 f) (v_s falls
   * as p_s grows: dv_s / dp_s = -v_s^2 / a^2), continued by its limit
   * v_s / a at f = 0; rarefaction: the integral of v/a over the pressure,
   * a ln(rho_s / rho_K) */
  E->rs = r;
  E->v = v;
  E->g = S->a2 * or_log(r / S->rsat);
  if (ps > S->p) {
    real dv = 1.0 / S->r - v;
    E->f = sqrt((ps - S->p) * dv);
    E->df = E->f > 0.0 ? (dv + (ps - S->p) * (v * v / S->a2)) / (2.0 * E->f) : v / S->a;
  } else {
    E->f = S->a * or_log(r / S->r);
    E->df = v / S->a;
  }
  return 1;
#else
  real L = or_log(r * S->irs);
  E->rs = r;
  E->v = v;
  E->g = S->a2 * L;
  if (ps > S->p) {
    real ig = 1.0 / sqrt(S->r * r);
    E->f = (S->a * (r - S->r)) * ig;
    E->df = ((r + S->r) * ig) * (v * S->hia);
  } else {
    E->f = S->a * (L - S->LK);
    E->df = v * S->ia;
  }
  return 1;
#endif
}

typedef struct {
  int phl, phr;
  or_side L, R;
  real izref; /* 1 / max(rho_l a_l, rho_r a_r) */
  real zref;  /* max(rho_l a_l, rho_r a_r) */
} or_rp;

typedef struct {
  real G1, G2, J11, J12, J21, J22, m2, z;
  real dzl, dzr; /* dz/dp_l*, dz/dp_r* */
  or_seval l, r;
} or_geval;

/* G = ([[p]] + z^2 [[v]],  f_l + f_r + z [[v]] + (u_r - u_l)) and its Jacobian
 * (eqs. 2p_RP:ex_sys, jacobian:ex_sys).  z from the kinetic relation
 * z = tau p_V ([[g]] + z^2 [[v^2]]/2) (eq. isoT:kin_rel1 with the kinetic
 * energy relative to the boundary), i.e. A z^2 - z + C = 0 with
 * A = tau p_V [[v^2]]/2 and C = tau p_V [[g]], root continuous at A -> 0;
 * dz/dp by implicit differentiation, where 2 A z - 1 = -sqrt(1 - 4 A C). */
static int or_eval_G(const or_material *M, const or_rp *R, real psl, real psr, or_geval *E) {
  if (!or_wave(M, &R->L, psl, &E->l)) return 0;
  if (!or_wave(M, &R->R, psr, &E->r)) return 0;
  real vl = E->l.v, vr = E->r.v;
  real pV = (R->phl == OR_VAP) ? psl : psr;
  real q = M->tau * pV;
  real jg = E->r.g - E->l.g;
  real jv2 = vr * vr - vl * vl;
  real A = 0.5 * q * jv2;
  real C = q * jg;
  real D = 1.0 - 4.0 * A * C;
  if (!(D >= 0.0) || !isfinite(D)) return 0;
  real sD = sqrt(D);
  real isD = 1.0 / sD;
  real z = 2.0 * C / (1.0 + sD);
#ifdef OR_PLAIN
  {
    /* derivatives as printed in eq. jacobian:ex_sys, (v* / a*)^2 with its
     * division; dz/dp = (dA/dp z^2 + dC/dp) / sqrt(D) */
    real a2l = R->L.a2, a2r = R->R.a2;
    real dAl = q * (vl * vl * vl / a2l), dAr = -(q * (vr * vr * vr / a2r));
    real dCl = -(q * vl), dCr = q * vr;
    if (R->phl == OR_VAP) {
      dAl += M->tau * jv2 / 2.0;
      dCl += M->tau * jg;
    } else {
      dAr += M->tau * jv2 / 2.0;
      dCr += M->tau * jg;
    }
    real dzl = (dAl * z * z + dCl) / sD, dzr = (dAr * z * z + dCr) / sD;
    real jv = vr - vl;
    real el = (vl / R->L.a) * (vl / R->L.a), er = (vr / R->R.a) * (vr / R->R.a);
    E->z = z;
    E->G1 = (psr - psl) + z * z * jv;
    E->G2 = (E->l.f + E->r.f) + z * jv + (R->R.u - R->L.u);
    E->J11 = -1.0 + 2.0 * z * dzl * jv + z * z * el;
    E->J12 = 1.0 + 2.0 * z * dzr * jv - z * z * er;
    E->J21 = E->l.df + dzl * jv + z * el;
    E->J22 = E->r.df + dzr * jv - z * er;
    if (!isfinite(E->G1) || !isfinite(E->G2)) return 0;
    real g1 = E->G1 / R->zref;
    E->m2 = sqrt(g1 * g1 + E->G2 * E->G2); /* unsquared merit */
    (void)isD;
    return 1;
  }
#endif
  /* d(v^2)/dp = -2 v^3 / a^2, dg/dp = v */
  real dAl = q * ((vl * vl * vl) * R->L.ia2);
  real dAr = -(q * ((vr * vr * vr) * R->R.ia2));
  real dCl = -(q * vl);
  real dCr = q * vr;
  if (R->phl == OR_VAP) {
    dAl += (0.5 * M->tau) * jv2;
    dCl += M->tau * jg;
  } else {
    dAr += (0.5 * M->tau) * jv2;
    dCr += M->tau * jg;
  }
  real dzl = (dAl * z * z + dCl) * isD;
  real dzr = (dAr * z * z + dCr) * isD;
  real jv = vr - vl;
  real el = (vl * vl) * R->L.ia2; /* = d[[v]]/dp_l* */
  real er = (vr * vr) * R->R.ia2; /* = -d[[v]]/dp_r* */
  E->z = z;
  E->dzl = dzl;
  E->dzr = dzr;
  E->G1 = (psr - psl) + z * z * jv;
  E->G2 = (E->l.f + E->r.f) + z * jv + (R->R.u - R->L.u);
  E->J11 = -1.0 + 2.0 * z * dzl * jv + z * z * el;
  E->J12 = 1.0 + 2.0 * z * dzr * jv - z * z * er;
  E->J21 = E->l.df + dzl * jv + z * el;
  E->J22 = E->r.df + dzr * jv - z * er;
  if (!isfinite(E->G1) || !isfinite(E->G2)) return 0;
  real a = E->G1 * R->izref;
  E->m2 = a * a + E->G2 * E->G2;
  return 1;
}

/* HLLC-type starting value: contact speed and liquid star density from the
 * left/right states (eq. HLLC:2p_nopt, mirrored for a liquid on the left),
 * liquid pressure law for the pressure; the vapour unknown is kept above
 * 1e-3 p_V so that it stays in the vapour state space. */
static void or_guess(const or_material *M, const or_rp *R, real *gl, real *gr) {
  const or_side *Ls = &R->L, *Rs = &R->R;
  real sl = Ls->u - Ls->a, sr = Rs->u + Rs->a;
  real num = (Rs->p - Ls->p) + Ls->r * Ls->u * (sl - Ls->u) - Rs->r * Rs->u * (sr - Rs->u);
  real den = Ls->r * (sl - Ls->u) - Rs->r * (sr - Rs->u);
  real ws = num / den;
  real rLs;
  if (R->phl == OR_LIQ)
    rLs = Ls->r * (sl - Ls->u) / (sl - ws);
  else
    rLs = Rs->r * (sr - Rs->u) / (sr - ws);
  real pg = or_pres(M, OR_LIQ, rLs);
  real pV = (R->phl == OR_VAP) ? Ls->p : Rs->p;
  real pvg = pg > 1e-3 * pV ? pg : 1e-3 * pV;
  if (R->phl == OR_VAP) {
    *gl = pvg;
    *gr = pg;
  } else {
    *gl = pg;
    *gr = pvg;
  }
}

#ifdef OR_PLAIN
/* Newton-Armijo from one starting point, plain: converged when a Newton step
 * below rtol (relative) has been taken, with G evaluated at the new point;
 * Armijo on the unsquared merit sqrt((G1/zref)^2 + G2^2), at most 20
 * halvings, the point kept when they fail only if the step is already
 * below 1e-8 (round-off floor).  The last step is never returned (last
 * stays 0). */
static int or_newton(const or_material *M, const or_rp *R, real xl, real xr, int maxit,
                     real rtol, real *ol, real *orr, or_geval *Eo, real *sl, real *sr,
                     int *last, int *iters) {
  or_geval E, Et;
  *sl = 0.0;
  *sr = 0.0;
  *last = 0;
  if (!or_eval_G(M, R, xl, xr, &E)) return 0;
  int it;
  for (it = 0; it < maxit; ++it) {
    real det = E.J11 * E.J22 - E.J12 * E.J21;
    if (!(det != 0.0) || !isfinite(det)) return 0;
    real dl = (-E.G1 * E.J22 + E.G2 * E.J12) / det;
    real dr = (-E.G2 * E.J11 + E.G1 * E.J21) / det;
    real sc = fabs(xl) > fabs(xr) ? fabs(xl) : fabs(xr);
    if (M->p0 > sc) sc = M->p0;
    real st = fabs(dl) > fabs(dr) ? fabs(dl) : fabs(dr);
    if (!isfinite(st)) return 0;
    if (st <= rtol * sc) {
      real tl = xl + dl, tr = xr + dr;
      if (or_eval_G(M, R, tl, tr, &Et)) {
        xl = tl;
        xr = tr;
        E = Et;
      }
      *ol = xl;
      *orr = xr;
      *Eo = E;
      *iters = it + 1;
      return 1;
    }
    real lam = 1.0;
    int acc = 0, k;
    for (k = 0; k <= 20; ++k) {
      real tl = xl + lam * dl, tr = xr + lam * dr;
      real c = 1.0 - 1e-4 * lam;
      if (or_eval_G(M, R, tl, tr, &Et) && Et.m2 <= c * E.m2) {
        xl = tl;
        xr = tr;
        E = Et;
        acc = 1;
        break;
      }
      lam *= 0.5;
    }
    if (!acc) {
      if (st <= 1e-8 * sc) {
        *ol = xl;
        *orr = xr;
        *Eo = E;
        *iters = it + 1;
        return 1;
      }
      return 0;
    }
  }
  return 0;
}

#else
/* Newton-Armijo from one starting point (Kelley's line search, Sec. 4);
 * 1 on convergence.  At an accepted point the Newton step is computed; if it
 * is below rtol (relative to max(|p_l*|, |p_r*|, p0)) it is the last one: it
 * is returned in (sl, sr), with last = 1, and the caller applies it to the unknowns and, to
 * first order, to the outputs, without evaluating G again (Newton's error
 * after that step is of the order of the step squared, far below round-off
 * for rtol = 1e-10).  Otherwise Armijo: halve lambda at most 20 times until
 * the squared merit ((G1/zref)^2 + G2^2) drops below (1 - 1e-4 lambda)^2
 * times its current value; if that fails the point is kept (last = 0) only
 * if the step is already below 1e-8 (round-off floor).  At
 * most maxit steps. */
static int or_newton(const or_material *M, const or_rp *R, real xl, real xr, int maxit,
                     real rtol, real *ol, real *orr, or_geval *Eo, real *sl, real *sr,
                     int *last, int *iters) {
  or_geval E, Et;
  *sl = 0.0;
  *sr = 0.0;
  *last = 0;
  if (!or_eval_G(M, R, xl, xr, &E)) return 0;
  int it;
  for (it = 0; it < maxit; ++it) {
    real det = E.J11 * E.J22 - E.J12 * E.J21;
    if (!(det != 0.0) || !isfinite(det)) return 0;
    real idet = 1.0 / det;
    real dl = (-E.G1 * E.J22 + E.G2 * E.J12) * idet;
    real dr = (-E.G2 * E.J11 + E.G1 * E.J21) * idet;
    real sc = fabs(xl) > fabs(xr) ? fabs(xl) : fabs(xr);
    if (M->p0 > sc) sc = M->p0;
    real st = fabs(dl) > fabs(dr) ? fabs(dl) : fabs(dr);
    if (!isfinite(st)) return 0;
    if (st <= rtol * sc) {
      *ol = xl;
      *orr = xr;
      *Eo = E;
      *sl = dl;
      *sr = dr;
      *last = 1;
      *iters = it + 1;
      return 1;
    }
    real lam = 1.0;
    int acc = 0, k;
    for (k = 0; k <= 20; ++k) {
      real tl = xl + lam * dl, tr = xr + lam * dr;
      real c = 1.0 - 1e-4 * lam;
      if (or_eval_G(M, R, tl, tr, &Et) && Et.m2 <= (c * c) * E.m2) {
        xl = tl;
        xr = tr;
        E = Et;
        acc = 1;
        break;
      }
      lam *= 0.5;
    }
    if (!acc) {
      if (st <= 1e-8 * sc) {
        *ol = xl;
        *orr = xr;
        *Eo = E;
        *iters = it + 1;
        return 1;
      }
      return 0;
    }
  }
  return 0;
}

#endif

/* Starting points, tried in this order until Newton-Armijo converges:
 * the caller's warm start (if any), the HLLC-type guess, and both unknowns
 * at the vapour state's own pressure. */
static int or_iface_solve(const or_material *M, int phl, real rl, real ml, int phr, real rr,
                       real mr, int have_guess, real gl, real gr, int maxit, real rtol,
                       or_iface *out) {
  memset(out, 0, sizeof(*out));
  if (!(rl > 0.0) || !(rr > 0.0) || phl == phr) return 0;
  or_rp R;
  R.phl = phl;
  R.phr = phr;
  or_side_init(M, phl, rl, ml, &R.L);
  or_side_init(M, phr, rr, mr, &R.R);
  real zl = rl * R.L.a, zr = rr * R.R.a;
  R.zref = zl > zr ? zl : zr;
  R.izref = 1.0 / R.zref;
  real xl = 0.0, xr = 0.0, dl = 0.0, dr = 0.0;
  or_geval E;
  int iters = 0, conv = 0, last = 0, attempt;
  for (attempt = 0; attempt < 3 && !conv; ++attempt) {
    real sl, sr;
    if (attempt == 0) {
      if (!have_guess) continue;
      sl = gl;
      sr = gr;
    } else if (attempt == 1) {
      or_guess(M, &R, &sl, &sr);
    } else {
      real pV = (phl == OR_VAP) ? R.L.p : R.R.p;
      sl = pV;
      sr = pV;
    }
    int it = 0;
    conv = or_newton(M, &R, sl, sr, maxit, rtol, &xl, &xr, &E, &dl, &dr, &last, &it);
    iters += it;
  }
  if (!conv) return 0;
  /* the last Newton step (dl, dr), if one was returned, applied to the root
   * and, through the derivatives the evaluation at (xl, xr) already holds, to
   * the outputs: v* by dv/dp = -v^2 / a^2, f_K by df_K/dp, z by dz/dp; rho* is
   * affine in p* and taken at the new point */
  real pl = xl, pr = xr;
  real vl = E.l.v, vr = E.r.v, fl = E.l.f, fr = E.r.f, z = E.z;
  if (last) {
    pl = xl + dl;
    pr = xr + dr;
    vl = vl - ((E.l.v * E.l.v) * R.L.ia2) * dl;
    vr = vr - ((E.r.v * E.r.v) * R.R.ia2) * dr;
    fl = fl + E.l.df * dl;
    fr = fr + E.r.df * dr;
    z = z + (E.dzl * dl + E.dzr * dr);
  }
  out->iters = iters;
  out->pl = pl;
  out->pr = pr;
  out->rl = or_rho_of_p(M, phl, pl);
  out->rr = or_rho_of_p(M, phr, pr);
  out->ul = R.L.u - fl;
  out->ur = R.R.u + fr;
  out->z = z;
  real uV, vV, pV;
  if (phl == OR_VAP) {
    uV = out->ul;
    vV = vl;
    pV = pl;
  } else {
    uV = out->ur;
    vV = vr;
    pV = pr;
  }
  out->w = uV + z * vV; /* from z = -rho_V (u_V - w) */
  out->F0 = -z;
  out->F1 = -z * uV + pV;
  out->ok = 1;
  return 1;
}

#ifndef OR_TANGENT
int oracle_iface_solve(const or_material *M, int phl, double rl, double ml, int phr, double rr,
                       double mr, int have_guess, double gl, double gr, int maxit, double rtol,
                       or_iface *out) {
  return or_iface_solve(M, phl, rl, ml, phr, rr, mr, have_guess, gl, gr, maxit, rtol, out);
}

/* G and its Jacobian at a given point (test hook for the analytic Jacobian) */
int oracle_iface_G(const or_material *M, int phl, real rl, real ml, int phr, real rr,
                   real mr, real psl, real psr, real *out6) {
  or_rp R;
  or_geval E;
  R.phl = phl;
  R.phr = phr;
  or_side_init(M, phl, rl, ml, &R.L);
  or_side_init(M, phr, rr, mr, &R.R);
  real zl = rl * R.L.a, zr = rr * R.R.a;
  R.zref = zl > zr ? zl : zr;
  R.izref = 1.0 / R.zref;
  if (!or_eval_G(M, &R, psl, psr, &E)) return 0;
  out6[0] = E.G1;
  out6[1] = E.G2;
  out6[2] = E.J11;
  out6[3] = E.J12;
  out6[4] = E.J21;
  out6[5] = E.J22;
  return 1;
}
#endif

#ifndef OR_TANGENT
/* ------------------------------------------------------------------ */
/* phase creation: cavitation and nucleation (Appendix, Sec. "Phase    */
/* Creation", steps (i)-(iii) and (v))                                 */
/* ------------------------------------------------------------------ */

/* Step (i): the Riemann problem of two states of one phase without phase
 * transition, f_l(p*) + f_r(p*) + (u_r - u_l) = 0 with the outer waves of
 * or_wave, by Newton from the mean pressure (stopped when a step is below
 * 1e-12 max(|p|, p_sat) or below 1e-13 a^2 rho(p)); a step that would leave
 * the phase's density range (rho* <= 0) is halved.  0 on success, 1 if no root with rho* > 0 was
 * found. */
static int or_single_rp(const or_material *M, const or_side *L, const or_side *R, real *ps) {
  real du = R->u - L->u;
  real p = 0.5 * (L->p + R->p);
  or_seval El, Er;
  for (int it = 0; it < 100; ++it) {
    if (!or_wave(M, L, p, &El) || !or_wave(M, R, p, &Er)) return 1;
    real dp = -(El.f + Er.f + du) / (El.df + Er.df);
    if (!isfinite(dp)) return 1;
    real pn = p + dp;
    int k = 0;
    while (!(or_rho_of_p(M, L->ph, pn) > 0.0) && k < 60) {
      dp = 0.5 * dp;
      pn = p + dp;
      ++k;
    }
    if (k == 60) return 1;
    real sc = fabs(p) > M->p0 ? fabs(p) : M->p0;
    p = pn;
    /* converged when the step is below 1e-12 of the pressure scale or below
     * 1e-13 of the density it implies: a stiff liquid resolves its density
     * only to 1e-16 relative, i.e. p* to about 1e-7 Pa (a step test on p
     * alone never passes for |p*| below about 1e5 Pa) */
    if (fabs(dp) <= 1e-12 * sc || fabs(dp) <= 1e-13 * (or_a2(M, L->ph) * or_rho_of_p(M, L->ph, p))) {
      *ps = p;
      return 0;
    }
  }
  return 1;
}

/* Mass flux z through a phase boundary from the kinetic relation (as in
 * or_eval_G) between the states l (left, phase phl) and r at pressures pl,
 * pr, and dz/dpl, dz/dpr. */
static int or_kinetic(const or_material *M, int phl, const or_seval *l, const or_seval *r,
                      real pl, real pr, real ia2l, real ia2r, real *z, real *dzl, real *dzr) {
  real vl = l->v, vr = r->v;
  real pV = phl == OR_VAP ? pl : pr;
  real q = M->tau * pV;
  real jg = r->g - l->g;
  real jv2 = vr * vr - vl * vl;
  real A = 0.5 * q * jv2;
  real C = q * jg;
  real D = 1.0 - 4.0 * A * C;
  if (!(D >= 0.0) || !isfinite(D)) return 0;
  real sD = sqrt(D);
  real isD = 1.0 / sD;
  real zz = 2.0 * C / (1.0 + sD);
  real dAl = q * ((vl * vl * vl) * ia2l);
  real dAr = -(q * ((vr * vr * vr) * ia2r));
  real dCl = -(q * vl);
  real dCr = q * vr;
  if (phl == OR_VAP) {
    dAl += (0.5 * M->tau) * jv2;
    dCl += M->tau * jg;
  } else {
    dAr += (0.5 * M->tau) * jv2;
    dCr += M->tau * jg;
  }
  *z = zz;
  *dzl = (dAl * zz * zz + dCl) * isD;
  *dzr = (dAr * zz * zz + dCr) * isD;
  return 1;
}

/* Step (ii): the Riemann problem of two states of phase `out` with a layer
 * of the other phase created between them: outer wave, star state (a),
 * phase boundary, new-phase state (b), phase boundary, star state (c),
 * outer wave.  Each phase boundary obeys the mass and momentum jump
 * conditions and the kinetic relation, as in the two-phase problem
 * (eq. 2p_RP:ex_sys); eliminating the new phase's velocity leaves
 *   E1 = (b - a) + z_l^2 (v_b - v_a),
 *   E2 = (c - b) + z_r^2 (v_c - v_b),
 *   E3 = f_L(a) + f_R(c) + z_l (v_b - v_a) + z_r (v_c - v_b) + (u_R - u_L). */
typedef struct {
  real E1, E2, E3, J[3][3], m2, zl, zr;
  or_seval a, b, c;
} or_ceval;

static int or_creation_eval(const or_material *M, const or_side *L, const or_side *R,
                            const or_side *S, real izref, real pa, real pb, real pc,
                            or_ceval *E) {
  if (!or_wave(M, L, pa, &E->a) || !or_wave(M, S, pb, &E->b) || !or_wave(M, R, pc, &E->c))
    return 0;
  real dla, dlb, drb, drc;
  if (!or_kinetic(M, L->ph, &E->a, &E->b, pa, pb, L->ia2, S->ia2, &E->zl, &dla, &dlb)) return 0;
  if (!or_kinetic(M, S->ph, &E->b, &E->c, pb, pc, S->ia2, R->ia2, &E->zr, &drb, &drc)) return 0;
  real zl = E->zl, zr = E->zr;
  real jl = E->b.v - E->a.v, jr = E->c.v - E->b.v;
  real ea = (E->a.v * E->a.v) * L->ia2; /* -dv/dp of each state */
  real eb = (E->b.v * E->b.v) * S->ia2;
  real ec = (E->c.v * E->c.v) * R->ia2;
  E->E1 = (pb - pa) + zl * zl * jl;
  E->E2 = (pc - pb) + zr * zr * jr;
  E->E3 = (E->a.f + E->c.f) + zl * jl + zr * jr + (R->u - L->u);
  E->J[0][0] = -1.0 + 2.0 * zl * dla * jl + zl * zl * ea;
  E->J[0][1] = 1.0 + 2.0 * zl * dlb * jl - zl * zl * eb;
  E->J[0][2] = 0.0;
  E->J[1][0] = 0.0;
  E->J[1][1] = -1.0 + 2.0 * zr * drb * jr + zr * zr * eb;
  E->J[1][2] = 1.0 + 2.0 * zr * drc * jr - zr * zr * ec;
  E->J[2][0] = E->a.df + dla * jl + zl * ea;
  E->J[2][1] = dlb * jl - zl * eb + drb * jr + zr * eb;
  E->J[2][2] = E->c.df + drc * jr - zr * ec;
  if (!isfinite(E->E1) || !isfinite(E->E2) || !isfinite(E->E3)) return 0;
  real s1 = E->E1 * izref, s2 = E->E2 * izref;
  E->m2 = s1 * s1 + s2 * s2 + E->E3 * E->E3;
  return 1;
}

/* 3x3 linear solve by Cramer's rule; 0 if singular */
static int or_solve3(const real J[3][3], const real *r, real *x) {
  real c0 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  real c1 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  real c2 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  real det = J[0][0] * c0 + J[0][1] * c1 + J[0][2] * c2;
  if (!(det != 0.0) || !isfinite(det)) return 0;
  real id = 1.0 / det;
  for (int k = 0; k < 3; ++k) {
    real A[3][3];
    memcpy(A, J, sizeof(A));
    for (int i = 0; i < 3; ++i) A[i][k] = r[i];
    real d = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
             A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
             A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    x[k] = d * id;
  }
  return 1;
}

typedef struct {
  real kind;                 /* 0 none, 1 cavitation, 2 nucleation */
  real p1;                   /* step (i) star pressure (0 if it has none) */
  real pa, pb, pc;           /* star pressures: outer phase left, new phase, outer phase right */
  real ra, rb, rc;           /* densities */
  real ua, ub, uc;           /* velocities */
  real zl, zr, wl, wr;       /* mass fluxes and speeds of the two phase boundaries */
  real Fl0, Fl1, Fr0, Fr1;   /* fluxes across them (mass, momentum) */
  real iters;
} or_creation;

/* Phase creation for one Riemann problem of phase ph (eqs. flux:cavitation,
 * flux:nucleation): step (i), the test p* < p_min (liquid: cavitation) or
 * p* > p_tilde (vapour: nucleation), a missing root counting as the test
 * passed, then step (ii) by Newton-Armijo on (E1, E2, E3) from all three
 * pressures at saturation, with the convergence rules of or_newton.
 * Returns 0 (no creation; p1 set), 1 (creation solved) or -1 (invalid
 * input or the solve failed). */
static int or_creation_rp(const or_material *M, int ph, real rl, real ml, real rr, real mr,
                          real p_min, real p_tilde, int maxit, real rtol, or_creation *out) {
  memset(out, 0, sizeof(*out));
  if (!(rl > 0.0) || !(rr > 0.0)) return -1;
  or_side L, R, S;
  or_side_init(M, ph, rl, ml, &L);
  or_side_init(M, ph, rr, mr, &R);
  real p1 = 0.0;
  int none = or_single_rp(M, &L, &R, &p1);
  out->p1 = none ? 0.0 : p1;
  int create = none ? 1 : (ph == OR_LIQ ? p1 < p_min : p1 > p_tilde);
  if (!create) return 0;
  int nph = 1 - ph;
  or_side_init(M, nph, nph == OR_VAP ? M->p0 / M->a2v : M->rhol0, 0.0, &S);
  real zL = rl * L.a, zR = rr * R.a;
  real izref = 1.0 / (zL > zR ? zL : zR);
  real x[3] = {M->p0, M->p0, M->p0};
  or_ceval E, Et;
  if (!or_creation_eval(M, &L, &R, &S, izref, x[0], x[1], x[2], &E)) return -1;
  int it, conv = 0;
  for (it = 0; it < maxit && !conv; ++it) {
    real rhs[3] = {-E.E1, -E.E2, -E.E3}, d[3];
    if (!or_solve3(E.J, rhs, d)) return -1;
    real sc = 0.0, st = 0.0;
    for (int i = 0; i < 3; ++i) {
      if (fabs(x[i]) > sc) sc = fabs(x[i]);
      if (fabs(d[i]) > st) st = fabs(d[i]);
    }
    if (M->p0 > sc) sc = M->p0;
    if (!isfinite(st)) return -1;
    if (st <= rtol * sc) {
      if (or_creation_eval(M, &L, &R, &S, izref, x[0] + d[0], x[1] + d[1], x[2] + d[2], &Et)) {
        for (int i = 0; i < 3; ++i) x[i] = x[i] + d[i];
        E = Et;
      }
      conv = 1;
      break;
    }
    real lam = 1.0;
    int acc = 0, k;
    for (k = 0; k <= 20; ++k) {
      real c = 1.0 - 1e-4 * lam;
      if (or_creation_eval(M, &L, &R, &S, izref, x[0] + lam * d[0], x[1] + lam * d[1],
                           x[2] + lam * d[2], &Et) &&
          Et.m2 <= (c * c) * E.m2) {
        for (int i = 0; i < 3; ++i) x[i] = x[i] + lam * d[i];
        E = Et;
        acc = 1;
        break;
      }
      lam *= 0.5;
    }
    if (!acc) {
      if (st <= 1e-8 * sc) conv = 1;
      else return -1;
      break;
    }
    if (k == 0 && st <= 1e-10 * sc) conv = 1;
  }
  if (!conv) return -1;
  out->kind = ph == OR_LIQ ? 1.0 : 2.0;
  out->pa = x[0];
  out->pb = x[1];
  out->pc = x[2];
  out->ra = E.a.rs;
  out->rb = E.b.rs;
  out->rc = E.c.rs;
  out->ua = L.u - E.a.f;
  out->uc = R.u + E.c.f;
  out->ub = out->ua - E.zl * (E.b.v - E.a.v);
  out->zl = E.zl;
  out->zr = E.zr;
  out->wl = out->ub + E.zl * E.b.v; /* z = -rho (u - w) on the new phase's side */
  out->wr = out->ub + E.zr * E.b.v;
  out->Fl0 = -E.zl;
  out->Fl1 = -E.zl * out->ub + x[1];
  out->Fr0 = -E.zr;
  out->Fr1 = -E.zr * out->ub + x[1];
  out->iters = it + 1;
  return 1;
}

int oracle_creation_rp(const or_material *M, int ph, double rl, double ml, double rr, double mr,
                       double p_min, double p_tilde, int maxit, double rtol, double *out20) {
  or_creation C;
  int st = or_creation_rp(M, ph, rl, ml, rr, mr, p_min, p_tilde, maxit, rtol, &C);
  memcpy(out20, &C, sizeof(C));
  return st;
}

/* n independent problems (threads over problems); out is [n][20] */
void oracle_creation_batch(const or_material *M, int n, const int *ph, const double *rl,
                           const double *ml, const double *rr, const double *mr, double p_min,
                           double p_tilde, int maxit, double rtol, int *status, double *out,
                           int n_threads) {
#pragma omp parallel for schedule(dynamic, 64) num_threads(n_threads > 0 ? n_threads : 1)
  for (int j = 0; j < n; ++j)
    status[j] = oracle_creation_rp(M, ph[j], rl[j], ml[j], rr[j], mr[j], p_min, p_tilde, maxit,
                                   rtol, out + (size_t)j * 20);
}
#endif

/* ------------------------------------------------------------------ */
/* one problem                                                         */
/* ------------------------------------------------------------------ */
typedef struct {
  int n, nif;
  real h;
  int phase_first;
  real *rho, *mom; /* n + nif slots */
  int *home;         /* background cell containing interface k */
  real *hl;        /* offset of interface k inside its home cell */
  real *pw;        /* 2 per interface: last converged star pressures */
  int *warm;
  real *t;
  int *status;
  long long *steps;
  /* replay of a previous run's decisions at the current step (NULL: decide) */
  const int *rp_count; /* [nif] pseudo-iteration counts */
  const int *rp_flags; /* [nif] event flags (merge, crossings) */
  int rp_cfl;          /* slot whose |u| + a set the time step (-1: take the max) */
  /* trace of one zone's dual time iterates (NULL: none) */
  struct or_trace *tr; /* where to record */
  int tr_k;            /* which interface */
  int tr_on;           /* set for the step to record */
} or_prob;

/* Trace record of one zone solve (oracle_run_trace): a header of 8 doubles
 * (m, tiny cell, cell left of the phase boundary, dt, count, lmax hit,
 * records, 0), per active cell (theta, h^n, predicted h^{n+1}, mov), then
 * for l = 0 .. count the iterate W^l (m x 2) and the phase-boundary speed of
 * the interface solve on W^l (the one that moves the lengths of W^{l+1}, or
 * of Part 2 for l = count).  A redo after a collapse restarts the record. */
typedef struct or_trace {
  double *buf;
  int cap, len;
} or_trace;

static void or_tr_put(or_trace *t, double x) {
  if (t && t->len < t->cap) t->buf[t->len] = x;
  if (t) t->len++;
}

typedef struct {
  int m;
  int slot[OR_MAXC];
  int ph[OR_MAXC];
  int mov[OR_MAXC];
  real U0[OR_MAXC][2];
  real hn[OR_MAXC];
  real hh[OR_MAXC]; /* end-of-step length predicted with the explicit speed */
  real th[OR_MAXC];
  real i1t[OR_MAXC]; /* 1 / (1 + theta) */
  real thr[OR_MAXC]; /* tol_i * theta_i dt: stop threshold per unit max(|W|,1) */
  int ic;   /* phase boundary lies between active cells ic and ic+1 */
  int tiny; /* active index of the tiny (or merged) cell */
  real FL[2], FR[2];
  /* phase boundaries in the zone (one, or two when the zones of two
   * neighbouring interfaces overlap): per boundary its cells and tiny cell
   * (icb[0], tinyb[0] are ic, tiny); per active cell the boundary that moves
   * it (bnd, -1 for a cell that does not move) */
  int nb;
  int icb[2], tinyb[2];
  int bnd[OR_MAXC];
} or_zone;

typedef struct {
  int count;
  int flags;
  int zlo;
} or_zlog;

static void or_phases(const or_prob *pb, int *ph) {
  int ns = pb->n + pb->nif, s, k = 0, cur = pb->phase_first;
  for (s = 0; s < ns; ++s) {
    while (k < pb->nif && pb->home[k] + k + 1 == s) {
      cur ^= 1;
      ++k;
    }
    ph[s] = cur;
  }
}

static void or_zone_range(const or_params *P, const or_prob *pb, int k, int *zlo, int *zhi,
                          int *tiny_right) {
  int ns = pb->n + pb->nif;
  int sL = pb->home[k] + k;
  real hL = pb->hl[k], hR = pb->h - hL;
  int tr = !(hL <= hR);
  int c = tr ? sL + 1 : sL;
  int lo = c - P->zone_half, hi = c + P->zone_half;
  if (lo < 0) lo = 0;
  if (hi > ns - 1) hi = ns - 1;
  *zlo = lo;
  *zhi = hi;
  *tiny_right = tr;
}

/* zone set-up: active cells, lengths, merge, pseudo-step fractions, for a
 * zone with nb phase boundaries (interfaces kb[0..nb-1], left to right),
 * each with its tiny side (trb), merge decision (mergeb) and predicted speed
 * (wb).  Returns 1, or 0 if the zone cannot be built; *vanish is set when
 * a merge of a two-boundary zone would leave the phase between the two
 * boundaries as a single cell bounded by both (the tiny piece would merge
 * into a piece of the other boundary's cut cell, or both tiny pieces into
 * the same cell): that phase is about to vanish. */
static int or_zone_build_n(const or_material *M, const or_params *P, const or_prob *pb, int nb,
                           const int *kb, const int *ph, int zlo, int zhi, const int *trb,
                           const int *mergeb, const real *wb, real dt, or_zone *Z, int *vanish) {
  int ns = pb->n + pb->nif;
  real h = pb->h;
  int sL[2], sR[2], skip[2] = {-1, -1}, into[2] = {-1, -1};
  real hL[2], hR[2];
  int b;
  *vanish = 0;
  for (b = 0; b < nb; ++b) {
    sL[b] = pb->home[kb[b]] + kb[b];
    sR[b] = sL[b] + 1;
    hL[b] = pb->hl[kb[b]];
    hR[b] = h - hL[b];
    if (mergeb[b]) {
      if (!trb[b]) {
        skip[b] = sL[b];
        into[b] = sL[b] - 1;
      } else {
        skip[b] = sR[b];
        into[b] = sR[b] + 1;
      }
      if (into[b] < zlo || into[b] > zhi || into[b] < 0 || into[b] >= ns) return 0;
    }
  }
  if (nb == 2) {
    if (sR[0] >= sL[1]) *vanish = 1; /* two boundaries in one background cell */
    for (b = 0; b < 2; ++b)
      if (into[b] >= 0 && (into[b] == sL[1 - b] || into[b] == sR[1 - b])) *vanish = 1;
    if (into[0] >= 0 && into[0] == into[1]) *vanish = 1;
    if (*vanish) return 0;
  }
  int m = 0, s;
  Z->nb = nb;
  for (b = 0; b < 2; ++b) {
    Z->icb[b] = -1;
    Z->tinyb[b] = -1;
  }
  for (s = zlo; s <= zhi; ++s) {
    if (s == skip[0] || s == skip[1]) continue;
    if (m >= OR_MAXC) return 0;
    Z->slot[m] = s;
    Z->ph[m] = ph[s];
    Z->U0[m][0] = pb->rho[s];
    Z->U0[m][1] = pb->mom[s];
    Z->hn[m] = h;
    Z->mov[m] = 0;
    Z->bnd[m] = -1;
    for (b = 0; b < nb; ++b) {
      if (s == sL[b]) {
        Z->hn[m] = hL[b];
        Z->mov[m] = 1;
        Z->bnd[m] = b;
      } else if (s == sR[b]) {
        Z->hn[m] = hR[b];
        Z->mov[m] = -1;
        Z->bnd[m] = b;
      }
    }
    for (b = 0; b < nb; ++b) {
      if (s == into[b]) {
        real ht = trb[b] ? hR[b] : hL[b];
        real hm = h + ht;
        Z->U0[m][0] = (h * pb->rho[s] + ht * pb->rho[skip[b]]) / hm;
        Z->U0[m][1] = (h * pb->mom[s] + ht * pb->mom[skip[b]]) / hm;
        Z->hn[m] = hm;
        Z->mov[m] = trb[b] ? -1 : 1;
        Z->bnd[m] = b;
      }
    }
    ++m;
  }
  Z->m = m;
  for (s = 0; s < m; ++s) {
    for (b = 0; b < nb; ++b) {
      if (Z->mov[s] == 1 && Z->bnd[s] == b) Z->icb[b] = s;
      int is_t = mergeb[b] ? (Z->slot[s] == into[b]) : (Z->slot[s] == (trb[b] ? sR[b] : sL[b]));
      if (is_t) Z->tinyb[b] = s;
    }
  }
  for (b = 0; b < nb; ++b)
    if (Z->icb[b] < 0 || Z->icb[b] + 1 >= m || Z->tinyb[b] < 0) return 0;
  Z->ic = Z->icb[0];
  Z->tiny = Z->tinyb[0];
  for (s = 0; s < m; ++s) {
    real wv = wb[Z->bnd[s] >= 0 ? Z->bnd[s] : 0];
    real hh = Z->hn[s] + ((double)Z->mov[s] * wv) * dt;
    real th = hh / h;
    if (th > P->theta_nb) th = P->theta_nb;
    Z->hh[s] = hh;
    Z->th[s] = th;
    Z->i1t[s] = 1.0 / (1.0 + th);
    int is_tiny = 0;
    for (b = 0; b < nb; ++b) is_tiny = is_tiny || s == Z->tinyb[b];
    Z->thr[s] = (is_tiny ? P->tol_tiny : P->tol_nb) * (th * dt);
    if (!(th > 0.0)) return 0;
  }
  /* bounding fluxes from U^n (Algorithm 1, Step 1: F_left / F_right) */
  if (zlo == 0)
    or_bflux(M, ph[0], 0, P->bc_left, pb->rho[0], pb->mom[0], Z->FL);
  else
    or_hll(M, ph[zlo], pb->rho[zlo - 1], pb->mom[zlo - 1], pb->rho[zlo], pb->mom[zlo], Z->FL);
  if (zhi == ns - 1)
    or_bflux(M, ph[ns - 1], 1, P->bc_right, pb->rho[ns - 1], pb->mom[ns - 1], Z->FR);
  else
    or_hll(M, ph[zhi], pb->rho[zhi], pb->mom[zhi], pb->rho[zhi + 1], pb->mom[zhi + 1], Z->FR);
  return 1;
}

/* the zone of one interface */
static int or_zone_build(const or_material *M, const or_params *P, const or_prob *pb, int k,
                         const int *ph, int zlo, int zhi, int tiny_right, int merge, real w,
                         real dt, or_zone *Z) {
  int vanish = 0;
  return or_zone_build_n(M, P, pb, 1, &k, ph, zlo, zhi, &tiny_right, &merge, &w, dt, Z, &vanish);
}

/* face fluxes of a zone iterate W; each phase-boundary face uses the
 * interface Riemann solver (boundary b starts from pw[2b], pw[2b+1], a guess
 * it takes when have is NULL or have[b] is set, and leaves its root there and
 * its speed in wout[b]), all other inner faces HLL. */
static int or_zone_fluxes_g(const or_material *M, const or_params *P, const or_zone *Z,
                            real W[][2], real F[][2], real *pw, const int *have, real *wout) {
  int c;
  F[0][0] = Z->FL[0];
  F[0][1] = Z->FL[1];
  F[Z->m][0] = Z->FR[0];
  F[Z->m][1] = Z->FR[1];
  for (c = 0; c + 1 < Z->m; ++c) {
    int b = c == Z->icb[0] ? 0 : ((Z->nb == 2 && c == Z->icb[1]) ? 1 : -1);
    if (b >= 0) {
      or_iface I;
      if (!or_iface_solve(M, Z->ph[c], W[c][0], W[c][1], Z->ph[c + 1], W[c + 1][0],
                              W[c + 1][1], have ? have[b] : 1, pw[2 * b], pw[2 * b + 1],
                              P->newton_maxit, P->newton_rtol, &I))
        return 0;
      pw[2 * b] = I.pl;
      pw[2 * b + 1] = I.pr;
      wout[b] = I.w;
      F[c + 1][0] = I.F0;
      F[c + 1][1] = I.F1;
    } else {
      or_hll(M, Z->ph[c], W[c][0], W[c][1], W[c + 1][0], W[c + 1][1], F[c + 1]);
    }
  }
  return 1;
}

static int or_zone_fluxes(const or_material *M, const or_params *P, const or_zone *Z,
                          real W[][2], real F[][2], real *pw, real *wout) {
  return or_zone_fluxes_g(M, P, Z, W, F, pw, NULL, wout);
}

static int or_state_ok(real r, real m) { return r > 0.0 && isfinite(r) && isfinite(m); }

#ifdef OR_TANGENT
#define OR_VAL(x) ((x).v)
#else
#define OR_VAL(x) (x)
#endif

/* Start of the interface solve of a dual time pass.  The paper fixes the
 * solver (Newton-Armijo to a tolerance, Appendix A), not where it starts
 * inside the dual time loop; the root it returns is the same to round-off.
 * hist[0..2] hold the roots of the three previous passes, newest first
 * (nh of them recorded).  With fewer than three the start is the previous
 * root (pw).  From the fourth pass on the roots settle geometrically with
 * the pseudo iterates, and each unknown is extrapolated one pass ahead:
 * a + (d1 / d0) d1 with a the newest root, d1 = a - (the one before),
 * d0 = (the one before) - (the one before that), when |d1| < |d0| (the
 * differences contract); otherwise that unknown starts at a.  The ratio is
 * taken from values only, so in the tangent build the start is a fixed
 * linear combination of earlier roots. */
static void or_dts_start(const real *pw, real hist[3][2], int nh, real *g) {
  int j;
  for (j = 0; j < 2; ++j) {
    g[j] = pw[j];
    if (nh >= 3) {
      real a = hist[0][j], d1 = hist[0][j] - hist[1][j], d0 = hist[1][j] - hist[2][j];
      if (fabs(OR_VAL(d1)) < fabs(OR_VAL(d0))) {
        double q = OR_VAL(d1) / OR_VAL(d0);
        g[j] = a + (real)q * d1;
      }
    }
  }
}

static void or_dts_record(real hist[3][2], int *nh, const real *root) {
  int j;
  for (j = 0; j < 2; ++j) {
    hist[2][j] = hist[1][j];
    hist[1][j] = hist[0][j];
    hist[0][j] = root[j];
  }
  if (*nh < 3) ++*nh;
}

/* Algorithm 2 on one zone. Returns 0 on success, or a status bit.
 * *shrink_cell is set when a moving cell fell below half of its predicted
 * end-of-step length (the length its pseudo step was sized for).
 * Pseudo step (eq. dual time tau diff with moving lengths):
 *   W^{l+1} = (W^l + theta rhs) / (1 + theta),
 *   rhs = (h^n U^n - dt (F_{i+1/2}(W^l) - F_{i-1/2}(W^l))) / h^{n,l+1};
 * stop test of Sec. 4, res_i < tol_i, evaluated without dividing:
 *   |(1 + theta_i)(W^{l+1} - W^l)| < tol_i (theta_i dt) max(|W^l|, 1)
 * for both components of every cell (tol_tiny on the tiny cell, tol_nb on
 * the others); in relative mode |W^{l+1} - W^l| < tol_rel max(|W^l|, 1). */
static int or_zone_dts(const or_material *M, const or_params *P, const or_zone *Z, real dt,
                       real *pw, real U1[][2], real *wstar, int *count, int *lmax_hit,
                       int *shrink_cell, int force_count, or_trace *tr) {
  real W[OR_MAXC][2], Wn[OR_MAXC][2], F[OR_MAXC + 1][2], hnew[OR_MAXC], ih[OR_MAXC];
  int c, l, m = Z->m, b;
  real w[2] = {0.0, 0.0};
  *shrink_cell = -1;
  *lmax_hit = 0;
  for (c = 0; c < m; ++c) {
    W[c][0] = Z->U0[c][0];
    W[c][1] = Z->U0[c][1];
  }
#ifdef OR_TANGENT
  (void)tr;
#define OR_TRACE_ITER()
#else
  if (tr) {
    tr->len = 0;
    or_tr_put(tr, m);
    or_tr_put(tr, Z->tiny);
    or_tr_put(tr, Z->ic);
    or_tr_put(tr, dt);
    or_tr_put(tr, 0.0);
    or_tr_put(tr, 0.0);
    or_tr_put(tr, 0.0);
    or_tr_put(tr, 0.0);
    for (c = 0; c < m; ++c) {
      or_tr_put(tr, Z->th[c]);
      or_tr_put(tr, Z->hn[c]);
      or_tr_put(tr, Z->hh[c]);
      or_tr_put(tr, Z->mov[c]);
    }
  }
#define OR_TRACE_ITER()                      \
  do {                                       \
    if (tr) {                                \
      int c_;                                \
      for (c_ = 0; c_ < m; ++c_) {           \
        or_tr_put(tr, W[c_][0]);             \
        or_tr_put(tr, W[c_][1]);             \
      }                                      \
      or_tr_put(tr, w[0]);                   \
    }                                        \
  } while (0)
#endif
  int cnt = 0, stop = 0;
  /* per boundary: the roots of the last passes and the next start */
  real hist[2][3][2], g[4];
  int nh[2] = {0, 0};
  /* Part 1: pseudo-time iterations (exactly force_count of them in a replay) */
  int lmax = force_count > 0 ? force_count : P->lmax;
  for (l = 0; l < lmax; ++l) {
    for (b = 0; b < Z->nb; ++b) or_dts_start(pw + 2 * b, hist[b], nh[b], g + 2 * b);
    if (!or_zone_fluxes(M, P, Z, W, F, g, w)) return OR_ST_NEWTON;
    for (b = 0; b < Z->nb; ++b) {
      pw[2 * b] = g[2 * b];
      pw[2 * b + 1] = g[2 * b + 1];
      or_dts_record(hist[b], &nh[b], g + 2 * b);
    }
    OR_TRACE_ITER();
    for (c = 0; c < m; ++c) {
      hnew[c] = Z->hn[c] + ((double)Z->mov[c] * w[Z->bnd[c] >= 0 ? Z->bnd[c] : 0]) * dt;
      ih[c] = 1.0 / hnew[c];
      if (Z->mov[c] != 0 && !(hnew[c] >= 0.5 * Z->hh[c])) {
        *shrink_cell = c;
        return OR_ST_MESH;
      }
    }
    int conv = 1;
    for (c = 0; c < m; ++c) {
      real th = Z->th[c], opt = 1.0 + th;
      int q;
      for (q = 0; q < 2; ++q) {
#ifdef OR_PLAIN
        /* Algorithm 2 update with the moving lengths of Sec. 3.4, as printed:
         * W^{l+1} = W^l/(1+r) + r/(1+r) ((h^n/h^{n,l+1}) U^n
         *           - (dt/h^{n,l+1}) (F_{i+1/2} - F_{i-1/2})),  r = dtau/dt = theta;
         * residual res_i = |(1 + dtau/dt)(W^{l+1} - W^l)| / (dtau max(|W^l|,1)) */
        real dtau = th * dt;
        real rhs = (Z->hn[c] / hnew[c]) * Z->U0[c][q] - (dt / hnew[c]) * (F[c + 1][q] - F[c][q]);
        Wn[c][q] = W[c][q] / (1.0 + th) + (th / (1.0 + th)) * rhs;
        real d = Wn[c][q] - W[c][q];
        real sc = fabs(W[c][q]) > 1.0 ? fabs(W[c][q]) : 1.0;
        real tol = c == Z->tiny ? P->tol_tiny : P->tol_nb;
        int ok = (P->tol_mode == 0) ? (fabs(opt * d) / (dtau * sc) < tol)
                                    : (fabs(d) < P->tol_rel * sc);
#else
        real rhs = (Z->hn[c] * Z->U0[c][q] - dt * (F[c + 1][q] - F[c][q])) * ih[c];
        Wn[c][q] = (W[c][q] + th * rhs) * Z->i1t[c];
        real d = Wn[c][q] - W[c][q];
        real sc = fabs(W[c][q]) > 1.0 ? fabs(W[c][q]) : 1.0;
        int ok = (P->tol_mode == 0) ? (fabs(opt * d) < Z->thr[c] * sc) : (fabs(d) < P->tol_rel * sc);
#endif
        conv = conv && ok;
      }
      if (!or_state_ok(Wn[c][0], Wn[c][1])) return OR_ST_NONPHYS;
    }
    for (c = 0; c < m; ++c) {
      W[c][0] = Wn[c][0];
      W[c][1] = Wn[c][1];
    }
    cnt = l + 1;
    stop = force_count > 0 ? cnt == force_count : conv;
    if (stop) break;
  }
  if (!stop) *lmax_hit = 1;
  *count = cnt;
  /* Part 2: fluxes from the accepted iterate, conservative update */
  for (b = 0; b < Z->nb; ++b) or_dts_start(pw + 2 * b, hist[b], nh[b], g + 2 * b);
  if (!or_zone_fluxes(M, P, Z, W, F, g, w)) return OR_ST_NEWTON;
  for (b = 0; b < Z->nb; ++b) {
    pw[2 * b] = g[2 * b];
    pw[2 * b + 1] = g[2 * b + 1];
  }
  OR_TRACE_ITER();
#ifndef OR_TANGENT
  if (tr && tr->cap >= 8) {
    tr->buf[4] = cnt;
    tr->buf[5] = !stop;
    tr->buf[6] = cnt + 1;
  }
#endif
#undef OR_TRACE_ITER
  for (c = 0; c < m; ++c) {
    hnew[c] = Z->hn[c] + ((double)Z->mov[c] * w[Z->bnd[c] >= 0 ? Z->bnd[c] : 0]) * dt;
    ih[c] = 1.0 / hnew[c];
    if (Z->mov[c] != 0 && !(hnew[c] >= 0.5 * Z->hh[c])) {
      *shrink_cell = c;
      return OR_ST_MESH;
    }
  }
  for (c = 0; c < m; ++c) {
    int q;
    for (q = 0; q < 2; ++q)
#ifdef OR_PLAIN
      U1[c][q] = (Z->hn[c] / hnew[c]) * Z->U0[c][q] - (dt / hnew[c]) * (F[c + 1][q] - F[c][q]);
#else
      U1[c][q] = (Z->hn[c] * Z->U0[c][q] - dt * (F[c + 1][q] - F[c][q])) * ih[c];
#endif
    if (!or_state_ok(U1[c][0], U1[c][1])) return OR_ST_NONPHYS;
  }
  for (b = 0; b < Z->nb; ++b) wstar[b] = w[b];
  return 0;
}

#ifndef OR_TANGENT
/* Newton on the implicit step of a zone (the Newton-like solver of the
 * paper's outlook), the alternative to or_zone_dts: unknowns the zone
 * iterates W, equations
 *   R_c(W) = (h_c(W) / h_c^n) W_c - U_c^n + (dt / h_c^n)(F_{c+1/2}(W) - F_{c-1/2}(W)),
 * h_c(W) = h_c^n + mov_c w(W) dt, the zone's outer faces from U^n.  From
 * W = U^n, each Newton step evaluates R at the base point W_k and at the
 * points moved along each unknown (forward differences, step
 * 1e-7 max(|W_j|, 1)); every interface solve of the step starts from the
 * same point, the previous base point's root (in the first step the recorded
 * root, or the solver's own guess without one, as the prediction), so that
 * no evaluation of a step waits for another.  The step dx solves J dx = -R;
 * it is the last when every component is below zn_rtol max(|W_j|, 1) or it
 * is the zn_maxit-th, otherwise W_{k+1} = W_k + dx.  Part 2 then takes the
 * fluxes and the boundary speed of that last base point.  R_c depends on
 * W_{c-1}, W_c and W_{c+1} only (each face flux on the two cells beside it,
 * the moving lengths on the interface face, whose cells are neighbours), so
 * the Jacobian is block tridiagonal in 2x2 blocks: the Newton system takes
 * the difference quotients of those blocks and is solved by or_block_tri.
 * Shrink and state checks and the return codes as in or_zone_dts (the
 * shrink check on every base point). */

/* inverse of a 2x2 matrix by its adjugate; 0 if 1/det is not finite */
static int or_inv2(const double A[2][2], double I[2][2]) {
  double det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
  double id = 1.0 / det;
  if (!isfinite(id)) return 0;
  I[0][0] = A[1][1] * id;
  I[0][1] = -A[0][1] * id;
  I[1][0] = -A[1][0] * id;
  I[1][1] = A[0][0] * id;
  return 1;
}

/* block tridiagonal system (block Thomas algorithm, no pivoting):
 *   L_c x_{c-1} + D_c x_c + U_c x_{c+1} = r_c,  c = 0 .. m-1
 * (L_0, U_{m-1} unused).  Forward: D'_0 = D_0, r'_0 = r_0,
 *   D'_c = D_c - (L_c D'_{c-1}^{-1}) U_{c-1},  r'_c = r_c - (L_c D'_{c-1}^{-1}) r'_{c-1};
 * back: x_{m-1} = D'_{m-1}^{-1} r'_{m-1},  x_c = D'_c^{-1} (r'_c - U_c x_{c+1}).
 * 2x2 products summed in index order.  0 if a D'_c has no finite inverse or
 * a result is not finite. */
static int or_block_tri(int m, double D[][2][2], double L[][2][2], double U[][2][2],
                        double r[][2], double x[][2]) {
  double I[OR_MAXC][2][2], rp[OR_MAXC][2];
  int c, i, j;
  for (c = 0; c < m; ++c) {
    double Dp[2][2];
    if (c == 0) {
      for (i = 0; i < 2; ++i) {
        rp[0][i] = r[0][i];
        for (j = 0; j < 2; ++j) Dp[i][j] = D[0][i][j];
      }
    } else {
      double Lf[2][2];
      for (i = 0; i < 2; ++i)
        for (j = 0; j < 2; ++j) Lf[i][j] = L[c][i][0] * I[c - 1][0][j] + L[c][i][1] * I[c - 1][1][j];
      for (i = 0; i < 2; ++i) {
        for (j = 0; j < 2; ++j)
          Dp[i][j] = D[c][i][j] - (Lf[i][0] * U[c - 1][0][j] + Lf[i][1] * U[c - 1][1][j]);
        rp[c][i] = r[c][i] - (Lf[i][0] * rp[c - 1][0] + Lf[i][1] * rp[c - 1][1]);
      }
    }
    if (!or_inv2(Dp, I[c])) return 0;
  }
  for (c = m - 1; c >= 0; --c) {
    double y[2];
    for (i = 0; i < 2; ++i)
      y[i] = c == m - 1 ? rp[c][i] : rp[c][i] - (U[c][i][0] * x[c + 1][0] + U[c][i][1] * x[c + 1][1]);
    for (i = 0; i < 2; ++i) {
      x[c][i] = I[c][i][0] * y[0] + I[c][i][1] * y[1];
      if (!isfinite(x[c][i])) return 0;
    }
  }
  return 1;
}

/* exported for the tests: blocks as flat arrays of m * 4 (row-major 2x2)
 * and m * 2 doubles */
int oracle_block_tri(int m, const double *D, const double *L, const double *U, const double *r,
                     double *x) {
  double Db[OR_MAXC][2][2], Lb[OR_MAXC][2][2], Ub[OR_MAXC][2][2], rb[OR_MAXC][2], xb[OR_MAXC][2];
  int c, i, j;
  if (m < 1 || m > OR_MAXC) return 0;
  for (c = 0; c < m; ++c)
    for (i = 0; i < 2; ++i) {
      rb[c][i] = r[2 * c + i];
      for (j = 0; j < 2; ++j) {
        Db[c][i][j] = D[4 * c + 2 * i + j];
        Lb[c][i][j] = L[4 * c + 2 * i + j];
        Ub[c][i][j] = U[4 * c + 2 * i + j];
      }
    }
  if (!or_block_tri(m, Db, Lb, Ub, rb, xb)) return 0;
  for (c = 0; c < m; ++c)
    for (i = 0; i < 2; ++i) x[2 * c + i] = xb[c][i];
  return 1;
}

static int or_zone_resid(const or_material *M, const or_params *P, const or_zone *Z, double dt,
                         double W[][2], double *pw, const int *have, double *R,
                         double F[][2], double *w, int check, int *shrink_cell) {
  int c, q;
  if (!or_zone_fluxes_g(M, P, Z, W, F, pw, have, w)) return OR_ST_NEWTON;
  for (c = 0; c < Z->m; ++c) {
    double hk = Z->hn[c] + ((double)Z->mov[c] * w[0]) * dt;
    if (check && Z->mov[c] != 0 && !(hk >= 0.5 * Z->hh[c])) {
      *shrink_cell = c;
      return OR_ST_MESH;
    }
    double ihn = 1.0 / Z->hn[c];
    for (q = 0; q < 2; ++q)
      R[2 * c + q] = (hk * ihn) * W[c][q] - Z->U0[c][q] + (dt * ihn) * (F[c + 1][q] - F[c][q]);
  }
  return 0;
}

/* rec_have, rec_pw: the recorded start of the boundary's interface solve
 * (the prediction's); pw: in, the prediction's root, out the last base
 * point's */
static int or_zone_newton(const or_material *M, const or_params *P, const or_zone *Z, double dt,
                          int rec_have, const double *rec_pw, double *pw, double U1[][2],
                          double *wstar, int *count, int *lmax_hit, int *shrink_cell) {
  int m = Z->m, n = 2 * m, c, q, j, it, conv = 0;
  double W[OR_MAXC][2], R[2 * OR_MAXC], Rp[2 * OR_MAXC], J[2 * OR_MAXC][2 * OR_MAXC];
  double Db[OR_MAXC][2][2], Lb[OR_MAXC][2][2], Ub[OR_MAXC][2][2], rb[OR_MAXC][2], d[OR_MAXC][2];
  double F[OR_MAXC + 1][2], Fp[OR_MAXC + 1][2], w[2] = {0.0, 0.0};
  *shrink_cell = -1;
  *lmax_hit = 0;
  *count = 0;
  for (c = 0; c < m; ++c) {
    W[c][0] = Z->U0[c][0];
    W[c][1] = Z->U0[c][1];
  }
  for (it = 0;; ++it) {
    /* the start of every interface solve of this step */
    const int have[1] = {it == 0 ? rec_have : 1};
    const double g0[2] = {it == 0 ? rec_pw[0] : pw[0], it == 0 ? rec_pw[1] : pw[1]};
    pw[0] = g0[0];
    pw[1] = g0[1];
    int st = or_zone_resid(M, P, Z, dt, W, pw, have, R, F, w, 1, shrink_cell);
    if (st) return st;
    for (j = 0; j < n; ++j) {
      int cj = j / 2, qj = j % 2, dummy;
      double xj = W[cj][qj];
      double e = 1e-7 * (fabs(xj) > 1.0 ? fabs(xj) : 1.0);
      double g[2] = {g0[0], g0[1]}, a[2];
      W[cj][qj] = xj + e;
      st = or_zone_resid(M, P, Z, dt, W, g, have, Rp, Fp, a, 0, &dummy);
      W[cj][qj] = xj;
      if (st) return st;
      for (q = 0; q < n; ++q) J[q][j] = (Rp[q] - R[q]) / e;
    }
    for (c = 0; c < m; ++c) {
      int a, b;
      for (a = 0; a < 2; ++a) {
        rb[c][a] = -R[2 * c + a];
        for (b = 0; b < 2; ++b) {
          Db[c][a][b] = J[2 * c + a][2 * c + b];
          Lb[c][a][b] = c > 0 ? J[2 * c + a][2 * (c - 1) + b] : 0.0;
          Ub[c][a][b] = c + 1 < m ? J[2 * c + a][2 * (c + 1) + b] : 0.0;
        }
      }
    }
    if (!or_block_tri(m, Db, Lb, Ub, rb, d)) return OR_ST_NEWTON;
    conv = 1;
    for (j = 0; j < n; ++j) {
      double xj = W[j / 2][j % 2];
      double sc = fabs(xj) > 1.0 ? fabs(xj) : 1.0;
      conv = conv && (fabs(d[j / 2][j % 2]) <= P->zn_rtol * sc);
    }
    *count = it + 1;
    if (conv || it + 1 >= P->zn_maxit) break;
    for (c = 0; c < m; ++c) {
      W[c][0] = W[c][0] + d[c][0];
      W[c][1] = W[c][1] + d[c][1];
      if (!or_state_ok(W[c][0], W[c][1])) return OR_ST_NONPHYS;
    }
  }
  if (!conv) *lmax_hit = 1;
  /* Part 2 with the last base point's fluxes and boundary speed */
  double ih[OR_MAXC];
  for (c = 0; c < m; ++c) {
    double hk = Z->hn[c] + ((double)Z->mov[c] * w[0]) * dt;
    ih[c] = 1.0 / hk;
    if (Z->mov[c] != 0 && !(hk >= 0.5 * Z->hh[c])) {
      *shrink_cell = c;
      return OR_ST_MESH;
    }
  }
  for (c = 0; c < m; ++c) {
    for (q = 0; q < 2; ++q)
      U1[c][q] = (Z->hn[c] * Z->U0[c][q] - dt * (F[c + 1][q] - F[c][q])) * ih[c];
    if (!or_state_ok(U1[c][0], U1[c][1])) return OR_ST_NONPHYS;
  }
  *wstar = w[0];
  return 0;
}
#endif

/* Predict, merge, solve and re-align one zone: the zone of interface kb[0]
 * (nb = 1), or the zone of the two neighbouring interfaces kb[0], kb[1]
 * whose zones overlap (nb = 2: their union, zlo..zhi, solved as one, with
 * both phase boundaries).  Writes the zone's new cell values into (rn, mn)
 * and each interface's log into lg[0..nb-1].  Returns 0 or a status bit. */
static int or_zone_step(const or_material *M, const or_params *P, or_prob *pb, int nb,
                        const int *kb, const int *ph, int zlo, int zhi, real dt, real *rn,
                        real *mn, or_zlog *lg) {
  real h = pb->h;
  int b, sL[2], sR[2], tr[2], merge[2] = {0, 0};
  real wp[2] = {0.0, 0.0};
  or_iface I[2];
  int force = 0, rflags[2] = {0, 0};
  for (b = 0; b < nb; ++b) {
    int lo, hi;
    sL[b] = pb->home[kb[b]] + kb[b];
    sR[b] = sL[b] + 1;
    or_zone_range(P, pb, kb[b], &lo, &hi, &tr[b]);
    lg[b].zlo = zlo;
    lg[b].flags = (tr[b] ? OR_FL_TINY_RIGHT : 0) | (nb == 2 ? OR_FL_PAIR : 0);
    lg[b].count = 0;
  }
  for (b = 0; b < nb; ++b) {
    int k = kb[b];
    /* explicit prediction of the phase-boundary speed from U^n */
    if (!or_iface_solve(M, ph[sL[b]], pb->rho[sL[b]], pb->mom[sL[b]], ph[sR[b]], pb->rho[sR[b]],
                        pb->mom[sR[b]], pb->warm[k], pb->pw[2 * k], pb->pw[2 * k + 1],
                        P->newton_maxit, P->newton_rtol, &I[b]))
      return OR_ST_NEWTON;
    wp[b] = I[b].w;
    real ht = tr[b] ? h - pb->hl[k] : pb->hl[k];
    real rate = tr[b] ? -wp[b] : wp[b];
    real hfl = P->alpha_floor * h;
    merge[b] = (ht < hfl) || (ht + (P->merge_safety * rate) * dt < hfl);
    if (pb->rp_count) {
      force = pb->rp_count[k];
      rflags[b] = pb->rp_flags[k];
      merge[b] = (rflags[b] & OR_FL_MERGED) != 0;
    }
  }
  int redo = 0;
  real U1[OR_MAXC][2];
  real wstar[2] = {0.0, 0.0};
  int count = 0, lmax_hit = 0;
  or_zone Z;
  for (;;) {
    real pw[4] = {I[0].pl, I[0].pr, I[1].pl, I[1].pr};
    int vanish = 0;
    if (!or_zone_build_n(M, P, pb, nb, kb, ph, zlo, zhi, tr, merge, wp, dt, &Z, &vanish))
      return vanish ? OR_ST_VANISH : OR_ST_MESH;
    int sc;
#ifndef OR_TANGENT
    int st = P->zone_solver == 1
                 ? or_zone_newton(M, P, &Z, dt, pb->warm[kb[0]], pb->pw + 2 * kb[0], pw, U1,
                                  wstar, &count, &lmax_hit, &sc)
                 : or_zone_dts(M, P, &Z, dt, pw, U1, wstar, &count, &lmax_hit, &sc, force,
                               (pb->tr_on && kb[0] == pb->tr_k) ? pb->tr : NULL);
#else
    int st = or_zone_dts(M, P, &Z, dt, pw, U1, wstar, &count, &lmax_hit, &sc, force, NULL);
#endif
    if (st == OR_ST_MESH) {
      /* a tiny cell fell below half its predicted length: solve again with
       * it merged (once per boundary) */
      int again = 0;
      for (b = 0; b < nb; ++b)
        if (!merge[b] && sc == Z.tinyb[b]) {
          merge[b] = 1;
          again = 1;
        }
      if (again) {
        redo = 1;
        continue;
      }
    }
    if (st) return st;
    for (b = 0; b < nb; ++b) {
      pb->pw[2 * kb[b]] = pw[2 * b];
      pb->pw[2 * kb[b] + 1] = pw[2 * b + 1];
    }
    break;
  }
  int c;
  for (c = 0; c < Z.m; ++c) {
    rn[Z.slot[c]] = U1[c][0];
    mn[Z.slot[c]] = U1[c][1];
  }
  for (b = 0; b < nb; ++b) {
    int k = kb[b];
    real hln = pb->hl[k] + wstar[b] * dt;
    int fl = lg[b].flags;
    if (merge[b]) {
      fl |= OR_FL_MERGED;
      if (!tr[b]) {
        if (pb->rp_count ? (rflags[b] & OR_FL_CROSS_L) != 0 : hln < 0.0) {
          pb->home[k] -= 1;
          pb->hl[k] = hln + h;
          rn[sL[b]] = rn[sR[b]];
          mn[sL[b]] = mn[sR[b]];
          fl |= OR_FL_CROSS_L;
        } else {
          rn[sL[b]] = rn[sL[b] - 1];
          mn[sL[b]] = mn[sL[b] - 1];
          pb->hl[k] = hln;
        }
      } else {
        if (pb->rp_count ? (rflags[b] & OR_FL_CROSS_R) != 0 : hln > h) {
          pb->home[k] += 1;
          pb->hl[k] = hln - h;
          rn[sR[b]] = rn[sL[b]];
          mn[sR[b]] = mn[sL[b]];
          fl |= OR_FL_CROSS_R;
        } else {
          rn[sR[b]] = rn[sR[b] + 1];
          mn[sR[b]] = mn[sR[b] + 1];
          pb->hl[k] = hln;
        }
      }
    } else {
      pb->hl[k] = hln;
    }
    pb->warm[k] = 1;
    if (redo) fl |= OR_FL_REDO;
    if (lmax_hit) fl |= OR_FL_LMAX;
    lg[b].flags = fl;
    lg[b].count = count;
  }
  return 0;
}

/* one physical step of one problem (Algorithm 1 with Algorithm 2 per zone) */
static void or_step(const or_material *M, const or_params *P, or_prob *pb, int *ph, real *F,
                    real *rn, real *mn, int *zmark, or_zlog *lg, int *cfl_slot) {
  int ns = pb->n + pb->nif, s, k;
  for (k = 0; k < pb->nif; ++k) {
    lg[k].count = 0;
    lg[k].flags = OR_FL_INACTIVE;
    lg[k].zlo = -1;
  }
  *cfl_slot = -1;
  if (*pb->status) return;
  if (!(*pb->t < P->t_end)) return;
  or_phases(pb, ph);
  /* CFL (eq. cfl_cond:unif): maximal |u| + a over all cells (the first
   * slot attaining it is reported) */
  real S = 0.0;
  int bad = 0, smax = -1;
  for (s = 0; s < ns; ++s) {
    real r = pb->rho[s], m = pb->mom[s];
    if (!or_state_ok(r, m)) {
      bad = 1;
      break;
    }
    real si = fabs(m / r) + sqrt(or_a2(M, ph[s]));
    if (si > S) {
      S = si;
      smax = s;
    }
  }
  if (!bad && pb->rp_cfl >= 0) {
    s = pb->rp_cfl;
    S = fabs(pb->mom[s] / pb->rho[s]) + sqrt(or_a2(M, ph[s]));
    smax = s;
  }
  *cfl_slot = smax;
  if (bad || !(S > 0.0) || !isfinite(S)) {
    *pb->status |= OR_ST_NONPHYS;
    return;
  }
  real dt = (P->cfl * pb->h) / S;
  real rem = P->t_end - *pb->t;
  int clipped = 0;
  if (dt >= rem) {
    dt = rem;
    clipped = 1;
  }
  /* zones: smaller cut piece +- Z slots.  With Algorithm 2, the zones of two
   * neighbouring interfaces that overlap are solved as one zone (their
   * union, both phase boundaries in it); any other overlap freezes the
   * problem.  zmark: the first interface of the zone holding a slot. */
  for (s = 0; s < ns; ++s) zmark[s] = -1;
  int prev_hi = -1;
  for (k = 0; k < pb->nif;) {
    int zlo, zhi, tr, nbk = 1;
    or_zone_range(P, pb, k, &zlo, &zhi, &tr);
    if (zlo <= prev_hi) {
      *pb->status |= OR_ST_OVERLAP;
      return;
    }
    if (k + 1 < pb->nif && P->zone_solver == 0) {
      int zlo1, zhi1, tr1;
      or_zone_range(P, pb, k + 1, &zlo1, &zhi1, &tr1);
      if (zlo1 <= zhi) {
        nbk = 2;
        zhi = zhi1;
      }
    }
    prev_hi = zhi;
    for (s = zlo; s <= zhi; ++s) zmark[s] = k;
    k += nbk;
  }
  /* Algorithm 1, Step 1: explicit update of every cell outside the zones */
  real lam = dt / pb->h;
  for (s = 0; s <= ns; ++s) {
    int need = (s - 1 >= 0 && zmark[s - 1] < 0) || (s < ns && zmark[s] < 0);
    if (!need) continue;
    if (s == 0)
      or_bflux(M, ph[0], 0, P->bc_left, pb->rho[0], pb->mom[0], &F[0]);
    else if (s == ns)
      or_bflux(M, ph[ns - 1], 1, P->bc_right, pb->rho[ns - 1], pb->mom[ns - 1], &F[2 * ns]);
    else
      or_hll(M, ph[s], pb->rho[s - 1], pb->mom[s - 1], pb->rho[s], pb->mom[s], &F[2 * s]);
  }
  for (s = 0; s < ns; ++s) {
    rn[s] = pb->rho[s];
    mn[s] = pb->mom[s];
    if (zmark[s] >= 0) continue;
    rn[s] = pb->rho[s] - lam * (F[2 * (s + 1)] - F[2 * s]);
    mn[s] = pb->mom[s] - lam * (F[2 * (s + 1) + 1] - F[2 * s + 1]);
  }
  /* Algorithm 1, Step 2: each zone by Algorithm 2 */
  int fail = 0;
  for (k = 0; k < pb->nif;) {
    int zlo, zhi, tr, b, nbk = 1;
    or_zone_range(P, pb, k, &zlo, &zhi, &tr);
    if (k + 1 < pb->nif && P->zone_solver == 0) {
      int zlo1, zhi1, tr1;
      or_zone_range(P, pb, k + 1, &zlo1, &zhi1, &tr1);
      if (zlo1 <= zhi) {
        nbk = 2;
        zhi = zhi1;
      }
    }
    int kb[2] = {k, k + 1}, homes[2], i;
    real hls[2];
    for (b = 0; b < nbk; ++b) {
      homes[b] = pb->home[kb[b]];
      hls[b] = pb->hl[kb[b]];
    }
    int st = or_zone_step(M, P, pb, nbk, kb, ph, zlo, zhi, dt, rn, mn, &lg[k]);
    if (st) {
      for (b = 0; b < nbk; ++b) {
        pb->home[kb[b]] = homes[b];
        pb->hl[kb[b]] = hls[b];
        lg[kb[b]].flags |= OR_FL_FAIL;
      }
      for (i = zlo; i <= zhi; ++i) {
        rn[i] = pb->rho[i];
        mn[i] = pb->mom[i];
      }
      fail |= st;
    }
    k += nbk;
  }
  memcpy(pb->rho, rn, sizeof(real) * ns);
  memcpy(pb->mom, mn, sizeof(real) * ns);
  if (fail) {
    *pb->status |= fail;
    return;
  }
  *pb->t = clipped ? P->t_end : *pb->t + dt;
  *pb->steps += 1;
}

/* ------------------------------------------------------------------ */
/* objective and batch driver                                          */
/* ------------------------------------------------------------------ */
/* Scalar objective of one problem: cx times the sum of its interface
 * positions plus the mass in the window [wa, wb],
 *   sum_k (x_left + home_k h + hl_k) cx + sum_s rho_s |slot_s ∩ [wa, wb]|,
 * slot s spanning background cell j = s - (interfaces left of s), or the
 * piece of it left / right of the interface that cuts it. */
static real or_objective(const or_prob *pb, double x_left, double cx, double wa, double wb) {
  int ns = pb->n + pb->nif, s, k = 0;
  real h = pb->h, L = 0.0;
  for (k = 0; k < pb->nif; ++k) L += cx * ((x_left + (double)pb->home[k] * h) + pb->hl[k]);
  k = 0;
  for (s = 0; s < ns; ++s) {
    while (k < pb->nif && pb->home[k] + k + 1 < s) ++k;
    int left_piece = k < pb->nif && pb->home[k] + k == s;
    int right_piece = k < pb->nif && pb->home[k] + k + 1 == s;
    int j = s - k - (right_piece ? 1 : 0);
    real a = x_left + (double)j * h, e = x_left + (double)(j + 1) * h;
    if (left_piece) e = a + pb->hl[k];
    if (right_piece) a = a + pb->hl[k];
    real lo = a > wa ? a : (real)wa, hi = e < wb ? e : (real)wb;
    if (hi > lo) L += pb->rho[s] * (hi - lo);
  }
  return L;
}

/* n_steps physical steps of one problem.  Logs (optional) are rows of
 * nif_tot (interfaces) and P (problems) entries per step; a replay reads
 * its decisions from the same layout. */
static void or_run_problem(const or_material *M, const or_params *Pp, or_prob *pb, int n_steps,
                           int nif_tot, int k0, int P, int p, int *log_count, int *log_flags,
                           int *log_zlo, int *log_cfl, const int *rp_count, const int *rp_flags,
                           const int *rp_cfl, int tr_step) {
  int ns = pb->n + pb->nif;
  int *ph = (int *)malloc(sizeof(int) * ns);
  int *zm = (int *)malloc(sizeof(int) * ns);
  real *F = (real *)malloc(sizeof(real) * 2 * (ns + 1));
  real *rn = (real *)malloc(sizeof(real) * ns);
  real *mn = (real *)malloc(sizeof(real) * ns);
  or_zlog *lg = (or_zlog *)malloc(sizeof(or_zlog) * (pb->nif > 0 ? pb->nif : 1));
  int n, k;
  for (n = 0; n < n_steps; ++n) {
    int cs;
    pb->rp_count = rp_count ? rp_count + (size_t)n * nif_tot + k0 : NULL;
    pb->rp_flags = rp_count ? rp_flags + (size_t)n * nif_tot + k0 : NULL;
    pb->rp_cfl = rp_cfl ? rp_cfl[(size_t)n * P + p] : -1;
    pb->tr_on = pb->tr != NULL && n == tr_step;
    or_step(M, Pp, pb, ph, F, rn, mn, zm, lg, &cs);
    if (log_count) {
      for (k = 0; k < pb->nif; ++k) {
        size_t o = (size_t)n * nif_tot + k0 + k;
        log_count[o] = lg[k].count;
        log_flags[o] = lg[k].flags;
        log_zlo[o] = lg[k].zlo;
      }
    }
    if (log_cfl) log_cfl[(size_t)n * P + p] = cs;
  }
  free(ph);
  free(zm);
  free(F);
  free(rn);
  free(mn);
  free(lg);
}

#ifndef OR_TANGENT
/* Runs n_steps physical steps on each of P independent problems (OpenMP
 * over problems).  Slot arrays are flattened with slot_off[P+1]; interface
 * arrays with iface_off[P+1].  Logs (optional) are [n_steps][n_iface]
 * (counts, flags, zone start) and [n_steps][P] (CFL slot); rp_* (optional)
 * replay a previous run's logs. */
static int or_run_batch(const or_material *M, const or_params *Pp, int P, const int *n_cells,
                        const double *h, const int *phase_first, const int *iface_off,
                        const long long *slot_off, int *home, double *hl, double *pw, int *warm,
                        double *rho, double *mom, double *t, int *status, long long *steps,
                        int n_steps, int *log_count, int *log_flags, int *log_zlo, int *log_cfl,
                        const int *rp_count, const int *rp_flags, const int *rp_cfl,
                        int n_threads, int tr_p, int tr_step, int tr_k, or_trace *tr) {
  int nif_tot = iface_off[P];
  int p;
  if (Pp->zone_half < 1 || 2 * Pp->zone_half + 1 > OR_MAXC) return -1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (p = 0; p < P; ++p) {
    or_prob pb;
    memset(&pb, 0, sizeof(pb));
    if (p == tr_p) {
      pb.tr = tr;
      pb.tr_k = tr_k;
    }
    int k0 = iface_off[p];
    pb.n = n_cells[p];
    pb.nif = iface_off[p + 1] - k0;
    pb.h = h[p];
    pb.phase_first = phase_first[p];
    pb.rho = rho + slot_off[p];
    pb.mom = mom + slot_off[p];
    pb.home = home + k0;
    pb.hl = hl + k0;
    pb.pw = pw + 2 * k0;
    pb.warm = warm + k0;
    pb.t = t + p;
    pb.status = status + p;
    pb.steps = steps + p;
    or_run_problem(M, Pp, &pb, n_steps, nif_tot, k0, P, p, log_count, log_flags, log_zlo,
                   log_cfl, rp_count, rp_flags, rp_cfl, tr_step);
  }
  return 0;
}

int oracle_run(const or_material *M, const or_params *Pp, int P, const int *n_cells,
               const double *h, const int *phase_first, const int *iface_off,
               const long long *slot_off, int *home, double *hl, double *pw, int *warm,
               double *rho, double *mom, double *t, int *status, long long *steps, int n_steps,
               int *log_count, int *log_flags, int *log_zlo, int *log_cfl, const int *rp_count,
               const int *rp_flags, const int *rp_cfl, int n_threads) {
  return or_run_batch(M, Pp, P, n_cells, h, phase_first, iface_off, slot_off, home, hl, pw, warm,
                      rho, mom, t, status, steps, n_steps, log_count, log_flags, log_zlo, log_cfl,
                      rp_count, rp_flags, rp_cfl, n_threads, -1, -1, -1, NULL);
}

/* As oracle_run, and records the dual time iterates of interface tr_k
 * (local to problem tr_p) at step tr_step of this call (layout: or_trace)
 * into buf[cap]; *len receives the record's length (larger than cap if it
 * did not fit; 0 if that zone was not solved at that step). */
int oracle_run_trace(const or_material *M, const or_params *Pp, int P, const int *n_cells,
                     const double *h, const int *phase_first, const int *iface_off,
                     const long long *slot_off, int *home, double *hl, double *pw, int *warm,
                     double *rho, double *mom, double *t, int *status, long long *steps,
                     int n_steps, int *log_count, int *log_flags, int *log_zlo, int *log_cfl,
                     const int *rp_count, const int *rp_flags, const int *rp_cfl, int n_threads,
                     int tr_p, int tr_step, int tr_k, double *buf, int cap, int *len) {
  or_trace tr = {buf, cap, 0};
  int rc = or_run_batch(M, Pp, P, n_cells, h, phase_first, iface_off, slot_off, home, hl, pw,
                        warm, rho, mom, t, status, steps, n_steps, log_count, log_flags, log_zlo,
                        log_cfl, rp_count, rp_flags, rp_cfl, n_threads, tr_p, tr_step, tr_k, &tr);
  *len = tr.len;
  return rc;
}

/* objective (see or_objective) of every problem at the given state */
void oracle_objective(int P, const int *n_cells, const double *h, const double *x_left,
                      const int *iface_off, const long long *slot_off, int *home, double *hl,
                      double *rho, double cx, double wa, double wb, double *out) {
  int p;
  for (p = 0; p < P; ++p) {
    or_prob pb;
    memset(&pb, 0, sizeof(pb));
    int k0 = iface_off[p];
    pb.n = n_cells[p];
    pb.nif = iface_off[p + 1] - k0;
    pb.h = h[p];
    pb.rho = rho + slot_off[p];
    pb.home = home + k0;
    pb.hl = hl + k0;
    out[p] = or_objective(&pb, x_left[p], cx, wa, wb);
  }
}
#else
/* Tangent run: the same steps with every state value carrying a derivative
 * along one direction (d* arrays: seeds in, derivatives out, in place), the
 * material constants with derivative dmat (order a2v, a2l, p0, rhol0, tau).
 * Writes each problem's objective and its directional derivative. */
OR_API int oracle_tan_run(const double *mat, const double *dmat, const or_params *Pp, int P,
                          const int *n_cells, const double *h, const double *x_left,
                          const int *phase_first, const int *iface_off, const long long *slot_off,
                          int *home, double *hl, double *dhl, double *pw, double *dpw, int *warm,
                          double *rho, double *drho, double *mom, double *dmom, double *t,
                          double *dtt, int *status, long long *steps, int n_steps, double cx,
                          double wa, double wb, double *obj, double *dobj, int n_threads) {
  or_material Md = {or_dual(mat[0], dmat[0]), or_dual(mat[1], dmat[1]), or_dual(mat[2], dmat[2]),
                    or_dual(mat[3], dmat[3]), or_dual(mat[4], dmat[4])};
  int nif_tot = iface_off[P];
  int p;
  if (Pp->zone_half < 1 || 2 * Pp->zone_half + 1 > OR_MAXC) return -1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (p = 0; p < P; ++p) {
    or_prob pb;
    int k0 = iface_off[p], nif = iface_off[p + 1] - k0, i;
    long long s0 = slot_off[p];
    int ns = (int)(slot_off[p + 1] - s0);
    real *r = (real *)malloc(sizeof(real) * (ns + 3 * (nif > 0 ? nif : 1) + 1));
    real *m = (real *)malloc(sizeof(real) * ns);
    real *hlk = r + ns, *pwk = hlk + (nif > 0 ? nif : 1), *tp = pwk + 2 * (nif > 0 ? nif : 1);
    for (i = 0; i < ns; ++i) {
      r[i] = or_dual(rho[s0 + i], drho[s0 + i]);
      m[i] = or_dual(mom[s0 + i], dmom[s0 + i]);
    }
    for (i = 0; i < nif; ++i) {
      hlk[i] = or_dual(hl[k0 + i], dhl[k0 + i]);
      pwk[2 * i] = or_dual(pw[2 * (k0 + i)], dpw[2 * (k0 + i)]);
      pwk[2 * i + 1] = or_dual(pw[2 * (k0 + i) + 1], dpw[2 * (k0 + i) + 1]);
    }
    *tp = or_dual(t[p], dtt[p]);
    pb.n = n_cells[p];
    pb.nif = nif;
    pb.h = h[p];
    pb.phase_first = phase_first[p];
    pb.rho = r;
    pb.mom = m;
    pb.home = home + k0;
    pb.hl = hlk;
    pb.pw = pwk;
    pb.warm = warm + k0;
    pb.t = tp;
    pb.status = status + p;
    pb.steps = steps + p;
    pb.tr = NULL;
    pb.tr_k = -1;
    pb.tr_on = 0;
    or_run_problem(&Md, Pp, &pb, n_steps, nif_tot, k0, P, p, NULL, NULL, NULL, NULL, NULL, NULL,
                   NULL, -1);
    real L = or_objective(&pb, x_left[p], cx, wa, wb);
    obj[p] = L.v;
    dobj[p] = L.d;
    for (i = 0; i < ns; ++i) {
      rho[s0 + i] = r[i].v;
      drho[s0 + i] = r[i].d;
      mom[s0 + i] = m[i].v;
      dmom[s0 + i] = m[i].d;
    }
    for (i = 0; i < nif; ++i) {
      hl[k0 + i] = hlk[i].v;
      dhl[k0 + i] = hlk[i].d;
      pw[2 * (k0 + i)] = pwk[2 * i].v;
      dpw[2 * (k0 + i)] = pwk[2 * i].d;
      pw[2 * (k0 + i) + 1] = pwk[2 * i + 1].v;
      dpw[2 * (k0 + i) + 1] = pwk[2 * i + 1].d;
    }
    t[p] = tp->v;
    dtt[p] = tp->d;
    free(r);
    free(m);
  }
  return 0;
}
#endif

#ifndef OR_TANGENT
/* ------------------------------------------------------------------ */
/* fixed-point check: Algorithm 2 to a tight tolerance vs a direct     */
/* Newton solve of the zone's implicit Euler system                    */
/* ------------------------------------------------------------------ */
/* residual R(W) = h^{n+1}(W) W - h^n U^n + dt (F_{c+1/2}(W) - F_{c-1/2}(W)) */
static int or_zone_residual(const or_material *M, const or_params *P, const or_zone *Z,
                            double dt, double W[][2], double *pw, double *R) {
  double F[OR_MAXC + 1][2];
  double w = 0.0;
  int c, q;
  if (!or_zone_fluxes(M, P, Z, W, F, pw, &w)) return 0;
  for (c = 0; c < Z->m; ++c) {
    double hnew = Z->hn[c] + ((double)Z->mov[c] * w) * dt;
    for (q = 0; q < 2; ++q)
      R[2 * c + q] = hnew * W[c][q] - Z->hn[c] * Z->U0[c][q] + dt * (F[c + 1][q] - F[c][q]);
  }
  return 1;
}

static int or_gauss(int n, double *A, double *b) {
  int i, j, k;
  for (k = 0; k < n; ++k) {
    int piv = k;
    for (i = k + 1; i < n; ++i)
      if (fabs(A[i * n + k]) > fabs(A[piv * n + k])) piv = i;
    if (A[piv * n + k] == 0.0) return 0;
    if (piv != k) {
      for (j = 0; j < n; ++j) {
        double tmp = A[k * n + j];
        A[k * n + j] = A[piv * n + j];
        A[piv * n + j] = tmp;
      }
      double tb = b[k];
      b[k] = b[piv];
      b[piv] = tb;
    }
    for (i = k + 1; i < n; ++i) {
      double f = A[i * n + k] / A[k * n + k];
      for (j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (j = i + 1; j < n; ++j) s -= A[i * n + j] * b[j];
    b[i] = s / A[i * n + i];
  }
  return 1;
}

/* For interface k of a single problem at its current state, repeats the
 * set-up of one step (CFL time step, prediction, merge decision), then
 *   (a) runs Algorithm 2 Part 1 with the given parameters and returns the
 *       last iterate in W_dts;
 *   (b) solves the zone's implicit Euler system R(W) = 0 by Newton with a
 *       central-difference Jacobian, started from U^n, into W_newton.
 * m_out gets the number of active zone cells (2 values per cell). */
int oracle_zone_fixed_point(const or_material *M, const or_params *Pp, int n_cells, double h,
                            int phase_first, int nif, double *rho, double *mom, int *home,
                            double *hl, double *pw, int *warm, int k, double *W_dts,
                            double *W_newton, int *m_out, double *dt_out) {
  or_prob pb;
  double t = 0.0;
  int status = 0;
  long long steps = 0;
  memset(&pb, 0, sizeof(pb));
  pb.n = n_cells;
  pb.nif = nif;
  pb.h = h;
  pb.phase_first = phase_first;
  pb.rho = rho;
  pb.mom = mom;
  pb.home = home;
  pb.hl = hl;
  pb.pw = pw;
  pb.warm = warm;
  pb.t = &t;
  pb.status = &status;
  pb.steps = &steps;
  int ns = n_cells + nif, s, c, q;
  int *ph = (int *)malloc(sizeof(int) * ns);
  or_phases(&pb, ph);
  double S = 0.0;
  for (s = 0; s < ns; ++s) {
    double si = fabs(mom[s] / rho[s]) + sqrt(or_a2(M, ph[s]));
    if (si > S) S = si;
  }
  double dt = (Pp->cfl * h) / S;
  *dt_out = dt;
  int zlo, zhi, tr;
  or_zone_range(Pp, &pb, k, &zlo, &zhi, &tr);
  int sL = home[k] + k, sR = sL + 1;
  or_iface I;
  if (!or_iface_solve(M, ph[sL], rho[sL], mom[sL], ph[sR], rho[sR], mom[sR], warm[k],
                          pw[2 * k], pw[2 * k + 1], Pp->newton_maxit, Pp->newton_rtol, &I)) {
    free(ph);
    return -1;
  }
  double ht = tr ? h - hl[k] : hl[k];
  double rate = tr ? -I.w : I.w;
  double hfl = Pp->alpha_floor * h;
  int merge = (ht < hfl) || (ht + (Pp->merge_safety * rate) * dt < hfl);
  or_zone Z;
  if (!or_zone_build(M, Pp, &pb, k, ph, zlo, zhi, tr, merge, I.w, dt, &Z)) {
    free(ph);
    return -2;
  }
  free(ph);
  *m_out = Z.m;
  /* (a) Algorithm 2, Part 1 only */
  double W[OR_MAXC][2], Wn[OR_MAXC][2], F[OR_MAXC + 1][2];
  double pwz[2] = {I.pl, I.pr};
  double w = 0.0;
  int l;
  for (c = 0; c < Z.m; ++c) {
    W[c][0] = Z.U0[c][0];
    W[c][1] = Z.U0[c][1];
  }
  for (l = 0; l < Pp->lmax; ++l) {
    if (!or_zone_fluxes(M, Pp, &Z, W, F, pwz, &w)) return -3;
    double rrel = 0.0;
    for (c = 0; c < Z.m; ++c) {
      double hnew = Z.hn[c] + ((double)Z.mov[c] * w) * dt;
      for (q = 0; q < 2; ++q) {
        double rhs = (Z.hn[c] * Z.U0[c][q] - dt * (F[c + 1][q] - F[c][q])) * (1.0 / hnew);
        Wn[c][q] = (W[c][q] + Z.th[c] * rhs) * Z.i1t[c];
        double sc = fabs(W[c][q]) > 1.0 ? fabs(W[c][q]) : 1.0;
        double rel = fabs(Wn[c][q] - W[c][q]) / sc;
        if (rel > rrel) rrel = rel;
      }
    }
    for (c = 0; c < Z.m; ++c) {
      W[c][0] = Wn[c][0];
      W[c][1] = Wn[c][1];
    }
    if (rrel < Pp->tol_rel) break;
  }
  for (c = 0; c < Z.m; ++c) {
    W_dts[2 * c] = W[c][0];
    W_dts[2 * c + 1] = W[c][1];
  }
  /* (b) Newton with a central-difference Jacobian */
  int n = 2 * Z.m, it, j;
  double X[2 * OR_MAXC], R0[2 * OR_MAXC], Rp[2 * OR_MAXC], Rm[2 * OR_MAXC];
  double *J = (double *)malloc(sizeof(double) * n * n);
  double Wt[OR_MAXC][2];
  for (c = 0; c < Z.m; ++c) {
    X[2 * c] = Z.U0[c][0];
    X[2 * c + 1] = Z.U0[c][1];
  }
  int ok = 0;
  for (it = 0; it < 60; ++it) {
    double pwn[2] = {I.pl, I.pr};
    for (c = 0; c < Z.m; ++c) {
      Wt[c][0] = X[2 * c];
      Wt[c][1] = X[2 * c + 1];
    }
    if (!or_zone_residual(M, Pp, &Z, dt, Wt, pwn, R0)) break;
    for (j = 0; j < n; ++j) {
      double e = 1e-6 * (fabs(X[j]) > 1e-3 ? fabs(X[j]) : 1e-3);
      double pa[2] = {pwn[0], pwn[1]}, pb2[2] = {pwn[0], pwn[1]};
      for (c = 0; c < Z.m; ++c) {
        Wt[c][0] = X[2 * c];
        Wt[c][1] = X[2 * c + 1];
      }
      Wt[j / 2][j % 2] = X[j] + e;
      if (!or_zone_residual(M, Pp, &Z, dt, Wt, pa, Rp)) goto done;
      Wt[j / 2][j % 2] = X[j] - e;
      if (!or_zone_residual(M, Pp, &Z, dt, Wt, pb2, Rm)) goto done;
      for (s = 0; s < n; ++s) J[s * n + j] = (Rp[s] - Rm[s]) / (2.0 * e);
    }
    for (s = 0; s < n; ++s) R0[s] = -R0[s];
    if (!or_gauss(n, J, R0)) break;
    double st = 0.0;
    for (s = 0; s < n; ++s) {
      double sc = fabs(X[s]) > 1.0 ? fabs(X[s]) : 1.0;
      double d = fabs(R0[s]) / sc;
      if (d > st) st = d;
      X[s] += R0[s];
    }
    if (st < 1e-14) {
      ok = 1;
      break;
    }
  }
done:
  free(J);
  for (s = 0; s < n; ++s) W_newton[s] = X[s];
  return ok ? 0 : -4;
}
#endif

#ifndef OR_TANGENT
/* ------------------------------------------------------------------ */
/* a created cell inside the mesh: appendix "Phase Creation", step     */
/* (iv), and the two phase boundaries of the steps that follow it      */
/* ------------------------------------------------------------------ */
/* A creation tube has n regular cells of length h and phase ph; slot n
 * holds the created cell once there is one.  The cell is created on the
 * face j (between cells j-1 and j, the face the Riemann problem of step (i)
 * failed on) and is bounded by two phase boundaries at x_j + dl and
 * x_j + dr; the neighbours take lengths h + dl (cell j-1) and h - dr
 * (cell j), the created cell dr - dl (the picture of the creation step in
 * Sec. 2: the face is gone, two boundary points move apart).  Steps:
 *   - CFL step over every cell, the created one included;
 *   - while there is no created cell: step (i) on every inner face; one
 *     failing face is a creation step: step (ii) there, its two
 *     neighbours updated with the boundary fluxes of step (v) and their
 *     new lengths, the new cell set to the middle star state of step (iv)
 *     with length (w_r - w_l) dt; every other cell explicitly (HLL);
 *   - with a created cell: Algorithm 1 with the zone "created cell +- Z
 *     cells", whose inner faces are HLL faces and the two phase
 *     boundaries (interface solver, eq. pb_flux:pt), Algorithm 2 with the
 *     moving lengths of the three cells next to the boundaries.
 * The created cell is never merged (its neighbours are of the other
 * phase); a neighbour shorter than h/2, a second creation in one problem
 * and a zone reaching past the domain are not modelled and freeze the
 * problem with a status bit. */
#define OR_CT_ST_NEWTON 1
#define OR_CT_ST_NONPHYS 2
#define OR_CT_ST_MESH 4
#define OR_CT_ST_MULTI 8
#define OR_CT_FL_CREATED 1
#define OR_CT_FL_LMAX 2
#define OR_CT_FL_INACTIVE 4

typedef struct {
  int n, ph;
  double h;
  double *rho, *mom; /* n + 1 slots */
  int *face;
  double *dl, *dr, *pw; /* pw: (p_l, p_r) of the left boundary, then of the right one */
  double *t;
  int *status, *steps;
  long long *iters;
} or_ctube;

/* step (i) alone: 1 if the Riemann problem of the two states creates a
 * layer of the other phase (as decided inside or_creation_rp) */
static int or_creation_test(const or_material *M, int ph, double rl, double ml, double rr,
                            double mr, double p_min, double p_tilde) {
  or_side L, R;
  or_side_init(M, ph, rl, ml, &L);
  or_side_init(M, ph, rr, mr, &R);
  double p1 = 0.0;
  int none = or_single_rp(M, &L, &R, &p1);
  return none ? 1 : (ph == OR_LIQ ? p1 < p_min : p1 > p_tilde);
}

/* flux on the regular face j (0 and n: the domain ends) from U */
static void or_ct_face(const or_material *M, const or_params *P, const or_ctube *c,
                       const double *r, const double *m, int j, double *F) {
  if (j == 0)
    or_bflux(M, c->ph, 0, P->bc_left, r[0], m[0], F);
  else if (j == c->n)
    or_bflux(M, c->ph, 1, P->bc_right, r[c->n - 1], m[c->n - 1], F);
  else
    or_hll(M, c->ph, r[j - 1], m[j - 1], r[j], m[j], F);
}

/* length of a zone cell when the left boundary moves with wl and the right
 * one with wr: kind 1 left neighbour, 2 created cell, 3 right neighbour */
static double or_ct_len(double hn, int kind, double wl, double wr, double dt) {
  if (kind == 1) return hn + wl * dt;
  if (kind == 2) return hn + (wr - wl) * dt;
  if (kind == 3) return hn - wr * dt;
  return hn;
}

typedef struct {
  int m, zc; /* cells, index of the created cell */
  int phn;   /* phase of the created cell */
  int kind[OR_MAXC];
  double U0[OR_MAXC][2], hn[OR_MAXC], hh[OR_MAXC], th[OR_MAXC], i1t[OR_MAXC], thr[OR_MAXC];
  double FL[2], FR[2];
} or_ctzone;

/* fluxes of a zone iterate: HLL inside the outer phase, the interface
 * solver on the two phase boundaries (warm starts pwl, pwr updated) */
static int or_ct_fluxes(const or_material *M, const or_params *P, int ph, const or_ctzone *Z,
                        double W[][2], double F[][2], double *pwl, double *pwr, double *wl,
                        double *wr) {
  int c;
  F[0][0] = Z->FL[0];
  F[0][1] = Z->FL[1];
  F[Z->m][0] = Z->FR[0];
  F[Z->m][1] = Z->FR[1];
  for (c = 0; c + 1 < Z->m; ++c) {
    if (c == Z->zc - 1 || c == Z->zc) {
      int left = c == Z->zc - 1;
      double *pw = left ? pwl : pwr;
      or_iface I;
      if (!or_iface_solve(M, left ? ph : Z->phn, W[c][0], W[c][1], left ? Z->phn : ph,
                          W[c + 1][0], W[c + 1][1], 1, pw[0], pw[1], P->newton_maxit,
                          P->newton_rtol, &I))
        return 0;
      pw[0] = I.pl;
      pw[1] = I.pr;
      if (left)
        *wl = I.w;
      else
        *wr = I.w;
      F[c + 1][0] = I.F0;
      F[c + 1][1] = I.F1;
    } else {
      or_hll(M, ph, W[c][0], W[c][1], W[c + 1][0], W[c + 1][1], F[c + 1]);
    }
  }
  return 1;
}

/* Algorithm 2 on the zone of the created cell (pseudo step and stop test as
 * in or_zone_dts); returns 0 or a status bit */
static int or_ct_dts(const or_material *M, const or_params *P, int ph, const or_ctzone *Z,
                     double dt, double *pwl, double *pwr, double U1[][2], double *wls,
                     double *wrs, int *count, int *lmax_hit) {
  double W[OR_MAXC][2], Wn[OR_MAXC][2], F[OR_MAXC + 1][2], hnew[OR_MAXC], ih[OR_MAXC];
  int c, l, m = Z->m, cnt = 0, stop = 0;
  double wl = 0.0, wr = 0.0;
  *lmax_hit = 0;
  for (c = 0; c < m; ++c) {
    W[c][0] = Z->U0[c][0];
    W[c][1] = Z->U0[c][1];
  }
  for (l = 0; l < P->lmax; ++l) {
    if (!or_ct_fluxes(M, P, ph, Z, W, F, pwl, pwr, &wl, &wr)) return OR_CT_ST_NEWTON;
    for (c = 0; c < m; ++c) {
      hnew[c] = or_ct_len(Z->hn[c], Z->kind[c], wl, wr, dt);
      ih[c] = 1.0 / hnew[c];
      if (Z->kind[c] != 0 && !(hnew[c] >= 0.5 * Z->hh[c])) return OR_CT_ST_MESH;
    }
    int conv = 1;
    for (c = 0; c < m; ++c) {
      double th = Z->th[c], opt = 1.0 + th;
      int q;
      for (q = 0; q < 2; ++q) {
        double rhs = (Z->hn[c] * Z->U0[c][q] - dt * (F[c + 1][q] - F[c][q])) * ih[c];
        Wn[c][q] = (W[c][q] + th * rhs) * Z->i1t[c];
        double d = Wn[c][q] - W[c][q];
        double sc = fabs(W[c][q]) > 1.0 ? fabs(W[c][q]) : 1.0;
        int ok = (P->tol_mode == 0) ? (fabs(opt * d) < Z->thr[c] * sc) : (fabs(d) < P->tol_rel * sc);
        conv = conv && ok;
      }
      if (!or_state_ok(Wn[c][0], Wn[c][1])) return OR_CT_ST_NONPHYS;
    }
    for (c = 0; c < m; ++c) {
      W[c][0] = Wn[c][0];
      W[c][1] = Wn[c][1];
    }
    cnt = l + 1;
    stop = conv;
    if (stop) break;
  }
  if (!stop) *lmax_hit = 1;
  *count = cnt;
  /* Part 2 */
  if (!or_ct_fluxes(M, P, ph, Z, W, F, pwl, pwr, &wl, &wr)) return OR_CT_ST_NEWTON;
  for (c = 0; c < m; ++c) {
    hnew[c] = or_ct_len(Z->hn[c], Z->kind[c], wl, wr, dt);
    ih[c] = 1.0 / hnew[c];
    if (Z->kind[c] != 0 && !(hnew[c] >= 0.5 * Z->hh[c])) return OR_CT_ST_MESH;
  }
  for (c = 0; c < m; ++c) {
    int q;
    for (q = 0; q < 2; ++q)
      U1[c][q] = (Z->hn[c] * Z->U0[c][q] - dt * (F[c + 1][q] - F[c][q])) * ih[c];
    if (!or_state_ok(U1[c][0], U1[c][1])) return OR_CT_ST_NONPHYS;
  }
  *wls = wl;
  *wrs = wr;
  return 0;
}

/* Newton on the implicit step of the zone, the alternative to Algorithm 2
 * that the paper's outlook names (a Newton-like solver for the small
 * implicit systems).  Unknowns the zone iterates W (2 per cell), equations
 *   R_c(W) = (h_c(W) / h_c^n) W_c - U_c^n + (dt / h_c^n)(F_{c+1/2}(W) - F_{c-1/2}(W))
 * with the lengths h_c(W) from the boundary speeds at W and the outer zone
 * faces from U^n (the fixed point of Algorithm 2).  From W = U^n: the
 * Jacobian by forward differences (step 1e-7 max(|W_j|, 1), boundary solves
 * warm-started from the current iterate's), the full step; converged when
 * every step component is below rtol max(|W_j|, 1) (the step is taken); at
 * most maxit steps (then flagged like l_max).  Part 2 as in Algorithm 2.
 * The shrink and state checks of Algorithm 2 apply to every iterate.  R_c
 * depends on W_{c-1}, W_c, W_{c+1} only (the created cell's length on both
 * boundary speeds, each neighbour's on its own boundary), so the 2x2 blocks
 * beside the diagonal of the difference Jacobian are kept and the system is
 * solved by or_block_tri, as for the batch path's zones. */
#define OR_CT_NMAX (2 * OR_MAXC)

static int or_ct_resid(const or_material *M, const or_params *P, int ph, const or_ctzone *Z,
                       double dt, double W[][2], double *pwl, double *pwr, double *R,
                       double *wl, double *wr, int check) {
  double F[OR_MAXC + 1][2];
  int c, q;
  if (!or_ct_fluxes(M, P, ph, Z, W, F, pwl, pwr, wl, wr)) return OR_CT_ST_NEWTON;
  for (c = 0; c < Z->m; ++c) {
    double hk = or_ct_len(Z->hn[c], Z->kind[c], *wl, *wr, dt);
    if (check && Z->kind[c] != 0 && !(hk >= 0.5 * Z->hh[c])) return OR_CT_ST_MESH;
    double ihn = 1.0 / Z->hn[c];
    for (q = 0; q < 2; ++q)
      R[2 * c + q] = (hk * ihn) * W[c][q] - Z->U0[c][q] + (dt * ihn) * (F[c + 1][q] - F[c][q]);
  }
  return 0;
}

static int or_ct_newton(const or_material *M, const or_params *P, int ph, const or_ctzone *Z,
                        double dt, double *pwl, double *pwr, int maxit, double rtol,
                        double U1[][2], double *wls, double *wrs, int *count, int *lmax_hit) {
  int m = Z->m, n = 2 * m, c, q, j, it, conv = 0;
  double W[OR_MAXC][2], R[OR_CT_NMAX], Rp[OR_CT_NMAX], J[OR_CT_NMAX][OR_CT_NMAX];
  double Db[OR_MAXC][2][2], Lb[OR_MAXC][2][2], Ub[OR_MAXC][2][2], rb[OR_MAXC][2], d[OR_MAXC][2];
  double wl = 0.0, wr = 0.0;
  *lmax_hit = 0;
  *count = 0;
  for (c = 0; c < m; ++c) {
    W[c][0] = Z->U0[c][0];
    W[c][1] = Z->U0[c][1];
  }
  for (it = 0; it < maxit && !conv; ++it) {
    int st = or_ct_resid(M, P, ph, Z, dt, W, pwl, pwr, R, &wl, &wr, 1);
    if (st) return st;
    for (j = 0; j < n; ++j) {
      int cj = j / 2, qj = j % 2;
      double xj = W[cj][qj];
      double e = 1e-7 * (fabs(xj) > 1.0 ? fabs(xj) : 1.0);
      double gl[2] = {pwl[0], pwl[1]}, gr[2] = {pwr[0], pwr[1]}, a, b2;
      W[cj][qj] = xj + e;
      st = or_ct_resid(M, P, ph, Z, dt, W, gl, gr, Rp, &a, &b2, 0);
      W[cj][qj] = xj;
      if (st) return st;
      for (q = 0; q < n; ++q) J[q][j] = (Rp[q] - R[q]) / e;
    }
    for (c = 0; c < m; ++c) {
      int a, b;
      for (a = 0; a < 2; ++a) {
        rb[c][a] = -R[2 * c + a];
        for (b = 0; b < 2; ++b) {
          Db[c][a][b] = J[2 * c + a][2 * c + b];
          Lb[c][a][b] = c > 0 ? J[2 * c + a][2 * (c - 1) + b] : 0.0;
          Ub[c][a][b] = c + 1 < m ? J[2 * c + a][2 * (c + 1) + b] : 0.0;
        }
      }
    }
    if (!or_block_tri(m, Db, Lb, Ub, rb, d)) return OR_CT_ST_NEWTON;
    conv = 1;
    for (j = 0; j < n; ++j) {
      double xj = W[j / 2][j % 2];
      double sc = fabs(xj) > 1.0 ? fabs(xj) : 1.0;
      conv = conv && (fabs(d[j / 2][j % 2]) <= rtol * sc);
    }
    for (c = 0; c < m; ++c) {
      W[c][0] = W[c][0] + d[c][0];
      W[c][1] = W[c][1] + d[c][1];
      if (!or_state_ok(W[c][0], W[c][1])) return OR_CT_ST_NONPHYS;
    }
    *count = it + 1;
  }
  if (!conv) *lmax_hit = 1;
  /* Part 2 */
  double F[OR_MAXC + 1][2], ih[OR_MAXC];
  if (!or_ct_fluxes(M, P, ph, Z, W, F, pwl, pwr, &wl, &wr)) return OR_CT_ST_NEWTON;
  for (c = 0; c < m; ++c) {
    double hk = or_ct_len(Z->hn[c], Z->kind[c], wl, wr, dt);
    ih[c] = 1.0 / hk;
    if (Z->kind[c] != 0 && !(hk >= 0.5 * Z->hh[c])) return OR_CT_ST_MESH;
  }
  for (c = 0; c < m; ++c) {
    for (q = 0; q < 2; ++q)
      U1[c][q] = (Z->hn[c] * Z->U0[c][q] - dt * (F[c + 1][q] - F[c][q])) * ih[c];
    if (!or_state_ok(U1[c][0], U1[c][1])) return OR_CT_ST_NONPHYS;
  }
  *wls = wl;
  *wrs = wr;
  return 0;
}

/* one physical step of one creation tube; *count, *flags: its log entry */
static void or_ct_step(const or_material *M, const or_params *P, double p_min, double p_tilde,
                       int solver, int zn_maxit, double zn_rtol, or_ctube *c, double *rn,
                       double *mn, double *F, int *count, int *flags) {
  int n = c->n, s, j;
  double h = c->h;
  double *r = c->rho, *m = c->mom;
  int j0 = *c->face;
  /* a tube that fails the checks at the start of its step (mesh, CFL)
   * logs the step as inactive: nothing of it was done */
  *count = 0;
  *flags = OR_CT_FL_INACTIVE;
  if (*c->status || !(*c->t < P->t_end)) return;
  if (j0 >= 0) {
    double dl = *c->dl, dr = *c->dr;
    if (!(h + dl >= 0.5 * h) || !(h - dr >= 0.5 * h) || !(dr - dl > 0.0) ||
        j0 - P->zone_half < 0 || j0 + P->zone_half > n) {
      *c->status |= OR_CT_ST_MESH;
      return;
    }
  }
  /* CFL (eq. cfl_cond:unif) over every cell, the created one included */
  double S = 0.0;
  int ns = j0 >= 0 ? n + 1 : n;
  for (s = 0; s < ns; ++s) {
    int phs = s < n ? c->ph : 1 - c->ph;
    if (!or_state_ok(r[s], m[s])) {
      *c->status |= OR_CT_ST_NONPHYS;
      return;
    }
    double si = fabs(m[s] / r[s]) + sqrt(or_a2(M, phs));
    if (si > S) S = si;
  }
  if (!(S > 0.0) || !isfinite(S)) {
    *c->status |= OR_CT_ST_NONPHYS;
    return;
  }
  *flags = 0;
  double dt = (P->cfl * h) / S;
  double rem = P->t_end - *c->t;
  int clipped = 0;
  if (dt >= rem) {
    dt = rem;
    clipped = 1;
  }
  double lam = dt / h;
  /* cells updated by the explicit sweep: [0, a) and [b, n) */
  int a = n, b = n, jc = -1;
  if (j0 < 0) {
    /* step (i) on every inner face */
    int nc = 0;
    for (j = 1; j < n; ++j)
      if (or_creation_test(M, c->ph, r[j - 1], m[j - 1], r[j], m[j], p_min, p_tilde)) {
        if (jc < 0) jc = j;
        ++nc;
      }
    if (nc > 1) {
      *c->status |= OR_CT_ST_MULTI;
      return;
    }
    if (jc >= 0) {
      a = jc - 1;
      b = jc + 1;
    }
  } else {
    a = j0 - P->zone_half;
    b = j0 + P->zone_half;
  }
  for (j = 0; j <= n; ++j)
    if (j <= a || j >= b) or_ct_face(M, P, c, r, m, j, &F[2 * j]);
  for (s = 0; s < n; ++s) {
    rn[s] = r[s];
    mn[s] = m[s];
    if (s >= a && s < b) continue;
    rn[s] = r[s] - lam * (F[2 * (s + 1)] - F[2 * s]);
    mn[s] = m[s] - lam * (F[2 * (s + 1) + 1] - F[2 * s + 1]);
  }
  rn[n] = r[n];
  mn[n] = m[n];
  int cnt = 0, fl = 0, st = 0;
  double ndl = 0.0, ndr = 0.0, pw4[4] = {0.0, 0.0, 0.0, 0.0};
  if (jc >= 0) {
    /* creation step: steps (ii), (iii), (v) on face jc, step (iv) */
    or_creation C;
    if (or_creation_rp(M, c->ph, r[jc - 1], m[jc - 1], r[jc], m[jc], p_min, p_tilde,
                       P->newton_maxit, P->newton_rtol, &C) != 1) {
      st = OR_CT_ST_NEWTON;
    } else {
      double h1l = h + C.wl * dt, h1r = h - C.wr * dt;
      ndl = C.wl * dt;
      ndr = C.wr * dt;
      if (!(h1l > 0.0) || !(h1r > 0.0) || !(ndr - ndl > 0.0)) {
        st = OR_CT_ST_MESH;
      } else {
        double il = 1.0 / h1l, ir = 1.0 / h1r;
        rn[jc - 1] = (h * r[jc - 1] - dt * (C.Fl0 - F[2 * (jc - 1)])) * il;
        mn[jc - 1] = (h * m[jc - 1] - dt * (C.Fl1 - F[2 * (jc - 1) + 1])) * il;
        rn[jc] = (h * r[jc] - dt * (F[2 * (jc + 1)] - C.Fr0)) * ir;
        mn[jc] = (h * m[jc] - dt * (F[2 * (jc + 1) + 1] - C.Fr1)) * ir;
        rn[n] = C.rb;
        mn[n] = C.rb * C.ub;
        pw4[0] = C.pa;
        pw4[1] = C.pb;
        pw4[2] = C.pb;
        pw4[3] = C.pc;
        if (!or_state_ok(rn[jc - 1], mn[jc - 1]) || !or_state_ok(rn[jc], mn[jc]) ||
            !or_state_ok(rn[n], mn[n]))
          st = OR_CT_ST_NONPHYS;
        fl = OR_CT_FL_CREATED;
      }
    }
  } else if (j0 >= 0) {
    /* Algorithm 2 on cells j0-Z .. j0-1, the created cell, j0 .. j0+Z-1 */
    int Zh = P->zone_half, k;
    double dl = *c->dl, dr = *c->dr;
    or_ctzone Z;
    Z.m = 2 * Zh + 1;
    Z.zc = Zh;
    Z.phn = 1 - c->ph;
    for (k = 0; k < Z.m; ++k) {
      int sl = k < Zh ? j0 - Zh + k : (k == Zh ? n : j0 + (k - Zh - 1));
      Z.U0[k][0] = r[sl];
      Z.U0[k][1] = m[sl];
      Z.kind[k] = k == Zh - 1 ? 1 : (k == Zh ? 2 : (k == Zh + 1 ? 3 : 0));
      Z.hn[k] = k == Zh - 1 ? h + dl : (k == Zh ? dr - dl : (k == Zh + 1 ? h - dr : h));
    }
    or_ct_face(M, P, c, r, m, a, Z.FL);
    or_ct_face(M, P, c, r, m, b, Z.FR);
    /* explicit prediction of both boundary speeds from U^n */
    or_iface Il, Ir;
    double *pw = c->pw;
    if (!or_iface_solve(M, c->ph, r[j0 - 1], m[j0 - 1], Z.phn, r[n], m[n], 1, pw[0], pw[1],
                        P->newton_maxit, P->newton_rtol, &Il) ||
        !or_iface_solve(M, Z.phn, r[n], m[n], c->ph, r[j0], m[j0], 1, pw[2], pw[3],
                        P->newton_maxit, P->newton_rtol, &Ir)) {
      st = OR_CT_ST_NEWTON;
    } else {
      for (k = 0; k < Z.m && !st; ++k) {
        double hh = or_ct_len(Z.hn[k], Z.kind[k], Il.w, Ir.w, dt);
        double th = hh / h;
        if (th > P->theta_nb) th = P->theta_nb;
        Z.hh[k] = hh;
        Z.th[k] = th;
        Z.i1t[k] = 1.0 / (1.0 + th);
        Z.thr[k] = (k == Zh ? P->tol_tiny : P->tol_nb) * (th * dt);
        if (!(th > 0.0)) st = OR_CT_ST_MESH;
      }
      double pwl[2] = {Il.pl, Il.pr}, pwr[2] = {Ir.pl, Ir.pr};
      double U1[OR_MAXC][2], wl = 0.0, wr = 0.0;
      int lh = 0;
      if (!st) {
        if (solver == 1)
          st = or_ct_newton(M, P, c->ph, &Z, dt, pwl, pwr, zn_maxit, zn_rtol, U1, &wl, &wr, &cnt,
                            &lh);
        else
          st = or_ct_dts(M, P, c->ph, &Z, dt, pwl, pwr, U1, &wl, &wr, &cnt, &lh);
      }
      if (!st) {
        for (k = 0; k < Z.m; ++k) {
          int sl = k < Zh ? j0 - Zh + k : (k == Zh ? n : j0 + (k - Zh - 1));
          rn[sl] = U1[k][0];
          mn[sl] = U1[k][1];
        }
        ndl = dl + wl * dt;
        ndr = dr + wr * dt;
        pw4[0] = pwl[0];
        pw4[1] = pwl[1];
        pw4[2] = pwr[0];
        pw4[3] = pwr[1];
        if (lh) fl |= OR_CT_FL_LMAX;
      }
    }
  }
  if (st) {
    *c->status |= st;
    *flags = fl;
    return;
  }
  memcpy(r, rn, sizeof(double) * (n + 1));
  memcpy(m, mn, sizeof(double) * (n + 1));
  if (jc >= 0) *c->face = jc;
  if (jc >= 0 || j0 >= 0) {
    *c->dl = ndl;
    *c->dr = ndr;
    memcpy(c->pw, pw4, sizeof(pw4));
  }
  *c->t = clipped ? P->t_end : *c->t + dt;
  *c->steps += 1;
  *c->iters += cnt;
  *count = cnt;
  *flags = fl;
}

/* n_steps steps of P independent creation tubes (OpenMP over tubes), the
 * zone solved by Algorithm 2 (solver 0) or by Newton (solver 1, at most
 * zn_maxit steps, tolerance zn_rtol).  Tube
 * p has n_cells[p] regular cells and n_cells[p] + 1 slots from off[p];
 * face, dl, dr, pw (4 per tube), t, status, steps, iters are its state.
 * Logs (optional) are [n_steps][P]. */
int oracle_ct_run(const or_material *M, const or_params *Pp, double p_min, double p_tilde,
                  int solver, int zn_maxit, double zn_rtol,
                  int P, const int *n_cells, const double *h, const int *phase,
                  const long long *off, double *rho, double *mom, int *face, double *dl,
                  double *dr, double *pw, double *t, int *status, int *steps, long long *iters,
                  int n_steps, int *log_count, int *log_flags, int n_threads) {
  int p;
  if (Pp->zone_half < 1 || 2 * Pp->zone_half + 1 > OR_MAXC) return -1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (p = 0; p < P; ++p) {
    or_ctube c;
    c.n = n_cells[p];
    c.ph = phase[p];
    c.h = h[p];
    c.rho = rho + off[p];
    c.mom = mom + off[p];
    c.face = face + p;
    c.dl = dl + p;
    c.dr = dr + p;
    c.pw = pw + 4 * (size_t)p;
    c.t = t + p;
    c.status = status + p;
    c.steps = steps + p;
    c.iters = iters + p;
    double *rn = (double *)malloc(sizeof(double) * (2 * (size_t)(c.n + 1) + 2 * (size_t)(c.n + 1)));
    double *mn = rn + (c.n + 1), *F = mn + (c.n + 1);
    int k;
    for (k = 0; k < n_steps; ++k) {
      int cnt, fl;
      if (!log_count && (*c.status || !(*c.t < Pp->t_end))) break;
      or_ct_step(M, Pp, p_min, p_tilde, solver, zn_maxit, zn_rtol, &c, rn, mn, F, &cnt, &fl);
      if (log_count) {
        log_count[(size_t)k * P + p] = cnt;
        log_flags[(size_t)k * P + p] = fl;
      }
    }
    free(rn);
  }
  return 0;
}
#endif
