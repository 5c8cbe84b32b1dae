/*
 * euler_oracle.c -- plain, slow, FP64 CPU oracle of the mixed explicit-implicit
 * scheme with dual time stepping applied to the full 1D Euler equations of an
 * ideal gas on a fixed mesh with one small cell (the first test of Sec. 4,
 * "stationary phase boundary without phase transition": the Lax shock tube
 * and its study of the local pseudo time step factors theta_i).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the package smoke check and the
 * bench's cpu_baseline leg may load it.  It shares no code, header or table
 * with the HIP library.  It is linked into the same shared object as the
 * isothermal oracle and borrows that file's fixed-order logarithm.
 *
 * What it follows:
 *   - the model mesh of Fig. 1: N cells of length h = (x_R - x_L)/N and one
 *     small cell I_k of length alpha h whose left face sits at x = 0, so the
 *     domain is [x_L, x_R + alpha h];
 *   - Godunov's method (eq. godunov_meth:unif) with the exact Riemann solution
 *     of the Euler equations sampled on the (fixed) face;
 *   - Algorithm 1 (explicit update of all cells except I_{k-1}, I_k, I_{k+1},
 *     saving F_left = F_{k-3/2} and F_right = F_{k+3/2}) and Algorithm 2
 *     (dual time stepping on the three cells with Delta tau_i = theta_i Delta t,
 *     then Part 2, the conservative update with fluxes of the accepted
 *     iterate);
 *   - the residual and stopping rule of Sec. 4: res_{k-1}, res_{k+1} < tol_nb
 *     and res_k < tol_k;
 *   - the time step of eq. cfl_cond:unif with the regular length h.
 *
 * Readings where the paper is silent: the wave speed bound S^n is
 * max_i(|u_i| + a_i) over all cells at t^n, the last step is clipped to
 * t_end (t = t_end after it) while its pseudo steps stay theta_i Delta t_ref
 * with the unclipped CFL step Delta t_ref, both outer boundaries are transmissive (boundary flux = F(U) of the
 * boundary cell), max(U, 1) in the residual is taken as max(|U|, 1) per
 * component, and the stop test is evaluated multiplied out,
 * |(1 + theta_i) dW| < tol_i theta_i Delta t max(|W|, 1).
 *
 * The exact Riemann solver is written from the wave curves of the ideal gas
 * (shock: Rankine-Hugoniot; rarefaction: isentrope and Riemann invariant),
 * Newton's method on the star pressure from the linearised (primitive
 * variable) guess, and sampling of the self-similar solution at x/t = 0.
 * Powers with non-integer exponents are exp(e log x) through fixed-order
 * routines so that every IEEE machine gives the same bits.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

double oracle_log(double x); /* fixed-order logarithm of the isothermal oracle */

#define EU_ST_VACUUM 1  /* a Riemann problem generates vacuum */
#define EU_ST_NEWTON 2  /* Newton on the star pressure did not converge */
#define EU_ST_NONPHYS 4 /* a cell left rho > 0, p > 0 */
#define EU_FL_LMAX 1    /* dual time stepping stopped at l_max */

#define EU_NEWTON_MAXIT 60

/* exp of a finite double: x = k ln2 + r with k = nearest integer to x/ln2 and
 * ln2 split into a head with trailing zero bits and a tail (Cody and Waite),
 * |r| <= ln2/2; exp(r) by its Taylor polynomial of degree 13 evaluated with
 * Estrin's scheme; then multiplied by 2^k through the exponent field (two
 * factors, so results near the range ends are still scaled exactly).
 * Plain IEEE operations in a fixed order; a few ulp accurate. */
double oracle_exp(double x) {
  if (x != x) return x;
  if (x > 709.782712893384) return INFINITY;
  if (x < -745.1332191019412) return 0.0;
  double kf = floor(x * 1.4426950408889634 + 0.5);
  double r = (x - kf * 0x1.62e42feep-1) - kf * 0x1.a39ef35793c76p-33;
  double r2 = r * r, r4 = r2 * r2, r8 = r4 * r4;
  double c0 = 1.0 + r, c1 = (1.0 / 2.0) + (1.0 / 6.0) * r;
  double c2 = (1.0 / 24.0) + (1.0 / 120.0) * r, c3 = (1.0 / 720.0) + (1.0 / 5040.0) * r;
  double c4 = (1.0 / 40320.0) + (1.0 / 362880.0) * r;
  double c5 = (1.0 / 3628800.0) + (1.0 / 39916800.0) * r;
  double c6 = (1.0 / 479001600.0) + (1.0 / 6227020800.0) * r;
  double d0 = c0 + c1 * r2, d1 = c2 + c3 * r2, d2 = c4 + c5 * r2;
  double e0 = d0 + d1 * r4, e1 = d2 + c6 * r4;
  double p = e0 + e1 * r8;
  int k = (int)kf;
  int k1 = k / 2, k2 = k - k1;
  uint64_t b1 = (uint64_t)(int64_t)(k1 + 1023) << 52, b2 = (uint64_t)(int64_t)(k2 + 1023) << 52;
  double s1, s2;
  memcpy(&s1, &b1, 8);
  memcpy(&s2, &b2, 8);
  return (p * s1) * s2;
}

/* x^e for x > 0 */
static double eu_pow(double x, double e) { return oracle_exp(e * oracle_log(x)); }

/* ideal gas constants derived from gamma once per call */
typedef struct {
  double g;    /* gamma */
  double gm1;  /* gamma - 1 */
  double e1;   /* (gamma - 1) / (2 gamma): exponent of p on the isentrope for a */
  double ig;   /* 1 / gamma */
  double e5;   /* 2 / (gamma - 1) */
  double e7;   /* 2 gamma / (gamma - 1) */
  double mu;   /* (gamma - 1) / (gamma + 1) */
  double gp;   /* 2 / (gamma + 1) */
  double sk;   /* (gamma + 1) / (2 gamma) */
} eu_gas;

static eu_gas eu_make_gas(double g) {
  eu_gas G;
  G.g = g;
  G.gm1 = g - 1.0;
  G.e1 = (g - 1.0) / (2.0 * g);
  G.ig = 1.0 / g;
  G.e5 = 2.0 / (g - 1.0);
  G.e7 = 2.0 * g / (g - 1.0);
  G.mu = (g - 1.0) / (g + 1.0);
  G.gp = 2.0 / (g + 1.0);
  G.sk = (g + 1.0) / (2.0 * g);
  return G;
}

/* Velocity jump across the K-wave connecting (rK, pK, aK) to pressure p:
 * a shock (p > pK) from the Rankine-Hugoniot conditions, else a rarefaction
 * from the isentrope and the Riemann invariant.  Also its derivative in p. */
static void eu_wave(const eu_gas *G, double p, double rK, double pK, double aK, double *f,
                    double *df) {
  if (p > pK) {
    double A = G->gp / rK, B = G->mu * pK;
    double q = sqrt(A / (p + B));
    *f = (p - pK) * q;
    *df = q * (1.0 - 0.5 * (p - pK) / (p + B));
  } else {
    double pr = p / pK;
    double t = eu_pow(pr, G->e1);
    *f = G->e5 * aK * (t - 1.0);
    *df = t / (rK * aK * pr);
  }
}

/* Star region of the Riemann problem (rL,uL,pL | rR,uR,pR): returns 0 and
 * the star pressure/velocity, EU_ST_VACUUM if the data generate vacuum,
 * EU_ST_NEWTON if Newton's method does not converge. */
static int eu_star(const eu_gas *G, const double *WL, const double *WR, double aL, double aR,
                   double *ps, double *us) {
  double rL = WL[0], uL = WL[1], pL = WL[2];
  double rR = WR[0], uR = WR[1], pR = WR[2];
  double du = uR - uL;
  if (G->e5 * (aL + aR) <= du) return EU_ST_VACUUM;
  double ppv = 0.5 * (pL + pR) - 0.125 * du * (rL + rR) * (aL + aR);
  double pfloor = 1e-6 * (pL < pR ? pL : pR);
  double p = ppv > pfloor ? ppv : pfloor;
  double fL, dfL, fR, dfR;
  int it;
  for (it = 0; it < EU_NEWTON_MAXIT; ++it) {
    eu_wave(G, p, rL, pL, aL, &fL, &dfL);
    eu_wave(G, p, rR, pR, aR, &fR, &dfR);
    double pn = p - (fL + fR + du) / (dfL + dfR);
    if (!(pn > 0.0)) pn = 0.5 * p;
    double ch = fabs(pn - p);
    p = pn;
    if (ch <= 1e-14 * pn) break;
  }
  if (it == EU_NEWTON_MAXIT || !(p > 0.0) || !isfinite(p)) return EU_ST_NEWTON;
  eu_wave(G, p, rL, pL, aL, &fL, &dfL);
  eu_wave(G, p, rR, pR, aR, &fR, &dfR);
  *ps = p;
  *us = 0.5 * (uL + uR) + 0.5 * (fR - fL);
  return 0;
}

/* Physical flux of the primitive state W = (rho, u, p). */
static void eu_flux(const eu_gas *G, const double *W, double *F) {
  double m = W[0] * W[1];
  double E = W[2] / G->gm1 + 0.5 * m * W[1];
  F[0] = m;
  F[1] = m * W[1] + W[2];
  F[2] = W[1] * (E + W[2]);
}

/* Exact Riemann solution sampled at x/t = 0 (the fixed face) and its flux.
 * star (optional): p*, u*, rho*_L, rho*_R.  Returns 0 or an EU_ST_ code. */
static int eu_godunov(const eu_gas *G, const double *WL, const double *WR, double *W0,
                      double *F, double *star) {
  double aL = sqrt(G->g * WL[2] / WL[0]), aR = sqrt(G->g * WR[2] / WR[0]);
  double ps, us;
  int st = eu_star(G, WL, WR, aL, aR, &ps, &us);
  if (st) return st;
  double rsL, rsR;
  {
    double q = ps / WL[2];
    rsL = ps > WL[2] ? WL[0] * ((q + G->mu) / (G->mu * q + 1.0)) : WL[0] * eu_pow(q, G->ig);
    q = ps / WR[2];
    rsR = ps > WR[2] ? WR[0] * ((q + G->mu) / (G->mu * q + 1.0)) : WR[0] * eu_pow(q, G->ig);
  }
  if (star) {
    star[0] = ps;
    star[1] = us;
    star[2] = rsL;
    star[3] = rsR;
  }
  if (us >= 0.0) { /* the face sees the left wave or the left star state */
    double rL = WL[0], uL = WL[1], pL = WL[2];
    if (ps > pL) { /* left shock */
      double S = uL - aL * sqrt(G->sk * (ps / pL) + G->e1);
      if (S >= 0.0) {
        memcpy(W0, WL, 3 * sizeof(double));
      } else {
        W0[0] = rsL;
        W0[1] = us;
        W0[2] = ps;
      }
    } else { /* left rarefaction */
      double Sh = uL - aL;
      if (Sh >= 0.0) {
        memcpy(W0, WL, 3 * sizeof(double));
      } else {
        double asL = aL * eu_pow(ps / pL, G->e1);
        double St = us - asL;
        if (St < 0.0) {
          W0[0] = rsL;
          W0[1] = us;
          W0[2] = ps;
        } else { /* the face is inside the fan: u - a = 0 there */
          double c = G->gp * (aL + 0.5 * G->gm1 * uL);
          double q = c / aL;
          W0[0] = rL * eu_pow(q, G->e5);
          W0[1] = c;
          W0[2] = pL * eu_pow(q, G->e7);
        }
      }
    }
  } else { /* right wave or right star state */
    double rR = WR[0], uR = WR[1], pR = WR[2];
    if (ps > pR) {
      double S = uR + aR * sqrt(G->sk * (ps / pR) + G->e1);
      if (S <= 0.0) {
        memcpy(W0, WR, 3 * sizeof(double));
      } else {
        W0[0] = rsR;
        W0[1] = us;
        W0[2] = ps;
      }
    } else {
      double Sh = uR + aR;
      if (Sh <= 0.0) {
        memcpy(W0, WR, 3 * sizeof(double));
      } else {
        double asR = aR * eu_pow(ps / pR, G->e1);
        double St = us + asR;
        if (St > 0.0) {
          W0[0] = rsR;
          W0[1] = us;
          W0[2] = ps;
        } else { /* inside the right fan: u + a = 0 there */
          double c = G->gp * (aR - 0.5 * G->gm1 * uR);
          double q = c / aR;
          W0[0] = rR * eu_pow(q, G->e5);
          W0[1] = -c;
          W0[2] = pR * eu_pow(q, G->e7);
        }
      }
    }
  }
  eu_flux(G, W0, F);
  return 0;
}

/* conserved (rho, m, E) -> primitive (rho, u, p); 0 if not physical */
static int eu_prim(const eu_gas *G, const double *U, double *W) {
  double r = U[0];
  double u = U[1] / r;
  double p = G->gm1 * (U[2] - 0.5 * U[1] * u);
  W[0] = r;
  W[1] = u;
  W[2] = p;
  return r > 0.0 && p > 0.0 && isfinite(r) && isfinite(p) && isfinite(u);
}

/* Godunov flux between two conserved states */
static int eu_face(const eu_gas *G, const double *UL, const double *UR, double *F) {
  double WL[3], WR[3], W0[3];
  if (!eu_prim(G, UL, WL) || !eu_prim(G, UR, WR)) return EU_ST_NONPHYS;
  return eu_godunov(G, WL, WR, W0, F, 0);
}

/* exported exact solver for the tests: W0 = state at x/t = 0, F its flux,
 * star = (p*, u*, rho*_L, rho*_R) */
int oracle_euler_riemann(double gamma, const double *WL, const double *WR, double *W0,
                         double *F, double *star) {
  eu_gas G = eu_make_gas(gamma);
  return eu_godunov(&G, WL, WR, W0, F, star);
}

typedef struct {
  double gamma, tol_nb, tol_k;
  int lmax;
} eu_params;

/* stop test of Sec. 4 for one cell */
static int eu_cell_done(const double *Wold, const double *Wnew, double th, double thr) {
  for (int c = 0; c < 3; ++c) {
    double d = (1.0 + th) * (Wnew[c] - Wold[c]);
    double s = fabs(Wold[c]);
    if (s < 1.0) s = 1.0;
    if (!(fabs(d) < thr * s)) return 0;
  }
  return 1;
}

/* One time step of one problem (Algorithm 1 with Algorithm 2 on the cells
 * k-1, k, k+1).  U is the problem's state, 3 arrays of n = N + 1 cells.
 * Returns 0 or the EU_ST_ bits of every failure met: the explicit part
 * evaluates all of its faces and the implicit part runs as well, so the bits
 * do not depend on the order of the two parts.  After a failure the state of
 * the problem is not meaningful.  *cnt = dual time iterations, *fl = EU_FL_
 * bits. */
static int eu_step(const eu_gas *G, const eu_params *P, int N, double h, double alpha,
                   double th_nb, double th_k, double dt, double dtref, int clip, double *rho,
                   double *mom, double *ene, double *F, int *cnt, int *fl) {
  int n = N + 1, k = N / 2;
  double hk = alpha * h;
  int st = 0;
  *cnt = 0;
  *fl = 0;
  /* Algorithm 1, Step 1 (a): fluxes of U^n on every face but the two faces of
   * the small cell; boundary faces transmissive.  F holds 3 (n + 1) values,
   * face j between cells j-1 and j. */
  for (int j = 0; j <= n; ++j) {
    double *Fj = F + 3 * j;
    if (j == 0 || j == n) {
      int i = j == 0 ? 0 : n - 1;
      double U[3] = {rho[i], mom[i], ene[i]}, W[3];
      if (!eu_prim(G, U, W)) {
        st |= EU_ST_NONPHYS;
        continue;
      }
      eu_flux(G, W, Fj);
      continue;
    }
    if (j == k || j == k + 1) continue;
    double UL[3] = {rho[j - 1], mom[j - 1], ene[j - 1]};
    double UR[3] = {rho[j], mom[j], ene[j]};
    st |= eu_face(G, UL, UR, Fj);
  }
  /* Algorithm 2 works on U^n of the three cells and the saved fluxes
   * F_left = F_{k-3/2}, F_right = F_{k+3/2} */
  double Un[3][3], Fleft[3], Fright[3];
  for (int q = 0; q < 3; ++q) {
    Un[q][0] = rho[k - 1 + q];
    Un[q][1] = mom[k - 1 + q];
    Un[q][2] = ene[k - 1 + q];
  }
  int stz = 0;
  {
    double Um2[3] = {rho[k - 2], mom[k - 2], ene[k - 2]};
    double Up2[3] = {rho[k + 2], mom[k + 2], ene[k + 2]};
    stz |= eu_face(G, Um2, Un[0], Fleft);
    stz |= eu_face(G, Un[2], Up2, Fright);
  }
  /* Step 1 (b): explicit update away from the small cell */
  double lam = dt / h;
  for (int i = 0; i < n; ++i) {
    if (i >= k - 1 && i <= k + 1) continue;
    double *Fl = F + 3 * i, *Fr = F + 3 * (i + 1);
    rho[i] = rho[i] - lam * (Fr[0] - Fl[0]);
    mom[i] = mom[i] - lam * (Fr[1] - Fl[1]);
    ene[i] = ene[i] - lam * (Fr[2] - Fl[2]);
  }
  if (stz) return st | stz;
  /* Algorithm 2, Part 1: dual time stepping from W^0 = U^n with the pseudo
   * steps Delta tau_i = theta_i Delta t_ref of Sec. 4, Delta t_ref the CFL step;
   * Delta t = Delta t_ref but on a step clipped to t_end, where the update
   * takes the ratio Delta tau_i / Delta t */
  double lamk = dt / hk;
  double tau[3] = {th_nb * dtref, th_k * dtref, th_nb * dtref};
  double th[3] = {th_nb, th_k, th_nb};
  if (clip)
    for (int q = 0; q < 3; ++q) th[q] = tau[q] / dt;
  double thr[3] = {P->tol_nb * tau[0], P->tol_k * tau[1], P->tol_nb * tau[2]};
  double W[3][3], Wn[3][3], Fkm[3], Fkp[3];
  memcpy(W, Un, sizeof(W));
  int l, done = 0;
  for (l = 0; l <= P->lmax; ++l) {
    stz = eu_face(G, W[0], W[1], Fkm) | eu_face(G, W[1], W[2], Fkp);
    if (stz) return st | stz;
    for (int c = 0; c < 3; ++c) {
      Wn[0][c] = (W[0][c] + th[0] * (Un[0][c] - lam * (Fkm[c] - Fleft[c]))) / (1.0 + th[0]);
      Wn[1][c] = (W[1][c] + th[1] * (Un[1][c] - lamk * (Fkp[c] - Fkm[c]))) / (1.0 + th[1]);
      Wn[2][c] = (W[2][c] + th[2] * (Un[2][c] - lam * (Fright[c] - Fkp[c]))) / (1.0 + th[2]);
    }
    done = 1;
    for (int q = 0; q < 3; ++q)
      if (!eu_cell_done(W[q], Wn[q], th[q], thr[q])) done = 0;
    memcpy(W, Wn, sizeof(W));
    if (done) break;
  }
  if (!done) {
    *fl |= EU_FL_LMAX;
    l = P->lmax;
  }
  *cnt = l + 1;
  /* Part 2: fluxes of the accepted iterate, conservative update */
  stz = eu_face(G, W[0], W[1], Fkm) | eu_face(G, W[1], W[2], Fkp);
  if (stz) return st | stz;
  double *cell[3] = {rho, mom, ene};
  for (int c = 0; c < 3; ++c) {
    cell[c][k - 1] = Un[0][c] - lam * (Fkm[c] - Fleft[c]);
    cell[c][k] = Un[1][c] - lamk * (Fkp[c] - Fkm[c]);
    cell[c][k + 1] = Un[2][c] - lam * (Fright[c] - Fkp[c]);
  }
  for (int i = k - 1; i <= k + 1; ++i) {
    double U[3] = {rho[i], mom[i], ene[i]}, Wp[3];
    if (!eu_prim(G, U, Wp)) st |= EU_ST_NONPHYS;
  }
  return st;
}

/* S^n = max_i (|u_i| + a_i); 0 if a cell is not physical */
static double eu_smax(const eu_gas *G, int n, const double *rho, const double *mom,
                      const double *ene) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    double U[3] = {rho[i], mom[i], ene[i]}, W[3];
    if (!eu_prim(G, U, W)) return 0.0;
    double v = fabs(W[1]) + sqrt(G->g * W[2] / W[0]);
    if (v > s) s = v;
  }
  return s;
}

/* Advances every problem by up to max_steps time steps, stopping a problem
 * at t_end or at its first failure.
 *   off[b]        first cell of problem b in rho/mom/ene (N[b] + 1 cells)
 *   N, h, alpha   regular cell count (even), regular length, small-cell ratio
 *   th_nb, th_k   theta_{k-1} = theta_{k+1} and theta_k
 *   cfl, t_end    C_CFL and the end time
 *   t, steps, status  per problem, read and updated
 *   iters         per problem, total dual time iterations (added to)
 *   log_cnt       NULL or [n_problems][max_steps] iteration count per step
 *                 of this call (0 where the problem did not step)
 *   log_flags     NULL or the same shape, EU_FL_ bits */
int oracle_euler_run(int n_problems, const long long *off, const int *N, const double *h,
                     const double *alpha, const double *th_nb, const double *th_k,
                     const double *cfl, const double *t_end, double gamma, double tol_nb,
                     double tol_k, int lmax, double *rho, double *mom, double *ene, double *t,
                     int *steps, int *status, long long *iters, int max_steps, int *log_cnt,
                     int *log_flags, int n_threads) {
  eu_params P = {gamma, tol_nb, tol_k, lmax};
  eu_gas G = eu_make_gas(gamma);
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (int b = 0; b < n_problems; ++b) {
    int n = N[b] + 1;
    double *r = rho + off[b], *m = mom + off[b], *e = ene + off[b];
    double *F = (double *)malloc(sizeof(double) * 3 * (size_t)(n + 1));
    for (int s = 0; s < max_steps; ++s) {
      if (status[b] || !(t[b] < t_end[b])) break;
      double S = eu_smax(&G, n, r, m, e);
      if (!(S > 0.0)) {
        status[b] |= EU_ST_NONPHYS;
        break;
      }
      double dtref = (cfl[b] * h[b]) / S;
      double dt = dtref;
      double rem = t_end[b] - t[b];
      int clip = 0;
      if (dt >= rem) {
        dt = rem;
        clip = 1;
      }
      int cnt = 0, fl = 0;
      int st = eu_step(&G, &P, N[b], h[b], alpha[b], th_nb[b], th_k[b], dt, dtref, clip, r, m, e, F, &cnt,
                       &fl);
      if (log_cnt) log_cnt[(size_t)b * max_steps + s] = cnt;
      if (log_flags) log_flags[(size_t)b * max_steps + s] = fl;
      if (st) {
        status[b] |= st;
        break;
      }
      iters[b] += cnt;
      t[b] = clip ? t_end[b] : t[b] + dt;
      steps[b] += 1;
    }
    free(F);
  }
  return 0;
}
