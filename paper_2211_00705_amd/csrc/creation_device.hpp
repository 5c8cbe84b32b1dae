// creation_device.hpp -- device side of phase creation for one Riemann
// problem of two states of one phase (appendix "Phase Creation", steps (i),
// (ii), (iii), (v)): the single-phase star pressure (step (i)) and the
// five-state problem with a layer of the other phase (step (ii)) and its
// outputs.  Shared by the batched creation kernels and the creation-tube
// path; every expression is evaluated in the order written.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/imexds_creation.h"
#include "imexds_device.hpp"

namespace imexds {
namespace {

// per-phase constants of the creation solve
__device__ __forceinline__ double c_ia2(const Mat& M, int ph) { return ph == VAP ? M.ia2v : M.ia2l; }

// Step (i): star pressure of the single-phase problem; 0 on success, 1 if no
// root with rho* > 0 was found.
__device__ int c_single_rp(const Mat& M, const Side& L, const Side& R, double& ps) {
  const double du = R.u - L.u;
  double p = 0.5 * (L.p + R.p);
  for (int it = 0; it < 100; ++it) {
    double rl, vl, gl, fl, dfl, rr, vr, gr, fr, dfr;
    // taken branches: selecting here makes the compiler address the
    // material constants through a stack copy
    const bool okl = d_wave<false>(M, L, p, rl, vl, gl, fl, dfl);
    const bool okr = d_wave<false>(M, R, p, rr, vr, gr, fr, dfr);
    if (!okl || !okr) return 1;
    double dp = -(fl + fr + du) / (dfl + dfr);
    if (!d_finite(dp)) return 1;
    double pn = p + dp;
    int k = 0;
    while (!(d_rho_of_p(M, L.ph, pn) > 0.0) && k < 60) {
      dp = 0.5 * dp;
      pn = p + dp;
      ++k;
    }
    if (k == 60) return 1;
    const double sc = fabs(p) > M.p0 ? fabs(p) : M.p0;
    p = pn;
    // converged when the step is below 1e-12 of the pressure scale or below
    // 1e-13 of the density it implies (the liquid resolves p* only to about
    // 1e-7 Pa through its density)
    if (fabs(dp) <= 1e-12 * sc || fabs(dp) <= 1e-13 * (d_a2(M, L.ph) * d_rho_of_p(M, L.ph, p))) {
      ps = p;
      return 0;
    }
  }
  return 1;
}

// one state of the five-state problem at its star pressure
struct CState {
  double rs, v, g, f, df;
};

// mass flux through a boundary between l (left, phase phl) and r from the
// kinetic relation, and its derivatives in the left and right pressure
__device__ __forceinline__ bool c_kinetic(const Mat& M, int phl, const CState& l, const CState& r,
                                          double pl, double pr, double ia2l, double ia2r,
                                          double& z, double& dzl, double& dzr) {
  const double vl = l.v, vr = r.v;
  const double pV = phl == VAP ? pl : pr;
  const double q = M.tau * pV;
  const double jg = r.g - l.g;
  const double jv2 = vr * vr - vl * vl;
  const double A = 0.5 * q * jv2;
  const double C = q * jg;
  const double D = 1.0 - 4.0 * A * C;
  if (!(D >= 0.0) || !d_finite(D)) return false;
  const double sD = sqrt(D);
  const double isD = 1.0 / sD;
  const double zz = 2.0 * C / (1.0 + sD);
  double dAl = q * ((vl * vl * vl) * ia2l);
  double dAr = -(q * ((vr * vr * vr) * ia2r));
  double dCl = -(q * vl);
  double dCr = q * vr;
  if (phl == VAP) {
    dAl += (0.5 * M.tau) * jv2;
    dCl += M.tau * jg;
  } else {
    dAr += (0.5 * M.tau) * jv2;
    dCr += M.tau * jg;
  }
  z = zz;
  dzl = (dAl * zz * zz + dCl) * isD;
  dzr = (dAr * zz * zz + dCr) * isD;
  return true;
}

struct CEval {
  double E1, E2, E3, J[3][3], m2, zl, zr;
  CState a, b, c;
};

__device__ bool c_eval(const Mat& M, const Side& L, const Side& R, const Side& S, double izref,
                       double pa, double pb, double pc, CEval& E) {
  if (!d_wave(M, L, pa, E.a.rs, E.a.v, E.a.g, E.a.f, E.a.df) ||
      !d_wave(M, S, pb, E.b.rs, E.b.v, E.b.g, E.b.f, E.b.df) ||
      !d_wave(M, R, pc, E.c.rs, E.c.v, E.c.g, E.c.f, E.c.df))
    return false;
  const double ia2o = c_ia2(M, L.ph), ia2n = c_ia2(M, S.ph);
  double dla, dlb, drb, drc;
  if (!c_kinetic(M, L.ph, E.a, E.b, pa, pb, ia2o, ia2n, E.zl, dla, dlb)) return false;
  if (!c_kinetic(M, S.ph, E.b, E.c, pb, pc, ia2n, ia2o, E.zr, drb, drc)) return false;
  const double zl = E.zl, zr = E.zr;
  const double jl = E.b.v - E.a.v, jr = E.c.v - E.b.v;
  const double ea = (E.a.v * E.a.v) * ia2o;
  const double eb = (E.b.v * E.b.v) * ia2n;
  const double ec = (E.c.v * E.c.v) * ia2o;
  E.E1 = (pb - pa) + zl * zl * jl;
  E.E2 = (pc - pb) + zr * zr * jr;
  E.E3 = (E.a.f + E.c.f) + zl * jl + zr * jr + (R.u - L.u);
  E.J[0][0] = -1.0 + 2.0 * zl * dla * jl + zl * zl * ea;
  E.J[0][1] = 1.0 + 2.0 * zl * dlb * jl - zl * zl * eb;
  E.J[0][2] = 0.0;
  E.J[1][0] = 0.0;
  E.J[1][1] = -1.0 + 2.0 * zr * drb * jr + zr * zr * eb;
  E.J[1][2] = 1.0 + 2.0 * zr * drc * jr - zr * zr * ec;
  E.J[2][0] = E.a.df + dla * jl + zl * ea;
  E.J[2][1] = dlb * jl - zl * eb + drb * jr + zr * eb;
  E.J[2][2] = E.c.df + drc * jr - zr * ec;
  if (!d_finite(E.E1) || !d_finite(E.E2) || !d_finite(E.E3)) return false;
  const double s1 = E.E1 * izref, s2 = E.E2 * izref;
  E.m2 = s1 * s1 + s2 * s2 + E.E3 * E.E3;
  return true;
}

// determinant of the 3x3 matrix whose column k is replaced by r (k = -1: none)
__device__ __forceinline__ double c_det(const double J[3][3], int k, const double* r) {
  double A[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A[i][j] = j == k ? r[i] : J[i][j];
  return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
         A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
         A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

// Cramer's rule; the determinant is expanded by cofactors of the first row
__device__ __forceinline__ bool c_solve3(const double J[3][3], const double* r, double* x) {
  const double c0 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c1 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c2 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double det = J[0][0] * c0 + J[0][1] * c1 + J[0][2] * c2;
  if (!(det != 0.0) || !d_finite(det)) return false;
  const double id = 1.0 / det;
#pragma unroll
  for (int k = 0; k < 3; ++k) x[k] = c_det(J, k, r) * id;
  return true;
}

// Step (ii) and outputs for a problem that step (i) sent to creation: fills
// the record o (already zero but P1) and returns 1, or -1 on failure.
__device__ int c_solve(const Mat& M, int ph, double rl, double ml, double rr, double mr,
                       int maxit, double rtol, double* o) {
  Side L, R, S;
  d_side(M, ph, rl, ml, L);
  d_side(M, ph, rr, mr, R);
  const int nph = 1 - ph;
  d_side(M, nph, nph == VAP ? M.rhov0 : M.rhol0, 0.0, S);
  const double aph = ph == VAP ? M.av : M.al;
  const double zL = rl * aph, zR = rr * aph;
  const double izref = 1.0 / (zL > zR ? zL : zR);
  double x0 = M.p0, x1 = M.p0, x2 = M.p0;
  CEval E, Et;
  if (!c_eval(M, L, R, S, izref, x0, x1, x2, E)) return -1;
  int it;
  bool conv = false;
  for (it = 0; it < maxit && !conv; ++it) {
    const double rhs[3] = {-E.E1, -E.E2, -E.E3};
    double d[3];
    if (!c_solve3(E.J, rhs, d)) return -1;
    double sc = 0.0, st = 0.0;
    const double xs[3] = {x0, x1, x2};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (fabs(xs[i]) > sc) sc = fabs(xs[i]);
      if (fabs(d[i]) > st) st = fabs(d[i]);
    }
    if (M.p0 > sc) sc = M.p0;
    if (!d_finite(st)) return -1;
    if (st <= rtol * sc) {
      if (c_eval(M, L, R, S, izref, x0 + d[0], x1 + d[1], x2 + d[2], Et)) {
        x0 = x0 + d[0];
        x1 = x1 + d[1];
        x2 = x2 + d[2];
        E = Et;
      }
      conv = true;
      break;
    }
    double lam = 1.0;
    bool acc = false;
    int k;
    for (k = 0; k <= 20; ++k) {
      const double c = 1.0 - 1e-4 * lam;
      if (c_eval(M, L, R, S, izref, x0 + lam * d[0], x1 + lam * d[1], x2 + lam * d[2], Et) &&
          Et.m2 <= (c * c) * E.m2) {
        x0 = x0 + lam * d[0];
        x1 = x1 + lam * d[1];
        x2 = x2 + lam * d[2];
        E = Et;
        acc = true;
        break;
      }
      lam *= 0.5;
    }
    if (!acc) {
      if (st <= 1e-8 * sc) {
        conv = true;
        break;
      }
      return -1;
    }
    if (k == 0 && st <= 1e-10 * sc) conv = true;
  }
  if (!conv) return -1;
  o[IMEXDS_CR_KIND] = ph == LIQ ? 1.0 : 2.0;
  o[IMEXDS_CR_PA] = x0;
  o[IMEXDS_CR_PB] = x1;
  o[IMEXDS_CR_PC] = x2;
  o[IMEXDS_CR_RA] = E.a.rs;
  o[IMEXDS_CR_RB] = E.b.rs;
  o[IMEXDS_CR_RC] = E.c.rs;
  const double ua = L.u - E.a.f;
  const double uc = R.u + E.c.f;
  const double ub = ua - E.zl * (E.b.v - E.a.v);
  o[IMEXDS_CR_UA] = ua;
  o[IMEXDS_CR_UB] = ub;
  o[IMEXDS_CR_UC] = uc;
  o[IMEXDS_CR_ZL] = E.zl;
  o[IMEXDS_CR_ZR] = E.zr;
  o[IMEXDS_CR_WL] = ub + E.zl * E.b.v;
  o[IMEXDS_CR_WR] = ub + E.zr * E.b.v;
  o[IMEXDS_CR_FL0] = -E.zl;
  o[IMEXDS_CR_FL1] = -E.zl * ub + x1;
  o[IMEXDS_CR_FR0] = -E.zr;
  o[IMEXDS_CR_FR1] = -E.zr * ub + x1;
  o[IMEXDS_CR_ITERS] = (double)(it + 1);
  return 1;
}

// step (i) and its decision alone: 1 if the problem creates a layer of the
// other phase (p* < p_min for a liquid, p* > p_tilde for a vapour, or no
// root), 0 if not; p1 gets the star pressure (0 without a root)
template <int PH>
__device__ __forceinline__ int c_creates_t(const Mat& M, double rl, double ml, double rr, double mr,
                                           double p_min, double p_tilde, double& p1) {
  Side L, R;
  d_side(M, PH, rl, ml, L);
  d_side(M, PH, rr, mr, R);
  p1 = 0.0;
  const int none = c_single_rp(M, L, R, p1);
  if (none) p1 = 0.0;
  return none ? 1 : (PH == LIQ ? p1 < p_min : p1 > p_tilde);
}

// (the phase as a constant: every per-phase constant is then read directly
// instead of selected)
__device__ __forceinline__ int c_creates(const Mat& M, int ph, double rl, double ml, double rr,
                                         double mr, double p_min, double p_tilde, double& p1) {
  return ph == LIQ ? c_creates_t<LIQ>(M, rl, ml, rr, mr, p_min, p_tilde, p1)
                   : c_creates_t<VAP>(M, rl, ml, rr, mr, p_min, p_tilde, p1);
}

}  // namespace
}  // namespace imexds
