// imexds_device.hpp -- device-side physics of the IMEX-DS step (gfx950).
//
// Phase laws and Gibbs energies (Sec. 5 eqs. eos:isoT_idgas, eos:isoT_lintait;
// Sec. 2.1 Maxwell construction), the HLL flux for same-phase faces, and the
// two-phase interface Riemann solve of Appendix A: Newton-Armijo on
// G(p_l*, p_r*) = ([[p]] + z^2 [[v]],  f_l + f_r + z [[v]] + (u_r - u_l)) with
// the analytic Jacobian (eq. jacobian:ex_sys), z from the kinetic relation
// z = tau p_V ([[g]] + z^2 [[v^2]] / 2) (eq. isoT:kin_rel1, kinetic energy
// relative to the boundary), and the boundary flux F_PB = (-z, -z u_V* + p_V*)
// (eq. pb_flux:pt).  All arithmetic is FP64 and the translation unit is
// compiled with -ffp-contract=off: each expression is evaluated in the
// order written, without fused multiply-adds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imexds {

constexpr int LIQ = 0;
constexpr int VAP = 1;

constexpr int ST_NEWTON = 1;
constexpr int ST_NONPHYS = 2;
constexpr int ST_MESH = 4;
constexpr int ST_OVERLAP = 8;

constexpr int FL_TINY_RIGHT = 1;
constexpr int FL_MERGED = 2;
constexpr int FL_REDO = 4;
constexpr int FL_LMAX = 8;
constexpr int FL_CROSS_L = 16;
constexpr int FL_CROSS_R = 32;
constexpr int FL_FAIL = 64;
constexpr int FL_INACTIVE = 128;

// Material: the five physical constants and three derived ones (square roots
// and the vapour saturation density), each computed once on the host with a
// correctly rounded operation.
struct Mat {
  double a2v, a2l, p0, rhol0, tau;
  double av, al;  // sqrt(a2v), sqrt(a2l)
  double rhov0;   // p0 / a2v
};

struct Par {
  double cfl, theta_nb, tol_nb, tol_tiny, tol_rel, alpha_floor, merge_safety, newton_rtol, t_end;
  int zone_half, tol_mode, lmax, bc_left, bc_right, newton_maxit;
};

__device__ __forceinline__ double d_a2(const Mat& M, int ph) { return ph == VAP ? M.a2v : M.a2l; }
__device__ __forceinline__ double d_a(const Mat& M, int ph) { return ph == VAP ? M.av : M.al; }

__device__ __forceinline__ double d_pres(const Mat& M, int ph, double r) {
  return ph == VAP ? M.a2v * r : M.p0 + M.a2l * (r - M.rhol0);
}

__device__ __forceinline__ double d_rho_of_p(const Mat& M, int ph, double p) {
  return ph == VAP ? p / M.a2v : M.rhol0 + (p - M.p0) / M.a2l;
}

// Natural logarithm of a positive finite double: x = 2^e m with m in
// [sqrt(1/2), sqrt(2)], ln m = 2 atanh(f), f = (m-1)/(m+1), by the atanh
// series through f^24/25 (Horner), plus e ln 2 with ln 2 split into a head
// with trailing zero bits and a tail (as in fdlibm).  Plain IEEE double
// operations in a fixed order: the result is the same on any IEEE machine,
// which keeps iteration counts that hinge on a logarithm reproducible.
__device__ __forceinline__ double d_log(double x) {
  if (!(x > 0.0)) return x == 0.0 ? -__builtin_inf() : __builtin_nan("");
  if (!__builtin_isfinite(x)) return x;
  unsigned long long b = (unsigned long long)__double_as_longlong(x);
  int ex = (int)((b >> 52) & 0x7ff);
  int e;
  if (ex == 0) {
    double y = x * 18014398509481984.0;
    b = (unsigned long long)__double_as_longlong(y);
    e = (int)((b >> 52) & 0x7ff) - 1023 - 54;
  } else {
    e = ex - 1023;
  }
  b = (b & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
  double m = __longlong_as_double((long long)b);
  if (m > 1.4142135623730951) {
    m = 0.5 * m;
    e += 1;
  }
  double f = (m - 1.0) / (m + 1.0);
  double s = f * f;
  double p = 1.0 / 25.0;
  p = p * s + 1.0 / 23.0;
  p = p * s + 1.0 / 21.0;
  p = p * s + 1.0 / 19.0;
  p = p * s + 1.0 / 17.0;
  p = p * s + 1.0 / 15.0;
  p = p * s + 1.0 / 13.0;
  p = p * s + 1.0 / 11.0;
  p = p * s + 1.0 / 9.0;
  p = p * s + 1.0 / 7.0;
  p = p * s + 1.0 / 5.0;
  p = p * s + 1.0 / 3.0;
  p = p * s + 1.0;
  double r = (2.0 * f) * p;
  double de = (double)e;
  return de * 0x1.62e42feep-1 + (de * 0x1.a39ef35793c76p-33 + r);
}

__device__ __forceinline__ double d_gibbs(const Mat& M, int ph, double r) {
  return ph == VAP ? M.a2v * d_log(r / M.rhov0) : M.a2l * d_log(r / M.rhol0);
}

__device__ __forceinline__ bool d_finite(double x) { return __builtin_isfinite(x); }

__device__ __forceinline__ bool d_state_ok(double r, double m) {
  return r > 0.0 && d_finite(r) && d_finite(m);
}

// HLL flux from primitive and conservative values of the two sides (Davis
// wave speeds min(u_l,u_r) - a, max(u_l,u_r) + a).
__device__ __forceinline__ void d_hll_prim(double a, double rl, double ml, double ul, double pl,
                                           double rr, double mr, double ur, double pr, double& F0,
                                           double& F1) {
  double sl = (ul < ur ? ul : ur) - a;
  double sr = (ul > ur ? ul : ur) + a;
  double fl0 = ml, fl1 = ml * ul + pl;
  double fr0 = mr, fr1 = mr * ur + pr;
  if (sl >= 0.0) {
    F0 = fl0;
    F1 = fl1;
  } else if (sr <= 0.0) {
    F0 = fr0;
    F1 = fr1;
  } else {
    double d = sr - sl, ss = sl * sr;
    F0 = ((sr * fl0 - sl * fr0) + ss * (rr - rl)) / d;
    F1 = ((sr * fl1 - sl * fr1) + ss * (mr - ml)) / d;
  }
}

__device__ __forceinline__ void d_hll(const Mat& M, int ph, double rl, double ml, double rr,
                                      double mr, double& F0, double& F1) {
  double ul = ml / rl, ur = mr / rr;
  d_hll_prim(d_a(M, ph), rl, ml, ul, d_pres(M, ph, rl), rr, mr, ur, d_pres(M, ph, rr), F0, F1);
}

// Flux through a domain boundary: HLL against the ghost (rho, -m) (wall) or
// (rho, m) (transmissive); the ghost sits outside the boundary.
__device__ __forceinline__ void d_bflux(const Mat& M, int ph, bool right_end, int bc, double r,
                                        double m, double& F0, double& F1) {
  double mg = (bc == 0) ? -m : m;
  if (right_end)
    d_hll(M, ph, r, m, r, mg, F0, F1);
  else
    d_hll(M, ph, r, mg, r, m, F0, F1);
}

// ---------------------------------------------------------------------------
// two-phase interface Riemann problem
// ---------------------------------------------------------------------------
struct RP {
  int phl, phr;
  double rl, ul, pl, rr, ur, pr;
};

struct GEval {
  double G1, G2, J11, J12, J21, J22;
  double rsl, rsr, fl, fr, z;
};

struct IfaceOut {
  double pl, pr, rl, rr, ul, ur, z, w, F0, F1;
  int iters;
};

// Outer-wave function f_K(p*) and its derivative; shock branch in the form
// a (rho* - rho_K) / sqrt(rho_K rho*), exact for pressure laws affine in rho.
__device__ __forceinline__ bool d_wave(const Mat& M, int ph, double rhoK, double pK, double ps,
                                       double& f, double& df, double& rs) {
  double r = d_rho_of_p(M, ph, ps);
  if (!(r > 0.0) || !d_finite(r)) return false;
  double a = d_a(M, ph);
  rs = r;
  if (ps > pK) {
    double g = sqrt(rhoK * r);
    f = a * (r - rhoK) / g;
    df = (r + rhoK) / ((2.0 * a * r) * g);
  } else {
    f = a * d_log(r / rhoK);
    df = 1.0 / (r * a);
  }
  return true;
}

// z(p_l*, p_r*) from A z^2 - z + C = 0 (root continuous at A = 0) and dz/dp.
__device__ __forceinline__ bool d_kinetic(const Mat& M, int phl, int phr, double rsl, double rsr,
                                          double psl, double psr, double& z, double& dzl,
                                          double& dzr) {
  double pV = (phl == VAP) ? psl : psr;
  double q = M.tau * pV;
  double vl = 1.0 / rsl, vr = 1.0 / rsr;
  double jg = d_gibbs(M, phr, rsr) - d_gibbs(M, phl, rsl);
  double jv2 = vr * vr - vl * vl;
  double A = 0.5 * q * jv2;
  double C = q * jg;
  double D = 1.0 - 4.0 * A * C;
  if (!(D >= 0.0) || !d_finite(D)) return false;
  double sD = sqrt(D);
  double zz = 2.0 * C / (1.0 + sD);
  double a2l = d_a2(M, phl), a2r = d_a2(M, phr);
  double dAl = 0.5 * q * (2.0 * vl * vl * vl / a2l);
  double dAr = 0.5 * q * (-2.0 * vr * vr * vr / a2r);
  double dCl = q * (-vl);
  double dCr = q * vr;
  if (phl == VAP) {
    dAl += 0.5 * M.tau * jv2;
    dCl += M.tau * jg;
  } else {
    dAr += 0.5 * M.tau * jv2;
    dCr += M.tau * jg;
  }
  dzl = (dAl * zz * zz + dCl) / sD;
  dzr = (dAr * zz * zz + dCr) / sD;
  z = zz;
  return true;
}

__device__ __forceinline__ bool d_eval_G(const Mat& M, const RP& R, double psl, double psr,
                                         GEval& E) {
  double dfl, dfr, dzl, dzr;
  if (!d_wave(M, R.phl, R.rl, R.pl, psl, E.fl, dfl, E.rsl)) return false;
  if (!d_wave(M, R.phr, R.rr, R.pr, psr, E.fr, dfr, E.rsr)) return false;
  if (!d_kinetic(M, R.phl, R.phr, E.rsl, E.rsr, psl, psr, E.z, dzl, dzr)) return false;
  double z = E.z;
  double vl = 1.0 / E.rsl, vr = 1.0 / E.rsr;
  double jv = vr - vl;
  double el = vl * vl / d_a2(M, R.phl);
  double er = vr * vr / d_a2(M, R.phr);
  E.G1 = (psr - psl) + z * z * jv;
  E.G2 = (E.fl + E.fr) + z * jv + (R.ur - R.ul);
  E.J11 = -1.0 + 2.0 * z * dzl * jv + z * z * el;
  E.J12 = 1.0 + 2.0 * z * dzr * jv - z * z * er;
  E.J21 = dfl + dzl * jv + z * el;
  E.J22 = dfr + dzr * jv - z * er;
  return d_finite(E.G1) && d_finite(E.G2);
}

__device__ __forceinline__ double d_merit(const GEval& E, double zref) {
  double a = E.G1 / zref, b = E.G2;
  return sqrt(a * a + b * b);
}

// Newton-Armijo from one start: full step accepted once the relative step is
// below rtol; otherwise halve the step (at most 20 times) until the merit
// decreases by the factor (1 - 1e-4 lambda); if no halving works the point
// is accepted only when the step is already below 1e-8 (round-off floor).
__device__ bool d_newton(const Mat& M, const RP& R, double zref, double xl, double xr, int maxit,
                         double rtol, double& ol, double& orr, GEval& Eo, int& iters) {
  GEval E, Et;
  if (!d_eval_G(M, R, xl, xr, E)) return false;
  for (int it = 0; it < maxit; ++it) {
    double det = E.J11 * E.J22 - E.J12 * E.J21;
    if (!(det != 0.0) || !d_finite(det)) return false;
    double dl = (-E.G1 * E.J22 + E.G2 * E.J12) / det;
    double dr = (-E.G2 * E.J11 + E.G1 * E.J21) / det;
    double sc = fabs(xl) > fabs(xr) ? fabs(xl) : fabs(xr);
    if (M.p0 > sc) sc = M.p0;
    double st = fabs(dl) > fabs(dr) ? fabs(dl) : fabs(dr);
    if (!d_finite(st)) return false;
    if (st <= rtol * sc) {
      double tl = xl + dl, tr = xr + dr;
      if (d_eval_G(M, R, tl, tr, Et)) {
        xl = tl;
        xr = tr;
        E = Et;
      }
      ol = xl;
      orr = xr;
      Eo = E;
      iters += it + 1;
      return true;
    }
    double m0 = d_merit(E, zref);
    double lam = 1.0;
    bool acc = false;
    for (int k = 0; k <= 20; ++k) {
      double tl = xl + lam * dl, tr = xr + lam * dr;
      if (d_eval_G(M, R, tl, tr, Et) && d_merit(Et, zref) <= (1.0 - 1e-4 * lam) * m0) {
        xl = tl;
        xr = tr;
        E = Et;
        acc = true;
        break;
      }
      lam *= 0.5;
    }
    if (!acc) {
      if (st <= 1e-8 * sc) {
        ol = xl;
        orr = xr;
        Eo = E;
        iters += it + 1;
        return true;
      }
      return false;
    }
  }
  iters += maxit;
  return false;
}

// HLLC-type start (eq. HLLC:2p_nopt, mirrored when the liquid is on the left):
// contact speed and liquid star density from the two states, liquid law for
// the pressure; the vapour unknown is kept at or above 1e-3 of the vapour
// pressure.
__device__ __forceinline__ void d_guess(const Mat& M, const RP& R, double& gl, double& gr) {
  double al = d_a(M, R.phl), ar = d_a(M, R.phr);
  double sl = R.ul - al, sr = R.ur + ar;
  double num = (R.pr - R.pl) + R.rl * R.ul * (sl - R.ul) - R.rr * R.ur * (sr - R.ur);
  double den = R.rl * (sl - R.ul) - R.rr * (sr - R.ur);
  double ws = num / den;
  double rLs = (R.phl == LIQ) ? R.rl * (sl - R.ul) / (sl - ws) : R.rr * (sr - R.ur) / (sr - ws);
  double pg = d_pres(M, LIQ, rLs);
  double pV = (R.phl == VAP) ? R.pl : R.pr;
  double pvg = pg > 1e-3 * pV ? pg : 1e-3 * pV;
  if (R.phl == VAP) {
    gl = pvg;
    gr = pg;
  } else {
    gl = pg;
    gr = pvg;
  }
}

// Interface solve from conservative states; starts tried in order: the warm
// start (if have_guess), the HLLC-type guess, both unknowns at the vapour
// pressure.  Returns false if none converges.
__device__ bool d_iface_solve(const Mat& M, int maxit, double rtol, int phl, double rl, double ml,
                              int phr, double rr, double mr, bool have_guess, double gl,
                              double gr, IfaceOut& out) {
  if (!(rl > 0.0) || !(rr > 0.0) || phl == phr) return false;
  RP R;
  R.phl = phl;
  R.phr = phr;
  R.rl = rl;
  R.rr = rr;
  R.ul = ml / rl;
  R.ur = mr / rr;
  R.pl = d_pres(M, phl, rl);
  R.pr = d_pres(M, phr, rr);
  double zl = rl * d_a(M, phl), zr = rr * d_a(M, phr);
  double zref = zl > zr ? zl : zr;
  double xl = 0.0, xr = 0.0;
  GEval E;
  int iters = 0;
  bool conv = false;
  for (int attempt = 0; attempt < 3 && !conv; ++attempt) {
    double sl, sr;
    if (attempt == 0) {
      if (!have_guess) continue;
      sl = gl;
      sr = gr;
    } else if (attempt == 1) {
      d_guess(M, R, sl, sr);
    } else {
      double pV = (phl == VAP) ? R.pl : R.pr;
      sl = pV;
      sr = pV;
    }
    conv = d_newton(M, R, zref, sl, sr, maxit, rtol, xl, xr, E, iters);
  }
  if (!conv) return false;
  out.iters = iters;
  out.pl = xl;
  out.pr = xr;
  out.rl = E.rsl;
  out.rr = E.rsr;
  out.ul = R.ul - E.fl;
  out.ur = R.ur + E.fr;
  out.z = E.z;
  double uV, rV, pV;
  if (phl == VAP) {
    uV = out.ul;
    rV = out.rl;
    pV = xl;
  } else {
    uV = out.ur;
    rV = out.rr;
    pV = xr;
  }
  out.w = uV + E.z / rV;
  out.F0 = -E.z;
  out.F1 = -E.z * uV + pV;
  return true;
}

}  // namespace imexds
