// imexds_device.hpp -- device-side physics of the IMEX-DS step (gfx950).
//
// Phase laws and Gibbs energies (Sec. 4 eqs. eos:isoT_idgas, eos:isoT_lintait;
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
constexpr int ST_VANISH = 16;

constexpr int FL_TINY_RIGHT = 1;
constexpr int FL_MERGED = 2;
constexpr int FL_REDO = 4;
constexpr int FL_LMAX = 8;
constexpr int FL_CROSS_L = 16;
constexpr int FL_CROSS_R = 32;
constexpr int FL_FAIL = 64;
constexpr int FL_INACTIVE = 128;
constexpr int FL_PAIR = 256;

// Material: the five physical constants and derived ones, each computed once
// on the host with one correctly rounded operation (sqrt or division) from
// the five, in the order listed.
struct Mat {
  double a2v, a2l, p0, rhol0, tau;
  double av, al;    // sqrt(a2v), sqrt(a2l)
  double rhov0;     // p0 / a2v
  double ia2v, ia2l;  // 1 / a2v, 1 / a2l
  double iav, ial;    // 1 / av, 1 / al
  double irv0, irl0;  // 1 / rhov0, 1 / rhol0
};

// The material constants in vector registers.  Kernels select them per lane
// by phase (vapour or liquid); from a struct in the kernel arguments the
// compiler turns such a select into a load from a selected address, which
// needs a copy of the struct in scratch memory.  OR-ing each constant's bits
// with a zero it cannot see through (a vector register set by one v_mov)
// keeps every value as it is but places it in a vector register.
__device__ __forceinline__ Mat d_mat_vregs(const Mat& src) {
  int vz;
  asm volatile("v_mov_b32 %0, 0" : "=v"(vz));
  Mat M = src;
#define D_MAT_VREG(x) x = __longlong_as_double(__double_as_longlong(x) | (long long)vz)
  D_MAT_VREG(M.a2v); D_MAT_VREG(M.a2l); D_MAT_VREG(M.p0); D_MAT_VREG(M.rhol0);
  D_MAT_VREG(M.tau); D_MAT_VREG(M.av); D_MAT_VREG(M.al); D_MAT_VREG(M.rhov0);
  D_MAT_VREG(M.ia2v); D_MAT_VREG(M.ia2l); D_MAT_VREG(M.iav); D_MAT_VREG(M.ial);
  D_MAT_VREG(M.irv0); D_MAT_VREG(M.irl0);
#undef D_MAT_VREG
  return M;
}

struct Par {
  double cfl, theta_nb, tol_nb, tol_tiny, tol_rel, alpha_floor, merge_safety, newton_rtol, t_end;
  int zone_half, tol_mode, lmax, bc_left, bc_right, newton_maxit;
  int zone_solver, zn_maxit;  // zone solver: 0 Algorithm 2, 1 Newton (at most zn_maxit steps)
  double zn_rtol;             // Newton: relative step tolerance
};

__device__ __forceinline__ double d_a2(const Mat& M, int ph) { return ph == VAP ? M.a2v : M.a2l; }
__device__ __forceinline__ double d_a(const Mat& M, int ph) { return ph == VAP ? M.av : M.al; }

__device__ __forceinline__ double d_pres(const Mat& M, int ph, double r) {
  return ph == VAP ? M.a2v * r : M.p0 + M.a2l * (r - M.rhol0);
}

// Inverse pressure law, used inside the interface solve (reciprocal form).
__device__ __forceinline__ double d_rho_of_p(const Mat& M, int ph, double p) {
  return ph == VAP ? p * M.ia2v : M.rhol0 + (p - M.p0) * M.ia2l;
}

// Natural logarithm of a positive finite double: x = 2^e m with m in
// [sqrt(1/2), sqrt(2)], ln m = 2 atanh(f), f = (m-1)/(m+1), by the atanh
// series through f^24/25 (Estrin's scheme), plus e ln 2 with ln 2 split into a head
// with trailing zero bits and a tail (as in fdlibm).  Plain IEEE double
// operations in a fixed order: the result is the same on any IEEE machine,
// which keeps iteration counts that hinge on a logarithm reproducible.  The
// subnormal scaling and the special arguments (0, negative, infinite, NaN)
// are selected rather than branched to: a lone wave pays an issue slot for
// every instruction, and the branches' mask bookkeeping costs more than the
// few unused operations.
template <bool SELECT = true>
__device__ __forceinline__ double d_log(double x) {
  if (!SELECT) {
    if (!(x > 0.0)) return x == 0.0 ? -__builtin_inf() : __builtin_nan("");
    if (!__builtin_isfinite(x)) return x;
  }
  const bool pos = x > 0.0;
  const bool fin = __builtin_isfinite(x);
  unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const int ex = (int)((b >> 52) & 0x7ff);
  const bool sub = ex == 0;
  const double y = x * 18014398509481984.0;
  const unsigned long long by = (unsigned long long)__double_as_longlong(y);
  b = sub ? by : b;
  int e = (int)((b >> 52) & 0x7ff) - 1023 - (sub ? 54 : 0);
  b = (b & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
  double m = __longlong_as_double((long long)b);
  const bool hi = m > 1.4142135623730951;
  m = hi ? 0.5 * m : m;
  e += hi ? 1 : 0;
  double f = (m - 1.0) / (m + 1.0);
  double s = f * f;
  double s2 = s * s, s4 = s2 * s2, s8 = s4 * s4;
  double q0 = 1.0 + (1.0 / 3.0) * s, q1 = (1.0 / 5.0) + (1.0 / 7.0) * s;
  double q2 = (1.0 / 9.0) + (1.0 / 11.0) * s, q3 = (1.0 / 13.0) + (1.0 / 15.0) * s;
  double q4 = (1.0 / 17.0) + (1.0 / 19.0) * s, q5 = (1.0 / 21.0) + (1.0 / 23.0) * s;
  double r0 = q0 + q1 * s2, r1 = q2 + q3 * s2, r2 = q4 + q5 * s2;
  double t0 = r0 + r1 * s4, t1 = r2 + (1.0 / 25.0) * s4;
  double p = t0 + t1 * s8;
  double r = (2.0 * f) * p;
  double de = (double)e;
  const double res = de * 0x1.62e42feep-1 + (de * 0x1.a39ef35793c76p-33 + r);
  const double spec = x == 0.0 ? -__builtin_inf() : (pos ? x : __builtin_nan(""));
  return (pos && fin) ? res : spec;
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

// Implicit zone of an interface: the smaller cut piece (ties: left) +- Z
// slots, clipped to the problem.  Slots are local to the problem.
__device__ __forceinline__ void d_zone_range(int sL, double hl, double h, int Z, int ns, int& zlo,
                                             int& zhi, bool& tiny_right) {
  double hR = h - hl;
  tiny_right = !(hl <= hR);
  int c = tiny_right ? sL + 1 : sL;
  zlo = c - Z < 0 ? 0 : c - Z;
  zhi = c + Z > ns - 1 ? ns - 1 : c + Z;
}

// ---------------------------------------------------------------------------
// two-phase interface Riemann problem
// ---------------------------------------------------------------------------
// Per-side data of one solve: the side's state and L_K = ln(rho_K / rho_K,sat),
// so that one logarithm per side and evaluation, L* = ln(rho* / rho_K,sat),
// yields both the Gibbs energy a^2 L* and the rarefaction wave a (L* - L_K).
struct Side {
  int ph;
  double r, u, p, LK;
};

struct RP {
  int phl;
  Side L, Rt;
  double izref;  // 1 / max(rho_l a_l, rho_r a_r)
};

// What one evaluation of G leaves behind: G, its Jacobian, the squared merit
// (G1 / zref)^2 + G2^2, z and dz/dp*, and per side rho*, v*, f_K and df_K/dp*.
struct GEval {
  double G1, G2, J11, J12, J21, J22, m2, z, dzl, dzr;
  double rsl, vl, fl, dfl, rsr, vr, fr, dfr;
};

struct IfaceOut {
  double pl, pr, rl, rr, ul, ur, z, w, F0, F1;
  int nev;  // evaluations of G (Newton steps and Armijo trials, all starts)
};

// u: the side's velocity m / r when the caller already has it (has_u)
__device__ __forceinline__ void d_side(const Mat& M, int ph, double r, double m, Side& S,
                                       bool has_u = false, double u = 0.0) {
  S.ph = ph;
  S.r = r;
  S.u = has_u ? u : m / r;
  S.p = d_pres(M, ph, r);
  S.LK = d_log(r * (ph == VAP ? M.irv0 : M.irl0));
}

// Outer wave of one side at star pressure ps: rho*, v*, Gibbs energy, f_K and
// df_K/dp*.  Shock branch sqrt(-[[p]][[v]]) written a (rho* - rho_K) /
// sqrt(rho_K rho*), exact for pressure laws affine in rho; rarefaction branch:
// the integral of v/a, a ln(rho*/rho_K).  SELECT: both branches are computed
// and one is selected (the two lanes of a pair solve, and the groups of a
// wave, take different branches anyway); otherwise the branch is taken.  False
// if rho* is not positive and finite, in which case the outputs are
// meaningless.
template <bool SELECT = true>
__device__ __forceinline__ bool d_wave(const Mat& M, const Side& S, double ps, double& rs,
                                       double& v, double& g, double& f, double& df) {
  const bool vap = S.ph == VAP;
  double r = d_rho_of_p(M, S.ph, ps);
  const bool ok = (r > 0.0) && d_finite(r);
  if (!SELECT && !ok) return false;
  v = 1.0 / r;
  double L = d_log<SELECT>(r * (vap ? M.irv0 : M.irl0));
  rs = r;
  g = (vap ? M.a2v : M.a2l) * L;
  const double a = vap ? M.av : M.al;
  const double ia = vap ? M.iav : M.ial;
  if (SELECT) {
    const bool shock = ps > S.p;
    const double ig = 1.0 / sqrt(S.r * r);
    const double fs = (a * (r - S.r)) * ig;
    const double dfs = ((r + S.r) * ig) * (v * (0.5 * ia));
    const double fr = a * (L - S.LK);
    const double dfr = v * ia;
    f = shock ? fs : fr;
    df = shock ? dfs : dfr;
  } else if (ps > S.p) {
    double ig = 1.0 / sqrt(S.r * r);
    f = (a * (r - S.r)) * ig;
    df = ((r + S.r) * ig) * (v * (0.5 * ia));
  } else {
    f = a * (L - S.LK);
    df = v * ia;
  }
  return ok;
}

// Value of the next / previous lane in the 16-lane row (a DPP row shift, a
// VALU move; a lane permute goes through the LDS crossbar, about 70 cycles).
// A lane whose source lies outside its row keeps its own value; the source
// lane must be active.
__device__ __forceinline__ double d_lane_next(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, 0x101, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), 0x101, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double d_lane_prev(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, 0x111, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), 0x111, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Value of lane + 1 / lane - 1 across the whole wave (DPP wave shift); the
// last / first lane keeps its own value, as __shfl_down / __shfl_up by one
// do.  Every lane must be active.
__device__ __forceinline__ int d_wave_next_i(int x) {
  return __builtin_amdgcn_update_dpp(x, x, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ int d_wave_prev_i(int x) {
  return __builtin_amdgcn_update_dpp(x, x, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ double d_wave_next(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = d_wave_next_i((int)b), hi = d_wave_next_i((int)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double d_wave_prev(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = d_wave_prev_i((int)b), hi = d_wave_prev_i((int)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Exchange with the pair's other lane.  The two lanes of a pair solve are an
// even lane and the odd one after it (lane and lane ^ 1), both active, so the
// exchange is one DPP quad permutation [1,0,3,2] per 32 bits: a VALU move
// that waits no longer than any other, where a lane permute goes through the
// LDS crossbar (about 70 cycles).
__device__ __forceinline__ int d_swap_i(int x) {
  return __builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false);
}
__device__ __forceinline__ double d_swap(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = d_swap_i((int)b), hi = d_swap_i((int)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// G(p_l*, p_r*) and its Jacobian.  z solves A z^2 - z + C = 0 with
// A = tau p_V [[v^2]] / 2, C = tau p_V [[g]] (root continuous at A = 0);
// dz/dp from differentiating that relation, using 2 A z - 1 = -sqrt(D).
// PAIR: two lanes evaluate together, the lane with side 0 the left outer
// wave and the one with side 1 the right one (same operations as one lane
// doing both), then swap them; everything after is computed on both lanes
// from identical values.  Straight-line code: the tests that make an
// evaluation invalid are combined into the result, and the outputs of an
// invalid evaluation are not used.
template <bool PAIR>
__device__ __forceinline__ bool d_eval_G_t(const Mat& M, const RP& R, double psl, double psr,
                                           int side, GEval& E) {
  double gl, gr, dfl, dfr;
  bool okw;
  if (PAIR) {
    double rs = 0.0, v = 0.0, g = 0.0, f = 0.0, df = 0.0;
    Side me;
    me.ph = side == 0 ? R.L.ph : R.Rt.ph;
    me.r = side == 0 ? R.L.r : R.Rt.r;
    me.u = side == 0 ? R.L.u : R.Rt.u;
    me.p = side == 0 ? R.L.p : R.Rt.p;
    me.LK = side == 0 ? R.L.LK : R.Rt.LK;
    const bool ok = d_wave(M, me, side == 0 ? psl : psr, rs, v, g, f, df);
    const double o_rs = d_swap(rs), o_v = d_swap(v), o_g = d_swap(g);
    const double o_f = d_swap(f), o_df = d_swap(df);
    const bool o_ok = d_swap_i(ok ? 1 : 0) != 0;
    okw = ok && o_ok;
    const bool s0 = side == 0;
    E.rsl = s0 ? rs : o_rs; E.vl = s0 ? v : o_v; gl = s0 ? g : o_g; E.fl = s0 ? f : o_f;
    dfl = s0 ? df : o_df;
    E.rsr = s0 ? o_rs : rs; E.vr = s0 ? o_v : v; gr = s0 ? o_g : g; E.fr = s0 ? o_f : f;
    dfr = s0 ? o_df : df;
  } else {
    const bool okl = d_wave(M, R.L, psl, E.rsl, E.vl, gl, E.fl, dfl);
    const bool okr = d_wave(M, R.Rt, psr, E.rsr, E.vr, gr, E.fr, dfr);
    okw = okl && okr;
  }
  const double vl = E.vl, vr = E.vr;
  const bool lvap = R.phl == VAP;
  const double ia2l = lvap ? M.ia2v : M.ia2l, ia2r = lvap ? M.ia2l : M.ia2v;
  const double pV = lvap ? psl : psr;
  const double q = M.tau * pV;
  const double jg = gr - gl;
  const double jv2 = vr * vr - vl * vl;
  const double A = 0.5 * q * jv2;
  const double C = q * jg;
  const double D = 1.0 - 4.0 * A * C;
  const bool okd = (D >= 0.0) && d_finite(D);
  const double sD = sqrt(D);
  const double isD = 1.0 / sD;
  const double z = 2.0 * C / (1.0 + sD);
  double dAl = q * ((vl * vl * vl) * ia2l);
  double dAr = -(q * ((vr * vr * vr) * ia2r));
  double dCl = -(q * vl);
  double dCr = q * vr;
  const double hjv2 = (0.5 * M.tau) * jv2, tjg = M.tau * jg;
  dAl = lvap ? dAl + hjv2 : dAl;
  dCl = lvap ? dCl + tjg : dCl;
  dAr = lvap ? dAr : dAr + hjv2;
  dCr = lvap ? dCr : dCr + tjg;
  const double dzl = (dAl * z * z + dCl) * isD;
  const double dzr = (dAr * z * z + dCr) * isD;
  const double jv = vr - vl;
  const double el = (vl * vl) * ia2l;
  const double er = (vr * vr) * ia2r;
  E.z = z;
  E.dzl = dzl;
  E.dzr = dzr;
  E.dfl = dfl;
  E.dfr = dfr;
  E.G1 = (psr - psl) + z * z * jv;
  E.G2 = (E.fl + E.fr) + z * jv + (R.Rt.u - R.L.u);
  E.J11 = -1.0 + 2.0 * z * dzl * jv + z * z * el;
  E.J12 = 1.0 + 2.0 * z * dzr * jv - z * z * er;
  E.J21 = dfl + dzl * jv + z * el;
  E.J22 = dfr + dzr * jv - z * er;
  const double a = E.G1 * R.izref;
  E.m2 = a * a + E.G2 * E.G2;
  return okw && okd && d_finite(E.G1) && d_finite(E.G2);
}

__device__ __forceinline__ bool d_eval_G(const Mat& M, const RP& R, double psl, double psr,
                                         GEval& E) {
  return d_eval_G_t<false>(M, R, psl, psr, 0, E);
}

// HLLC-type start (eq. HLLC:2p_nopt, mirrored when the liquid is on the left):
// contact speed and liquid star density from the two states, liquid law for
// the pressure; the vapour unknown is kept at or above 1e-3 of the vapour
// pressure.
__device__ __forceinline__ void d_guess(const Mat& M, const RP& R, double& gl, double& gr) {
  const Side &Ls = R.L, &Rs = R.Rt;
  double sl = Ls.u - d_a(M, Ls.ph), sr = Rs.u + d_a(M, Rs.ph);
  double num = (Rs.p - Ls.p) + Ls.r * Ls.u * (sl - Ls.u) - Rs.r * Rs.u * (sr - Rs.u);
  double den = Ls.r * (sl - Ls.u) - Rs.r * (sr - Rs.u);
  double ws = num / den;
  double rLs = (R.phl == LIQ) ? Ls.r * (sl - Ls.u) / (sl - ws) : Rs.r * (sr - Rs.u) / (sr - ws);
  double pg = d_pres(M, LIQ, rLs);
  double pV = (R.phl == VAP) ? Ls.p : Rs.p;
  double pvg = pg > 1e-3 * pV ? pg : 1e-3 * pV;
  if (R.phl == VAP) {
    gl = pvg;
    gr = pg;
  } else {
    gl = pg;
    gr = pvg;
  }
}

// Interface solve by Newton-Armijo from conservative states.  Starts are
// tried in order (the warm start if have_guess, the HLLC-type guess, both
// unknowns at the vapour pressure) until one converges.  From an accepted
// point: a Newton step below rtol (relative to max(|p_l*|, |p_r*|, p0)) is the
// last one; it is added to the root and, to first order, to the outputs
// (rho* exactly, being affine in p*; v*, f_K and z through the derivatives the
// evaluation at the point holds), with no further evaluation of G: Newton's
// error after the step is of the order of its square.  Otherwise the step is
// halved (at most 20 times) until the squared merit falls below
// (1 - 1e-4 lambda)^2 times the current one; if no halving passes, the point
// is kept when the step is already below 1e-8 (round-off floor), else the
// start fails; at most maxit steps per start.  Written as one loop with a
// single evaluation site so that lanes at different stages share it.
// PAIR: two lanes solve together (see d_eval_G_t): the lane with side 0, an
// even lane, passes the left state in (rl, ml), the one with side 1, the odd
// lane after it, the right state in (rr, mr); each sets up its own side and
// the two swap them (d_swap); both lanes return the same result.  has_u: the
// caller passes its side's velocity m / r in u_own (PAIR only).
template <bool PAIR>
__device__ __forceinline__ bool d_iface_solve_t(const Mat& M, int maxit, double rtol, int phl,
                                                double rl, double ml, int phr, double rr,
                                                double mr, bool have_guess, double gl, double gr,
                                                int side, IfaceOut& out, bool has_u = false,
                                                double u_own = 0.0) {
  RP R;
  R.phl = phl;
  if (PAIR) {
    Side own;
    d_side(M, side == 0 ? phl : phr, side == 0 ? rl : rr, side == 0 ? ml : mr, own, has_u, u_own);
    const double o_r = d_swap(own.r), o_u = d_swap(own.u);
    const double o_p = d_swap(own.p), o_LK = d_swap(own.LK);
    R.L.ph = phl;
    R.Rt.ph = phr;
    R.L.r = side == 0 ? own.r : o_r;
    R.L.u = side == 0 ? own.u : o_u;
    R.L.p = side == 0 ? own.p : o_p;
    R.L.LK = side == 0 ? own.LK : o_LK;
    R.Rt.r = side == 0 ? o_r : own.r;
    R.Rt.u = side == 0 ? o_u : own.u;
    R.Rt.p = side == 0 ? o_p : own.p;
    R.Rt.LK = side == 0 ? o_LK : own.LK;
    rl = R.L.r;
    rr = R.Rt.r;
    if (!(rl > 0.0) || !(rr > 0.0) || phl == phr) return false;
  } else {
    if (!(rl > 0.0) || !(rr > 0.0) || phl == phr) return false;
    d_side(M, phl, rl, ml, R.L);
    d_side(M, phr, rr, mr, R.Rt);
  }
  const double zl = rl * d_a(M, phl), zr = rr * d_a(M, phr);
  R.izref = 1.0 / (zl > zr ? zl : zr);
  int attempt = have_guess ? 0 : 1;
  double tl, tr;  // point to evaluate next
  if (attempt == 0) {
    tl = gl;
    tr = gr;
  } else {
    d_guess(M, R, tl, tr);
  }
  // accepted point and what survives it: squared merit and the outputs
  double xl = 0.0, xr = 0.0, m2 = 0.0, z = 0.0, vl = 0.0, fl = 0.0, vr = 0.0, fr = 0.0;
  double dl = 0.0, dr = 0.0, st = 0.0, sc = 0.0, lam = 1.0;
  int k = 0, it = 0, mode = 0;  // 0: start point, 1: Armijo trial
  int nev = 0;
  for (;;) {
    GEval Et;
    const bool valid = d_eval_G_t<PAIR>(M, R, tl, tr, side, Et);
    ++nev;
    bool done = false, take = false, next = false, acc = false;
    if (mode == 0) {
      if (!valid) {
        next = true;
      } else {
        acc = true;
        it = 0;
        take = true;
      }
    } else {
      const double c = 1.0 - 1e-4 * lam;
      if (valid && Et.m2 <= (c * c) * m2) {
        acc = true;
        ++it;
        take = true;
      } else {
        lam *= 0.5;
        ++k;
        if (k > 20) {
          if (st <= 1e-8 * sc)
            done = true;
          else
            next = true;
        } else {
          tl = xl + lam * dl;
          tr = xr + lam * dr;
        }
      }
    }
    if (acc) {
      xl = tl;
      xr = tr;
      m2 = Et.m2;
      z = Et.z;
      vl = Et.vl;
      fl = Et.fl;
      vr = Et.vr;
      fr = Et.fr;
    }
    if (take) {
      const double det = Et.J11 * Et.J22 - Et.J12 * Et.J21;
      if (it >= maxit || !(det != 0.0) || !d_finite(det)) {
        next = true;
      } else {
        const double idet = 1.0 / det;
        dl = (-Et.G1 * Et.J22 + Et.G2 * Et.J12) * idet;
        dr = (-Et.G2 * Et.J11 + Et.G1 * Et.J21) * idet;
        sc = fabs(xl) > fabs(xr) ? fabs(xl) : fabs(xr);
        if (M.p0 > sc) sc = M.p0;
        st = fabs(dl) > fabs(dr) ? fabs(dl) : fabs(dr);
        if (!d_finite(st)) {
          next = true;
        } else if (st <= rtol * sc) {
          // the last step, to first order; Et is the accepted point's evaluation
          const double ia2l = phl == VAP ? M.ia2v : M.ia2l;
          const double ia2r = phr == VAP ? M.ia2v : M.ia2l;
          xl = xl + dl;
          xr = xr + dr;
          vl = vl - ((Et.vl * Et.vl) * ia2l) * dl;
          vr = vr - ((Et.vr * Et.vr) * ia2r) * dr;
          fl = fl + Et.dfl * dl;
          fr = fr + Et.dfr * dr;
          z = z + (Et.dzl * dl + Et.dzr * dr);
          done = true;
        } else {
          mode = 1;
          lam = 1.0;
          k = 0;
          tl = xl + dl;
          tr = xr + dr;
        }
      }
    }
    if (done) break;
    if (next) {
      ++attempt;
      if (attempt >= 3) return false;
      if (attempt == 1) {
        d_guess(M, R, tl, tr);
      } else {
        tl = (phl == VAP) ? R.L.p : R.Rt.p;
        tr = tl;
      }
      mode = 0;
    }
  }
  out.pl = xl;
  out.pr = xr;
  out.rl = d_rho_of_p(M, phl, xl);
  out.rr = d_rho_of_p(M, phr, xr);
  out.ul = R.L.u - fl;
  out.ur = R.Rt.u + fr;
  out.z = z;
  double uV, vV, pV;
  if (phl == VAP) {
    uV = out.ul;
    vV = vl;
    pV = xl;
  } else {
    uV = out.ur;
    vV = vr;
    pV = xr;
  }
  out.w = uV + z * vV;
  out.F0 = -z;
  out.F1 = -z * uV + pV;
  out.nev = nev;
  return true;
}

__device__ __forceinline__ bool d_iface_solve(const Mat& M, int maxit, double rtol, int phl,
                                              double rl, double ml, int phr, double rr, double mr,
                                              bool have_guess, double gl, double gr,
                                              IfaceOut& out) {
  return d_iface_solve_t<false>(M, maxit, rtol, phl, rl, ml, phr, rr, mr, have_guess, gl, gr, 0,
                                out);
}

// Start of the interface solve of the next dual time pass.  The solver's
// root does not depend on where it starts (to round-off); the start only
// decides how many Newton steps it takes.  The roots of the last three passes
// (r0 newest, then r1, r2; nh of them recorded since the zone was set up)
// settle geometrically with the pseudo iterates: with fewer than three the
// start is the newest root, else each unknown is extrapolated one pass ahead,
// r0 + (d1 / d0) d1 with d1 = r0 - r1, d0 = r1 - r2, when |d1| < |d0|, and
// starts at r0 otherwise.
struct DtsRoots {
  double r0l, r0r, r1l, r1r, r2l, r2r;
  int nh;
};

__device__ __forceinline__ void d_dts_reset(DtsRoots& H) { H.nh = 0; }

// Records the newest root and returns the start of the next pass.
__device__ __forceinline__ void d_dts_record(DtsRoots& H, double pl, double pr, double& gl,
                                             double& gr) {
  H.r2l = H.r1l;
  H.r2r = H.r1r;
  H.r1l = H.r0l;
  H.r1r = H.r0r;
  H.r0l = pl;
  H.r0r = pr;
  if (H.nh < 3) ++H.nh;
  gl = pl;
  gr = pr;
  if (H.nh >= 3) {
    const double d1l = H.r0l - H.r1l, d0l = H.r1l - H.r2l;
    const double d1r = H.r0r - H.r1r, d0r = H.r1r - H.r2r;
    if (fabs(d1l) < fabs(d0l)) gl = H.r0l + (d1l / d0l) * d1l;
    if (fabs(d1r) < fabs(d0r)) gr = H.r0r + (d1r / d0r) * d1r;
  }
}

}  // namespace imexds
