// euler.hip -- the explicit-implicit scheme with dual time stepping for the
// full 1D Euler equations of an ideal gas on a fixed mesh with one small cell
// per problem (Sec. 4, first test; Algorithms 1 and 2), kernels and the host
// runtime behind include/imexds_euler.h.
//
// Kernels, one step of every problem:
//   k_eu_bulk  (tiles of cells) : Algorithm 1 Step 1 -- exact Godunov fluxes
//                                 on the faces of every cell but I_{k-1..k+1}
//                                 and their explicit update; epilogue: the
//                                 per-problem max(|u| + a) of the new state
//                                 (next CFL step) and the OR of failure bits,
//                                 one atomic per wave each.
//   k_eu_zone  (1 or 2 lanes per problem): Algorithm 2 on I_{k-1}, I_k,
//                                 I_{k+1}: F_{k-3/2}, F_{k+3/2} from U^n, dual
//                                 time iterations, Part 2; with 2 lanes the two
//                                 Riemann problems of an iteration run side by
//                                 side and the fluxes are swapped.
//   k_eu_fin   (lane per problem): t += dt, steps, status, the next dt.
// k_eu_bulk and k_eu_zone read only U^n and write disjoint cells of U^{n+1},
// so they run concurrently on two streams.
//
// Every expression is evaluated in the order written (-ffp-contract=off, no
// reassociation): results are bitwise those of any IEEE FP64 evaluation of
// the same expressions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/imexds_euler.h"
#include "imexds_device.hpp"

namespace eu {

constexpr int ST_VACUUM = 1, ST_NEWTON = 2, ST_NONPHYS = 4;
constexpr int FL_LMAX = 1;
constexpr int NEWTON_MAXIT = 60;
constexpr int ROW = 62;  // cells updated per 64-lane row of the sweep
constexpr unsigned long long NAN_BITS = 0x7FF8000000000000ull;

// ideal-gas constants, derived once on the host from gamma
struct Gas {
  double g, gm1, e1, ig, e5, e7, mu, gp, sk;
};

struct Args {
  Gas G;
  double tol_nb, tol_k;
  int lmax;
  int P;
  const long long* off;  // [P] first cell of the problem
  const int* N;          // [P]
  const double* h;
  const double* alpha;
  const double* thnb;
  const double* thk;
  const double* cfl;
  const double* tend;
  const int* tile_prob;
  const int* tile_start;
  const int* tile_len;
  const double *r0, *m0, *e0;  // U^n
  double *r1, *m1, *e1;        // U^{n+1}
  double* t;
  double* dt;
  double* dtr;              // the CFL step Delta t_ref (dt unless clipped to t_end)
  int* clipped;
  int* status;
  int* steps;
  long long* iters;
  int* cnt;                 // dual time iterations of this step
  int* fail;                // failure bits of this step
  unsigned long long* S;    // bit pattern of max(|u| + a) of the new state
  int* log_cnt;             // [log_max][P] or null
  int* log_fl;
  int log_row;              // row of this step (or -1)
  int zone_ppw;             // problems per wave in the dual time kernel
};

// exp of a finite double (Cody-Waite reduction by ln 2 with a head/tail split
// of ln 2, Taylor polynomial of degree 13 by Estrin's scheme, scaling by two
// powers of two built in the exponent field)
__device__ __forceinline__ double d_exp(double x) {
  if (x != x) return x;
  if (x > 709.782712893384) return __builtin_inf();
  if (x < -745.1332191019412) return 0.0;
  const double kf = floor(x * 1.4426950408889634 + 0.5);
  const double r = (x - kf * 0x1.62e42feep-1) - kf * 0x1.a39ef35793c76p-33;
  const double r2 = r * r, r4 = r2 * r2, r8 = r4 * r4;
  const double c0 = 1.0 + r, c1 = (1.0 / 2.0) + (1.0 / 6.0) * r;
  const double c2 = (1.0 / 24.0) + (1.0 / 120.0) * r, c3 = (1.0 / 720.0) + (1.0 / 5040.0) * r;
  const double c4 = (1.0 / 40320.0) + (1.0 / 362880.0) * r;
  const double c5 = (1.0 / 3628800.0) + (1.0 / 39916800.0) * r;
  const double c6 = (1.0 / 479001600.0) + (1.0 / 6227020800.0) * r;
  const double d0 = c0 + c1 * r2, d1 = c2 + c3 * r2, d2 = c4 + c5 * r2;
  const double q0 = d0 + d1 * r4, q1 = d2 + c6 * r4;
  const double poly = q0 + q1 * r8;
  const int k = (int)kf;
  const int ka = k / 2, kb = k - ka;
  const double sa = __longlong_as_double((long long)(ka + 1023) << 52);
  const double sb = __longlong_as_double((long long)(kb + 1023) << 52);
  return (poly * sa) * sb;
}

__device__ __forceinline__ double d_pow(double x, double e) {
  return d_exp(e * imexds::d_log(x));
}

// conserved -> primitive; false unless rho > 0, p > 0 and all finite
__device__ __forceinline__ bool d_prim(const Gas& G, double r, double m, double E, double& u,
                                       double& p) {
  u = m / r;
  p = G.gm1 * (E - 0.5 * m * u);
  return r > 0.0 && p > 0.0 && __builtin_isfinite(r) && __builtin_isfinite(p) &&
         __builtin_isfinite(u);
}

__device__ __forceinline__ void d_flux(const Gas& G, double r, double u, double p, double& F0,
                                       double& F1, double& F2) {
  const double m = r * u;
  const double E = p / G.gm1 + 0.5 * m * u;
  F0 = m;
  F1 = m * u + p;
  F2 = u * (E + p);
}

// velocity change across the wave from (rK, pK, aK) to pressure p, and its
// derivative: Rankine-Hugoniot branch for p > pK, isentrope otherwise
__device__ __forceinline__ void d_wave(const Gas& G, double p, double rK, double pK, double aK,
                                       double& f, double& df) {
  if (p > pK) {
    const double A = G.gp / rK, B = G.mu * pK;
    const double q = sqrt(A / (p + B));
    f = (p - pK) * q;
    df = q * (1.0 - 0.5 * (p - pK) / (p + B));
  } else {
    const double pr = p / pK;
    const double t = d_pow(pr, G.e1);
    f = G.e5 * aK * (t - 1.0);
    df = t / (rK * aK * pr);
  }
}

// Exact Riemann solution of (rL,uL,pL | rR,uR,pR) sampled on the face
// (x/t = 0) and its flux; returns 0 or ST_VACUUM / ST_NEWTON.
__device__ int d_godunov(const Gas& G, double rL, double uL, double pL, double rR, double uR,
                         double pR, double& F0, double& F1, double& F2) {
  const double aL = sqrt(G.g * pL / rL), aR = sqrt(G.g * pR / rR);
  const double du = uR - uL;
  if (G.e5 * (aL + aR) <= du) return ST_VACUUM;
  // Newton on f_L(p) + f_R(p) + du = 0 from the linearised guess
  const double ppv = 0.5 * (pL + pR) - 0.125 * du * (rL + rR) * (aL + aR);
  const double pfloor = 1e-6 * (pL < pR ? pL : pR);
  double p = ppv > pfloor ? ppv : pfloor;
  double fL, dfL, fR, dfR;
  int it;
  for (it = 0; it < NEWTON_MAXIT; ++it) {
    d_wave(G, p, rL, pL, aL, fL, dfL);
    d_wave(G, p, rR, pR, aR, fR, dfR);
    double pn = p - (fL + fR + du) / (dfL + dfR);
    if (!(pn > 0.0)) pn = 0.5 * p;
    const double ch = fabs(pn - p);
    p = pn;
    if (ch <= 1e-14 * pn) break;
  }
  if (it == NEWTON_MAXIT || !(p > 0.0) || !__builtin_isfinite(p)) return ST_NEWTON;
  d_wave(G, p, rL, pL, aL, fL, dfL);
  d_wave(G, p, rR, pR, aR, fR, dfR);
  const double ps = p;
  const double us = 0.5 * (uL + uR) + 0.5 * (fR - fL);
  // the side of the contact the face sees, then the wave of that side
  const bool left = us >= 0.0;
  const double rK = left ? rL : rR, uK = left ? uL : uR, pK = left ? pL : pR;
  const double aK = left ? aL : aR;
  const double sg = left ? -1.0 : 1.0;  // direction of the outer wave
  double r, u, pp;
  const double q = ps / pK;
  if (ps > pK) {  // shock
    const double S = uK + sg * (aK * sqrt(G.sk * q + G.e1));
    const bool outside = left ? S >= 0.0 : S <= 0.0;
    if (outside) {
      r = rK;
      u = uK;
      pp = pK;
    } else {
      r = rK * ((q + G.mu) / (G.mu * q + 1.0));
      u = us;
      pp = ps;
    }
  } else {  // rarefaction
    const double Sh = uK + sg * aK;
    const bool outside = left ? Sh >= 0.0 : Sh <= 0.0;
    if (outside) {
      r = rK;
      u = uK;
      pp = pK;
    } else {
      const double as = aK * d_pow(q, G.e1);
      const double St = us + sg * as;
      const bool star = left ? St < 0.0 : St > 0.0;
      if (star) {
        r = rK * d_pow(q, G.ig);
        u = us;
        pp = ps;
      } else {  // inside the fan: u -+ a = 0 on the face
        const double c = left ? G.gp * (aK + 0.5 * G.gm1 * uK) : G.gp * (aK - 0.5 * G.gm1 * uK);
        const double qa = c / aK;
        r = rK * d_pow(qa, G.e5);
        u = left ? c : -c;
        pp = pK * d_pow(qa, G.e7);
      }
    }
  }
  d_flux(G, r, u, pp, F0, F1, F2);
  return 0;
}

// flux between two conserved states, failure bits as the return value
__device__ __forceinline__ int d_face(const Gas& G, double rl, double ml, double El, double rr,
                                      double mr, double Er, double& F0, double& F1,
                                      double& F2) {
  double ul, pl, ur, pr;
  const bool okl = d_prim(G, rl, ml, El, ul, pl);
  const bool okr = d_prim(G, rr, mr, Er, ur, pr);
  if (!okl || !okr) return ST_NONPHYS;
  return d_godunov(G, rl, ul, pl, rr, ur, pr, F0, F1, F2);
}

__device__ __forceinline__ unsigned long long d_speed_bits(const Gas& G, double r, double m,
                                                           double E) {
  double u, p;
  if (!d_prim(G, r, m, E, u, p)) return NAN_BITS;
  return (unsigned long long)__double_as_longlong(fabs(u) + sqrt(G.g * p / r));
}

__device__ __forceinline__ unsigned long long d_wave_max(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

__device__ __forceinline__ int d_wave_or(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// explicit sweep.  A workgroup is 4 waves, each R rows of 62 cells; in a row
// lane j holds cell base-1+j, computes the flux on the face to its right
// (its right neighbour's state comes by a lane shuffle), takes its left face
// from lane j-1, and lanes 1..62 update their cell.
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(256) void k_eu_bulk(Args A, int tile_begin) {
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int tile = tile_begin + blockIdx.x;
  const int p = A.tile_prob[tile];
  const int t0 = A.tile_start[tile];
  const int tend = t0 + A.tile_len[tile];
  const long long o = A.off[p];
  const int n = A.N[p] + 1;
  const int k = A.N[p] / 2;
  const double dt = A.dt[p];
  const double* __restrict__ r0 = A.r0 + o;
  const double* __restrict__ m0 = A.m0 + o;
  const double* __restrict__ E0 = A.e0 + o;
  double* __restrict__ r1 = A.r1 + o;
  double* __restrict__ m1 = A.m1 + o;
  double* __restrict__ E1 = A.e1 + o;
  if (dt == 0.0) {  // frozen or finished: carry the state over
    for (int c = t0 + (int)threadIdx.x; c < tend; c += 256) {
      if (c >= k - 1 && c <= k + 1) continue;
      r1[c] = r0[c];
      m1[c] = m0[c];
      E1[c] = E0[c];
    }
    return;
  }
  const Gas& G = A.G;
  const double lam = dt / A.h[p];
  int code = 0;
  unsigned long long vmax = 0;
#pragma unroll 1
  for (int row = 0; row < R; ++row) {
    const int base = t0 + (wv * R + row) * ROW;
    if (base >= tend) break;  // uniform over the wave
    const int s = base - 1 + lane;
    const int se = s < 0 ? 0 : (s > n - 1 ? n - 1 : s);
    const double rho = r0[se], mom = m0[se], ene = E0[se];
    double u, pr;
    const bool ok = d_prim(G, rho, mom, ene, u, pr);
    const double rR = __shfl_down(rho, 1, 64);
    const double uR = __shfl_down(u, 1, 64);
    const double pR = __shfl_down(pr, 1, 64);
    const int okR = __shfl_down((int)ok, 1, 64);
    // flux on face s+1 (between cells s and s+1)
    double F0 = 0.0, F1 = 0.0, F2 = 0.0;
    const int j = s + 1;
    if (lane <= ROW && j <= n && j != k && j != k + 1) {
      if (j == 0 || j == n) {  // transmissive boundary: flux of the boundary cell
        if (ok)
          d_flux(G, rho, u, pr, F0, F1, F2);
        else
          code |= ST_NONPHYS;
      } else if (!ok || !okR) {
        code |= ST_NONPHYS;
      } else {
        code |= d_godunov(G, rho, u, pr, rR, uR, pR, F0, F1, F2);
      }
    }
    const double G0 = __shfl_up(F0, 1, 64);
    const double G1 = __shfl_up(F1, 1, 64);
    const double G2 = __shfl_up(F2, 1, 64);
    if (lane >= 1 && lane <= ROW && s < tend && (s < k - 1 || s > k + 1)) {
      const double rn = rho - lam * (F0 - G0);
      const double mn = mom - lam * (F1 - G1);
      const double En = ene - lam * (F2 - G2);
      r1[s] = rn;
      m1[s] = mn;
      E1[s] = En;
      const unsigned long long v = d_speed_bits(G, rn, mn, En);
      vmax = v > vmax ? v : vmax;
    }
  }
  vmax = d_wave_max(vmax);
  code = d_wave_or(code);
  if (lane == 0) {
    if (vmax) atomicMax(A.S + p, vmax);
    if (code) atomicOr(A.fail + p, code);
  }
}

// CFL bound of the initial state (every cell)
__global__ __launch_bounds__(256) void k_eu_cfl(Args A, int tile_begin) {
  const int tile = tile_begin + blockIdx.x;
  const int p = A.tile_prob[tile];
  const int t0 = A.tile_start[tile];
  const int tend = t0 + A.tile_len[tile];
  const long long o = A.off[p];
  unsigned long long vmax = 0;
  for (int c = t0 + (int)threadIdx.x; c < tend; c += 256) {
    const unsigned long long v = d_speed_bits(A.G, A.r0[o + c], A.m0[o + c], A.e0[o + c]);
    vmax = v > vmax ? v : vmax;
  }
  vmax = d_wave_max(vmax);
  if ((threadIdx.x & 63) == 0 && vmax) atomicMax(A.S + p, vmax);
}

// ---------------------------------------------------------------------------
// dual time stepping on I_{k-1}, I_k, I_{k+1}.  L lanes per problem (1 or 2).
// With L = 2 both lanes hold the three iterates; lane 0 evaluates the face
// k-1/2 and lane 1 the face k+1/2 (and F_{k-3/2}, F_{k+3/2} likewise), the
// fluxes are swapped, and both lanes apply the same updates and stop test.
// A pair never splits: both lanes take every branch together.
// ---------------------------------------------------------------------------
template <int L>
__global__ __launch_bounds__(64) void k_eu_zone(Args A) {
  // a workgroup is one wave holding zone_ppw problems in its first lanes.
  // Each problem is a serial chain of dual time iterations; packing 32 of
  // them per wave (the default) leaves the other SIMDs to the sweep that runs
  // beside this kernel, which measured faster than fewer problems per wave
  const int lane = (int)threadIdx.x;
  if (lane >= A.zone_ppw * L) return;
  const int p = blockIdx.x * A.zone_ppw + lane / L;
  const int side = L == 2 ? (lane & 1) : 0;
  if (p >= A.P) return;  // pairs are whole: both lanes of a pair see the same p
  const long long o = A.off[p];
  const int k = A.N[p] / 2;
  const double* __restrict__ r0 = A.r0 + o;
  const double* __restrict__ m0 = A.m0 + o;
  const double* __restrict__ E0 = A.e0 + o;
  double* __restrict__ r1 = A.r1 + o;
  double* __restrict__ m1 = A.m1 + o;
  double* __restrict__ E1 = A.e1 + o;
  const double dt = A.dt[p];
  const bool writer = side == 0;
  if (dt == 0.0) {
    if (writer) {
      for (int c = k - 1; c <= k + 1; ++c) {
        r1[c] = r0[c];
        m1[c] = m0[c];
        E1[c] = E0[c];
      }
      if (A.log_row >= 0) {
        A.log_cnt[(long long)A.log_row * A.P + p] = 0;
        A.log_fl[(long long)A.log_row * A.P + p] = 0;
      }
    }
    return;
  }
  const Gas& G = A.G;
  const double h = A.h[p];
  const double hk = A.alpha[p] * h;
  const double lam = dt / h, lamk = dt / hk;
  // pseudo steps Delta tau_i = theta_i Delta t_ref (Sec. 4); the update uses
  // Delta tau_i / Delta t, which is theta_i unless the step was clipped
  const double dtr = A.dtr[p];
  const double tau0 = A.thnb[p] * dtr, tau1 = A.thk[p] * dtr;
  double th0 = A.thnb[p], th1 = A.thk[p];
  if (A.clipped[p]) {
    th0 = tau0 / dt;
    th1 = tau1 / dt;
  }
  const double thr0 = A.tol_nb * tau0, thr1 = A.tol_k * tau1;
  // U^n of the three cells: a = k-1, b = k, c = k+1
  const double ra = r0[k - 1], ma = m0[k - 1], Ea = E0[k - 1];
  const double rb = r0[k], mb = m0[k], Eb = E0[k];
  const double rc = r0[k + 1], mc = m0[k + 1], Ec = E0[k + 1];
  int code = 0, cnt = 0, fl = 0;
  double Fl0 = 0, Fl1 = 0, Fl2 = 0, Fr0 = 0, Fr1 = 0, Fr2 = 0;  // F_left, F_right
  // F_{k-3/2} from (U_{k-2}, U_{k-1}) and F_{k+3/2} from (U_{k+1}, U_{k+2})
#pragma unroll 1
  for (int f = side; f < 2; f += L) {
    const bool lf = f == 0;
    double X0, X1, X2;
    const int cl = lf ? k - 2 : k + 1;
    const int c = cl + 1;
    const int e = d_face(G, r0[cl], m0[cl], E0[cl], r0[c], m0[c], E0[c], X0, X1, X2);
    code |= e;
    if (lf) {
      Fl0 = X0; Fl1 = X1; Fl2 = X2;
    } else {
      Fr0 = X0; Fr1 = X1; Fr2 = X2;
    }
  }
  if (L == 2) {
    // lane 0 has F_left, lane 1 F_right: exchange
    const double y0 = __shfl_xor(side ? Fr0 : Fl0, 1, 64);
    const double y1 = __shfl_xor(side ? Fr1 : Fl1, 1, 64);
    const double y2 = __shfl_xor(side ? Fr2 : Fl2, 1, 64);
    const int yc = __shfl_xor(code, 1, 64);
    if (side) {
      Fl0 = y0; Fl1 = y1; Fl2 = y2;
    } else {
      Fr0 = y0; Fr1 = y1; Fr2 = y2;
    }
    code |= yc;
  }
  double Wa0 = ra, Wa1 = ma, Wa2 = Ea, Wb0 = rb, Wb1 = mb, Wb2 = Eb, Wc0 = rc, Wc1 = mc, Wc2 = Ec;
  double Km0 = 0, Km1 = 0, Km2 = 0, Kp0 = 0, Kp1 = 0, Kp2 = 0;  // F_{k-1/2}, F_{k+1/2}
  bool done = false, part2 = false;
  if (code == 0) {
    // Part 1; the pass with part2 set evaluates the fluxes of the accepted
    // iterate for Part 2 and leaves the loop
#pragma unroll 1
    for (int l = 0;; ++l) {
      part2 = done || l == A.lmax + 1;
      // the two faces of the small cell at the current iterate
      int ec = 0;
#pragma unroll 1
      for (int f = side; f < 2; f += L) {
        const bool lf = f == 0;
        double X0, X1, X2;
        const double x0 = lf ? Wa0 : Wb0, x1 = lf ? Wa1 : Wb1, x2 = lf ? Wa2 : Wb2;
        const double y0 = lf ? Wb0 : Wc0, y1 = lf ? Wb1 : Wc1, y2 = lf ? Wb2 : Wc2;
        ec |= d_face(G, x0, x1, x2, y0, y1, y2, X0, X1, X2);
        if (lf) {
          Km0 = X0; Km1 = X1; Km2 = X2;
        } else {
          Kp0 = X0; Kp1 = X1; Kp2 = X2;
        }
      }
      if (L == 2) {
        const double y0 = __shfl_xor(side ? Kp0 : Km0, 1, 64);
        const double y1 = __shfl_xor(side ? Kp1 : Km1, 1, 64);
        const double y2 = __shfl_xor(side ? Kp2 : Km2, 1, 64);
        ec |= __shfl_xor(ec, 1, 64);
        if (side) {
          Km0 = y0; Km1 = y1; Km2 = y2;
        } else {
          Kp0 = y0; Kp1 = y1; Kp2 = y2;
        }
      }
      if (ec) {
        code |= ec;
        if (!part2) cnt = 0;  // a failure inside Part 1 reports no iterations
        break;
      }
      if (part2) break;
      // pseudo step (eq. dual time tau diff with Delta tau_i = theta_i dt)
      const double na0 = (Wa0 + th0 * (ra - lam * (Km0 - Fl0))) / (1.0 + th0);
      const double na1 = (Wa1 + th0 * (ma - lam * (Km1 - Fl1))) / (1.0 + th0);
      const double na2 = (Wa2 + th0 * (Ea - lam * (Km2 - Fl2))) / (1.0 + th0);
      const double nb0 = (Wb0 + th1 * (rb - lamk * (Kp0 - Km0))) / (1.0 + th1);
      const double nb1 = (Wb1 + th1 * (mb - lamk * (Kp1 - Km1))) / (1.0 + th1);
      const double nb2 = (Wb2 + th1 * (Eb - lamk * (Kp2 - Km2))) / (1.0 + th1);
      const double nc0 = (Wc0 + th0 * (rc - lam * (Fr0 - Kp0))) / (1.0 + th0);
      const double nc1 = (Wc1 + th0 * (mc - lam * (Fr1 - Kp1))) / (1.0 + th0);
      const double nc2 = (Wc2 + th0 * (Ec - lam * (Fr2 - Kp2))) / (1.0 + th0);
      // stop test of Sec. 4, multiplied out
      bool ok = true;
#define EU_TEST(Wo, Wn, th, thr)                                   \
  {                                                                \
    const double d = (1.0 + th) * (Wn - Wo);                       \
    double sc = fabs(Wo);                                          \
    if (sc < 1.0) sc = 1.0;                                        \
    ok = ok && (fabs(d) < thr * sc);                               \
  }
      EU_TEST(Wa0, na0, th0, thr0) EU_TEST(Wa1, na1, th0, thr0) EU_TEST(Wa2, na2, th0, thr0)
      EU_TEST(Wb0, nb0, th1, thr1) EU_TEST(Wb1, nb1, th1, thr1) EU_TEST(Wb2, nb2, th1, thr1)
      EU_TEST(Wc0, nc0, th0, thr0) EU_TEST(Wc1, nc1, th0, thr0) EU_TEST(Wc2, nc2, th0, thr0)
#undef EU_TEST
      Wa0 = na0; Wa1 = na1; Wa2 = na2;
      Wb0 = nb0; Wb1 = nb1; Wb2 = nb2;
      Wc0 = nc0; Wc1 = nc1; Wc2 = nc2;
      done = ok;
      cnt = l + 1;
    }
    if (part2 && !done) fl |= FL_LMAX;
  }
  if (writer) {
    if (code == 0) {
      // Part 2: conservative update with the fluxes of the accepted iterate
      const double na0 = ra - lam * (Km0 - Fl0), na1 = ma - lam * (Km1 - Fl1),
                   na2 = Ea - lam * (Km2 - Fl2);
      const double nb0 = rb - lamk * (Kp0 - Km0), nb1 = mb - lamk * (Kp1 - Km1),
                   nb2 = Eb - lamk * (Kp2 - Km2);
      const double nc0 = rc - lam * (Fr0 - Kp0), nc1 = mc - lam * (Fr1 - Kp1),
                   nc2 = Ec - lam * (Fr2 - Kp2);
      r1[k - 1] = na0; m1[k - 1] = na1; E1[k - 1] = na2;
      r1[k] = nb0; m1[k] = nb1; E1[k] = nb2;
      r1[k + 1] = nc0; m1[k + 1] = nc1; E1[k + 1] = nc2;
      const unsigned long long va = d_speed_bits(G, na0, na1, na2);
      const unsigned long long vb = d_speed_bits(G, nb0, nb1, nb2);
      const unsigned long long vc = d_speed_bits(G, nc0, nc1, nc2);
      if (va == NAN_BITS || vb == NAN_BITS || vc == NAN_BITS) code |= ST_NONPHYS;
      unsigned long long v = va > vb ? va : vb;
      v = vc > v ? vc : v;
      atomicMax(A.S + p, v);
    }
    if (code) atomicOr(A.fail + p, code);
    A.cnt[p] = cnt;
    if (A.log_row >= 0) {
      A.log_cnt[(long long)A.log_row * A.P + p] = cnt;
      A.log_fl[(long long)A.log_row * A.P + p] = fl;
    }
  }
}

// ---------------------------------------------------------------------------
// per-problem bookkeeping between steps
// ---------------------------------------------------------------------------
__global__ void k_eu_fin(Args A, int init) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= A.P) return;
  double dt = A.dt[p];
  int st = A.status[p];
  double t = A.t[p];
  const double tend = A.tend[p];
  if (!init && dt > 0.0) {
    const int f = A.fail[p];
    if (f) {
      st |= f;
    } else {
      t = A.clipped[p] ? tend : t + dt;
      A.steps[p] += 1;
      A.iters[p] += A.cnt[p];
    }
  }
  double ndt = 0.0, nref = 0.0;
  int clip = 0;
  if (st == 0 && t < tend) {
    const double S = __longlong_as_double((long long)A.S[p]);
    if (!(S > 0.0) || !__builtin_isfinite(S)) {
      st |= ST_NONPHYS;
    } else {
      nref = (A.cfl[p] * A.h[p]) / S;
      ndt = nref;
      const double rem = tend - t;
      if (ndt >= rem) {
        ndt = rem;
        clip = 1;
      }
    }
  }
  A.dt[p] = st == 0 ? ndt : 0.0;
  A.dtr[p] = st == 0 ? nref : 0.0;
  A.t[p] = t;
  A.status[p] = st;
  A.clipped[p] = clip;
  A.S[p] = 0ull;
  A.fail[p] = 0;
  A.cnt[p] = 0;
}

}  // namespace eu

// ===========================================================================
// host runtime
// ===========================================================================
struct imexds_eu_ctx {
  int device = 0;
  hipStream_t user = nullptr, ms = nullptr, zs = nullptr;
  hipEvent_t ev_in = nullptr, ev_fork = nullptr, ev_join = nullptr, ev_out = nullptr;
  eu::Gas gas{};
  double tol_nb = 0, tol_k = 0;
  int lmax = 0;
  int P = 0;
  long long ncell = 0;
  std::vector<int> h_N;
  std::vector<long long> h_off;
  std::vector<int> h_tile_first;  // [P + 1] first tile of each problem
  // device
  long long* off = nullptr;
  int *N = nullptr, *clipped = nullptr, *status = nullptr, *steps = nullptr, *cnt = nullptr,
      *fail = nullptr;
  double *h = nullptr, *alpha = nullptr, *thnb = nullptr, *thk = nullptr, *cfl = nullptr,
         *tend = nullptr, *t = nullptr, *dt = nullptr, *dtr = nullptr;
  long long* iters = nullptr;
  unsigned long long* S = nullptr;
  double* U[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
  int cur = 0;
  int *tile_prob = nullptr, *tile_start = nullptr, *tile_len = nullptr;
  int n_tiles = 0, tile_class = 1024, zone_lanes = 2, zone_ppw = 32;
  int *log_cnt = nullptr, *log_fl = nullptr;
  int log_max = 0, log_row = 0;
  bool have_state = false;
  // timing
  bool timing = false;
  std::vector<hipEvent_t> tev;  // 6 per step: step begin, bulk 0/1, zone 0/1, step end
  int timed_steps = 0;
};

namespace {

constexpr int TIMED_MAX = 4096;

template <class T>
int dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc((void**)p, n * sizeof(T)) == hipSuccess ? 0 : IMEXDS_ERR_OOM;
}

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

int hip_err(hipError_t e) { return e == hipSuccess ? 0 : IMEXDS_ERR_HIP; }

int tile_cells_of(int cls) { return (cls / 256) * 4 * eu::ROW; }

void release(imexds_eu_ctx* c) {
  dfree(c->off);
  dfree(c->N);
  dfree(c->clipped);
  dfree(c->status);
  dfree(c->steps);
  dfree(c->cnt);
  dfree(c->fail);
  dfree(c->h);
  dfree(c->alpha);
  dfree(c->thnb);
  dfree(c->thk);
  dfree(c->cfl);
  dfree(c->tend);
  dfree(c->t);
  dfree(c->dt);
  dfree(c->dtr);
  dfree(c->iters);
  dfree(c->S);
  for (int b = 0; b < 2; ++b)
    for (int q = 0; q < 3; ++q) dfree(c->U[b][q]);
  dfree(c->tile_prob);
  dfree(c->tile_start);
  dfree(c->tile_len);
  dfree(c->log_cnt);
  dfree(c->log_fl);
  for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
  c->tev.clear();
  for (hipEvent_t* e : {&c->ev_in, &c->ev_fork, &c->ev_join, &c->ev_out})
    if (*e) (void)hipEventDestroy(*e), *e = nullptr;
  if (c->ms) (void)hipStreamDestroy(c->ms);
  if (c->zs) (void)hipStreamDestroy(c->zs);
  c->ms = c->zs = nullptr;
}

int build_tiles(imexds_eu_ctx* c) {
  dfree(c->tile_prob);
  dfree(c->tile_start);
  dfree(c->tile_len);
  const int T = tile_cells_of(c->tile_class);
  std::vector<int> tp, ts, tl;
  c->h_tile_first.assign(c->P + 1, 0);
  for (int p = 0; p < c->P; ++p) {
    c->h_tile_first[p] = (int)tp.size();
    const int n = c->h_N[p] + 1;
    for (int s = 0; s < n; s += T) {
      tp.push_back(p);
      ts.push_back(s);
      tl.push_back(std::min(T, n - s));
    }
  }
  c->n_tiles = (int)tp.size();
  c->h_tile_first[c->P] = c->n_tiles;
  int e = dalloc(&c->tile_prob, tp.size());
  if (!e) e = dalloc(&c->tile_start, ts.size());
  if (!e) e = dalloc(&c->tile_len, tl.size());
  if (e) return e;
  if (c->n_tiles) {
    e = hip_err(hipMemcpy(c->tile_prob, tp.data(), tp.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!e) e = hip_err(hipMemcpy(c->tile_start, ts.data(), ts.size() * sizeof(int),
                                  hipMemcpyHostToDevice));
    if (!e) e = hip_err(hipMemcpy(c->tile_len, tl.data(), tl.size() * sizeof(int),
                                  hipMemcpyHostToDevice));
  }
  return e;
}

eu::Args make_args(const imexds_eu_ctx* c, int parity) {
  eu::Args A{};
  A.G = c->gas;
  A.tol_nb = c->tol_nb;
  A.tol_k = c->tol_k;
  A.lmax = c->lmax;
  A.P = c->P;
  A.off = c->off;
  A.N = c->N;
  A.h = c->h;
  A.alpha = c->alpha;
  A.thnb = c->thnb;
  A.thk = c->thk;
  A.cfl = c->cfl;
  A.tend = c->tend;
  A.tile_prob = c->tile_prob;
  A.tile_start = c->tile_start;
  A.tile_len = c->tile_len;
  A.r0 = c->U[parity][0];
  A.m0 = c->U[parity][1];
  A.e0 = c->U[parity][2];
  A.r1 = c->U[parity ^ 1][0];
  A.m1 = c->U[parity ^ 1][1];
  A.e1 = c->U[parity ^ 1][2];
  A.t = c->t;
  A.dt = c->dt;
  A.dtr = c->dtr;
  A.clipped = c->clipped;
  A.status = c->status;
  A.steps = c->steps;
  A.iters = c->iters;
  A.cnt = c->cnt;
  A.fail = c->fail;
  A.S = c->S;
  A.log_cnt = c->log_cnt;
  A.log_fl = c->log_fl;
  A.log_row = (c->log_cnt && c->log_row < c->log_max) ? c->log_row : -1;
  A.zone_ppw = c->zone_ppw;
  return A;
}

hipError_t launch_bulk(const eu::Args& A, int cls, int n_tiles, hipStream_t s,
                       int tile_begin = 0) {
  if (n_tiles <= 0) return hipSuccess;
  switch (cls) {
    case 256: eu::k_eu_bulk<1><<<n_tiles, 256, 0, s>>>(A, tile_begin); break;
    case 512: eu::k_eu_bulk<2><<<n_tiles, 256, 0, s>>>(A, tile_begin); break;
    case 1024: eu::k_eu_bulk<4><<<n_tiles, 256, 0, s>>>(A, tile_begin); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zone(const eu::Args& A, int lanes, hipStream_t s) {
  if (A.P <= 0) return hipSuccess;
  const int blocks = (A.P + A.zone_ppw - 1) / A.zone_ppw;
  if (lanes == 2)
    eu::k_eu_zone<2><<<blocks, 64, 0, s>>>(A);
  else
    eu::k_eu_zone<1><<<blocks, 64, 0, s>>>(A);
  return hipGetLastError();
}

hipError_t launch_fin(const eu::Args& A, int init, hipStream_t s) {
  const int blocks = A.P > 0 ? (A.P + 255) / 256 : 1;
  eu::k_eu_fin<<<blocks, 256, 0, s>>>(A, init);
  return hipGetLastError();
}

// orders the context's streams after the caller's stream
int enter(imexds_eu_ctx* c) {
  int e = hip_err(hipSetDevice(c->device));
  if (!e) e = hip_err(hipEventRecord(c->ev_in, c->user));
  if (!e) e = hip_err(hipStreamWaitEvent(c->ms, c->ev_in, 0));
  return e;
}

// orders the caller's stream after the context's main stream
int leave(imexds_eu_ctx* c) {
  int e = hip_err(hipEventRecord(c->ev_out, c->ms));
  if (!e) e = hip_err(hipStreamWaitEvent(c->user, c->ev_out, 0));
  return e;
}

hipEvent_t timing_event(imexds_eu_ctx* c, int i) {
  while ((int)c->tev.size() <= i) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->tev.push_back(e);
  }
  return c->tev[i];
}

int one_step(imexds_eu_ctx* c) {
  eu::Args A = make_args(c, c->cur);
  hipEvent_t tb = nullptr, b0 = nullptr, b1 = nullptr, z0 = nullptr, z1 = nullptr,
             te = nullptr;
  const bool tm = c->timing && c->timed_steps < TIMED_MAX;
  if (tm) {
    const int i = 6 * c->timed_steps;
    tb = timing_event(c, i);
    b0 = timing_event(c, i + 1);
    b1 = timing_event(c, i + 2);
    z0 = timing_event(c, i + 3);
    z1 = timing_event(c, i + 4);
    te = timing_event(c, i + 5);
    if (!tb || !b0 || !b1 || !z0 || !z1 || !te) return IMEXDS_ERR_HIP;
    if (hipEventRecord(tb, c->ms) != hipSuccess) return IMEXDS_ERR_HIP;
  }
  int e = hip_err(hipEventRecord(c->ev_fork, c->ms));
  if (!e) e = hip_err(hipStreamWaitEvent(c->zs, c->ev_fork, 0));
  if (!e && tm) e = hip_err(hipEventRecord(z0, c->zs));
  if (!e) e = hip_err(launch_zone(A, c->zone_lanes, c->zs));
  if (!e && tm) e = hip_err(hipEventRecord(z1, c->zs));
  if (!e && tm) e = hip_err(hipEventRecord(b0, c->ms));
  if (!e) e = hip_err(launch_bulk(A, c->tile_class, c->n_tiles, c->ms));
  if (!e && tm) e = hip_err(hipEventRecord(b1, c->ms));
  if (!e) e = hip_err(hipEventRecord(c->ev_join, c->zs));
  if (!e) e = hip_err(hipStreamWaitEvent(c->ms, c->ev_join, 0));
  if (!e) e = hip_err(launch_fin(A, 0, c->ms));
  if (!e && tm) e = hip_err(hipEventRecord(te, c->ms));
  if (e) return e;
  if (tm) c->timed_steps += 1;
  c->cur ^= 1;
  c->log_row += 1;
  return 0;
}

// The arguments of problem p alone: per-problem arrays shifted to p, one
// problem, no log (the cell arrays and the tile table stay global).
eu::Args problem_args(const eu::Args& A, int p) {
  eu::Args B = A;
  B.P = 1;
  B.off += p;
  B.N += p;
  B.h += p;
  B.alpha += p;
  B.thnb += p;
  B.thk += p;
  B.cfl += p;
  B.tend += p;
  B.t += p;
  B.dt += p;
  B.dtr += p;
  B.clipped += p;
  B.status += p;
  B.steps += p;
  B.iters += p;
  B.cnt += p;
  B.fail += p;
  B.S += p;
  B.log_cnt = nullptr;
  B.log_fl = nullptr;
  B.log_row = -1;
  return B;
}

// One step launched problem by problem on the main stream: the unbatched form.
int one_step_per_problem(imexds_eu_ctx* c) {
  eu::Args A = make_args(c, c->cur);
  int e = 0;
  for (int p = 0; p < c->P && !e; ++p) {
    const eu::Args B = problem_args(A, p);
    const int t0 = c->h_tile_first[p], nt = c->h_tile_first[p + 1] - t0;
    e = hip_err(launch_bulk(A, c->tile_class, nt, c->ms, t0));
    if (!e) e = hip_err(launch_zone(B, c->zone_lanes, c->ms));
    if (!e) e = hip_err(launch_fin(B, 0, c->ms));
  }
  if (e) return e;
  c->cur ^= 1;
  c->log_row += 1;
  return 0;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

extern "C" {

int imexds_eu_create(imexds_eu_ctx** out, const imexds_eu_params* par,
                     const imexds_eu_batch* b, void* hip_stream) {
  if (!out) return IMEXDS_ERR_INVALID_ARG;
  *out = nullptr;
  if (!par || !b || b->n_problems < 0) return IMEXDS_ERR_INVALID_ARG;
  if (!(std::isfinite(par->gamma) && par->gamma > 1.0) || !finite_pos(par->tol_nb) ||
      !finite_pos(par->tol_k) || par->lmax < 0 || par->lmax > 2000000000)
    return IMEXDS_ERR_INVALID_ARG;
  const int P = b->n_problems;
  if (P > 0 && (!b->N || !b->h || !b->alpha || !b->theta_nb || !b->theta_k || !b->cfl ||
                !b->t_end))
    return IMEXDS_ERR_INVALID_ARG;
  long long ncell = 0;
  std::vector<long long> off(P + 1, 0);
  for (int p = 0; p < P; ++p) {
    const int N = b->N[p];
    if (N < 4 || N % 2 || N > (1 << 28)) return IMEXDS_ERR_INVALID_ARG;
    if (!finite_pos(b->h[p]) || !finite_pos(b->alpha[p]) || b->alpha[p] > 1.0 ||
        !finite_pos(b->theta_nb[p]) || b->theta_nb[p] > 1.0 || !finite_pos(b->theta_k[p]) ||
        b->theta_k[p] > 1.0 || !finite_pos(b->cfl[p]) || !(b->t_end[p] >= 0.0) ||
        std::isnan(b->t_end[p]))
      return IMEXDS_ERR_INVALID_ARG;
    off[p + 1] = off[p] + N + 1;
  }
  ncell = off[P];
  imexds_eu_ctx* c = new (std::nothrow) imexds_eu_ctx();
  if (!c) return IMEXDS_ERR_OOM;
  int e = hip_err(hipGetDevice(&c->device));
  c->user = (hipStream_t)hip_stream;
  if (!e) e = hip_err(hipStreamCreateWithFlags(&c->ms, hipStreamNonBlocking));
  if (!e) e = hip_err(hipStreamCreateWithFlags(&c->zs, hipStreamNonBlocking));
  for (hipEvent_t* ev : {&c->ev_in, &c->ev_fork, &c->ev_join, &c->ev_out})
    if (!e) e = hip_err(hipEventCreateWithFlags(ev, hipEventDisableTiming));
  const double g = par->gamma;
  c->gas.g = g;
  c->gas.gm1 = g - 1.0;
  c->gas.e1 = (g - 1.0) / (2.0 * g);
  c->gas.ig = 1.0 / g;
  c->gas.e5 = 2.0 / (g - 1.0);
  c->gas.e7 = 2.0 * g / (g - 1.0);
  c->gas.mu = (g - 1.0) / (g + 1.0);
  c->gas.gp = 2.0 / (g + 1.0);
  c->gas.sk = (g + 1.0) / (2.0 * g);
  c->tol_nb = par->tol_nb;
  c->tol_k = par->tol_k;
  c->lmax = par->lmax;
  c->P = P;
  c->ncell = ncell;
  c->h_N.assign(b->N, b->N + P);
  c->h_off = off;
  if (!e) e = dalloc(&c->off, P + 1);
  if (!e) e = dalloc(&c->N, P);
  for (int** q : {&c->clipped, &c->status, &c->steps, &c->cnt, &c->fail})
    if (!e) e = dalloc(q, P);
  for (double** q : {&c->h, &c->alpha, &c->thnb, &c->thk, &c->cfl, &c->tend, &c->t, &c->dt,
                     &c->dtr})
    if (!e) e = dalloc(q, P);
  if (!e) e = dalloc(&c->iters, P);
  if (!e) e = dalloc(&c->S, P);
  for (int bb = 0; bb < 2; ++bb)
    for (int q = 0; q < 3; ++q)
      if (!e) e = dalloc(&c->U[bb][q], ncell);
  auto up = [&](void* d, const void* h, size_t bytes) {
    if (!e && bytes) e = hip_err(hipMemcpy(d, h, bytes, hipMemcpyHostToDevice));
  };
  up(c->off, off.data(), (P + 1) * sizeof(long long));
  up(c->N, b->N, P * sizeof(int));
  up(c->h, b->h, P * sizeof(double));
  up(c->alpha, b->alpha, P * sizeof(double));
  up(c->thnb, b->theta_nb, P * sizeof(double));
  up(c->thk, b->theta_k, P * sizeof(double));
  up(c->cfl, b->cfl, P * sizeof(double));
  up(c->tend, b->t_end, P * sizeof(double));
  if (!e) e = build_tiles(c);
  if (e) {
    release(c);
    delete c;
    return e;
  }
  *out = c;
  return 0;
}

int imexds_eu_set_state(imexds_eu_ctx* c, const double* rho, const double* mom,
                        const double* ene) {
  if (!c || (c->ncell && (!rho || !mom || !ene))) return IMEXDS_ERR_INVALID_ARG;
  int e = enter(c);
  const size_t bytes = (size_t)c->ncell * sizeof(double);
  c->cur = 0;
  const double* src[3] = {rho, mom, ene};
  for (int q = 0; q < 3; ++q)
    if (!e && bytes)
      e = hip_err(hipMemcpyAsync(c->U[0][q], src[q], bytes, hipMemcpyDeviceToDevice, c->ms));
  const size_t P = (size_t)c->P;
  if (!e) e = hip_err(hipMemsetAsync(c->t, 0, P * sizeof(double), c->ms));
  if (!e) e = hip_err(hipMemsetAsync(c->dt, 0, P * sizeof(double), c->ms));
  if (!e) e = hip_err(hipMemsetAsync(c->dtr, 0, P * sizeof(double), c->ms));
  for (int* q : {c->clipped, c->status, c->steps, c->cnt, c->fail})
    if (!e) e = hip_err(hipMemsetAsync(q, 0, P * sizeof(int), c->ms));
  if (!e) e = hip_err(hipMemsetAsync(c->iters, 0, P * sizeof(long long), c->ms));
  if (!e) e = hip_err(hipMemsetAsync(c->S, 0, P * sizeof(unsigned long long), c->ms));
  eu::Args A = make_args(c, 0);
  if (!e && c->n_tiles) {
    eu::k_eu_cfl<<<c->n_tiles, 256, 0, c->ms>>>(A, 0);
    e = hip_err(hipGetLastError());
  }
  if (!e) e = hip_err(launch_fin(A, 1, c->ms));
  c->log_row = 0;
  if (!e) e = leave(c);
  c->have_state = e == 0;
  return e;
}

int imexds_eu_step(imexds_eu_ctx* c, int32_t n_steps) {
  if (!c || n_steps < 0) return IMEXDS_ERR_INVALID_ARG;
  if (!c->have_state) return IMEXDS_ERR_NO_STATE;
  int e = enter(c);
  for (int i = 0; i < n_steps && !e; ++i) e = one_step(c);
  if (!e) e = leave(c);
  return e;
}

int imexds_eu_step_per_problem(imexds_eu_ctx* c, int32_t n_steps) {
  if (!c || n_steps < 0) return IMEXDS_ERR_INVALID_ARG;
  if (!c->have_state) return IMEXDS_ERR_NO_STATE;
  int e = enter(c);
  for (int i = 0; i < n_steps && !e; ++i) e = one_step_per_problem(c);
  if (!e) e = leave(c);
  return e;
}

int imexds_eu_run(imexds_eu_ctx* c, int32_t max_steps, int32_t check_every,
                  int32_t* steps_done) {
  if (!c || max_steps < 0 || check_every <= 0) return IMEXDS_ERR_INVALID_ARG;
  if (!c->have_state) return IMEXDS_ERR_NO_STATE;
  int done = 0, e = 0;
  std::vector<double> t(c->P), te(c->P);
  std::vector<int> st(c->P);
  if (c->P)
    e = hip_err(hipMemcpy(te.data(), c->tend, c->P * sizeof(double), hipMemcpyDeviceToHost));
  while (!e && done < max_steps) {
    const int n = std::min(check_every, max_steps - done);
    e = imexds_eu_step(c, n);
    if (e) break;
    done += n;
    e = imexds_eu_get_problems(c, t.data(), st.data(), nullptr, nullptr);
    bool active = false;
    for (int p = 0; p < c->P && !e; ++p) active = active || (st[p] == 0 && t[p] < te[p]);
    if (!active) break;
  }
  if (steps_done) *steps_done = done;
  return e;
}

int imexds_eu_get_state(imexds_eu_ctx* c, double* rho, double* mom, double* ene) {
  if (!c || (c->ncell && (!rho || !mom || !ene))) return IMEXDS_ERR_INVALID_ARG;
  if (!c->have_state) return IMEXDS_ERR_NO_STATE;
  int e = enter(c);
  double* dst[3] = {rho, mom, ene};
  const size_t bytes = (size_t)c->ncell * sizeof(double);
  for (int q = 0; q < 3; ++q)
    if (!e && bytes)
      e = hip_err(hipMemcpyAsync(dst[q], c->U[c->cur][q], bytes, hipMemcpyDeviceToDevice, c->ms));
  if (!e) e = leave(c);
  return e;
}

int imexds_eu_get_problems(imexds_eu_ctx* c, double* t, int32_t* status, int32_t* steps,
                           int64_t* iters) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  if (!c->have_state) return IMEXDS_ERR_NO_STATE;
  int e = enter(c);
  if (!e) e = hip_err(hipStreamSynchronize(c->ms));
  const size_t P = (size_t)c->P;
  if (P) {
    if (!e && t) e = hip_err(hipMemcpy(t, c->t, P * sizeof(double), hipMemcpyDeviceToHost));
    if (!e && status)
      e = hip_err(hipMemcpy(status, c->status, P * sizeof(int), hipMemcpyDeviceToHost));
    if (!e && steps)
      e = hip_err(hipMemcpy(steps, c->steps, P * sizeof(int), hipMemcpyDeviceToHost));
    if (!e && iters)
      e = hip_err(hipMemcpy(iters, c->iters, P * sizeof(long long), hipMemcpyDeviceToHost));
  }
  return e;
}

int imexds_eu_enable_log(imexds_eu_ctx* c, int32_t max_steps) {
  if (!c || max_steps < 0) return IMEXDS_ERR_INVALID_ARG;
  int e = hip_err(hipSetDevice(c->device));
  if (!e) e = hip_err(hipStreamSynchronize(c->ms));
  dfree(c->log_cnt);
  dfree(c->log_fl);
  c->log_max = 0;
  c->log_row = 0;
  if (e || max_steps == 0) return e;
  const size_t n = (size_t)max_steps * (size_t)std::max(c->P, 1);
  e = dalloc(&c->log_cnt, n);
  if (!e) e = dalloc(&c->log_fl, n);
  if (!e) e = hip_err(hipMemset(c->log_cnt, 0, n * sizeof(int)));
  if (!e) e = hip_err(hipMemset(c->log_fl, 0, n * sizeof(int)));
  if (e) {
    dfree(c->log_cnt);
    dfree(c->log_fl);
    return e;
  }
  c->log_max = max_steps;
  return 0;
}

int imexds_eu_get_log(imexds_eu_ctx* c, int32_t* count, int32_t* flags, int32_t* rows) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  int e = hip_err(hipSetDevice(c->device));
  if (!e) e = hip_err(hipStreamSynchronize(c->ms));
  const int r = std::min(c->log_row, c->log_max);
  if (rows) *rows = r;
  const size_t n = (size_t)r * (size_t)c->P;
  if (!e && n && count)
    e = hip_err(hipMemcpy(count, c->log_cnt, n * sizeof(int), hipMemcpyDeviceToHost));
  if (!e && n && flags)
    e = hip_err(hipMemcpy(flags, c->log_fl, n * sizeof(int), hipMemcpyDeviceToHost));
  return e;
}

int imexds_eu_set_launch(imexds_eu_ctx* c, int32_t tile_cells, int32_t zone_lanes,
                         int32_t zone_problems_per_wave) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  if (tile_cells != 256 && tile_cells != 512 && tile_cells != 1024)
    return IMEXDS_ERR_INVALID_ARG;
  if (zone_lanes != 1 && zone_lanes != 2) return IMEXDS_ERR_INVALID_ARG;
  if (zone_problems_per_wave < 1 || zone_problems_per_wave * zone_lanes > 64)
    return IMEXDS_ERR_INVALID_ARG;
  int e = hip_err(hipSetDevice(c->device));
  if (!e) e = hip_err(hipStreamSynchronize(c->ms));
  if (e) return e;
  c->zone_lanes = zone_lanes;
  c->zone_ppw = zone_problems_per_wave;
  if (tile_cells != c->tile_class) {
    c->tile_class = tile_cells;
    e = build_tiles(c);
  }
  return e;
}

int imexds_eu_get_sizes(imexds_eu_ctx* c, int32_t* n_problems, int64_t* n_cells) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  if (n_problems) *n_problems = c->P;
  if (n_cells) *n_cells = c->ncell;
  return 0;
}

int imexds_eu_time_kernels(imexds_eu_ctx* c, int32_t on) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  int e = hip_err(hipSetDevice(c->device));
  if (!e) e = hip_err(hipStreamSynchronize(c->ms));
  c->timing = on != 0;
  c->timed_steps = 0;
  return e;
}

int imexds_eu_last_timing(imexds_eu_ctx* c, double* bulk_ms, double* zone_ms, double* step_ms) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  int e = hip_err(hipSetDevice(c->device));
  if (!e) e = hip_err(hipStreamSynchronize(c->ms));
  if (!e) e = hip_err(hipStreamSynchronize(c->zs));
  double sb = 0, sz = 0, ss = 0;
  const int n = c->timed_steps;
  for (int i = 0; i < n && !e; ++i) {
    float a = 0, bz = 0, s = 0;
    e = hip_err(hipEventElapsedTime(&a, c->tev[6 * i + 1], c->tev[6 * i + 2]));
    if (!e) e = hip_err(hipEventElapsedTime(&bz, c->tev[6 * i + 3], c->tev[6 * i + 4]));
    if (!e) e = hip_err(hipEventElapsedTime(&s, c->tev[6 * i], c->tev[6 * i + 5]));
    sb += a;
    sz += bz;
    ss += s;
  }
  const double d = n > 0 ? (double)n : 1.0;
  if (bulk_ms) *bulk_ms = sb / d;
  if (zone_ms) *zone_ms = sz / d;
  if (step_ms) *step_ms = ss / d;
  return e;
}

void imexds_eu_destroy(imexds_eu_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->ms) (void)hipStreamSynchronize(c->ms);
  if (c->zs) (void)hipStreamSynchronize(c->zs);
  release(c);
  delete c;
}

}  // extern "C"
