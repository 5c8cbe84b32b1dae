// ctube.hip -- creation tubes: phase creation inside the mesh of the
// isothermal two-phase scheme (appendix "Phase Creation", step (iv), and the
// two phase boundaries of the following steps: Algorithms 1 and 2), kernels
// and the host runtime behind include/imexds_ctube.h.
//
// A tube has N regular cells of one phase; slot N holds the cell created on
// face j (between cells j-1 and j).  Kernels, one step of every tube:
//   k_ct_detect (tiles of cells): step (i) on every inner face of the tubes
//                                 that have no created cell yet; a creating
//                                 face is recorded (atomic min, count).
//   k_ct_bulk   (tiles of cells): Algorithm 1 Step 1, HLL fluxes and the
//                                 explicit update of every cell outside the
//                                 implicit range (the zone, or the two
//                                 neighbours of a creating face); epilogue:
//                                 max(|u| + a) of the new state per tube and
//                                 failure bits, one atomic per wave each.
//   k_ct_create (lane per tube)  : the creation step (step (ii) on the face,
//                                 the neighbours, the new cell).
//   k_ct_zone   (1, 2 or 4 lanes per tube): Algorithm 2 on the created
//                                 cell +- Z cells with both phase boundaries
//                                 solved by the interface solver (2 lanes:
//                                 one per boundary, side by side; 4: two per
//                                 boundary, one per side of its problem).
//   k_ct_newton (7 groups of 1, 2 or 4 lanes per tube): instead of
//                                 k_ct_zone when the zone is solved by
//                                 Newton (zone +- 1).
//   k_ct_fin    (lane per tube)  : t, steps, status, the mesh check and the
//                                 next dt.
// k_ct_bulk and k_ct_create + k_ct_zone read U^n only and write disjoint
// slots of U^{n+1}, so they run concurrently on two streams.
//
// Every expression is evaluated in the order written (-ffp-contract=off):
// results are bitwise those of any IEEE FP64 evaluation of the same
// expressions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <new>
#include <vector>

#include "../../include/imexds_ctube.h"
#include "creation_device.hpp"
#include "imexds_device.hpp"

namespace ct {

using imexds::d_a;
using imexds::d_bflux;
using imexds::d_finite;
using imexds::d_hll;
using imexds::d_state_ok;
using imexds::IfaceOut;
using imexds::Mat;

constexpr int ST_NEWTON = IMEXDS_CT_ST_NEWTON, ST_NONPHYS = IMEXDS_CT_ST_NONPHYS,
              ST_MESH = IMEXDS_CT_ST_MESH, ST_MULTI = IMEXDS_CT_ST_MULTI;
constexpr int FL_CREATED = IMEXDS_CT_FL_CREATED, FL_LMAX = IMEXDS_CT_FL_LMAX,
              FL_INACTIVE = IMEXDS_CT_FL_INACTIVE;
constexpr int TILE = 256;  // cells per workgroup of the sweep and the detection
constexpr unsigned long long NAN_BITS = 0x7FF8000000000000ull;

struct Args {
  Mat M;
  double cfl, theta_nb, tol_nb, tol_tiny, tol_rel, t_end, newton_rtol, p_min, p_tilde;
  int tol_mode, lmax, Z, bc_left, bc_right, newton_maxit;
  int P;
  const long long* off;  // [P] first slot of the tube
  const int* N;
  const double* h;
  const int* phase;
  const int* tile_prob;
  const int* tile_start;
  const double *r0, *m0;  // U^n
  double *r1, *m1;        // U^{n+1}
  int* face;              // created cell's face (-1: none)
  double *dl, *dr;        // its boundaries relative to that face
  double* pw;             // [4P] warm starts of the two boundaries
  double* t;
  double* dt;
  int* clipped;
  int* status;
  int* steps;
  long long* iters;
  int* cnt;                // dual time iterations of this step
  int* fail;               // failure bits of this step
  unsigned long long* S;   // bit pattern of max(|u| + a) of the new state
  int* cface;              // smallest creating face of this step (INT_MAX: none)
  int* ccount;             // creating faces of this step
  int* log_cnt;
  int* log_fl;
  int log_row;
  int zone_ppw;
  int zn_maxit;     // Newton zone solver: at most this many steps
  double zn_rtol;   // and this relative step tolerance
};

__device__ __forceinline__ unsigned long long speed_bits(const Mat& M, int ph, double r,
                                                         double m) {
  if (!d_state_ok(r, m)) return NAN_BITS;
  return (unsigned long long)__double_as_longlong(fabs(m / r) + d_a(M, ph));
}

__device__ __forceinline__ unsigned long long wave_max(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// flux on the regular face j of a tube (0 and N: the domain ends)
__device__ __forceinline__ void face_flux(const Args& A, int ph, int N, const double* r,
                                          const double* m, int j, double& F0, double& F1) {
  if (j == 0)
    d_bflux(A.M, ph, false, A.bc_left, r[0], m[0], F0, F1);
  else if (j == N)
    d_bflux(A.M, ph, true, A.bc_right, r[N - 1], m[N - 1], F0, F1);
  else
    d_hll(A.M, ph, r[j - 1], m[j - 1], r[j], m[j], F0, F1);
}

// cells [a, b) left to k_ct_zone this step; a = b = N: none
__device__ __forceinline__ void implicit_range(const Args& A, int p, int N, int& a, int& b) {
  const int j0 = A.face[p];
  a = N;
  b = N;
  if (j0 >= 0) {
    a = j0 - A.Z;
    b = j0 + A.Z;
  } else if (A.ccount[p] == 1) {
    a = A.cface[p] - 1;
    b = A.cface[p] + 1;
  }
  a = a < 0 ? 0 : a;
  b = b > N ? N : b;
}

// length of a zone cell with the left boundary moving at wl and the right
// one at wr: kind 1 left neighbour, 2 created cell, 3 right neighbour
__device__ __forceinline__ double cell_len(double hn, int kind, double wl, double wr, double dt) {
  if (kind == 1) return hn + wl * dt;
  if (kind == 2) return hn + (wr - wl) * dt;
  if (kind == 3) return hn - wr * dt;
  return hn;
}

// ---------------------------------------------------------------------------
// step (i) on the inner faces of tubes without a created cell
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TILE) void k_ct_detect(Args A, int tile_begin) {
  const int tile = tile_begin + (int)blockIdx.x;
  const int p = A.tile_prob[tile];
  if (A.dt[p] == 0.0 || A.face[p] >= 0) return;  // uniform over the workgroup
  const int j = A.tile_start[tile] + (int)threadIdx.x;  // face between cells j-1 and j
  const int N = A.N[p];
  if (j < 1 || j >= N) return;
  const long long o = A.off[p];
  double p1;
  if (imexds::c_creates(A.M, A.phase[p], A.r0[o + j - 1], A.m0[o + j - 1], A.r0[o + j],
                        A.m0[o + j], A.p_min, A.p_tilde, p1)) {
    atomicMin(A.cface + p, j);
    atomicAdd(A.ccount + p, 1);
  }
}

// ---------------------------------------------------------------------------
// explicit sweep: one lane per cell, both faces by HLL
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TILE) void k_ct_bulk(Args A, int tile_begin) {
  const int tile = tile_begin + (int)blockIdx.x;
  const int p = A.tile_prob[tile];
  const int N = A.N[p];
  const int s = A.tile_start[tile] + (int)threadIdx.x;
  const long long o = A.off[p];
  const double* __restrict__ r0 = A.r0 + o;
  const double* __restrict__ m0 = A.m0 + o;
  double* __restrict__ r1 = A.r1 + o;
  double* __restrict__ m1 = A.m1 + o;
  const double dt = A.dt[p];
  int a, b;
  implicit_range(A, p, N, a, b);
  const bool mine = s < N && (s < a || s >= b);
  if (dt == 0.0) {  // frozen or finished: carry the state over
    if (mine) {
      r1[s] = r0[s];
      m1[s] = m0[s];
    }
    return;
  }
  const int ph = A.phase[p];
  const double lam = dt / A.h[p];
  unsigned long long v = 0;
  if (mine) {
    double FL0, FL1, FR0, FR1;
    face_flux(A, ph, N, r0, m0, s, FL0, FL1);
    face_flux(A, ph, N, r0, m0, s + 1, FR0, FR1);
    const double rn = r0[s] - lam * (FR0 - FL0);
    const double mn = m0[s] - lam * (FR1 - FL1);
    r1[s] = rn;
    m1[s] = mn;
    v = speed_bits(A.M, ph, rn, mn);
  }
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0 && v) atomicMax(A.S + p, v);
}

// CFL bound of the initial state
__global__ __launch_bounds__(TILE) void k_ct_cfl(Args A) {
  const int tile = blockIdx.x;
  const int p = A.tile_prob[tile];
  const int s = A.tile_start[tile] + (int)threadIdx.x;
  const long long o = A.off[p];
  unsigned long long v = 0;
  if (s < A.N[p]) v = speed_bits(A.M, A.phase[p], A.r0[o + s], A.m0[o + s]);
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0 && v) atomicMax(A.S + p, v);
}

// ---------------------------------------------------------------------------
// the creation step (steps (ii), (iii), (v) on the creating face, step (iv)),
// a lane per tube; the tubes with more than one creating face fail here
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_ct_create(Args A) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= A.P) return;
  const double dt = A.dt[p];
  const int cc = A.ccount[p];
  if (dt == 0.0 || A.face[p] >= 0 || cc == 0) return;  // k_ct_zone's tubes
  const long long lrow = A.log_row >= 0 ? (long long)A.log_row * A.P + p : -1;
  int code = 0, fl = 0;
  if (cc > 1) {
    code = ST_MULTI;
  } else {
    const Mat& M = A.M;
    const long long o = A.off[p];
    const int N = A.N[p];
    const double* __restrict__ r0 = A.r0 + o;
    const double* __restrict__ m0 = A.m0 + o;
    double* __restrict__ r1 = A.r1 + o;
    double* __restrict__ m1 = A.m1 + o;
    const int ph = A.phase[p], phn = 1 - ph;
    const double h = A.h[p];
    const int jc = A.cface[p];
    double C[IMEXDS_CR_FIELDS];
#pragma unroll
    for (int i = 0; i < IMEXDS_CR_FIELDS; ++i) C[i] = 0.0;
    if (imexds::c_solve(M, ph, r0[jc - 1], m0[jc - 1], r0[jc], m0[jc], A.newton_maxit,
                        A.newton_rtol, C) != 1) {
      code = ST_NEWTON;
    } else {
      const double wl = C[IMEXDS_CR_WL], wr = C[IMEXDS_CR_WR];
      const double h1l = h + wl * dt, h1r = h - wr * dt;
      const double ndl = wl * dt, ndr = wr * dt;
      if (!(h1l > 0.0) || !(h1r > 0.0) || !(ndr - ndl > 0.0)) {
        code = ST_MESH;
      } else {
        double F0, F1, G0, G1;
        face_flux(A, ph, N, r0, m0, jc - 1, F0, F1);
        face_flux(A, ph, N, r0, m0, jc + 1, G0, G1);
        const double il = 1.0 / h1l, ir = 1.0 / h1r;
        const double ra = (h * r0[jc - 1] - dt * (C[IMEXDS_CR_FL0] - F0)) * il;
        const double ma = (h * m0[jc - 1] - dt * (C[IMEXDS_CR_FL1] - F1)) * il;
        const double rc = (h * r0[jc] - dt * (G0 - C[IMEXDS_CR_FR0])) * ir;
        const double mc = (h * m0[jc] - dt * (G1 - C[IMEXDS_CR_FR1])) * ir;
        const double rb = C[IMEXDS_CR_RB], mb = C[IMEXDS_CR_RB] * C[IMEXDS_CR_UB];
        r1[jc - 1] = ra;
        m1[jc - 1] = ma;
        r1[jc] = rc;
        m1[jc] = mc;
        r1[N] = rb;
        m1[N] = mb;
        if (!d_state_ok(ra, ma) || !d_state_ok(rc, mc) || !d_state_ok(rb, mb)) {
          code = ST_NONPHYS;
        } else {
          A.dl[p] = ndl;
          A.dr[p] = ndr;
          double* pw = A.pw + 4 * (long long)p;
          pw[0] = C[IMEXDS_CR_PA];
          pw[1] = C[IMEXDS_CR_PB];
          pw[2] = C[IMEXDS_CR_PB];
          pw[3] = C[IMEXDS_CR_PC];
          const unsigned long long va = speed_bits(M, ph, ra, ma);
          const unsigned long long vc = speed_bits(M, ph, rc, mc);
          const unsigned long long vb = speed_bits(M, phn, rb, mb);
          unsigned long long v = va > vc ? va : vc;
          v = vb > v ? vb : v;
          atomicMax(A.S + p, v);
        }
        fl = FL_CREATED;
      }
    }
  }
  if (code) atomicOr(A.fail + p, code);
  A.cnt[p] = 0;
  if (lrow >= 0) {
    A.log_cnt[lrow] = 0;
    A.log_fl[lrow] = fl;
  }
}

// ---------------------------------------------------------------------------
// Algorithm 2 on the created cell +- Z cells (and the carry-over of frozen
// tubes).  L lanes per tube; with L = 2 lane `side` solves boundary `side`
// (0 left, 1 right) and the two swap fluxes and speeds, so both hold the same
// iterates and take every branch together.  Pass -1 of the loop is the
// explicit prediction of the boundary speeds from U^n, passes 0 .. are the
// pseudo steps, and the pass after the last one (stopped, or l = lmax)
// evaluates the fluxes of the accepted iterate for Part 2: one call site of
// the interface solver.
// ---------------------------------------------------------------------------
template <int Z, int L>
__global__ __launch_bounds__(64) void k_ct_zone(Args A) {
  constexpr int MC = 2 * Z + 1;
  constexpr int XB = L == 4 ? 2 : 1;  // lane distance between the two boundaries' lanes
  const int lane = (int)threadIdx.x;
  if (lane >= A.zone_ppw * L) return;
  const int p = blockIdx.x * A.zone_ppw + lane / L;
  const int sub = lane & (L - 1);
  const int side = L == 4 ? (sub >> 1) : sub;  // the boundary this lane solves (L = 1: both)
  const int half = L == 4 ? (sub & 1) : 0;     // L = 4: the side of that boundary's problem
  if (p >= A.P) return;  // the lanes of a tube are whole
  const bool writer = sub == 0;
  const long long o = A.off[p];
  const int N = A.N[p];
  const double* __restrict__ r0 = A.r0 + o;
  const double* __restrict__ m0 = A.m0 + o;
  double* __restrict__ r1 = A.r1 + o;
  double* __restrict__ m1 = A.m1 + o;
  const double dt = A.dt[p];
  const long long lrow = A.log_row >= 0 ? (long long)A.log_row * A.P + p : -1;
  const int j0 = A.face[p];
  if (dt == 0.0 || j0 < 0) {
    if (dt != 0.0 && A.ccount[p] != 0) return;  // k_ct_create's tubes
    if (writer) {
      if (dt == 0.0) {
        int a, b;
        implicit_range(A, p, N, a, b);
        for (int c = a; c < b; ++c) {
          r1[c] = r0[c];
          m1[c] = m0[c];
        }
      }
      // the created slot, unused or frozen, is carried over
      r1[N] = r0[N];
      m1[N] = m0[N];
      if (dt != 0.0) A.cnt[p] = 0;
      if (lrow >= 0) {
        A.log_cnt[lrow] = 0;
        A.log_fl[lrow] = dt == 0.0 ? FL_INACTIVE : 0;
      }
    }
    return;
  }
  const Mat& M = A.M;
  const int ph = A.phase[p], phn = 1 - ph;
  const double h = A.h[p];
  int code = 0, cnt = 0, fl = 0;
  const double dl = A.dl[p], dr = A.dr[p];
  double* pwp = A.pw + 4 * (long long)p;
  double U0[MC][2], hn[MC], hh[MC], th[MC], i1t[MC], thr[MC], W[MC][2];
  int kind[MC];
#pragma unroll
  for (int k = 0; k < MC; ++k) {
    const int sl = k < Z ? j0 - Z + k : (k == Z ? N : j0 + (k - Z - 1));
    U0[k][0] = r0[sl];
    U0[k][1] = m0[sl];
    W[k][0] = U0[k][0];
    W[k][1] = U0[k][1];
    kind[k] = k == Z - 1 ? 1 : (k == Z ? 2 : (k == Z + 1 ? 3 : 0));
    hn[k] = k == Z - 1 ? h + dl : (k == Z ? dr - dl : (k == Z + 1 ? h - dr : h));
    hh[k] = hn[k];
    th[k] = 0.0;
    i1t[k] = 1.0;
    thr[k] = 0.0;
  }
  double F[MC + 1][2];
  face_flux(A, ph, N, r0, m0, j0 - Z, F[0][0], F[0][1]);
  face_flux(A, ph, N, r0, m0, j0 + Z, F[MC][0], F[MC][1]);
  // boundary speeds and warm starts (pl0, pl1) of the left boundary,
  // (pr0, pr1) of the right one
  double wl = 0.0, wr = 0.0;
  double pl0 = pwp[0], pl1 = pwp[1], pr0 = pwp[2], pr1 = pwp[3];
  bool stop = false;
#pragma unroll 1
  for (int l = -1;; ++l) {
    const bool part2 = l >= 0 && (stop || l == A.lmax);
    // the two phase boundaries at the current iterate (pass -1: U^n = W)
    int ec = 0;
    double bl0 = 0.0, bl1 = 0.0, br0 = 0.0, br1 = 0.0;
#pragma unroll 1
    for (int f = side; f < 2; f += (L == 1 ? 1 : 2)) {
      const bool lf = f == 0;
      IfaceOut I;
      // L = 4: the two lanes of a boundary split its problem by side
      if (!imexds::d_iface_solve_t<L == 4>(M, A.newton_maxit, A.newton_rtol, lf ? ph : phn,
                                           lf ? W[Z - 1][0] : W[Z][0], lf ? W[Z - 1][1] : W[Z][1],
                                           lf ? phn : ph, lf ? W[Z][0] : W[Z + 1][0],
                                           lf ? W[Z][1] : W[Z + 1][1], true, lf ? pl0 : pr0,
                                           lf ? pl1 : pr1, half, I)) {
        ec = 1;
      } else if (lf) {
        wl = I.w;
        pl0 = I.pl;
        pl1 = I.pr;
        bl0 = I.F0;
        bl1 = I.F1;
      } else {
        wr = I.w;
        pr0 = I.pl;
        pr1 = I.pr;
        br0 = I.F0;
        br1 = I.F1;
      }
    }
    if (L > 1) {
      const double y0 = __shfl_xor(side ? br0 : bl0, XB, 64);
      const double y1 = __shfl_xor(side ? br1 : bl1, XB, 64);
      const double yw = __shfl_xor(side ? wr : wl, XB, 64);
      ec |= __shfl_xor(ec, XB, 64);
      if (side) {
        bl0 = y0;
        bl1 = y1;
        wl = yw;
      } else {
        br0 = y0;
        br1 = y1;
        wr = yw;
      }
    }
    if (ec) {
      code = ST_NEWTON;
      break;
    }
    if (l < 0) {
      // predicted end-of-step lengths and the pseudo step fractions
#pragma unroll
      for (int k = 0; k < MC; ++k) {
        const double hk = cell_len(hn[k], kind[k], wl, wr, dt);
        double t = hk / h;
        if (t > A.theta_nb) t = A.theta_nb;
        hh[k] = hk;
        th[k] = t;
        i1t[k] = 1.0 / (1.0 + t);
        thr[k] = (k == Z ? A.tol_tiny : A.tol_nb) * (t * dt);
        if (!(t > 0.0)) code = ST_MESH;
      }
      if (code) break;
      continue;
    }
    F[Z][0] = bl0;
    F[Z][1] = bl1;
    F[Z + 1][0] = br0;
    F[Z + 1][1] = br1;
#pragma unroll
    for (int c = 0; c + 1 < MC; ++c)
      if (c != Z - 1 && c != Z)
        d_hll(M, ph, W[c][0], W[c][1], W[c + 1][0], W[c + 1][1], F[c + 1][0], F[c + 1][1]);
    double ih[MC];
    bool shrink = false;
#pragma unroll
    for (int k = 0; k < MC; ++k) {
      const double hk = cell_len(hn[k], kind[k], wl, wr, dt);
      ih[k] = 1.0 / hk;
      if (kind[k] != 0 && !(hk >= 0.5 * hh[k])) shrink = true;
    }
    if (shrink) {
      code = ST_MESH;
      break;
    }
    if (part2) {
      // Part 2: conservative update with the fluxes of the accepted iterate
#pragma unroll
      for (int k = 0; k < MC; ++k) {
        const double u0 = (hn[k] * U0[k][0] - dt * (F[k + 1][0] - F[k][0])) * ih[k];
        const double u1 = (hn[k] * U0[k][1] - dt * (F[k + 1][1] - F[k][1])) * ih[k];
        W[k][0] = u0;
        W[k][1] = u1;
        if (!d_state_ok(u0, u1)) code = ST_NONPHYS;
      }
      break;
    }
    bool conv = true, okst = true;
#pragma unroll
    for (int k = 0; k < MC; ++k) {
      const double opt = 1.0 + th[k];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const double rhs = (hn[k] * U0[k][q] - dt * (F[k + 1][q] - F[k][q])) * ih[k];
        const double wn = (W[k][q] + th[k] * rhs) * i1t[k];
        const double d = wn - W[k][q];
        const double sc = fabs(W[k][q]) > 1.0 ? fabs(W[k][q]) : 1.0;
        const bool ok = A.tol_mode == 0 ? (fabs(opt * d) < thr[k] * sc)
                                        : (fabs(d) < A.tol_rel * sc);
        conv = conv && ok;
        W[k][q] = wn;
      }
      okst = okst && d_state_ok(W[k][0], W[k][1]);
    }
    if (!okst) {
      code = ST_NONPHYS;
      break;
    }
    cnt = l + 1;
    stop = conv;
  }
  if (!code && !stop) fl |= FL_LMAX;
  if (L > 1) {
    // the writer takes the right boundary's warm start from its partner
    const double q0 = __shfl_xor(pr0, XB, 64), q1 = __shfl_xor(pr1, XB, 64);
    if (side == 0) {
      pr0 = q0;
      pr1 = q1;
    }
  }
  if (writer) {
    unsigned long long vmax = 0;
    if (!code) {
#pragma unroll
      for (int k = 0; k < MC; ++k) {
        const int sl = k < Z ? j0 - Z + k : (k == Z ? N : j0 + (k - Z - 1));
        r1[sl] = W[k][0];
        m1[sl] = W[k][1];
        const unsigned long long v = speed_bits(M, k == Z ? phn : ph, W[k][0], W[k][1]);
        vmax = v > vmax ? v : vmax;
      }
      A.dl[p] = dl + wl * dt;
      A.dr[p] = dr + wr * dt;
      pwp[0] = pl0;
      pwp[1] = pl1;
      pwp[2] = pr0;
      pwp[3] = pr1;
      atomicMax(A.S + p, vmax);
    } else {
      atomicOr(A.fail + p, code);
    }
    A.cnt[p] = code ? 0 : cnt;
    if (lrow >= 0) {
      A.log_cnt[lrow] = code ? 0 : cnt;
      A.log_fl[lrow] = code ? 0 : fl;
    }
  }
}

// ---------------------------------------------------------------------------
// Newton on the implicit step of the zone (created cell +- Z), the
// alternative to Algorithm 2 (the paper's outlook: a Newton-like solver for
// the small implicit systems).  Unknowns: the 2 (2 Z + 1) values of the
// zone's cells; residual
//   R_c(W) = (h_c(W) / h_c^n) W_c - U_c^n + (dt / h_c^n)(F_{c+1/2}(W) - F_{c-1/2}(W)),
// (the lengths of the created cell and its two neighbours from the boundary
// speeds at W, HLL on the other inner faces, the zone's outer faces from
// U^n); Jacobian by forward differences (step 1e-7 max(|W_j|, 1), boundary
// solves warm-started from the base point's) of which the 2x2 blocks beside
// the diagonal are kept (each row couples its two neighbours only), the
// block Thomas algorithm, full steps from W = U^n, converged when every step
// component is below zn_rtol max(|W_j|, 1); at most zn_maxit steps.
// A tube has 1 + 2 (2 Z + 1) groups of L lanes (L = 1, 2, 4 as in
// k_ct_zone).  Every group evaluates the prediction and each base point
// (identical inputs and warm starts, so identical results without any
// exchange); then group g >= 1 evaluates the point moved along unknown
// g - 1 -- the difference columns side by side -- and every lane gathers the
// blocks and runs the same block solve.  Per Newton step two evaluations in
// sequence instead of 1 + 2 (2 Z + 1).
// ---------------------------------------------------------------------------
template <int Z, int L>
__device__ __forceinline__ int newton_tubes_per_wave(int ppw) {
  const int cap = 64 / ((2 * (2 * Z + 1) + 1) * L);
  return ppw < cap ? ppw : cap;
}

template <int Z, int L>
__global__ __launch_bounds__(64) void k_ct_newton(Args A) {
  constexpr int MC = 2 * Z + 1, NV = 2 * MC, G = NV + 1, TL = G * L;
  constexpr int XB = L == 4 ? 2 : 1;
  const int tpw = newton_tubes_per_wave<Z, L>(A.zone_ppw);
  const int lane = (int)threadIdx.x;
  if (lane >= tpw * TL) return;
  const int p = blockIdx.x * tpw + lane / TL;
  const int tl = lane % TL;      // lane within the tube
  const int grp = tl / L;        // 0: base points only; g >= 1: column g - 1
  const int sub = tl % L;
  const int side = L == 4 ? (sub >> 1) : sub;
  const int half = L == 4 ? (sub & 1) : 0;
  const int lane0 = lane - tl;   // the tube's first lane
  if (p >= A.P) return;          // the lanes of a tube are whole
  const bool writer = tl == 0;
  const long long o = A.off[p];
  const int N = A.N[p];
  const double* __restrict__ r0 = A.r0 + o;
  const double* __restrict__ m0 = A.m0 + o;
  double* __restrict__ r1 = A.r1 + o;
  double* __restrict__ m1 = A.m1 + o;
  const double dt = A.dt[p];
  const long long lrow = A.log_row >= 0 ? (long long)A.log_row * A.P + p : -1;
  const int j0 = A.face[p];
  if (dt == 0.0 || j0 < 0) {
    if (dt != 0.0 && A.ccount[p] != 0) return;  // k_ct_create's tubes
    if (writer) {
      if (dt == 0.0) {
        int a, b;
        implicit_range(A, p, N, a, b);
        for (int c = a; c < b; ++c) {
          r1[c] = r0[c];
          m1[c] = m0[c];
        }
      }
      r1[N] = r0[N];
      m1[N] = m0[N];
      if (dt != 0.0) A.cnt[p] = 0;
      if (lrow >= 0) {
        A.log_cnt[lrow] = 0;
        A.log_fl[lrow] = dt == 0.0 ? FL_INACTIVE : 0;
      }
    }
    return;
  }
  const Mat& M = A.M;
  const int ph = A.phase[p], phn = 1 - ph;
  const double h = A.h[p];
  const double dl = A.dl[p], dr = A.dr[p];
  double* pwp = A.pw + 4 * (long long)p;
  // zone cells: j0 - Z .. j0 - 2 (kind 0), j0 - 1 (kind 1), the created cell
  // (kind 2), j0 (kind 3), j0 + 1 .. j0 + Z - 1 (kind 0)
  double U0[MC][2], W[MC][2], hn[MC], ihn[MC], hh[MC];
  int slot[MC], kind[MC];
#pragma unroll
  for (int k = 0; k < MC; ++k) {
    slot[k] = k < Z ? j0 - Z + k : (k == Z ? N : j0 + (k - Z - 1));
    kind[k] = k == Z - 1 ? 1 : (k == Z ? 2 : (k == Z + 1 ? 3 : 0));
    hn[k] = k == Z - 1 ? h + dl : (k == Z ? dr - dl : (k == Z + 1 ? h - dr : h));
  }
#pragma unroll
  for (int k = 0; k < MC; ++k) {
    U0[k][0] = r0[slot[k]];
    U0[k][1] = m0[slot[k]];
    W[k][0] = U0[k][0];
    W[k][1] = U0[k][1];
    ihn[k] = 1.0 / hn[k];
    hh[k] = hn[k];
  }
  double FL0, FL1, FR0, FR1;
  face_flux(A, ph, N, r0, m0, j0 - Z, FL0, FL1);
  face_flux(A, ph, N, r0, m0, j0 + Z, FR0, FR1);
  double wl = 0.0, wr = 0.0;
  double pl0 = pwp[0], pl1 = pwp[1], pr0 = pwp[2], pr1 = pwp[3];  // current warm starts
  double gl0 = 0.0, gl1 = 0.0, gr0 = 0.0, gr1 = 0.0;              // the base point's
  double R[NV], Jc[NV];  // residual at the base point; this group's column
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    R[i] = 0.0;
    Jc[i] = 0.0;
  }
  const int colj = grp - 1;  // this group's unknown (groups >= 1)
  int code = 0, it = 0, phase = -2;  // -2: prediction, -1: base point, 0: columns
  double ecol = 0.0;
  bool final_pass = false, conv = false;
#pragma unroll 1
  for (;;) {
    const bool fd = phase == 0;
    const bool moved = fd && grp > 0;
    // the point: W, or (groups >= 1 in the column pass) W moved along colj
    double X[MC][2];
#pragma unroll
    for (int k = 0; k < MC; ++k)
#pragma unroll
      for (int q = 0; q < 2; ++q) X[k][q] = (moved && colj == 2 * k + q) ? W[k][q] + ecol : W[k][q];
    int ec = 0;
    double bl0 = 0.0, bl1 = 0.0, br0 = 0.0, br1 = 0.0, ewl = 0.0, ewr = 0.0;
    double npl0 = 0.0, npl1 = 0.0, npr0 = 0.0, npr1 = 0.0;
#pragma unroll 1
    for (int f = side; f < 2; f += (L == 1 ? 1 : 2)) {
      const bool lf = f == 0;
      IfaceOut I;
      const double g0 = fd ? (lf ? gl0 : gr0) : (lf ? pl0 : pr0);
      const double g1 = fd ? (lf ? gl1 : gr1) : (lf ? pl1 : pr1);
      if (!imexds::d_iface_solve_t<L == 4>(M, A.newton_maxit, A.newton_rtol, lf ? ph : phn,
                                           lf ? X[Z - 1][0] : X[Z][0], lf ? X[Z - 1][1] : X[Z][1],
                                           lf ? phn : ph, lf ? X[Z][0] : X[Z + 1][0],
                                           lf ? X[Z][1] : X[Z + 1][1], true, g0, g1, half, I)) {
        ec = 1;
      } else if (lf) {
        ewl = I.w;
        npl0 = I.pl;
        npl1 = I.pr;
        bl0 = I.F0;
        bl1 = I.F1;
      } else {
        ewr = I.w;
        npr0 = I.pl;
        npr1 = I.pr;
        br0 = I.F0;
        br1 = I.F1;
      }
    }
    if (L > 1) {
      const double y0 = __shfl_xor(side ? br0 : bl0, XB, 64);
      const double y1 = __shfl_xor(side ? br1 : bl1, XB, 64);
      const double yw = __shfl_xor(side ? ewr : ewl, XB, 64);
      const double q0 = __shfl_xor(side ? npr0 : npl0, XB, 64);
      const double q1 = __shfl_xor(side ? npr1 : npl1, XB, 64);
      ec |= __shfl_xor(ec, XB, 64);
      if (side) {
        bl0 = y0;
        bl1 = y1;
        ewl = yw;
        npl0 = q0;
        npl1 = q1;
      } else {
        br0 = y0;
        br1 = y1;
        ewr = yw;
        npr0 = q0;
        npr1 = q1;
      }
    }
    // a failed solve in any group of the tube fails the zone (group 0's
    // column-pass evaluation repeats the base point and cannot fail)
    const unsigned long long failm = __ballot(ec != 0);
    const unsigned long long tm = ((1ull << TL) - 1ull) << lane0;
    if (failm & tm) {
      code = ST_NEWTON;
      break;
    }
    if (!fd) {  // prediction and base points carry the warm starts on
      wl = ewl;
      wr = ewr;
      pl0 = npl0;
      pl1 = npl1;
      pr0 = npr0;
      pr1 = npr1;
    }
    if (phase == -2) {
      bool bad = false;
#pragma unroll
      for (int k = 0; k < MC; ++k) {
        hh[k] = cell_len(hn[k], kind[k], wl, wr, dt);
        if (!(hh[k] / h > 0.0)) bad = true;  // a predicted length that vanishes
      }
      if (bad) {
        code = ST_MESH;
        break;
      }
      phase = -1;
      continue;
    }
    // faces of the point: the zone's outer faces from U^n, the two phase
    // boundaries, HLL on the other inner faces
    double F[MC + 1][2];
    F[0][0] = FL0;
    F[0][1] = FL1;
    F[MC][0] = FR0;
    F[MC][1] = FR1;
    F[Z][0] = bl0;
    F[Z][1] = bl1;
    F[Z + 1][0] = br0;
    F[Z + 1][1] = br1;
#pragma unroll
    for (int c = 0; c + 1 < MC; ++c)
      if (c != Z - 1 && c != Z)
        d_hll(M, ph, X[c][0], X[c][1], X[c + 1][0], X[c + 1][1], F[c + 1][0], F[c + 1][1]);
    double hk[MC];
    bool shrink = false;
#pragma unroll
    for (int k = 0; k < MC; ++k) {
      hk[k] = cell_len(hn[k], kind[k], ewl, ewr, dt);
      if (!fd && !(hk[k] >= 0.5 * hh[k])) shrink = true;
    }
    if (shrink) {
      code = ST_MESH;
      break;
    }
    if (final_pass) {
      // Part 2: conservative update with the fluxes of the accepted iterate
#pragma unroll
      for (int k = 0; k < MC; ++k) {
        const double ih = 1.0 / hk[k];
        const double u0 = (hn[k] * U0[k][0] - dt * (F[k + 1][0] - F[k][0])) * ih;
        const double u1 = (hn[k] * U0[k][1] - dt * (F[k + 1][1] - F[k][1])) * ih;
        W[k][0] = u0;
        W[k][1] = u1;
        if (!d_state_ok(u0, u1)) code = ST_NONPHYS;
      }
      break;
    }
    double RX[NV];
#pragma unroll
    for (int k = 0; k < MC; ++k)
#pragma unroll
      for (int q = 0; q < 2; ++q)
        RX[2 * k + q] = (hk[k] * ihn[k]) * X[k][q] - U0[k][q] + (dt * ihn[k]) * (F[k + 1][q] - F[k][q]);
    if (!fd) {
#pragma unroll
      for (int i = 0; i < NV; ++i) R[i] = RX[i];
      gl0 = pl0;
      gl1 = pl1;
      gr0 = pr0;
      gr1 = pr1;
      // this group's column step
      double xj = 0.0;
#pragma unroll
      for (int k = 0; k < MC; ++k)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          if (2 * k + q == colj) xj = W[k][q];
      ecol = 1e-7 * (fabs(xj) > 1.0 ? fabs(xj) : 1.0);
      phase = 0;
      continue;
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) Jc[i] = (RX[i] - R[i]) / ecol;
    // block tridiagonal solve (block Thomas, the oracle's order of
    // operations): group j + 1 holds column j; cell k's blocks D_k, L_k and
    // U_{k-1} come from the groups of cells k, k - 1 and k
    double Ib[MC][2][2], rp[MC][2], Ub[MC][2][2], dx[MC][2], d[NV];
    bool sing = false;
#pragma unroll
    for (int k = 0; k < MC; ++k) {
      double Dp[2][2], rc[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        rc[a] = -R[2 * k + a];
#pragma unroll
        for (int c = 0; c < 2; ++c) Dp[a][c] = __shfl(Jc[2 * k + a], lane0 + (2 * k + c + 1) * L, 64);
      }
      if (k > 0) {
        double Lc[2][2], Lf[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            Lc[a][c] = __shfl(Jc[2 * k + a], lane0 + (2 * (k - 1) + c + 1) * L, 64);
            Ub[k - 1][a][c] = __shfl(Jc[2 * (k - 1) + a], lane0 + (2 * k + c + 1) * L, 64);
          }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            Lf[a][c] = Lc[a][0] * Ib[k - 1][0][c] + Lc[a][1] * Ib[k - 1][1][c];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
#pragma unroll
          for (int c = 0; c < 2; ++c)
            Dp[a][c] = Dp[a][c] - (Lf[a][0] * Ub[k - 1][0][c] + Lf[a][1] * Ub[k - 1][1][c]);
          rc[a] = rc[a] - (Lf[a][0] * rp[k - 1][0] + Lf[a][1] * rp[k - 1][1]);
        }
      }
      rp[k][0] = rc[0];
      rp[k][1] = rc[1];
      const double det = Dp[0][0] * Dp[1][1] - Dp[0][1] * Dp[1][0];
      const double id = 1.0 / det;
      if (!d_finite(id)) sing = true;
      Ib[k][0][0] = Dp[1][1] * id;
      Ib[k][0][1] = -Dp[0][1] * id;
      Ib[k][1][0] = -Dp[1][0] * id;
      Ib[k][1][1] = Dp[0][0] * id;
    }
#pragma unroll
    for (int k = MC - 1; k >= 0; --k) {
      double y[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        y[a] = k == MC - 1 ? rp[k][a]
                           : rp[k][a] - (Ub[k][a][0] * dx[k + 1][0] + Ub[k][a][1] * dx[k + 1][1]);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        dx[k][a] = Ib[k][a][0] * y[0] + Ib[k][a][1] * y[1];
        if (!d_finite(dx[k][a])) sing = true;
        d[2 * k + a] = dx[k][a];
      }
    }
    if (sing) {
      code = ST_NEWTON;
      break;
    }
    conv = true;
#pragma unroll
    for (int k = 0; k < MC; ++k)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const double sc = fabs(W[k][q]) > 1.0 ? fabs(W[k][q]) : 1.0;
        conv = conv && (fabs(d[2 * k + q]) <= A.zn_rtol * sc);
      }
    bool okst = true;
#pragma unroll
    for (int k = 0; k < MC; ++k) {
      W[k][0] = W[k][0] + d[2 * k];
      W[k][1] = W[k][1] + d[2 * k + 1];
      okst = okst && d_state_ok(W[k][0], W[k][1]);
    }
    if (!okst) {
      code = ST_NONPHYS;
      break;
    }
    it += 1;
    final_pass = conv || it == A.zn_maxit;
    phase = -1;
  }
  const int fl = (!code && !conv) ? FL_LMAX : 0;
  if (writer) {
    if (!code) {
      unsigned long long vmax = 0;
#pragma unroll
      for (int k = 0; k < MC; ++k) {
        r1[slot[k]] = W[k][0];
        m1[slot[k]] = W[k][1];
        const unsigned long long v = speed_bits(M, k == Z ? phn : ph, W[k][0], W[k][1]);
        vmax = v > vmax ? v : vmax;
      }
      A.dl[p] = dl + wl * dt;
      A.dr[p] = dr + wr * dt;
      pwp[0] = pl0;
      pwp[1] = pl1;
      pwp[2] = pr0;
      pwp[3] = pr1;
      atomicMax(A.S + p, vmax);
    } else {
      atomicOr(A.fail + p, code);
    }
    A.cnt[p] = code ? 0 : it;
    if (lrow >= 0) {
      A.log_cnt[lrow] = code ? 0 : it;
      A.log_fl[lrow] = code ? 0 : fl;
    }
  }
}

// ---------------------------------------------------------------------------
// per-tube bookkeeping between steps
// ---------------------------------------------------------------------------
__global__ void k_ct_fin(Args A, int init) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= A.P) return;
  double dt = A.dt[p];
  int st = A.status[p];
  double t = A.t[p];
  if (!init && dt > 0.0) {
    const int f = A.fail[p];
    if (f) {
      st |= f;
    } else {
      t = A.clipped[p] ? A.t_end : t + dt;
      A.steps[p] += 1;
      A.iters[p] += A.cnt[p];
      // a creation step succeeded: the created cell's face (set here, not
      // in k_ct_zone, because the sweep reads it during the step)
      if (A.face[p] < 0 && A.ccount[p] == 1) A.face[p] = A.cface[p];
    }
  }
  double ndt = 0.0;
  int clip = 0;
  if (st == 0 && t < A.t_end) {
    const int j0 = A.face[p];
    const double h = A.h[p];
    bool mesh_ok = true;
    if (j0 >= 0) {
      const double dl = A.dl[p], dr = A.dr[p];
      mesh_ok = (h + dl >= 0.5 * h) && (h - dr >= 0.5 * h) && (dr - dl > 0.0) &&
                j0 - A.Z >= 0 && j0 + A.Z <= A.N[p];
    }
    const double S = __longlong_as_double((long long)A.S[p]);
    if (!mesh_ok) {
      st |= ST_MESH;
    } else if (!(S > 0.0) || !__builtin_isfinite(S)) {
      st |= ST_NONPHYS;
    } else {
      ndt = (A.cfl * h) / S;
      const double rem = A.t_end - t;
      if (ndt >= rem) {
        ndt = rem;
        clip = 1;
      }
    }
  }
  A.dt[p] = st == 0 ? ndt : 0.0;
  A.t[p] = t;
  A.status[p] = st;
  A.clipped[p] = clip;
  A.S[p] = 0ull;
  A.fail[p] = 0;
  A.cnt[p] = 0;
  A.cface[p] = INT_MAX;
  A.ccount[p] = 0;
}

}  // namespace ct

// ===========================================================================
// host runtime
// ===========================================================================
struct imexds_ct_ctx {
  int device = 0;
  hipStream_t user = nullptr, ms = nullptr, zs = nullptr;
  hipEvent_t ev_in = nullptr, ev_fork = nullptr, ev_join = nullptr, ev_out = nullptr;
  ct::Args base{};  // material and parameters
  int P = 0;
  long long nslot = 0;
  std::vector<int> h_N;
  std::vector<int> h_tile_first;  // [P + 1] first tile of each tube
  // device
  long long* off = nullptr;
  int *N = nullptr, *phase = nullptr, *face = nullptr, *clipped = nullptr, *status = nullptr,
      *steps = nullptr, *cnt = nullptr, *fail = nullptr, *cface = nullptr, *ccount = nullptr;
  double *h = nullptr, *dl = nullptr, *dr = nullptr, *pw = nullptr, *t = nullptr, *dt = nullptr;
  long long* iters = nullptr;
  unsigned long long* S = nullptr;
  double* U[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  int cur = 0;
  int *tile_prob = nullptr, *tile_start = nullptr;
  int n_tiles = 0, zone_lanes = 4, zone_ppw = 2;
  int zone_solver = IMEXDS_CT_SOLVER_DTS, zn_maxit = 30;
  double zn_rtol = 1e-10;
  int *log_cnt = nullptr, *log_fl = nullptr;
  int log_max = 0, log_row = 0;
  bool have_state = false;
  bool timing = false;
  std::vector<hipEvent_t> tev;  // 6 per step: begin, bulk 0/1, zone 0/1, end
  int timed_steps = 0;
};

namespace {

constexpr int CT_TIMED_MAX = 4096;

template <class T>
int ct_alloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc((void**)p, n * sizeof(T)) == hipSuccess ? 0 : IMEXDS_ERR_OOM;
}

template <class T>
void ct_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

int ct_err(hipError_t e) { return e == hipSuccess ? 0 : IMEXDS_ERR_HIP; }

void ct_release(imexds_ct_ctx* c) {
  ct_free(c->off);
  for (int** q : {&c->N, &c->phase, &c->face, &c->clipped, &c->status, &c->steps, &c->cnt,
                  &c->fail, &c->cface, &c->ccount, &c->tile_prob, &c->tile_start, &c->log_cnt,
                  &c->log_fl})
    ct_free(*q);
  for (double** q : {&c->h, &c->dl, &c->dr, &c->pw, &c->t, &c->dt}) ct_free(*q);
  ct_free(c->iters);
  ct_free(c->S);
  for (int b = 0; b < 2; ++b)
    for (int q = 0; q < 2; ++q) ct_free(c->U[b][q]);
  for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
  c->tev.clear();
  for (hipEvent_t* e : {&c->ev_in, &c->ev_fork, &c->ev_join, &c->ev_out})
    if (*e) (void)hipEventDestroy(*e), *e = nullptr;
  if (c->ms) (void)hipStreamDestroy(c->ms);
  if (c->zs) (void)hipStreamDestroy(c->zs);
  c->ms = c->zs = nullptr;
}

ct::Args ct_args(const imexds_ct_ctx* c, int parity) {
  ct::Args A = c->base;
  A.P = c->P;
  A.off = c->off;
  A.N = c->N;
  A.h = c->h;
  A.phase = c->phase;
  A.tile_prob = c->tile_prob;
  A.tile_start = c->tile_start;
  A.r0 = c->U[parity][0];
  A.m0 = c->U[parity][1];
  A.r1 = c->U[parity ^ 1][0];
  A.m1 = c->U[parity ^ 1][1];
  A.face = c->face;
  A.dl = c->dl;
  A.dr = c->dr;
  A.pw = c->pw;
  A.t = c->t;
  A.dt = c->dt;
  A.clipped = c->clipped;
  A.status = c->status;
  A.steps = c->steps;
  A.iters = c->iters;
  A.cnt = c->cnt;
  A.fail = c->fail;
  A.S = c->S;
  A.cface = c->cface;
  A.ccount = c->ccount;
  A.log_cnt = c->log_cnt;
  A.log_fl = c->log_fl;
  A.log_row = (c->log_cnt && c->log_row < c->log_max) ? c->log_row : -1;
  A.zone_ppw = c->zone_ppw;
  A.zn_maxit = c->zn_maxit;
  A.zn_rtol = c->zn_rtol;
  return A;
}

hipError_t ct_launch_zone(const ct::Args& A, int lanes, hipStream_t s) {
  if (A.P <= 0) return hipSuccess;
  const int blocks = (A.P + A.zone_ppw - 1) / A.zone_ppw;
  const int key = A.Z * 10 + lanes;
  switch (key) {
    case 11: ct::k_ct_zone<1, 1><<<blocks, 64, 0, s>>>(A); break;
    case 12: ct::k_ct_zone<1, 2><<<blocks, 64, 0, s>>>(A); break;
    case 14: ct::k_ct_zone<1, 4><<<blocks, 64, 0, s>>>(A); break;
    case 21: ct::k_ct_zone<2, 1><<<blocks, 64, 0, s>>>(A); break;
    case 22: ct::k_ct_zone<2, 2><<<blocks, 64, 0, s>>>(A); break;
    case 24: ct::k_ct_zone<2, 4><<<blocks, 64, 0, s>>>(A); break;
    case 31: ct::k_ct_zone<3, 1><<<blocks, 64, 0, s>>>(A); break;
    case 32: ct::k_ct_zone<3, 2><<<blocks, 64, 0, s>>>(A); break;
    case 34: ct::k_ct_zone<3, 4><<<blocks, 64, 0, s>>>(A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t ct_launch_newton(const ct::Args& A, int lanes, hipStream_t s) {
  if (A.P <= 0) return hipSuccess;
  // tubes per wave as in ct::newton_tubes_per_wave: 1 + 2 (2 Z + 1) lane
  // groups per tube
  const int cap = 64 / ((2 * (2 * A.Z + 1) + 1) * lanes);
  const int tpw = A.zone_ppw < cap ? A.zone_ppw : cap;
  const int blocks = (A.P + tpw - 1) / tpw;
  switch (A.Z * 10 + lanes) {
    case 11: ct::k_ct_newton<1, 1><<<blocks, 64, 0, s>>>(A); break;
    case 12: ct::k_ct_newton<1, 2><<<blocks, 64, 0, s>>>(A); break;
    case 14: ct::k_ct_newton<1, 4><<<blocks, 64, 0, s>>>(A); break;
    case 21: ct::k_ct_newton<2, 1><<<blocks, 64, 0, s>>>(A); break;
    case 22: ct::k_ct_newton<2, 2><<<blocks, 64, 0, s>>>(A); break;
    case 24: ct::k_ct_newton<2, 4><<<blocks, 64, 0, s>>>(A); break;
    case 31: ct::k_ct_newton<3, 1><<<blocks, 64, 0, s>>>(A); break;
    case 32: ct::k_ct_newton<3, 2><<<blocks, 64, 0, s>>>(A); break;
    case 34: ct::k_ct_newton<3, 4><<<blocks, 64, 0, s>>>(A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t ct_launch_fin(const ct::Args& A, int init, hipStream_t s) {
  const int blocks = A.P > 0 ? (A.P + 255) / 256 : 1;
  ct::k_ct_fin<<<blocks, 256, 0, s>>>(A, init);
  return hipGetLastError();
}

int ct_enter(imexds_ct_ctx* c) {
  int e = ct_err(hipSetDevice(c->device));
  if (!e) e = ct_err(hipEventRecord(c->ev_in, c->user));
  if (!e) e = ct_err(hipStreamWaitEvent(c->ms, c->ev_in, 0));
  return e;
}

int ct_leave(imexds_ct_ctx* c) {
  int e = ct_err(hipEventRecord(c->ev_out, c->ms));
  if (!e) e = ct_err(hipStreamWaitEvent(c->user, c->ev_out, 0));
  return e;
}

hipEvent_t ct_timing_event(imexds_ct_ctx* c, int i) {
  while ((int)c->tev.size() <= i) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->tev.push_back(e);
  }
  return c->tev[i];
}

int ct_one_step(imexds_ct_ctx* c) {
  ct::Args A = ct_args(c, c->cur);
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  const bool tm = c->timing && c->timed_steps < CT_TIMED_MAX;
  if (tm) {
    for (int i = 0; i < 6; ++i) {
      ev[i] = ct_timing_event(c, 6 * c->timed_steps + i);
      if (!ev[i]) return IMEXDS_ERR_HIP;
    }
    if (hipEventRecord(ev[0], c->ms) != hipSuccess) return IMEXDS_ERR_HIP;
  }
  int e = 0;
  if (c->n_tiles) {
    ct::k_ct_detect<<<c->n_tiles, ct::TILE, 0, c->ms>>>(A, 0);
    e = ct_err(hipGetLastError());
  }
  if (!e) e = ct_err(hipEventRecord(c->ev_fork, c->ms));
  if (!e) e = ct_err(hipStreamWaitEvent(c->zs, c->ev_fork, 0));
  if (!e && tm) e = ct_err(hipEventRecord(ev[3], c->zs));
  if (!e && A.P > 0) {
    ct::k_ct_create<<<(A.P + 63) / 64, 64, 0, c->zs>>>(A);
    e = ct_err(hipGetLastError());
  }
  if (!e)
    e = ct_err(c->zone_solver == IMEXDS_CT_SOLVER_NEWTON ? ct_launch_newton(A, c->zone_lanes, c->zs)
                                                         : ct_launch_zone(A, c->zone_lanes, c->zs));
  if (!e && tm) e = ct_err(hipEventRecord(ev[4], c->zs));
  if (!e && tm) e = ct_err(hipEventRecord(ev[1], c->ms));
  if (!e && c->n_tiles) {
    ct::k_ct_bulk<<<c->n_tiles, ct::TILE, 0, c->ms>>>(A, 0);
    e = ct_err(hipGetLastError());
  }
  if (!e && tm) e = ct_err(hipEventRecord(ev[2], c->ms));
  if (!e) e = ct_err(hipEventRecord(c->ev_join, c->zs));
  if (!e) e = ct_err(hipStreamWaitEvent(c->ms, c->ev_join, 0));
  if (!e) e = ct_err(ct_launch_fin(A, 0, c->ms));
  if (!e && tm) e = ct_err(hipEventRecord(ev[5], c->ms));
  if (e) return e;
  if (tm) c->timed_steps += 1;
  c->cur ^= 1;
  c->log_row += 1;
  return 0;
}

// The arguments of tube p alone: per-tube arrays shifted to p, one tube, no
// log (the cell arrays and the tile table stay global).
ct::Args ct_problem_args(const ct::Args& A, int p) {
  ct::Args B = A;
  B.P = 1;
  B.off += p;
  B.N += p;
  B.h += p;
  B.phase += p;
  B.face += p;
  B.dl += p;
  B.dr += p;
  B.pw += 4 * (long long)p;
  B.t += p;
  B.dt += p;
  B.clipped += p;
  B.status += p;
  B.steps += p;
  B.iters += p;
  B.cnt += p;
  B.fail += p;
  B.S += p;
  B.cface += p;
  B.ccount += p;
  B.log_cnt = nullptr;
  B.log_fl = nullptr;
  B.log_row = -1;
  return B;
}

// One step launched tube by tube on the main stream: the unbatched form.
int ct_one_step_per_problem(imexds_ct_ctx* c) {
  ct::Args A = ct_args(c, c->cur);
  A.log_cnt = nullptr;
  A.log_fl = nullptr;
  A.log_row = -1;
  int e = 0;
  for (int p = 0; p < c->P && !e; ++p) {
    const ct::Args B = ct_problem_args(A, p);
    const int t0 = c->h_tile_first[p], nt = c->h_tile_first[p + 1] - t0;
    if (nt > 0) {
      ct::k_ct_detect<<<nt, ct::TILE, 0, c->ms>>>(A, t0);
      e = ct_err(hipGetLastError());
      if (!e) {
        ct::k_ct_bulk<<<nt, ct::TILE, 0, c->ms>>>(A, t0);
        e = ct_err(hipGetLastError());
      }
    }
    if (!e) {
      ct::k_ct_create<<<1, 64, 0, c->ms>>>(B);
      e = ct_err(hipGetLastError());
    }
    if (!e)
      e = ct_err(c->zone_solver == IMEXDS_CT_SOLVER_NEWTON ? ct_launch_newton(B, c->zone_lanes, c->ms)
                                                           : ct_launch_zone(B, c->zone_lanes, c->ms));
    if (!e) e = ct_err(ct_launch_fin(B, 0, c->ms));
  }
  if (e) return e;
  c->cur ^= 1;
  c->log_row += 1;
  return 0;
}

bool ct_pos(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

extern "C" {

int imexds_ct_create(imexds_ct_ctx** out, const imexds_material* mat, const imexds_params* par,
                     double p_min, double p_tilde, const imexds_ct_batch* b, void* hip_stream) {
  if (!out) return IMEXDS_ERR_INVALID_ARG;
  *out = nullptr;
  if (!mat || !par || !b || b->n_problems < 0) return IMEXDS_ERR_INVALID_ARG;
  if (!ct_pos(mat->a2_vap) || !ct_pos(mat->a2_liq) || !ct_pos(mat->p_sat) ||
      !ct_pos(mat->rho_liq_sat) || !ct_pos(mat->tau) || !std::isfinite(p_min) ||
      !std::isfinite(p_tilde))
    return IMEXDS_ERR_INVALID_ARG;
  if (!ct_pos(par->cfl) || par->zone_half < 1 || par->zone_half > 3 || !ct_pos(par->theta_nb) ||
      par->theta_nb > 1.0 || (par->tol_mode != IMEXDS_TOL_PAPER && par->tol_mode != IMEXDS_TOL_REL) ||
      !ct_pos(par->tol_nb) || !ct_pos(par->tol_tiny) || !ct_pos(par->tol_rel) || par->lmax < 1 ||
      (par->bc_left != 0 && par->bc_left != 1) || (par->bc_right != 0 && par->bc_right != 1) ||
      par->newton_maxit < 1 || !ct_pos(par->newton_rtol) || !(par->t_end >= 0.0))
    return IMEXDS_ERR_INVALID_ARG;
  const int P = b->n_problems;
  if (P > 0 && (!b->n_cells || !b->h || !b->phase)) return IMEXDS_ERR_INVALID_ARG;
  std::vector<long long> off(P + 1, 0);
  for (int p = 0; p < P; ++p) {
    const int N = b->n_cells[p];
    if (N < 4 || N > (1 << 28) || !ct_pos(b->h[p]) || (b->phase[p] != 0 && b->phase[p] != 1))
      return IMEXDS_ERR_INVALID_ARG;
    off[p + 1] = off[p] + N + 1;
  }
  imexds_ct_ctx* c = new (std::nothrow) imexds_ct_ctx();
  if (!c) return IMEXDS_ERR_OOM;
  int e = ct_err(hipGetDevice(&c->device));
  c->user = (hipStream_t)hip_stream;
  if (!e) e = ct_err(hipStreamCreateWithFlags(&c->ms, hipStreamNonBlocking));
  if (!e) e = ct_err(hipStreamCreateWithFlags(&c->zs, hipStreamNonBlocking));
  for (hipEvent_t* ev : {&c->ev_in, &c->ev_fork, &c->ev_join, &c->ev_out})
    if (!e) e = ct_err(hipEventCreateWithFlags(ev, hipEventDisableTiming));
  ct::Args& B = c->base;
  B.M.a2v = mat->a2_vap;
  B.M.a2l = mat->a2_liq;
  B.M.p0 = mat->p_sat;
  B.M.rhol0 = mat->rho_liq_sat;
  B.M.tau = mat->tau;
  B.M.av = std::sqrt(mat->a2_vap);
  B.M.al = std::sqrt(mat->a2_liq);
  B.M.rhov0 = mat->p_sat / mat->a2_vap;
  B.M.ia2v = 1.0 / B.M.a2v;
  B.M.ia2l = 1.0 / B.M.a2l;
  B.M.iav = 1.0 / B.M.av;
  B.M.ial = 1.0 / B.M.al;
  B.M.irv0 = 1.0 / B.M.rhov0;
  B.M.irl0 = 1.0 / B.M.rhol0;
  B.cfl = par->cfl;
  B.theta_nb = par->theta_nb;
  B.tol_nb = par->tol_nb;
  B.tol_tiny = par->tol_tiny;
  B.tol_rel = par->tol_rel;
  B.t_end = par->t_end;
  B.newton_rtol = par->newton_rtol;
  B.p_min = p_min;
  B.p_tilde = p_tilde;
  B.tol_mode = par->tol_mode;
  B.lmax = par->lmax;
  B.Z = par->zone_half;
  B.bc_left = par->bc_left;
  B.bc_right = par->bc_right;
  B.newton_maxit = par->newton_maxit;
  c->P = P;
  c->nslot = off[P];
  c->h_N.assign(b->n_cells, b->n_cells + P);
  // tiles of TILE regular cells, problem by problem
  std::vector<int> tp, ts;
  c->h_tile_first.assign(P + 1, 0);
  for (int p = 0; p < P; ++p) {
    c->h_tile_first[p] = (int)tp.size();
    for (int s = 0; s < b->n_cells[p]; s += ct::TILE) {
      tp.push_back(p);
      ts.push_back(s);
    }
  }
  c->n_tiles = (int)tp.size();
  c->h_tile_first[P] = c->n_tiles;
  if (!e) e = ct_alloc(&c->off, P + 1);
  for (int** q : {&c->N, &c->phase, &c->face, &c->clipped, &c->status, &c->steps, &c->cnt,
                  &c->fail, &c->cface, &c->ccount})
    if (!e) e = ct_alloc(q, P);
  for (double** q : {&c->h, &c->dl, &c->dr, &c->t, &c->dt})
    if (!e) e = ct_alloc(q, P);
  if (!e) e = ct_alloc(&c->pw, 4 * (size_t)P);
  if (!e) e = ct_alloc(&c->iters, P);
  if (!e) e = ct_alloc(&c->S, P);
  for (int bb = 0; bb < 2; ++bb)
    for (int q = 0; q < 2; ++q)
      if (!e) e = ct_alloc(&c->U[bb][q], c->nslot);
  if (!e) e = ct_alloc(&c->tile_prob, tp.size());
  if (!e) e = ct_alloc(&c->tile_start, ts.size());
  auto up = [&](void* d, const void* hsrc, size_t bytes) {
    if (!e && bytes) e = ct_err(hipMemcpy(d, hsrc, bytes, hipMemcpyHostToDevice));
  };
  up(c->off, off.data(), (P + 1) * sizeof(long long));
  up(c->N, b->n_cells, P * sizeof(int));
  up(c->phase, b->phase, P * sizeof(int));
  up(c->h, b->h, P * sizeof(double));
  up(c->tile_prob, tp.data(), tp.size() * sizeof(int));
  up(c->tile_start, ts.data(), ts.size() * sizeof(int));
  if (e) {
    ct_release(c);
    delete c;
    return e;
  }
  *out = c;
  return 0;
}

int imexds_ct_set_state(imexds_ct_ctx* c, const double* rho, const double* mom) {
  if (!c || (c->nslot && (!rho || !mom))) return IMEXDS_ERR_INVALID_ARG;
  int e = ct_enter(c);
  const size_t bytes = (size_t)c->nslot * sizeof(double);
  c->cur = 0;
  if (!e && bytes) e = ct_err(hipMemcpyAsync(c->U[0][0], rho, bytes, hipMemcpyDeviceToDevice, c->ms));
  if (!e && bytes) e = ct_err(hipMemcpyAsync(c->U[0][1], mom, bytes, hipMemcpyDeviceToDevice, c->ms));
  const size_t P = (size_t)c->P;
  if (!e && P) e = ct_err(hipMemsetAsync(c->face, 0xff, P * sizeof(int), c->ms));  // -1
  for (double* q : {c->dl, c->dr, c->t, c->dt})
    if (!e && P) e = ct_err(hipMemsetAsync(q, 0, P * sizeof(double), c->ms));
  if (!e && P) e = ct_err(hipMemsetAsync(c->pw, 0, 4 * P * sizeof(double), c->ms));
  for (int* q : {c->clipped, c->status, c->steps, c->cnt, c->fail, c->ccount})
    if (!e && P) e = ct_err(hipMemsetAsync(q, 0, P * sizeof(int), c->ms));
  if (!e && P) e = ct_err(hipMemsetAsync(c->iters, 0, P * sizeof(long long), c->ms));
  if (!e && P) e = ct_err(hipMemsetAsync(c->S, 0, P * sizeof(unsigned long long), c->ms));
  ct::Args A = ct_args(c, 0);
  if (!e && c->n_tiles) {
    ct::k_ct_cfl<<<c->n_tiles, ct::TILE, 0, c->ms>>>(A);
    e = ct_err(hipGetLastError());
  }
  if (!e) e = ct_err(ct_launch_fin(A, 1, c->ms));
  c->log_row = 0;
  if (!e) e = ct_leave(c);
  c->have_state = e == 0;
  return e;
}

int imexds_ct_step(imexds_ct_ctx* c, int32_t n_steps) {
  if (!c || n_steps < 0) return IMEXDS_ERR_INVALID_ARG;
  if (!c->have_state) return IMEXDS_ERR_NO_STATE;
  int e = ct_enter(c);
  for (int i = 0; i < n_steps && !e; ++i) e = ct_one_step(c);
  if (!e) e = ct_leave(c);
  return e;
}

int imexds_ct_step_per_problem(imexds_ct_ctx* c, int32_t n_steps) {
  if (!c || n_steps < 0) return IMEXDS_ERR_INVALID_ARG;
  if (!c->have_state) return IMEXDS_ERR_NO_STATE;
  int e = ct_enter(c);
  for (int i = 0; i < n_steps && !e; ++i) e = ct_one_step_per_problem(c);
  if (!e) e = ct_leave(c);
  return e;
}

int imexds_ct_get_problems(imexds_ct_ctx* c, double* t, int32_t* status, int32_t* steps,
                           int64_t* iters, int32_t* face, double* dl, double* dr) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  if (!c->have_state) return IMEXDS_ERR_NO_STATE;
  int e = ct_enter(c);
  if (!e) e = ct_err(hipStreamSynchronize(c->ms));
  const size_t P = (size_t)c->P;
  auto down = [&](void* hdst, const void* d, size_t bytes) {
    if (!e && hdst && bytes) e = ct_err(hipMemcpy(hdst, d, bytes, hipMemcpyDeviceToHost));
  };
  down(t, c->t, P * sizeof(double));
  down(status, c->status, P * sizeof(int));
  down(steps, c->steps, P * sizeof(int));
  down(iters, c->iters, P * sizeof(long long));
  down(face, c->face, P * sizeof(int));
  down(dl, c->dl, P * sizeof(double));
  down(dr, c->dr, P * sizeof(double));
  return e;
}

int imexds_ct_run(imexds_ct_ctx* c, int32_t max_steps, int32_t check_every,
                  int32_t* steps_done) {
  if (!c || max_steps < 0 || check_every <= 0) return IMEXDS_ERR_INVALID_ARG;
  if (!c->have_state) return IMEXDS_ERR_NO_STATE;
  int done = 0, e = 0;
  std::vector<double> t(c->P);
  std::vector<int> st(c->P);
  while (!e && done < max_steps) {
    const int n = std::min(check_every, max_steps - done);
    e = imexds_ct_step(c, n);
    if (e) break;
    done += n;
    e = imexds_ct_get_problems(c, t.data(), st.data(), nullptr, nullptr, nullptr, nullptr,
                               nullptr);
    bool active = false;
    for (int p = 0; p < c->P && !e; ++p) active = active || (st[p] == 0 && t[p] < c->base.t_end);
    if (!active) break;
  }
  if (steps_done) *steps_done = done;
  return e;
}

int imexds_ct_get_state(imexds_ct_ctx* c, double* rho, double* mom) {
  if (!c || (c->nslot && (!rho || !mom))) return IMEXDS_ERR_INVALID_ARG;
  if (!c->have_state) return IMEXDS_ERR_NO_STATE;
  int e = ct_enter(c);
  const size_t bytes = (size_t)c->nslot * sizeof(double);
  if (!e && bytes)
    e = ct_err(hipMemcpyAsync(rho, c->U[c->cur][0], bytes, hipMemcpyDeviceToDevice, c->ms));
  if (!e && bytes)
    e = ct_err(hipMemcpyAsync(mom, c->U[c->cur][1], bytes, hipMemcpyDeviceToDevice, c->ms));
  if (!e) e = ct_leave(c);
  return e;
}

int imexds_ct_enable_log(imexds_ct_ctx* c, int32_t max_steps) {
  if (!c || max_steps < 0) return IMEXDS_ERR_INVALID_ARG;
  int e = ct_err(hipSetDevice(c->device));
  if (!e) e = ct_err(hipStreamSynchronize(c->ms));
  ct_free(c->log_cnt);
  ct_free(c->log_fl);
  c->log_max = 0;
  c->log_row = 0;
  if (e || max_steps == 0) return e;
  const size_t n = (size_t)max_steps * (size_t)std::max(c->P, 1);
  e = ct_alloc(&c->log_cnt, n);
  if (!e) e = ct_alloc(&c->log_fl, n);
  if (!e) e = ct_err(hipMemset(c->log_cnt, 0, n * sizeof(int)));
  if (!e) e = ct_err(hipMemset(c->log_fl, 0, n * sizeof(int)));
  if (e) {
    ct_free(c->log_cnt);
    ct_free(c->log_fl);
    return e;
  }
  c->log_max = max_steps;
  return 0;
}

int imexds_ct_get_log(imexds_ct_ctx* c, int32_t* count, int32_t* flags, int32_t* rows) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  int e = ct_err(hipSetDevice(c->device));
  if (!e) e = ct_err(hipStreamSynchronize(c->ms));
  const int r = std::min(c->log_row, c->log_max);
  if (rows) *rows = r;
  const size_t n = (size_t)r * (size_t)c->P;
  if (!e && n && count)
    e = ct_err(hipMemcpy(count, c->log_cnt, n * sizeof(int), hipMemcpyDeviceToHost));
  if (!e && n && flags)
    e = ct_err(hipMemcpy(flags, c->log_fl, n * sizeof(int), hipMemcpyDeviceToHost));
  return e;
}

int imexds_ct_set_launch(imexds_ct_ctx* c, int32_t zone_lanes, int32_t zone_problems_per_wave) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  if (zone_lanes != 1 && zone_lanes != 2 && zone_lanes != 4) return IMEXDS_ERR_INVALID_ARG;
  if (zone_problems_per_wave < 1 || zone_problems_per_wave * zone_lanes > 64)
    return IMEXDS_ERR_INVALID_ARG;
  int e = ct_err(hipSetDevice(c->device));
  if (!e) e = ct_err(hipStreamSynchronize(c->ms));
  if (e) return e;
  c->zone_lanes = zone_lanes;
  c->zone_ppw = zone_problems_per_wave;
  return 0;
}

int imexds_ct_set_solver(imexds_ct_ctx* c, int32_t solver, int32_t maxit, double rtol) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  if (solver != IMEXDS_CT_SOLVER_DTS && solver != IMEXDS_CT_SOLVER_NEWTON)
    return IMEXDS_ERR_INVALID_ARG;
  if (maxit < 1 || !ct_pos(rtol)) return IMEXDS_ERR_INVALID_ARG;
  int e = ct_err(hipSetDevice(c->device));
  if (!e) e = ct_err(hipStreamSynchronize(c->ms));
  if (!e) e = ct_err(hipStreamSynchronize(c->zs));
  if (e) return e;
  c->zone_solver = solver;
  c->zn_maxit = maxit;
  c->zn_rtol = rtol;
  return 0;
}

int imexds_ct_get_sizes(imexds_ct_ctx* c, int32_t* n_problems, int64_t* n_slots) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  if (n_problems) *n_problems = c->P;
  if (n_slots) *n_slots = c->nslot;
  return 0;
}

int imexds_ct_time_kernels(imexds_ct_ctx* c, int32_t on) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  int e = ct_err(hipSetDevice(c->device));
  if (!e) e = ct_err(hipStreamSynchronize(c->ms));
  c->timing = on != 0;
  c->timed_steps = 0;
  return e;
}

int imexds_ct_last_timing(imexds_ct_ctx* c, double* bulk_ms, double* zone_ms, double* step_ms) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  int e = ct_err(hipSetDevice(c->device));
  if (!e) e = ct_err(hipStreamSynchronize(c->ms));
  if (!e) e = ct_err(hipStreamSynchronize(c->zs));
  double sb = 0, sz = 0, ss = 0;
  const int n = c->timed_steps;
  for (int i = 0; i < n && !e; ++i) {
    float x = 0, y = 0, z = 0;
    e = ct_err(hipEventElapsedTime(&x, c->tev[6 * i + 1], c->tev[6 * i + 2]));
    if (!e) e = ct_err(hipEventElapsedTime(&y, c->tev[6 * i + 3], c->tev[6 * i + 4]));
    if (!e) e = ct_err(hipEventElapsedTime(&z, c->tev[6 * i], c->tev[6 * i + 5]));
    sb += x;
    sz += y;
    ss += z;
  }
  const double d = n > 0 ? (double)n : 1.0;
  if (bulk_ms) *bulk_ms = sb / d;
  if (zone_ms) *zone_ms = sz / d;
  if (step_ms) *step_ms = ss / d;
  return e;
}

void imexds_ct_destroy(imexds_ct_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->ms) (void)hipStreamSynchronize(c->ms);
  if (c->zs) (void)hipStreamSynchronize(c->zs);
  ct_release(c);
  delete c;
}

}  // extern "C"
