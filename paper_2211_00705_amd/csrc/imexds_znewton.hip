// imexds_znewton.hip -- the interface zones of one step solved by Newton on
// their implicit step instead of Algorithm 2 (the Newton-like solver for the
// small implicit systems that the paper's outlook names).  Everything around
// the solve is the zone step of k_zone: the prediction of the boundary speed
// from U^n, the merge test, the zone (tiny cut piece +- Z slots, a merged
// piece folded into its neighbour), the redo with a merge when the tiny cell
// collapses, Part 2, the interface advance and re-split, the records, logs
// and the CFL contribution.
//
// The solve: unknowns the zone cells' values W (2 per cell), residual
//   R_i(W) = (h_i(W) / h_i^n) W_i - U_i^n + (dt / h_i^n)(F_{i+1/2}(W) - F_{i-1/2}(W)),
// h_i(W) = h_i^n + mov_i w(W) dt, the zone's outer faces from U^n.  From
// W = U^n each Newton step evaluates R at the base point and at the points
// moved along each unknown (forward differences, step 1e-7 max(|W_j|, 1));
// every interface solve of a step starts from the previous base point's root
// (in a zone's first step from the recorded root, as the prediction).  Of the
// difference Jacobian the 2x2 blocks next to the diagonal are kept (R_i
// depends on W_{i-1}, W_i, W_{i+1} only), solved by the block Thomas
// algorithm.  The step is the last when every component is below
// zn_rtol max(|W_j|, 1) or it is the zn_maxit-th (then flagged like l_max);
// else W moves by the full step.  Part 2 takes the last base point's fluxes
// and boundary speed.  The kernel works on 2 Z + 1 cells; cells past the
// zone (the folded piece's position is left out) are identity rows with
// zero right-hand sides, which leave the zone cells' results as in the
// compact system.
//
// A zone has G = 1 + 2 MC groups of one lane, or of two lanes (the pair form
// of the interface solver: one lane per side of the interface problem).  In
// a round group 0 evaluates the base point and group g >= 1 the point moved
// along unknown g - 1, all side by side; the base point's residual, root and
// boundary speed are then read from group 0, and every lane gathers the three
// blocks of each cell's row and runs the same block solve.  The first round
// is also the prediction (the base point is U^n); unless the prediction
// merges the tiny piece, it is the first Newton step too.
#include "imexds_device.hpp"
#include "imexds_kernels.hpp"

namespace imexds {
namespace {

constexpr unsigned long long NT_NAN_BITS = 0x7FF8000000000000ull;

__device__ __forceinline__ unsigned long long nt_speed_bits(const Mat& M, int ph, double r,
                                                            double m) {
  if (!d_state_ok(r, m)) return NT_NAN_BITS;
  return (unsigned long long)__double_as_longlong(fabs(m / r) + d_a(M, ph));
}

template <int ZH, int LG>
__global__ __launch_bounds__(64) void k_zone_nt(StepArgs A, int if_begin, int if_end) {
  constexpr int MC = 2 * ZH + 1, NV = 2 * MC, G = NV + 1, TL = LG * G, ZPW = 64 / TL;
  const Mat& M = A.mat;
  const Par& P = A.par;
  const int lane = (int)threadIdx.x;
  if (lane >= ZPW * TL) return;
  const int tl = lane % TL;
  const int grp = tl / LG, half = LG == 2 ? (tl & 1) : 0;
  const int lane0 = lane - tl;
  const int k = if_begin + (int)blockIdx.x * ZPW + lane / TL;
  if (k >= if_end) return;  // the lanes of a zone are whole
  const bool writer = tl == 0;
  const int p = A.iface_prob[k];
  const int kk = A.iface_local[k];
  const double dt = A.dt[p];
  const int home = A.rec_home0[k];
  const double hl = A.rec_hl0[k];
  const double rpw0 = A.rec_pw0[2 * k], rpw1 = A.rec_pw0[2 * k + 1];
  const int warm = A.rec_warm0[k];
  int row = -1;
  if (A.log_count && A.log_row) {
    row = *A.log_row;
    if (row >= A.log_max) row = -1;
  }
  const long long so = A.slot_off[p];
  const int ns = (int)(A.slot_off[p + 1] - so);
  const int sL = home + kk;
  if (dt == 0.0 || sL < 0 || sL + 1 >= ns) {
    if (writer) {
      if (dt != 0.0) atomicOr(A.fail_acc + p, ST_MESH);
      A.rec_home1[k] = home;
      A.rec_hl1[k] = hl;
      A.rec_pw1[2 * k] = rpw0;
      A.rec_pw1[2 * k + 1] = rpw1;
      A.rec_warm1[k] = warm;
      if (row >= 0) {
        const long long o = (long long)row * A.n_iface + k;
        A.log_count[o] = 0;
        A.log_flags[o] = dt == 0.0 ? FL_INACTIVE : FL_FAIL;
        A.log_zlo[o] = -1;
      }
    }
    return;
  }
  const double h = A.h[p];
  const int phl = A.phase_first[p] ^ (kk & 1), phr = phl ^ 1;
  int zlo, zhi;
  bool tr;
  d_zone_range(sL, hl, h, ZH, ns, zlo, zhi, tr);
  const int nr = zhi - zlo + 1, iL = sL - zlo, iR = iL + 1;
  const double* r0 = A.rho0 + so;
  const double* m0 = A.mom0 + so;
  double Ur[MC], Um[MC];
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    Ur[i] = i < nr ? r0[zlo + i] : 1.0;
    Um[i] = i < nr ? m0[zlo + i] : 0.0;
  }
  double FL0, FL1, FR0, FR1;
  {
    const int phz = (zlo <= sL) ? phl : phr;
    if (zlo == 0)
      d_bflux(M, phz, false, P.bc_left, r0[0], m0[0], FL0, FL1);
    else
      d_hll(M, phz, r0[zlo - 1], m0[zlo - 1], r0[zlo], m0[zlo], FL0, FL1);
    const int phe = (zhi <= sL) ? phl : phr;
    if (zhi == ns - 1)
      d_bflux(M, phe, true, P.bc_right, r0[ns - 1], m0[ns - 1], FR0, FR1);
    else
      d_hll(M, phe, r0[zhi], m0[zhi], r0[zhi + 1], m0[zhi + 1], FR0, FR1);
  }
  // zone state
  bool merge = false, redo = false;
  int skip = -1, into = -1, ic = 0, icr = 1, tiny = 0;
  double Mr = 0.0, Mm = 0.0, hn_l = 0.0, hn_r = 0.0, hh_l = 0.0, hh_r = 0.0;
  double wp = 0.0;
  double W0[MC], W1[MC];
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    W0[i] = Ur[i];
    W1[i] = Um[i];
  }
  double pw0 = 0.0, pw1 = 0.0, w = 0.0;
  const int colj = grp - 1;
  int status = 0, it = 0;
  bool pred = true, conv = false, finished = false;
  double wstar = 0.0;
  // (re)builds the zone after the prediction or a redo: the folded piece and
  // its merged content, the interface cells, the lengths; false (status set)
  // when the zone cannot be built
  auto build_zone = [&]() -> bool {
    skip = -1;
    into = -1;
    if (merge) {
      skip = tr ? iR : iL;
      into = tr ? iR + 1 : iL - 1;
      if (into < 0 || into >= nr) status = ST_MESH;
    }
    if (status) return false;
    double rskip = 0.0, mskip = 0.0, rin = 0.0, min_ = 0.0;
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      if (i == skip) {
        rskip = Ur[i];
        mskip = Um[i];
      }
      if (i == into) {
        rin = Ur[i];
        min_ = Um[i];
      }
    }
    const double hLp = hl, hRp = h - hl;
    const double ht = tr ? hRp : hLp;
    const double hm = h + ht;
    if (merge) {
      Mr = (h * rin + ht * rskip) / hm;
      Mm = (h * min_ + ht * mskip) / hm;
    }
    ic = (merge && !tr) ? into : iL;
    icr = (merge && tr) ? into : iR;
    tiny = merge ? into : (tr ? iR : iL);
    hn_l = (merge && !tr) ? hm : hLp;
    hn_r = (merge && tr) ? hm : hRp;
    hh_l = hn_l + (1.0 * wp) * dt;
    hh_r = hn_r + (-1.0 * wp) * dt;
    const double hh_f = h + (0.0 * wp) * dt;
    double th_l = hh_l / h, th_r = hh_r / h, th_f = hh_f / h;
    if (th_l > P.theta_nb) th_l = P.theta_nb;
    if (th_r > P.theta_nb) th_r = P.theta_nb;
    if (th_f > P.theta_nb) th_f = P.theta_nb;
    if (!(th_l > 0.0) || !(th_r > 0.0) || !(th_f > 0.0)) {
      status = ST_MESH;
      return false;
    }
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      W0[i] = (i == into) ? Mr : Ur[i];
      W1[i] = (i == into) ? Mm : Um[i];
    }
    it = 0;
    conv = false;
    return true;
  };
#pragma unroll 1
  for (;;) {
    // One Newton step: group 0 evaluates the base point W, group g >= 1 the
    // point moved along unknown colj = g - 1 when that unknown belongs to the
    // zone (component ccmp of zone cell ccell, zone cells in slot order and
    // the folded piece left out, at position cpos).  The first round is also
    // the prediction (group 0's point is U^n at the cut); without a merge it
    // is the first Newton step as well, since W = U^n there.
    const int mm = skip >= 0 ? nr - 1 : nr;
    const int ccell = colj >> 1, ccmp = colj & 1;
    const int cpos = ccell + ((skip >= 0 && ccell >= skip) ? 1 : 0);
    const bool moved = colj >= 0 && ccell < mm;
    double xj = 0.0;
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      if (cpos == i && ccmp == 0) xj = W0[i];
      if (cpos == i && ccmp == 1) xj = W1[i];
    }
    const double ecol = 1e-7 * (fabs(xj) > 1.0 ? fabs(xj) : 1.0);
    double X0[MC], X1[MC];
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      X0[i] = (moved && cpos == i && ccmp == 0) ? W0[i] + ecol : W0[i];
      X1[i] = (moved && cpos == i && ccmp == 1) ? W1[i] + ecol : W1[i];
    }
    // the interface problem: positions iL, iR (prediction) or ic, icr
    const int a = pred ? iL : ic, b = pred ? iR : icr;
    double ql0 = 0.0, ql1 = 0.0, qr0 = 0.0, qr1 = 0.0;
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      if (i == a) {
        ql0 = X0[i];
        ql1 = X1[i];
      }
      if (i == b) {
        qr0 = X0[i];
        qr1 = X1[i];
      }
    }
    // every solve of a step starts from the previous base point's root; in
    // the first step of a (re)built zone, as the prediction, from the
    // recorded root (or the solver's guess without one)
    const bool rs = it == 0;
    const bool hg = rs ? warm != 0 : true;
    const double g0 = rs ? rpw0 : pw0;
    const double g1 = rs ? rpw1 : pw1;
    IfaceOut o;
    const bool okl = d_iface_solve_t<LG == 2>(M, P.newton_maxit, P.newton_rtol, phl, ql0, ql1,
                                              phr, qr0, qr1, hg, g0, g1, half, o);
    const unsigned long long zm = ((1ull << TL) - 1ull) << lane0;
    const unsigned long long failm = __ballot(!okl) & zm;
    // the base point's solve first (group 0); a moved point's failure counts
    // after the base point's shrink test
    const unsigned long long bm = ((1ull << LG) - 1ull) << lane0;
    if (failm & bm) {
      status = ST_NEWTON;
      break;
    }
    // the base point's boundary speed and root, from group 0
    const double bw = __shfl(o.w, lane0, 64);
    const double bpl = __shfl(o.pl, lane0, 64);
    const double bpr = __shfl(o.pr, lane0, 64);
    if (pred) {
      pred = false;
      wp = bw;
      const double ht = tr ? h - hl : hl;
      const double rate = tr ? -wp : wp;
      const double hfl = P.alpha_floor * h;
      merge = (ht < hfl) || (ht + (P.merge_safety * rate) * dt < hfl);
      if (!build_zone()) break;
      if (merge) continue;  // the zone changed: this round's points are not its own
    }
    const double we = o.w;
    // right face of each zone position at the point
    double FR_0[MC], FR_1[MC];
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      FR_0[i] = 0.0;
      FR_1[i] = 0.0;
      if (i >= nr || i == skip) continue;
      if (i == nr - 1) {
        FR_0[i] = FR0;
        FR_1[i] = FR1;
      } else if (i == ic) {
        FR_0[i] = o.F0;
        FR_1[i] = o.F1;
      } else if (i + 1 < MC) {
        const int ph = (zlo + i <= sL) ? phl : phr;
        d_hll(M, ph, X0[i], X1[i], X0[i + 1], X1[i + 1], FR_0[i], FR_1[i]);
      }
    }
    const double hk_l = hn_l + (1.0 * we) * dt;
    const double hk_r = hn_r + (-1.0 * we) * dt;
    const double hk_f = h + (0.0 * we) * dt;
    {  // shrink test at the base point
      const double bk_l = hn_l + (1.0 * bw) * dt;
      const double bk_r = hn_r + (-1.0 * bw) * dt;
      const bool bl = !(bk_l >= 0.5 * hh_l), br = !(bk_r >= 0.5 * hh_r);
      int shrink = -1;
      if (bl && br)
        shrink = ic < icr ? ic : icr;
      else if (bl)
        shrink = ic;
      else if (br)
        shrink = icr;
      if (shrink >= 0) {
        if (!merge && shrink == tiny) {
          merge = true;
          redo = true;
          if (!build_zone()) break;
          continue;
        }
        status = ST_MESH;
        break;
      }
    }
    if (failm) {
      status = ST_NEWTON;
      break;
    }
    pw0 = bpl;
    pw1 = bpr;
    w = bw;
    // residual of every zone position at the point
    double RX[NV];
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      RX[2 * i] = 0.0;
      RX[2 * i + 1] = 0.0;
      if (i >= nr || i == skip) continue;
      double fl0, fl1;
      if (i == 0) {
        fl0 = FL0;
        fl1 = FL1;
      } else if (i >= 2 && skip == i - 1) {
        fl0 = FR_0[i >= 2 ? i - 2 : 0];
        fl1 = FR_1[i >= 2 ? i - 2 : 0];
      } else {
        fl0 = FR_0[i - 1];
        fl1 = FR_1[i - 1];
      }
      const double u0r = (i == into) ? Mr : Ur[i];
      const double u0m = (i == into) ? Mm : Um[i];
      const double hni = (i == ic) ? hn_l : ((i == icr) ? hn_r : h);
      const double hki = (i == ic) ? hk_l : ((i == icr) ? hk_r : hk_f);
      const double ihn = 1.0 / hni;
      RX[2 * i] = (hki * ihn) * X0[i] - u0r + (dt * ihn) * (FR_0[i] - fl0);
      RX[2 * i + 1] = (hki * ihn) * X1[i] - u0m + (dt * ihn) * (FR_1[i] - fl1);
    }
    // the base point's residual, from group 0, and this group's difference
    // column (group 0's is not used)
    double R[NV], Jc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      R[i] = __shfl(RX[i], lane0, 64);
      Jc[i] = (RX[i] - R[i]) / ecol;
    }
    // rows in zone-cell order (the folded piece's position left out)
    double Jk[NV], Rk[NV];
#pragma unroll
    for (int c = 0; c < MC; ++c) {
      const bool sh = skip >= 0 && c >= skip;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const double j1 = c + 1 < MC ? Jc[2 * (c + 1) + a] : 0.0;
        const double r1 = c + 1 < MC ? R[2 * (c + 1) + a] : 0.0;
        Jk[2 * c + a] = sh ? j1 : Jc[2 * c + a];
        Rk[2 * c + a] = sh ? r1 : R[2 * c + a];
      }
    }
    // block tridiagonal solve (block Thomas, the oracle's order of
    // operations): group j + 1 holds column j; cell c's blocks D_c, L_c and
    // U_{c-1} are gathered from the groups of cells c, c - 1 and c.  Cells
    // c >= mm are identity rows with zero right-hand sides: their L, U blocks
    // are zero, so they leave the zone cells' forward sweep untouched and
    // give x_c = +-0, which subtracts nothing from the last zone cell.
    double Ib[MC][2][2], rp[MC][2], Ub[MC][2][2], dx[MC][2];
    bool sing = false;
#pragma unroll
    for (int c = 0; c < MC; ++c) {
      const bool ac = c < mm;
      double Dp[2][2], rc[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        rc[a] = ac ? -Rk[2 * c + a] : 0.0;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const double v = __shfl(Jk[2 * c + a], lane0 + LG * (2 * c + b + 1), 64);
          Dp[a][b] = ac ? v : (a == b ? 1.0 : 0.0);
        }
      }
      if (c > 0) {
        double Lc[2][2], Lf[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const double lv = __shfl(Jk[2 * c + a], lane0 + LG * (2 * (c - 1) + b + 1), 64);
            const double uv = __shfl(Jk[2 * (c - 1) + a], lane0 + LG * (2 * c + b + 1), 64);
            Lc[a][b] = ac ? lv : 0.0;
            Ub[c - 1][a][b] = ac ? uv : 0.0;
          }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            Lf[a][b] = Lc[a][0] * Ib[c - 1][0][b] + Lc[a][1] * Ib[c - 1][1][b];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
#pragma unroll
          for (int b = 0; b < 2; ++b)
            Dp[a][b] = Dp[a][b] - (Lf[a][0] * Ub[c - 1][0][b] + Lf[a][1] * Ub[c - 1][1][b]);
          rc[a] = rc[a] - (Lf[a][0] * rp[c - 1][0] + Lf[a][1] * rp[c - 1][1]);
        }
      }
      rp[c][0] = rc[0];
      rp[c][1] = rc[1];
      const double det = Dp[0][0] * Dp[1][1] - Dp[0][1] * Dp[1][0];
      const double id = 1.0 / det;
      if (ac && !d_finite(id)) sing = true;
      Ib[c][0][0] = Dp[1][1] * id;
      Ib[c][0][1] = -Dp[0][1] * id;
      Ib[c][1][0] = -Dp[1][0] * id;
      Ib[c][1][1] = Dp[0][0] * id;
    }
#pragma unroll
    for (int c = MC - 1; c >= 0; --c) {
      double y[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        y[a] = c == MC - 1 ? rp[c][a]
                           : rp[c][a] - (Ub[c][a][0] * dx[c + 1][0] + Ub[c][a][1] * dx[c + 1][1]);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        dx[c][a] = Ib[c][a][0] * y[0] + Ib[c][a][1] * y[1];
        if (c < mm && !d_finite(dx[c][a])) sing = true;
      }
    }
    if (sing) {
      status = ST_NEWTON;
      break;
    }
    // the step of each zone position's values
    double e0[MC], e1[MC];
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      const bool sh = skip >= 0 && i > skip;
      e0[i] = (sh && i > 0) ? dx[i > 0 ? i - 1 : 0][0] : dx[i][0];
      e1[i] = (sh && i > 0) ? dx[i > 0 ? i - 1 : 0][1] : dx[i][1];
    }
    conv = true;
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      if (i >= nr || i == skip) continue;
      const double s0 = fabs(W0[i]) > 1.0 ? fabs(W0[i]) : 1.0;
      const double s1 = fabs(W1[i]) > 1.0 ? fabs(W1[i]) : 1.0;
      conv = conv && (fabs(e0[i]) <= P.zn_rtol * s0) && (fabs(e1[i]) <= P.zn_rtol * s1);
    }
    it += 1;
    if (conv || it >= P.zn_maxit) {
      // Part 2 with the base point's fluxes and boundary speed (group 0's;
      // the write-back is lane 0's)
      bool okw = true;
#pragma unroll
      for (int i = 0; i < MC; ++i) {
        if (i >= nr || i == skip) continue;
        double fl0, fl1;
        if (i == 0) {
          fl0 = FL0;
          fl1 = FL1;
        } else if (i >= 2 && skip == i - 1) {
          fl0 = FR_0[i >= 2 ? i - 2 : 0];
          fl1 = FR_1[i >= 2 ? i - 2 : 0];
        } else {
          fl0 = FR_0[i - 1];
          fl1 = FR_1[i - 1];
        }
        const double u0r = (i == into) ? Mr : Ur[i];
        const double u0m = (i == into) ? Mm : Um[i];
        const double hni = (i == ic) ? hn_l : ((i == icr) ? hn_r : h);
        const double hki = (i == ic) ? hk_l : ((i == icr) ? hk_r : hk_f);
        const double ih = 1.0 / hki;
        const double n0 = (hni * u0r - dt * (FR_0[i] - fl0)) * ih;
        const double n1 = (hni * u0m - dt * (FR_1[i] - fl1)) * ih;
        if (!d_state_ok(n0, n1)) okw = false;
        W0[i] = n0;
        W1[i] = n1;
      }
      if (!okw) {
        status = ST_NONPHYS;
      } else {
        wstar = w;
        finished = true;
      }
      break;
    }
    bool okst = true;
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      if (i >= nr || i == skip) continue;
      W0[i] = W0[i] + e0[i];
      W1[i] = W1[i] + e1[i];
      okst = okst && d_state_ok(W0[i], W1[i]);
    }
    if (!okst) {
      status = ST_NONPHYS;
      break;
    }
  }
  if (!writer) return;

  // ---------------- write-back (success or failure), as k_zone ----------------
  double* r1 = A.rho1 + so;
  double* m1 = A.mom1 + so;
  int flags = tr ? FL_TINY_RIGHT : 0;
  int count = 0;
  int nhome = home;
  double nhl = hl;
  if (finished) {
    const double hln = hl + wstar * dt;
    if (merge) {
      flags |= FL_MERGED;
      int src;
      if (!tr) {
        if (hln < 0.0) {
          nhome = home - 1;
          nhl = hln + h;
          src = iR;
          flags |= FL_CROSS_L;
        } else {
          nhl = hln;
          src = into;
        }
      } else {
        if (hln > h) {
          nhome = home + 1;
          nhl = hln - h;
          src = iL;
          flags |= FL_CROSS_R;
        } else {
          nhl = hln;
          src = into;
        }
      }
      double cr = 0.0, cm = 0.0;
#pragma unroll
      for (int i = 0; i < MC; ++i)
        if (i == src) {
          cr = W0[i];
          cm = W1[i];
        }
#pragma unroll
      for (int i = 0; i < MC; ++i)
        if (i == skip) {
          W0[i] = cr;
          W1[i] = cm;
        }
    } else {
      nhl = hln;
    }
    if (redo) flags |= FL_REDO;
    if (!conv) flags |= FL_LMAX;
    count = it;
    A.rec_pw1[2 * k] = pw0;
    A.rec_pw1[2 * k + 1] = pw1;
    A.rec_warm1[k] = 1;
    if (A.st_pseudo) atomicAdd(A.st_pseudo, (unsigned long long)count);
    if (merge && A.st_merges) atomicAdd(A.st_merges, 1ull);
    if (!conv && A.st_lmax) atomicAdd(A.st_lmax, 1ull);
  } else {
    flags |= FL_FAIL;
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      W0[i] = Ur[i];
      W1[i] = Um[i];
    }
    A.rec_pw1[2 * k] = rpw0;
    A.rec_pw1[2 * k + 1] = rpw1;
    A.rec_warm1[k] = warm;
    atomicOr(A.fail_acc + p, status);
  }
  if (A.st_events) {
    const int ev = ((flags & FL_MERGED) ? 1 : 0) + ((flags & FL_REDO) ? 1 : 0) +
                   ((flags & (FL_CROSS_L | FL_CROSS_R)) ? 1 : 0);
    if (ev) atomicAdd(A.st_events, (unsigned long long)ev);
  }
  A.rec_home1[k] = nhome;
  A.rec_hl1[k] = nhl;
  const int nsL = nhome + kk;
  unsigned long long vmax = 0;
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    if (i < nr) {
      r1[zlo + i] = W0[i];
      m1[zlo + i] = W1[i];
      const int ph = (zlo + i <= nsL) ? phl : phr;
      const unsigned long long bt = nt_speed_bits(M, ph, W0[i], W1[i]);
      vmax = bt > vmax ? bt : vmax;
    }
  }
  atomicMax(A.S_acc + p, vmax);
  if (row >= 0) {
    const long long o2 = (long long)row * A.n_iface + k;
    A.log_count[o2] = count;
    A.log_flags[o2] = flags;
    A.log_zlo[o2] = zlo;
  }
}

}  // namespace

template <int ZH, int LG>
hipError_t launch_nt(const StepArgs& A, int if_begin, int n, hipStream_t s) {
  constexpr int zpw = 64 / (LG * (2 * (2 * ZH + 1) + 1));
  k_zone_nt<ZH, LG><<<(n + zpw - 1) / zpw, 64, 0, s>>>(A, if_begin, if_begin + n);
  return hipGetLastError();
}

hipError_t launch_zone_newton(const StepArgs& A, int if_begin, int if_end, int lanes,
                              hipStream_t s) {
  const int n = if_end - if_begin;
  if (n <= 0) return hipSuccess;
  const bool pair = lanes != 1;
  switch (A.par.zone_half) {
    case 1: return pair ? launch_nt<1, 2>(A, if_begin, n, s) : launch_nt<1, 1>(A, if_begin, n, s);
    case 2: return pair ? launch_nt<2, 2>(A, if_begin, n, s) : launch_nt<2, 1>(A, if_begin, n, s);
    case 3: return pair ? launch_nt<3, 2>(A, if_begin, n, s) : launch_nt<3, 1>(A, if_begin, n, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace imexds
