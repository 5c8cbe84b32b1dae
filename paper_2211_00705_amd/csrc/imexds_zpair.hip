// imexds_zpair.hip -- implicit zones holding two phase boundaries (gfx950).
//
// When the zones (tiny cut piece +- Z slots) of two neighbouring interfaces
// of a problem overlap, their union is solved as one zone with both phase
// boundaries in it: Algorithm 2 (Part 1 and Part 2) over all its cells, two
// interface Riemann solves per pseudo iteration, each boundary with its own
// prediction, merge test, moving cells, redo after a collapse and re-split
// (Sec. 3.4, grid alignment of Sec. 2.3 applied per boundary).  A merge that
// would leave the phase between the two boundaries as a single cell bounded
// by both (the tiny piece merging into a piece of the other boundary's cut
// cell, or both tiny pieces into one cell) sets ST_VANISH and freezes the
// problem.  The single-boundary kernels leave such interfaces to this one.
//
// Two lanes per zone: both hold the whole zone and compute every step of it
// identically, except the interface solves: lane b solves boundary b and the
// two swap their results.  Candidates: lane pair j of block q takes interface
// if_begin + 32 q + j and works on it when it leads a pair (its zone overlaps
// the next interface's); every other lane pair leaves at once.  Zone cells
// are addressed by position 0..nr-1 in the slot range zlo..zhi; a merged-away
// piece keeps its position (inactive) and its content sits in the merged
// cell.  Every operation is the one the CPU oracle performs, in its order.
#include "imexds_device.hpp"
#include "imexds_kernels.hpp"

namespace imexds {

namespace {

// CFL contribution of one cell: |m / rho| + a as bits, or a NaN pattern (above
// every finite non-negative double in an unsigned max) if non-physical
__device__ __forceinline__ unsigned long long zp_speed_bits(const Mat& M, int ph, double r,
                                                            double m) {
  if (!d_state_ok(r, m)) return 0x7FF8000000000000ull;
  return (unsigned long long)__double_as_longlong(fabs(m / r) + d_a(M, ph));
}

// value of the partner lane of a two-lane group (both lanes must call)
__device__ __forceinline__ double zp_other(double x) { return __shfl_xor(x, 1, 64); }
__device__ __forceinline__ int zp_otheri(int x) { return __shfl_xor(x, 1, 64); }

}  // namespace

template <int ZH>
__global__ __launch_bounds__(64) void k_zone_pair(StepArgs A, int if_begin, int if_end) {
  constexpr int MC = 2 * ZH + 1;
  constexpr int MP = 2 * MC;  // positions of the union of two zones (at most 2 MC - 1)
  constexpr int S_PRED = 1, S_ITER = 2;
  const Mat& M = A.mat;
  const Par& P = A.par;
  const int lane = threadIdx.x;
  const int me = lane & 1;  // the boundary whose interface solve this lane runs
  const int k = if_begin + (int)blockIdx.x * 32 + (lane >> 1);
  if (k >= if_end) return;
  const int p = A.iface_prob[k];
  const int kk = A.iface_local[k];
  const int nif = A.iface_off[p + 1] - A.iface_off[p];
  const double dt = A.dt[p];
  const long long so = A.slot_off[p];
  const int ns = (int)(A.slot_off[p + 1] - so);
  const double h = A.h[p];
  if (dt == 0.0 || P.zone_solver != 0) return;
  if (!d_pair_lead(A, k, kk, nif, ns, h)) return;
  // both lanes of the pair are here, with identical values from now on
  if (me == 0 && A.pair_seen) atomicOr(A.pair_seen, 1);

  int row = -1;
  if (A.log_count && A.log_row) {
    row = *A.log_row;
    if (row >= A.log_max) row = -1;
  }
  const int phl0 = A.phase_first[p] ^ (kk & 1);  // phase left of boundary 0
  // per boundary b (interface k + b): records of the step's start
  int home[2], sL[2], iL[2], warm[2];
  double hl[2], rpw0[2], rpw1[2];
  bool tr[2];
  int zlo = 0, zhi = 0;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    home[b] = A.rec_home0[k + b];
    hl[b] = A.rec_hl0[k + b];
    rpw0[b] = A.rec_pw0[2 * (k + b)];
    rpw1[b] = A.rec_pw0[2 * (k + b) + 1];
    warm[b] = A.rec_warm0[k + b];
    sL[b] = home[b] + kk + b;
    int lo, hi;
    d_zone_range(sL[b], hl[b], h, ZH, ns, lo, hi, tr[b]);
    if (b == 0) zlo = lo;
    if (b == 1) zhi = hi;
  }
  const int nr = zhi - zlo + 1;
#pragma unroll
  for (int b = 0; b < 2; ++b) iL[b] = sL[b] - zlo;
  // phase of the slot at zone position i (boundaries at the step's start)
  auto ph_of = [&](int i, int s0, int s1) {
    const int s = zlo + i;
    return s <= s0 ? phl0 : (s <= s1 ? (phl0 ^ 1) : phl0);
  };
  const double* r0 = A.rho0 + so;
  const double* m0 = A.mom0 + so;
  double Ur[MP], Um[MP];
#pragma unroll
  for (int i = 0; i < MP; ++i) {
    Ur[i] = i < nr ? r0[zlo + i] : 1.0;
    Um[i] = i < nr ? m0[zlo + i] : 0.0;
  }
  // bounding fluxes from U^n (Algorithm 1: F_left, F_right)
  double FL0, FL1, FR0, FR1;
  {
    const int phz = ph_of(0, sL[0], sL[1]);
    if (zlo == 0)
      d_bflux(M, phz, false, P.bc_left, r0[0], m0[0], FL0, FL1);
    else
      d_hll(M, phz, r0[zlo - 1], m0[zlo - 1], r0[zlo], m0[zlo], FL0, FL1);
    const int phe = ph_of(nr - 1, sL[0], sL[1]);
    if (zhi == ns - 1)
      d_bflux(M, phe, true, P.bc_right, r0[ns - 1], m0[ns - 1], FR0, FR1);
    else
      d_hll(M, phe, r0[zhi], m0[zhi], r0[zhi + 1], m0[zhi + 1], FR0, FR1);
  }

  // per boundary: merge, merged cell, cells next to it, tiny cell, lengths,
  // pseudo steps, prediction, roots
  bool merge[2] = {false, false};
  int skip[2] = {-1, -1}, into[2] = {-1, -1}, ic[2] = {0, 0}, icr[2] = {1, 1}, tiny[2] = {0, 0};
  double Mr[2] = {0.0, 0.0}, Mm[2] = {0.0, 0.0};
  double hn_l[2] = {0.0, 0.0}, hn_r[2] = {0.0, 0.0}, hh_l[2] = {0.0, 0.0}, hh_r[2] = {0.0, 0.0};
  double th_l[2] = {0.0, 0.0}, th_r[2] = {0.0, 0.0}, it_l[2] = {0.0, 0.0}, it_r[2] = {0.0, 0.0};
  double th_f = 0.0, it_f = 0.0;
  double Ipl[2] = {0.0, 0.0}, Ipr[2] = {0.0, 0.0}, wp[2] = {0.0, 0.0};
  double pw0[2] = {0.0, 0.0}, pw1[2] = {0.0, 0.0}, gn0[2] = {0.0, 0.0}, gn1[2] = {0.0, 0.0};
  DtsRoots H[2];
  d_dts_reset(H[0]);
  d_dts_reset(H[1]);
  double W0[MP], W1[MP];
#pragma unroll
  for (int i = 0; i < MP; ++i) {
    W0[i] = Ur[i];
    W1[i] = Um[i];
  }
  bool redo = false, stop = false, finished = false;
  int l = 0, cnt = 0, status = 0, stage = S_PRED;
  double wstar[2] = {0.0, 0.0};
  unsigned nsolve = 0, nev = 0;

  for (;;) {
    // ---------------- the two interface solves (lane b: boundary b) ----------------
    const bool pred = stage == S_PRED;
    double ql0 = 0.0, ql1 = 0.0, qr0 = 0.0, qr1 = 0.0;
    {
      // this lane's boundary, selected (an array indexed by the lane would
      // live in scratch memory)
      const int iLm = me ? iL[1] : iL[0];
      const int a = pred ? iLm : (me ? ic[1] : ic[0]);
      const int c = pred ? iLm + 1 : (me ? icr[1] : icr[0]);
#pragma unroll
      for (int i = 0; i < MP; ++i) {
        const double x0 = pred ? Ur[i] : W0[i], x1 = pred ? Um[i] : W1[i];
        if (i == a) {
          ql0 = x0;
          ql1 = x1;
        }
        if (i == c) {
          qr0 = x0;
          qr1 = x1;
        }
      }
    }
    const int phl_me = me == 0 ? phl0 : (phl0 ^ 1);
    const bool hg = pred ? (me ? warm[1] : warm[0]) != 0 : true;
    const double g0 = pred ? (me ? rpw0[1] : rpw0[0]) : (me ? gn0[1] : gn0[0]);
    const double g1 = pred ? (me ? rpw1[1] : rpw1[0]) : (me ? gn1[1] : gn1[0]);
    IfaceOut o;
    const bool ok_me = d_iface_solve(M, P.newton_maxit, P.newton_rtol, phl_me, ql0, ql1,
                                     phl_me ^ 1, qr0, qr1, hg, g0, g1, o);
    if (ok_me) {
      ++nsolve;
      nev += (unsigned)o.nev;
    }
    // both boundaries' results on both lanes
    bool okb[2];
    double opl[2], opr[2], ow[2], oF0[2], oF1[2];
    {
      const int ok_o = zp_otheri(ok_me ? 1 : 0);
      const double pl_o = zp_other(o.pl), pr_o = zp_other(o.pr), w_o = zp_other(o.w);
      const double F0_o = zp_other(o.F0), F1_o = zp_other(o.F1);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const bool mine = b == me;
        okb[b] = mine ? ok_me : ok_o != 0;
        opl[b] = mine ? o.pl : pl_o;
        opr[b] = mine ? o.pr : pr_o;
        ow[b] = mine ? o.w : w_o;
        oF0[b] = mine ? o.F0 : F0_o;
        oF1[b] = mine ? o.F1 : F1_o;
      }
    }

    bool setup = false;
    if (pred) {
      if (!okb[0] || !okb[1]) {
        status = ST_NEWTON;
      } else {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          Ipl[b] = opl[b];
          Ipr[b] = opr[b];
          wp[b] = ow[b];
          const double ht = tr[b] ? h - hl[b] : hl[b];
          const double rate = tr[b] ? -wp[b] : wp[b];
          const double hfl = P.alpha_floor * h;
          merge[b] = (ht < hfl) || (ht + (P.merge_safety * rate) * dt < hfl);
        }
        setup = true;
      }
    } else if (!okb[0] || !okb[1]) {
      status = ST_NEWTON;
    } else {
      const bool part2 = stop || (l == P.lmax);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        pw0[b] = opl[b];
        pw1[b] = opr[b];
        d_dts_record(H[b], pw0[b], pw1[b], gn0[b], gn1[b]);
      }
      // right-face flux of every active position
      double FRa0[MP], FRa1[MP];
      const int cur0 = sL[0], cur1 = sL[1];
#pragma unroll
      for (int i = 0; i < MP; ++i) {
        FRa0[i] = 0.0;
        FRa1[i] = 0.0;
        if (i >= nr || i == skip[0] || i == skip[1]) continue;
        if (i == nr - 1) {
          FRa0[i] = FR0;
          FRa1[i] = FR1;
        } else if (i == ic[0]) {
          FRa0[i] = oF0[0];
          FRa1[i] = oF1[0];
        } else if (i == ic[1]) {
          FRa0[i] = oF0[1];
          FRa1[i] = oF1[1];
        } else if (i + 1 < MP) {
          d_hll(M, ph_of(i, cur0, cur1), W0[i], W1[i], W0[i + 1], W1[i + 1], FRa0[i], FRa1[i]);
        }
      }
      // new lengths of the four moving cells; collapse check (first position)
      double hnew_l[2], hnew_r[2], ih_l[2], ih_r[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        hnew_l[b] = hn_l[b] + (1.0 * ow[b]) * dt;
        hnew_r[b] = hn_r[b] + (-1.0 * ow[b]) * dt;
        ih_l[b] = 1.0 / hnew_l[b];
        ih_r[b] = 1.0 / hnew_r[b];
      }
      const double ih_f = 1.0 / (h + (0.0 * ow[0]) * dt);
      int shrink = MP;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (!(hnew_l[b] >= 0.5 * hh_l[b]) && ic[b] < shrink) shrink = ic[b];
        if (!(hnew_r[b] >= 0.5 * hh_r[b]) && icr[b] < shrink) shrink = icr[b];
      }
      if (shrink < MP) {
        // a tiny cell that collapsed: solve again with it merged (once per
        // boundary); any other collapse fails the zone
        bool again = false;
#pragma unroll
        for (int b = 0; b < 2; ++b)
          if (!merge[b] && shrink == tiny[b]) {
            merge[b] = true;
            again = true;
          }
        if (again) {
          redo = true;
          setup = true;
        } else {
          status = ST_MESH;
        }
      } else {
        // Part 1 pseudo step (eq. dual time tau diff, moving lengths) with the
        // stop test of Sec. 4 written without divisions; or Part 2
        const bool paper = P.tol_mode == 0;
        bool okw = true, conv = true;
#pragma unroll
        for (int i = 0; i < MP; ++i) {
          if (i >= nr || i == skip[0] || i == skip[1]) continue;
          double fl0, fl1;
          if (i == 0) {
            fl0 = FL0;
            fl1 = FL1;
          } else if (i >= 2 && (skip[0] == i - 1 || skip[1] == i - 1)) {
            fl0 = FRa0[i >= 2 ? i - 2 : 0];
            fl1 = FRa1[i >= 2 ? i - 2 : 0];
          } else {
            fl0 = FRa0[i - 1];
            fl1 = FRa1[i - 1];
          }
          const double u0r = (i == into[0]) ? Mr[0] : ((i == into[1]) ? Mr[1] : Ur[i]);
          const double u0m = (i == into[0]) ? Mm[0] : ((i == into[1]) ? Mm[1] : Um[i]);
          const double hni = (i == ic[0])    ? hn_l[0]
                             : (i == icr[0]) ? hn_r[0]
                             : (i == ic[1])  ? hn_l[1]
                             : (i == icr[1]) ? hn_r[1]
                                             : h;
          const double ihi = (i == ic[0])    ? ih_l[0]
                             : (i == icr[0]) ? ih_r[0]
                             : (i == ic[1])  ? ih_l[1]
                             : (i == icr[1]) ? ih_r[1]
                                             : ih_f;
          const double rhs0 = (hni * u0r - dt * (FRa0[i] - fl0)) * ihi;
          const double rhs1 = (hni * u0m - dt * (FRa1[i] - fl1)) * ihi;
          double n0, n1;
          if (part2) {
            n0 = rhs0;
            n1 = rhs1;
          } else {
            const double t = (i == ic[0])    ? th_l[0]
                             : (i == icr[0]) ? th_r[0]
                             : (i == ic[1])  ? th_l[1]
                             : (i == icr[1]) ? th_r[1]
                                             : th_f;
            const double i1 = (i == ic[0])    ? it_l[0]
                              : (i == icr[0]) ? it_r[0]
                              : (i == ic[1])  ? it_l[1]
                              : (i == icr[1]) ? it_r[1]
                                              : it_f;
            const double opt = 1.0 + t;
            const bool is_tiny = i == tiny[0] || i == tiny[1];
            const double thr = (is_tiny ? P.tol_tiny : P.tol_nb) * (t * dt);
            n0 = (W0[i] + t * rhs0) * i1;
            n1 = (W1[i] + t * rhs1) * i1;
            const double d0 = n0 - W0[i], d1 = n1 - W1[i];
            const double s0 = fabs(W0[i]) > 1.0 ? fabs(W0[i]) : 1.0;
            const double s1 = fabs(W1[i]) > 1.0 ? fabs(W1[i]) : 1.0;
            const bool c0 = paper ? fabs(opt * d0) < thr * s0 : fabs(d0) < P.tol_rel * s0;
            const bool c1 = paper ? fabs(opt * d1) < thr * s1 : fabs(d1) < P.tol_rel * s1;
            conv = conv && c0 && c1;
          }
          if (!d_state_ok(n0, n1)) okw = false;
          W0[i] = n0;
          W1[i] = n1;
        }
        if (!okw) {
          status = ST_NONPHYS;
        } else if (part2) {
          wstar[0] = ow[0];
          wstar[1] = ow[1];
          finished = true;
        } else {
          cnt = l + 1;
          ++l;
          stop = conv;
        }
      }
    }

    // ---------------- (re)build the zone: merges, lengths, pseudo steps ----------------
    if (setup && !status) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        skip[b] = -1;
        into[b] = -1;
        if (merge[b]) {
          skip[b] = tr[b] ? iL[b] + 1 : iL[b];
          into[b] = tr[b] ? iL[b] + 2 : iL[b] - 1;
          if (into[b] < 0 || into[b] >= nr) status = ST_MESH;
        }
      }
      if (!status) {
        // a merge into a piece of the other boundary's cut cell, or both
        // into one cell: the phase between the boundaries would vanish
        bool vanish = iL[0] + 1 >= iL[1];
#pragma unroll
        for (int b = 0; b < 2; ++b)
          if (into[b] >= 0 && (into[b] == iL[1 - b] || into[b] == iL[1 - b] + 1)) vanish = true;
        if (into[0] >= 0 && into[0] == into[1]) vanish = true;
        if (vanish) status = ST_VANISH;
      }
      if (!status) {
        const double hh_f = h + (0.0 * wp[0]) * dt;
        th_f = hh_f / h;
        if (th_f > P.theta_nb) th_f = P.theta_nb;
        it_f = 1.0 / (1.0 + th_f);
        bool bad = !(th_f > 0.0);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          double rskip = 0.0, mskip = 0.0, rin = 0.0, min_ = 0.0;
#pragma unroll
          for (int i = 0; i < MP; ++i) {
            if (i == skip[b]) {
              rskip = Ur[i];
              mskip = Um[i];
            }
            if (i == into[b]) {
              rin = Ur[i];
              min_ = Um[i];
            }
          }
          const double hLp = hl[b], hRp = h - hl[b];
          const double ht = tr[b] ? hRp : hLp;
          const double hm = h + ht;
          if (merge[b]) {
            Mr[b] = (h * rin + ht * rskip) / hm;
            Mm[b] = (h * min_ + ht * mskip) / hm;
          }
          ic[b] = (merge[b] && !tr[b]) ? into[b] : iL[b];
          icr[b] = (merge[b] && tr[b]) ? into[b] : iL[b] + 1;
          tiny[b] = merge[b] ? into[b] : (tr[b] ? iL[b] + 1 : iL[b]);
          hn_l[b] = (merge[b] && !tr[b]) ? hm : hLp;
          hn_r[b] = (merge[b] && tr[b]) ? hm : hRp;
          hh_l[b] = hn_l[b] + (1.0 * wp[b]) * dt;
          hh_r[b] = hn_r[b] + (-1.0 * wp[b]) * dt;
          th_l[b] = hh_l[b] / h;
          if (th_l[b] > P.theta_nb) th_l[b] = P.theta_nb;
          th_r[b] = hh_r[b] / h;
          if (th_r[b] > P.theta_nb) th_r[b] = P.theta_nb;
          it_l[b] = 1.0 / (1.0 + th_l[b]);
          it_r[b] = 1.0 / (1.0 + th_r[b]);
          bad = bad || !(th_l[b] > 0.0) || !(th_r[b] > 0.0);
          pw0[b] = Ipl[b];
          pw1[b] = Ipr[b];
          gn0[b] = Ipl[b];
          gn1[b] = Ipr[b];
          d_dts_reset(H[b]);
        }
#pragma unroll
        for (int i = 0; i < MP; ++i) {
          W0[i] = (i == into[0]) ? Mr[0] : ((i == into[1]) ? Mr[1] : Ur[i]);
          W1[i] = (i == into[0]) ? Mm[0] : ((i == into[1]) ? Mm[1] : Um[i]);
        }
        if (bad) status = ST_MESH;
        l = 0;
        cnt = 0;
        stop = false;
        stage = S_ITER;
      }
    }
    if (status || finished) break;
  }

  // ---------------- write-back (success or failure) ----------------
  double* r1 = A.rho1 + so;
  double* m1 = A.mom1 + so;
  int flags[2], nhome[2];
  double nhl[2];
  int count = 0;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    flags[b] = (tr[b] ? FL_TINY_RIGHT : 0) | FL_PAIR;
    nhome[b] = home[b];
    nhl[b] = hl[b];
  }
  if (finished) {
    // the interface advance and re-split of each boundary, in order
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const double hln = hl[b] + wstar[b] * dt;
      if (merge[b]) {
        flags[b] |= FL_MERGED;
        int src;  // position whose value fills the emptied piece
        if (!tr[b]) {
          if (hln < 0.0) {
            nhome[b] = home[b] - 1;
            nhl[b] = hln + h;
            src = iL[b] + 1;
            flags[b] |= FL_CROSS_L;
          } else {
            nhl[b] = hln;
            src = into[b];
          }
        } else {
          if (hln > h) {
            nhome[b] = home[b] + 1;
            nhl[b] = hln - h;
            src = iL[b];
            flags[b] |= FL_CROSS_R;
          } else {
            nhl[b] = hln;
            src = into[b];
          }
        }
        double cr = 0.0, cm = 0.0;
#pragma unroll
        for (int i = 0; i < MP; ++i)
          if (i == src) {
            cr = W0[i];
            cm = W1[i];
          }
#pragma unroll
        for (int i = 0; i < MP; ++i)
          if (i == skip[b]) {
            W0[i] = cr;
            W1[i] = cm;
          }
      } else {
        nhl[b] = hln;
      }
      if (redo) flags[b] |= FL_REDO;
      if (!stop) flags[b] |= FL_LMAX;
    }
    count = cnt;
  } else {
#pragma unroll
    for (int b = 0; b < 2; ++b) flags[b] |= FL_FAIL;
#pragma unroll
    for (int i = 0; i < MP; ++i) {
      W0[i] = Ur[i];
      W1[i] = Um[i];
    }
  }
  // lane b writes boundary b's record and log; lane 0 the cells
  {
    const int b = me, kb = k + me;
    if (finished) {
      A.rec_pw1[2 * kb] = pw0[b];
      A.rec_pw1[2 * kb + 1] = pw1[b];
      A.rec_warm1[kb] = 1;
      if (A.st_pseudo) atomicAdd(A.st_pseudo, (unsigned long long)count);
      if (merge[b] && A.st_merges) atomicAdd(A.st_merges, 1ull);
      if (!stop && A.st_lmax) atomicAdd(A.st_lmax, 1ull);
    } else {
      A.rec_pw1[2 * kb] = rpw0[b];
      A.rec_pw1[2 * kb + 1] = rpw1[b];
      A.rec_warm1[kb] = warm[b];
      if (b == 0) atomicOr(A.fail_acc + p, status);
    }
    if (A.st_newton) {
      atomicAdd(A.st_newton, (unsigned long long)nev);
      atomicAdd(A.st_solves, (unsigned long long)nsolve);
      const int ev = ((flags[b] & FL_MERGED) ? 1 : 0) + ((flags[b] & FL_REDO) ? 1 : 0) +
                     ((flags[b] & (FL_CROSS_L | FL_CROSS_R)) ? 1 : 0);
      if (ev) atomicAdd(A.st_events, (unsigned long long)ev);
      if (b == 0 && A.st_pairs) atomicAdd(A.st_pairs, 1ull);
    }
    A.rec_home1[kb] = nhome[b];
    A.rec_hl1[kb] = nhl[b];
    if (row >= 0) {
      const long long o2 = (long long)row * A.n_iface + kb;
      A.log_count[o2] = count;
      A.log_flags[o2] = flags[b];
      A.log_zlo[o2] = zlo;
    }
    if (A.tape) {
      double* T = A.tape + kb * A.tape_stride;
      T[TH_COUNT] = count;
      T[TH_FLAGS] = flags[b];
      T[TH_ZLO] = zlo;
      T[TH_WSTAR] = wstar[b];
    }
  }
  if (me == 0) {
    const int nsL0 = nhome[0] + kk, nsL1 = nhome[1] + kk + 1;
    unsigned long long vmax = 0;
#pragma unroll
    for (int i = 0; i < MP; ++i) {
      if (i < nr) {
        r1[zlo + i] = W0[i];
        m1[zlo + i] = W1[i];
        const unsigned long long sb = zp_speed_bits(M, ph_of(i, nsL0, nsL1), W0[i], W1[i]);
        vmax = sb > vmax ? sb : vmax;
      }
    }
    atomicMax(A.S_acc + p, vmax);
  }
}

hipError_t launch_zone_pair(const StepArgs& A, int if_begin, int if_end, hipStream_t s) {
  const int n = if_end - if_begin;
  if (n <= 1 || A.par.zone_solver != 0) return hipSuccess;
  const int blocks = (n + 31) / 32;
  switch (A.par.zone_half) {
    case 1: k_zone_pair<1><<<blocks, 64, 0, s>>>(A, if_begin, if_end); break;
    case 2: k_zone_pair<2><<<blocks, 64, 0, s>>>(A, if_begin, if_end); break;
    case 3: k_zone_pair<3><<<blocks, 64, 0, s>>>(A, if_begin, if_end); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace imexds
