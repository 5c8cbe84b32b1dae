// imexds_zone8.hip -- implicit zones with eight lanes per zone (gfx950).
//
// Same computation as k_zone (prediction of the boundary speed, merge test,
// Algorithm 2 Part 1 and Part 2 with moving cut cells, interface advance and
// re-split), with the work of one zone spread over an 8-lane group so that
// each lane's instruction stream per pseudo iteration is short:
//   * lane c holds active zone cell c (the cells of the zone range without
//     the merged-away piece, left to right): its iterate, U^n, h^n, theta;
//   * lane c computes the flux on the face to its right (HLL; the zone's
//     F_right on the last cell) and takes its left-face flux from lane c-1;
//   * the interface solve runs on the two lanes next to the phase boundary,
//     one outer wave each (d_iface_solve_t<true>), and its flux and speed are
//     broadcast to the group;
//   * the stop test is an AND over the group.
// Every operation is the one k_zone (and the CPU oracle) performs, in the same
// order, so results are bit for bit those of k_zone.  A wave holds up to
// eight groups (the launch's zones per group); groups fetch zones from the
// shared counter until none is left.
#include "imexds_device.hpp"
#include "imexds_kernels.hpp"

namespace imexds {

namespace {

__device__ __forceinline__ unsigned long long z8_bits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}

__device__ __forceinline__ unsigned long long z8_speed_bits(const Mat& M, int ph, double r,
                                                            double m) {
  if (!d_state_ok(r, m)) return 0x7FF8000000000000ull;
  return z8_bits(fabs(m / r) + d_a(M, ph));
}

// value of lane gb + c of this lane's group
__device__ __forceinline__ double z8_get(double x, int gb, int c) { return __shfl(x, gb + c, 64); }
__device__ __forceinline__ int z8_geti(int x, int gb, int c) { return __shfl(x, gb + c, 64); }

// group-wide AND / OR of a per-lane flag (lanes of the group only)
__device__ __forceinline__ bool z8_all(bool v, int gb) {
  const unsigned long long b = __ballot(v ? 1 : 0);
  return ((b >> gb) & 0xffull) == 0xffull;
}
__device__ __forceinline__ bool z8_any(bool v, int gb) {
  const unsigned long long b = __ballot(v ? 1 : 0);
  return ((b >> gb) & 0xffull) != 0ull;
}

__device__ __forceinline__ unsigned long long z8_max_u64(unsigned long long v) {
#pragma unroll
  for (int off = 4; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 8);
    v = o > v ? o : v;
  }
  return v;
}

}  // namespace

template <int ZH>
__global__ __launch_bounds__(64) void k_zone8(StepArgs A, int if_begin, int if_end) {
  constexpr int MC = 2 * ZH + 1;
  constexpr int S_FETCH = 0, S_PRED = 1, S_ITER = 2, S_EXIT = 3;
  static_assert(MC <= 8, "a zone must fit an 8-lane group");
  // The material constants are read in every pass of the dual time loop.
  // Uniform values live in scalar registers, which this kernel runs out of
  // (the spills cost a v_readlane each in the loop); it has vector registers
  // to spare at its occupancy.
  const Mat Mv = d_mat_vregs(A.mat);
  const Mat& M = Mv;
  const Par& P = A.par;
  const int lane = threadIdx.x;
  const double tol_nb = P.tol_nb, tol_tiny = P.tol_tiny;
  const int c = lane & 7;       // cell (lane) index inside the group
  const int gb = lane & ~7;     // first lane of the group
  // zone groups per wave: A.zones_per_group clamped to 1..8 (fewer groups
  // per wave: less divergence between zones, more waves)
  const int gpw = A.zones_per_group < 1 ? 1 : (A.zones_per_group > 8 ? 8 : A.zones_per_group);
  if ((lane >> 3) >= gpw) return;  // whole groups leave together

  // group-wide (identical on the 8 lanes)
  int k = 0, p = 0, kk = 0, ns = 0, sL = 0, zlo = 0, nr = 0, iL = 0, iR = 1, m = 0;
  long long so = 0;
  double h = 0.0, dt = 0.0, hl = 0.0, rpw0 = 0.0, rpw1 = 0.0;
  int phl = 0, phr = 1, home = 0, warm = 0, row = -1;
  bool tr = false, merge = false, redo = false, stop = false;
  int skip = -1, into = -1, ic = 0, tiny = 0, l = 0, cnt = 0;
  double FL0 = 0.0, FL1 = 0.0, FR0 = 0.0, FR1 = 0.0, Ipl = 0.0, Ipr = 0.0, wp = 0.0;
  double pw0 = 0.0, pw1 = 0.0, hh_l = 0.0, hh_r = 0.0;
  // start of the next pass's interface solve and the roots it comes from
  // (identical on the group's lanes)
  double gn0 = 0.0, gn1 = 0.0;
  DtsRoots H;
  d_dts_reset(H);
  // per lane: U^n of zone position c (and of position c + 1), and the active cell c
  double Ur = 1.0, Um = 0.0, nUr = 1.0, nUm = 0.0, Uu = 0.0, nUu = 0.0;
  int pos = -1;  // zone position of active cell c (-1: lane idle)
  double W0 = 1.0, W1 = 0.0, U00 = 1.0, U01 = 0.0, hn = 0.0, th = 0.0, it1 = 0.0, mv = 0.0;
  double tol = 0.0;
  int ph = 0;
  int stage = S_FETCH;
  // per lane: interface solves this lane led (side 0) in the current zone
  // step and their evaluations of G (summed over the group at write-back)
  unsigned nsolve = 0, nev = 0;
  // the first zone of a group is its own index in the grid, further ones come
  // from the counter: 4096 groups pulling from one address at once would
  // queue behind each other for tens of microseconds
  const int g_self = (int)blockIdx.x * gpw + (lane >> 3);
  const int g_all = (int)gridDim.x * gpw;
  bool first = true;

  for (;;) {
    // ---------------- fetch a zone ----------------
    while (stage == S_FETCH) {
      int t = 0;
      if (c == 0) t = first ? g_self : g_all + atomicAdd(A.zone_ctr, 1);
      first = false;
      k = if_begin + z8_geti(t, gb, 0);
      if (k >= if_end) {
        stage = S_EXIT;
        break;
      }
      p = A.iface_prob[k];
      kk = A.iface_local[k];
      dt = A.dt[p];
      home = A.rec_home0[k];
      hl = A.rec_hl0[k];
      rpw0 = A.rec_pw0[2 * k];
      rpw1 = A.rec_pw0[2 * k + 1];
      warm = A.rec_warm0[k];
      row = -1;
      if (A.log_count && A.log_row) {
        row = *A.log_row;
        if (row >= A.log_max) row = -1;
      }
      so = A.slot_off[p];
      ns = (int)(A.slot_off[p + 1] - so);
      sL = home + kk;
      if (dt == 0.0 || sL < 0 || sL + 1 >= ns) {
        if (c == 0) {
          if (dt != 0.0) atomicOr(A.fail_acc + p, ST_MESH);
          A.rec_home1[k] = home;
          A.rec_hl1[k] = hl;
          A.rec_pw1[2 * k] = rpw0;
          A.rec_pw1[2 * k + 1] = rpw1;
          A.rec_warm1[k] = warm;
          if (row >= 0) {
            long long o = (long long)row * A.n_iface + k;
            A.log_count[o] = 0;
            A.log_flags[o] = dt == 0.0 ? FL_INACTIVE : FL_FAIL;
            A.log_zlo[o] = -1;
          }
          if (A.tape) A.tape[k * A.tape_stride + TH_FLAGS] = dt == 0.0 ? FL_INACTIVE : FL_FAIL;
        }
        continue;
      }
      h = A.h[p];
      {
        // an interface whose zone overlaps a neighbour's is solved with it
        // in one zone by k_zone_pair
        const int nif = A.iface_off[p + 1] - A.iface_off[p];
        if (d_pair_lead(A, k - 1, kk - 1, nif, ns, h) || d_pair_lead(A, k, kk, nif, ns, h))
          continue;
      }
      phl = A.phase_first[p] ^ (kk & 1);
      phr = phl ^ 1;
      int zhi;
      d_zone_range(sL, hl, h, ZH, ns, zlo, zhi, tr);
      nr = zhi - zlo + 1;
      iL = sL - zlo;
      iR = iL + 1;
      const double* r0 = A.rho0 + so;
      const double* m0 = A.mom0 + so;
      Ur = 1.0;
      Um = 0.0;
      if (c < nr) {
        Ur = r0[zlo + c];
        Um = m0[zlo + c];
      }
      nUr = d_lane_next(Ur);
      nUm = d_lane_next(Um);
      Uu = Um / Ur;
      nUu = d_lane_next(Uu);
      // bounding fluxes from U^n: F_left on lane 0, F_right on lane 1
      {
        double f0 = 0.0, f1 = 0.0;
        if (c == 0) {
          const int phz = (zlo <= sL) ? phl : phr;
          if (zlo == 0)
            d_bflux(M, phz, false, P.bc_left, r0[0], m0[0], f0, f1);
          else
            d_hll(M, phz, r0[zlo - 1], m0[zlo - 1], r0[zlo], m0[zlo], f0, f1);
        } else if (c == 1) {
          const int phe = (zhi <= sL) ? phl : phr;
          if (zhi == ns - 1)
            d_bflux(M, phe, true, P.bc_right, r0[ns - 1], m0[ns - 1], f0, f1);
          else
            d_hll(M, phe, r0[zhi], m0[zhi], r0[zhi + 1], m0[zhi + 1], f0, f1);
        }
        FL0 = z8_get(f0, gb, 0);
        FL1 = z8_get(f1, gb, 0);
        FR0 = z8_get(f0, gb, 1);
        FR1 = z8_get(f1, gb, 1);
      }
      merge = false;
      redo = false;
      pos = -1;
      nsolve = 0;
      nev = 0;
      stage = S_PRED;
    }
    if (stage == S_EXIT) break;
    // the right neighbour's iterate for this pass's HLL flux, read ahead of the
    // interface solve (which leaves it unchanged) so the exchange overlaps it
    const double nW0 = d_lane_next(W0);
    const double nW1 = d_lane_next(W1);
    // the lane's velocity and its right neighbour's, for the HLL flux and the
    // interface solve's set-up
    const double uo = W1 / W0;
    const double nu = d_lane_next(uo);

    // ---------------- one interface solve (two lanes of the group) ----------------
    const bool pred = stage == S_PRED;
    // prediction: zone positions iL, iR hold the two sides; iteration:
    // active cells ic, ic + 1.  The pair solve runs on an even lane and the
    // odd one after it (its exchanges are DPP quad permutations): on a0, a0 + 1
    // for an even a0, else on a0 - 1, a0, which take their states from the
    // right neighbour's values (U^n of the next zone position, the next
    // active cell's iterate).
    const int a0 = pred ? iL : ic;
    const int p0 = a0 & ~1;
    const bool shifted = (a0 & 1) != 0;
    int side = -1;
    if (c == p0) side = 0;
    if (c == p0 + 1) side = 1;
    IfaceOut o;
    o.pl = o.pr = o.rl = o.rr = o.ul = o.ur = o.z = o.w = o.F0 = o.F1 = 0.0;
    o.nev = 0;
    int okl = 0;
    if (side >= 0) {
      const double x0 = pred ? (shifted ? nUr : Ur) : (shifted ? nW0 : W0);
      const double x1 = pred ? (shifted ? nUm : Um) : (shifted ? nW1 : W1);
      const double xu = pred ? (shifted ? nUu : Uu) : (shifted ? nu : uo);
      const bool hg = pred ? warm != 0 : true;
      const double g0 = pred ? rpw0 : gn0, g1 = pred ? rpw1 : gn1;
      okl = d_iface_solve_t<true>(M, P.newton_maxit, P.newton_rtol, phl, x0, x1, phr, x0, x1, hg,
                                  g0, g1, side, o, true, xu)
                ? 1
                : 0;
      if (side == 0 && okl) {
        ++nsolve;
        nev += (unsigned)o.nev;
      }
    }
    const bool ok = z8_geti(okl, gb, a0) != 0;
    const double opl = z8_get(o.pl, gb, a0), opr = z8_get(o.pr, gb, a0);
    const double ow = z8_get(o.w, gb, a0), oF0 = z8_get(o.F0, gb, a0),
                 oF1 = z8_get(o.F1, gb, a0);

    // ---------------- stage-specific work ----------------
    int status = 0;
    bool setup = false, finished = false;
    double wstar = 0.0;
    if (pred) {
      if (!ok) {
        status = ST_NEWTON;
      } else {
        Ipl = opl;
        Ipr = opr;
        wp = ow;
        if (A.tape && c == 0) {
          double* T = A.tape + k * A.tape_stride;
          T[TH_IPL] = Ipl;
          T[TH_IPR] = Ipr;
          T[TH_WP] = wp;
        }
        const double ht = tr ? h - hl : hl;
        const double rate = tr ? -wp : wp;
        const double hfl = P.alpha_floor * h;
        merge = (ht < hfl) || (ht + (P.merge_safety * rate) * dt < hfl);
        setup = true;
      }
    } else if (!ok) {
      status = ST_NEWTON;
    } else {
      const bool part2 = stop || (l == P.lmax);
      pw0 = opl;
      pw1 = opr;
      d_dts_record(H, pw0, pw1, gn0, gn1);
      const double w = ow;
      if (A.tape) {  // W^l (by zone position) and its interface root
        double* e = A.tape + k * A.tape_stride + TAPE_HDR + (long long)l * (2 * MC + 2);
        if (pos >= 0) {
          e[pos] = W0;
          e[MC + pos] = W1;
        }
        if (c == 0) {
          e[2 * MC] = pw0;
          e[2 * MC + 1] = pw1;
        }
      }
      // flux on the right face of cell c, left face from lane c - 1
      double Fr0 = 0.0, Fr1 = 0.0;
      if (c < m) {
        if (c == m - 1) {
          Fr0 = FR0;
          Fr1 = FR1;
        } else if (c == ic) {
          Fr0 = oF0;
          Fr1 = oF1;
        } else {
          d_hll_prim(d_a(M, ph), W0, W1, uo, d_pres(M, ph, W0), nW0, nW1, nu, d_pres(M, ph, nW0),
                     Fr0, Fr1);
        }
      }
      double Fl0 = d_lane_prev(Fr0);
      double Fl1 = d_lane_prev(Fr1);
      if (c == 0) {
        Fl0 = FL0;
        Fl1 = FL1;
      }
      // new lengths of the two moving cells; collapse check
      const double hnew = hn + (mv * w) * dt;
      const double ih = 1.0 / hnew;
      bool shr = false;
      if (c == ic) shr = !(hnew >= 0.5 * hh_l);
      if (c == ic + 1) shr = !(hnew >= 0.5 * hh_r);
      const bool bl = z8_any(shr && c == ic, gb), br = z8_any(shr && c == ic + 1, gb);
      int shrink = -1;  // zone position
      // zone position of active cell q: the set-up's pos of lane q
      auto pos_of = [&](int q) { return q < m ? ((skip >= 0 && q >= skip) ? q + 1 : q) : -1; };
      {
        const int pic = pos_of(ic), pir = pos_of(ic + 1);
        if (bl && br)
          shrink = pic < pir ? pic : pir;
        else if (bl)
          shrink = pic;
        else if (br)
          shrink = pir;
      }
      if (shrink >= 0) {
        const int ptiny = pos_of(tiny);
        if (!merge && shrink == ptiny) {
          merge = true;
          redo = true;
          setup = true;
        } else {
          status = ST_MESH;
        }
      } else {
        // Part 1 pseudo step (eq. dual time tau diff, moving lengths) with the
        // stop test of Sec. 4; or Part 2, the conservative update
        const bool paper = P.tol_mode == 0;
        bool okw = true, conv = true;
        if (c < m) {
          const double rhs0 = (hn * U00 - dt * (Fr0 - Fl0)) * ih;
          const double rhs1 = (hn * U01 - dt * (Fr1 - Fl1)) * ih;
          double n0, n1;
          if (part2) {
            n0 = rhs0;
            n1 = rhs1;
          } else {
            const double opt = 1.0 + th;
            const double thr = tol * (th * dt);
            n0 = (W0 + th * rhs0) * it1;
            n1 = (W1 + th * rhs1) * it1;
            const double d0 = n0 - W0, d1 = n1 - W1;
            const double s0 = fabs(W0) > 1.0 ? fabs(W0) : 1.0;
            const double s1 = fabs(W1) > 1.0 ? fabs(W1) : 1.0;
            const bool c0 = paper ? fabs(opt * d0) < thr * s0 : fabs(d0) < P.tol_rel * s0;
            const bool c1 = paper ? fabs(opt * d1) < thr * s1 : fabs(d1) < P.tol_rel * s1;
            conv = c0 && c1;
          }
          okw = d_state_ok(n0, n1);
          W0 = n0;
          W1 = n1;
        }
        okw = z8_all(okw, gb);
        conv = z8_all(conv, gb);
        if (!okw) {
          status = ST_NONPHYS;
        } else if (part2) {
          wstar = w;
          finished = true;
        } else {
          cnt = l + 1;
          ++l;
          stop = conv;
        }
      }
    }

    // ---------------- (re)build the zone: merge, lengths, pseudo steps ----------------
    if (setup && !status) {
      skip = -1;
      into = -1;
      if (merge) {
        skip = tr ? iR : iL;
        into = tr ? iR + 1 : iL - 1;
        if (into < 0 || into >= nr) status = ST_MESH;
      }
      if (!status) {
        m = merge ? nr - 1 : nr;
        pos = (c < m) ? ((skip >= 0 && c >= skip) ? c + 1 : c) : -1;
        const double rpos = z8_get(Ur, gb, pos >= 0 ? pos : 0);
        const double mpos = z8_get(Um, gb, pos >= 0 ? pos : 0);
        const double rskip = z8_get(Ur, gb, skip >= 0 ? skip : 0);
        const double mskip = z8_get(Um, gb, skip >= 0 ? skip : 0);
        const double hLp = hl, hRp = h - hl;
        const double ht = tr ? hRp : hLp;
        const double hm = h + ht;
        // active-cell indices of the two cells next to the boundary and of the
        // tiny (or merged) cell
        const int ic_pos = (merge && !tr) ? into : iL;
        ic = (skip >= 0 && ic_pos > skip) ? ic_pos - 1 : ic_pos;
        const int tpos = merge ? into : (tr ? iR : iL);
        tiny = (skip >= 0 && tpos > skip) ? tpos - 1 : tpos;
        const double hn_l = (merge && !tr) ? hm : hLp;
        const double hn_r = (merge && tr) ? hm : hRp;
        hh_l = hn_l + (1.0 * wp) * dt;
        hh_r = hn_r + (-1.0 * wp) * dt;
        const double hh_f = h + (0.0 * wp) * dt;
        double th_l = hh_l / h;
        if (th_l > P.theta_nb) th_l = P.theta_nb;
        double th_r = hh_r / h;
        if (th_r > P.theta_nb) th_r = P.theta_nb;
        double th_f = hh_f / h;
        if (th_f > P.theta_nb) th_f = P.theta_nb;
        const double it_l = 1.0 / (1.0 + th_l), it_r = 1.0 / (1.0 + th_r);
        const double it_f = 1.0 / (1.0 + th_f);
        const bool bad = !(th_l > 0.0) || !(th_r > 0.0) || !(th_f > 0.0);
        if (pos >= 0) {
          if (pos == into) {
            U00 = (h * rpos + ht * rskip) / hm;
            U01 = (h * mpos + ht * mskip) / hm;
          } else {
            U00 = rpos;
            U01 = mpos;
          }
          W0 = U00;
          W1 = U01;
          hn = (c == ic) ? hn_l : ((c == ic + 1) ? hn_r : h);
          mv = (c == ic) ? 1.0 : ((c == ic + 1) ? -1.0 : 0.0);
          th = (c == ic) ? th_l : ((c == ic + 1) ? th_r : th_f);
          it1 = (c == ic) ? it_l : ((c == ic + 1) ? it_r : it_f);
          tol = tol_nb;
          if (c == tiny) tol = tol_tiny;
          ph = (zlo + pos <= sL) ? phl : phr;
        } else {
          W0 = 1.0;
          W1 = 0.0;
          U00 = 1.0;
          U01 = 0.0;
          hn = h;
          mv = 0.0;
          th = th_f;
          it1 = it_f;
          tol = tol_nb;
          ph = phl;
        }
        if (bad) status = ST_MESH;
        pw0 = Ipl;
        pw1 = Ipr;
        gn0 = Ipl;
        gn1 = Ipr;
        d_dts_reset(H);
        l = 0;
        cnt = 0;
        stop = false;
        stage = S_ITER;
      }
    }

    if (!status && !finished) continue;

    // ---------------- write-back (success or failure) ----------------
    double* r1 = A.rho1 + so;
    double* m1 = A.mom1 + so;
    int flags = tr ? FL_TINY_RIGHT : 0;
    int count = 0;
    int nhome = home;
    double nhl = hl;
    unsigned long long vmax = 0;
    if (finished) {
      const double hln = hl + wstar * dt;
      int src = -1;  // zone position whose value fills the emptied piece
      if (merge) {
        flags |= FL_MERGED;
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
      } else {
        nhl = hln;
      }
      if (redo) flags |= FL_REDO;
      if (!stop) flags |= FL_LMAX;
      count = cnt;
      const int nsL = nhome + kk;
      if (pos >= 0) {
        r1[zlo + pos] = W0;
        m1[zlo + pos] = W1;
        vmax = z8_speed_bits(M, (zlo + pos <= nsL) ? phl : phr, W0, W1);
        if (pos == src) {
          r1[zlo + skip] = W0;
          m1[zlo + skip] = W1;
          const unsigned long long b2 =
              z8_speed_bits(M, (zlo + skip <= nsL) ? phl : phr, W0, W1);
          vmax = b2 > vmax ? b2 : vmax;
        }
      }
      if (c == 0) {
        A.rec_pw1[2 * k] = pw0;
        A.rec_pw1[2 * k + 1] = pw1;
        A.rec_warm1[k] = 1;
        if (A.st_pseudo) atomicAdd(A.st_pseudo, (unsigned long long)count);
        if (merge && A.st_merges) atomicAdd(A.st_merges, 1ull);
        if (!stop && A.st_lmax) atomicAdd(A.st_lmax, 1ull);
      }
    } else {
      flags |= FL_FAIL;
      const int nsL = nhome + kk;
      if (c < nr) {  // the zone keeps U^n
        r1[zlo + c] = Ur;
        m1[zlo + c] = Um;
        vmax = z8_speed_bits(M, (zlo + c <= nsL) ? phl : phr, Ur, Um);
      }
      if (c == 0) {
        A.rec_pw1[2 * k] = rpw0;
        A.rec_pw1[2 * k + 1] = rpw1;
        A.rec_warm1[k] = warm;
        atomicOr(A.fail_acc + p, status);
      }
    }
    vmax = z8_max_u64(vmax);
    if (A.st_newton) {
      unsigned long long sv = ((unsigned long long)nsolve << 32) | nev;
#pragma unroll
      for (int off = 4; off > 0; off >>= 1) sv += __shfl_xor(sv, off, 8);
      if (c == 0) {
        atomicAdd(A.st_newton, sv & 0xffffffffull);
        atomicAdd(A.st_solves, sv >> 32);
        const int ev = ((flags & FL_MERGED) ? 1 : 0) + ((flags & FL_REDO) ? 1 : 0) +
                       ((flags & (FL_CROSS_L | FL_CROSS_R)) ? 1 : 0);
        if (ev) atomicAdd(A.st_events, (unsigned long long)ev);
      }
    }
    if (c == 0) {
      A.rec_home1[k] = nhome;
      A.rec_hl1[k] = nhl;
      atomicMax(A.S_acc + p, vmax);
      if (row >= 0) {
        long long o2 = (long long)row * A.n_iface + k;
        A.log_count[o2] = count;
        A.log_flags[o2] = flags;
        A.log_zlo[o2] = zlo;
      }
      if (A.tape) {
        double* T = A.tape + k * A.tape_stride;
        T[TH_COUNT] = count;
        T[TH_FLAGS] = flags;
        T[TH_ZLO] = zlo;
        T[TH_WSTAR] = wstar;
      }
    }
    stage = S_FETCH;
  }
}

hipError_t launch_zone8(const StepArgs& A, int if_begin, int if_end, int groups, hipStream_t s) {
  const int n = if_end - if_begin;
  if (n <= 0) return hipSuccess;
  const int gpw = A.zones_per_group < 1 ? 1 : (A.zones_per_group > 8 ? 8 : A.zones_per_group);
  const int need = (n + gpw - 1) / gpw;  // waves of gpw zone groups
  if (groups <= 0 || groups > need) groups = need;
  switch (A.par.zone_half) {
    case 1: k_zone8<1><<<groups, 64, 0, s>>>(A, if_begin, if_end); break;
    case 2: k_zone8<2><<<groups, 64, 0, s>>>(A, if_begin, if_end); break;
    case 3: k_zone8<3><<<groups, 64, 0, s>>>(A, if_begin, if_end); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace imexds
