// imexds_kernels.hip -- gfx950 kernels of one IMEX-DS physical step.
//
// One step of every problem is three launches:
//   k_bulk   (tiles of cells)  : Algorithm 1 Step 1 -- HLL fluxes on the faces
//                                of every cell outside the implicit zones and
//                                the explicit update of those cells; fused
//                                epilogue: per-problem max(|u| + a) of the new
//                                state (CFL, eq. cfl_cond:unif) via one 64-bit
//                                atomicMax per wave.
//   k_zone   (lanes pull zones): prediction of the boundary speed, merge test,
//                                Algorithm 2 (Part 1 dual time stepping with
//                                local pseudo steps, Part 2 conservative update
//                                with moving cut cells), interface advance and
//                                re-split; CFL contribution of its cells.
//   k_finalize (one lane / problem): t += dt, status, next dt, overlap test.
// k_bulk and k_zone read only U^n and write disjoint slots of U^{n+1}, so they
// run concurrently on two streams.
#include "imexds_device.hpp"
#include "imexds_kernels.hpp"

namespace imexds {

__device__ __forceinline__ unsigned long long d_bits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}

constexpr unsigned long long NAN_BITS = 0x7FF8000000000000ull;

// CFL contribution of one cell: |m / rho| + a, or a NaN pattern (which wins
// every unsigned max against a finite non-negative double) if non-physical.
__device__ __forceinline__ unsigned long long d_speed_bits(const Mat& M, int ph, double r,
                                                           double m) {
  if (!d_state_ok(r, m)) return NAN_BITS;
  return d_bits(fabs(m / r) + d_a(M, ph));
}

__device__ __forceinline__ unsigned long long d_wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// ---------------------------------------------------------------------------
// bulk sweep
// ---------------------------------------------------------------------------
// A workgroup is 4 waves; each wave handles R rows of 62 cells.  In a row,
// lane j holds cell base-1+j (lane 0 and lane 63 are the halo), computes the
// flux on the face to its right from its own and its right neighbour's
// values (exchanged with a lane shuffle), takes the flux of its left face
// from lane j-1, and lanes 1..62 update their cell.  No LDS tile, no
// barrier in the sweep: occupancy stays high and all R rows' loads are in
// flight together.
template <int R>
__global__ __launch_bounds__(256) void k_bulk(StepArgs A, int tile_begin) {
  constexpr int OUT = 62;
  __shared__ int s_zlo[MAX_IF_PER_PROB], s_zhi[MAX_IF_PER_PROB], s_sR[MAX_IF_PER_PROB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int tile = tile_begin + blockIdx.x;
  const int p = A.tile_prob[tile];
  const int t0 = A.tile_start[tile];
  const int tend = t0 + A.tile_len[tile];
  const long long so = A.slot_off[p];
  const int ns = (int)(A.slot_off[p + 1] - so);
  const double* __restrict__ r0 = A.rho0 + so;
  const double* __restrict__ m0 = A.mom0 + so;
  double* __restrict__ r1 = A.rho1 + so;
  double* __restrict__ m1 = A.mom1 + so;
  const double dt = A.dt[p];

  if (dt == 0.0) {  // frozen or finished: carry the state over
    for (int c = t0 + tid; c < tend; c += 256) {
      r1[c] = r0[c];
      m1[c] = m0[c];
    }
    return;
  }
  const Mat& M = A.mat;
  const double h = A.h[p];
  const double lam = dt / h;
  const int i0 = A.iface_off[p];
  const int nif = A.iface_off[p + 1] - i0;
  const int pf = A.phase_first[p];
  const bool wallL = A.par.bc_left == 0, wallR = A.par.bc_right == 0;
  if (tid < nif) {
    int zlo, zhi;
    bool tr;
    int sL = A.rec_home0[i0 + tid] + tid;
    d_zone_range(sL, A.rec_hl0[i0 + tid], h, A.par.zone_half, ns, zlo, zhi, tr);
    s_zlo[tid] = zlo;
    s_zhi[tid] = zhi;
    s_sR[tid] = sL + 1;
  }
  __syncthreads();

  // loads of all rows first
  double rr[R], mm[R];
  int ss[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int s = t0 + (wv * R + r) * OUT - 1 + lane;
    ss[r] = s;
    int se = s < 0 ? 0 : (s > ns - 1 ? ns - 1 : s);
    double rv = r0[se], mv = m0[se];
    if ((s < 0 && wallL) || (s >= ns && wallR)) mv = -mv;
    rr[r] = rv;
    mm[r] = mv;
  }

  unsigned long long vmax = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int s = ss[r];
    const int rowbase = t0 + (wv * R + r) * OUT;
    if (rowbase >= tend) break;  // uniform over the wave
    const int se = s < 0 ? 0 : (s > ns - 1 ? ns - 1 : s);
    int ph = pf;
    bool zone = false;
    for (int j = 0; j < nif; ++j) {
      ph ^= (s_sR[j] <= se) ? 1 : 0;
      zone = zone || (s >= s_zlo[j] && s <= s_zhi[j]);
    }
    const double rho = rr[r], mom = mm[r];
    const double u = mom / rho;
    const double pr = d_pres(M, ph, rho);
    const double rhoR = d_wave_next(rho);
    const double momR = d_wave_next(mom);
    const double uR = d_wave_next(u);
    const double prR = d_wave_next(pr);
    double F0, F1;  // flux on the face between s and s+1 (phase of s)
    d_hll_prim(d_a(M, ph), rho, mom, u, pr, rhoR, momR, uR, prR, F0, F1);
    const double G0 = d_wave_prev(F0);
    const double G1 = d_wave_prev(F1);
    if (lane >= 1 && lane <= OUT && s < tend && !zone) {
      double rn = rho - lam * (F0 - G0);
      double mn = mom - lam * (F1 - G1);
      r1[s] = rn;
      m1[s] = mn;
      unsigned long long b = d_speed_bits(M, ph, rn, mn);
      vmax = b > vmax ? b : vmax;
    }
  }
  vmax = d_wave_max_u64(vmax);
  if (lane == 0 && vmax) atomicMax(A.S_acc + p, vmax);
}

// CFL over all slots of the current state (first step after a state load).
__global__ __launch_bounds__(256) void k_cfl(StepArgs A, int tile_begin) {
  __shared__ int s_sR[MAX_IF_PER_PROB];
  const int tid = threadIdx.x;
  const int tile = tile_begin + blockIdx.x;
  const int p = A.tile_prob[tile];
  const int t0 = A.tile_start[tile];
  const int len = A.tile_len[tile];
  const long long so = A.slot_off[p];
  const int i0 = A.iface_off[p];
  const int nif = A.iface_off[p + 1] - i0;
  const int pf = A.phase_first[p];
  if (tid < nif) s_sR[tid] = A.rec_home0[i0 + tid] + tid + 1;
  __syncthreads();
  unsigned long long vmax = 0;
  for (int c = tid; c < len; c += 256) {
    int s = t0 + c;
    int ph = pf;
    for (int j = 0; j < nif; ++j) ph ^= (s_sR[j] <= s) ? 1 : 0;
    unsigned long long b = d_speed_bits(A.mat, ph, A.rho0[so + s], A.mom0[so + s]);
    vmax = b > vmax ? b : vmax;
  }
  vmax = d_wave_max_u64(vmax);
  if ((tid & 63) == 0 && vmax) atomicMax(A.S_acc + p, vmax);
}

// ---------------------------------------------------------------------------
// implicit zones
// ---------------------------------------------------------------------------
// Each active lane runs a state machine: fetch a zone (atomic counter), solve
// the predicting Riemann problem, then one pseudo-time iteration per pass
// (each pass ends with Part 2 when the stop test or lmax says so), then the
// write-back, and fetch the next zone.  Every pass calls the interface solver
// exactly once, so all lanes of a wave execute the same solver code together
// whatever zone or iteration they are at.  Zone cells are addressed by their
// position 0..nr-1 in the slot range zlo..zhi; the merged-away piece (if
// any) is position `skip` and its content sits in position `into`.
template <int ZH>
__global__ __launch_bounds__(64) void k_zone(StepArgs A, int if_begin, int if_end) {
  constexpr int MC = 2 * ZH + 1;
  constexpr int S_FETCH = 0, S_PRED = 1, S_ITER = 2, S_EXIT = 3;
  if ((int)threadIdx.x >= A.zones_per_group) return;
  const Mat& M = A.mat;
  const Par& P = A.par;

  int k = 0, p = 0, kk = 0, ns = 0, sL = 0, zlo = 0, nr = 0, iL = 0, iR = 1;
  long long so = 0;
  double h = 0.0, dt = 0.0;
  int phl = 0, phr = 1;
  bool tr = false;
  int home = 0, warm = 0;
  double hl = 0.0, rpw0 = 0.0, rpw1 = 0.0;
  double Ur[MC], Um[MC];  // U^n over the zone range
  double FL0 = 0.0, FL1 = 0.0, FR0 = 0.0, FR1 = 0.0;
  double Ipl = 0.0, Ipr = 0.0, wp = 0.0;
  bool merge = false, redo = false;
  int skip = -1, into = -1, ic = 0, icr = 1, tiny = 0;
  double Mr = 0.0, Mm = 0.0;  // U^n of the merged cell (position into)
  // Only the two cells next to the boundary (positions ic, icr) move; every
  // other zone cell has length h and theta = min(theta_nb, 1).
  double hn_l = 0.0, hn_r = 0.0, th_l = 0.0, th_r = 0.0, it_l = 0.0, it_r = 0.0;
  double hh_l = 0.0, hh_r = 0.0;  // predicted end lengths of positions ic, icr
  double th_f = 0.0, it_f = 0.0;  // theta and 1/(1+theta) of a fixed full cell
  double W0[MC], W1[MC];
  double pw0 = 0.0, pw1 = 0.0;
  // start of the next pass's interface solve and the roots it comes from
  double gn0 = 0.0, gn1 = 0.0;
  DtsRoots H;
  d_dts_reset(H);
  int l = 0, cnt = 0;
  bool stop = false;
  int row = -1;
#pragma unroll
  for (int i = 0; i < MC; ++i) Ur[i] = Um[i] = W0[i] = W1[i] = 0.0;
  int stage = S_FETCH;
  unsigned nsolve = 0, nev = 0;  // interface solves of this zone step, evaluations of G
  // first zone: the lane's own index in the grid; then the counter
  const int g_self = (int)blockIdx.x * A.zones_per_group + (int)threadIdx.x;
  const int g_all = (int)gridDim.x * A.zones_per_group;
  bool first = true;

  for (;;) {
    // ---------------- fetch a zone that needs work ----------------
    while (stage == S_FETCH) {
      k = if_begin + (first ? g_self : g_all + atomicAdd(A.zone_ctr, 1));
      first = false;
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
        // frozen/finished (or a record outside its problem: freeze, touch nothing)
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
#pragma unroll
      for (int i = 0; i < MC; ++i) {
        if (i < nr) {
          Ur[i] = r0[zlo + i];
          Um[i] = m0[zlo + i];
        } else {
          Ur[i] = 1.0;
          Um[i] = 0.0;
        }
      }
      // bounding fluxes from U^n (Algorithm 1: F_left, F_right)
      int phz = (zlo <= sL) ? phl : phr;
      if (zlo == 0)
        d_bflux(M, phz, false, P.bc_left, r0[0], m0[0], FL0, FL1);
      else
        d_hll(M, phz, r0[zlo - 1], m0[zlo - 1], r0[zlo], m0[zlo], FL0, FL1);
      int phe = (zhi <= sL) ? phl : phr;
      if (zhi == ns - 1)
        d_bflux(M, phe, true, P.bc_right, r0[ns - 1], m0[ns - 1], FR0, FR1);
      else
        d_hll(M, phe, r0[zhi], m0[zhi], r0[zhi + 1], m0[zhi + 1], FR0, FR1);
      merge = false;
      redo = false;
      nsolve = 0;
      nev = 0;
      stage = S_PRED;
    }
    if (stage == S_EXIT) break;

    // ---------------- one interface Riemann solve ----------------
    double ql0 = 0.0, ql1 = 0.0, qr0 = 0.0, qr1 = 0.0, g0, g1;
    bool hg;
    {
      const bool pred = stage == S_PRED;
      const int a = pred ? iL : ic, b = pred ? iR : icr;
#pragma unroll
      for (int i = 0; i < MC; ++i) {
        const double x0 = pred ? Ur[i] : W0[i], x1 = pred ? Um[i] : W1[i];
        if (i == a) {
          ql0 = x0;
          ql1 = x1;
        }
        if (i == b) {
          qr0 = x0;
          qr1 = x1;
        }
      }
      hg = pred ? warm != 0 : true;
      g0 = pred ? rpw0 : gn0;
      g1 = pred ? rpw1 : gn1;
    }
    IfaceOut o;
    const bool ok = d_iface_solve(M, P.newton_maxit, P.newton_rtol, phl, ql0, ql1, phr, qr0, qr1,
                                  hg, g0, g1, o);
    if (ok) {
      ++nsolve;
      nev += (unsigned)o.nev;
    }

    // ---------------- stage-specific work ----------------
    int status = 0;
    bool setup = false, finished = false;
    double wstar = 0.0;
    if (stage == S_PRED) {
      if (!ok) {
        status = ST_NEWTON;
      } else {
        Ipl = o.pl;
        Ipr = o.pr;
        wp = o.w;
        if (A.tape) {
          double* T = A.tape + k * A.tape_stride;
          T[TH_IPL] = Ipl;
          T[TH_IPR] = Ipr;
          T[TH_WP] = wp;
        }
        double ht = tr ? h - hl : hl;
        double rate = tr ? -wp : wp;
        double hfl = P.alpha_floor * h;
        merge = (ht < hfl) || (ht + (P.merge_safety * rate) * dt < hfl);
        setup = true;
      }
    } else if (!ok) {
      status = ST_NEWTON;
    } else {
      const bool part2 = stop || (l == P.lmax);
      pw0 = o.pl;
      pw1 = o.pr;
      d_dts_record(H, pw0, pw1, gn0, gn1);
      const double w = o.w;
      if (A.tape) {  // W^l and its interface root
        double* e = A.tape + k * A.tape_stride + TAPE_HDR + (long long)l * (2 * MC + 2);
#pragma unroll
        for (int i = 0; i < MC; ++i) {
          e[i] = W0[i];
          e[MC + i] = W1[i];
        }
        e[2 * MC] = pw0;
        e[2 * MC + 1] = pw1;
      }
      // fluxes of the iterate: right face of each active position
      double FRa0[MC], FRa1[MC];
#pragma unroll
      for (int i = 0; i < MC; ++i) {
        FRa0[i] = 0.0;
        FRa1[i] = 0.0;
        if (i >= nr || i == skip) continue;
        if (i == nr - 1) {
          FRa0[i] = FR0;
          FRa1[i] = FR1;
        } else if (i == ic) {
          FRa0[i] = o.F0;
          FRa1[i] = o.F1;
        } else if (i + 1 < MC) {
          int ph = (zlo + i <= sL) ? phl : phr;
          d_hll(M, ph, W0[i], W1[i], W0[i + 1], W1[i + 1], FRa0[i], FRa1[i]);
        }
      }
      // new lengths (only the two cells next to the boundary move); collapse check
      const double hnew_l = hn_l + (1.0 * w) * dt;
      const double hnew_r = hn_r + (-1.0 * w) * dt;
      const double ih_l = 1.0 / hnew_l, ih_r = 1.0 / hnew_r;
      const double ih_f = 1.0 / (h + (0.0 * w) * dt);
      int shrink = -1;
      {
        const bool bl = !(hnew_l >= 0.5 * hh_l), br = !(hnew_r >= 0.5 * hh_r);
        if (bl && br)
          shrink = ic < icr ? ic : icr;
        else if (bl)
          shrink = ic;
        else if (br)
          shrink = icr;
      }
      if (shrink >= 0) {
        if (!merge && shrink == tiny) {
          merge = true;
          redo = true;
          setup = true;
        } else {
          status = ST_MESH;
        }
      } else {
        // Part 1 pseudo step (eq. dual time tau diff, moving lengths) with the
        // stop test of Sec. 4 written without divisions:
        //   |(1 + theta) d| < tol_i (theta dt) max(|W|, 1)  per component;
        // or Part 2: the conservative update from the accepted iterate.
        const bool paper = P.tol_mode == 0;
        bool okw = true, conv = true;
#pragma unroll
        for (int i = 0; i < MC; ++i) {
          if (i >= nr || i == skip) continue;
          double fl0, fl1;
          if (i == 0) {
            fl0 = FL0;
            fl1 = FL1;
          } else if (i >= 2 && skip == i - 1) {
            fl0 = FRa0[i >= 2 ? i - 2 : 0];
            fl1 = FRa1[i >= 2 ? i - 2 : 0];
          } else {
            fl0 = FRa0[i - 1];
            fl1 = FRa1[i - 1];
          }
          const double u0r = (i == into) ? Mr : Ur[i];
          const double u0m = (i == into) ? Mm : Um[i];
          const double hni = (i == ic) ? hn_l : ((i == icr) ? hn_r : h);
          const double ihi = (i == ic) ? ih_l : ((i == icr) ? ih_r : ih_f);
          const double rhs0 = (hni * u0r - dt * (FRa0[i] - fl0)) * ihi;
          const double rhs1 = (hni * u0m - dt * (FRa1[i] - fl1)) * ihi;
          double n0, n1;
          if (part2) {
            n0 = rhs0;
            n1 = rhs1;
          } else {
            const double t = (i == ic) ? th_l : ((i == icr) ? th_r : th_f);
            const double i1 = (i == ic) ? it_l : ((i == icr) ? it_r : it_f);
            const double opt = 1.0 + t;
            const double thr = (i == tiny ? P.tol_tiny : P.tol_nb) * (t * dt);
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
        // lengths at t^n, predicted end lengths and pseudo steps
        // theta = min(theta_nb, h_end / h) (Sec. 4: theta_k = alpha, 0.9 otherwise)
        hn_l = (merge && !tr) ? hm : hLp;
        hn_r = (merge && tr) ? hm : hRp;
        hh_l = hn_l + (1.0 * wp) * dt;
        hh_r = hn_r + (-1.0 * wp) * dt;
        const double hh_f = h + (0.0 * wp) * dt;
        th_l = hh_l / h;
        if (th_l > P.theta_nb) th_l = P.theta_nb;
        th_r = hh_r / h;
        if (th_r > P.theta_nb) th_r = P.theta_nb;
        th_f = hh_f / h;
        if (th_f > P.theta_nb) th_f = P.theta_nb;
        it_l = 1.0 / (1.0 + th_l);
        it_r = 1.0 / (1.0 + th_r);
        it_f = 1.0 / (1.0 + th_f);
        bool bad = !(th_l > 0.0) || !(th_r > 0.0) || !(th_f > 0.0);
#pragma unroll
        for (int i = 0; i < MC; ++i) {
          W0[i] = (i == into) ? Mr : Ur[i];
          W1[i] = (i == into) ? Mm : Um[i];
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
    if (finished) {
      double hln = hl + wstar * dt;
      if (merge) {
        flags |= FL_MERGED;
        int src;  // position whose value fills the emptied piece
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
      if (!stop) flags |= FL_LMAX;
      count = cnt;
      A.rec_pw1[2 * k] = pw0;
      A.rec_pw1[2 * k + 1] = pw1;
      A.rec_warm1[k] = 1;
      if (A.st_pseudo) atomicAdd(A.st_pseudo, (unsigned long long)count);
      if (merge && A.st_merges) atomicAdd(A.st_merges, 1ull);
      if (!stop && A.st_lmax) atomicAdd(A.st_lmax, 1ull);
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
    if (A.st_newton) {
      atomicAdd(A.st_newton, (unsigned long long)nev);
      atomicAdd(A.st_solves, (unsigned long long)nsolve);
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
        int ph = (zlo + i <= nsL) ? phl : phr;
        unsigned long long b = d_speed_bits(M, ph, W0[i], W1[i]);
        vmax = b > vmax ? b : vmax;
      }
    }
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
    stage = S_FETCH;
  }
}

// ---------------------------------------------------------------------------
// per-problem bookkeeping between steps
// ---------------------------------------------------------------------------
__global__ void k_finalize(StepArgs A, int p_begin, int p_end, int init, int bump_row) {
  const int p = p_begin + blockIdx.x * blockDim.x + threadIdx.x;
  if (p == p_begin) {
    if (bump_row && A.log_row) *A.log_row += 1;
    *A.zone_ctr = 0;
  }
  if (p >= p_end) return;
  const Par& P = A.par;
  double dt = A.dt[p];
  int st = A.status[p];
  double t = A.t[p];
  if (!init && dt > 0.0) {
    int f = A.fail_acc[p];
    if (f)
      st |= f;
    else {
      t = A.clipped[p] ? P.t_end : t + dt;
      A.steps[p] += 1;
    }
  }
  double ndt = 0.0;
  int clip = 0;
  if (st == 0 && t < P.t_end) {
    double S = __longlong_as_double((long long)A.S_acc[p]);
    if (!(S > 0.0) || !d_finite(S)) {
      st |= ST_NONPHYS;
    } else {
      const long long so = A.slot_off[p];
      const int ns = (int)(A.slot_off[p + 1] - so);
      const int i0 = A.iface_off[p], nif = A.iface_off[p + 1] - i0;
      const double h = A.h[p];
      // zones must be disjoint, except that with Algorithm 2 the zones of
      // two neighbouring interfaces may overlap (solved as one zone)
      int prev_hi = -1;
      for (int j = 0; j < nif;) {
        int zlo, zhi;
        bool tr;
        d_zone_range(A.rec_home1[i0 + j] + j, A.rec_hl1[i0 + j], h, P.zone_half, ns, zlo, zhi, tr);
        if (zlo <= prev_hi) {
          st |= ST_OVERLAP;
          break;
        }
        int nb = 1;
        if (j + 1 < nif && P.zone_solver == 0) {
          int zlo1, zhi1;
          bool tr1;
          d_zone_range(A.rec_home1[i0 + j + 1] + j + 1, A.rec_hl1[i0 + j + 1], h, P.zone_half, ns,
                       zlo1, zhi1, tr1);
          if (zlo1 <= zhi) {
            nb = 2;
            zhi = zhi1;
          }
        }
        prev_hi = zhi;
        j += nb;
      }
      if (st == 0) {
        ndt = (P.cfl * h) / S;
        double rem = P.t_end - t;
        if (ndt >= rem) {
          ndt = rem;
          clip = 1;
        }
      }
    }
  }
  A.dt[p] = st == 0 ? ndt : 0.0;
  A.t[p] = t;
  A.status[p] = st;
  A.clipped[p] = clip;
  A.S_acc[p] = 0ull;
  A.fail_acc[p] = 0;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
int bulk_tile_cells(int tile_class) { return (tile_class / 256) * 4 * 62; }

hipError_t launch_bulk(const StepArgs& A, int tile_class, int tile_begin, int n_tiles,
                       hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  switch (tile_class) {
    case 256: k_bulk<1><<<n_tiles, 256, 0, s>>>(A, tile_begin); break;
    case 512: k_bulk<2><<<n_tiles, 256, 0, s>>>(A, tile_begin); break;
    case 1024: k_bulk<4><<<n_tiles, 256, 0, s>>>(A, tile_begin); break;
    case 2048: k_bulk<8><<<n_tiles, 256, 0, s>>>(A, tile_begin); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cfl(const StepArgs& A, int tile_begin, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  k_cfl<<<n_tiles, 256, 0, s>>>(A, tile_begin);
  return hipGetLastError();
}

hipError_t launch_zone(const StepArgs& A, int if_begin, int if_end, int groups, hipStream_t s) {
  int n = if_end - if_begin;
  if (n <= 0) return hipSuccess;
  int need = (n + A.zones_per_group - 1) / A.zones_per_group;
  if (groups <= 0 || groups > need) groups = need;
  switch (A.par.zone_half) {
    case 1: k_zone<1><<<groups, 64, 0, s>>>(A, if_begin, if_end); break;
    case 2: k_zone<2><<<groups, 64, 0, s>>>(A, if_begin, if_end); break;
    case 3: k_zone<3><<<groups, 64, 0, s>>>(A, if_begin, if_end); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The per-step records of a recorded step copied into its tape slot: the
// interface cells and cut lengths (N each), dt, the clip flag and the step
// counter (P each).  One launch instead of five copies.
__global__ void k_tape_copy(const int* home, const double* hl, const double* dt, const int* clip,
                            const long long* steps, int* t_home, double* t_hl, double* t_dt,
                            int* t_clip, long long* t_steps, int N, int P) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) {
    t_home[i] = home[i];
    t_hl[i] = hl[i];
  }
  if (i < P) {
    t_dt[i] = dt[i];
    t_clip[i] = clip[i];
    t_steps[i] = steps[i];
  }
}

hipError_t launch_tape_copy(const int* home, const double* hl, const double* dt, const int* clip,
                            const long long* steps, int* t_home, double* t_hl, double* t_dt,
                            int* t_clip, long long* t_steps, int N, int P, hipStream_t s) {
  const int n = N > P ? N : P;
  if (n <= 0) return hipSuccess;
  k_tape_copy<<<(n + 255) / 256, 256, 0, s>>>(home, hl, dt, clip, steps, t_home, t_hl, t_dt,
                                              t_clip, t_steps, N, P);
  return hipGetLastError();
}

hipError_t launch_finalize(const StepArgs& A, int p_begin, int p_end, int init, int bump_row,
                           hipStream_t s) {
  int n = p_end - p_begin;
  int blocks = n > 0 ? (n + 255) / 256 : 1;
  k_finalize<<<blocks, 256, 0, s>>>(A, p_begin, p_end, init, bump_row);
  return hipGetLastError();
}

}  // namespace imexds
