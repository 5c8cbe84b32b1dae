// imexds_kernels.hip -- gfx950 kernels of one IMEX-DS physical step.
//
// One step of every problem is three launches:
//   k_bulk   (tiles of cells)  : Algorithm 1 Step 1 -- HLL fluxes on every face
//                                next to a cell outside the implicit zones and
//                                the explicit update of those cells; fused
//                                epilogue: per-problem max(|u| + a) of the new
//                                state (CFL, eq. cfl_cond:unif) via one 64-bit
//                                atomicMax per workgroup.
//   k_zone   (one lane / zone) : prediction of the boundary speed, merge test,
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
template <int CPT>
__global__ __launch_bounds__(256) void k_bulk(StepArgs A, int tile_begin) {
  constexpr int T = 256 * CPT;
  __shared__ double s_r[T + 2], s_m[T + 2], s_u[T + 2], s_p[T + 2];
  __shared__ double s_F0[T + 1], s_F1[T + 1];
  __shared__ int s_zlo[MAX_IF_PER_PROB], s_zhi[MAX_IF_PER_PROB], s_sR[MAX_IF_PER_PROB];
  __shared__ unsigned long long s_red[4];

  const int tid = threadIdx.x;
  const int tile = tile_begin + blockIdx.x;
  const int p = A.tile_prob[tile];
  const int t0 = A.tile_start[tile];
  const int len = A.tile_len[tile];
  const long long so = A.slot_off[p];
  const int ns = (int)(A.slot_off[p + 1] - so);
  const double* __restrict__ r0 = A.rho0 + so;
  const double* __restrict__ m0 = A.mom0 + so;
  double* __restrict__ r1 = A.rho1 + so;
  double* __restrict__ m1 = A.mom1 + so;
  const double dt = A.dt[p];

  if (dt == 0.0) {  // frozen or finished: carry the state over
    for (int c = tid; c < len; c += 256) {
      r1[t0 + c] = r0[t0 + c];
      m1[t0 + c] = m0[t0 + c];
    }
    return;
  }
  const Mat& M = A.mat;
  const double h = A.h[p];
  const double lam = dt / h;
  const int i0 = A.iface_off[p];
  const int nif = A.iface_off[p + 1] - i0;
  const int pf = A.phase_first[p];
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

  auto phase_of = [&](int s) {
    int ph = pf;
    for (int j = 0; j < nif; ++j) ph ^= (s_sR[j] <= s) ? 1 : 0;
    return ph;
  };
  auto in_zone = [&](int s) {
    bool z = false;
    for (int j = 0; j < nif; ++j) z = z || (s >= s_zlo[j] && s <= s_zhi[j]);
    return z;
  };

  // stage the tile and a one-cell halo (ghost states at the domain ends)
  for (int i = tid; i < len + 2; i += 256) {
    int s = t0 - 1 + i;
    double r, m;
    int ph;
    if (s < 0) {
      r = r0[0];
      m = (A.par.bc_left == 0) ? -m0[0] : m0[0];
      ph = phase_of(0);
    } else if (s >= ns) {
      r = r0[ns - 1];
      m = (A.par.bc_right == 0) ? -m0[ns - 1] : m0[ns - 1];
      ph = phase_of(ns - 1);
    } else {
      r = r0[s];
      m = m0[s];
      ph = phase_of(s);
    }
    s_r[i] = r;
    s_m[i] = m;
    s_u[i] = m / r;
    s_p[i] = d_pres(M, ph, r);
  }
  __syncthreads();

  // face i lies between staged entries i and i+1 (slots t0-1+i and t0+i)
  for (int i = tid; i < len + 1; i += 256) {
    int sl = t0 - 1 + i, sr = t0 + i;
    bool need = (sl >= 0 && !in_zone(sl)) || (sr < ns && !in_zone(sr));
    if (need) {
      int ph = phase_of(sl >= 0 ? sl : sr);
      double F0, F1;
      d_hll_prim(d_a(M, ph), s_r[i], s_m[i], s_u[i], s_p[i], s_r[i + 1], s_m[i + 1], s_u[i + 1],
                 s_p[i + 1], F0, F1);
      s_F0[i] = F0;
      s_F1[i] = F1;
    }
  }
  __syncthreads();

  unsigned long long vmax = 0;
  for (int c = tid; c < len; c += 256) {
    int s = t0 + c;
    if (in_zone(s)) continue;
    double r = s_r[c + 1] - lam * (s_F0[c + 1] - s_F0[c]);
    double m = s_m[c + 1] - lam * (s_F1[c + 1] - s_F1[c]);
    r1[s] = r;
    m1[s] = m;
    unsigned long long b = d_speed_bits(M, phase_of(s), r, m);
    vmax = b > vmax ? b : vmax;
  }
  vmax = d_wave_max_u64(vmax);
  if ((tid & 63) == 0) s_red[tid >> 6] = vmax;
  __syncthreads();
  if (tid == 0) {
    unsigned long long v = s_red[0];
    for (int w = 1; w < 4; ++w) v = s_red[w] > v ? s_red[w] : v;
    if (v) atomicMax(A.S_acc + p, v);
  }
}

// CFL over all slots of the current state (first step after a state load).
template <int CPT>
__global__ __launch_bounds__(256) void k_cfl(StepArgs A, int tile_begin) {
  __shared__ int s_sR[MAX_IF_PER_PROB];
  __shared__ unsigned long long s_red[4];
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
  if ((tid & 63) == 0) s_red[tid >> 6] = vmax;
  __syncthreads();
  if (tid == 0) {
    unsigned long long v = s_red[0];
    for (int w = 1; w < 4; ++w) v = s_red[w] > v ? s_red[w] : v;
    if (v) atomicMax(A.S_acc + p, v);
  }
}

// ---------------------------------------------------------------------------
// implicit zones
// ---------------------------------------------------------------------------
// Interface flux of a zone iterate; warm start in/out through pw.
__device__ __noinline__ bool d_zone_iface(const Mat& M, const Par& P, int phl, double rl, double ml,
                                          int phr, double rr, double mr, double& pw0, double& pw1,
                                          double& F0, double& F1, double& w) {
  IfaceOut o;
  if (!d_iface_solve(M, P.newton_maxit, P.newton_rtol, phl, rl, ml, phr, rr, mr, true, pw0, pw1,
                     o))
    return false;
  pw0 = o.pl;
  pw1 = o.pr;
  F0 = o.F0;
  F1 = o.F1;
  w = o.w;
  return true;
}

template <int ZH>
__global__ __launch_bounds__(64) void k_zone(StepArgs A, int if_begin, int if_end) {
  constexpr int MC = 2 * ZH + 1;
  const int lane = threadIdx.x;
  if (lane >= A.zones_per_group) return;
  const int k = if_begin + blockIdx.x * A.zones_per_group + lane;
  if (k >= if_end) return;
  const Mat& M = A.mat;
  const Par& P = A.par;
  const int p = A.iface_prob[k];
  const int kk = A.iface_local[k];
  const double dt = A.dt[p];
  int home = A.rec_home0[k];
  double hl = A.rec_hl0[k];
  double pwa = A.rec_pw0[2 * k], pwb = A.rec_pw0[2 * k + 1];
  int warm = A.rec_warm0[k];
  int row = -1;
  if (A.log_count && A.log_row) {
    row = *A.log_row;
    if (row >= A.log_max) row = -1;
  }
  if (dt == 0.0) {
    A.rec_home1[k] = home;
    A.rec_hl1[k] = hl;
    A.rec_pw1[2 * k] = pwa;
    A.rec_pw1[2 * k + 1] = pwb;
    A.rec_warm1[k] = warm;
    if (row >= 0) {
      long long o = (long long)row * A.n_iface + k;
      A.log_count[o] = 0;
      A.log_flags[o] = FL_INACTIVE;
      A.log_zlo[o] = -1;
    }
    return;
  }
  const long long so = A.slot_off[p];
  const int ns = (int)(A.slot_off[p + 1] - so);
  const double h = A.h[p];
  const double* __restrict__ r0 = A.rho0 + so;
  const double* __restrict__ m0 = A.mom0 + so;
  double* __restrict__ r1 = A.rho1 + so;
  double* __restrict__ m1 = A.mom1 + so;
  const int sL = home + kk, sR = sL + 1;
  if (sL < 0 || sR >= ns) {  // interface record outside its problem: freeze, touch nothing
    atomicOr(A.fail_acc + p, ST_MESH);
    A.rec_home1[k] = home;
    A.rec_hl1[k] = hl;
    A.rec_pw1[2 * k] = pwa;
    A.rec_pw1[2 * k + 1] = pwb;
    A.rec_warm1[k] = warm;
    return;
  }
  const int phl = A.phase_first[p] ^ (kk & 1), phr = phl ^ 1;
  int zlo, zhi;
  bool tr;
  d_zone_range(sL, hl, h, ZH, ns, zlo, zhi, tr);
  const int nr = zhi - zlo + 1;
  const int iL = sL - zlo, iR = iL + 1;

  double Ur[MC], Um[MC];
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
  double FL0, FL1, FR0, FR1;
  {
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
  }

  int status = 0, flags = tr ? FL_TINY_RIGHT : 0, count = 0;
  bool merge = false, redo = false, lmax_hit = false;
  double wstar = 0.0;
  double U1r[MC], U1m[MC];
  int skip = -1, into = -1;
  // prediction of the boundary speed from U^n
  double Ipl = 0.0, Ipr = 0.0, wp = 0.0;
  {
    double F0, F1;
    double g0 = pwa, g1 = pwb;
    IfaceOut o;
    if (!d_iface_solve(M, P.newton_maxit, P.newton_rtol, phl, r0[sL], m0[sL], phr, r0[sR], m0[sR],
                       warm != 0, g0, g1, o)) {
      status = ST_NEWTON;
    } else {
      Ipl = o.pl;
      Ipr = o.pr;
      wp = o.w;
    }
    (void)F0;
    (void)F1;
  }
  if (!status) {
    double ht = tr ? h - hl : hl;
    double rate = tr ? -wp : wp;
    double hfl = P.alpha_floor * h;
    merge = (ht < hfl) || (ht + (P.merge_safety * rate) * dt < hfl);
  }

  for (int attempt = 0; attempt < 2 && !status; ++attempt) {
    // ---- zone set-up in range positions 0..nr-1 ----
    skip = -1;
    into = -1;
    if (merge) {
      skip = tr ? iR : iL;
      into = tr ? iR + 1 : iL - 1;
      if (into < 0 || into >= nr) {
        status = ST_MESH;
        break;
      }
    }
    double U0r[MC], U0m[MC], hn[MC], hh[MC], th[MC];
    int mov[MC];
    bool act[MC];
    double rskip = 0.0, mskip = 0.0;
    if (merge) {
      rskip = r0[zlo + skip];
      mskip = m0[zlo + skip];
    }
    const double hLp = hl, hRp = h - hl;
    bool bad = false;
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      act[i] = (i < nr) && (i != skip);
      U0r[i] = Ur[i];
      U0m[i] = Um[i];
      hn[i] = h;
      mov[i] = 0;
      if (i == iL) {
        hn[i] = hLp;
        mov[i] = 1;
      } else if (i == iR) {
        hn[i] = hRp;
        mov[i] = -1;
      }
      if (i == into) {
        double ht = tr ? hRp : hLp;
        double hm = h + ht;
        U0r[i] = (h * Ur[i] + ht * rskip) / hm;
        U0m[i] = (h * Um[i] + ht * mskip) / hm;
        hn[i] = hm;
        mov[i] = tr ? -1 : 1;
      }
      double hx = hn[i] + ((double)mov[i] * wp) * dt;
      double t = hx / h;
      if (t > P.theta_nb) t = P.theta_nb;
      hh[i] = hx;
      th[i] = t;
      if (act[i] && !(t > 0.0)) bad = true;
    }
    if (bad) {
      status = ST_MESH;
      break;
    }
    // interface between active positions ic (left) and icr (right)
    const int ic = (merge && !tr) ? into : iL;
    const int icr = (merge && tr) ? into : iR;
    const int tiny = merge ? into : (tr ? iR : iL);
    int last = nr - 1;

    double W0[MC], W1[MC];
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      W0[i] = U0r[i];
      W1[i] = U0m[i];
    }
    double pw0 = Ipl, pw1 = Ipr;
    int shrink = -1;
    bool stop = false;
    int cnt = 0;
    double w = 0.0;
    // ---- Part 1: pseudo-time iterations, then Part 2 with l == lmax marker ----
    for (int l = 0; l <= P.lmax; ++l) {
      const bool part2 = (l == P.lmax) || stop;
      // fluxes of the iterate
      double Wl0 = 0.0, Wl1 = 0.0, Wr0 = 0.0, Wr1 = 0.0;
#pragma unroll
      for (int i = 0; i < MC; ++i) {
        if (i == ic) {
          Wl0 = W0[i];
          Wl1 = W1[i];
        }
        if (i == icr) {
          Wr0 = W0[i];
          Wr1 = W1[i];
        }
      }
      double Fi0, Fi1;
      if (!d_zone_iface(M, P, phl, Wl0, Wl1, phr, Wr0, Wr1, pw0, pw1, Fi0, Fi1, w)) {
        status = ST_NEWTON;
        break;
      }
      double FR0a[MC], FR1a[MC];  // flux on the right face of each active position
#pragma unroll
      for (int i = 0; i < MC; ++i) {
        FR0a[i] = 0.0;
        FR1a[i] = 0.0;
        if (!act[i]) continue;
        if (i == last) {
          FR0a[i] = FR0;
          FR1a[i] = FR1;
        } else if (i == ic) {
          FR0a[i] = Fi0;
          FR1a[i] = Fi1;
        } else if (i + 1 < MC) {
          int ph = (zlo + i <= sL) ? phl : phr;
          d_hll(M, ph, W0[i], W1[i], W0[i + 1], W1[i + 1], FR0a[i], FR1a[i]);
        }
      }
      double hnew[MC];
#pragma unroll
      for (int i = 0; i < MC; ++i) {
        hnew[i] = hn[i] + ((double)mov[i] * w) * dt;
        if (shrink < 0 && act[i] && mov[i] != 0 && !(hnew[i] >= 0.5 * hh[i])) shrink = i;
      }
      if (shrink >= 0) {
        status = ST_MESH;
        break;
      }
      if (part2) {
        bool okp = true;
#pragma unroll
        for (int i = 0; i < MC; ++i) {
          if (!act[i]) continue;
          double fl0, fl1;
          if (i == 0) {
            fl0 = FL0;
            fl1 = FL1;
          } else if (i >= 2 && skip == i - 1) {
            fl0 = FR0a[i >= 2 ? i - 2 : 0];
            fl1 = FR1a[i >= 2 ? i - 2 : 0];
          } else {
            fl0 = FR0a[i - 1];
            fl1 = FR1a[i - 1];
          }
          U1r[i] = (hn[i] * U0r[i] - dt * (FR0a[i] - fl0)) / hnew[i];
          U1m[i] = (hn[i] * U0m[i] - dt * (FR1a[i] - fl1)) / hnew[i];
          if (!d_state_ok(U1r[i], U1m[i])) okp = false;
        }
        if (!okp) status = ST_NONPHYS;
        wstar = w;
        break;
      }
      // Part 1 update (eq. dual time tau diff with moving lengths) and residuals
      double N0[MC], N1[MC];
      double rmax_nb = 0.0, r_tiny = 0.0, rrel = 0.0;
      bool okw = true;
#pragma unroll
      for (int i = 0; i < MC; ++i) {
        N0[i] = W0[i];
        N1[i] = W1[i];
        if (!act[i]) continue;
        double fl0, fl1;
        if (i == 0) {
          fl0 = FL0;
          fl1 = FL1;
        } else if (i >= 2 && skip == i - 1) {
          fl0 = FR0a[i >= 2 ? i - 2 : 0];
          fl1 = FR1a[i >= 2 ? i - 2 : 0];
        } else {
          fl0 = FR0a[i - 1];
          fl1 = FR1a[i - 1];
        }
        const double t = th[i];
        double rc = 0.0, rr = 0.0;
        {
          double rhs = (hn[i] * U0r[i] - dt * (FR0a[i] - fl0)) / hnew[i];
          N0[i] = (W0[i] + t * rhs) / (1.0 + t);
          double d = N0[i] - W0[i];
          double sc = fabs(W0[i]) > 1.0 ? fabs(W0[i]) : 1.0;
          double res = fabs((1.0 + t) * d) / ((t * dt) * sc);
          double rel = fabs(d) / sc;
          if (res > rc) rc = res;
          if (rel > rr) rr = rel;
        }
        {
          double rhs = (hn[i] * U0m[i] - dt * (FR1a[i] - fl1)) / hnew[i];
          N1[i] = (W1[i] + t * rhs) / (1.0 + t);
          double d = N1[i] - W1[i];
          double sc = fabs(W1[i]) > 1.0 ? fabs(W1[i]) : 1.0;
          double res = fabs((1.0 + t) * d) / ((t * dt) * sc);
          double rel = fabs(d) / sc;
          if (res > rc) rc = res;
          if (rel > rr) rr = rel;
        }
        if (!d_state_ok(N0[i], N1[i])) okw = false;
        if (i == tiny)
          r_tiny = rc;
        else if (rc > rmax_nb)
          rmax_nb = rc;
        if (rr > rrel) rrel = rr;
      }
      if (!okw) {
        status = ST_NONPHYS;
        break;
      }
#pragma unroll
      for (int i = 0; i < MC; ++i) {
        W0[i] = N0[i];
        W1[i] = N1[i];
      }
      cnt = l + 1;
      if (P.tol_mode == 0)
        stop = (rmax_nb < P.tol_nb) && (r_tiny < P.tol_tiny);
      else
        stop = rrel < P.tol_rel;
    }
    if (status == ST_MESH && !merge && shrink == tiny && attempt == 0) {
      status = 0;
      merge = true;
      redo = true;
      continue;
    }
    if (status) break;
    lmax_hit = !stop;
    count = cnt;
    pwa = pw0;
    pwb = pw1;
    break;
  }

  // ---- write back ----
  double Fr[MC], Fm[MC];
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    Fr[i] = Ur[i];
    Fm[i] = Um[i];
  }
  int nhome = home;
  double nhl = hl;
  if (!status) {
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      if (i < nr && i != skip) {
        Fr[i] = U1r[i];
        Fm[i] = U1m[i];
      }
    }
    double hln = hl + wstar * dt;
    if (merge) {
      flags |= FL_MERGED;
      double cr = 0.0, cm = 0.0;  // value copied into the emptied piece
      if (!tr) {
        if (hln < 0.0) {
          nhome = home - 1;
          nhl = hln + h;
#pragma unroll
          for (int i = 0; i < MC; ++i)
            if (i == iR) {
              cr = Fr[i];
              cm = Fm[i];
            }
          flags |= FL_CROSS_L;
        } else {
#pragma unroll
          for (int i = 0; i < MC; ++i)
            if (i == into) {
              cr = Fr[i];
              cm = Fm[i];
            }
          nhl = hln;
        }
      } else {
        if (hln > h) {
          nhome = home + 1;
          nhl = hln - h;
#pragma unroll
          for (int i = 0; i < MC; ++i)
            if (i == iL) {
              cr = Fr[i];
              cm = Fm[i];
            }
          flags |= FL_CROSS_R;
        } else {
#pragma unroll
          for (int i = 0; i < MC; ++i)
            if (i == into) {
              cr = Fr[i];
              cm = Fm[i];
            }
          nhl = hln;
        }
      }
#pragma unroll
      for (int i = 0; i < MC; ++i)
        if (i == skip) {
          Fr[i] = cr;
          Fm[i] = cm;
        }
    } else {
      nhl = hln;
    }
    if (redo) flags |= FL_REDO;
    if (lmax_hit) flags |= FL_LMAX;
    A.rec_pw1[2 * k] = pwa;
    A.rec_pw1[2 * k + 1] = pwb;
    A.rec_warm1[k] = 1;
  } else {
    flags |= FL_FAIL;
    count = 0;
    A.rec_pw1[2 * k] = A.rec_pw0[2 * k];
    A.rec_pw1[2 * k + 1] = A.rec_pw0[2 * k + 1];
    A.rec_warm1[k] = warm;
    atomicOr(A.fail_acc + p, status);
  }
  A.rec_home1[k] = nhome;
  A.rec_hl1[k] = nhl;
  const int nsL = nhome + kk;
  unsigned long long vmax = 0;
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    if (i < nr) {
      r1[zlo + i] = Fr[i];
      m1[zlo + i] = Fm[i];
      int ph = (zlo + i <= nsL) ? phl : phr;
      unsigned long long b = d_speed_bits(M, ph, Fr[i], Fm[i]);
      vmax = b > vmax ? b : vmax;
    }
  }
  atomicMax(A.S_acc + p, vmax);
  if (!status) {
    if (A.st_pseudo) atomicAdd(A.st_pseudo, (unsigned long long)count);
    if (merge && A.st_merges) atomicAdd(A.st_merges, 1ull);
    if (lmax_hit && A.st_lmax) atomicAdd(A.st_lmax, 1ull);
  }
  if (row >= 0) {
    long long o = (long long)row * A.n_iface + k;
    A.log_count[o] = count;
    A.log_flags[o] = flags;
    A.log_zlo[o] = zlo;
  }
}

// ---------------------------------------------------------------------------
// per-problem bookkeeping between steps
// ---------------------------------------------------------------------------
__global__ void k_finalize(StepArgs A, int p_begin, int p_end, int init, int bump_row) {
  const int p = p_begin + blockIdx.x * blockDim.x + threadIdx.x;
  if (bump_row && p == p_begin && A.log_row) *A.log_row += 1;
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
      int prev_hi = -1;
      for (int j = 0; j < nif; ++j) {
        int zlo, zhi;
        bool tr;
        d_zone_range(A.rec_home1[i0 + j] + j, A.rec_hl1[i0 + j], h, P.zone_half, ns, zlo, zhi, tr);
        if (zlo <= prev_hi) {
          st |= ST_OVERLAP;
          break;
        }
        prev_hi = zhi;
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
hipError_t launch_bulk(const StepArgs& A, int tile_cells, int tile_begin, int n_tiles,
                       hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  switch (tile_cells) {
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
  k_cfl<1><<<n_tiles, 256, 0, s>>>(A, tile_begin);
  return hipGetLastError();
}

hipError_t launch_zone(const StepArgs& A, int if_begin, int if_end, hipStream_t s) {
  int n = if_end - if_begin;
  if (n <= 0) return hipSuccess;
  int groups = (n + A.zones_per_group - 1) / A.zones_per_group;
  switch (A.par.zone_half) {
    case 1: k_zone<1><<<groups, 64, 0, s>>>(A, if_begin, if_end); break;
    case 2: k_zone<2><<<groups, 64, 0, s>>>(A, if_begin, if_end); break;
    case 3: k_zone<3><<<groups, 64, 0, s>>>(A, if_begin, if_end); break;
    default: return hipErrorInvalidValue;
  }
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
