// imexds_adjoint.hip -- reverse-mode adjoint of one IMEX-DS step (gfx950).
//
// The step is the discrete map U^n -> U^{n+1} of the forward kernels with all
// of its decisions frozen (pseudo-iteration count, merge and crossing events,
// HLL branches, the cell that set the CFL time step), as recorded on the
// forward's tape.  Its adjoint runs in three launches per step; the first
// two touch disjoint cells and may run at the same time:
//   k_zone_adj  (one lane per zone): reverse of the interface advance and
//               re-split, of Part 2 and of every pseudo iteration of Part 1
//               (Algorithm 2) in reverse order from the stored iterates, of
//               the pseudo-step fractions theta = min(theta_nb, h_end / h)
//               and of the predicting solve, and of the zone set-up (merge
//               average, cut lengths).  Each interface solve is reversed at
//               its root by the implicit function theorem: with G(p*; x) = 0
//               (Appendix A, eq. 2p_RP:ex_sys), the adjoint of the inputs x
//               is dO/dx^T b - dG/dx^T mu with J^T mu = dO/dp*^T b, J the
//               Jacobian of eq. jacobian:ex_sys.  It leaves the adjoints of
//               the zone's edge fluxes F_left / F_right.
//   k_bulk_adj  (tiles of cells): transposed three-point stencil of the
//               explicit HLL update (Algorithm 1 Step 1) on the faces between
//               bulk cells, and the dependence of the update on dt; per tile
//               it also leaves the maximum of |u| + a and the first slot
//               attaining it.
//   k_fin_adj   (one lane per problem): the faces next to zone cells (the
//               stencil's terms there plus the edge-flux adjoints), then the
//               adjoint of dt = C h / max(|u| + a) (eq. cfl_cond:unif)
//               through that slot, or of a clipped last step through t.
// Everything is FP64; sums run in a fixed order (no atomics), so the adjoint
// is reproducible run to run.
#include "imexds_device.hpp"
#include "imexds_kernels.hpp"

namespace imexds {

// J^T b of the physical flux F(U) = (m, m u + p(rho)) of one phase:
// dF/drho = (0, a^2 - u^2), dF/dm = (1, 2u).
__device__ __forceinline__ void d_flux_jt(double a2, double u, double b0, double b1, double& gr,
                                          double& gm) {
  gr += b1 * (a2 - u * u);
  gm += b0 + 2.0 * u * b1;
}

// Reverse of d_hll: adds (dF/dU_l)^T b and (dF/dU_r)^T b, with the branch
// and the min / max choices of the forward, to (grl, gml) and (grr, gmr),
// which the caller passes in at zero.
__device__ __forceinline__ void d_hll_adj(const Mat& M, int ph, double rl, double ml, double rr,
                                          double mr, double b0, double b1, double& grl,
                                          double& gml, double& grr, double& gmr) {
  const double a = d_a(M, ph), a2 = d_a2(M, ph);
  const double ul = ml / rl, ur = mr / rr;
  const double sl = (ul < ur ? ul : ur) - a;
  const double sr = (ul > ur ? ul : ur) + a;
  if (sl >= 0.0 || sr <= 0.0) {
    // one-sided: the flux is the physical flux of the upwind side.  Both
    // sides' outputs are updated with selected values (updating one side
    // chosen at run time makes the compiler keep the caller's accumulators
    // in scratch memory); every caller passes them in at zero, so adding a
    // zero leaves the other side unchanged.
    const bool left = sl >= 0.0;
    double tr = 0.0, tm = 0.0;
    d_flux_jt(a2, left ? ul : ur, b0, b1, tr, tm);
    grl += left ? tr : 0.0;
    gml += left ? tm : 0.0;
    grr += left ? 0.0 : tr;
    gmr += left ? 0.0 : tm;
    return;
  }
  const double pl = d_pres(M, ph, rl), pr = d_pres(M, ph, rr);
  const double fl0 = ml, fl1 = ml * ul + pl, fr0 = mr, fr1 = mr * ur + pr;
  const double id = 1.0 / (sr - sl), ss = sl * sr;
  const double dU0 = rr - rl, dU1 = mr - ml;
  const double F0 = ((sr * fl0 - sl * fr0) + ss * dU0) * id;
  const double F1 = ((sr * fl1 - sl * fr1) + ss * dU1) * id;
  // F = (sr F_l - sl F_r + sl sr (U_r - U_l)) / (sr - sl)
  double tr = 0.0, tm = 0.0;
  d_flux_jt(a2, ul, b0, b1, tr, tm);
  grl += (sr * id) * tr - (ss * id) * b0;
  gml += (sr * id) * tm - (ss * id) * b1;
  tr = tm = 0.0;
  d_flux_jt(a2, ur, b0, b1, tr, tm);
  grr += (-sl * id) * tr + (ss * id) * b0;
  gmr += (-sl * id) * tm + (ss * id) * b1;
  // dF/dsl = (-F_r + sr dU + F) / (sr - sl), dF/dsr = (F_l + sl dU - F) / (sr - sl)
  const double gsl = (b0 * ((-fr0 + sr * dU0) + F0) + b1 * ((-fr1 + sr * dU1) + F1)) * id;
  const double gsr = (b0 * ((fl0 + sl * dU0) - F0) + b1 * ((fl1 + sl * dU1) - F1)) * id;
  double gul = 0.0, gur = 0.0;
  if (ul < ur)
    gul += gsl;
  else
    gur += gsl;
  if (ul > ur)
    gul += gsr;
  else
    gur += gsr;
  // u = m / rho
  grl += -gul * (ul / rl);
  gml += gul / rl;
  grr += -gur * (ur / rr);
  gmr += gur / rr;
}

// Linearisation of one interface solve at its root (p_l*, p_r*): the outputs
// F_PB = (F0, F1) and w, and what their reverse needs.
struct IfaceLin {
  double F0, F1, w;
  double z, zt;             // z and dz/dtau at fixed p*
  double dzl, dzr;          // dz/dp_l*, dz/dp_r*
  double J11, J12, J21, J22;
  double jv;                // [[v]] = v_r* - v_l*
  double ul, ur, rl, rr;    // side states
  double dfl, dfr;          // df_K / dp_K*
  double dfl_r, dfr_r;      // df_K / drho_K (side density)
  double uVs, vV, dvV;      // vapour star velocity, specific volume, dv_V*/dp_V*
  bool lvap;
};

// Outer wave of one side (as d_wave) with the derivative of f_K with respect
// to the side's density: shock -a (rho* + rho_K) / (2 rho_K sqrt(rho_K rho*)),
// rarefaction -a / rho_K.
__device__ __forceinline__ void d_wave_lin(const Mat& M, int ph, double rK, double ps, double& v,
                                           double& g, double& f, double& df, double& dfr) {
  const bool vap = ph == VAP;
  const double a = vap ? M.av : M.al, ia = vap ? M.iav : M.ial;
  const double irs = vap ? M.irv0 : M.irl0;
  const double r = d_rho_of_p(M, ph, ps);
  v = 1.0 / r;
  const double L = d_log(r * irs);
  g = (vap ? M.a2v : M.a2l) * L;
  if (ps > d_pres(M, ph, rK)) {
    const double ig = 1.0 / sqrt(rK * r);
    f = (a * (r - rK)) * ig;
    df = ((r + rK) * ig) * (v * (0.5 * ia));
    dfr = -(a * (r + rK) * ig) / (2.0 * rK);
  } else {
    f = a * (L - d_log(rK * irs));
    df = v * ia;
    dfr = -a / rK;
  }
}

// The linearisation from the two outer waves (d_wave_lin of each side).
__device__ __forceinline__ void d_iface_lin_w(const Mat& M, int phl, double rl, double ml,
                                              double rr, double mr, double psl, double psr,
                                              double vl, double gl, double fl, double dfl,
                                              double dfl_r, double vr, double gr, double fr,
                                              double dfr, double dfr_r, IfaceLin& Q) {
  const bool lvap = phl == VAP;
  Q.lvap = lvap;
  Q.rl = rl;
  Q.rr = rr;
  Q.ul = ml / rl;
  Q.ur = mr / rr;
  Q.dfl = dfl;
  Q.dfl_r = dfl_r;
  Q.dfr = dfr;
  Q.dfr_r = dfr_r;
  const double ia2l = lvap ? M.ia2v : M.ia2l, ia2r = lvap ? M.ia2l : M.ia2v;
  const double pV = lvap ? psl : psr;
  const double q = M.tau * pV;
  const double jg = gr - gl;
  const double jv2 = vr * vr - vl * vl;
  const double A = 0.5 * q * jv2;
  const double C = q * jg;
  const double sD = sqrt(1.0 - 4.0 * A * C);
  const double isD = 1.0 / sD;
  const double z = 2.0 * C / (1.0 + sD);
  double dAl = q * ((vl * vl * vl) * ia2l);
  double dAr = -(q * ((vr * vr * vr) * ia2r));
  double dCl = -(q * vl);
  double dCr = q * vr;
  if (lvap) {
    dAl += (0.5 * M.tau) * jv2;
    dCl += M.tau * jg;
  } else {
    dAr += (0.5 * M.tau) * jv2;
    dCr += M.tau * jg;
  }
  Q.dzl = (dAl * z * z + dCl) * isD;
  Q.dzr = (dAr * z * z + dCr) * isD;
  // A and C are linear in tau: dz/dtau = (A_tau z^2 + C_tau) / sqrt(D)
  Q.zt = ((0.5 * pV * jv2) * z * z + pV * jg) * isD;
  const double jv = vr - vl;
  const double el = (vl * vl) * ia2l, er = (vr * vr) * ia2r;
  Q.jv = jv;
  Q.z = z;
  Q.J11 = -1.0 + 2.0 * z * Q.dzl * jv + z * z * el;
  Q.J12 = 1.0 + 2.0 * z * Q.dzr * jv - z * z * er;
  Q.J21 = Q.dfl + Q.dzl * jv + z * el;
  Q.J22 = Q.dfr + Q.dzr * jv - z * er;
  if (lvap) {
    Q.uVs = Q.ul - fl;
    Q.vV = vl;
    Q.dvV = -(vl * vl) * ia2l;
  } else {
    Q.uVs = Q.ur + fr;
    Q.vV = vr;
    Q.dvV = -(vr * vr) * ia2r;
  }
  Q.w = Q.uVs + z * Q.vV;
  Q.F0 = -z;
  Q.F1 = -z * Q.uVs + pV;
}

__device__ __forceinline__ void d_iface_lin(const Mat& M, int phl, double rl, double ml,
                                            double rr, double mr, double psl, double psr,
                                            IfaceLin& Q) {
  double vl, gl, fl, dfl, dfl_r, vr, gr, fr, dfr, dfr_r;
  d_wave_lin(M, phl, rl, psl, vl, gl, fl, dfl, dfl_r);
  d_wave_lin(M, phl ^ 1, rr, psr, vr, gr, fr, dfr, dfr_r);
  d_iface_lin_w(M, phl, rl, ml, rr, mr, psl, psr, vl, gl, fl, dfl, dfl_r, vr, gr, fr, dfr, dfr_r,
                Q);
}

// Reverse of one interface solve: adjoints (b0, b1, bw) of (F0, F1, w) to the
// two side states and tau.
__device__ __forceinline__ void d_iface_adj(const IfaceLin& Q, double b0, double b1, double bw,
                                            double& grl, double& gml, double& grr, double& gmr,
                                            double& gtau) {
  // F0 = -z, F1 = -z u_V* + p_V*, w = u_V* + z v_V*
  const double gz = (-b0 - Q.uVs * b1) + Q.vV * bw;
  const double guV = -Q.z * b1 + bw;
  const double gpV = b1 + (Q.z * bw) * Q.dvV;
  double gpl = gz * Q.dzl, gpr = gz * Q.dzr;
  if (Q.lvap)
    gpl += -guV * Q.dfl + gpV;  // u_V* = u_l - f_l
  else
    gpr += guV * Q.dfr + gpV;  // u_V* = u_r + f_r
  // J^T mu = dO/dp*^T b
  const double idet = 1.0 / (Q.J11 * Q.J22 - Q.J12 * Q.J21);
  const double mu1 = (Q.J22 * gpl - Q.J21 * gpr) * idet;
  const double mu2 = (Q.J11 * gpr - Q.J12 * gpl) * idet;
  // direct dependence at fixed p*: u_V* through the vapour side's velocity
  // (selected, not branched: a conditional update of one of two accumulators
  // put them in scratch memory)
  gtau += gz * Q.zt;
  {
    const double rV = Q.lvap ? Q.rl : Q.rr, uV = Q.lvap ? Q.ul : Q.ur;
    const double dV = Q.lvap ? -Q.dfl_r : Q.dfr_r;
    const double gr = guV * (-(uV / rV) + dV), gm = guV / rV;
    const double grl1 = grl + gr, gml1 = gml + gm, grr1 = grr + gr, gmr1 = gmr + gm;
    grl = Q.lvap ? grl1 : grl;
    gml = Q.lvap ? gml1 : gml;
    grr = Q.lvap ? grr : grr1;
    gmr = Q.lvap ? gmr : gmr1;
  }
  // minus dG/dx^T mu: G1 = (p_r* - p_l*) + z^2 [[v]],
  // G2 = f_l + f_r + z [[v]] + (u_r - u_l)
  grl -= mu2 * (Q.dfl_r + Q.ul / Q.rl);
  gml += mu2 / Q.rl;
  grr -= mu2 * (Q.dfr_r - Q.ur / Q.rr);
  gmr -= mu2 / Q.rr;
  gtau -= mu1 * (2.0 * Q.z * Q.jv * Q.zt) + mu2 * (Q.jv * Q.zt);
}

// ---------------------------------------------------------------------------
// zone pass
// ---------------------------------------------------------------------------
// Reverse of one pass over the zone: given the adjoint gO of its output (the
// next iterate, or U^{n+1} in Part 2), accumulates the adjoints of the input
// iterate W (into gWr/gWm, which the caller zeroes), of U0, of the moving
// lengths and thetas, of dt, tau and the edge fluxes.
template <int MC>
struct ZoneRev {
  // set-up, fixed over the passes of one zone step
  int nr, skip, into, ic, icr, zlo, sL, phl, phr;
  double h, dt, hn_l, hn_r, th_l, th_r, th_f, it_l, it_r, it_f;
  double FL0, FL1, FR0, FR1;
  double U0r[MC], U0m[MC];
  // adjoint accumulators
  double gU0r[MC], gU0m[MC];
  double ghn_l, ghn_r, gth_l, gth_r, gdt, gtau, gFL0, gFL1, gFR0, gFR1;
};

template <int MC>
__device__ __forceinline__ void d_pass_rev(const Mat& M, ZoneRev<MC>& Z, bool part2,
                                           const double* Wr, const double* Wm, double rpl,
                                           double rpr, const double* Nr, const double* Nm,
                                           const double* gOr, const double* gOm, double& gw,
                                           double* gWr, double* gWm) {
  // forward fluxes of W: right face of each active position
  double Fr0[MC], Fr1[MC];
  IfaceLin Q;
  double qr0 = 1.0, qm0 = 0.0, qr1 = 1.0, qm1 = 0.0;
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    if (i == Z.ic) {
      qr0 = Wr[i];
      qm0 = Wm[i];
    }
    if (i == Z.icr) {
      qr1 = Wr[i];
      qm1 = Wm[i];
    }
  }
  d_iface_lin(M, Z.phl, qr0, qm0, qr1, qm1, rpl, rpr, Q);
  const double w = Q.w;
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    Fr0[i] = 0.0;
    Fr1[i] = 0.0;
    if (i >= Z.nr || i == Z.skip) continue;
    if (i == Z.nr - 1) {
      Fr0[i] = Z.FR0;
      Fr1[i] = Z.FR1;
    } else if (i == Z.ic) {
      Fr0[i] = Q.F0;
      Fr1[i] = Q.F1;
    } else if (i + 1 < MC) {
      const int ph = (Z.zlo + i <= Z.sL) ? Z.phl : Z.phr;
      d_hll(M, ph, Wr[i], Wm[i], Wr[i + 1], Wm[i + 1], Fr0[i], Fr1[i]);
    }
  }
  const double hnew_l = Z.hn_l + (1.0 * w) * Z.dt;
  const double hnew_r = Z.hn_r + (-1.0 * w) * Z.dt;
  const double ih_l = 1.0 / hnew_l, ih_r = 1.0 / hnew_r, ih_f = 1.0 / Z.h;
  double gF0[MC], gF1[MC];  // adjoints of the right-face fluxes
#pragma unroll
  for (int i = 0; i < MC; ++i) gF0[i] = gF1[i] = 0.0;
  double gl0 = 0.0, gl1 = 0.0;  // adjoint of F_left of position 0
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    if (i >= Z.nr || i == Z.skip) continue;
    double fl0, fl1;
    if (i == 0) {
      fl0 = Z.FL0;
      fl1 = Z.FL1;
    } else if (i >= 2 && Z.skip == i - 1) {
      fl0 = Fr0[i >= 2 ? i - 2 : 0];
      fl1 = Fr1[i >= 2 ? i - 2 : 0];
    } else {
      fl0 = Fr0[i - 1];
      fl1 = Fr1[i - 1];
    }
    const bool mvl = i == Z.ic, mvr = i == Z.icr;
    const double hni = mvl ? Z.hn_l : (mvr ? Z.hn_r : Z.h);
    const double ihi = mvl ? ih_l : (mvr ? ih_r : ih_f);
    const double d0 = Fr0[i] - fl0, d1 = Fr1[i] - fl1;
    const double rhs0 = (hni * Z.U0r[i] - Z.dt * d0) * ihi;
    const double rhs1 = (hni * Z.U0m[i] - Z.dt * d1) * ihi;
    double gr0, gr1;  // adjoint of rhs
    if (part2) {
      gr0 = gOr[i];
      gr1 = gOm[i];
    } else {
      // W^{l+1} = (W^l + theta rhs) / (1 + theta)
      const double th = mvl ? Z.th_l : (mvr ? Z.th_r : Z.th_f);
      const double it = mvl ? Z.it_l : (mvr ? Z.it_r : Z.it_f);
      gWr[i] += it * gOr[i];
      gWm[i] += it * gOm[i];
      gr0 = (th * it) * gOr[i];
      gr1 = (th * it) * gOm[i];
      const double gth = it * ((rhs0 - Nr[i]) * gOr[i] + (rhs1 - Nm[i]) * gOm[i]);
      if (mvl) Z.gth_l += gth;
      if (mvr) Z.gth_r += gth;
    }
    // rhs = (h^n U0 - dt (F_right - F_left)) / h^{l+1}
    Z.gU0r[i] += (hni * ihi) * gr0;
    Z.gU0m[i] += (hni * ihi) * gr1;
    const double gfr0 = -(Z.dt * ihi) * gr0, gfr1 = -(Z.dt * ihi) * gr1;
    gF0[i] += gfr0;
    gF1[i] += gfr1;
    if (i == 0) {
      gl0 -= gfr0;
      gl1 -= gfr1;
    } else if (i >= 2 && Z.skip == i - 1) {
      gF0[i >= 2 ? i - 2 : 0] -= gfr0;
      gF1[i >= 2 ? i - 2 : 0] -= gfr1;
    } else {
      gF0[i - 1] -= gfr0;
      gF1[i - 1] -= gfr1;
    }
    Z.gdt -= ihi * (d0 * gr0 + d1 * gr1);
    if (mvl || mvr) {
      const double ghn = ihi * (Z.U0r[i] * gr0 + Z.U0m[i] * gr1);
      const double ghnew = -ihi * (rhs0 * gr0 + rhs1 * gr1);
      if (mvl) {  // h^{l+1} = h^n + w dt
        Z.ghn_l += ghn + ghnew;
        gw += Z.dt * ghnew;
        Z.gdt += w * ghnew;
      } else {  // h^{l+1} = h^n - w dt
        Z.ghn_r += ghn + ghnew;
        gw -= Z.dt * ghnew;
        Z.gdt -= w * ghnew;
      }
    }
  }
  Z.gFL0 += gl0;
  Z.gFL1 += gl1;
  // fluxes of W -> W
  double gq_r0 = 0.0, gq_m0 = 0.0, gq_r1 = 0.0, gq_m1 = 0.0;
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    if (i >= Z.nr || i == Z.skip) continue;
    if (i == Z.nr - 1) {
      Z.gFR0 += gF0[i];
      Z.gFR1 += gF1[i];
    } else if (i == Z.ic) {
      d_iface_adj(Q, gF0[i], gF1[i], gw, gq_r0, gq_m0, gq_r1, gq_m1, Z.gtau);
    } else if (i + 1 < MC) {
      const int ph = (Z.zlo + i <= Z.sL) ? Z.phl : Z.phr;
      double a0 = 0.0, a1 = 0.0, c0 = 0.0, c1 = 0.0;
      d_hll_adj(M, ph, Wr[i], Wm[i], Wr[i + 1], Wm[i + 1], gF0[i], gF1[i], a0, a1, c0, c1);
      gWr[i] += a0;
      gWm[i] += a1;
      gWr[i + 1] += c0;
      gWm[i + 1] += c1;
    }
  }
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    if (i == Z.ic) {
      gWr[i] += gq_r0;
      gWm[i] += gq_m0;
    }
    if (i == Z.icr) {
      gWr[i] += gq_r1;
      gWm[i] += gq_m1;
    }
  }
}

template <int ZH>
__global__ __launch_bounds__(64) void k_zone_adj(StepArgs A, AdjArgs B) {
  constexpr int MC = 2 * ZH + 1;
  constexpr int E = 2 * MC + 2;
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k >= A.n_iface) return;
  const Mat& M = A.mat;
  const Par& P = A.par;
  const int p = A.iface_prob[k], kk = A.iface_local[k];
  const double dt = A.dt[p];
  const double* T = A.tape + k * A.tape_stride;
  const int flags = (int)T[TH_FLAGS];
  double* zo = B.zadj + 5 * (long long)k;
#pragma unroll
  for (int j = 0; j < 5; ++j) zo[j] = 0.0;
  if (dt == 0.0 || (flags & FL_INACTIVE)) return;  // the bulk pass carries the whole problem
  const long long so = A.slot_off[p];
  const int ns = (int)(A.slot_off[p + 1] - so);
  const double h = A.h[p];
  const int home = A.rec_home0[k];
  const double hl = A.rec_hl0[k];
  const int sL = home + kk;
  const int phl = A.phase_first[p] ^ (kk & 1), phr = phl ^ 1;
  int zlo, zhi;
  bool tr;
  d_zone_range(sL, hl, h, ZH, ns, zlo, zhi, tr);
  const int nr = zhi - zlo + 1, iL = sL - zlo, iR = iL + 1;
  const double* r0 = A.rho0 + so;
  const double* m0 = A.mom0 + so;
  const double* g1r = B.gr1 + so;
  const double* g1m = B.gm1 + so;
  double* g0r = B.gr0 + so;
  double* g0m = B.gm0 + so;
  if ((flags & FL_FAIL) || sL < 0 || sL + 1 >= ns) {  // cells and record left at t^n
    for (int i = 0; i < nr; ++i) {
      g0r[zlo + i] = g1r[zlo + i];
      g0m[zlo + i] = g1m[zlo + i];
    }
    return;
  }
  double Ur[MC], Um[MC], Br[MC], Bm[MC];
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    const bool in = i < nr;
    Ur[i] = in ? r0[zlo + i] : 1.0;
    Um[i] = in ? m0[zlo + i] : 0.0;
    Br[i] = in ? g1r[zlo + i] : 0.0;
    Bm[i] = in ? g1m[zlo + i] : 0.0;
  }
  const bool merge = (flags & FL_MERGED) != 0;
  int cnt = (int)T[TH_COUNT];
  cnt = cnt < 0 ? 0 : (cnt > P.lmax ? P.lmax : cnt);
  const double wp = T[TH_WP], wstar = T[TH_WSTAR];

  ZoneRev<MC> Z;
  Z.nr = nr;
  Z.zlo = zlo;
  Z.sL = sL;
  Z.phl = phl;
  Z.phr = phr;
  Z.h = h;
  Z.dt = dt;
  Z.skip = merge ? (tr ? iR : iL) : -1;
  Z.into = merge ? (tr ? iR + 1 : iL - 1) : -1;
  Z.ic = (merge && !tr) ? Z.into : iL;
  Z.icr = (merge && tr) ? Z.into : iR;
  const double ht = tr ? h - hl : hl;
  const double hm = h + ht;
  double rskip = 0.0, mskip = 0.0, rin = 0.0, min_ = 0.0;
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    if (i == Z.skip) {
      rskip = Ur[i];
      mskip = Um[i];
    }
    if (i == Z.into) {
      rin = Ur[i];
      min_ = Um[i];
    }
  }
  const double Mr = merge ? (h * rin + ht * rskip) / hm : 0.0;
  const double Mm = merge ? (h * min_ + ht * mskip) / hm : 0.0;
  Z.hn_l = (merge && !tr) ? hm : hl;
  Z.hn_r = (merge && tr) ? hm : h - hl;
  const double hh_l = Z.hn_l + (1.0 * wp) * dt;
  const double hh_r = Z.hn_r + (-1.0 * wp) * dt;
  const bool cl_l = hh_l / h > P.theta_nb, cl_r = hh_r / h > P.theta_nb;
  Z.th_l = cl_l ? P.theta_nb : hh_l / h;
  Z.th_r = cl_r ? P.theta_nb : hh_r / h;
  const double thf = (h + (0.0 * wp) * dt) / h;
  Z.th_f = thf > P.theta_nb ? P.theta_nb : thf;
  Z.it_l = 1.0 / (1.0 + Z.th_l);
  Z.it_r = 1.0 / (1.0 + Z.th_r);
  Z.it_f = 1.0 / (1.0 + Z.th_f);
  const int phz = (zlo <= sL) ? phl : phr;
  const int phe = (zhi <= sL) ? phl : phr;
  if (zlo == 0)
    d_bflux(M, phz, false, P.bc_left, r0[0], m0[0], Z.FL0, Z.FL1);
  else
    d_hll(M, phz, r0[zlo - 1], m0[zlo - 1], r0[zlo], m0[zlo], Z.FL0, Z.FL1);
  if (zhi == ns - 1)
    d_bflux(M, phe, true, P.bc_right, r0[ns - 1], m0[ns - 1], Z.FR0, Z.FR1);
  else
    d_hll(M, phe, r0[zhi], m0[zhi], r0[zhi + 1], m0[zhi + 1], Z.FR0, Z.FR1);
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    Z.U0r[i] = (i == Z.into) ? Mr : Ur[i];
    Z.U0m[i] = (i == Z.into) ? Mm : Um[i];
    Z.gU0r[i] = Z.gU0m[i] = 0.0;
  }
  Z.ghn_l = Z.ghn_r = Z.gth_l = Z.gth_r = Z.gdt = Z.gtau = 0.0;
  Z.gFL0 = Z.gFL1 = Z.gFR0 = Z.gFR1 = 0.0;

  // reverse of the write-back: the emptied piece copied the value of `src`
  double gOr[MC], gOm[MC];
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    gOr[i] = (i == Z.skip || i >= nr) ? 0.0 : Br[i];
    gOm[i] = (i == Z.skip || i >= nr) ? 0.0 : Bm[i];
  }
  if (merge) {
    int src;
    if (!tr)
      src = (flags & FL_CROSS_L) ? iR : Z.into;
    else
      src = (flags & FL_CROSS_R) ? iL : Z.into;
    double sr_ = 0.0, sm_ = 0.0;
#pragma unroll
    for (int i = 0; i < MC; ++i)
      if (i == Z.skip) {
        sr_ = Br[i];
        sm_ = Bm[i];
      }
#pragma unroll
    for (int i = 0; i < MC; ++i)
      if (i == src) {
        gOr[i] += sr_;
        gOm[i] += sm_;
      }
  }
  // hl^{n+1} = hl^n + w* dt (+- h after a crossing)
  const double ghl1 = B.hl_bar[k];
  double ghl = ghl1;
  double gw = ghl1 * dt;
  Z.gdt += ghl1 * wstar;

  // Part 2 at W^count, then the pseudo iterations in reverse
  double Wr[MC], Wm[MC], Nr[MC], Nm[MC], gWr[MC], gWm[MC];
  const double* e = T + TAPE_HDR + (long long)cnt * E;
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    Wr[i] = e[i];
    Wm[i] = e[MC + i];
    gWr[i] = gWm[i] = 0.0;
  }
  d_pass_rev<MC>(M, Z, true, Wr, Wm, e[2 * MC], e[2 * MC + 1], Wr, Wm, gOr, gOm, gw, gWr, gWm);
  for (int l = cnt - 1; l >= 0; --l) {
    const double* el = T + TAPE_HDR + (long long)l * E;
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      Nr[i] = Wr[i];
      Nm[i] = Wm[i];
      Wr[i] = el[i];
      Wm[i] = el[MC + i];
      gOr[i] = gWr[i];
      gOm[i] = gWm[i];
      gWr[i] = gWm[i] = 0.0;
    }
    double gwl = 0.0;
    d_pass_rev<MC>(M, Z, false, Wr, Wm, el[2 * MC], el[2 * MC + 1], Nr, Nm, gOr, gOm, gwl, gWr,
                   gWm);
  }
  // W^0 = U0
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    Z.gU0r[i] += gWr[i];
    Z.gU0m[i] += gWm[i];
  }
  // theta = min(theta_nb, h_end / h), h_end = h^n +- w_pred dt
  double gwp = 0.0;
  if (!cl_l) {
    const double g = Z.gth_l / h;
    Z.ghn_l += g;
    gwp += g * dt;
    Z.gdt += g * wp;
  }
  if (!cl_r) {
    const double g = Z.gth_r / h;
    Z.ghn_r += g;
    gwp -= g * dt;
    Z.gdt -= g * wp;
  }
  // zone set-up: U0 from U^n (merge average), lengths from hl
  double Gr[MC], Gm[MC];
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    Gr[i] = (i == Z.into) ? (h / hm) * Z.gU0r[i] : Z.gU0r[i];
    Gm[i] = (i == Z.into) ? (h / hm) * Z.gU0m[i] : Z.gU0m[i];
  }
  if (merge) {
    double gir = 0.0, gim = 0.0;
#pragma unroll
    for (int i = 0; i < MC; ++i)
      if (i == Z.into) {
        gir = Z.gU0r[i];
        gim = Z.gU0m[i];
      }
#pragma unroll
    for (int i = 0; i < MC; ++i)
      if (i == Z.skip) {  // U0 of the skipped piece is unused: only the average reads it
        Gr[i] = (ht / hm) * gir;
        Gm[i] = (ht / hm) * gim;
      }
    // d/dht of (h U_into + ht U_skip) / (h + ht) = (U_skip - M) / hm; h^n of the merged cell = hm
    double ght = ((rskip - Mr) * gir + (mskip - Mm) * gim) / hm;
    if (!tr) {
      ght += Z.ghn_l;
      ghl -= Z.ghn_r;  // h^n_r = h - hl
      ghl += ght;      // ht = hl
    } else {
      ght += Z.ghn_r;
      ghl += Z.ghn_l;  // h^n_l = hl
      ghl -= ght;      // ht = h - hl
    }
  } else {
    ghl += Z.ghn_l - Z.ghn_r;
  }
  // predicting solve on U^n of the two cut pieces
  if (gwp != 0.0) {
    double qr0 = 1.0, qm0 = 0.0, qr1 = 1.0, qm1 = 0.0;
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      if (i == iL) {
        qr0 = Ur[i];
        qm0 = Um[i];
      }
      if (i == iR) {
        qr1 = Ur[i];
        qm1 = Um[i];
      }
    }
    IfaceLin Q;
    d_iface_lin(M, phl, qr0, qm0, qr1, qm1, T[TH_IPL], T[TH_IPR], Q);
    double a0 = 0.0, a1 = 0.0, c0 = 0.0, c1 = 0.0;
    d_iface_adj(Q, 0.0, 0.0, gwp, a0, a1, c0, c1, Z.gtau);
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      if (i == iL) {
        Gr[i] += a0;
        Gm[i] += a1;
      }
      if (i == iR) {
        Gr[i] += c0;
        Gm[i] += c1;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < MC; ++i)
    if (i < nr) {
      g0r[zlo + i] = Gr[i];
      g0m[zlo + i] = Gm[i];
    }
  zo[0] = Z.gFL0;
  zo[1] = Z.gFL1;
  zo[2] = Z.gFR0;
  zo[3] = Z.gFR1;
  zo[4] = Z.gdt;
  B.tau_bar[k] += Z.gtau;
  B.hl_bar[k] = ghl;
}

// ---------------------------------------------------------------------------
// zone pass with eight lanes per zone
// ---------------------------------------------------------------------------
// The same reverse as k_zone_adj, with the zone spread over an 8-lane group
// as in k_zone8: lane c holds active cell c (its iterate, U0, lengths,
// theta and their adjoints) and the face to its right; the interface solve
// is linearised and reversed on the lane left of the phase boundary.  Sums
// over the group run in a fixed shuffle order.
namespace {

__device__ __forceinline__ double a8_get(double x, int gb, int c) { return __shfl(x, gb + c, 64); }

__device__ __forceinline__ double a8_sum(double v) {
#pragma unroll
  for (int off = 4; off > 0; off >>= 1) v += __shfl_xor(v, off, 8);
  return v;
}

struct ZoneRev8 {
  int c, gb, m, ic, zlo, sL, phl, phr;
  double h, dt, FL0, FL1, FR0, FR1;
  // own active cell
  double U00, U01, hn, mv, th, it1;
  int ph;
  // own adjoint accumulators
  double gU00, gU01, ghn, gth, gdt, gtau, gFL0, gFL1, gFR0, gFR1;
};

// The interface linearisations of up to four passes at once: pair j of the
// group (lanes 2j, 2j + 1) takes pass l_hi - j, the even lane the left outer
// wave (active cell ic, tape position pic), the odd one the right (ic + 1,
// pic1); they exchange them by DPP quad permutation and the even lane
// completes the linearisation and stores it in slots[pass & 3] (A8_LIN
// doubles).  Lanes without a pass of their own (j >= nb) repeat pass l_hi
// and store nothing.  Every lane of the group must be active.
constexpr int A8_LIN = 23;

__device__ __forceinline__ void a8_lin_batch(const Mat& M, const ZoneRev8& Z, const double* T,
                                             int E, int MC, int l_hi, int nb, int pic, int pic1,
                                             double (*slots)[A8_LIN]) {
  const int j = Z.c >> 1, side = Z.c & 1;
  const int lp = j < nb ? l_hi - j : l_hi;
  const double* el = T + TAPE_HDR + (long long)lp * E;
  const int pc = side ? pic1 : pic;
  const double Wr = el[pc], Wm = el[MC + pc];
  const double rpl = el[2 * MC], rpr = el[2 * MC + 1];
  double v, g, f, df, dr;
  d_wave_lin(M, side ? Z.phr : Z.phl, Wr, side ? rpr : rpl, v, g, f, df, dr);
  const double oWr = d_swap(Wr), oWm = d_swap(Wm), ov = d_swap(v), og = d_swap(g);
  const double of = d_swap(f), odf = d_swap(df), odr = d_swap(dr);
  if (side == 0 && j < nb) {
    IfaceLin Q;
    d_iface_lin_w(M, Z.phl, Wr, Wm, oWr, oWm, rpl, rpr, v, g, f, df, dr, ov, og, of, odf, odr, Q);
    double* q = slots[lp & 3];
    q[0] = Q.F0; q[1] = Q.F1; q[2] = Q.w; q[3] = Q.z; q[4] = Q.zt; q[5] = Q.dzl; q[6] = Q.dzr;
    q[7] = Q.J11; q[8] = Q.J12; q[9] = Q.J21; q[10] = Q.J22; q[11] = Q.jv; q[12] = Q.ul;
    q[13] = Q.ur; q[14] = Q.rl; q[15] = Q.rr; q[16] = Q.dfl; q[17] = Q.dfr; q[18] = Q.dfl_r;
    q[19] = Q.dfr_r; q[20] = Q.uVs; q[21] = Q.vV; q[22] = Q.dvV;
  }
}

__device__ __forceinline__ void a8_lin_load(const double* q, int phl, IfaceLin& Q) {
  Q.F0 = q[0]; Q.F1 = q[1]; Q.w = q[2]; Q.z = q[3]; Q.zt = q[4]; Q.dzl = q[5]; Q.dzr = q[6];
  Q.J11 = q[7]; Q.J12 = q[8]; Q.J21 = q[9]; Q.J22 = q[10]; Q.jv = q[11]; Q.ul = q[12];
  Q.ur = q[13]; Q.rl = q[14]; Q.rr = q[15]; Q.dfl = q[16]; Q.dfr = q[17]; Q.dfl_r = q[18];
  Q.dfr_r = q[19]; Q.uVs = q[20]; Q.vV = q[21]; Q.dvV = q[22];
  Q.lvap = phl == VAP;
}

// One pass of the zone (a pseudo iteration, or Part 2) reversed: own iterate
// (W0, W1), next iterate (N0, N1), adjoint of this lane's output (gO0, gO1);
// gwx is the adjoint of the boundary speed from outside the pass (Part 2:
// the interface advance; counted once); Q the pass's interface linearisation
// (read on lane ic).  Adds the adjoint of the own iterate to (gW0, gW1).
__device__ __forceinline__ void a8_pass_rev(const Mat& M, ZoneRev8& Z, bool part2, double W0,
                                            double W1, const IfaceLin& Q, double N0, double N1,
                                            double gO0, double gO1, double gwx, double& gW0,
                                            double& gW1) {
  // Neighbour values come by DPP row shifts: the 8-lane groups sit inside the
  // 16-lane rows, and the lanes whose shift would cross a group boundary
  // (lane 7 from the next group, lane 0 from the previous) do not use them.
  const int c = Z.c;
  const double nW0 = d_lane_next(W0), nW1 = d_lane_next(W1);
  // the boundary's flux is used on lane ic, which holds it; its speed on
  // the two moving cells ic and ic + 1 (every other cell has mv = 0 and
  // keeps its length whatever the speed)
  const double F0pb = Q.F0, F1pb = Q.F1;
  const double wprev = d_lane_prev(Q.w);
  const double w = c == Z.ic ? Q.w : (c == Z.ic + 1 ? wprev : 0.0);
  const bool act = c < Z.m;
  double Fr0 = 0.0, Fr1 = 0.0;
  if (act) {
    if (c == Z.m - 1) {
      Fr0 = Z.FR0;
      Fr1 = Z.FR1;
    } else if (c == Z.ic) {
      Fr0 = F0pb;
      Fr1 = F1pb;
    } else {
      d_hll(M, Z.ph, W0, W1, nW0, nW1, Fr0, Fr1);
    }
  }
  double Fl0 = d_lane_prev(Fr0), Fl1 = d_lane_prev(Fr1);
  if (c == 0) {
    Fl0 = Z.FL0;
    Fl1 = Z.FL1;
  }
  double gfr0 = 0.0, gfr1 = 0.0, gfl0 = 0.0, gfl1 = 0.0, gwl = 0.0;
  if (act) {
    const double hnew = Z.hn + (Z.mv * w) * Z.dt;
    const double ih = 1.0 / hnew;
    const double d0 = Fr0 - Fl0, d1 = Fr1 - Fl1;
    const double rhs0 = (Z.hn * Z.U00 - Z.dt * d0) * ih;
    const double rhs1 = (Z.hn * Z.U01 - Z.dt * d1) * ih;
    double gr0, gr1;
    if (part2) {
      gr0 = gO0;
      gr1 = gO1;
    } else {
      gW0 += Z.it1 * gO0;
      gW1 += Z.it1 * gO1;
      gr0 = (Z.th * Z.it1) * gO0;
      gr1 = (Z.th * Z.it1) * gO1;
      Z.gth += Z.it1 * ((rhs0 - N0) * gO0 + (rhs1 - N1) * gO1);
    }
    Z.gU00 += (Z.hn * ih) * gr0;
    Z.gU01 += (Z.hn * ih) * gr1;
    gfr0 = -(Z.dt * ih) * gr0;
    gfr1 = -(Z.dt * ih) * gr1;
    gfl0 = -gfr0;
    gfl1 = -gfr1;
    Z.gdt -= ih * (d0 * gr0 + d1 * gr1);
    if (Z.mv != 0.0) {
      const double ghnew = -ih * (rhs0 * gr0 + rhs1 * gr1);
      Z.ghn += ih * (Z.U00 * gr0 + Z.U01 * gr1) + ghnew;
      gwl = Z.mv * (Z.dt * ghnew);
      Z.gdt += Z.mv * (w * ghnew);
    }
  }
  // adjoint of the flux on the right face of c: own part plus the left-face
  // part of cell c + 1
  double gF0 = gfr0 + d_lane_next(gfl0), gF1 = gfr1 + d_lane_next(gfl1);
  if (c == 0) {
    Z.gFL0 += gfl0;
    Z.gFL1 += gfl1;
  }
  if (act && c == Z.m - 1) {
    Z.gFR0 += gfr0;
    Z.gFR1 += gfr1;
  }
  // only the moving cells ic and ic + 1 carry a speed adjoint; it is needed
  // on lane ic
  const double gw = (gwl + d_lane_next(gwl)) + gwx;
  double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;  // own / right neighbour
  if (act && c < Z.m - 1) {
    if (c == Z.ic)
      d_iface_adj(Q, gF0, gF1, gw, a0, a1, b0, b1, Z.gtau);
    else
      d_hll_adj(M, Z.ph, W0, W1, nW0, nW1, gF0, gF1, a0, a1, b0, b1);
  }
  gW0 += a0 + d_lane_prev(b0) * (c > 0 ? 1.0 : 0.0);
  gW1 += a1 + d_lane_prev(b1) * (c > 0 ? 1.0 : 0.0);
}

}  // namespace

template <int ZH>
__global__ __launch_bounds__(64) void k_zone_adj8(StepArgs A, AdjArgs B) {
  constexpr int MC = 2 * ZH + 1;
  constexpr int E = 2 * MC + 2;
  static_assert(MC <= 8, "a zone must fit an 8-lane group");
  // the interface linearisations of four passes per group (a8_lin_batch)
  __shared__ double s_lin[8][4][A8_LIN];
  const int c = threadIdx.x & 7, gb = threadIdx.x & ~7;
  const int k = (blockIdx.x * 64 + threadIdx.x) >> 3;
  if (k >= A.n_iface) return;  // uniform over the group
  const Mat& M = A.mat;
  const Par& P = A.par;
  const double theta_nb = P.theta_nb;
  const int p = A.iface_prob[k], kk = A.iface_local[k];
  const double dt = A.dt[p];
  const double* T = A.tape + k * A.tape_stride;
  const int flags = (int)T[TH_FLAGS];
  if (c == 0) {
    double* zo = B.zadj + 5 * (long long)k;
#pragma unroll
    for (int j = 0; j < 5; ++j) zo[j] = 0.0;
  }
  if (dt == 0.0 || (flags & FL_INACTIVE)) return;
  const long long so = A.slot_off[p];
  const int ns = (int)(A.slot_off[p + 1] - so);
  const double h = A.h[p];
  const int home = A.rec_home0[k];
  const double hl = A.rec_hl0[k];
  const int sL = home + kk;
  const int phl = A.phase_first[p] ^ (kk & 1), phr = phl ^ 1;
  int zlo, zhi;
  bool tr;
  d_zone_range(sL, hl, h, ZH, ns, zlo, zhi, tr);
  const int nr = zhi - zlo + 1, iL = sL - zlo, iR = iL + 1;
  const double* r0 = A.rho0 + so;
  const double* m0 = A.mom0 + so;
  const double* g1r = B.gr1 + so;
  const double* g1m = B.gm1 + so;
  double* g0r = B.gr0 + so;
  double* g0m = B.gm0 + so;
  if ((flags & FL_FAIL) || sL < 0 || sL + 1 >= ns) {  // cells and record left at t^n
    if (c < nr) {
      g0r[zlo + c] = g1r[zlo + c];
      g0m[zlo + c] = g1m[zlo + c];
    }
    return;
  }
  // U^n and the adjoint of U^{n+1} of zone position c
  double Ur = 1.0, Um = 0.0, Br = 0.0, Bm = 0.0;
  if (c < nr) {
    Ur = r0[zlo + c];
    Um = m0[zlo + c];
    Br = g1r[zlo + c];
    Bm = g1m[zlo + c];
  }
  const bool merge = (flags & FL_MERGED) != 0;
  int cnt = (int)T[TH_COUNT];
  cnt = cnt < 0 ? 0 : (cnt > P.lmax ? P.lmax : cnt);
  const double wp = T[TH_WP], wstar = T[TH_WSTAR];
  const int skip = merge ? (tr ? iR : iL) : -1;
  const int into = merge ? (tr ? iR + 1 : iL - 1) : -1;
  ZoneRev8 Z;
  Z.c = c;
  Z.gb = gb;
  Z.m = merge ? nr - 1 : nr;
  Z.zlo = zlo;
  Z.sL = sL;
  Z.phl = phl;
  Z.phr = phr;
  Z.h = h;
  Z.dt = dt;
  const int ic_pos = (merge && !tr) ? into : iL;
  Z.ic = (skip >= 0 && ic_pos > skip) ? ic_pos - 1 : ic_pos;
  const int pos = c < Z.m ? ((skip >= 0 && c >= skip) ? c + 1 : c) : -1;
  const double ht = tr ? h - hl : hl;
  const double hm = h + ht;
  const double rpos = a8_get(Ur, gb, pos >= 0 ? pos : 0), mpos = a8_get(Um, gb, pos >= 0 ? pos : 0);
  const double rskip = a8_get(Ur, gb, skip >= 0 ? skip : 0);
  const double mskip = a8_get(Um, gb, skip >= 0 ? skip : 0);
  const double Mr = merge ? (h * a8_get(Ur, gb, into >= 0 ? into : 0) + ht * rskip) / hm : 0.0;
  const double Mm = merge ? (h * a8_get(Um, gb, into >= 0 ? into : 0) + ht * mskip) / hm : 0.0;
  const double hn_l = (merge && !tr) ? hm : hl;
  const double hn_r = (merge && tr) ? hm : h - hl;
  const double hh_l = hn_l + (1.0 * wp) * dt;
  const double hh_r = hn_r + (-1.0 * wp) * dt;
  const bool cl_l = hh_l / h > theta_nb, cl_r = hh_r / h > theta_nb;
  const double th_l = cl_l ? theta_nb : hh_l / h;
  const double th_r = cl_r ? theta_nb : hh_r / h;
  const double thf = (h + (0.0 * wp) * dt) / h;
  const double th_f = thf > theta_nb ? theta_nb : thf;
  const bool mvl = c == Z.ic, mvr = c == Z.ic + 1;
  Z.U00 = pos == into ? Mr : rpos;
  Z.U01 = pos == into ? Mm : mpos;
  Z.hn = mvl ? hn_l : (mvr ? hn_r : h);
  Z.mv = mvl ? 1.0 : (mvr ? -1.0 : 0.0);
  Z.th = mvl ? th_l : (mvr ? th_r : th_f);
  Z.it1 = 1.0 / (1.0 + Z.th);
  Z.ph = (zlo + (pos >= 0 ? pos : 0) <= sL) ? phl : phr;
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
    Z.FL0 = a8_get(f0, gb, 0);
    Z.FL1 = a8_get(f1, gb, 0);
    Z.FR0 = a8_get(f0, gb, 1);
    Z.FR1 = a8_get(f1, gb, 1);
  }
  Z.gU00 = Z.gU01 = Z.ghn = Z.gth = Z.gdt = Z.gtau = 0.0;
  Z.gFL0 = Z.gFL1 = Z.gFR0 = Z.gFR1 = 0.0;

  // reverse of the write-back: the emptied piece copied the value of `src`.
  // (Lane exchanges run with all eight lanes active: a lane masked off in a
  // branch does not provide its value.)
  const double bpos0 = a8_get(Br, gb, pos >= 0 ? pos : 0);
  const double bpos1 = a8_get(Bm, gb, pos >= 0 ? pos : 0);
  double gO0 = pos >= 0 ? bpos0 : 0.0, gO1 = pos >= 0 ? bpos1 : 0.0;
  int src = -1;
  if (merge) src = !tr ? ((flags & FL_CROSS_L) ? iR : into) : ((flags & FL_CROSS_R) ? iL : into);
  {
    const double sr_ = a8_get(Br, gb, skip >= 0 ? skip : 0);
    const double sm_ = a8_get(Bm, gb, skip >= 0 ? skip : 0);
    if (merge && pos == src) {
      gO0 += sr_;
      gO1 += sm_;
    }
  }
  // hl^{n+1} = hl^n + w* dt (+- h after a crossing)
  const double ghl1 = B.hl_bar[k];
  double ghl = ghl1;
  Z.gdt += (c == 0) ? ghl1 * wstar : 0.0;

  // Part 2 at W^count, then the pseudo iterations in reverse.  The interface
  // linearisations at the tape's roots do not depend on the adjoints: they
  // are computed four passes at a time by the group's four lane pairs
  // (a8_lin_batch, every fourth pass; the pass counter is common to the
  // groups of the wave, so they batch together) and each pass's lane ic
  // reads its own from LDS.  Each pass's iterate is read from the tape one
  // pass ahead, so that the loads overlap the pass before.
  const int gi = (int)threadIdx.x >> 3;
  const int pic = (skip >= 0 && Z.ic >= skip) ? Z.ic + 1 : Z.ic;
  const int pic1 = (skip >= 0 && Z.ic + 1 >= skip) ? Z.ic + 2 : Z.ic + 1;
  const int ep = pos >= 0 ? pos : 0;
  const double* e = T + TAPE_HDR + (long long)cnt * E;
  double W0 = e[ep], W1 = e[MC + ep];
  double gW0 = 0.0, gW1 = 0.0;
  double tW0 = 0.0, tW1 = 0.0;
  if (cnt > 0) {
    const double* el = T + TAPE_HDR + (long long)(cnt - 1) * E;
    tW0 = el[ep];
    tW1 = el[MC + ep];
  }
  for (int i = 0; i <= cnt; ++i) {
    const int l = cnt - i;
    if ((i & 3) == 0) a8_lin_batch(M, Z, T, E, MC, l, l + 1 < 4 ? l + 1 : 4, pic, pic1, s_lin[gi]);
    IfaceLin Q;
    Q.F0 = Q.F1 = Q.w = 0.0;
    if (c == Z.ic) a8_lin_load(s_lin[gi][l & 3], phl, Q);
    if (i == 0) {
      a8_pass_rev(M, Z, true, W0, W1, Q, W0, W1, gO0, gO1, (c == Z.ic) ? ghl1 * dt : 0.0, gW0,
                  gW1);
    } else {
      const double N0 = W0, N1 = W1;
      W0 = tW0;
      W1 = tW1;
      if (l > 0) {
        const double* en = T + TAPE_HDR + (long long)(l - 1) * E;
        tW0 = en[ep];
        tW1 = en[MC + ep];
      }
      const double o0 = gW0, o1 = gW1;
      gW0 = gW1 = 0.0;
      a8_pass_rev(M, Z, false, W0, W1, Q, N0, N1, o0, o1, 0.0, gW0, gW1);
    }
  }
  // W^0 = U0
  Z.gU00 += gW0;
  Z.gU01 += gW1;
  // theta = min(theta_nb, h_end / h), h_end = h^n +- w_pred dt (moving cells)
  double gwp_l = 0.0;
  if ((mvl && !cl_l) || (mvr && !cl_r)) {
    const double g = Z.gth / h;
    Z.ghn += g;
    gwp_l = Z.mv * (g * dt);
    Z.gdt += Z.mv * (g * wp);
  }
  const double gwp = a8_sum(gwp_l);
  // lengths at t^n from hl (the moving cells' h^n)
  const double ghn_l = a8_get(Z.ghn, gb, Z.ic), ghn_r = a8_get(Z.ghn, gb, Z.ic + 1);
  // zone set-up: U0 from U^n (merge average) -> adjoint by zone position
  const double gi_r = (pos == into) ? Z.gU00 : 0.0, gi_m = (pos == into) ? Z.gU01 : 0.0;
  const double gir = a8_sum(gi_r), gim = a8_sum(gi_m);  // adjoint of the merged cell's U0
  double Gown0 = (pos == into) ? (h / hm) * Z.gU00 : Z.gU00;
  double Gown1 = (pos == into) ? (h / hm) * Z.gU01 : Z.gU01;
  // lane j (zone position j) takes the adjoint of the active cell at j
  const int cj = (skip >= 0 && c > skip) ? c - 1 : c;
  double G0 = a8_get(Gown0, gb, cj), G1 = a8_get(Gown1, gb, cj);
  if (c == skip) {
    G0 = (ht / hm) * gir;
    G1 = (ht / hm) * gim;
  }
  if (merge) {
    double ght = ((rskip - Mr) * gir + (mskip - Mm) * gim) / hm;
    if (!tr) {
      ght += ghn_l;
      ghl -= ghn_r;
      ghl += ght;
    } else {
      ght += ghn_r;
      ghl += ghn_l;
      ghl -= ght;
    }
  } else {
    ghl += ghn_l - ghn_r;
  }
  // predicting solve on U^n of the two cut pieces (positions iL, iR)
  double gtau_p = 0.0;
  {
    const double nUr = a8_get(Ur, gb, c < 7 ? c + 1 : 7), nUm = a8_get(Um, gb, c < 7 ? c + 1 : 7);
    double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
    if (c == iL && gwp != 0.0) {
      IfaceLin Q;
      d_iface_lin(M, phl, Ur, Um, nUr, nUm, T[TH_IPL], T[TH_IPR], Q);
      d_iface_adj(Q, 0.0, 0.0, gwp, a0, a1, b0, b1, gtau_p);
    }
    const double fb0 = a8_get(b0, gb, c > 0 ? c - 1 : 0), fb1 = a8_get(b1, gb, c > 0 ? c - 1 : 0);
    G0 += a0;
    G1 += a1;
    if (c == iR) {
      G0 += fb0;
      G1 += fb1;
    }
  }
  if (c < nr) {
    g0r[zlo + c] = G0;
    g0m[zlo + c] = G1;
  }
  const double sdt = a8_sum(Z.gdt), stau = a8_sum(Z.gtau + gtau_p);
  const double sFL0 = a8_sum(Z.gFL0), sFL1 = a8_sum(Z.gFL1);
  const double sFR0 = a8_sum(Z.gFR0), sFR1 = a8_sum(Z.gFR1);
  if (c == 0) {
    double* zo = B.zadj + 5 * (long long)k;
    zo[0] = sFL0;
    zo[1] = sFL1;
    zo[2] = sFR0;
    zo[3] = sFR1;
    zo[4] = sdt;
    B.tau_bar[k] += stau;
    B.hl_bar[k] = ghl;
  }
}

// ---------------------------------------------------------------------------
// bulk pass
// ---------------------------------------------------------------------------
__device__ __forceinline__ double d_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Lane j of a row holds cell s = base - 1 + j (lane 0 / 63: halo) and handles
// the face between s and s+1: its adjoint is
//   gF = lam (gU^{n+1}_{s+1} [s+1 bulk] - gU^{n+1}_s [s bulk])
//        + gF_left of a zone starting at s+1 + gF_right of a zone ending at s,
// sent through the HLL Jacobians to s (own lane) and s+1 (shuffled up).
// Cells outside the domain are the wall / transmissive ghosts of the
// boundary cells, so their adjoints fold back onto those.  The faces with a
// zone cell on either side need the zone pass's results, so they are left to
// the per-problem pass (d_edge_faces) and zone cells are not written: the
// zone pass can run at the same time.
template <int R>
__global__ __launch_bounds__(256) void k_bulk_adj(StepArgs A, AdjArgs B) {
  constexpr int OUT = 62;
  __shared__ int s_zlo[MAX_IF_PER_PROB], s_zhi[MAX_IF_PER_PROB], s_sR[MAX_IF_PER_PROB];
  __shared__ double s_red[4];
  __shared__ unsigned long long s_mx[4];
  __shared__ int s_ix[4];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int tile = blockIdx.x;
  const int p = A.tile_prob[tile];
  const int t0 = A.tile_start[tile];
  const int tend = t0 + A.tile_len[tile];
  const long long so = A.slot_off[p];
  const int ns = (int)(A.slot_off[p + 1] - so);
  const double* __restrict__ r0 = A.rho0 + so;
  const double* __restrict__ m0 = A.mom0 + so;
  const double* __restrict__ g1r = B.gr1 + so;
  const double* __restrict__ g1m = B.gm1 + so;
  double* __restrict__ g0r = B.gr0 + so;
  double* __restrict__ g0m = B.gm0 + so;
  const double dt = A.dt[p];
  if (dt == 0.0) {  // frozen: U^{n+1} = U^n
    for (int c = t0 + tid; c < tend; c += 256) {
      g0r[c] = g1r[c];
      g0m[c] = g1m[c];
    }
    if (tid == 0) {
      B.tile_gdt[tile] = 0.0;
      B.tile_smax[tile] = 0ull;
      B.tile_sidx[tile] = -1;
    }
    return;
  }
  const Mat& M = A.mat;
  const double h = A.h[p];
  const double lam = dt / h;
  const int i0 = A.iface_off[p];
  const int nif = A.iface_off[p + 1] - i0;
  const int pf = A.phase_first[p];
  const int bcL = A.par.bc_left, bcR = A.par.bc_right;
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

  double rr[R], mm[R], br[R], bm[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int s = t0 + (wv * R + r) * OUT - 1 + lane;
    const int se = s < 0 ? 0 : (s > ns - 1 ? ns - 1 : s);
    double rv = r0[se], mv = m0[se];
    if ((s < 0 && bcL == 0) || (s >= ns && bcR == 0)) mv = -mv;
    rr[r] = rv;
    mm[r] = mv;
    const bool in = s >= 0 && s < ns;
    br[r] = in ? g1r[se] : 0.0;
    bm[r] = in ? g1m[se] : 0.0;
  }

  double gdt = 0.0;
  unsigned long long vmax = 0;
  int vidx = 0x7fffffff;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int s = t0 + (wv * R + r) * OUT - 1 + lane;
    const int rowbase = t0 + (wv * R + r) * OUT;
    if (rowbase >= tend) break;  // uniform over the wave
    const bool in = s >= 0 && s < ns;
    const int se = s < 0 ? 0 : (s > ns - 1 ? ns - 1 : s);
    int ph = pf;
    bool zone = false;
    for (int j = 0; j < nif; ++j) {
      ph ^= (s_sR[j] <= se) ? 1 : 0;
      zone = zone || (s >= s_zlo[j] && s <= s_zhi[j]);
    }
    const bool bulk = in && !zone;
    // a face with a zone cell on either side is the per-problem pass's (the
    // shift runs on every lane: a lane masked off would not provide its value)
    const int zoneR = d_wave_next_i(zone ? 1 : 0);
    const bool edge = zone || zoneR != 0;
    const double rho = rr[r], mom = mm[r];
    const double u = mom / rho;
    const double pr = d_pres(M, ph, rho);
    const double rhoR = d_wave_next(rho);
    const double momR = d_wave_next(mom);
    const double uR = d_wave_next(u);
    const double prR = d_wave_next(pr);
    const double bR0 = d_wave_next(br[r]);
    const double bR1 = d_wave_next(bm[r]);
    const int bulkR = d_wave_next_i(bulk ? 1 : 0);
    double F0, F1;  // forward flux on the face s | s+1
    d_hll_prim(d_a(M, ph), rho, mom, u, pr, rhoR, momR, uR, prR, F0, F1);
    const double Fl0 = d_wave_prev(F0);
    const double Fl1 = d_wave_prev(F1);
    // adjoint of the face flux
    double gf0 = 0.0, gf1 = 0.0;
    if (bulkR && !edge) {
      gf0 += lam * bR0;
      gf1 += lam * bR1;
    }
    if (bulk && !edge) {
      gf0 -= lam * br[r];
      gf1 -= lam * bm[r];
    }
    double cl_r = 0.0, cl_m = 0.0, cr_r = 0.0, cr_m = 0.0;
    if (gf0 != 0.0 || gf1 != 0.0)
      d_hll_adj(M, ph, rho, mom, rhoR, momR, gf0, gf1, cl_r, cl_m, cr_r, cr_m);
    if (s == -1) {  // left ghost: fold onto cell 0, which lane j+1 holds
      cr_r += cl_r;
      cr_m += (bcL == 0) ? -cl_m : cl_m;
    }
    if (s == ns - 1) {  // right neighbour is the ghost of this cell
      cl_r += cr_r;
      cl_m += (bcR == 0) ? -cr_m : cr_m;
    }
    const double from_r = d_wave_prev(cr_r);
    const double from_m = d_wave_prev(cr_m);
    if (lane >= 1 && lane <= OUT && s < tend && in) {
      if (bulk) {  // zone cells: the zone pass's
        gdt -= ((F0 - Fl0) * br[r] + (F1 - Fl1) * bm[r]) / h;
        g0r[s] = br[r] + cl_r + from_r;
        g0m[s] = bm[r] + cl_m + from_m;
      }
      const unsigned long long b =
          (unsigned long long)__double_as_longlong(fabs(mom / rho) + d_a(M, ph));
      if (b > vmax || (b == vmax && s < vidx)) {
        vmax = b;
        vidx = s;
      }
    }
  }
  gdt = d_wave_sum(gdt);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long om = __shfl_xor(vmax, off, 64);
    const int oi = __shfl_xor(vidx, off, 64);
    if (om > vmax || (om == vmax && oi < vidx)) {
      vmax = om;
      vidx = oi;
    }
  }
  if (lane == 0) {
    s_red[wv] = gdt;
    s_mx[wv] = vmax;
    s_ix[wv] = vidx;
  }
  __syncthreads();
  if (tid == 0) {
    double g = 0.0;
    unsigned long long mx = 0;
    int ix = 0x7fffffff;
    for (int w = 0; w < 4; ++w) {
      g += s_red[w];
      if (s_mx[w] > mx || (s_mx[w] == mx && s_ix[w] < ix)) {
        mx = s_mx[w];
        ix = s_ix[w];
      }
    }
    B.tile_gdt[tile] = g;
    B.tile_smax[tile] = mx;
    B.tile_sidx[tile] = ix;
  }
}

// ---------------------------------------------------------------------------
// per-problem pass: dt and t
// ---------------------------------------------------------------------------
// The faces that k_bulk_adj left out, those with a zone cell on
// either side (each zone's two bounding faces, a face between two adjacent
// zones once), of problem p: the face adjoint as k_bulk_adj forms it, sent
// through the HLL Jacobians to both cells (ghosts folded back), added to
// their adjoints.  One thread per problem, after the zone and bulk passes.
__device__ void d_edge_faces(const StepArgs& A, const AdjArgs& B, int p, double dt) {
  const Mat& M = A.mat;
  const Par& P = A.par;
  const long long so = A.slot_off[p];
  const int ns = (int)(A.slot_off[p + 1] - so);
  const double h = A.h[p];
  const double lam = dt / h;
  const int i0 = A.iface_off[p];
  const int nif = A.iface_off[p + 1] - i0;
  const int pf = A.phase_first[p];
  const int bcL = P.bc_left, bcR = P.bc_right;
  const double* r0 = A.rho0 + so;
  const double* m0 = A.mom0 + so;
  const double* g1r = B.gr1 + so;
  const double* g1m = B.gm1 + so;
  double* g0r = B.gr0 + so;
  double* g0m = B.gm0 + so;
  auto zone_of = [&](int j, int& lo, int& hi) {
    bool tr;
    d_zone_range(A.rec_home0[i0 + j] + j, A.rec_hl0[i0 + j], h, P.zone_half, ns, lo, hi, tr);
  };
  // the face between slots a and a + 1 (a = -1, ns - 1: a ghost on one side)
  auto face = [&](int a) {
    const int se = a < 0 ? 0 : a, seR = a + 1 > ns - 1 ? ns - 1 : a + 1;
    int ph = pf;
    bool zl = false, zr = false;
    double gf0 = 0.0, gf1 = 0.0;
    for (int j = 0; j < nif; ++j) {
      int lo, hi;
      zone_of(j, lo, hi);
      ph ^= (A.rec_home0[i0 + j] + j + 1 <= se) ? 1 : 0;
      zl = zl || (a >= lo && a <= hi);
      zr = zr || (a + 1 >= lo && a + 1 <= hi);
      const double* zg = B.zadj + 5 * (long long)(i0 + j);
      if (lo == a + 1) {
        gf0 += zg[0];
        gf1 += zg[1];
      }
      if (hi == a) {
        gf0 += zg[2];
        gf1 += zg[3];
      }
    }
    const bool bulkL = a >= 0 && !zl, bulkR = a + 1 < ns && !zr;
    if (bulkR) {
      gf0 += lam * g1r[a + 1];
      gf1 += lam * g1m[a + 1];
    }
    if (bulkL) {
      gf0 -= lam * g1r[a];
      gf1 -= lam * g1m[a];
    }
    if (gf0 == 0.0 && gf1 == 0.0) return;
    double rl = r0[se], ml = m0[se], rr = r0[seR], mr = m0[seR];
    if (a < 0 && bcL == 0) ml = -ml;
    if (a + 1 >= ns && bcR == 0) mr = -mr;
    double cl_r = 0.0, cl_m = 0.0, cr_r = 0.0, cr_m = 0.0;
    d_hll_adj(M, ph, rl, ml, rr, mr, gf0, gf1, cl_r, cl_m, cr_r, cr_m);
    if (a == -1) {
      cr_r += cl_r;
      cr_m += (bcL == 0) ? -cl_m : cl_m;
    }
    if (a == ns - 1) {
      cl_r += cr_r;
      cl_m += (bcR == 0) ? -cr_m : cr_m;
    }
    if (a >= 0) {
      g0r[a] += cl_r;
      g0m[a] += cl_m;
    }
    if (a + 1 < ns) {
      g0r[a + 1] += cr_r;
      g0m[a + 1] += cr_m;
    }
  };
  int last = -2;
  for (int j = 0; j < nif; ++j) {
    int lo, hi;
    zone_of(j, lo, hi);
    if (lo - 1 != last) face(lo - 1);
    face(hi);
    last = hi;
  }
}

__global__ void k_fin_adj(StepArgs A, AdjArgs B, int P) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const double dt = A.dt[p];
  if (dt == 0.0) return;
  d_edge_faces(A, B, p, dt);
  double gdt = 0.0;
  unsigned long long mx = 0;
  int ix = 0x7fffffff;
  for (int t = B.tile_off[p]; t < B.tile_off[p + 1]; ++t) {
    gdt += B.tile_gdt[t];
    if (B.tile_smax[t] > mx || (B.tile_smax[t] == mx && B.tile_sidx[t] < ix)) {
      mx = B.tile_smax[t];
      ix = B.tile_sidx[t];
    }
  }
  for (int k = A.iface_off[p]; k < A.iface_off[p + 1]; ++k) gdt += B.zadj[5 * (long long)k + 4];
  const double tb = B.t_bar[p];
  const bool advanced = B.steps1[p] > B.steps0[p];
  const bool clipped = A.clipped[p] != 0;
  double ntb = tb;  // t^{n+1} = t^n (failed step) or t^n + dt
  if (advanced && clipped) ntb = 0.0;  // t^{n+1} = t_end
  if (advanced && !clipped) gdt += tb;
  if (clipped) {
    ntb -= gdt;  // dt = t_end - t^n
  } else if (ix >= 0 && ix != 0x7fffffff) {
    // dt = C h / S, S = |u| + a at slot ix: dS adjoint = -dt / S * gdt
    const double S = __longlong_as_double((long long)mx);
    const double gS = -(dt / S) * gdt;
    const long long so = A.slot_off[p];
    const double r = A.rho0[so + ix], m = A.mom0[so + ix];
    const double u = m / r;
    const double sg = u < 0.0 ? -1.0 : 1.0;
    B.gr0[so + ix] += gS * sg * (-(u / r));
    B.gm0[so + ix] += gS * sg / r;
  }
  B.t_bar[p] = ntb;
}

// Fixed-order sum of n doubles by one workgroup (deterministic).
__global__ __launch_bounds__(256) void k_sum(const double* x, int n, double* out) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += x[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

hipError_t launch_zone_adj(const StepArgs& A, const AdjArgs& B, int lanes, hipStream_t s) {
  if (A.n_iface <= 0) return hipSuccess;
  if (lanes == 8) {
    const int waves = (A.n_iface + 7) / 8;
    switch (A.par.zone_half) {
      case 1: k_zone_adj8<1><<<waves, 64, 0, s>>>(A, B); break;
      case 2: k_zone_adj8<2><<<waves, 64, 0, s>>>(A, B); break;
      case 3: k_zone_adj8<3><<<waves, 64, 0, s>>>(A, B); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const int blocks = (A.n_iface + 63) / 64;
  switch (A.par.zone_half) {
    case 1: k_zone_adj<1><<<blocks, 64, 0, s>>>(A, B); break;
    case 2: k_zone_adj<2><<<blocks, 64, 0, s>>>(A, B); break;
    case 3: k_zone_adj<3><<<blocks, 64, 0, s>>>(A, B); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bulk_adj(const StepArgs& A, const AdjArgs& B, int tile_class, int n_tiles,
                           hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  switch (tile_class) {
    case 256: k_bulk_adj<1><<<n_tiles, 256, 0, s>>>(A, B); break;
    case 512: k_bulk_adj<2><<<n_tiles, 256, 0, s>>>(A, B); break;
    case 1024: k_bulk_adj<4><<<n_tiles, 256, 0, s>>>(A, B); break;
    case 2048: k_bulk_adj<8><<<n_tiles, 256, 0, s>>>(A, B); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finalize_adj(const StepArgs& A, const AdjArgs& B, int P, hipStream_t s) {
  if (P <= 0) return hipSuccess;
  k_fin_adj<<<(P + 255) / 256, 256, 0, s>>>(A, B, P);
  return hipGetLastError();
}

hipError_t launch_sum(const double* x, int n, double* out, hipStream_t s) {
  k_sum<<<1, 256, 0, s>>>(x, n, out);
  return hipGetLastError();
}

}  // namespace imexds
