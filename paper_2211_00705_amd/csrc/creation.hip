// creation.hip -- phase creation (cavitation, nucleation) for batches of
// single-phase Riemann problems: kernel and C ABI of include/imexds_creation.h.
//
// Three passes, one lane per problem each.  Pass 0 (k_cr_partition) queues
// the problems by phase.  Pass 1 (k_cr_detect): step (i), a scalar Newton on
// the single-phase star pressure with the outer waves of the interface solver
// (d_wave), for every problem in that order; those that create a new phase
// are queued by phase.  Pass 2 (k_cr_solve): step (ii), a three-unknown
// Newton-Armijo on the star pressures of the five-state problem, over the
// queues, so that a wave's lanes share a phase and a path (2.6x faster than
// one pass over interleaved liquid and vapour problems).  Each problem's
// arithmetic does not depend on its place in a queue.  Every expression is
// written in the order of its definition and evaluated without contraction,
// so results are bitwise those of any IEEE FP64 evaluation of the same
// expressions.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/imexds_creation.h"
#include "imexds_device.hpp"

namespace imexds {
namespace {

// per-phase constants of the creation solve
__device__ __forceinline__ double c_ia2(const Mat& M, int ph) { return ph == VAP ? M.ia2v : M.ia2l; }

// Step (i): star pressure of the single-phase problem; 0 on success, 1 if no
// root with rho* > 0 was found.
__device__ int c_single_rp(const Mat& M, const Side& L, const Side& R, double& ps) {
  const double du = R.u - L.u;
  double p = 0.5 * (L.p + R.p);
  for (int it = 0; it < 100; ++it) {
    double rl, vl, gl, fl, dfl, rr, vr, gr, fr, dfr;
    if (!d_wave(M, L, p, rl, vl, gl, fl, dfl) || !d_wave(M, R, p, rr, vr, gr, fr, dfr)) return 1;
    double dp = -(fl + fr + du) / (dfl + dfr);
    if (!d_finite(dp)) return 1;
    double pn = p + dp;
    int k = 0;
    while (!(d_rho_of_p(M, L.ph, pn) > 0.0) && k < 60) {
      dp = 0.5 * dp;
      pn = p + dp;
      ++k;
    }
    if (k == 60) return 1;
    const double sc = fabs(p) > M.p0 ? fabs(p) : M.p0;
    p = pn;
    // converged when the step is below 1e-12 of the pressure scale or below
    // 1e-13 of the density it implies (the liquid resolves p* only to about
    // 1e-7 Pa through its density)
    if (fabs(dp) <= 1e-12 * sc || fabs(dp) <= 1e-13 * (d_a2(M, L.ph) * d_rho_of_p(M, L.ph, p))) {
      ps = p;
      return 0;
    }
  }
  return 1;
}

// one state of the five-state problem at its star pressure
struct CState {
  double rs, v, g, f, df;
};

// mass flux through a boundary between l (left, phase phl) and r from the
// kinetic relation, and its derivatives in the left and right pressure
__device__ __forceinline__ bool c_kinetic(const Mat& M, int phl, const CState& l, const CState& r,
                                          double pl, double pr, double ia2l, double ia2r,
                                          double& z, double& dzl, double& dzr) {
  const double vl = l.v, vr = r.v;
  const double pV = phl == VAP ? pl : pr;
  const double q = M.tau * pV;
  const double jg = r.g - l.g;
  const double jv2 = vr * vr - vl * vl;
  const double A = 0.5 * q * jv2;
  const double C = q * jg;
  const double D = 1.0 - 4.0 * A * C;
  if (!(D >= 0.0) || !d_finite(D)) return false;
  const double sD = sqrt(D);
  const double isD = 1.0 / sD;
  const double zz = 2.0 * C / (1.0 + sD);
  double dAl = q * ((vl * vl * vl) * ia2l);
  double dAr = -(q * ((vr * vr * vr) * ia2r));
  double dCl = -(q * vl);
  double dCr = q * vr;
  if (phl == VAP) {
    dAl += (0.5 * M.tau) * jv2;
    dCl += M.tau * jg;
  } else {
    dAr += (0.5 * M.tau) * jv2;
    dCr += M.tau * jg;
  }
  z = zz;
  dzl = (dAl * zz * zz + dCl) * isD;
  dzr = (dAr * zz * zz + dCr) * isD;
  return true;
}

struct CEval {
  double E1, E2, E3, J[3][3], m2, zl, zr;
  CState a, b, c;
};

__device__ bool c_eval(const Mat& M, const Side& L, const Side& R, const Side& S, double izref,
                       double pa, double pb, double pc, CEval& E) {
  if (!d_wave(M, L, pa, E.a.rs, E.a.v, E.a.g, E.a.f, E.a.df) ||
      !d_wave(M, S, pb, E.b.rs, E.b.v, E.b.g, E.b.f, E.b.df) ||
      !d_wave(M, R, pc, E.c.rs, E.c.v, E.c.g, E.c.f, E.c.df))
    return false;
  const double ia2o = c_ia2(M, L.ph), ia2n = c_ia2(M, S.ph);
  double dla, dlb, drb, drc;
  if (!c_kinetic(M, L.ph, E.a, E.b, pa, pb, ia2o, ia2n, E.zl, dla, dlb)) return false;
  if (!c_kinetic(M, S.ph, E.b, E.c, pb, pc, ia2n, ia2o, E.zr, drb, drc)) return false;
  const double zl = E.zl, zr = E.zr;
  const double jl = E.b.v - E.a.v, jr = E.c.v - E.b.v;
  const double ea = (E.a.v * E.a.v) * ia2o;
  const double eb = (E.b.v * E.b.v) * ia2n;
  const double ec = (E.c.v * E.c.v) * ia2o;
  E.E1 = (pb - pa) + zl * zl * jl;
  E.E2 = (pc - pb) + zr * zr * jr;
  E.E3 = (E.a.f + E.c.f) + zl * jl + zr * jr + (R.u - L.u);
  E.J[0][0] = -1.0 + 2.0 * zl * dla * jl + zl * zl * ea;
  E.J[0][1] = 1.0 + 2.0 * zl * dlb * jl - zl * zl * eb;
  E.J[0][2] = 0.0;
  E.J[1][0] = 0.0;
  E.J[1][1] = -1.0 + 2.0 * zr * drb * jr + zr * zr * eb;
  E.J[1][2] = 1.0 + 2.0 * zr * drc * jr - zr * zr * ec;
  E.J[2][0] = E.a.df + dla * jl + zl * ea;
  E.J[2][1] = dlb * jl - zl * eb + drb * jr + zr * eb;
  E.J[2][2] = E.c.df + drc * jr - zr * ec;
  if (!d_finite(E.E1) || !d_finite(E.E2) || !d_finite(E.E3)) return false;
  const double s1 = E.E1 * izref, s2 = E.E2 * izref;
  E.m2 = s1 * s1 + s2 * s2 + E.E3 * E.E3;
  return true;
}

// determinant of the 3x3 matrix whose column k is replaced by r (k = -1: none)
__device__ __forceinline__ double c_det(const double J[3][3], int k, const double* r) {
  double A[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A[i][j] = j == k ? r[i] : J[i][j];
  return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
         A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
         A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

// Cramer's rule; the determinant is expanded by cofactors of the first row
__device__ __forceinline__ bool c_solve3(const double J[3][3], const double* r, double* x) {
  const double c0 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c1 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c2 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double det = J[0][0] * c0 + J[0][1] * c1 + J[0][2] * c2;
  if (!(det != 0.0) || !d_finite(det)) return false;
  const double id = 1.0 / det;
#pragma unroll
  for (int k = 0; k < 3; ++k) x[k] = c_det(J, k, r) * id;
  return true;
}

// Step (ii) and outputs for a problem that step (i) sent to creation: fills
// the record o (already zero but P1) and returns 1, or -1 on failure.
__device__ int c_solve(const Mat& M, int ph, double rl, double ml, double rr, double mr,
                       int maxit, double rtol, double* o) {
  Side L, R, S;
  d_side(M, ph, rl, ml, L);
  d_side(M, ph, rr, mr, R);
  const int nph = 1 - ph;
  d_side(M, nph, nph == VAP ? M.rhov0 : M.rhol0, 0.0, S);
  const double aph = ph == VAP ? M.av : M.al;
  const double zL = rl * aph, zR = rr * aph;
  const double izref = 1.0 / (zL > zR ? zL : zR);
  double x0 = M.p0, x1 = M.p0, x2 = M.p0;
  CEval E, Et;
  if (!c_eval(M, L, R, S, izref, x0, x1, x2, E)) return -1;
  int it;
  bool conv = false;
  for (it = 0; it < maxit && !conv; ++it) {
    const double rhs[3] = {-E.E1, -E.E2, -E.E3};
    double d[3];
    if (!c_solve3(E.J, rhs, d)) return -1;
    double sc = 0.0, st = 0.0;
    const double xs[3] = {x0, x1, x2};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (fabs(xs[i]) > sc) sc = fabs(xs[i]);
      if (fabs(d[i]) > st) st = fabs(d[i]);
    }
    if (M.p0 > sc) sc = M.p0;
    if (!d_finite(st)) return -1;
    if (st <= rtol * sc) {
      if (c_eval(M, L, R, S, izref, x0 + d[0], x1 + d[1], x2 + d[2], Et)) {
        x0 = x0 + d[0];
        x1 = x1 + d[1];
        x2 = x2 + d[2];
        E = Et;
      }
      conv = true;
      break;
    }
    double lam = 1.0;
    bool acc = false;
    int k;
    for (k = 0; k <= 20; ++k) {
      const double c = 1.0 - 1e-4 * lam;
      if (c_eval(M, L, R, S, izref, x0 + lam * d[0], x1 + lam * d[1], x2 + lam * d[2], Et) &&
          Et.m2 <= (c * c) * E.m2) {
        x0 = x0 + lam * d[0];
        x1 = x1 + lam * d[1];
        x2 = x2 + lam * d[2];
        E = Et;
        acc = true;
        break;
      }
      lam *= 0.5;
    }
    if (!acc) {
      if (st <= 1e-8 * sc) {
        conv = true;
        break;
      }
      return -1;
    }
    if (k == 0 && st <= 1e-10 * sc) conv = true;
  }
  if (!conv) return -1;
  o[IMEXDS_CR_KIND] = ph == LIQ ? 1.0 : 2.0;
  o[IMEXDS_CR_PA] = x0;
  o[IMEXDS_CR_PB] = x1;
  o[IMEXDS_CR_PC] = x2;
  o[IMEXDS_CR_RA] = E.a.rs;
  o[IMEXDS_CR_RB] = E.b.rs;
  o[IMEXDS_CR_RC] = E.c.rs;
  const double ua = L.u - E.a.f;
  const double uc = R.u + E.c.f;
  const double ub = ua - E.zl * (E.b.v - E.a.v);
  o[IMEXDS_CR_UA] = ua;
  o[IMEXDS_CR_UB] = ub;
  o[IMEXDS_CR_UC] = uc;
  o[IMEXDS_CR_ZL] = E.zl;
  o[IMEXDS_CR_ZR] = E.zr;
  o[IMEXDS_CR_WL] = ub + E.zl * E.b.v;
  o[IMEXDS_CR_WR] = ub + E.zr * E.b.v;
  o[IMEXDS_CR_FL0] = -E.zl;
  o[IMEXDS_CR_FL1] = -E.zl * ub + x1;
  o[IMEXDS_CR_FR0] = -E.zr;
  o[IMEXDS_CR_FR1] = -E.zr * ub + x1;
  o[IMEXDS_CR_ITERS] = (double)(it + 1);
  return 1;
}

__global__ void k_cr_init(int* ctr) {
  if (threadIdx.x < 4) ctr[threadIdx.x] = 0;
}

// lane's rank among the lanes of its wave whose bit is set in mask
__device__ __forceinline__ int c_rank(unsigned long long mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

constexpr int CR_BLOCK = 1024;  // threads per workgroup of the queueing passes

// Appends the lanes whose flag is set to a queue: front (from index 0 up) or
// back (from n - 1 down).  Counts are summed per workgroup in LDS, so each
// workgroup makes one atomic per end (atomics on one address serialise:
// one per wave cost 0.37 ms per 2^20 problems).  Every thread of the
// workgroup must call it.
__device__ __forceinline__ void c_enqueue(bool front, bool back, int j, int n, int* ctr_front,
                                          int* ctr_back, int* q) {
  __shared__ int s_cnt[2][CR_BLOCK / 64];
  __shared__ int s_base[2];
  const unsigned long long mf = __ballot(front);
  const unsigned long long mb = __ballot(back);
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  if (lane == 0) {
    s_cnt[0][w] = __popcll(mf);
    s_cnt[1][w] = __popcll(mb);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int tf = 0, tb = 0;
    for (int v = 0; v < CR_BLOCK / 64; ++v) {
      tf += s_cnt[0][v];
      tb += s_cnt[1][v];
    }
    s_base[0] = tf ? atomicAdd(ctr_front, tf) : 0;
    s_base[1] = tb ? atomicAdd(ctr_back, tb) : 0;
  }
  __syncthreads();
  int of = s_base[0], ob = s_base[1];
  for (int v = 0; v < w; ++v) {
    of += s_cnt[0][v];
    ob += s_cnt[1][v];
  }
  if (front) q[of + c_rank(mf)] = j;
  if (back) q[n - 1 - (ob + c_rank(mb))] = j;
}

// Pass 0: queue A holds the liquid problems from its front and all others
// from its back, so that step (i) runs on lanes of one phase.
__global__ __launch_bounds__(CR_BLOCK) void k_cr_partition(int n, const int* __restrict__ phase,
                                                      int* ctr, int* qa) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = j < n;
  const bool liq = active && phase[j] == LIQ;
  c_enqueue(liq, active && !liq, (int)j, n, ctr + 0, ctr + 1, qa);
}

// Pass 1: validation and step (i) for every problem (in queue A order); a
// problem that creates a new phase goes to queue B: liquid ones from its
// front, vapour ones from its back; status 2 meanwhile.
__global__ __launch_bounds__(CR_BLOCK) void k_cr_detect(Mat M, int n, const int* __restrict__ phase,
                                                   const double* __restrict__ rl,
                                                   const double* __restrict__ ml,
                                                   const double* __restrict__ rr,
                                                   const double* __restrict__ mr, double p_min,
                                                   double p_tilde, int* __restrict__ status,
                                                   double* __restrict__ out, int* ctr,
                                                   const int* qa, int* q) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = t < n;
  const int cl = ctr[0];
  const long long j = !active ? 0 : (t < cl ? qa[t] : qa[n - 1 - (int)(t - cl)]);
  int create = 0, ph = 0;
  if (active) {
    double* oj = out + j * IMEXDS_CR_FIELDS;
#pragma unroll
    for (int i = 0; i < IMEXDS_CR_FIELDS; ++i) oj[i] = 0.0;
    ph = phase[j];
    const double a = rl[j], b = rr[j];
    if (!(a > 0.0) || !(b > 0.0) || (ph != LIQ && ph != VAP)) {
      status[j] = -1;
    } else {
      Side L, R;
      d_side(M, ph, a, ml[j], L);
      d_side(M, ph, b, mr[j], R);
      double p1 = 0.0;
      const int none = c_single_rp(M, L, R, p1);
      oj[IMEXDS_CR_P1] = none ? 0.0 : p1;
      create = none ? 1 : (ph == LIQ ? p1 < p_min : p1 > p_tilde);
      status[j] = create ? 2 : 0;
    }
  }
  c_enqueue(create && ph == LIQ, create && ph == VAP, (int)j, n, ctr + 2, ctr + 3, q);
}

// Pass 2: step (ii) over the queues, liquid problems first, so that the
// lanes of a wave share one phase and one path through the solve.
__global__ __launch_bounds__(256) void k_cr_solve(Mat M, int n, const int* __restrict__ phase,
                                                  const double* __restrict__ rl,
                                                  const double* __restrict__ ml,
                                                  const double* __restrict__ rr,
                                                  const double* __restrict__ mr, int maxit,
                                                  double rtol, int* __restrict__ status,
                                                  double* __restrict__ out, const int* ctr,
                                                  const int* q) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int cl = ctr[2], cv = ctr[3];
  int j;
  if (t < cl)
    j = q[t];
  else if (t - cl < cv)
    j = q[n - 1 - (int)(t - cl)];
  else
    return;
  double o[IMEXDS_CR_FIELDS];
  double* oj = out + (long long)j * IMEXDS_CR_FIELDS;
#pragma unroll
  for (int i = 0; i < IMEXDS_CR_FIELDS; ++i) o[i] = 0.0;
  o[IMEXDS_CR_P1] = oj[IMEXDS_CR_P1];
  const int st = c_solve(M, phase[j], rl[j], ml[j], rr[j], mr[j], maxit, rtol, o);
  status[j] = st;
  if (st == 1) {
#pragma unroll
    for (int i = 0; i < IMEXDS_CR_FIELDS; ++i) oj[i] = o[i];
  }
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace
}  // namespace imexds

extern "C" int imexds_creation_rp(const imexds_material* mat, int32_t n, const int32_t* phase,
                                  const double* rho_l, const double* mom_l, const double* rho_r,
                                  const double* mom_r, double p_min, double p_tilde, int32_t maxit,
                                  double rtol, int32_t* status, double* out, void* hip_stream) {
  using namespace imexds;
  if (!mat || n < 0 || maxit < 1 || !finite_pos(rtol)) return IMEXDS_ERR_INVALID_ARG;
  if (!finite_pos(mat->a2_vap) || !finite_pos(mat->a2_liq) || !finite_pos(mat->p_sat) ||
      !finite_pos(mat->rho_liq_sat) || !finite_pos(mat->tau) || !std::isfinite(p_min) ||
      !std::isfinite(p_tilde))
    return IMEXDS_ERR_INVALID_ARG;
  if (n == 0) return IMEXDS_OK;
  if (!phase || !rho_l || !mom_l || !rho_r || !mom_r || !status || !out)
    return IMEXDS_ERR_INVALID_ARG;
  // the same derived constants as the time-stepping context
  Mat M{};
  M.a2v = mat->a2_vap;
  M.a2l = mat->a2_liq;
  M.p0 = mat->p_sat;
  M.rhol0 = mat->rho_liq_sat;
  M.tau = mat->tau;
  M.av = std::sqrt(mat->a2_vap);
  M.al = std::sqrt(mat->a2_liq);
  M.rhov0 = mat->p_sat / mat->a2_vap;
  M.ia2v = 1.0 / M.a2v;
  M.ia2l = 1.0 / M.a2l;
  M.iav = 1.0 / M.av;
  M.ial = 1.0 / M.al;
  M.irv0 = 1.0 / M.rhov0;
  M.irl0 = 1.0 / M.rhol0;
  // scratch: four queue counters and two queues of n problem indices,
  // stream-ordered, released after the solve pass
  hipStream_t s = (hipStream_t)hip_stream;
  int* scratch = nullptr;
  const size_t bytes = sizeof(int) * (2 * (size_t)n + 4);
  if (hipMallocAsync((void**)&scratch, bytes, s) != hipSuccess) return IMEXDS_ERR_OOM;
  int* ctr = scratch;
  int* qa = scratch + 4;
  int* q = qa + n;
  const int blocks = (int)(((long long)n + 255) / 256);
  const int qblocks = (int)(((long long)n + CR_BLOCK - 1) / CR_BLOCK);
  k_cr_init<<<1, 64, 0, s>>>(ctr);
  k_cr_partition<<<qblocks, CR_BLOCK, 0, s>>>(n, phase, ctr, qa);
  k_cr_detect<<<qblocks, CR_BLOCK, 0, s>>>(M, n, phase, rho_l, mom_l, rho_r, mom_r, p_min,
                                           p_tilde, status, out, ctr, qa, q);
  k_cr_solve<<<blocks, 256, 0, s>>>(M, n, phase, rho_l, mom_l, rho_r, mom_r, maxit, rtol, status,
                                    out, ctr, q);
  const hipError_t le = hipGetLastError();
  const hipError_t fe = hipFreeAsync(scratch, s);
  if (le != hipSuccess || fe != hipSuccess) return IMEXDS_ERR_HIP;
  return IMEXDS_OK;
}
