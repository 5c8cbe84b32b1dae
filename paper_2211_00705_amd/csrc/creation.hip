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
#include <mutex>

#include "../../include/imexds_creation.h"
#include "creation_device.hpp"

// Fixed scratch of imexds_creation_rp_noalloc: the four queue counters and
// both queues for up to IMEXDS_CR_NOALLOC_MAX problems (8 MiB + 16 B).  Every
// device the library runs on holds one copy for the life of the process.
// Host code never passes this name to a kernel (on the host it only stands
// for the symbol): it uses the device address that hipGetSymbolAddress
// returns, looked up once per device.
static __device__ __align__(256) int scratch[4 + 2 * IMEXDS_CR_NOALLOC_MAX];

namespace imexds {
namespace {

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

// Material constants as the time-stepping context derives them; false if the
// arguments are invalid.
bool cr_prepare(const imexds_material* mat, int32_t n, int32_t maxit, double rtol, double p_min,
                double p_tilde, Mat& M) {
  if (!mat || n < 0 || maxit < 1 || !finite_pos(rtol)) return false;
  if (!finite_pos(mat->a2_vap) || !finite_pos(mat->a2_liq) || !finite_pos(mat->p_sat) ||
      !finite_pos(mat->rho_liq_sat) || !finite_pos(mat->tau) || !std::isfinite(p_min) ||
      !std::isfinite(p_tilde))
    return false;
  M = Mat{};
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
  return true;
}

// The three passes on stream s over n > 0 problems, with buf = four queue
// counters followed by two queues of n problem indices (device memory of
// 4 (2 n + 4) bytes).  The counters are cleared by a kernel (k_cr_init), not
// by a memset, so the sequence may be captured in a graph.
void cr_launch(const Mat& M, int32_t n, const int32_t* phase, const double* rho_l,
               const double* mom_l, const double* rho_r, const double* mom_r, double p_min,
               double p_tilde, int32_t maxit, double rtol, int32_t* status, double* out,
               int* buf, hipStream_t s) {
  int* ctr = buf;
  int* qa = buf + 4;
  int* q = qa + n;
  const int blocks = (int)(((long long)n + 255) / 256);
  const int qblocks = (int)(((long long)n + CR_BLOCK - 1) / CR_BLOCK);
  k_cr_init<<<1, 64, 0, s>>>(ctr);
  k_cr_partition<<<qblocks, CR_BLOCK, 0, s>>>(n, phase, ctr, qa);
  k_cr_detect<<<qblocks, CR_BLOCK, 0, s>>>(M, n, phase, rho_l, mom_l, rho_r, mom_r, p_min,
                                           p_tilde, status, out, ctr, qa, q);
  k_cr_solve<<<blocks, 256, 0, s>>>(M, n, phase, rho_l, mom_l, rho_r, mom_r, maxit, rtol, status,
                                    out, ctr, q);
}

constexpr int CR_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
int* g_scratch_ptr[CR_MAX_DEVICES] = {};

// Device address of this device's scratch (looked up once per device, with
// that device current); nullptr on failure.
int* cr_scratch_ptr(int dev) {
  if (dev < 0 || dev >= CR_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = (int*)ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace imexds

extern "C" int imexds_creation_rp(const imexds_material* mat, int32_t n, const int32_t* phase,
                                  const double* rho_l, const double* mom_l, const double* rho_r,
                                  const double* mom_r, double p_min, double p_tilde, int32_t maxit,
                                  double rtol, int32_t* status, double* out, void* hip_stream) {
  using namespace imexds;
  Mat M;
  if (!cr_prepare(mat, n, maxit, rtol, p_min, p_tilde, M)) return IMEXDS_ERR_INVALID_ARG;
  if (n == 0) return IMEXDS_OK;
  if (!phase || !rho_l || !mom_l || !rho_r || !mom_r || !status || !out)
    return IMEXDS_ERR_INVALID_ARG;
  // scratch: four queue counters and two queues of n problem indices,
  // stream-ordered, released after the solve pass
  hipStream_t s = (hipStream_t)hip_stream;
  int* buf = nullptr;
  const size_t bytes = sizeof(int) * (2 * (size_t)n + 4);
  if (hipMallocAsync((void**)&buf, bytes, s) != hipSuccess) return IMEXDS_ERR_OOM;
  cr_launch(M, n, phase, rho_l, mom_l, rho_r, mom_r, p_min, p_tilde, maxit, rtol, status, out,
            buf, s);
  const hipError_t le = hipGetLastError();
  const hipError_t fe = hipFreeAsync(buf, s);
  if (le != hipSuccess || fe != hipSuccess) return IMEXDS_ERR_HIP;
  return IMEXDS_OK;
}

extern "C" int imexds_creation_rp_noalloc(const imexds_material* mat, int32_t n,
                                          const int32_t* phase, const double* rho_l,
                                          const double* mom_l, const double* rho_r,
                                          const double* mom_r, double p_min, double p_tilde,
                                          int32_t maxit, double rtol, int32_t* status,
                                          double* out, void* hip_stream) {
  using namespace imexds;
  Mat M;
  if (!cr_prepare(mat, n, maxit, rtol, p_min, p_tilde, M)) return IMEXDS_ERR_INVALID_ARG;
  if (n > IMEXDS_CR_NOALLOC_MAX) return IMEXDS_ERR_TOO_LARGE;
  if (n == 0) return IMEXDS_OK;
  if (!phase || !rho_l || !mom_l || !rho_r || !mom_r || !status || !out)
    return IMEXDS_ERR_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return IMEXDS_ERR_HIP;
  int* scratch_dev = cr_scratch_ptr(dev);
  if (!scratch_dev) return IMEXDS_ERR_HIP;
  cr_launch(M, n, phase, rho_l, mom_l, rho_r, mom_r, p_min, p_tilde, maxit, rtol, status, out,
            scratch_dev, (hipStream_t)hip_stream);
  if (hipGetLastError() != hipSuccess) return IMEXDS_ERR_HIP;
  return IMEXDS_OK;
}
