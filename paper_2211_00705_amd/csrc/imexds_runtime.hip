// imexds_runtime.hip -- host runtime behind the C ABI of include/imexds.h.
//
// The context owns every device buffer: ping-pong state arrays (rho, rho u)
// in structure-of-arrays FP64 layout over the flat slot index of all problems,
// ping-pong interface records, per-problem scalars (t, dt, status, CFL
// accumulator) and the tile table of the bulk sweep.  Work goes to two
// streams owned by the context, both at the default priority: the bulk sweep
// and the per-problem bookkeeping on the main one, the implicit zones on the
// second, joined by events each step.  Repeated steps are captured once into
// a HIP graph (an even number of steps, so the ping-pong parity returns) and
// replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/imexds.h"
#include "imexds_kernels.hpp"

using imexds::StepArgs;

namespace {

// device counters of the zone kernels (imexds_stats): dual time iterations,
// merges, lmax hits, evaluations of G, interface solves, mesh events, zone
// steps with two phase boundaries
constexpr int N_STATS = 7;

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
};

struct Snapshot {
  double *rho = nullptr, *mom = nullptr;
  int *home = nullptr, *warm = nullptr, *status = nullptr, *clipped = nullptr;
  double *hl = nullptr, *pw = nullptr, *dt = nullptr, *t = nullptr;
  long long* steps = nullptr;
  unsigned long long* stats = nullptr;
  int parity = 0;
};

}  // namespace

// The recorded steps of one checkpoint segment.
struct Tape {
  double* U = nullptr;          // [C][2][S] rho^n, (rho u)^n
  int* home = nullptr;          // [C][NIF]
  double* hl = nullptr;         // [C][NIF]
  double* dt = nullptr;         // [C][P]
  int* clip = nullptr;          // [C][P]
  long long* steps = nullptr;   // [C+1][P]
  double* zone = nullptr;       // [C][NIF][stride]
  int seg = -1;                 // checkpoint segment recorded in it (-1: none)
};

struct imexds_ctx {
  int device = 0;
  hipStream_t user = nullptr;  // the caller's stream
  hipStream_t ms = nullptr;    // main stream of the context
  hipStream_t zs = nullptr;    // zone stream of the context
  hipStream_t ps = nullptr;    // stream of the zones with two phase boundaries
  std::vector<hipEvent_t> fork_ev, join_ev, join2_ev;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
  std::vector<hipEvent_t> bulk_ev;  // pairs around bulk launches when timing
  std::vector<hipEvent_t> zone_ev;  // pairs around zone launches when timing
  // begin / end events of the stepping calls since the last statistics
  // read-out, and the device time they have accounted for so far
  std::vector<hipEvent_t> call_ev;
  int n_call_ev = 0;
  double acc_gpu_ms = 0.0;
  imexds::Mat mat{};
  imexds::Par par{};
  int P = 0, NIF = 0;
  long long S = 0;
  std::vector<long long> h_slot_off;
  std::vector<int> h_n_cells, h_phase_first, h_iface_off, h_home0, h_iface_prob, h_iface_local;
  std::vector<double> h_h, h_x_left, h_hl0;
  // static layout on the device
  long long* d_slot_off = nullptr;
  double* d_h = nullptr;
  int *d_phase_first = nullptr, *d_iface_off = nullptr, *d_iface_prob = nullptr,
      *d_iface_local = nullptr;
  int *d_tile_prob = nullptr, *d_tile_start = nullptr, *d_tile_len = nullptr;
  int n_tiles = 0, tile_cells = 1024, zones_per_group = 16, zone_groups = 0, graph_steps = 8;
  int zone_lanes = 1;  // lanes per zone: 1 (k_zone) or 8 (k_zone8)
  std::vector<int> h_tile_off;  // [P+1] tiles of each problem
  // evolving state
  double *d_rho[2] = {nullptr, nullptr}, *d_mom[2] = {nullptr, nullptr};
  int* d_home[2] = {nullptr, nullptr};
  double* d_hl[2] = {nullptr, nullptr};
  double* d_pw[2] = {nullptr, nullptr};
  int* d_warm[2] = {nullptr, nullptr};
  double *d_dt = nullptr, *d_t = nullptr;
  int *d_status = nullptr, *d_clipped = nullptr, *d_fail = nullptr;
  long long* d_steps = nullptr;
  unsigned long long* d_S = nullptr;
  unsigned long long* d_stats = nullptr;  // pseudo, merges, lmax, G evaluations, solves, events,
                                          // zone steps with two boundaries
  int* d_pair_seen = nullptr;  // a zone with two boundaries was solved (adjoint refuses)
  int max_nif = 0;             // most interfaces in one problem
  bool adj_pairs = false;      // the last checkpointed forward solved such a zone
  int* d_zone_ctr = nullptr;
  int *d_log_count = nullptr, *d_log_flags = nullptr, *d_log_zlo = nullptr, *d_log_row = nullptr;
  int log_max = 0;
  int parity = 0;
  bool has_state = false;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t ev_rev = nullptr, ev_rec = nullptr;  // the adjoint's two streams
  // reverse sweeps of a recorded segment, by the adjoint buffer they start
  // from (index bit 0), full or shorter last segment (bit 1) and tape (bit
  // 2); recorded segments, by the state parity they start at (bit 0), length
  // (bit 1) and tape (bit 2)
  hipGraphExec_t rev_gexec[8] = {};
  int rev_len[8] = {};
  hipGraphExec_t rec_gexec[8] = {};
  int rec_len[8] = {};
  bool time_bulk = false;
  int bulk_launches = 0;
  double last_total_ms = 0.0, last_bulk_ms = 0.0;
  bool timed = false;
  std::vector<void*> allocs;
  // adjoint: checkpoints of the last checkpointed forward, one segment's tape
  std::vector<Snapshot> ck;
  Snapshot ck_end;
  bool ck_end_valid = false;
  int adj_steps = 0, adj_every = 0;
  bool adj_ready = false;
  int tape_steps = 0;      // segment length the tape buffers hold
  long long tape_stride = 0;
  // Two tapes: while the reverse sweep reads one segment's tape, the
  // segment before it is recomputed into the other (tape[1] allocated by the
  // adjoint when there is more than one segment and memory allows)
  Tape tape[2];
  int n_tapes = 0;
  double *d_gr[2] = {nullptr, nullptr}, *d_gm[2] = {nullptr, nullptr};
  double *d_hlbar = nullptr, *d_taubar = nullptr, *d_zadj = nullptr, *d_tbar = nullptr;
  double* d_tgdt = nullptr;
  unsigned long long* d_tsmax = nullptr;
  int* d_tsidx = nullptr;
  int adj_tiles = 0;
  int* d_tile_off = nullptr;
};

namespace {

thread_local char g_err[512];

int hip_fail(hipError_t e, const char* what) {
  snprintf(g_err, sizeof(g_err), "%s: %s", what, hipGetErrorString(e));
  return IMEXDS_ERR_HIP;
}

#define CK(expr)                                  \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

template <class T>
int dalloc(imexds_ctx* c, T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    snprintf(g_err, sizeof(g_err), "hipMalloc of %zu bytes failed", n * sizeof(T));
    return IMEXDS_ERR_OOM;
  }
  c->allocs.push_back((void*)*p);
  return 0;
}

#define AL(ptr, n)                          \
  do {                                      \
    int r_ = dalloc(c, &(ptr), (size_t)(n)); \
    if (r_) return r_;                      \
  } while (0)

void drop_step_graph(imexds_ctx* c) {
  if (c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
}

void drop_adjoint_graphs(imexds_ctx* c) {
  for (int a = 0; a < 8; ++a) {
    if (c->rev_gexec[a]) (void)hipGraphExecDestroy(c->rev_gexec[a]);
    c->rev_gexec[a] = nullptr;
    c->rev_len[a] = 0;
    if (c->rec_gexec[a]) (void)hipGraphExecDestroy(c->rec_gexec[a]);
    c->rec_gexec[a] = nullptr;
    c->rec_len[a] = 0;
  }
}

// Captured graphs hold the launch arguments (material, parameters, buffers)
// by value: any change of them drops the graphs.
void drop_graph(imexds_ctx* c) {
  drop_step_graph(c);
  drop_adjoint_graphs(c);
}

StepArgs make_args(imexds_ctx* c, int parity, bool init) {
  StepArgs A;
  memset(&A, 0, sizeof(A));
  A.mat = c->mat;
  A.par = c->par;
  A.slot_off = c->d_slot_off;
  A.h = c->d_h;
  A.phase_first = c->d_phase_first;
  A.iface_off = c->d_iface_off;
  A.iface_prob = c->d_iface_prob;
  A.iface_local = c->d_iface_local;
  A.tile_prob = c->d_tile_prob;
  A.tile_start = c->d_tile_start;
  A.tile_len = c->d_tile_len;
  int a = parity, b = init ? parity : parity ^ 1;
  A.rho0 = c->d_rho[a];
  A.mom0 = c->d_mom[a];
  A.rho1 = c->d_rho[b];
  A.mom1 = c->d_mom[b];
  A.rec_home0 = c->d_home[a];
  A.rec_hl0 = c->d_hl[a];
  A.rec_pw0 = c->d_pw[a];
  A.rec_warm0 = c->d_warm[a];
  A.rec_home1 = c->d_home[b];
  A.rec_hl1 = c->d_hl[b];
  A.rec_pw1 = c->d_pw[b];
  A.rec_warm1 = c->d_warm[b];
  A.dt = c->d_dt;
  A.t = c->d_t;
  A.status = c->d_status;
  A.clipped = c->d_clipped;
  A.steps = c->d_steps;
  A.S_acc = c->d_S;
  A.fail_acc = c->d_fail;
  if (c->log_max > 0) {
    A.log_count = c->d_log_count;
    A.log_flags = c->d_log_flags;
    A.log_zlo = c->d_log_zlo;
    A.log_row = c->d_log_row;
    A.log_max = c->log_max;
  }
  A.n_iface = c->NIF;
  A.st_pseudo = c->d_stats;
  A.st_merges = c->d_stats + 1;
  A.st_lmax = c->d_stats + 2;
  A.st_newton = c->d_stats + 3;
  A.st_solves = c->d_stats + 4;
  A.st_events = c->d_stats + 5;
  A.st_pairs = c->d_stats + 6;
  A.pair_seen = c->d_pair_seen;
  A.zone_ctr = c->d_zone_ctr;
  A.zones_per_group = c->zones_per_group;
  return A;
}

int build_tiles(imexds_ctx* c, int tile_cells) {
  std::vector<int> tp, ts, tl;
  c->h_tile_off.assign(c->P + 1, 0);
  const int cells = imexds::bulk_tile_cells(tile_cells);
  for (int p = 0; p < c->P; ++p) {
    int ns = (int)(c->h_slot_off[p + 1] - c->h_slot_off[p]);
    for (int s = 0; s < ns; s += cells) {
      tp.push_back(p);
      ts.push_back(s);
      tl.push_back(std::min(cells, ns - s));
    }
    c->h_tile_off[p + 1] = (int)tp.size();
  }
  int n = (int)tp.size();
  int *np = nullptr, *nst = nullptr, *nl = nullptr;
  if (n > 0) {
    CK(hipMalloc((void**)&np, sizeof(int) * n));
    CK(hipMalloc((void**)&nst, sizeof(int) * n));
    CK(hipMalloc((void**)&nl, sizeof(int) * n));
    CK(hipMemcpy(np, tp.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    CK(hipMemcpy(nst, ts.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    CK(hipMemcpy(nl, tl.data(), sizeof(int) * n, hipMemcpyHostToDevice));
  }
  int* toff = nullptr;
  CK(hipMalloc((void**)&toff, sizeof(int) * (c->P + 1)));
  CK(hipMemcpy(toff, c->h_tile_off.data(), sizeof(int) * (c->P + 1), hipMemcpyHostToDevice));
  if (c->d_tile_prob) {
    (void)hipFree(c->d_tile_prob);
    (void)hipFree(c->d_tile_start);
    (void)hipFree(c->d_tile_len);
  }
  if (c->d_tile_off) (void)hipFree(c->d_tile_off);
  c->d_tile_off = toff;
  c->d_tile_prob = np;
  c->d_tile_start = nst;
  c->d_tile_len = nl;
  c->n_tiles = n;
  c->tile_cells = tile_cells;
  return 0;
}

// zones with two phase boundaries can occur (Algorithm 2, a problem with
// more than one interface)
bool pairs_possible(const imexds_ctx* c) {
  return c->par.zone_solver == IMEXDS_ZONE_DTS && c->max_nif >= 2;
}

// The zone kernels of interfaces [k0, k1) on stream s; with pairs, also the
// zones holding two phase boundaries (after the others, same stream).
hipError_t launch_zones(imexds_ctx* c, const StepArgs& A, int k0, int k1, int groups,
                        hipStream_t s, bool pairs = true) {
  if (c->par.zone_solver == IMEXDS_ZONE_NEWTON)
    return imexds::launch_zone_newton(A, k0, k1, c->zone_lanes, s);
  const hipError_t e = c->zone_lanes == 8 ? imexds::launch_zone8(A, k0, k1, groups, s)
                                          : imexds::launch_zone(A, k0, k1, groups, s);
  if (e != hipSuccess || !pairs || !pairs_possible(c)) return e;
  return imexds::launch_zone_pair(A, k0, k1, s);
}

// One physical step of every problem, enqueued on c->ms (zones on c->zs).
int enqueue_step(imexds_ctx* c, int ev_slot) {
  StepArgs A = make_args(c, c->parity, false);
  hipEvent_t ef = c->fork_ev[ev_slot], ej = c->join_ev[ev_slot];
  if (c->time_bulk) {
    // timing mode: the bulk sweep runs alone between its two events, then the
    // zones on the same stream (no overlap), so the events see the kernel only
    size_t need = 2 * (size_t)(c->bulk_launches + 1);
    while (c->bulk_ev.size() < need) {
      hipEvent_t e;
      CK(hipEventCreate(&e));
      c->bulk_ev.push_back(e);
    }
    CK(hipEventRecord(c->bulk_ev[2 * c->bulk_launches], c->ms));
    CK(imexds::launch_bulk(A, c->tile_cells, 0, c->n_tiles, c->ms));
    CK(hipEventRecord(c->bulk_ev[2 * c->bulk_launches + 1], c->ms));
    while (c->zone_ev.size() < need) {
      hipEvent_t e;
      CK(hipEventCreate(&e));
      c->zone_ev.push_back(e);
    }
    CK(hipEventRecord(c->zone_ev[2 * c->bulk_launches], c->ms));
    if (c->NIF > 0) CK(launch_zones(c, A, 0, c->NIF, c->zone_groups, c->ms));
    CK(hipEventRecord(c->zone_ev[2 * c->bulk_launches + 1], c->ms));
    c->bulk_launches++;
    CK(imexds::launch_finalize(A, 0, c->P, 0, 1, c->ms));
    c->parity ^= 1;
    return 0;
  }
  // zones with one boundary on zs, those with two on ps, beside the bulk
  const bool pairs = c->NIF > 0 && pairs_possible(c);
  if (c->NIF > 0) {
    CK(hipEventRecord(ef, c->ms));
    CK(hipStreamWaitEvent(c->zs, ef, 0));
    CK(launch_zones(c, A, 0, c->NIF, c->zone_groups, c->zs, false));
    if (pairs) {
      CK(hipStreamWaitEvent(c->ps, ef, 0));
      CK(imexds::launch_zone_pair(A, 0, c->NIF, c->ps));
    }
  }
  CK(imexds::launch_bulk(A, c->tile_cells, 0, c->n_tiles, c->ms));
  if (c->NIF > 0) {
    CK(hipEventRecord(ej, c->zs));
    CK(hipStreamWaitEvent(c->ms, ej, 0));
    if (pairs) {
      CK(hipEventRecord(c->join2_ev[ev_slot], c->ps));
      CK(hipStreamWaitEvent(c->ms, c->join2_ev[ev_slot], 0));
    }
  }
  CK(imexds::launch_finalize(A, 0, c->P, 0, 1, c->ms));
  c->parity ^= 1;
  return 0;
}

int ensure_events(imexds_ctx* c, size_t n) {
  while (c->fork_ev.size() < n) {
    hipEvent_t a, b, d;
    CK(hipEventCreateWithFlags(&a, hipEventDisableTiming));
    CK(hipEventCreateWithFlags(&b, hipEventDisableTiming));
    CK(hipEventCreateWithFlags(&d, hipEventDisableTiming));
    c->fork_ev.push_back(a);
    c->join_ev.push_back(b);
    c->join2_ev.push_back(d);
  }
  return 0;
}

int capture_graph(imexds_ctx* c) {
  drop_step_graph(c);
  int G = c->graph_steps;
  int r = ensure_events(c, (size_t)G);
  if (r) return r;
  int par0 = c->parity;
  CK(hipStreamBeginCapture(c->ms, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < G; ++i) {
    r = enqueue_step(c, i);
    if (r) {
      hipGraph_t g;
      (void)hipStreamEndCapture(c->ms, &g);
      if (g) (void)hipGraphDestroy(g);
      c->parity = par0;
      return r;
    }
  }
  hipGraph_t g = nullptr;
  CK(hipStreamEndCapture(c->ms, &g));
  c->parity = par0;  // capturing does not run anything
  hipError_t e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->gexec = nullptr;
    return hip_fail(e, "hipGraphInstantiate");
  }
  return 0;
}

int begin_call(imexds_ctx* c) {
  CK(hipSetDevice(c->device));
  CK(hipEventRecord(c->ev_in, c->user));
  CK(hipStreamWaitEvent(c->ms, c->ev_in, 0));
  return 0;
}

int end_call(imexds_ctx* c) {
  CK(hipEventRecord(c->ev_out, c->ms));
  CK(hipStreamWaitEvent(c->user, c->ev_out, 0));
  return 0;
}

// Device time of the stepping calls: each call records a pair of events;
// completed pairs are folded into acc_gpu_ms (all of them, waiting, when
// `wait`; else those already done, and the oldest ones once many are
// pending, so that the event list stays bounded).
int fold_call_events(imexds_ctx* c, bool wait) {
  int done = 0;
  for (; done < c->n_call_ev; ++done) {
    hipEvent_t e0 = c->call_ev[2 * done], e1 = c->call_ev[2 * done + 1];
    if (wait || c->n_call_ev - done > 256) {
      CK(hipEventSynchronize(e1));
    } else {
      hipError_t q = hipEventQuery(e1);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
    }
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, e0, e1));
    c->acc_gpu_ms += ms;
  }
  if (done > 0) {  // keep the pending pairs at the front, recycle the folded ones
    std::rotate(c->call_ev.begin(), c->call_ev.begin() + 2 * done,
                c->call_ev.begin() + 2 * c->n_call_ev);
    c->n_call_ev -= done;
  }
  return 0;
}

int call_begin(imexds_ctx* c) {
  int r = fold_call_events(c, false);
  if (r) return r;
  while (c->call_ev.size() < 2 * (size_t)(c->n_call_ev + 1)) {
    hipEvent_t e;
    CK(hipEventCreate(&e));
    c->call_ev.push_back(e);
  }
  CK(hipEventRecord(c->call_ev[2 * c->n_call_ev], c->ms));
  return 0;
}

int call_end(imexds_ctx* c) {
  CK(hipEventRecord(c->call_ev[2 * c->n_call_ev + 1], c->ms));
  c->n_call_ev++;
  return 0;
}

int init_dt(imexds_ctx* c) {
  StepArgs A = make_args(c, c->parity, true);
  CK(imexds::launch_cfl(A, 0, c->n_tiles, c->ms));
  CK(imexds::launch_finalize(A, 0, c->P, 1, 0, c->ms));
  return 0;
}

int snap_take(imexds_ctx* c, Snapshot& s) {
  size_t S = (size_t)std::max<long long>(c->S, 1), N = (size_t)std::max(c->NIF, 1),
         P = (size_t)std::max(c->P, 1);
  CK(hipMalloc((void**)&s.rho, S * 8));
  CK(hipMalloc((void**)&s.mom, S * 8));
  CK(hipMalloc((void**)&s.home, N * 4));
  CK(hipMalloc((void**)&s.warm, N * 4));
  CK(hipMalloc((void**)&s.hl, N * 8));
  CK(hipMalloc((void**)&s.pw, 2 * N * 8));
  CK(hipMalloc((void**)&s.dt, P * 8));
  CK(hipMalloc((void**)&s.t, P * 8));
  CK(hipMalloc((void**)&s.status, P * 4));
  CK(hipMalloc((void**)&s.clipped, P * 4));
  CK(hipMalloc((void**)&s.steps, P * 8));
  CK(hipMalloc((void**)&s.stats, N_STATS * 8));
  int a = c->parity;
  s.parity = a;
  hipStream_t m = c->ms;
  CK(hipMemcpyAsync(s.rho, c->d_rho[a], S * 8, hipMemcpyDeviceToDevice, m));
  CK(hipMemcpyAsync(s.mom, c->d_mom[a], S * 8, hipMemcpyDeviceToDevice, m));
  if (c->NIF > 0) {
    CK(hipMemcpyAsync(s.home, c->d_home[a], N * 4, hipMemcpyDeviceToDevice, m));
    CK(hipMemcpyAsync(s.warm, c->d_warm[a], N * 4, hipMemcpyDeviceToDevice, m));
    CK(hipMemcpyAsync(s.hl, c->d_hl[a], N * 8, hipMemcpyDeviceToDevice, m));
    CK(hipMemcpyAsync(s.pw, c->d_pw[a], 2 * N * 8, hipMemcpyDeviceToDevice, m));
  }
  CK(hipMemcpyAsync(s.dt, c->d_dt, P * 8, hipMemcpyDeviceToDevice, m));
  CK(hipMemcpyAsync(s.t, c->d_t, P * 8, hipMemcpyDeviceToDevice, m));
  CK(hipMemcpyAsync(s.status, c->d_status, P * 4, hipMemcpyDeviceToDevice, m));
  CK(hipMemcpyAsync(s.clipped, c->d_clipped, P * 4, hipMemcpyDeviceToDevice, m));
  CK(hipMemcpyAsync(s.steps, c->d_steps, P * 8, hipMemcpyDeviceToDevice, m));
  CK(hipMemcpyAsync(s.stats, c->d_stats, N_STATS * 8, hipMemcpyDeviceToDevice, m));
  return 0;
}

// Copies the snapshot back into the live state on stream m (the main stream
// by default) and, with `sync`, waits for it.
int snap_restore(imexds_ctx* c, Snapshot& s, hipStream_t m = nullptr, bool sync = true) {
  size_t S = (size_t)std::max<long long>(c->S, 1), N = (size_t)std::max(c->NIF, 1),
         P = (size_t)std::max(c->P, 1);
  int a = s.parity;
  c->parity = a;
  if (!m) m = c->ms;
  CK(hipMemcpyAsync(c->d_rho[a], s.rho, S * 8, hipMemcpyDeviceToDevice, m));
  CK(hipMemcpyAsync(c->d_mom[a], s.mom, S * 8, hipMemcpyDeviceToDevice, m));
  if (c->NIF > 0) {
    CK(hipMemcpyAsync(c->d_home[a], s.home, N * 4, hipMemcpyDeviceToDevice, m));
    CK(hipMemcpyAsync(c->d_warm[a], s.warm, N * 4, hipMemcpyDeviceToDevice, m));
    CK(hipMemcpyAsync(c->d_hl[a], s.hl, N * 8, hipMemcpyDeviceToDevice, m));
    CK(hipMemcpyAsync(c->d_pw[a], s.pw, 2 * N * 8, hipMemcpyDeviceToDevice, m));
  }
  CK(hipMemcpyAsync(c->d_dt, s.dt, P * 8, hipMemcpyDeviceToDevice, m));
  CK(hipMemcpyAsync(c->d_t, s.t, P * 8, hipMemcpyDeviceToDevice, m));
  CK(hipMemcpyAsync(c->d_status, s.status, P * 4, hipMemcpyDeviceToDevice, m));
  CK(hipMemcpyAsync(c->d_clipped, s.clipped, P * 4, hipMemcpyDeviceToDevice, m));
  CK(hipMemcpyAsync(c->d_steps, s.steps, P * 8, hipMemcpyDeviceToDevice, m));
  CK(hipMemcpyAsync(c->d_stats, s.stats, N_STATS * 8, hipMemcpyDeviceToDevice, m));
  if (sync) CK(hipStreamSynchronize(m));
  return 0;
}

void snap_free(Snapshot& s) {
  void* ps[] = {s.rho, s.mom, s.home, s.warm, s.status, s.clipped, s.hl,
                s.pw,  s.dt,  s.t,    s.steps, s.stats};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  s = Snapshot();
}

int steps_impl(imexds_ctx* c, int n) {
  int r;
  if (c->time_bulk || c->graph_steps <= 0) {
    r = ensure_events(c, 1);
    if (r) return r;
    for (int i = 0; i < n; ++i)
      if ((r = enqueue_step(c, 0))) return r;
    return 0;
  }
  int done = 0;
  r = ensure_events(c, 1);
  if (r) return r;
  if (c->parity != 0 && n > 0) {  // graphs start at parity 0
    if ((r = enqueue_step(c, 0))) return r;
    ++done;
  }
  int G = c->graph_steps;
  if (n - done >= G) {
    if (!c->gexec && (r = capture_graph(c))) return r;
    while (n - done >= G) {
      CK(hipGraphLaunch(c->gexec, c->ms));
      done += G;
    }
  }
  while (done < n) {
    if ((r = enqueue_step(c, 0))) return r;
    ++done;
  }
  return 0;
}

void free_one_tape(Tape& T) {
  void* ps[] = {T.U, T.home, T.hl, T.dt, T.clip, T.steps, T.zone};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  T = Tape();
}

void free_tape(imexds_ctx* c) {
  drop_adjoint_graphs(c);
  free_one_tape(c->tape[0]);
  free_one_tape(c->tape[1]);
  c->n_tapes = 0;
  c->tape_steps = 0;
}

void free_checkpoints(imexds_ctx* c) {
  c->tape[0].seg = c->tape[1].seg = -1;
  for (Snapshot& s : c->ck) snap_free(s);
  c->ck.clear();
  if (c->ck_end_valid) snap_free(c->ck_end);
  c->ck_end_valid = false;
  c->adj_ready = false;
}

void free_adjoint(imexds_ctx* c) {
  free_checkpoints(c);
  free_tape(c);
  void* ps[] = {c->d_gr[0], c->d_gr[1], c->d_gm[0], c->d_gm[1], c->d_hlbar, c->d_taubar,
                c->d_zadj, c->d_tbar, c->d_tgdt, c->d_tsmax, c->d_tsidx};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  c->d_gr[0] = c->d_gr[1] = c->d_gm[0] = c->d_gm[1] = nullptr;
  c->d_hlbar = c->d_taubar = c->d_zadj = c->d_tbar = c->d_tgdt = nullptr;
  c->d_tsmax = nullptr;
  c->d_tsidx = nullptr;
  c->adj_tiles = 0;
}

template <class T>
int halloc(T** p, size_t n) {
  *p = nullptr;
  if (hipMalloc((void**)p, (n ? n : 1) * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    snprintf(g_err, sizeof(g_err), "hipMalloc of %zu bytes failed (adjoint buffers)",
             (n ? n : 1) * sizeof(T));
    return IMEXDS_ERR_OOM;
  }
  return 0;
}

#define HA(ptr, n)                          \
  do {                                      \
    int r_ = halloc(&(ptr), (size_t)(n));   \
    if (r_) return r_;                      \
  } while (0)

int alloc_tape(imexds_ctx* c, Tape& T) {
  const size_t S = (size_t)c->S, N = (size_t)c->NIF, P = (size_t)c->P;
  const size_t C = (size_t)c->tape_steps;
  HA(T.U, C * 2 * S);
  HA(T.home, C * N);
  HA(T.hl, C * N);
  HA(T.dt, C * P);
  HA(T.clip, C * P);
  HA(T.steps, (C + 1) * P);
  HA(T.zone, C * N * (size_t)c->tape_stride);
  T.seg = -1;
  return 0;
}

// The second tape, for recomputing a segment while the one after it is
// reversed; false (and one tape) when it does not fit in device memory.
bool ensure_second_tape(imexds_ctx* c) {
  if (c->n_tapes >= 2) return true;
  if (alloc_tape(c, c->tape[1])) {
    free_one_tape(c->tape[1]);
    (void)hipGetLastError();
    return false;
  }
  c->n_tapes = 2;
  return true;
}

// Tape of one segment of C steps and the adjoint work arrays.
int ensure_adjoint_buffers(imexds_ctx* c, int C) {
  const size_t S = (size_t)c->S, N = (size_t)c->NIF, P = (size_t)c->P;
  const long long stride = imexds::tape_stride(c->par.zone_half, c->par.lmax);
  if (c->tape_steps != C || c->tape_stride != stride) {
    free_tape(c);
    c->tape_steps = C;
    c->tape_stride = stride;
    int r = alloc_tape(c, c->tape[0]);
    if (r) {
      free_tape(c);
      return r;
    }
    c->n_tapes = 1;
  }
  if (!c->d_gr[0]) {
    for (int a = 0; a < 2; ++a) {
      HA(c->d_gr[a], S);
      HA(c->d_gm[a], S);
    }
    HA(c->d_hlbar, N);
    HA(c->d_taubar, N);
    HA(c->d_zadj, 5 * N);
    HA(c->d_tbar, P);
  }
  if (c->adj_tiles != c->n_tiles) {
    drop_adjoint_graphs(c);
    if (c->d_tgdt) (void)hipFree(c->d_tgdt);
    if (c->d_tsmax) (void)hipFree(c->d_tsmax);
    if (c->d_tsidx) (void)hipFree(c->d_tsidx);
    c->d_tgdt = nullptr;
    c->d_tsmax = nullptr;
    c->d_tsidx = nullptr;
    c->adj_tiles = 0;
    HA(c->d_tgdt, (size_t)c->n_tiles);
    HA(c->d_tsmax, (size_t)c->n_tiles);
    HA(c->d_tsidx, (size_t)c->n_tiles);
    c->adj_tiles = c->n_tiles;
  }
  return 0;
}

// Enqueues `len` steps from the restored checkpoint, keeping for each step
// its input state, records, dt and the zone tape.  Step j reads its state
// from tape slot j and writes the next one straight into slot j + 1 (the
// last step into the live state buffer, which the segment's caller reads);
// the zones run on zs beside the bulk sweep, as in a plain step.
int enqueue_record(imexds_ctx* c, Tape& T, int len, hipStream_t m) {
  const size_t S = (size_t)c->S, N = (size_t)c->NIF, P = (size_t)c->P;
  if (S && len > 0) {
    CK(hipMemcpyAsync(T.U, c->d_rho[c->parity], S * 8, hipMemcpyDeviceToDevice, m));
    CK(hipMemcpyAsync(T.U + S, c->d_mom[c->parity], S * 8, hipMemcpyDeviceToDevice, m));
  }
  for (int j = 0; j < len; ++j) {
    const int a = c->parity;
    CK(imexds::launch_tape_copy(c->d_home[a], c->d_hl[a], c->d_dt, c->d_clipped, c->d_steps,
                                T.home + j * N, T.hl + j * N, T.dt + j * P, T.clip + j * P,
                                T.steps + j * P, (int)N, (int)P, m));
    StepArgs A = make_args(c, a, false);
    A.rho0 = T.U + (size_t)j * 2 * S;
    A.mom0 = A.rho0 + S;
    if (j + 1 < len) {
      A.rho1 = T.U + (size_t)(j + 1) * 2 * S;
      A.mom1 = A.rho1 + S;
    }
    A.log_count = A.log_flags = A.log_zlo = A.log_row = nullptr;
    A.log_max = 0;
    A.st_pseudo = A.st_merges = A.st_lmax = nullptr;
    A.st_newton = A.st_solves = A.st_events = A.st_pairs = nullptr;
    A.tape = T.zone + (size_t)j * N * (size_t)c->tape_stride;
    A.tape_stride = c->tape_stride;
    if (N) {
      CK(hipEventRecord(c->fork_ev[j], m));
      CK(hipStreamWaitEvent(c->zs, c->fork_ev[j], 0));
      CK(launch_zones(c, A, 0, c->NIF, c->zone_groups, c->zs));
    }
    CK(imexds::launch_bulk(A, c->tile_cells, 0, c->n_tiles, m));
    if (N) {
      CK(hipEventRecord(c->join_ev[j], c->zs));
      CK(hipStreamWaitEvent(m, c->join_ev[j], 0));
    }
    CK(imexds::launch_finalize(A, 0, c->P, 0, 0, m));
    c->parity ^= 1;
  }
  CK(hipMemcpyAsync(T.steps + (size_t)len * P, c->d_steps, P * 8, hipMemcpyDeviceToDevice, m));
  return 0;
}

// Records a segment of `len` steps, captured into a graph (kept per start
// parity and segment kind for the next segment of the same shape: the
// reverse sweep records every checkpointed segment again) and replayed.
// Launched one by one, the cross-stream waits of the zone/bulk overlap
// would cost more than the overlap saves.
int record_segment(imexds_ctx* c, int t, int len, hipStream_t m) {
  if (len < 0 || len > c->tape_steps || t < 0 || t >= c->n_tapes) return IMEXDS_ERR_INVALID_ARG;
  Tape& T = c->tape[t];
  if (len == 0 || c->P <= 0) return enqueue_record(c, T, len, m);
  const int p0 = c->parity;
  const int slot = p0 + (len != c->tape_steps ? 2 : 0) + 4 * t;
  if (!c->rec_gexec[slot] || c->rec_len[slot] != len) {
    if (c->rec_gexec[slot]) (void)hipGraphExecDestroy(c->rec_gexec[slot]);
    c->rec_gexec[slot] = nullptr;
    c->rec_len[slot] = 0;
    int r = ensure_events(c, (size_t)len);
    if (r) return r;
    CK(hipStreamBeginCapture(m, hipStreamCaptureModeThreadLocal));
    r = enqueue_record(c, T, len, m);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(m, &g);
    c->parity = p0;
    if (r || ee != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return r ? r : hip_fail(ee, "hipStreamEndCapture");
    }
    const hipError_t e = hipGraphInstantiate(&c->rec_gexec[slot], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->rec_gexec[slot] = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
    c->rec_len[slot] = len;
  }
  CK(hipGraphLaunch(c->rec_gexec[slot], m));
  c->parity = p0 ^ (len & 1);
  return 0;
}

// Reverse of step j of the recorded segment: adjoint buffers cur -> cur ^ 1.
// The bulk pass leaves the faces next to zone cells to the per-problem pass,
// so it does not wait for the zone pass, which runs on zs beside it (the
// steps are captured into a graph: launched one by one, the cross-stream
// waits would cost more than the overlap saves).
int reverse_step(imexds_ctx* c, const Tape& T, int j, int cur) {
  const size_t S = (size_t)c->S, N = (size_t)c->NIF, P = (size_t)c->P;
  StepArgs A = make_args(c, 0, false);
  A.rho0 = T.U + (size_t)j * 2 * S;
  A.mom0 = A.rho0 + S;
  A.rec_home0 = T.home + (size_t)j * N;
  A.rec_hl0 = T.hl + (size_t)j * N;
  A.dt = T.dt + (size_t)j * P;
  A.clipped = T.clip + (size_t)j * P;
  A.tape = T.zone + (size_t)j * N * (size_t)c->tape_stride;
  A.tape_stride = c->tape_stride;
  imexds::AdjArgs B;
  B.gr1 = c->d_gr[cur];
  B.gm1 = c->d_gm[cur];
  B.gr0 = c->d_gr[cur ^ 1];
  B.gm0 = c->d_gm[cur ^ 1];
  B.hl_bar = c->d_hlbar;
  B.tau_bar = c->d_taubar;
  B.zadj = c->d_zadj;
  B.tile_gdt = c->d_tgdt;
  B.tile_smax = c->d_tsmax;
  B.tile_sidx = c->d_tsidx;
  B.tile_off = c->d_tile_off;
  B.steps0 = T.steps + (size_t)j * P;
  B.steps1 = T.steps + (size_t)(j + 1) * P;
  B.t_bar = c->d_tbar;
  if (N) {
    CK(hipEventRecord(c->fork_ev[j], c->ms));
    CK(hipStreamWaitEvent(c->zs, c->fork_ev[j], 0));
    CK(imexds::launch_zone_adj(A, B, c->zone_lanes, c->zs));
  }
  CK(imexds::launch_bulk_adj(A, B, c->tile_cells, c->n_tiles, c->ms));
  if (N) {
    CK(hipEventRecord(c->join_ev[j], c->zs));
    CK(hipStreamWaitEvent(c->ms, c->join_ev[j], 0));
  }
  CK(imexds::launch_finalize_adj(A, B, c->P, c->ms));
  return 0;
}

// Reverse sweep of the recorded segment (steps len - 1 .. 0) from adjoint
// buffer cur, captured into a graph and replayed.  The graph is kept per
// start buffer and segment kind (`last`: the shorter last segment) for the
// next sweep of the same length: every full checkpointed segment is one.
int reverse_segment(imexds_ctx* c, int t, int len, int cur, bool last) {
  if (len <= 0 || c->P <= 0) return 0;
  const Tape& T = c->tape[t];
  const int slot = cur + (last ? 2 : 0) + 4 * t;
  if (!c->rev_gexec[slot] || c->rev_len[slot] != len) {
    if (c->rev_gexec[slot]) (void)hipGraphExecDestroy(c->rev_gexec[slot]);
    c->rev_gexec[slot] = nullptr;
    c->rev_len[slot] = 0;
    int r = ensure_events(c, (size_t)len);
    if (r) return r;
    CK(hipStreamBeginCapture(c->ms, hipStreamCaptureModeThreadLocal));
    int b = cur;
    for (int j = len - 1; j >= 0 && !r; --j) {
      r = reverse_step(c, T, j, b);
      b ^= 1;
    }
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(c->ms, &g);
    if (r || ee != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return r ? r : hip_fail(ee, "hipStreamEndCapture");
    }
    const hipError_t e = hipGraphInstantiate(&c->rev_gexec[slot], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->rev_gexec[slot] = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
    c->rev_len[slot] = len;
  }
  CK(hipGraphLaunch(c->rev_gexec[slot], c->ms));
  return 0;
}

}  // namespace

extern "C" {

const char* imexds_strerror(int code) {
  switch (code) {
    case IMEXDS_OK: return "ok";
    case IMEXDS_ERR_INVALID_ARG: return "invalid argument";
    case IMEXDS_ERR_OOM: return "out of device memory";
    case IMEXDS_ERR_HIP: return g_err[0] ? g_err : "HIP runtime error";
    case IMEXDS_ERR_NO_STATE: return "no state loaded (call imexds_set_state first)";
    case IMEXDS_ERR_UNSUPPORTED: return "unsupported configuration";
    case IMEXDS_ERR_TOO_LARGE: return "size above the entry point's fixed maximum";
    default: return "unknown error";
  }
}

void imexds_destroy(imexds_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->ms) (void)hipStreamSynchronize(c->ms);
  if (c->zs) (void)hipStreamSynchronize(c->zs);
  if (c->ps) (void)hipStreamSynchronize(c->ps);
  drop_graph(c);
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->d_tile_prob) (void)hipFree(c->d_tile_prob);
  if (c->d_tile_start) (void)hipFree(c->d_tile_start);
  if (c->d_tile_len) (void)hipFree(c->d_tile_len);
  if (c->d_tile_off) (void)hipFree(c->d_tile_off);
  free_adjoint(c);
  if (c->d_log_count) (void)hipFree(c->d_log_count);
  if (c->d_log_flags) (void)hipFree(c->d_log_flags);
  if (c->d_log_zlo) (void)hipFree(c->d_log_zlo);
  for (auto e : c->fork_ev) (void)hipEventDestroy(e);
  for (auto e : c->join_ev) (void)hipEventDestroy(e);
  for (auto e : c->join2_ev) (void)hipEventDestroy(e);
  for (auto e : c->bulk_ev) (void)hipEventDestroy(e);
  for (auto e : c->zone_ev) (void)hipEventDestroy(e);
  for (auto e : c->call_ev) (void)hipEventDestroy(e);
  hipEvent_t es[] = {c->ev_in, c->ev_out, c->ev_t0, c->ev_t1, c->ev_rev, c->ev_rec};
  for (auto e : es)
    if (e) (void)hipEventDestroy(e);
  if (c->ms) (void)hipStreamDestroy(c->ms);
  if (c->zs) (void)hipStreamDestroy(c->zs);
  if (c->ps) (void)hipStreamDestroy(c->ps);
  delete c;
}

static int create_impl(imexds_ctx* c, const imexds_material* mat, const imexds_params* par,
                       const imexds_batch* b) {
  const int P = b->n_problems;
  if (P < 0) return IMEXDS_ERR_INVALID_ARG;
  if (!(par->cfl > 0.0) || par->zone_half < 1 || par->zone_half > 3 || !(par->theta_nb > 0.0) ||
      par->lmax < 1 || par->newton_maxit < 1 || !(par->newton_rtol > 0.0) ||
      (par->tol_mode != IMEXDS_TOL_PAPER && par->tol_mode != IMEXDS_TOL_REL) ||
      par->bc_left < 0 || par->bc_left > 1 || par->bc_right < 0 || par->bc_right > 1 ||
      !(par->alpha_floor >= 0.0) || !(par->merge_safety >= 0.0) || !(par->t_end > 0.0))
    return IMEXDS_ERR_INVALID_ARG;
  if (!(mat->a2_vap > 0.0) || !(mat->a2_liq > 0.0) || !(mat->p_sat > 0.0) ||
      !(mat->rho_liq_sat > 0.0) || !(mat->tau >= 0.0))
    return IMEXDS_ERR_INVALID_ARG;
  if (P > 0 && (!b->n_cells || !b->h || !b->x_left || !b->phase_first || !b->iface_off))
    return IMEXDS_ERR_INVALID_ARG;
  c->P = P;
  c->h_n_cells.assign(P, 0);
  c->h_h.assign(P, 0.0);
  c->h_x_left.assign(P, 0.0);
  c->h_phase_first.assign(P, 0);
  c->h_iface_off.assign(P + 1, 0);
  c->h_slot_off.assign(P + 1, 0);
  if (P > 0 && b->iface_off[0] != 0) return IMEXDS_ERR_INVALID_ARG;
  for (int p = 0; p < P; ++p) {
    int n = b->n_cells[p];
    int nif = b->iface_off[p + 1] - b->iface_off[p];
    if (n < 1 || nif < 0 || nif > imexds::MAX_IF_PER_PROB || !(b->h[p] > 0.0) ||
        (b->phase_first[p] != 0 && b->phase_first[p] != 1))
      return IMEXDS_ERR_INVALID_ARG;
    c->h_n_cells[p] = n;
    c->h_h[p] = b->h[p];
    c->h_x_left[p] = b->x_left[p];
    c->h_phase_first[p] = b->phase_first[p];
    c->h_iface_off[p + 1] = b->iface_off[p + 1];
    c->h_slot_off[p + 1] = c->h_slot_off[p] + n + nif;
    if (nif > c->max_nif) c->max_nif = nif;
  }
  c->NIF = P > 0 ? b->iface_off[P] : 0;
  c->S = c->h_slot_off[P];
  if (c->NIF > 0 && (!b->home || !b->hl)) return IMEXDS_ERR_INVALID_ARG;
  c->h_home0.assign(b->home, b->home + c->NIF);
  c->h_hl0.assign(b->hl, b->hl + c->NIF);
  c->h_iface_prob.assign(c->NIF, 0);
  c->h_iface_local.assign(c->NIF, 0);
  for (int p = 0; p < P; ++p) {
    int prev = -1;
    for (int k = b->iface_off[p]; k < b->iface_off[p + 1]; ++k) {
      int j = b->home[k];
      double hl = b->hl[k];
      if (j <= prev || j >= c->h_n_cells[p] || !(hl >= 0.0) || !(hl <= b->h[p]))
        return IMEXDS_ERR_INVALID_ARG;
      prev = j;
      c->h_iface_prob[k] = p;
      c->h_iface_local[k] = k - b->iface_off[p];
    }
  }
  c->mat.a2v = mat->a2_vap;
  c->mat.a2l = mat->a2_liq;
  c->mat.p0 = mat->p_sat;
  c->mat.rhol0 = mat->rho_liq_sat;
  c->mat.tau = mat->tau;
  c->mat.av = std::sqrt(mat->a2_vap);
  c->mat.al = std::sqrt(mat->a2_liq);
  c->mat.rhov0 = mat->p_sat / mat->a2_vap;
  c->mat.ia2v = 1.0 / c->mat.a2v;
  c->mat.ia2l = 1.0 / c->mat.a2l;
  c->mat.iav = 1.0 / c->mat.av;
  c->mat.ial = 1.0 / c->mat.al;
  c->mat.irv0 = 1.0 / c->mat.rhov0;
  c->mat.irl0 = 1.0 / c->mat.rhol0;
  c->par.cfl = par->cfl;
  c->par.theta_nb = par->theta_nb;
  c->par.tol_nb = par->tol_nb;
  c->par.tol_tiny = par->tol_tiny;
  c->par.tol_rel = par->tol_rel;
  c->par.alpha_floor = par->alpha_floor;
  c->par.merge_safety = par->merge_safety;
  c->par.newton_rtol = par->newton_rtol;
  c->par.t_end = par->t_end;
  c->par.zone_half = par->zone_half;
  c->par.tol_mode = par->tol_mode;
  c->par.lmax = par->lmax;
  c->par.bc_left = par->bc_left;
  c->par.bc_right = par->bc_right;
  c->par.newton_maxit = par->newton_maxit;
  c->par.zone_solver = IMEXDS_ZONE_DTS;
  c->par.zn_maxit = 30;
  c->par.zn_rtol = 1e-10;

  CK(hipGetDevice(&c->device));
  CK(hipStreamCreateWithFlags(&c->ms, hipStreamNonBlocking));
  CK(hipStreamCreateWithFlags(&c->zs, hipStreamNonBlocking));
  CK(hipStreamCreateWithFlags(&c->ps, hipStreamNonBlocking));
  CK(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
  CK(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
  CK(hipEventCreate(&c->ev_t0));
  CK(hipEventCreate(&c->ev_t1));
  CK(hipEventCreateWithFlags(&c->ev_rev, hipEventDisableTiming));
  CK(hipEventCreateWithFlags(&c->ev_rec, hipEventDisableTiming));
  int r = ensure_events(c, 1);
  if (r) return r;

  size_t Pn = (size_t)P, N = (size_t)c->NIF, S = (size_t)c->S;
  AL(c->d_slot_off, Pn + 1);
  AL(c->d_h, Pn);
  AL(c->d_phase_first, Pn);
  AL(c->d_iface_off, Pn + 1);
  AL(c->d_iface_prob, N);
  AL(c->d_iface_local, N);
  for (int a = 0; a < 2; ++a) {
    AL(c->d_rho[a], S);
    AL(c->d_mom[a], S);
    AL(c->d_home[a], N);
    AL(c->d_hl[a], N);
    AL(c->d_pw[a], 2 * N);
    AL(c->d_warm[a], N);
  }
  AL(c->d_dt, Pn);
  AL(c->d_t, Pn);
  AL(c->d_status, Pn);
  AL(c->d_clipped, Pn);
  AL(c->d_fail, Pn);
  AL(c->d_steps, Pn);
  AL(c->d_S, Pn);
  AL(c->d_stats, N_STATS);
  AL(c->d_pair_seen, 1);
  AL(c->d_log_row, 1);
  AL(c->d_zone_ctr, 1);
  CK(hipMemcpy(c->d_slot_off, c->h_slot_off.data(), (Pn + 1) * 8, hipMemcpyHostToDevice));
  if (P > 0) {
    CK(hipMemcpy(c->d_h, c->h_h.data(), Pn * 8, hipMemcpyHostToDevice));
    CK(hipMemcpy(c->d_phase_first, c->h_phase_first.data(), Pn * 4, hipMemcpyHostToDevice));
  }
  CK(hipMemcpy(c->d_iface_off, c->h_iface_off.data(), (Pn + 1) * 4, hipMemcpyHostToDevice));
  if (N > 0) {
    CK(hipMemcpy(c->d_iface_prob, c->h_iface_prob.data(), N * 4, hipMemcpyHostToDevice));
    CK(hipMemcpy(c->d_iface_local, c->h_iface_local.data(), N * 4, hipMemcpyHostToDevice));
  }
  CK(hipMemset(c->d_log_row, 0, 4));
  CK(hipMemset(c->d_zone_ctr, 0, 4));
  return build_tiles(c, c->tile_cells);
}

int imexds_create(imexds_ctx** out, const imexds_material* mat, const imexds_params* par,
                  const imexds_batch* batch, void* hip_stream) {
  if (!out) return IMEXDS_ERR_INVALID_ARG;
  *out = nullptr;
  if (!mat || !par || !batch) return IMEXDS_ERR_INVALID_ARG;
  imexds_ctx* c = new (std::nothrow) imexds_ctx();
  if (!c) return IMEXDS_ERR_OOM;
  c->user = (hipStream_t)hip_stream;
  int r = create_impl(c, mat, par, batch);
  if (r) {
    imexds_destroy(c);
    return r;
  }
  *out = c;
  return 0;
}

int imexds_set_state(imexds_ctx* c, const double* rho, const double* mom) {
  if (!c || (c->S > 0 && (!rho || !mom))) return IMEXDS_ERR_INVALID_ARG;
  int r = begin_call(c);
  if (r) return r;
  size_t S = (size_t)c->S, N = (size_t)c->NIF, P = (size_t)c->P;
  c->parity = 0;
  hipStream_t m = c->ms;
  if (S) {
    CK(hipMemcpyAsync(c->d_rho[0], rho, S * 8, hipMemcpyDeviceToDevice, m));
    CK(hipMemcpyAsync(c->d_mom[0], mom, S * 8, hipMemcpyDeviceToDevice, m));
  }
  if (N) {
    CK(hipMemcpyAsync(c->d_home[0], c->h_home0.data(), N * 4, hipMemcpyHostToDevice, m));
    CK(hipMemcpyAsync(c->d_hl[0], c->h_hl0.data(), N * 8, hipMemcpyHostToDevice, m));
    CK(hipMemsetAsync(c->d_pw[0], 0, 2 * N * 8, m));
    CK(hipMemsetAsync(c->d_warm[0], 0, N * 4, m));
  }
  if (P) {
    CK(hipMemsetAsync(c->d_t, 0, P * 8, m));
    CK(hipMemsetAsync(c->d_dt, 0, P * 8, m));
    CK(hipMemsetAsync(c->d_status, 0, P * 4, m));
    CK(hipMemsetAsync(c->d_clipped, 0, P * 4, m));
    CK(hipMemsetAsync(c->d_fail, 0, P * 4, m));
    CK(hipMemsetAsync(c->d_steps, 0, P * 8, m));
    CK(hipMemsetAsync(c->d_S, 0, P * 8, m));
  }
  CK(hipMemsetAsync(c->d_stats, 0, N_STATS * 8, m));
  c->n_call_ev = 0;
  c->acc_gpu_ms = 0.0;
  CK(hipMemsetAsync(c->d_log_row, 0, 4, m));
  CK(hipMemsetAsync(c->d_zone_ctr, 0, 4, m));
  // host->device copies above read pageable host memory: finish them here
  CK(hipStreamSynchronize(m));
  if (P) {
    r = init_dt(c);
    if (r) return r;
  }
  c->has_state = true;
  free_checkpoints(c);
  return end_call(c);
}

int imexds_step(imexds_ctx* c, int32_t n_steps) {
  if (!c || n_steps < 0) return IMEXDS_ERR_INVALID_ARG;
  if (!c->has_state) return IMEXDS_ERR_NO_STATE;
  int r = begin_call(c);
  if (r) return r;
  c->adj_ready = false;
  c->bulk_launches = 0;
  if ((r = call_begin(c))) return r;
  CK(hipEventRecord(c->ev_t0, c->ms));
  if (c->P > 0 && (r = steps_impl(c, n_steps))) return r;
  CK(hipEventRecord(c->ev_t1, c->ms));
  if ((r = call_end(c))) return r;
  c->timed = true;
  return end_call(c);
}

int imexds_step_per_problem(imexds_ctx* c, int32_t n_steps) {
  if (!c || n_steps < 0) return IMEXDS_ERR_INVALID_ARG;
  if (!c->has_state) return IMEXDS_ERR_NO_STATE;
  int r = begin_call(c);
  if (r) return r;
  c->adj_ready = false;
  c->bulk_launches = 0;
  if ((r = call_begin(c))) return r;
  CK(hipEventRecord(c->ev_t0, c->ms));
  for (int n = 0; n < n_steps; ++n) {
    StepArgs A = make_args(c, c->parity, false);
    for (int p = 0; p < c->P; ++p) {
      int k0 = c->h_iface_off[p], k1 = c->h_iface_off[p + 1];
      if (k1 > k0) CK(launch_zones(c, A, k0, k1, 0, c->ms));
      int t0 = c->h_tile_off[p], t1 = c->h_tile_off[p + 1];
      CK(imexds::launch_bulk(A, c->tile_cells, t0, t1 - t0, c->ms));
      CK(imexds::launch_finalize(A, p, p + 1, 0, p == c->P - 1, c->ms));
    }
    c->parity ^= 1;
  }
  CK(hipEventRecord(c->ev_t1, c->ms));
  if ((r = call_end(c))) return r;
  c->timed = true;
  return end_call(c);
}

int imexds_run(imexds_ctx* c, int32_t max_steps, int32_t check_every, int32_t* steps_done) {
  if (!c || max_steps < 0 || check_every < 1) return IMEXDS_ERR_INVALID_ARG;
  if (!c->has_state) return IMEXDS_ERR_NO_STATE;
  int r = begin_call(c);
  if (r) return r;
  c->adj_ready = false;
  int done = 0;
  std::vector<double> dt(c->P);
  if ((r = call_begin(c))) return r;
  CK(hipEventRecord(c->ev_t0, c->ms));
  while (done < max_steps && c->P > 0) {
    CK(hipMemcpyAsync(dt.data(), c->d_dt, sizeof(double) * c->P, hipMemcpyDeviceToHost, c->ms));
    CK(hipStreamSynchronize(c->ms));
    bool any = false;
    for (double d : dt) any = any || d > 0.0;
    if (!any) break;
    int n = std::min(check_every, max_steps - done);
    if ((r = steps_impl(c, n))) return r;
    done += n;
  }
  CK(hipEventRecord(c->ev_t1, c->ms));
  if ((r = call_end(c))) return r;
  c->timed = true;
  if (steps_done) *steps_done = done;
  return end_call(c);
}

int imexds_get_state(imexds_ctx* c, double* rho, double* mom) {
  if (!c || (c->S > 0 && (!rho || !mom))) return IMEXDS_ERR_INVALID_ARG;
  if (!c->has_state) return IMEXDS_ERR_NO_STATE;
  int r = begin_call(c);
  if (r) return r;
  size_t S = (size_t)c->S;
  if (S) {
    CK(hipMemcpyAsync(rho, c->d_rho[c->parity], S * 8, hipMemcpyDeviceToDevice, c->ms));
    CK(hipMemcpyAsync(mom, c->d_mom[c->parity], S * 8, hipMemcpyDeviceToDevice, c->ms));
  }
  return end_call(c);
}

int imexds_get_interfaces(imexds_ctx* c, int32_t* home, double* hl, double* x_iface) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  if (!c->has_state) return IMEXDS_ERR_NO_STATE;
  CK(hipSetDevice(c->device));
  size_t N = (size_t)c->NIF;
  if (!N) return 0;
  std::vector<int> hh(N);
  std::vector<double> ll(N);
  CK(hipMemcpyAsync(hh.data(), c->d_home[c->parity], N * 4, hipMemcpyDeviceToHost, c->ms));
  CK(hipMemcpyAsync(ll.data(), c->d_hl[c->parity], N * 8, hipMemcpyDeviceToHost, c->ms));
  CK(hipStreamSynchronize(c->ms));
  for (size_t k = 0; k < N; ++k) {
    if (home) home[k] = hh[k];
    if (hl) hl[k] = ll[k];
    if (x_iface) {
      int p = c->h_iface_prob[k];
      x_iface[k] = c->h_x_left[p] + hh[k] * c->h_h[p] + ll[k];
    }
  }
  return 0;
}

int imexds_get_problems(imexds_ctx* c, double* t, int32_t* status, int64_t* steps) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  if (!c->has_state) return IMEXDS_ERR_NO_STATE;
  CK(hipSetDevice(c->device));
  size_t P = (size_t)c->P;
  if (!P) return 0;
  if (t) CK(hipMemcpyAsync(t, c->d_t, P * 8, hipMemcpyDeviceToHost, c->ms));
  if (status) CK(hipMemcpyAsync(status, c->d_status, P * 4, hipMemcpyDeviceToHost, c->ms));
  if (steps) CK(hipMemcpyAsync(steps, c->d_steps, P * 8, hipMemcpyDeviceToHost, c->ms));
  CK(hipStreamSynchronize(c->ms));
  return 0;
}

int imexds_enable_log(imexds_ctx* c, int32_t max_steps) {
  if (!c || max_steps < 0) return IMEXDS_ERR_INVALID_ARG;
  CK(hipSetDevice(c->device));
  CK(hipStreamSynchronize(c->ms));
  drop_graph(c);
  if (c->d_log_count) {
    (void)hipFree(c->d_log_count);
    (void)hipFree(c->d_log_flags);
    (void)hipFree(c->d_log_zlo);
    c->d_log_count = c->d_log_flags = c->d_log_zlo = nullptr;
  }
  c->log_max = 0;
  if (max_steps > 0 && c->NIF > 0) {
    size_t n = (size_t)max_steps * (size_t)c->NIF;
    if (hipMalloc((void**)&c->d_log_count, n * 4) != hipSuccess ||
        hipMalloc((void**)&c->d_log_flags, n * 4) != hipSuccess ||
        hipMalloc((void**)&c->d_log_zlo, n * 4) != hipSuccess)
      return IMEXDS_ERR_OOM;
    c->log_max = max_steps;
  }
  CK(hipMemset(c->d_log_row, 0, 4));
  return 0;
}

int imexds_get_log(imexds_ctx* c, int32_t* count, int32_t* flags, int32_t* zlo, int32_t* rows) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  CK(hipSetDevice(c->device));
  int row = 0;
  CK(hipMemcpyAsync(&row, c->d_log_row, 4, hipMemcpyDeviceToHost, c->ms));
  CK(hipStreamSynchronize(c->ms));
  int n = std::min(row, c->log_max);
  if (rows) *rows = n;
  size_t cnt = (size_t)n * (size_t)c->NIF;
  if (cnt) {
    if (count) CK(hipMemcpy(count, c->d_log_count, cnt * 4, hipMemcpyDeviceToHost));
    if (flags) CK(hipMemcpy(flags, c->d_log_flags, cnt * 4, hipMemcpyDeviceToHost));
    if (zlo) CK(hipMemcpy(zlo, c->d_log_zlo, cnt * 4, hipMemcpyDeviceToHost));
  }
  return 0;
}

int imexds_get_stats(imexds_ctx* c, imexds_stats* out) {
  if (!c || !out) return IMEXDS_ERR_INVALID_ARG;
  CK(hipSetDevice(c->device));
  memset(out, 0, sizeof(*out));
  unsigned long long st[N_STATS] = {};
  CK(hipMemcpyAsync(st, c->d_stats, N_STATS * 8, hipMemcpyDeviceToHost, c->ms));
  size_t P = (size_t)c->P;
  std::vector<long long> steps(P);
  std::vector<int> status(P);
  std::vector<double> dt(P);
  if (P) {
    CK(hipMemcpyAsync(steps.data(), c->d_steps, P * 8, hipMemcpyDeviceToHost, c->ms));
    CK(hipMemcpyAsync(status.data(), c->d_status, P * 4, hipMemcpyDeviceToHost, c->ms));
    CK(hipMemcpyAsync(dt.data(), c->d_dt, P * 8, hipMemcpyDeviceToHost, c->ms));
  }
  CK(hipStreamSynchronize(c->ms));
  for (size_t p = 0; p < P; ++p) {
    out->steps += steps[p];
    out->cell_updates += steps[p] * (c->h_slot_off[p + 1] - c->h_slot_off[p]);
    if (status[p]) out->n_failed++;
    if (dt[p] > 0.0) out->n_active++;
  }
  out->pseudo_iters = (int64_t)st[0];
  out->merges = (int64_t)st[1];
  out->lmax_hits = (int64_t)st[2];
  out->newton_iters = (int64_t)st[3];
  out->iface_solves = (int64_t)st[4];
  out->events = (int64_t)st[5];
  out->pair_zones = (int64_t)st[6];
  int r = fold_call_events(c, true);
  if (r) return r;
  out->gpu_ms = c->acc_gpu_ms;
  return 0;
}

int imexds_set_launch(imexds_ctx* c, int32_t tile_cells, int32_t zones_per_group,
                      int32_t zone_groups, int32_t graph_steps, int32_t zone_lanes) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  if (tile_cells != 256 && tile_cells != 512 && tile_cells != 1024 && tile_cells != 2048)
    return IMEXDS_ERR_INVALID_ARG;
  if (zone_lanes != 1 && zone_lanes != 8) return IMEXDS_ERR_INVALID_ARG;
  if (zones_per_group < 1 || zones_per_group > 64 || zone_groups < 0 || graph_steps < 0 ||
      (graph_steps & 1) || graph_steps > 512)
    return IMEXDS_ERR_INVALID_ARG;
  CK(hipSetDevice(c->device));
  CK(hipStreamSynchronize(c->ms));
  drop_graph(c);
  c->zones_per_group = zones_per_group;
  c->zone_groups = zone_groups;
  c->graph_steps = graph_steps;
  c->zone_lanes = zone_lanes;
  if (tile_cells != c->tile_cells) return build_tiles(c, tile_cells);
  return 0;
}

int imexds_set_zone_solver(imexds_ctx* c, int32_t solver, int32_t maxit, double rtol) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  if (solver != IMEXDS_ZONE_DTS && solver != IMEXDS_ZONE_NEWTON) return IMEXDS_ERR_INVALID_ARG;
  if (maxit < 1 || !(rtol > 0.0) || !std::isfinite(rtol)) return IMEXDS_ERR_INVALID_ARG;
  CK(hipSetDevice(c->device));
  CK(hipStreamSynchronize(c->ms));
  CK(hipStreamSynchronize(c->zs));
  CK(hipStreamSynchronize(c->ps));
  c->par.zone_solver = solver;
  c->par.zn_maxit = maxit;
  c->par.zn_rtol = rtol;
  c->adj_ready = false;
  drop_graph(c);
  return 0;
}

int imexds_autotune(imexds_ctx* c, int32_t steps_per_trial, int32_t* tile_cells,
                    int32_t* zones_per_group, int32_t* zone_groups, int32_t* zone_lanes,
                    double* ms_per_step) {
  if (!c || steps_per_trial < 1) return IMEXDS_ERR_INVALID_ARG;
  if (!c->has_state) return IMEXDS_ERR_NO_STATE;
  CK(hipSetDevice(c->device));
  CK(hipStreamSynchronize(c->user));
  c->adj_ready = false;
  Snapshot s;
  int r = snap_take(c, s);
  if (r) {
    snap_free(s);
    return r;
  }
  struct Cfg {
    int t, z, g, n;
  };
  std::vector<Cfg> cfgs;
  // one lane per zone: zones spread one per lane over many waves, or fewer
  // lanes pulling several zones each; eight lanes per zone: one wave per
  // eight zones, or fewer waves pulling zones
  const int zl[] = {4, 8, 16, 64};
  const int gf[] = {0, 1, 2, 4};  // 0: all zones at once; else groups = CUs * f
  for (int z : zl)
    for (int f : gf) cfgs.push_back({1024, z, f == 0 ? 0 : 256 * f, 1});
  const int g8[] = {2, 4, 8};  // zone groups (of eight lanes) per wave
  for (int z : g8)
    for (int f : gf) cfgs.push_back({1024, z, f == 0 ? 0 : 256 * f, 8});
  int best_t = c->tile_cells, best_z = c->zones_per_group, best_g = c->zone_groups,
      best_n = c->zone_lanes;
  double best = 1e300;
  int G = c->graph_steps;
  auto trial = [&](const Cfg& q, double& per) -> int {
    int rr = imexds_set_launch(c, q.t, q.z, q.g, G, q.n);
    if (rr) return rr;
    if ((rr = snap_restore(c, s))) return rr;
    if ((rr = steps_impl(c, 2))) return rr;  // warm-up (also captures the graph)
    if ((rr = snap_restore(c, s))) return rr;
    CK(hipEventRecord(c->ev_t0, c->ms));
    if ((rr = steps_impl(c, steps_per_trial))) return rr;
    CK(hipEventRecord(c->ev_t1, c->ms));
    CK(hipEventSynchronize(c->ev_t1));
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, c->ev_t0, c->ev_t1));
    per = ms / steps_per_trial;
    return 0;
  };
  // stage 1: zone launch shape at a mid tile size; stage 2: tile size
  for (const Cfg& q : cfgs) {
    double per = 0.0;
    if ((r = trial(q, per))) break;
    if (per < best) {
      best = per;
      best_z = q.z;
      best_g = q.g;
      best_t = q.t;
      best_n = q.n;
    }
  }
  if (!r) {
    const int tiles[] = {256, 512, 2048};
    for (int t : tiles) {
      double per = 0.0;
      if ((r = trial({t, best_z, best_g, best_n}, per))) break;
      if (per < best) {
        best = per;
        best_t = t;
      }
    }
  }
  int r2 = imexds_set_launch(c, best_t, best_z, best_g, G, best_n);
  int r3 = snap_restore(c, s);
  snap_free(s);
  if (r) return r;
  if (r2) return r2;
  if (r3) return r3;
  if (tile_cells) *tile_cells = best_t;
  if (zones_per_group) *zones_per_group = best_z;
  if (zone_groups) *zone_groups = best_g;
  if (zone_lanes) *zone_lanes = best_n;
  if (ms_per_step) *ms_per_step = best;
  return 0;
}

int imexds_get_sizes(imexds_ctx* c, int32_t* n_problems, int32_t* n_iface, int64_t* n_slots) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  if (n_problems) *n_problems = c->P;
  if (n_iface) *n_iface = c->NIF;
  if (n_slots) *n_slots = c->S;
  return 0;
}

int imexds_last_timing(imexds_ctx* c, double* total_ms, double* bulk_ms_per_launch) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  CK(hipSetDevice(c->device));
  if (!c->timed) return IMEXDS_ERR_NO_STATE;
  CK(hipEventSynchronize(c->ev_t1));
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, c->ev_t0, c->ev_t1));
  if (total_ms) *total_ms = ms;
  if (bulk_ms_per_launch) {
    double sum = 0.0;
    for (int i = 0; i < c->bulk_launches; ++i) {
      float b = 0.f;
      CK(hipEventElapsedTime(&b, c->bulk_ev[2 * i], c->bulk_ev[2 * i + 1]));
      sum += b;
    }
    *bulk_ms_per_launch = c->bulk_launches ? sum / c->bulk_launches : 0.0;
  }
  return 0;
}

int imexds_time_bulk(imexds_ctx* c, int32_t on) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  c->time_bulk = on != 0;
  return 0;
}

int imexds_kernel_timing(imexds_ctx* c, double* bulk_ms, double* zone_ms, int32_t* launches) {
  if (!c) return IMEXDS_ERR_INVALID_ARG;
  CK(hipSetDevice(c->device));
  if (!c->timed) return IMEXDS_ERR_NO_STATE;
  CK(hipEventSynchronize(c->ev_t1));
  const int n = c->bulk_launches;
  double sb = 0.0, sz = 0.0;
  for (int i = 0; i < n; ++i) {
    float b = 0.f, z = 0.f;
    CK(hipEventElapsedTime(&b, c->bulk_ev[2 * i], c->bulk_ev[2 * i + 1]));
    CK(hipEventElapsedTime(&z, c->zone_ev[2 * i], c->zone_ev[2 * i + 1]));
    sb += b;
    sz += z;
  }
  if (bulk_ms) *bulk_ms = n ? sb / n : 0.0;
  if (zone_ms) *zone_ms = n ? sz / n : 0.0;
  if (launches) *launches = n;
  return 0;
}

int imexds_set_tau(imexds_ctx* c, double tau) {
  if (!c || !(tau >= 0.0) || !std::isfinite(tau)) return IMEXDS_ERR_INVALID_ARG;
  CK(hipSetDevice(c->device));
  CK(hipStreamSynchronize(c->ms));
  drop_graph(c);  // the captured launches hold the material by value
  c->mat.tau = tau;
  c->adj_ready = false;
  return 0;
}

int imexds_forward_ckpt(imexds_ctx* c, int32_t n_steps, int32_t ckpt_every) {
  if (!c || n_steps < 0 || ckpt_every < 1) return IMEXDS_ERR_INVALID_ARG;
  if (!c->has_state) return IMEXDS_ERR_NO_STATE;
  if (c->par.zone_solver != IMEXDS_ZONE_DTS) {
    snprintf(g_err, sizeof(g_err), "the adjoint covers the dual time zone solver only");
    return IMEXDS_ERR_UNSUPPORTED;
  }
  int r = begin_call(c);
  if (r) return r;
  CK(hipStreamSynchronize(c->ms));
  free_checkpoints(c);
  c->bulk_launches = 0;
  CK(hipMemsetAsync(c->d_pair_seen, 0, 4, c->ms));
  CK(hipEventRecord(c->ev_t0, c->ms));
  const int nck = (n_steps + ckpt_every - 1) / ckpt_every;
  c->ck.resize(nck);
  // the last segment is run with its tape recorded: the reverse sweep starts
  // there without re-running it
  if (nck > 0 && (r = ensure_adjoint_buffers(c, std::max(1, std::min(ckpt_every, n_steps)))))
    return r;
  for (int j = 0; j < nck; ++j) {
    if ((r = snap_take(c, c->ck[j]))) return r;
    const int len = std::min(ckpt_every, n_steps - j * ckpt_every);
    if (c->P > 0) {
      if (j == nck - 1) {
        if ((r = record_segment(c, 0, len, c->ms))) return r;
        c->tape[0].seg = j;
      } else if ((r = steps_impl(c, len))) {
        return r;
      }
    }
  }
  if ((r = snap_take(c, c->ck_end))) return r;
  c->ck_end_valid = true;
  CK(hipEventRecord(c->ev_t1, c->ms));
  int seen = 0;
  CK(hipMemcpyAsync(&seen, c->d_pair_seen, 4, hipMemcpyDeviceToHost, c->ms));
  CK(hipStreamSynchronize(c->ms));
  c->adj_pairs = seen != 0;
  c->timed = true;
  c->adj_steps = n_steps;
  c->adj_every = ckpt_every;
  c->adj_ready = true;
  return end_call(c);
}

int imexds_adjoint(imexds_ctx* c, const double* gL_rho, const double* gL_mom,
                   const double* gL_hl, double* g_rho0, double* g_mom0, double* g_hl0,
                   double* g_tau) {
  if (!c || (c->S > 0 && (!gL_rho || !gL_mom || !g_rho0 || !g_mom0)) || !g_tau)
    return IMEXDS_ERR_INVALID_ARG;
  if (!c->adj_ready) {
    snprintf(g_err, sizeof(g_err), "imexds_adjoint needs a preceding imexds_forward_ckpt");
    return IMEXDS_ERR_NO_STATE;
  }
  if (c->adj_pairs) {
    snprintf(g_err, sizeof(g_err),
             "the adjoint does not cover zones holding two phase boundaries, which the "
             "recorded forward solved");
    return IMEXDS_ERR_UNSUPPORTED;
  }
  int r = begin_call(c);
  if (r) return r;
  const int n = c->adj_steps, C = c->adj_every;
  if ((r = ensure_adjoint_buffers(c, std::max(1, std::min(C, n))))) return r;
  const size_t S = (size_t)c->S, N = (size_t)c->NIF, P = (size_t)c->P;
  hipStream_t m = c->ms;
  CK(hipEventRecord(c->ev_t0, m));
  if (S) {
    CK(hipMemcpyAsync(c->d_gr[0], gL_rho, S * 8, hipMemcpyDeviceToDevice, m));
    CK(hipMemcpyAsync(c->d_gm[0], gL_mom, S * 8, hipMemcpyDeviceToDevice, m));
  }
  if (N) {
    if (gL_hl)
      CK(hipMemcpyAsync(c->d_hlbar, gL_hl, N * 8, hipMemcpyDeviceToDevice, m));
    else
      CK(hipMemsetAsync(c->d_hlbar, 0, N * 8, m));
    CK(hipMemsetAsync(c->d_taubar, 0, N * 8, m));
  }
  if (P) CK(hipMemsetAsync(c->d_tbar, 0, P * 8, m));
  int cur = 0;
  const int nck = (int)c->ck.size();
  // the tape that holds the last segment (imexds_forward_ckpt recorded it)
  int t = (c->n_tapes > 1 && c->tape[1].seg == nck - 1) ? 1 : 0;
  // With two tapes, while segment seg is reversed on ms the segment before
  // it is recomputed into the other tape on ps, after the reverse sweep that
  // last read that tape: each reads only its own tape, checkpoint and
  // buffers.  With one tape, each segment is recomputed and then reversed.
  const bool two = nck > 1 && ensure_second_tape(c);
  hipStream_t q = c->ps;
  for (int seg = nck - 1; seg >= 0; --seg) {
    const int len = std::min(C, n - seg * C);
    if (c->tape[t].seg != seg) {
      if ((r = snap_restore(c, c->ck[seg]))) return r;
      if ((r = record_segment(c, t, len, m))) return r;
      c->tape[t].seg = seg;
    }
    const bool ahead = two && seg > 0;
    if (ahead) {
      const int u = t ^ 1;
      CK(hipEventRecord(c->ev_rev, m));
      CK(hipStreamWaitEvent(q, c->ev_rev, 0));
      if ((r = snap_restore(c, c->ck[seg - 1], q, false))) return r;
      if ((r = record_segment(c, u, std::min(C, n - (seg - 1) * C), q))) return r;
      c->tape[u].seg = seg - 1;
      CK(hipEventRecord(c->ev_rec, q));
    }
    if ((r = reverse_segment(c, t, len, cur, len != C))) return r;
    cur ^= len & 1;
    if (ahead) {
      CK(hipStreamWaitEvent(m, c->ev_rec, 0));
      t ^= 1;
    }
  }
  if (S) {
    CK(hipMemcpyAsync(g_rho0, c->d_gr[cur], S * 8, hipMemcpyDeviceToDevice, m));
    CK(hipMemcpyAsync(g_mom0, c->d_gm[cur], S * 8, hipMemcpyDeviceToDevice, m));
  }
  if (N && g_hl0) CK(hipMemcpyAsync(g_hl0, c->d_hlbar, N * 8, hipMemcpyDeviceToDevice, m));
  if (N)
    CK(imexds::launch_sum(c->d_taubar, c->NIF, g_tau, m));
  else
    CK(hipMemsetAsync(g_tau, 0, 8, m));
  CK(hipEventRecord(c->ev_t1, m));
  c->timed = true;
  if ((r = snap_restore(c, c->ck_end))) return r;  // leave the end state in place
  return end_call(c);
}

}  // extern "C"
