// imexds_kernels.hpp -- kernel arguments and launchers shared by the kernels
// and the host runtime of the IMEX-DS library.
#pragma once

#include <hip/hip_runtime.h>

#include "imexds_device.hpp"

namespace imexds {

constexpr int MAX_IF_PER_PROB = 64;

// Everything one step needs, passed by value to each kernel.  "0" buffers
// hold the state at t^n, "1" buffers receive t^{n+1}.
struct StepArgs {
  Mat mat;
  Par par;
  const long long* slot_off;  // [P+1]
  const double* h;            // [P]
  const int* phase_first;     // [P]
  const int* iface_off;       // [P+1]
  const int* iface_prob;      // [NIF]
  const int* iface_local;     // [NIF] index of the interface inside its problem
  const int* tile_prob;       // [tiles]
  const int* tile_start;      // [tiles] first slot of the tile, local to the problem
  const int* tile_len;        // [tiles]
  const double* rho0;
  const double* mom0;
  double* rho1;
  double* mom1;
  const int* rec_home0;
  const double* rec_hl0;
  const double* rec_pw0;
  const int* rec_warm0;
  int* rec_home1;
  double* rec_hl1;
  double* rec_pw1;
  int* rec_warm1;
  double* dt;
  double* t;
  int* status;
  int* clipped;
  long long* steps;
  unsigned long long* S_acc;  // bit patterns of non-negative doubles (max = numeric max)
  int* fail_acc;
  int* log_count;
  int* log_flags;
  int* log_zlo;
  int* log_row;
  int log_max;
  int n_iface;
  unsigned long long* st_pseudo;
  unsigned long long* st_merges;
  unsigned long long* st_lmax;
  unsigned long long* st_newton;  // evaluations of G in the interface solves
  unsigned long long* st_solves;  // interface solves
  unsigned long long* st_events;  // merges, redos and re-homings of interfaces
  unsigned long long* st_pairs;   // zone steps with two phase boundaries
  int* pair_seen;                 // set to 1 when a zone with two boundaries is solved
  int* zone_ctr;  // zones handed out so far in this step (reset by k_finalize)
  int zones_per_group;
  // zone tape of this step (nullptr: none).  Per interface, tape_stride
  // doubles: a header of TAPE_HDR values, then for l = 0..count the iterate
  // W^l of the zone (MC densities, MC momenta, MC = 2 zone_half + 1) and the
  // interface root (p_l*, p_r*) at W^l; entry `count` is the accepted iterate
  // of Part 2.
  double* tape;
  long long tape_stride;
};

// tape header: predicting root (2), predicted speed, count, log flags, zone
// start, accepted boundary speed w*
constexpr int TAPE_HDR = 8;
constexpr int TH_IPL = 0, TH_IPR = 1, TH_WP = 2, TH_COUNT = 3, TH_FLAGS = 4, TH_ZLO = 5,
              TH_WSTAR = 6;
inline long long tape_entry(int zone_half) { return 2 * (2 * zone_half + 1) + 2; }
inline long long tape_stride(int zone_half, int lmax) {
  return TAPE_HDR + (long long)(lmax + 1) * tape_entry(zone_half);
}

// Reverse sweep of one step (adjoint): arrays of adjoints ("g" = dL/d of).
struct AdjArgs {
  const double* gr1;  // [S] adjoint of rho^{n+1}
  const double* gm1;  // [S] adjoint of (rho u)^{n+1}
  double* gr0;        // [S] out: adjoint of rho^n
  double* gm0;
  double* hl_bar;     // [NIF] in: adjoint of hl^{n+1}; out: of hl^n
  double* tau_bar;    // [NIF] accumulated adjoint of tau per zone
  double* zadj;       // [NIF * 5] zone pass -> per-problem pass: adjoints of F_left, F_right, dt
  double* tile_gdt;   // [tiles] bulk cells' part of the adjoint of dt
  unsigned long long* tile_smax;  // [tiles] max |u| + a (bit pattern) over the tile
  int* tile_sidx;     // [tiles] first slot attaining it
  const int* tile_off;  // [P+1] tiles of each problem
  const long long* steps0;  // [P] step counters before and after the step
  const long long* steps1;  //     (t advanced iff they differ)
  double* t_bar;        // [P] adjoint of t
};

// Bulk tiles: tile_class in {256, 512, 1024, 2048} gives R = tile_class / 256
// rows of 62 cells per wave, 4 waves per workgroup: bulk_tile_cells() cells.
int bulk_tile_cells(int tile_class);
hipError_t launch_bulk(const StepArgs& A, int tile_class, int tile_begin, int n_tiles,
                       hipStream_t s);
hipError_t launch_cfl(const StepArgs& A, int tile_begin, int n_tiles, hipStream_t s);
// groups <= 0: one lane per zone; else that many workgroups whose lanes pull
// zones from the shared counter until none is left.
hipError_t launch_zone(const StepArgs& A, int if_begin, int if_end, int groups, hipStream_t s);
// the same zones with eight lanes per zone, eight zones per wave; groups <= 0:
// enough waves for all zones, else that many waves pulling zones
hipError_t launch_zone8(const StepArgs& A, int if_begin, int if_end, int groups, hipStream_t s);
// zones holding the two phase boundaries of neighbouring interfaces whose
// zones overlap (Algorithm 2 only; every interface of [if_begin, if_end) is
// a candidate)
hipError_t launch_zone_pair(const StepArgs& A, int if_begin, int if_end, hipStream_t s);

// Whether interface k (local index kk of the nif of its problem; ns slots,
// background width h) and interface k + 1 have overlapping zones (records of
// the step's start).  With Algorithm 2 such a pair is one zone; the
// single-boundary zone kernels leave both interfaces to k_zone_pair.
__device__ __forceinline__ bool d_pair_lead(const StepArgs& A, int k, int kk, int nif, int ns,
                                            double h) {
  if (kk < 0 || kk + 1 >= nif) return false;
  const int s0 = A.rec_home0[k] + kk, s1 = A.rec_home0[k + 1] + kk + 1;
  if (s0 < 0 || s1 < s0 + 2 || s1 + 1 >= ns) return false;  // records outside their problem
  int zlo0, zhi0, zlo1, zhi1;
  bool t0, t1;
  d_zone_range(A.rec_home0[k] + kk, A.rec_hl0[k], h, A.par.zone_half, ns, zlo0, zhi0, t0);
  d_zone_range(A.rec_home0[k + 1] + kk + 1, A.rec_hl0[k + 1], h, A.par.zone_half, ns, zlo1,
               zhi1, t1);
  return zlo1 <= zhi0;
}
// copies one step's records (N interface cells and cut lengths; P of dt,
// clip flags, step counters) into a tape slot
hipError_t launch_tape_copy(const int* home, const double* hl, const double* dt, const int* clip,
                            const long long* steps, int* t_home, double* t_hl, double* t_dt,
                            int* t_clip, long long* t_steps, int N, int P, hipStream_t s);
hipError_t launch_finalize(const StepArgs& A, int p_begin, int p_end, int init, int bump_row,
                           hipStream_t s);
// the zones solved by Newton on their implicit step (zone_half 1 or 2):
// 1 + 4 zone_half + 2 groups per zone of one lane (lanes == 1) or of two
// lanes (the pair form of the interface solver)
hipError_t launch_zone_newton(const StepArgs& A, int if_begin, int if_end, int lanes,
                              hipStream_t s);

// adjoint of one step: zone pass, then bulk pass, then per-problem pass
// lanes: 1 (one lane per zone) or 8 (eight lanes per zone)
hipError_t launch_zone_adj(const StepArgs& A, const AdjArgs& B, int lanes, hipStream_t s);
hipError_t launch_bulk_adj(const StepArgs& A, const AdjArgs& B, int tile_class, int n_tiles,
                           hipStream_t s);
hipError_t launch_finalize_adj(const StepArgs& A, const AdjArgs& B, int P, hipStream_t s);
hipError_t launch_sum(const double* x, int n, double* out, hipStream_t s);

}  // namespace imexds
