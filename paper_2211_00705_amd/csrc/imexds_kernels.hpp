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
  int* zone_ctr;  // zones handed out so far in this step (reset by k_finalize)
  int zones_per_group;
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
hipError_t launch_finalize(const StepArgs& A, int p_begin, int p_end, int init, int bump_row,
                           hipStream_t s);

}  // namespace imexds
