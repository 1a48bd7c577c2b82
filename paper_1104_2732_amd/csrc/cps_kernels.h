// Kernel argument blocks and launchers shared by the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cpselect.h"
#include "cp_state.h"

namespace cps {

constexpr int kWaveSize = 64;
constexpr int kSelectBlock = 512;
constexpr int kSelectUnroll = 4;
constexpr int kGroup = 16;       // workgroups per first-level arrival counter
constexpr int kMaxGroups = 256;  // so at most 4096 workgroups

// Grid-synchronisation words of the single-array kernel, each on its own 128-byte line.
// Workgroups arrive on grp[bid / kGroup]; the last of each group arrives on `top`; the last
// overall advances the state and bumps `gen`, on which the others wait.  gcur hands out
// write offsets in the gather buffer.
struct SyncCtl {
  uint32_t top;
  uint32_t gen;
  uint32_t pad0[30];
  uint64_t gcur;
  uint64_t pad1[15];
  uint32_t grp[kMaxGroups][32];
};

template <typename T> struct SelectArgs {
  const T *x;
  int64_t n, k;
  CpState *st;
  SyncCtl *sync;
  double *sd;          // per-workgroup partials, 8 fields x slot_stride
  int64_t *si;         // per-workgroup integer partials, 8 fields x slot_stride
  int64_t slot_stride;
  T *z[2];             // split buffers: one region of seg_R elements per wavefront
  int64_t seg_R;
  T *zf;               // gather buffer, cfg.zcap elements
  cps_result *out;
  cps_stats *stats;    // may be null
  CpConfig cfg;
  int64_t spin_limit;
};

template <typename T> hipError_t launch_select(const SelectArgs<T> &a, int grid, hipStream_t stream);
template <typename T> int select_max_blocks_per_cu();
template <typename T>
hipError_t launch_objective(const T *x, int64_t n, int64_t k, const double *ys, int64_t ny,
                            cps_eval *out, double *pd, int64_t *pi, int nb, hipStream_t stream);

}  // namespace cps
