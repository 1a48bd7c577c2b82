// Kernel argument blocks and launchers shared by the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cpselect.h"
#include "cp_state.h"

namespace cps {

constexpr int kSelectBlock = 256;
constexpr int kSelectUnroll = 4;

// Grid-synchronisation words of the single-array kernel.  `arrive` counts workgroups
// that finished the current pass; `gen` is bumped by the last one when the next pass
// may start; curL / curR hand out write offsets for the split of the current pass.
struct SyncCtl {
  uint32_t arrive;
  uint32_t gen;
  uint32_t pad0, pad1;
  uint64_t curL, curR;
};

template <typename T> struct SelectArgs {
  const T *x;
  int64_t n, k;
  CpState *st;
  SyncCtl *sync;
  double *sd;          // per-workgroup partials, 8 fields x slot_stride
  int64_t *si;         // per-workgroup integer partials, 8 fields x slot_stride
  int64_t slot_stride;
  T *z[2];             // split buffers, zcap elements each
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
