// Work order and descriptor checks of the batched selection.  Scalar code shared by the
// batched kernel and the host replay of its queue (tests/cpp), so both take the same
// decisions on the same descriptors.
#pragma once

#include <stdint.h>

#include "cp_state.h"

namespace cps {

constexpr int kBatchSortMax = 4096;  // arrays sorted largest-first in LDS up to this count

// Sort key of array j: its size (clamped to [0, 2^50]) above the complement of its index, so
// that a descending sort puts larger arrays first and, among equal sizes, lower indices first.
// Keys of the padding slots of the sort (j >= count) are 0, below every array's key.
CPS_HD inline uint64_t lpt_key(int64_t size, int64_t j) {
  int64_t sz = size < 0 ? 0 : size;
  if (sz > ((int64_t)1 << 50)) sz = (int64_t)1 << 50;
  return ((uint64_t)sz << 12) | (uint64_t)(kBatchSortMax - 1 - j);
}

CPS_HD inline int64_t lpt_index(uint64_t key) {
  return (int64_t)(kBatchSortMax - 1 - (key & (uint64_t)(kBatchSortMax - 1)));
}

// One compare-exchange of the descending bitonic network over order[0..m) (m a power of two),
// at stage (kk, jj), for element i: a no-op unless i is the lower index of its pair.
CPS_HD inline void bitonic_exchange(uint64_t *order, int64_t i, int64_t jj, int64_t kk) {
  const int64_t p = i ^ jj;
  if (p <= i) return;
  const uint64_t x0 = order[i], x1 = order[p];
  const bool desc = (i & kk) == 0;
  if (desc ? (x0 < x1) : (x0 > x1)) {
    order[i] = x1;
    order[p] = x0;
  }
}

// An array descriptor the kernel can run: a non-null pointer aligned to the element size,
// at least one element and a rank in [1, n].  Anything else gets status BADARG and is never
// read.
CPS_HD inline bool batch_array_valid(uint64_t addr, int64_t n, int64_t k, uint32_t esize) {
  return addr != 0 && n >= 1 && k >= 1 && k <= n && (addr % esize) == 0;
}

}  // namespace cps
