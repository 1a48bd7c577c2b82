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

// Workgroups of one array: arrays of more than `chunk` elements are split into contiguous
// parts of about `chunk` elements, one workgroup each, at most `tmax` of them (1 when teams
// are off: tmax <= 1 or chunk <= 0).  Non-increasing in the size, so in the largest-first
// order the arrays with more than one workgroup come first.
CPS_HD inline int32_t team_blocks(int64_t size, int64_t chunk, int32_t tmax) {
  if (tmax <= 1 || chunk <= 0 || size <= chunk) return 1;
  const int64_t b = (size + chunk - 1) / chunk;
  return b > tmax ? tmax : (int32_t)b;
}

// After the largest-first sort, slot j of the order holds (first work item of the array in
// slot j) << 32 | (its index): the work items are the arrays' workgroup parts in that order,
// the B parts of one array consecutive.  Work item q belongs to the last slot whose first item
// is <= q (a binary search over the slots), as part q - first.
CPS_HD inline uint64_t item_entry(int64_t first_item, int64_t index) {
  return ((uint64_t)first_item << 32) | (uint64_t)index;
}
CPS_HD inline int64_t item_first(uint64_t e) { return (int64_t)(e >> 32); }
CPS_HD inline int64_t item_index(uint64_t e) { return (int64_t)(e & 0xffffffffull); }

// The slot of work item q among slots [0, count) (entries from item_entry, first items
// non-decreasing, slot 0's first item 0).
CPS_HD inline int64_t item_slot(const uint64_t *order, int64_t count, int64_t q) {
  int64_t lo = 0, hi = count - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (item_first(order[mid]) <= q) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// An array descriptor the kernel can run: a non-null pointer aligned to the element size,
// at least one element and a rank in [1, n].  Anything else gets status BADARG and is never
// read.
CPS_HD inline bool batch_array_valid(uint64_t addr, int64_t n, int64_t k, uint32_t esize) {
  return addr != 0 && n >= 1 && k >= 1 && k <= n && (addr % esize) == 0;
}

}  // namespace cps
