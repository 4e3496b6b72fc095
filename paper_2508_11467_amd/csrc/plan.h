// The merge-tree plan on the host: the recursive split of Section 4.2.1 at
// k = floor(m/2) down to leaves of at most `leaf` rows, for a batch of
// problems, with the descriptors the kernels read.  Host code only (no HIP
// calls), so it also builds and runs in the host sanitizer check.
#pragma once

#include <cstdint>
#include <vector>

#include "bdc_internal.h"

namespace bdc {

struct HostPlan {
  std::vector<LeafDesc> leaves;       // left to right, problem by problem
  std::vector<NodeDesc> nodes;        // by height 1, 2, ... (id = index), left to right in a height
  std::vector<int> level_count;       // merges of height h + 1
  std::vector<int> level_max_m;       // their largest size
  std::vector<int64_t> prob;          // 5 x batch: n, vector offset, matrix offset, first U item, first V^T item
  std::vector<int32_t> uprob, vprob;  // final-pass work item -> problem (U, V^T)
  int64_t total_n = 0, total_n2 = 0, total_cols = 0, total_tiles = 0;
  int root_id0 = -1;                  // first problem's root merge, if it has one
};

// sizes: batch problem sizes (>= 0); leaf >= 4
HostPlan build_host_plan(const int64_t* sizes, int64_t batch, int leaf);

}  // namespace bdc
