// Grouped-launch planning, shared by the grouped entry points and the
// serving runtime.
#pragma once

#include "host.hpp"

namespace mg {

struct GroupPlan {
    int mode = 0;
    const GroupedKernel *gk = nullptr;
    std::vector<GroupDesc> descs;   // sorted by descending per-tile cost
    std::vector<int> src;           // index of each descriptor's problem in the caller's list
    int total_tiles = 0;
    int nwg = 0;
};

const GroupedKernel *grouped_kernel(int mode);
int grouped_choose(int mode, int64_t m, int64_t n, int64_t k);
int grouped_choose_alone(int mode, int64_t m, int64_t n, int64_t k);

// Validate the problems (one mode), choose each problem's tile configuration
// and lay the tiles out; empty outputs are dropped.  `force` = 0 or 1 puts
// every problem on that option of the grouped kernel (tuning); -1 chooses.
int build_group_plan(const gemm_problem_t *ps, int32_t count, GroupPlan &plan, int force = -1);

// Copy the descriptors to the stream's device workspace (stream-ordered).
int upload_descs(const GroupPlan &plan, hipStream_t s, const GroupDesc **dev_out);

// Launch the persistent kernel over descriptors already on the device, with
// zeroed work-queue counters (the launch leaves them zeroed again).
int enqueue_group(const GroupPlan &plan, const GroupDesc *dev_descs, int32_t *counters, hipStream_t s);

// 256 bytes of zeroed device memory for a grouped launch's work queue.
int alloc_counters(int32_t **out);

}  // namespace mg
