// Grouped-launch planning, shared by the grouped entry points and the
// serving runtime.
#pragma once

#include "host.hpp"

namespace mg {

struct GroupPlan {
    int mode = 0;
    const GroupedKernel *gk = nullptr;
    std::vector<GroupDesc> descs;      // one per non-empty problem, in the caller's order
    std::vector<int> src;              // index of each descriptor's problem in the caller's list
    std::vector<int32_t> wg_first;     // nwg + 1 offsets into `tiles`
    std::vector<GroupTile> tiles;      // every workgroup's tile list, concatenated
    int total_tiles = 0;
    int nwg = 0;
};

const GroupedKernel *grouped_kernel(int mode);
int grouped_choose(int mode, int64_t m, int64_t n, int64_t k);
int grouped_choose_alone(int mode, int64_t m, int64_t n, int64_t k);

// Validate the problems (one mode), choose each problem's tile configuration
// and build the static schedule; empty outputs are dropped.  `force` = 0 or 1
// puts every problem on that option of the grouped kernel (tuning); -1
// chooses.
int build_group_plan(const gemm_problem_t *ps, int32_t count, GroupPlan &plan, int force = -1);

// The plan's device image (descriptors and schedule): its size, and its
// bytes written to host memory.
size_t plan_image_bytes(const GroupPlan &plan);
void plan_image_write(const GroupPlan &plan, void *dst);

// Copy the plan's image to the stream's device workspace (stream-ordered).
int upload_plan(const GroupPlan &plan, hipStream_t s, const void **dev_out);

// Launch the persistent kernel over a plan image already on the device.
int enqueue_group(const GroupPlan &plan, const void *dev_image, hipStream_t s);

}  // namespace mg
