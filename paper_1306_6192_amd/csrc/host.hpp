// Host-side internals shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace mg {

// Record a failure for gemm_last_error() and return `code`.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define MG_HIP(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return ::mg::fail(GEMM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t elem_size(int mode);
bool mode_known(int mode);

// Synchronous argument checks; no HIP call, no memory access.
int validate(const gemm_problem_t *p);

// Number of compute units of the current device (256 if it cannot be read).
int num_cus();

// Kernel configuration table of a mode.
const KernelCfg *configs(int mode, int *count);

// The TileProblem of one problem for one configuration and split-K factor
// (split is normalised so that no split is empty; C is left to the caller
// when split > 1).
struct Launch {
    TileProblem P;
    int nwg;
    int splits;
    int64_t ws_bytes;
};
Launch make_launch(const gemm_problem_t &p, const KernelCfg &kc, int split);

// Enqueue one plain product with an explicit configuration.  `ws` must hold
// `Launch::ws_bytes` when the split is above 1.
int enqueue_plain(const gemm_problem_t &p, int cfg, int split, void *ws, hipStream_t s);

// Whether the problem's shape, strides and alignment meet the configuration's
// chunk requirement, and the configuration actually run for it: a chunked
// configuration the problem does not meet is replaced by the any-shape one of
// the same tile size (both sum every element in the same order).
bool cfg_eligible(const gemm_problem_t &p, const KernelCfg &kc);
bool presplit_shape_ok(int64_t n, int64_t k);
int split_grain(int mode);
int effective_cfg(const gemm_problem_t &p, int cfg);

// Split-K workspace bytes the (cfg, split) choice needs for this problem.
int64_t plain_ws_bytes(const gemm_problem_t &p, int cfg, int split);

// Tuning table.
void tuner_choose(int mode, int64_t m, int64_t n, int64_t k, int *cfg, int *split);
void heuristic_choose(int mode, int64_t m, int64_t n, int64_t k, int *cfg, int *split);
// floor(log2(d)) (0 for d <= 1): the bucket of a dimension in the tables.
int dim_bucket(int64_t d);
// The grouped table's tile option for a problem launched alone (0 or 1: the
// larger or the smaller of the grouped kernel's alone configurations) for
// the bucket of (m, n, k); false when the bucket has not been measured.
bool tuner_grouped_alone(int mode, int64_t m, int64_t n, int64_t k, int *alone);
void tuner_record_grouped(int mode, int64_t m, int64_t n, int64_t k, int alone);
// The measured efficiency of a two-tile grouped kernel's small tile relative
// to its large one in a mixed batch (the planner's cost model weighs the
// padded tile area by it); < 0 when not measured.
double tuner_grouped_eff(int mode);
// The grouped kernel variant measured fastest on a mixed batch (0 when not
// measured); recorded together with the efficiency.
int tuner_grouped_variant(int mode);
void tuner_record_grouped_eff(int mode, double eff, int variant);

// A device buffer owned by the library that grows on demand.  Growth waits
// for `s` to drain before freeing the old allocation.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t need, hipStream_t s);
    void release();
};

// Per-stream library workspace (split-K slabs, grouped descriptors).
DevBuf *stream_workspace(hipStream_t s, int slot);

// Serialises host-side use of one (device, stream)'s workspaces: a caller
// holds it from a workspace's ensure() until the work that reads the
// workspace is enqueued, so that a caller on another host thread using the
// same stream cannot free and replace the buffer in between.
std::unique_lock<std::mutex> lock_stream_workspaces(hipStream_t s);

uint64_t now_ns();

// Address of the allocation-free entry point's device scratch on the current
// device (looked up once per device).
int noalloc_scratch(void **out);

}  // namespace mg
