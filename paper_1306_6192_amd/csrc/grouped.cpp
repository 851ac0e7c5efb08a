// Grouped product: many independent problems in one persistent launch, and
// its capture into a HIP graph.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>

#include "grouped.hpp"

namespace mg {

// Per-problem choice between the grouped kernel's two tile configurations:
// the tuning table's measured choice for the problem's shape bucket, else a
// cost model that weighs the padded tile area against the lower sustained
// rate of the small tile.
static int grouped_model(int mode, int64_t m, int64_t n, bool alone) {
    const GroupedKernel *gk = grouped_kernel(mode);
    int count = 0;
    const KernelCfg *t = configs(mode, &count);
    double best = 1e300;
    int pick = 0;
    for (int c = 0; c < 2; ++c) {
        const KernelCfg &kc = t[gk->cfg_idx[c]];
        const double tiles = (double)((m + kc.bm - 1) / kc.bm) * (double)((n + kc.bn - 1) / kc.bn);
        const double eff = (kc.bm * kc.bn >= 16384) ? 1.0 : 0.6;
        // alone, rounds of resident workgroups count: a mid-size product on
        // the large tile would leave most CUs idle
        const double slots = (double)num_cus() * std::max(1, gk->wg_per_cu);
        const double cost = (alone ? std::ceil(tiles / slots) : tiles) * kc.bm * kc.bn / eff;
        if (cost < best * 0.999) {
            best = cost;
            pick = c;
        }
    }
    return pick;
}

int grouped_choose(int mode, int64_t m, int64_t n, int64_t k) {
    int in_batch = 0, alone = 0;
    if (tuner_grouped_choice(mode, m, n, k, &in_batch, &alone)) return in_batch;
    return grouped_model(mode, m, n, false);
}

// The same choice for a problem launched on its own (a serving batch of one):
// the two tiles give the same bits, so the one that finishes first is taken.
int grouped_choose_alone(int mode, int64_t m, int64_t n, int64_t k) {
    int in_batch = 0, alone = 0;
    if (tuner_grouped_choice(mode, m, n, k, &in_batch, &alone)) return alone;
    return grouped_model(mode, m, n, true);
}

const GroupedKernel *grouped_kernel(int mode) {
    if (mode == GEMM_MODE_F32) return f32_grouped();
    return lp_grouped(mode);
}

int build_group_plan(const gemm_problem_t *ps, int32_t count, GroupPlan &plan, int force) {
    if (count < 0) return fail(GEMM_EINVAL, "negative problem count");
    if (count > 0 && !ps) return fail(GEMM_EINVAL, "problem array is NULL");
    plan.descs.clear();
    plan.src.clear();
    plan.total_tiles = 0;
    plan.mode = count > 0 ? ps[0].mode : GEMM_MODE_F32;
    for (int i = 0; i < count; ++i) {
        int rc = validate(&ps[i]);
        if (rc != GEMM_OK) {
            char why[256];
            snprintf(why, sizeof(why), "%s", gemm_last_error());
            return fail(rc, "problem %d: %s", i, why);
        }
        if (ps[i].mode != plan.mode) return fail(GEMM_EINVAL, "problem %d: all problems must share one mode", i);
    }
    plan.gk = grouped_kernel(plan.mode);
    if (!plan.gk) return fail(GEMM_EUNSUPPORTED, "mode %d has no grouped kernel", plan.mode);
    int tcount = 0;
    const KernelCfg *t = configs(plan.mode, &tcount);
    struct Item {
        GroupDesc d;
        double cost;
        int tiles;
        int src;
    };
    // A launch whose chosen tiles would not fill every resident-workgroup
    // slot runs every problem on the smaller tile instead (the tile does not
    // change the bits): a handful of mid-size problems then spread over the
    // chip rather than over a fraction of it.
    const int small = t[plan.gk->cfg_idx[1]].bm * t[plan.gk->cfg_idx[1]].bn <
                              t[plan.gk->cfg_idx[0]].bm * t[plan.gk->cfg_idx[0]].bn
                          ? 1
                          : 0;
    int64_t chosen_tiles = 0;
    for (int i = 0; i < count; ++i) {
        const gemm_problem_t &p = ps[i];
        if (p.m == 0 || p.n == 0) continue;
        const KernelCfg &kc = t[plan.gk->cfg_idx[force >= 0 ? force : grouped_choose(p.mode, p.m, p.n, p.k)]];
        chosen_tiles += ((p.m + kc.bm - 1) / kc.bm) * ((p.n + kc.bn - 1) / kc.bn);
    }
    const bool underfilled = force < 0 && chosen_tiles < (int64_t)num_cus() * plan.gk->wg_per_cu;
    std::vector<Item> items;
    items.reserve(count);
    for (int i = 0; i < count; ++i) {
        const gemm_problem_t &p = ps[i];
        if (p.m == 0 || p.n == 0) continue;
        Item it;
        memset(&it.d, 0, sizeof(it.d));
        it.src = i;
        it.d.cfg = force >= 0 ? force : underfilled ? small : grouped_choose(p.mode, p.m, p.n, p.k);
        const KernelCfg &kc = t[plan.gk->cfg_idx[it.d.cfg]];
        it.d.P = make_launch(p, kc, 1).P;
        it.tiles = it.d.P.tiles_m * it.d.P.tiles_n;
        it.cost = (double)kc.bm * kc.bn * (double)std::max<int64_t>(p.k, 1);
        items.push_back(it);
    }
    // Longest tiles first: workgroups take tiles from a queue in this order,
    // so the costliest tiles start first and the cheap ones fill the tail.
    std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) { return a.cost > b.cost; });
    int64_t start = 0;
    for (auto &it : items) {
        it.d.tile_start = (int32_t)start;
        start += it.tiles;
        if (start > INT32_MAX) return fail(GEMM_EUNSUPPORTED, "grouped launch above 2^31 tiles");
        plan.descs.push_back(it.d);
        plan.src.push_back(it.src);
    }
    plan.total_tiles = (int)start;
    plan.nwg = (int)std::min<int64_t>(start, (int64_t)num_cus() * plan.gk->wg_per_cu);
    return GEMM_OK;
}

int enqueue_group(const GroupPlan &plan, const GroupDesc *dev_descs, int32_t *counters, hipStream_t s) {
    if (plan.total_tiles == 0) return GEMM_OK;
    GroupedArgs G;
    G.descs = dev_descs;
    G.count = (int32_t)plan.descs.size();
    G.total_tiles = plan.total_tiles;
    G.counters = counters;
    MG_HIP(plan.gk->launch(G, plan.nwg, s));
    return GEMM_OK;
}

int alloc_counters(int32_t **out) {
    *out = nullptr;
    void *p = nullptr;
    if (hipMalloc(&p, 256) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GEMM_ENOMEM, "work-queue counters");
    }
    if (hipMemset(p, 0, 256) != hipSuccess) {
        (void)hipFree(p);
        return fail(GEMM_EHIP, "zeroing work-queue counters failed");
    }
    *out = static_cast<int32_t *>(p);
    return GEMM_OK;
}

// The work-queue counters of a stream's grouped launches (zeroed once; every
// launch leaves them at zero).
static std::mutex g_cnt_mu;
static std::map<std::pair<int, hipStream_t>, int32_t *> g_cnt;

static int stream_counters(hipStream_t s, int32_t **out) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_cnt_mu);
    int32_t *&c = g_cnt[{dev, s}];
    if (!c) {
        int rc = alloc_counters(&c);
        if (rc != GEMM_OK) return rc;
    }
    *out = c;
    return GEMM_OK;
}

// Pinned host staging of the descriptor upload: a ring of buffers per
// (device, stream), so that the host only waits for the copy issued
// kRing calls earlier and can run ahead of the device by that many calls.
// Callers on one stream take the stage's lock for the whole upload.
static const int kRing = 4;
struct HostStage {
    std::mutex mu;
    void *host[kRing] = {};
    size_t bytes[kRing] = {};
    hipEvent_t ev[kRing] = {};
    int next = 0;
};
static std::mutex g_stage_mu;
static std::map<std::pair<int, hipStream_t>, HostStage *> g_stage;

int upload_descs(const GroupPlan &plan, hipStream_t s, const GroupDesc **dev_out) {
    const size_t bytes = plan.descs.size() * sizeof(GroupDesc);
    DevBuf *db = stream_workspace(s, 1);
    int rc = db->ensure(std::max<size_t>(bytes, 256), s);
    if (rc != GEMM_OK) return rc;
    int dev = 0;
    (void)hipGetDevice(&dev);
    HostStage *st;
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        HostStage *&p = g_stage[{dev, s}];
        if (!p) p = new HostStage();
        st = p;
    }
    std::lock_guard<std::mutex> lk(st->mu);
    const int b = st->next;
    st->next = (b + 1) % kRing;
    if (st->ev[b]) MG_HIP(hipEventSynchronize(st->ev[b]));
    else MG_HIP(hipEventCreateWithFlags(&st->ev[b], hipEventDisableTiming));
    if (st->bytes[b] < bytes) {
        if (st->host[b]) MG_HIP(hipHostFree(st->host[b]));
        st->host[b] = nullptr;
        st->bytes[b] = 0;
        MG_HIP(hipHostMalloc(&st->host[b], std::max<size_t>(bytes, 4096), hipHostMallocDefault));
        st->bytes[b] = std::max<size_t>(bytes, 4096);
    }
    memcpy(st->host[b], plan.descs.data(), bytes);
    MG_HIP(hipMemcpyAsync(db->ptr, st->host[b], bytes, hipMemcpyHostToDevice, s));
    MG_HIP(hipEventRecord(st->ev[b], s));
    *dev_out = static_cast<const GroupDesc *>(db->ptr);
    return GEMM_OK;
}

// Median of `reps` event-timed runs of `run` on stream `s`, after one
// untimed run.
template <class F>
static int time_median(hipStream_t s, int reps, F run, float *ms_out) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MG_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(GEMM_EHIP, "event creation failed");
    }
    std::vector<float> ts;
    int rc = run();
    for (int r = 0; r < reps && rc == GEMM_OK; ++r) {
        (void)hipEventRecord(e0, s);
        rc = run();
        (void)hipEventRecord(e1, s);
        if (rc == GEMM_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(GEMM_EHIP, "event sync failed");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ts.push_back(ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != GEMM_OK) return rc;
    std::sort(ts.begin(), ts.end());
    *ms_out = ts[ts.size() / 2];
    return GEMM_OK;
}

struct GroupGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *descs = nullptr;
    int32_t *counters = nullptr;
};

}  // namespace mg

using namespace mg;

extern "C" {

int gemm_grouped(const gemm_problem_t *ps, int32_t count, void *stream) {
    clear_error();
    GroupPlan plan;
    int rc = build_group_plan(ps, count, plan);
    if (rc != GEMM_OK || plan.total_tiles == 0) return rc;
    hipStream_t s = (hipStream_t)stream;
    const GroupDesc *dd = nullptr;
    int32_t *cnt = nullptr;
    rc = stream_counters(s, &cnt);
    if (rc != GEMM_OK) return rc;
    std::unique_lock<std::mutex> ws_lock = lock_stream_workspaces(s);
    rc = upload_descs(plan, s, &dd);
    if (rc != GEMM_OK) return rc;
    return enqueue_group(plan, dd, cnt, s);
}

int gemm_grouped_graph_create(const gemm_problem_t *ps, int32_t count, void **graph_out) {
    clear_error();
    if (!graph_out) return fail(GEMM_EINVAL, "graph_out is NULL");
    *graph_out = nullptr;
    GroupPlan plan;
    int rc = build_group_plan(ps, count, plan);
    if (rc != GEMM_OK) return rc;
    GroupGraph *g = new GroupGraph();
    if (plan.total_tiles > 0) {
        const size_t bytes = plan.descs.size() * sizeof(GroupDesc);
        hipStream_t cs = nullptr;
        rc = alloc_counters(&g->counters);
        if (rc != GEMM_OK) {
            delete g;
            return rc;
        }
        hipError_t e = hipMalloc(&g->descs, bytes);
        if (e == hipSuccess) e = hipMemcpy(g->descs, plan.descs.data(), bytes, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            rc = enqueue_group(plan, static_cast<const GroupDesc *>(g->descs), g->counters, cs);
            hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
            if (rc == GEMM_OK && e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess && rc == GEMM_OK) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (cs) (void)hipStreamDestroy(cs);
        if (e != hipSuccess || rc != GEMM_OK) {
            if (g->exec) (void)hipGraphExecDestroy(g->exec);
            if (g->graph) (void)hipGraphDestroy(g->graph);
            if (g->descs) (void)hipFree(g->descs);
            if (g->counters) (void)hipFree(g->counters);
            delete g;
            if (rc != GEMM_OK) return rc;
            return fail(GEMM_EHIP, "graph capture failed: %s", hipGetErrorString(e));
        }
    }
    *graph_out = g;
    return GEMM_OK;
}

int gemm_tune_grouped(int32_t mode, int64_t m, int64_t n, int64_t k, void *stream) {
    clear_error();
    if (!mode_known(mode)) return fail(GEMM_EINVAL, "unknown mode %d", mode);
    if (m <= 0 || n <= 0 || k <= 0) return fail(GEMM_EINVAL, "tuning needs a non-empty product");
    if (m > 65536 || n > 65536 || k > 65536) return fail(GEMM_EUNSUPPORTED, "tuning shapes are limited to 65536");
    const GroupedKernel *gk = grouped_kernel(mode);
    if (!gk) return fail(GEMM_EUNSUPPORTED, "mode %d has no grouped kernel", mode);
    int tcount = 0;
    const KernelCfg *t = configs(mode, &tcount);
    hipStream_t s = (hipStream_t)stream;
    const int64_t es = (int64_t)elem_size(mode);
    // A batch of identical problems, enough that the option with fewer tiles
    // fills every resident-workgroup slot twice (at most 256 problems and
    // 1 GiB of operands), each with operands of its own.
    int64_t fewest = INT64_MAX;
    for (int o = 0; o < 2; ++o) {
        const KernelCfg &kc = t[gk->cfg_idx[o]];
        fewest = std::min<int64_t>(fewest, ((m + kc.bm - 1) / kc.bm) * ((n + kc.bn - 1) / kc.bn));
    }
    const int64_t slots = (int64_t)num_cus() * std::max(1, gk->wg_per_cu);
    int64_t count = std::min<int64_t>(256, std::max<int64_t>(1, (2 * slots + fewest - 1) / fewest));
    const int64_t abytes = (m * k * es + 255) / 256 * 256, bbytes = (k * n * es + 255) / 256 * 256,
                  cbytes = (m * n * 4 + 255) / 256 * 256;
    const int64_t per = abytes + bbytes + cbytes;
    while (count > 1 && count * per > ((int64_t)1 << 30)) count = (count + 1) / 2;
    uint8_t *buf = nullptr;
    void *descs = nullptr;
    int32_t *counters = nullptr;
    if (hipMalloc(&buf, (size_t)(count * per)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GEMM_ENOMEM, "grouped tuning buffers do not fit");
    }
    std::vector<gemm_problem_t> ps((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        gemm_problem_t &p = ps[(size_t)i];
        memset(&p, 0, sizeof(p));
        uint8_t *base = buf + i * per;
        p.mode = mode;
        p.m = m;
        p.n = n;
        p.k = k;
        p.A = base;
        p.lda = k;
        p.B = base + abytes;
        p.ldb = n;
        p.C = reinterpret_cast<float *>(base + abytes + bbytes);
        p.ldc = n;
        p.scale_a = p.scale_b = 1.f;
    }
    int rc = GEMM_OK;
    // non-zero operands: the clock under load depends on the data
    if (launch_fill_tuning(buf, count * per / es, (int)es, 3u, s) != hipSuccess)
        rc = fail(GEMM_EHIP, "filling the tuning operands failed");
    if (rc == GEMM_OK) rc = alloc_counters(&counters);
    float batch_ms[2] = {0.f, 0.f}, alone_ms[2] = {0.f, 0.f};
    for (int o = 0; o < 2 && rc == GEMM_OK; ++o) {
        GroupPlan plan;
        rc = build_group_plan(ps.data(), (int32_t)count, plan, o);
        if (rc != GEMM_OK) break;
        const size_t bytes = plan.descs.size() * sizeof(GroupDesc);
        if (descs) (void)hipFree(descs);
        descs = nullptr;
        if (hipMalloc(&descs, bytes) != hipSuccess ||
            hipMemcpy(descs, plan.descs.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(GEMM_EHIP, "grouped tuning descriptors");
            break;
        }
        rc = time_median(s, 7, [&] { return enqueue_group(plan, static_cast<const GroupDesc *>(descs), counters, s); },
                         &batch_ms[o]);
        if (rc != GEMM_OK) break;
        rc = time_median(s, 7, [&] { return enqueue_plain(ps[0], gk->cfg_idx[o], 1, nullptr, s); }, &alone_ms[o]);
    }
    if (rc == GEMM_OK && hipStreamSynchronize(s) != hipSuccess) rc = fail(GEMM_EHIP, "stream sync failed");
    if (descs) (void)hipFree(descs);
    if (counters) (void)hipFree(counters);
    (void)hipFree(buf);
    if (rc != GEMM_OK) return rc;
    tuner_record_grouped(mode, m, n, k, batch_ms[1] < batch_ms[0] ? 1 : 0, alone_ms[1] < alone_ms[0] ? 1 : 0);
    return GEMM_OK;
}

int gemm_grouped_info(int32_t mode, int32_t info[4]) {
    clear_error();
    if (!mode_known(mode)) return fail(GEMM_EINVAL, "unknown mode %d", mode);
    if (!info) return fail(GEMM_EINVAL, "info is NULL");
    const GroupedKernel *gk = grouped_kernel(mode);
    if (!gk) return fail(GEMM_EUNSUPPORTED, "mode %d has no grouped kernel", mode);
    info[0] = gk->cfg_idx[0];
    info[1] = gk->cfg_idx[1];
    info[2] = gk->wg_per_cu;
    info[3] = gk->lds_bytes;
    return GEMM_OK;
}

int gemm_grouped_lookup(int32_t mode, int64_t m, int64_t n, int64_t k, int32_t out[3]) {
    clear_error();
    if (!mode_known(mode)) return fail(GEMM_EINVAL, "unknown mode %d", mode);
    if (!out) return fail(GEMM_EINVAL, "out is NULL");
    if (m < 0 || n < 0 || k < 0) return fail(GEMM_EINVAL, "negative dimension");
    const GroupedKernel *gk = grouped_kernel(mode);
    if (!gk) return fail(GEMM_EUNSUPPORTED, "mode %d has no grouped kernel", mode);
    int in_batch = 0, alone = 0;
    const bool measured = tuner_grouped_choice(mode, m, n, k, &in_batch, &alone);
    out[0] = gk->cfg_idx[grouped_choose(mode, m, n, k)];
    out[1] = gk->cfg_idx[grouped_choose_alone(mode, m, n, k)];
    out[2] = measured ? 1 : 0;
    return GEMM_OK;
}

int gemm_grouped_plan(const gemm_problem_t *ps, int32_t count, int32_t *cfg_out) {
    clear_error();
    if (count > 0 && !cfg_out) return fail(GEMM_EINVAL, "cfg_out is NULL");
    GroupPlan plan;
    int rc = build_group_plan(ps, count, plan);
    if (rc != GEMM_OK) return rc;
    for (int i = 0; i < count; ++i) cfg_out[i] = -1;
    for (size_t j = 0; j < plan.descs.size(); ++j) cfg_out[plan.src[j]] = plan.gk->cfg_idx[plan.descs[j].cfg];
    return GEMM_OK;
}

int gemm_graph_launch(void *graph, void *stream) {
    clear_error();
    if (!graph) return fail(GEMM_EINVAL, "graph is NULL");
    GroupGraph *g = static_cast<GroupGraph *>(graph);
    if (!g->exec) return GEMM_OK;  // an empty group
    MG_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return GEMM_OK;
}

int gemm_graph_destroy(void *graph) {
    clear_error();
    if (!graph) return fail(GEMM_EINVAL, "graph is NULL");
    GroupGraph *g = static_cast<GroupGraph *>(graph);
    if (g->exec) {
        // replays may still be running on some stream: wait before freeing
        (void)hipDeviceSynchronize();
        (void)hipGraphExecDestroy(g->exec);
    }
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->descs) (void)hipFree(g->descs);
    if (g->counters) (void)hipFree(g->counters);
    delete g;
    return GEMM_OK;
}

}  // extern "C"
