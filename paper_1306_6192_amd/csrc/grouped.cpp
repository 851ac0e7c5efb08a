// Grouped product: many independent problems in one persistent launch, and
// its capture into a HIP graph.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <queue>
#include <vector>

#include "grouped.hpp"

namespace mg {

// Default efficiency of the small tile relative to the large one in the
// cost model, where the tuning table has no measured value for the mode.
static const double kDefaultSmallEff = 0.6;

// Cost model of the choice between the grouped kernel's two tile
// configurations: the padded tile area, weighed by the small tile's lower
// sustained rate (`small_eff`); alone, in rounds of resident workgroups.
static int grouped_model(int mode, int64_t m, int64_t n, bool alone, double small_eff) {
    const GroupedKernel *gk = grouped_kernel(mode);
    int count = 0;
    const KernelCfg *t = configs(mode, &count);
    double best = 1e300;
    int pick = 0;
    for (int c = 0; c < 2; ++c) {
        const KernelCfg &kc = t[alone ? gk->alone_idx[c] : gk->cfg_idx[c]];
        const double tiles = (double)((m + kc.bm - 1) / kc.bm) * (double)((n + kc.bn - 1) / kc.bn);
        const double eff = (kc.bm * kc.bn >= 16384) ? 1.0 : small_eff;
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

// Set by gemm_tune_grouped_mix while it plans its candidates.
static thread_local double t_eff_override = -1.0;
static thread_local int t_variant_override = -1;

static double small_eff_of(int mode) {
    if (t_eff_override > 0) return t_eff_override;
    const double e = tuner_grouped_eff(mode);
    return e > 0 ? e : kDefaultSmallEff;
}

// In a batch: the cost model with the small-tile efficiency the autotuner
// measured on a mixed batch (gemm_tune_grouped_mix).  Per-shape choices
// measured on batches of one shape chose the small tile where a mixed batch
// runs faster on the large one, so the batch choice is the calibrated model.
int grouped_choose(int mode, int64_t m, int64_t n, int64_t k) {
    (void)k;
    return grouped_model(mode, m, n, false, small_eff_of(mode));
}

// The same choice for a problem launched on its own (a serving batch of one):
// the two tiles give the same bits, so the one measured to finish first for
// the shape's bucket is taken, else the model's.
int grouped_choose_alone(int mode, int64_t m, int64_t n, int64_t k) {
    int alone = 0;
    if (tuner_grouped_alone(mode, m, n, k, &alone)) return alone;
    return grouped_model(mode, m, n, true, small_eff_of(mode));
}

// Variant v (0 or 1) of the mode's grouped kernel (null for another v).
static const GroupedKernel *grouped_variant(int mode, int v) {
    if (v < 0 || v > 1) return nullptr;
    return mode == GEMM_MODE_F32 ? f32_grouped(v) : lp_grouped(mode, v);
}

// The mode's grouped kernel: the variant the autotuner measured fastest on a
// mixed batch (gemm_tune_grouped_mix), else (also for a variant this mode
// does not have) variant 0.
static int grouped_variant_of(int mode) {
    const int v = t_variant_override >= 0 ? t_variant_override : tuner_grouped_variant(mode);
    return grouped_variant(mode, v) ? v : 0;
}

const GroupedKernel *grouped_kernel(int mode) { return grouped_variant(mode, grouped_variant_of(mode)); }

// Cost of one output tile in the static schedule, in microseconds of one
// workgroup: its k-tiles, each bounded by the operand bytes it moves (16 KB
// at the workgroup's share of HBM bandwidth) or by its MFMA work at the
// mode's rate (whichever is longer), plus the accumulator store and the
// per-tile overhead.
static double tile_cost_us(int mode, const KernelCfg &kc, int64_t k, int wg_per_cu) {
    const double cus = (double)num_cus();
    const double slots = cus * std::max(1, wg_per_cu);
    const double bw = 8.0e6 / slots;                    // bytes per microsecond per workgroup
    double peak;                                        // flop per microsecond per workgroup
    switch (mode) {
        case GEMM_MODE_F32: peak = 157.3e6; break;
        case GEMM_MODE_F8E4M3: peak = 5000.0e6; break;
        case GEMM_MODE_F32_SPLIT_BF16X3: peak = 2500.0e6 / 3.0; break;
        default: peak = 2500.0e6; break;
    }
    peak /= slots;
    const int64_t nkt = std::max<int64_t>(1, (k + kc.bk - 1) / kc.bk);
    const double es = (double)elem_size(mode);
    const double kt_bytes = (double)(kc.bm + kc.bn) * kc.bk * es;
    const double kt_flops = 2.0 * kc.bm * kc.bn * kc.bk;
    const double per_kt = std::max(kt_bytes / bw, kt_flops / peak);
    return (double)nkt * per_kt + (double)kc.bm * kc.bn * 4.0 / bw + 1.0;
}

// Static schedule of the grouped launch.  Workgroup w runs on XCD w % 8 (the
// dispatcher deals workgroups out round-robin), and each XCD has an L2 of its
// own, so the tiles of a problem are kept on one XCD where the balance
// allows: problems are placed whole, costliest first, on the least-loaded
// XCD, except those costing more than a quarter of an XCD's fair share,
// whose tiles are placed one by one.  Within an XCD, tiles are dealt
// costliest first over its workgroups in snake order.  The schedule depends
// on the problem list only.
// Tile t of problem p (in the grouped row order of the plain launch: groups
// of 8 tile rows, column by column within a group).
static GroupTile tile_entry(const GroupPlan &plan, const KernelCfg *t, int p, int tile) {
    const GroupDesc &d = plan.descs[p];
    const KernelCfg &kc = t[plan.gk->cfg_idx[d.cfg]];
    const int group_m = 8;
    const int per_group = group_m * d.P.tiles_n;
    const int g = tile / per_group;
    const int first_m = g * group_m;
    const int gsz = std::min(d.P.tiles_m - first_m, group_m);
    const int in = tile - g * per_group;
    GroupTile e;
    e.p = p;
    e.m0 = (first_m + in % gsz) * kc.bm;
    e.n0 = (in / gsz) * kc.bn;
    e.nkt = std::max(1, (d.P.k + kc.bk - 1) / kc.bk);
    return e;
}

static void build_schedule(GroupPlan &plan, const std::vector<double> &prob_cost,
                           const std::vector<int> &prob_tiles) {
    int tcount = 0;
    const KernelCfg *tab = configs(plan.mode, &tcount);
    const int np = (int)plan.descs.size();
    const int nwg = plan.nwg;
    const int nx = std::min(GEMM_NUM_XCD, nwg);
    typedef std::pair<double, int> L;   // (load per resident workgroup, index)
    // XCD x hosts workgroups x, x + 8, ... below nwg
    std::vector<double> xcap(nx, 0.0);
    for (int w = 0; w < nwg; ++w) xcap[w % GEMM_NUM_XCD] += 1.0;
    std::priority_queue<L, std::vector<L>, std::greater<L>> xheap;
    for (int x = 0; x < nx; ++x) xheap.push({0.0, x});
    double total = 0.0;
    for (int p = 0; p < np; ++p) total += prob_cost[p] * prob_tiles[p];
    std::vector<int> order(np);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return prob_cost[a] * prob_tiles[a] > prob_cost[b] * prob_tiles[b];
    });
    // tiles grouped by XCD: (problem, tile) in placement order
    std::vector<std::vector<std::pair<int, int>>> xt(nx);
    const double split_above = 0.25 * total / nx;
    auto place = [&](int p, int t0, int t1, double c) {
        L top = xheap.top();
        xheap.pop();
        for (int t = t0; t < t1; ++t) xt[top.second].push_back({p, t});
        top.first += c * (t1 - t0) / xcap[top.second];
        xheap.push(top);
    };
    for (int p : order) {
        const int nt = prob_tiles[p];
        if (prob_cost[p] * nt > split_above)
            for (int t = 0; t < nt; ++t) place(p, t, t + 1, prob_cost[p]);
        else
            place(p, 0, nt, prob_cost[p]);
    }
    // within an XCD: costliest first, dealt over the XCD's workgroups in
    // snake order (w0 .. wn, wn .. w0, ...), which balances runs of equal
    // costs like the longest-processing-time rule at linear cost
    std::vector<int> wg_of;
    std::vector<std::pair<int, int>> flat;
    flat.reserve(plan.total_tiles);
    wg_of.reserve(plan.total_tiles);
    std::vector<int32_t> count(nwg, 0);
    for (int x = 0; x < nx; ++x) {
        auto &v = xt[x];
        std::stable_sort(v.begin(), v.end(), [&](const std::pair<int, int> &a, const std::pair<int, int> &b) {
            return prob_cost[a.first] > prob_cost[b.first];
        });
        const int nw = (nwg - x + GEMM_NUM_XCD - 1) / GEMM_NUM_XCD;   // workgroups x, x + 8, ...
        for (size_t i = 0; i < v.size(); ++i) {
            const int round = (int)(i / nw), j = (int)(i % nw);
            const int w = x + GEMM_NUM_XCD * ((round & 1) ? nw - 1 - j : j);
            flat.push_back(v[i]);
            wg_of.push_back(w);
            ++count[w];
        }
    }
    // counting sort by workgroup (placement order kept within a workgroup)
    plan.wg_first.assign(nwg + 1, 0);
    for (int w = 0; w < nwg; ++w) plan.wg_first[w + 1] = plan.wg_first[w] + count[w];
    std::vector<int32_t> pos(plan.wg_first.begin(), plan.wg_first.end() - 1);
    plan.tiles.resize(flat.size());
    for (size_t i = 0; i < flat.size(); ++i)
        plan.tiles[pos[wg_of[i]]++] = tile_entry(plan, tab, flat[i].first, flat[i].second);
}

int build_group_plan(const gemm_problem_t *ps, int32_t count, GroupPlan &plan, int force) {
    if (count < 0) return fail(GEMM_EINVAL, "negative problem count");
    if (count > 0 && !ps) return fail(GEMM_EINVAL, "problem array is NULL");
    plan.descs.clear();
    plan.src.clear();
    plan.tiles.clear();
    plan.wg_first.clear();
    plan.total_tiles = 0;
    plan.nwg = 0;
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
    // A launch whose chosen tiles would not fill every resident-workgroup
    // slot runs every problem on the smaller tile instead (the tile does not
    // change the bits): a handful of mid-size problems then spread over the
    // chip rather than over a fraction of it.
    const int small = t[plan.gk->cfg_idx[1]].bm * t[plan.gk->cfg_idx[1]].bn <
                              t[plan.gk->cfg_idx[0]].bm * t[plan.gk->cfg_idx[0]].bn
                          ? 1
                          : 0;
    int64_t chosen_tiles = 0;
    std::vector<int8_t> choice(count, 0);
    for (int i = 0; i < count; ++i) {
        const gemm_problem_t &p = ps[i];
        if (p.m == 0 || p.n == 0) continue;
        choice[i] = (int8_t)(force >= 0 ? force : grouped_choose(p.mode, p.m, p.n, p.k));
        const KernelCfg &kc = t[plan.gk->cfg_idx[choice[i]]];
        chosen_tiles += ((p.m + kc.bm - 1) / kc.bm) * ((p.n + kc.bn - 1) / kc.bn);
    }
    const int64_t slots = (int64_t)num_cus() * plan.gk->wg_per_cu;
    const bool underfilled = force < 0 && chosen_tiles < slots;
    std::vector<double> cost;
    std::vector<int> ntiles;
    cost.reserve(count);
    ntiles.reserve(count);
    plan.descs.reserve(count);
    plan.src.reserve(count);
    int64_t total = 0;
    for (int i = 0; i < count; ++i) {
        const gemm_problem_t &p = ps[i];
        if (p.m == 0 || p.n == 0) continue;
        GroupDesc d;
        memset(&d, 0, sizeof(d));
        d.cfg = underfilled ? small : choice[i];
        const KernelCfg &kc = t[plan.gk->cfg_idx[d.cfg]];
        d.P = make_launch(p, kc, 1).P;
        const int64_t nt = (int64_t)d.P.tiles_m * d.P.tiles_n;
        total += nt;
        if (total > INT32_MAX) return fail(GEMM_EUNSUPPORTED, "grouped launch above 2^31 tiles");
        plan.descs.push_back(d);
        plan.src.push_back(i);
        cost.push_back(tile_cost_us(plan.mode, kc, p.k, plan.gk->wg_per_cu));
        ntiles.push_back((int)nt);
    }
    plan.total_tiles = (int)total;
    plan.nwg = (int)std::min<int64_t>(total, slots);
    if (total > 0) build_schedule(plan, cost, ntiles);
    return GEMM_OK;
}

// The plan's device image: descriptors, then the workgroups' list offsets,
// then the tile lists, each part 256-byte aligned.
static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

size_t plan_image_bytes(const GroupPlan &plan) {
    return align256(plan.descs.size() * sizeof(GroupDesc)) + align256(plan.wg_first.size() * sizeof(int32_t)) +
           align256(plan.tiles.size() * sizeof(GroupTile));
}

void plan_image_write(const GroupPlan &plan, void *dst) {
    uint8_t *d = static_cast<uint8_t *>(dst);
    memcpy(d, plan.descs.data(), plan.descs.size() * sizeof(GroupDesc));
    d += align256(plan.descs.size() * sizeof(GroupDesc));
    memcpy(d, plan.wg_first.data(), plan.wg_first.size() * sizeof(int32_t));
    d += align256(plan.wg_first.size() * sizeof(int32_t));
    memcpy(d, plan.tiles.data(), plan.tiles.size() * sizeof(GroupTile));
}

int enqueue_group(const GroupPlan &plan, const void *dev_image, hipStream_t s) {
    if (plan.total_tiles == 0) return GEMM_OK;
    const uint8_t *d = static_cast<const uint8_t *>(dev_image);
    GroupedArgs G;
    G.descs = reinterpret_cast<const GroupDesc *>(d);
    d += align256(plan.descs.size() * sizeof(GroupDesc));
    G.wg_first = reinterpret_cast<const int32_t *>(d);
    d += align256(plan.wg_first.size() * sizeof(int32_t));
    G.tiles = reinterpret_cast<const GroupTile *>(d);
    MG_HIP(plan.gk->launch(G, plan.nwg, s));
    return GEMM_OK;
}

// Pinned host staging of the plan upload: a ring of buffers per (device,
// stream), so that the host only waits for the copy issued kRing calls
// earlier and can run ahead of the device by that many calls.  Callers on
// one stream take the stage's lock for the whole upload.
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

int upload_plan(const GroupPlan &plan, hipStream_t s, const void **dev_out) {
    const size_t bytes = plan_image_bytes(plan);
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
    plan_image_write(plan, st->host[b]);
    MG_HIP(hipMemcpyAsync(db->ptr, st->host[b], bytes, hipMemcpyHostToDevice, s));
    MG_HIP(hipEventRecord(st->ev[b], s));
    *dev_out = db->ptr;
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
    void *image = nullptr;   // the plan's device image (graph-owned)
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
    const void *img = nullptr;
    std::unique_lock<std::mutex> ws_lock = lock_stream_workspaces(s);
    rc = upload_plan(plan, s, &img);
    if (rc != GEMM_OK) return rc;
    return enqueue_group(plan, img, s);
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
        const size_t bytes = plan_image_bytes(plan);
        std::vector<uint8_t> host(bytes);
        plan_image_write(plan, host.data());
        hipStream_t cs = nullptr;
        hipError_t e = hipMalloc(&g->image, bytes);
        if (e == hipSuccess) e = hipMemcpy(g->image, host.data(), bytes, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            rc = enqueue_group(plan, g->image, cs);
            hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
            if (rc == GEMM_OK && e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess && rc == GEMM_OK) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (cs) (void)hipStreamDestroy(cs);
        if (e != hipSuccess || rc != GEMM_OK) {
            if (g->exec) (void)hipGraphExecDestroy(g->exec);
            if (g->graph) (void)hipGraphDestroy(g->graph);
            if (g->image) (void)hipFree(g->image);
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
    hipStream_t s = (hipStream_t)stream;
    const int64_t es = (int64_t)elem_size(mode);
    const int64_t abytes = (m * k * es + 255) / 256 * 256, bbytes = (k * n * es + 255) / 256 * 256,
                  cbytes = (m * n * 4 + 255) / 256 * 256;
    uint8_t *buf = nullptr;
    if (hipMalloc(&buf, (size_t)(abytes + bbytes + cbytes)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GEMM_ENOMEM, "grouped tuning buffers do not fit");
    }
    gemm_problem_t p;
    memset(&p, 0, sizeof(p));
    p.mode = mode;
    p.m = m;
    p.n = n;
    p.k = k;
    p.A = buf;
    p.lda = k;
    p.B = buf + abytes;
    p.ldb = n;
    p.C = reinterpret_cast<float *>(buf + abytes + bbytes);
    p.ldc = n;
    p.scale_a = p.scale_b = 1.f;
    int rc = GEMM_OK;
    // non-zero operands: the clock under load depends on the data
    if (launch_fill_tuning(buf, (abytes + bbytes + cbytes) / es, (int)es, 3u, s) != hipSuccess)
        rc = fail(GEMM_EHIP, "filling the tuning operands failed");
    float alone_ms[2] = {0.f, 0.f};
    for (int o = 0; o < 2 && rc == GEMM_OK; ++o)
        rc = time_median(s, 7, [&] { return enqueue_plain(p, gk->alone_idx[o], 1, nullptr, s); }, &alone_ms[o]);
    if (rc == GEMM_OK && hipStreamSynchronize(s) != hipSuccess) rc = fail(GEMM_EHIP, "stream sync failed");
    (void)hipFree(buf);
    if (rc != GEMM_OK) return rc;
    tuner_record_grouped(mode, m, n, k, alone_ms[1] < alone_ms[0] ? 1 : 0);
    return GEMM_OK;
}

int gemm_tune_grouped_mix(const gemm_problem_t *ps, int32_t count, void *stream) {
    clear_error();
    if (count <= 0 || !ps) return fail(GEMM_EINVAL, "tuning needs a non-empty problem list");
    GroupPlan check;
    int rc = build_group_plan(ps, count, check);
    if (rc != GEMM_OK) return rc;
    if (check.total_tiles == 0) return fail(GEMM_EINVAL, "tuning needs a non-empty product");
    const int mode = check.mode;
    hipStream_t s = (hipStream_t)stream;
    // candidates: variant 0 (one tile), and variant 1 (two tiles) under each
    // candidate small-tile efficiency; the first (variant 0 at the default
    // efficiency) is kept unless another is more than 1 % faster
    static const double grid[] = {0.3, 0.45, kDefaultSmallEff, 0.75, 0.9, 1.0, 1.25, 1.6};
    const int ng = (int)(sizeof(grid) / sizeof(grid[0]));
    struct Cand {
        int variant;
        double eff;
    };
    std::vector<Cand> cands{{0, kDefaultSmallEff}};
    for (int g = 0; g < ng; ++g) cands.push_back({1, grid[g]});
    const int nc = (int)cands.size();
    std::vector<std::pair<int, std::vector<int32_t>>> seen;   // (variant, tile choices)
    std::vector<int> plan_of(nc, -1);
    std::vector<float> best_ms;
    void *image = nullptr;
    size_t image_bytes = 0;
    for (int pass = 0; pass < 2 && rc == GEMM_OK; ++pass) {
        for (int c = 0; c < nc && rc == GEMM_OK; ++c) {
            t_variant_override = cands[c].variant;
            t_eff_override = cands[c].eff;
            GroupPlan plan;
            rc = build_group_plan(ps, count, plan);
            t_eff_override = -1.0;
            t_variant_override = -1;
            if (rc != GEMM_OK) break;
            // candidates that give the same kernel and tile choices share one timing
            std::vector<int32_t> choice(plan.descs.size());
            for (size_t i = 0; i < plan.descs.size(); ++i) choice[i] = plan.descs[i].cfg;
            int id = -1;
            for (size_t j = 0; j < seen.size(); ++j)
                if (seen[j].first == cands[c].variant && seen[j].second == choice) id = (int)j;
            if (id < 0) {
                id = (int)seen.size();
                seen.emplace_back(cands[c].variant, choice);
                best_ms.push_back(1e30f);
            }
            plan_of[c] = id;
            const size_t bytes = plan_image_bytes(plan);
            std::vector<uint8_t> host(bytes);
            plan_image_write(plan, host.data());
            // the previous candidate's launches have completed (time_median
            // synchronises), so its image may be overwritten or replaced
            if (bytes > image_bytes) {
                if (image) (void)hipFree(image);
                image = nullptr;
                image_bytes = 0;
                if (hipMalloc(&image, bytes) != hipSuccess) {
                    (void)hipGetLastError();
                    rc = fail(GEMM_EHIP, "grouped tuning descriptors");
                    break;
                }
                image_bytes = bytes;
            }
            if (hipMemcpy(image, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
                (void)hipGetLastError();
                rc = fail(GEMM_EHIP, "grouped tuning descriptors");
                break;
            }
            float ms = 0.f;
            rc = time_median(s, 7, [&] { return enqueue_group(plan, image, s); }, &ms);
            if (rc == GEMM_OK) best_ms[id] = std::min(best_ms[id], ms);
        }
    }
    t_eff_override = -1.0;
    t_variant_override = -1;
    if (rc == GEMM_OK && hipStreamSynchronize(s) != hipSuccess) rc = fail(GEMM_EHIP, "stream sync failed");
    if (image) (void)hipFree(image);
    if (rc != GEMM_OK) return rc;
    int pick = 0;
    for (int c = 1; c < nc; ++c)
        if (best_ms[plan_of[c]] < 0.99f * best_ms[plan_of[pick]]) pick = c;
    tuner_record_grouped_eff(mode, cands[pick].eff, cands[pick].variant);
    return GEMM_OK;
}

int gemm_grouped_info(int32_t mode, int32_t info[7]) {
    clear_error();
    if (!mode_known(mode)) return fail(GEMM_EINVAL, "unknown mode %d", mode);
    if (!info) return fail(GEMM_EINVAL, "info is NULL");
    const GroupedKernel *gk = grouped_kernel(mode);
    if (!gk) return fail(GEMM_EUNSUPPORTED, "mode %d has no grouped kernel", mode);
    info[0] = gk->cfg_idx[0];
    info[1] = gk->cfg_idx[1];
    info[2] = gk->wg_per_cu;
    info[3] = gk->lds_bytes;
    info[4] = gk->alone_idx[0];
    info[5] = gk->alone_idx[1];
    info[6] = grouped_variant_of(mode);
    return GEMM_OK;
}

int gemm_grouped_lookup(int32_t mode, int64_t m, int64_t n, int64_t k, int32_t out[3]) {
    clear_error();
    if (!mode_known(mode)) return fail(GEMM_EINVAL, "unknown mode %d", mode);
    if (!out) return fail(GEMM_EINVAL, "out is NULL");
    if (m < 0 || n < 0 || k < 0) return fail(GEMM_EINVAL, "negative dimension");
    const GroupedKernel *gk = grouped_kernel(mode);
    if (!gk) return fail(GEMM_EUNSUPPORTED, "mode %d has no grouped kernel", mode);
    int alone = 0;
    const bool measured = tuner_grouped_alone(mode, m, n, k, &alone) && tuner_grouped_eff(mode) > 0;
    out[0] = gk->cfg_idx[grouped_choose(mode, m, n, k)];
    out[1] = gk->alone_idx[grouped_choose_alone(mode, m, n, k)];
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

int gemm_grouped_schedule(const gemm_problem_t *ps, int32_t count, int32_t *nwg_out, int32_t *ntiles_out,
                          int32_t *wg_first, int32_t *tile_problem, int32_t *tile_m0, int32_t *tile_n0) {
    clear_error();
    if (!nwg_out || !ntiles_out) return fail(GEMM_EINVAL, "nwg_out or ntiles_out is NULL");
    GroupPlan plan;
    int rc = build_group_plan(ps, count, plan);
    if (rc != GEMM_OK) return rc;
    *nwg_out = plan.nwg;
    *ntiles_out = plan.total_tiles;
    if (wg_first)
        for (int w = 0; w <= plan.nwg && plan.nwg > 0; ++w) wg_first[w] = plan.wg_first[w];
    for (int i = 0; i < plan.total_tiles; ++i) {
        const GroupTile &e = plan.tiles[i];
        if (tile_problem) tile_problem[i] = plan.src[e.p];
        if (tile_m0) tile_m0[i] = e.m0;
        if (tile_n0) tile_n0[i] = e.n0;
    }
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
    if (g->image) (void)hipFree(g->image);
    delete g;
    return GEMM_OK;
}

}  // extern "C"
