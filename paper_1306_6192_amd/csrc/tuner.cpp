// Tile-configuration autotuner: tables of (config, split-K) choices for plain
// launches and of tile choices for grouped launches, filled by measurement on
// the device (gemm_tune, gemm_tune_bucket, gemm_tune_grouped) and consulted
// before a cost model.  Plain choices are keyed by the exact (mode, m, n, k)
// or, failing that, by its log2 bucket (floor(log2) of each dimension), so
// shapes never measured still get a measured choice of a neighbouring shape;
// grouped choices are keyed by bucket.  Every choice depends on (mode, m, n,
// k) only, never on load, so a shape gets the same configuration -- and
// therefore the same summation order -- on every path.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "host.hpp"

namespace mg {

typedef std::tuple<int, int64_t, int64_t, int64_t> Key;
typedef std::tuple<int, int, int, int> BKey;   // mode, log2 buckets of m, n, k

static std::mutex g_mu;
static std::map<Key, std::pair<int, int>> g_table;          // exact shape -> (cfg, split)
static std::map<BKey, std::pair<int, int>> g_plain_bucket;  // bucket -> (cfg, split)
static std::map<BKey, int> g_grouped;                       // bucket -> option alone
static double g_grouped_eff[GEMM_NUM_MODES] = {-1, -1, -1, -1, -1};   // small-tile efficiency (< 0: unset)
static int g_grouped_variant[GEMM_NUM_MODES] = {-1, -1, -1, -1, -1};  // grouped kernel variant (< 0: unset)
static bool g_env_loaded = false;

int dim_bucket(int64_t d) {
    int b = 0;
    while (d > 1) {
        d >>= 1;
        ++b;
    }
    return b;
}

static BKey bucket_of(int mode, int64_t m, int64_t n, int64_t k) {
    return BKey(mode, dim_bucket(m), dim_bucket(n), dim_bucket(k));
}

static int load_file_locked(const char *path);

// Relative sustained efficiency of a workgroup tile (larger tiles reuse each
// staged operand more often and hide the per-k-tile barrier better).
static double tile_eff(const KernelCfg &kc) {
    const double area = (double)kc.bm * kc.bn;
    if (area >= 65536) return 1.00;
    if (area >= 32768) return 0.92;
    if (area >= 16384) return 0.82;
    if (area >= 8192) return 0.62;
    return 0.45;
}

void heuristic_choose(int mode, int64_t m, int64_t n, int64_t k, int *cfg_out, int *split_out) {
    int count = 0;
    const KernelCfg *t = configs(mode, &count);
    *cfg_out = 0;
    *split_out = 1;
    if (!t || count == 0 || m == 0 || n == 0 || k == 0) return;
    const double cus = (double)num_cus();
    double best = 1e300;
    for (int c = 0; c < count; ++c) {
        const KernelCfg &kc = t[c];
        // chunked (asynchronous-copy) tiles need k and n in whole 16-byte
        // chunks; where they apply they sustain 1.4x (16-bit) to 3.5x (FP8),
        // 1.1x (FP32) and 1.15-1.2x (binary64, complex) the register-staged
        // tile's rate at 8192^3 (measured; the complex 128x128 one beats the
        // register-staged 256x128 one although tile_eff favours the latter)
        if (kc.chunk && (k % kc.chunk || n % kc.chunk)) continue;
        if (kc.presplit && !presplit_shape_ok(n, k)) continue;
        // the pre-split split-BF16x3 path runs at about 1.75x the register-
        // staged split tile at 8192^3 (its operands are split once, not once
        // per output tile)
        double bonus = kc.presplit ? 1.75 : 1.0;
        if (kc.chunk) bonus = mode == GEMM_MODE_F32 ? 1.1 : (mode == GEMM_MODE_F64 || mode == GEMM_MODE_C32) ? 1.15 : 1.7;
        const int64_t tiles = ((m + kc.bm - 1) / kc.bm) * ((n + kc.bn - 1) / kc.bn);
        const int64_t nkt = (k + split_grain(mode) - 1) / split_grain(mode) * (split_grain(mode) / kc.bk);
        // the binary64 and complex families have no split-K
        const int max_split = mode < GEMM_NUM_MODES ? 16 : 1;
        for (int split = 1; split <= max_split; split *= 2) {
            if (split > 1 && nkt / split < 4) break;
            const int64_t per = (nkt + split - 1) / split;
            const int64_t wgs = tiles * split;
            const double slots = cus * std::max(1, kc.wg_per_cu);
            const double rounds = std::ceil((double)wgs / slots);
            // time ~ rounds * (work of one CU slot-set) / efficiency
            const double per_round = (double)std::max(1, kc.wg_per_cu) * kc.bm * kc.bn * (double)(per * kc.bk);
            double cost = rounds * per_round / (tile_eff(kc) * bonus);
            // split-K pays for writing and re-reading the partial slabs
            if (split > 1) cost += (double)(split + 1) * (double)m * n * 64.0 / cus;
            // a launch that cannot reach every CU also leaves HBM bandwidth idle
            if ((double)wgs < cus) cost *= 1.0 + 0.25 * (1.0 - (double)wgs / cus);
            if (cost < best * 0.999) {
                best = cost;
                *cfg_out = c;
                *split_out = split;
            }
        }
    }
}

static void load_env_locked() {
    if (g_env_loaded) return;
    g_env_loaded = true;
    const char *env = getenv("MI355GEMM_TUNE_FILE");
    if (env && *env) (void)load_file_locked(env);
}

void tuner_choose(int mode, int64_t m, int64_t n, int64_t k, int *cfg, int *split) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        load_env_locked();
        auto it = g_table.find(Key(mode, m, n, k));
        if (it != g_table.end()) {
            *cfg = it->second.first;
            *split = it->second.second;
            return;
        }
        auto ib = g_plain_bucket.find(bucket_of(mode, m, n, k));
        if (ib != g_plain_bucket.end()) {
            *cfg = ib->second.first;
            *split = ib->second.second;
            return;
        }
    }
    heuristic_choose(mode, m, n, k, cfg, split);
}

bool tuner_grouped_alone(int mode, int64_t m, int64_t n, int64_t k, int *alone) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_env_locked();
    auto it = g_grouped.find(bucket_of(mode, m, n, k));
    if (it == g_grouped.end()) return false;
    *alone = it->second;
    return true;
}

void tuner_record_grouped(int mode, int64_t m, int64_t n, int64_t k, int alone) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_grouped[bucket_of(mode, m, n, k)] = alone;
}

double tuner_grouped_eff(int mode) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_env_locked();
    return mode_known(mode) ? g_grouped_eff[mode] : -1.0;
}

void tuner_record_grouped_eff(int mode, double eff, int variant) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!mode_known(mode)) return;
    g_grouped_eff[mode] = eff;
    g_grouped_variant[mode] = variant;
}

int tuner_grouped_variant(int mode) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_env_locked();
    return mode_known(mode) && g_grouped_variant[mode] >= 0 ? g_grouped_variant[mode] : 0;
}

// One JSON object per line, in one of four forms (the forms gemm_tuner_save
// writes; lines in any other form are skipped):
//   {"mode": M, "m": m, "n": n, "k": k, "cfg": C, "split": S}
//   {"bucket": "plain", "mode": M, "bm": a, "bn": b, "bk": c, "cfg": C, "split": S}
//   {"bucket": "grouped", "mode": M, "bm": a, "bn": b, "bk": c, "alone": U}
//   {"grouped_eff": M, "eff": E, "variant": V}  (", variant" optional: 0)
static int load_file_locked(const char *path) {
    FILE *f = fopen(path, "r");
    if (!f) return fail(GEMM_ENOTFOUND, "cannot open tuning file %s", path);
    char line[512];
    int n_ok = 0;
    while (fgets(line, sizeof(line), f)) {
        int mode, cfg, split, bm, bn, bk;
        long long m, n, k;
        int count = 0;
        if (sscanf(line, " {\"mode\": %d, \"m\": %lld, \"n\": %lld, \"k\": %lld, \"cfg\": %d, \"split\": %d",
                   &mode, &m, &n, &k, &cfg, &split) == 6) {
            if (!mode_known(mode)) continue;
            configs(mode, &count);
            if (cfg >= 0 && cfg < count && split >= 1) {
                g_table[Key(mode, m, n, k)] = {cfg, split};
                ++n_ok;
            }
        } else if (sscanf(line,
                          " {\"bucket\": \"plain\", \"mode\": %d, \"bm\": %d, \"bn\": %d, \"bk\": %d, "
                          "\"cfg\": %d, \"split\": %d",
                          &mode, &bm, &bn, &bk, &cfg, &split) == 6) {
            if (!mode_known(mode)) continue;
            configs(mode, &count);
            if (cfg >= 0 && cfg < count && split >= 1) {
                g_plain_bucket[BKey(mode, bm, bn, bk)] = {cfg, split};
                ++n_ok;
            }
        } else if (sscanf(line,
                          " {\"bucket\": \"grouped\", \"mode\": %d, \"bm\": %d, \"bn\": %d, \"bk\": %d, "
                          "\"alone\": %d",
                          &mode, &bm, &bn, &bk, &cfg) == 5 ||
                   sscanf(line,
                          " {\"bucket\": \"grouped\", \"mode\": %d, \"bm\": %d, \"bn\": %d, \"bk\": %d, "
                          "\"tile\": %d, \"alone\": %d",
                          &mode, &bm, &bn, &bk, &split, &cfg) == 6) {
            // (the second form also carries an in-batch tile, which the
            // calibrated cost model now decides; only the alone choice is kept)
            if (!mode_known(mode) || cfg < 0 || cfg > 1) continue;
            g_grouped[BKey(mode, bm, bn, bk)] = cfg;
            ++n_ok;
        } else {
            double eff = 0;
            int variant = 0;
            const int got = sscanf(line, " {\"grouped_eff\": %d, \"eff\": %lf, \"variant\": %d", &mode, &eff,
                                   &variant);
            if (got >= 2 && mode_known(mode) && eff > 0 && eff <= 4 && variant >= 0 && variant <= 1) {
                g_grouped_eff[mode] = eff;
                g_grouped_variant[mode] = got == 3 ? variant : 0;
                ++n_ok;
            }
        }
    }
    fclose(f);
    return n_ok;
}

// Time one (cfg, split) choice: median of `reps` event-timed launches.
static int time_choice(const gemm_problem_t &p, int cfg, int split, void *ws, hipStream_t s, float *ms_out) {
    hipEvent_t e0, e1;
    MG_HIP(hipEventCreate(&e0));
    MG_HIP(hipEventCreate(&e1));
    const int reps = 5;
    float ts[reps];
    int rc = enqueue_plain(p, cfg, split, ws, s);  // warm-up
    for (int r = 0; r < reps && rc == GEMM_OK; ++r) {
        (void)hipEventRecord(e0, s);
        rc = enqueue_plain(p, cfg, split, ws, s);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) rc = fail(GEMM_EHIP, "event sync failed");
        (void)hipEventElapsedTime(&ts[r], e0, e1);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != GEMM_OK) return rc;
    std::sort(ts, ts + reps);
    *ms_out = ts[reps / 2];
    return GEMM_OK;
}

}  // namespace mg

using namespace mg;

extern "C" {

int gemm_tuner_lookup(int32_t mode, int64_t m, int64_t n, int64_t k, int32_t *cfg, int32_t *split_k) {
    clear_error();
    if (!mode_known(mode)) return fail(GEMM_EINVAL, "unknown mode %d", mode);
    if (!cfg || !split_k) return fail(GEMM_EINVAL, "NULL output");
    if (m < 0 || n < 0 || k < 0) return fail(GEMM_EINVAL, "negative dimension");
    int c = 0, s = 1;
    tuner_choose(mode, m, n, k, &c, &s);
    *cfg = c;
    *split_k = s;
    return GEMM_OK;
}

int gemm_tuner_load(const char *path) {
    clear_error();
    if (!path) return fail(GEMM_EINVAL, "path is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    const int rc = load_file_locked(path);
    return rc < 0 ? rc : GEMM_OK;
}

int gemm_tuner_save(const char *path) {
    clear_error();
    if (!path) return fail(GEMM_EINVAL, "path is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    FILE *f = fopen(path, "w");
    if (!f) return fail(GEMM_ENOTFOUND, "cannot write %s", path);
    for (auto &kv : g_table) {
        fprintf(f, "{\"mode\": %d, \"m\": %lld, \"n\": %lld, \"k\": %lld, \"cfg\": %d, \"split\": %d}\n",
                std::get<0>(kv.first), (long long)std::get<1>(kv.first), (long long)std::get<2>(kv.first),
                (long long)std::get<3>(kv.first), kv.second.first, kv.second.second);
    }
    for (auto &kv : g_plain_bucket)
        fprintf(f,
                "{\"bucket\": \"plain\", \"mode\": %d, \"bm\": %d, \"bn\": %d, \"bk\": %d, \"cfg\": %d, "
                "\"split\": %d}\n",
                std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
                kv.second.first, kv.second.second);
    for (auto &kv : g_grouped)
        fprintf(f, "{\"bucket\": \"grouped\", \"mode\": %d, \"bm\": %d, \"bn\": %d, \"bk\": %d, \"alone\": %d}\n",
                std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
                kv.second);
    for (int m = 0; m < GEMM_NUM_MODES; ++m)
        if (g_grouped_eff[m] > 0)
            fprintf(f, "{\"grouped_eff\": %d, \"eff\": %.3f, \"variant\": %d}\n", m, g_grouped_eff[m],
                    std::max(0, g_grouped_variant[m]));
    fclose(f);
    return GEMM_OK;
}

}  // extern "C"

namespace mg {

// Time every legal (configuration, split) of one shape; *cfg_out gets the
// fastest, *split_out its requested split factor and *norm_split_out the
// factor make_launch normalises it to for this shape.
static int tune_plain(int32_t mode, int64_t m, int64_t n, int64_t k, void *stream, int *cfg_out, int *split_out,
                      int *norm_split_out) {
    if (!mode_known(mode)) return fail(GEMM_EINVAL, "unknown mode %d", mode);
    if (m <= 0 || n <= 0 || k <= 0) return fail(GEMM_EINVAL, "tuning needs a non-empty product");
    int count = 0;
    const KernelCfg *t = configs(mode, &count);
    if (!t || count == 0) return fail(GEMM_EUNSUPPORTED, "mode %d has no kernels", mode);
    hipStream_t s = (hipStream_t)stream;
    const size_t es = elem_size(mode);
    void *A = nullptr, *B = nullptr, *C = nullptr, *ws = nullptr;
    int64_t ws_need = 0;
    gemm_problem_t p;
    memset(&p, 0, sizeof(p));
    p.mode = mode;
    p.m = m;
    p.n = n;
    p.k = k;
    p.lda = k;
    p.ldb = n;
    p.ldc = n;
    p.scale_a = p.scale_b = 1.f;
    for (int c = 0; c < count; ++c)
        for (int sp = 1; sp <= 16; sp *= 2) ws_need = std::max(ws_need, plain_ws_bytes(p, c, sp));
    int rc = GEMM_OK;
    if (hipMalloc(&A, (size_t)m * k * es) != hipSuccess || hipMalloc(&B, (size_t)k * n * es) != hipSuccess ||
        hipMalloc(&C, (size_t)m * n * 4) != hipSuccess ||
        (ws_need > 0 && hipMalloc(&ws, (size_t)ws_need) != hipSuccess)) {
        (void)hipGetLastError();
        rc = fail(GEMM_ENOMEM, "tuning buffers do not fit");
    }
    int best_c = 0, best_s = 1, best_req = 1;
    float best_ms = 1e30f;
    struct Cand {
        int cfg, split;
        float ms;
    };
    std::vector<Cand> cands;
    if (rc == GEMM_OK) {
        // non-zero operands: the clock under load depends on the data
        if (launch_fill_tuning(A, m * k, (int)es, 1u, s) != hipSuccess ||
            launch_fill_tuning(B, k * n, (int)es, 2u, s) != hipSuccess)
            rc = fail(GEMM_EHIP, "filling the tuning operands failed");
        p.A = A;
        p.B = B;
        p.C = static_cast<float *>(C);
        for (int c = 0; c < count && rc == GEMM_OK; ++c) {
            if (!cfg_eligible(p, t[c])) continue;
            const int64_t nkt = (k + split_grain(mode) - 1) / split_grain(mode);
            int last_split = 0;
            for (int sp = 1; sp <= 16 && rc == GEMM_OK; sp *= 2) {
                if (sp > 1 && nkt / sp < 4) break;
                const int eff = make_launch(p, t[c], sp).splits;
                if (eff == last_split) continue;
                last_split = eff;
                float ms = 0.f;
                rc = time_choice(p, c, sp, ws, s, &ms);
                if (rc == GEMM_OK) cands.push_back({c, sp, ms});
            }
        }
    }
    // Candidates within 3 % of the fastest are timed again, three rounds in
    // turn, and the lowest sum of the four medians wins: a single median
    // cannot tell choices that close apart.
    if (rc == GEMM_OK && !cands.empty()) {
        float first = 1e30f;
        for (const Cand &c : cands) first = std::min(first, c.ms);
        std::vector<Cand> close;
        for (const Cand &c : cands)
            if (c.ms <= first * 1.03f) close.push_back(c);
        for (int round = 0; round < 3 && close.size() > 1 && rc == GEMM_OK; ++round)
            for (Cand &c : close) {
                float ms = 0.f;
                rc = time_choice(p, c.cfg, c.split, ws, s, &ms);
                c.ms += ms;
                if (rc != GEMM_OK) break;
            }
        for (const Cand &c : close)
            if (c.ms < best_ms) {
                best_ms = c.ms;
                best_c = c.cfg;
                best_req = c.split;
                best_s = make_launch(p, t[c.cfg], c.split).splits;
            }
    }
    if (A) (void)hipFree(A);
    if (B) (void)hipFree(B);
    if (C) (void)hipFree(C);
    if (ws) (void)hipFree(ws);
    if (rc != GEMM_OK) return rc;
    *cfg_out = best_c;
    *split_out = best_req;
    *norm_split_out = best_s;
    return GEMM_OK;
}

}  // namespace mg

extern "C" {

int gemm_tune(int32_t mode, int64_t m, int64_t n, int64_t k, void *stream) {
    clear_error();
    int cfg = 0, req = 1, split = 1;
    const int rc = tune_plain(mode, m, n, k, stream, &cfg, &req, &split);
    if (rc != GEMM_OK) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[Key(mode, m, n, k)] = {cfg, split};
    return GEMM_OK;
}

int gemm_tune_bucket(int32_t mode, int64_t m, int64_t n, int64_t k, void *stream) {
    clear_error();
    int cfg = 0, req = 1, split = 1;
    const int rc = tune_plain(mode, m, n, k, stream, &cfg, &req, &split);
    if (rc != GEMM_OK) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    g_plain_bucket[bucket_of(mode, m, n, k)] = {cfg, req};
    return GEMM_OK;
}

}  // extern "C"
