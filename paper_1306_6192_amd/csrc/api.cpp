// C-ABI of the plain product, operand preparation, comparison reduction and
// diagnostics.  Argument validation happens here, before any HIP call.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>

#include "host.hpp"

namespace mg {

static thread_local char t_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_err, sizeof(t_err), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { t_err[0] = 0; }

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t elem_size(int mode) {
    switch (mode) {
        case GEMM_MODE_F32:
        case GEMM_MODE_F32_SPLIT_BF16X3: return 4;
        case GEMM_MODE_BF16:
        case GEMM_MODE_F16: return 2;
        case GEMM_MODE_F8E4M3: return 1;
        default: return 0;
    }
}

bool mode_known(int mode) { return mode >= 0 && mode < GEMM_NUM_MODES; }

// Largest dimension the kernels index with 32-bit tile arithmetic.
static const int64_t kMaxDim = (int64_t)1 << 30;

static bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

int validate(const gemm_problem_t *p) {
    if (!p) return fail(GEMM_EINVAL, "problem pointer is NULL");
    if (!mode_known(p->mode)) return fail(GEMM_EINVAL, "unknown mode %d", p->mode);
    if (p->flags != 0) return fail(GEMM_EINVAL, "flags must be 0 (got %d)", p->flags);
    if (p->m < 0 || p->n < 0 || p->k < 0)
        return fail(GEMM_EINVAL, "negative dimension (m=%lld n=%lld k=%lld)", (long long)p->m,
                    (long long)p->n, (long long)p->k);
    if (p->m > kMaxDim || p->n > kMaxDim || p->k > kMaxDim)
        return fail(GEMM_EUNSUPPORTED, "dimension above 2^30");
    if (p->lda < std::max<int64_t>(1, p->k))
        return fail(GEMM_EINVAL, "lda=%lld < max(1,k=%lld)", (long long)p->lda, (long long)p->k);
    if (p->ldb < std::max<int64_t>(1, p->n))
        return fail(GEMM_EINVAL, "ldb=%lld < max(1,n=%lld)", (long long)p->ldb, (long long)p->n);
    if (p->ldc < std::max<int64_t>(1, p->n))
        return fail(GEMM_EINVAL, "ldc=%lld < max(1,n=%lld)", (long long)p->ldc, (long long)p->n);
    const bool out_empty = p->m == 0 || p->n == 0;
    if (!out_empty && !p->C) return fail(GEMM_EINVAL, "C is NULL for a non-empty output");
    if (!out_empty && p->k > 0 && (!p->A || !p->B))
        return fail(GEMM_EINVAL, "A or B is NULL for a non-empty product");
    if (p->mode == GEMM_MODE_F8E4M3) {
        if (!(std::isfinite(p->scale_a) && p->scale_a > 0.f && std::isfinite(p->scale_b) &&
              p->scale_b > 0.f))
            return fail(GEMM_EINVAL, "FP8 scales must be finite and > 0");
    }
    if (!out_empty && p->k > 0) {
        const size_t es = elem_size(p->mode);
        const size_t cbytes = ((size_t)(p->m - 1) * p->ldc + p->n) * 4;
        const size_t abytes = ((size_t)(p->m - 1) * p->lda + p->k) * es;
        const size_t bbytes = ((size_t)(p->k - 1) * p->ldb + p->n) * es;
        if (overlaps(p->C, cbytes, p->A, abytes) || overlaps(p->C, cbytes, p->B, bbytes))
            return fail(GEMM_EINVAL, "C overlaps A or B");
    }
    return GEMM_OK;
}

int num_cus() {
    static int cached = -1;
    if (cached > 0) return cached;
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
        cached = n;
    else
        return 256;
    return cached;
}

const KernelCfg *configs(int mode, int *count) {
    if (mode == GEMM_MODE_F32) return f32_configs(count);
    if (mode == GEMM_MODE_F64) return f64_configs(count);
    if (mode == GEMM_MODE_C32) return c32_configs(count);
    return lp_configs(mode, count);
}

int split_grain(int mode) {
    switch (mode) {
        case GEMM_MODE_BF16:
        case GEMM_MODE_F16: return 64;
        case GEMM_MODE_F8E4M3: return 128;
        default: return 32;
    }
}

static bool vec_ok(const void *ptr, int64_t ld, size_t es) {
    return ((uintptr_t)ptr % 16 == 0) && ((ld * (int64_t)es) % 16 == 0);
}

Launch make_launch(const gemm_problem_t &p, const KernelCfg &kc, int split) {
    Launch L;
    TileProblem &P = L.P;
    memset(&P, 0, sizeof(P));
    const size_t es = elem_size(p.mode);
    P.A = p.A;
    P.B = p.B;
    P.C = p.C;
    P.lda = p.lda;
    P.ldb = p.ldb;
    P.ldc = p.ldc;
    P.m = (int32_t)p.m;
    P.n = (int32_t)p.n;
    P.k = (int32_t)p.k;
    P.tiles_m = (int32_t)((p.m + kc.bm - 1) / kc.bm);
    P.tiles_n = (int32_t)((p.n + kc.bn - 1) / kc.bn);
    // Split-K boundaries are placed on multiples of the mode's largest k-tile
    // (`grain`), so every configuration of a mode splits k at the same places
    // and sums each element in the same order.
    const int grain = split_grain(p.mode);
    const int ngr = (int)((p.k + grain - 1) / grain);
    split = std::max(1, std::min(split, std::max(1, ngr)));
    int per = (ngr + split - 1) / split;
    if (per < 1) per = 1;
    split = std::max(1, (ngr + per - 1) / per);
    P.splits = split;
    P.kt_per_split = per * (grain / kc.bk);
    P.vec = (vec_ok(p.A, p.lda, es) ? 1 : 0) | (vec_ok(p.B, p.ldb, es) ? 2 : 0) |
            (vec_ok(p.C, p.ldc, 4) ? 4 : 0);
    P.scale = p.mode == GEMM_MODE_F8E4M3 ? p.scale_a * p.scale_b : 1.f;
    P.split_stride = ((int64_t)p.m * p.n + 3) / 4 * 4;
    L.splits = split;
    L.nwg = P.tiles_m * P.tiles_n * split;
    L.ws_bytes = split > 1 ? (int64_t)split * P.split_stride * 4 : 0;
    return L;
}

// The pre-split path runs a BF16 product over an inner dimension of 3 k16
// (k rounded up to 16), which the tile indexes with 32-bit integers.
bool presplit_shape_ok(int64_t n, int64_t k) {
    const int64_t k16 = (k + 15) / 16 * 16;
    return n % 8 == 0 && n >= 8 && 3 * k16 <= (int64_t)INT32_MAX;
}

bool cfg_eligible(const gemm_problem_t &p, const KernelCfg &kc) {
    if (kc.presplit) return presplit_shape_ok(p.n, p.k);
    if (kc.chunk == 0) return true;
    const int64_t c = kc.chunk;
    return p.k % c == 0 && p.n % c == 0 && p.n >= c && p.lda % c == 0 && p.ldb % c == 0 &&
           (uintptr_t)p.A % 16 == 0 && (uintptr_t)p.B % 16 == 0;
}

int effective_cfg(const gemm_problem_t &p, int cfg) {
    int count = 0;
    const KernelCfg *t = configs(p.mode, &count);
    if (!t || cfg < 0 || cfg >= count || cfg_eligible(p, t[cfg])) return cfg;
    for (int c = 0; c < count; ++c)
        if (t[c].chunk == 0 && !t[c].presplit && t[c].bm == t[cfg].bm && t[c].bn == t[cfg].bn) return c;
    return 0;
}

// Bytes of the interleaved operand copies of the pre-split path (A' then B',
// each 256-byte aligned).
static int64_t presplit_bytes(const gemm_problem_t &p, int64_t *b_off) {
    const int64_t k16 = (p.k + 15) / 16 * 16;
    const int64_t a = ((int64_t)p.m * 3 * k16 * 2 + 255) / 256 * 256;
    *b_off = a;
    return a + ((int64_t)3 * k16 * p.n * 2 + 255) / 256 * 256;
}

int64_t plain_ws_bytes(const gemm_problem_t &p, int cfg, int split) {
    int count = 0;
    const KernelCfg *t = configs(p.mode, &count);
    if (!t || cfg < 0 || cfg >= count || p.m == 0 || p.n == 0 || p.k == 0) return 0;
    const KernelCfg &kc = t[effective_cfg(p, cfg)];
    int64_t ws = (make_launch(p, kc, split).ws_bytes + 255) / 256 * 256;
    if (kc.presplit) {
        int64_t b_off = 0;
        ws += presplit_bytes(p, &b_off);
    }
    return ws;
}

int enqueue_plain(const gemm_problem_t &p, int cfg, int split, void *ws, hipStream_t s) {
    if (p.m == 0 || p.n == 0) return GEMM_OK;
    if (p.k == 0) {
        MG_HIP(launch_fill_zero(p.C, p.ldc, (int)p.m, (int)p.n, s));
        return GEMM_OK;
    }
    int count = 0;
    const KernelCfg *t = configs(p.mode, &count);
    if (!t || count == 0) return fail(GEMM_EUNSUPPORTED, "mode %d has no kernels", p.mode);
    if (cfg < 0 || cfg >= count) return fail(GEMM_EINVAL, "config %d out of range [0,%d)", cfg, count);
    cfg = effective_cfg(p, cfg);
    Launch L = make_launch(p, t[cfg], split);
    if (L.splits > 1) {
        if (!ws) return fail(GEMM_EINTERNAL, "split-K workspace missing");
        L.P.C = static_cast<float *>(ws);
    }
    if (t[cfg].presplit) {
        // interleaved bfloat16 operands after the split-K slabs; the product
        // runs over 3 k16 with three BF16 k-tiles per 32-k split grain
        if (!ws) return fail(GEMM_EINTERNAL, "pre-split workspace missing");
        int64_t b_off = 0;
        presplit_bytes(p, &b_off);
        uint8_t *base = static_cast<uint8_t *>(ws) + (L.ws_bytes + 255) / 256 * 256;
        uint16_t *Ap = reinterpret_cast<uint16_t *>(base);
        uint16_t *Bp = reinterpret_cast<uint16_t *>(base + b_off);
        const int64_t k16 = (p.k + 15) / 16 * 16;
        MG_HIP(launch_presplit(static_cast<const float *>(p.A), p.lda, static_cast<const float *>(p.B), p.ldb,
                               (int)p.m, (int)p.n, (int)p.k, Ap, Bp, s));
        L.P.A = Ap;
        L.P.B = Bp;
        L.P.lda = 3 * k16;
        L.P.ldb = p.n;
        L.P.k = (int32_t)(3 * k16);
        L.P.kt_per_split = L.P.kt_per_split * 3;
        L.P.vec = 3;
    }
    MG_HIP(t[cfg].plain(L.P, L.nwg, s));
    if (L.splits > 1)
        MG_HIP(launch_splitk_reduce(static_cast<const float *>(ws), L.P.split_stride, L.splits, L.P.scale,
                                    p.C, p.ldc, (int)p.m, (int)p.n, s));
    return GEMM_OK;
}

// ---------------------------------------------------------------------------
// Device buffers.

int DevBuf::ensure(size_t need, hipStream_t s) {
    if (need <= bytes) return GEMM_OK;
    if (ptr) {
        MG_HIP(hipStreamSynchronize(s));
        MG_HIP(hipFree(ptr));
        ptr = nullptr;
        bytes = 0;
    }
    size_t sz = std::max<size_t>(need, 1 << 20);
    sz = (sz + 255) / 256 * 256;
    if (hipMalloc(&ptr, sz) != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return fail(GEMM_ENOMEM, "workspace allocation of %zu bytes failed", sz);
    }
    bytes = sz;
    return GEMM_OK;
}

void DevBuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

struct StreamWs {
    std::mutex mu;   // held by the caller from ensure() to the enqueue of the work that uses a slot
    DevBuf slot[4];
};
static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, StreamWs *> g_ws;

static StreamWs *stream_ws(hipStream_t s) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_ws_mu);
    StreamWs *&w = g_ws[{dev, s}];
    if (!w) w = new StreamWs();
    return w;
}

DevBuf *stream_workspace(hipStream_t s, int slot) { return &stream_ws(s)->slot[slot]; }

std::unique_lock<std::mutex> lock_stream_workspaces(hipStream_t s) {
    return std::unique_lock<std::mutex>(stream_ws(s)->mu);
}

// ---------------------------------------------------------------------------
// Scratch of gemm_plain_noalloc: split-K partial slabs and split-BF16x3
// operand copies of at most GEMM_NOALLOC_SCRATCH_BYTES, in a device array that
// every GPU the library runs on holds until the process ends.  Host code never
// passes the array's name to a kernel or a copy (on the host it is only a
// stand-in for the symbol): it uses the per-device address
// hipGetSymbolAddress returns, taken once per device with that device
// current.
static __device__ __align__(256) uint8_t scratch[GEMM_NOALLOC_SCRATCH_BYTES];

static const int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxScratchDevices];

int noalloc_scratch(void **out) {
    *out = nullptr;
    int dev = 0;
    MG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(GEMM_EUNSUPPORTED, "device %d: at most %d devices", dev,
                                                          kMaxScratchDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(GEMM_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return GEMM_OK;
}

}  // namespace mg

using namespace mg;

extern "C" {

const char *gemm_last_error(void) { return t_err; }

int gemm_version(void) { return 1; }

uint64_t gemm_now_ns(void) { return now_ns(); }

int gemm_num_configs(int32_t mode) {
    clear_error();
    if (mode < 0 || mode >= GEMM_NUM_KERNEL_FAMILIES) return fail(GEMM_EINVAL, "unknown mode %d", mode);
    int count = 0;
    configs(mode, &count);
    return count;
}

int gemm_config_info(int32_t mode, int32_t cfg, int32_t info[6]) {
    clear_error();
    if (mode < 0 || mode >= GEMM_NUM_KERNEL_FAMILIES) return fail(GEMM_EINVAL, "unknown mode %d", mode);
    if (!info) return fail(GEMM_EINVAL, "info is NULL");
    int count = 0;
    const KernelCfg *t = configs(mode, &count);
    if (cfg < 0 || cfg >= count) return fail(GEMM_EINVAL, "config %d out of range", cfg);
    info[0] = t[cfg].bm;
    info[1] = t[cfg].bn;
    info[2] = t[cfg].bk;
    info[3] = t[cfg].waves;
    info[4] = t[cfg].lds_bytes;
    info[5] = t[cfg].mfma_k;
    return GEMM_OK;
}

int gemm_config_chunk(int32_t mode, int32_t cfg) {
    clear_error();
    if (mode < 0 || mode >= GEMM_NUM_KERNEL_FAMILIES) return fail(GEMM_EINVAL, "unknown mode %d", mode);
    int count = 0;
    const KernelCfg *t = configs(mode, &count);
    if (cfg < 0 || cfg >= count) return fail(GEMM_EINVAL, "config %d out of range", cfg);
    return t[cfg].chunk;
}

static int plain_common(const gemm_problem_t *p, int cfg, int split, void *stream) {
    int rc = validate(p);
    if (rc != GEMM_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (p->m == 0 || p->n == 0) return GEMM_OK;
    void *ws = nullptr;
    std::unique_lock<std::mutex> ws_lock = lock_stream_workspaces(s);
    if (p->k > 0) {
        int count = 0;
        configs(p->mode, &count);
        if (count == 0) return fail(GEMM_EUNSUPPORTED, "mode %d has no kernels", p->mode);
        const int64_t need = plain_ws_bytes(*p, cfg, split);
        if (need > 0) {
            DevBuf *b = stream_workspace(s, 0);
            rc = b->ensure((size_t)need, s);
            if (rc != GEMM_OK) return rc;
            ws = b->ptr;
        }
    }
    return enqueue_plain(*p, cfg, split, ws, s);
}

int gemm_plain(const gemm_problem_t *p, void *stream) {
    clear_error();
    int rc = validate(p);
    if (rc != GEMM_OK) return rc;
    int cfg = 0, split = 1;
    tuner_choose(p->mode, p->m, p->n, p->k, &cfg, &split);
    return plain_common(p, cfg, split, stream);
}

int gemm_plain_cfg(const gemm_problem_t *p, int32_t cfg, int32_t split_k, void *stream) {
    clear_error();
    if (split_k < 1) return fail(GEMM_EINVAL, "split_k must be >= 1");
    int rc = validate(p);
    if (rc != GEMM_OK) return rc;
    int count = 0;
    configs(p->mode, &count);
    if (count == 0) return fail(GEMM_EUNSUPPORTED, "mode %d has no kernels", p->mode);
    if (cfg < 0 || cfg >= count) return fail(GEMM_EINVAL, "config %d out of range [0,%d)", cfg, count);
    return plain_common(p, cfg, split_k, stream);
}

int gemm_plain_workspace_bytes(const gemm_problem_t *p, uint64_t *bytes_out) {
    clear_error();
    if (!bytes_out) return fail(GEMM_EINVAL, "bytes_out is NULL");
    *bytes_out = 0;
    int rc = validate(p);
    if (rc != GEMM_OK) return rc;
    if (p->m == 0 || p->n == 0 || p->k == 0) return GEMM_OK;
    int cfg = 0, split = 1;
    tuner_choose(p->mode, p->m, p->n, p->k, &cfg, &split);
    *bytes_out = (uint64_t)plain_ws_bytes(*p, cfg, split);
    return GEMM_OK;
}

// Allocation-free plain product: gemm_plain's plan, with its workspace in a
// fixed device array instead of the per-stream library workspace.
int gemm_plain_noalloc(const gemm_problem_t *p, void *stream) {
    clear_error();
    int rc = validate(p);
    if (rc != GEMM_OK) return rc;
    if (p->m == 0 || p->n == 0) return GEMM_OK;
    int cfg = 0, split = 1;
    void *ws = nullptr;
    if (p->k > 0) {
        int count = 0;
        configs(p->mode, &count);
        if (count == 0) return fail(GEMM_EUNSUPPORTED, "mode %d has no kernels", p->mode);
        tuner_choose(p->mode, p->m, p->n, p->k, &cfg, &split);
        const int64_t need = plain_ws_bytes(*p, cfg, split);
        if (need > GEMM_NOALLOC_SCRATCH_BYTES)
            return fail(GEMM_EINVAL,
                        "this product needs %lld bytes of workspace; gemm_plain_noalloc holds at most %lld "
                        "(use gemm_plain)",
                        (long long)need, (long long)GEMM_NOALLOC_SCRATCH_BYTES);
        if (need > 0) {
            rc = noalloc_scratch(&ws);
            if (rc != GEMM_OK) return rc;
        }
    }
    return enqueue_plain(*p, cfg, split, ws, (hipStream_t)stream);
}

int gemm_convert_f32(const float *x, int64_t count, int32_t to_mode, void *out, void *stream) {
    clear_error();
    if (count < 0) return fail(GEMM_EINVAL, "negative count");
    if (to_mode != GEMM_MODE_BF16 && to_mode != GEMM_MODE_F16)
        return fail(GEMM_EINVAL, "to_mode must be BF16 or F16");
    if (count == 0) return GEMM_OK;
    if (!x || !out) return fail(GEMM_EINVAL, "NULL buffer");
    if (overlaps(x, (size_t)count * 4, out, (size_t)count * 2)) return fail(GEMM_EINVAL, "buffers overlap");
    MG_HIP(launch_convert_f32(x, count, to_mode, out, (hipStream_t)stream));
    return GEMM_OK;
}

int gemm_quantize_e4m3(const float *x, int64_t count, uint8_t *q, float *scale_out, void *stream) {
    clear_error();
    if (count < 0) return fail(GEMM_EINVAL, "negative count");
    if (!scale_out) return fail(GEMM_EINVAL, "scale_out is NULL");
    if (count > 0 && (!x || !q)) return fail(GEMM_EINVAL, "NULL buffer");
    if (count > 0 && overlaps(x, (size_t)count * 4, q, (size_t)count)) return fail(GEMM_EINVAL, "buffers overlap");
    hipStream_t s = (hipStream_t)stream;
    std::unique_lock<std::mutex> ws_lock = lock_stream_workspaces(s);
    DevBuf *b = stream_workspace(s, 2);
    int rc = b->ensure(4096, s);
    if (rc != GEMM_OK) return rc;
    MG_HIP(launch_quantize_e4m3(x, count, q, scale_out, static_cast<uint32_t *>(b->ptr), s));
    return GEMM_OK;
}

int gemm_errnorm(const float *C, int64_t ldc, const double *R, int64_t ldr, int64_t m, int64_t n,
                 double *out3, void *stream) {
    clear_error();
    if (m < 0 || n < 0) return fail(GEMM_EINVAL, "negative dimension");
    if (!out3) return fail(GEMM_EINVAL, "out3 is NULL");
    if (ldc < std::max<int64_t>(1, n) || ldr < std::max<int64_t>(1, n)) return fail(GEMM_EINVAL, "bad ld");
    if (m * n > 0 && (!C || !R)) return fail(GEMM_EINVAL, "NULL matrix");
    hipStream_t s = (hipStream_t)stream;
    const int nparts = 2048;
    std::unique_lock<std::mutex> ws_lock = lock_stream_workspaces(s);
    DevBuf *b = stream_workspace(s, 2);
    int rc = b->ensure(4096 + (size_t)nparts * 3 * sizeof(double), s);
    if (rc != GEMM_OK) return rc;
    double *partials = reinterpret_cast<double *>(static_cast<char *>(b->ptr) + 4096);
    MG_HIP(launch_errnorm(C, ldc, R, ldr, m, n, out3, partials, nparts, s));
    return GEMM_OK;
}

}  // extern "C"
