/*
 * mi355gemm -- dense matrix product C = A * B on AMD Instinct MI355X (gfx950).
 *
 * The operation is the standard ("Cauchy") product of the paper's
 * Implementation section (the equation for c_ij):
 *
 *     c_ij = sum_{r=0}^{k-1} a_ir * b_rj,     0 <= i < m, 0 <= j < n,
 *
 * for a row-major m x k matrix A and a row-major k x n matrix B.  The paper's
 * (n x m) * (m x p) maps onto (m x k) * (k x n) here.  C is overwritten (no
 * alpha/beta), as the paper's loops zero each c_ij before accumulating.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All functions are extern "C", never throw, and return an int status
 *    (gemm_status_t).  On failure gemm_last_error() describes the cause.
 *  - Matrix pointers are DEVICE pointers on the current HIP device, owned by
 *    the caller, row-major, with row strides (lda, ldb, ldc) in ELEMENTS.
 *    The caller keeps them alive until the enqueued work has completed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued asynchronously; nothing synchronises the host unless
 *    stated.
 *  - Argument validation happens before any HIP call and touches no memory:
 *    m, n, k >= 0; lda >= max(1,k); ldb >= max(1,n); ldc >= max(1,n);
 *    non-NULL pointers for non-empty operands; a known mode; FP8 scales
 *    finite and > 0; C must not overlap A or B.  Violations return
 *    GEMM_EINVAL (or GEMM_EUNSUPPORTED for a mode an entry point lacks, and
 *    for m, n or k above 2^30).  Offsets are formed in 64 bits: C and the
 *    operands may hold more than 2^31 elements.
 *  - k == 0 writes zeros to C (the empty sum); m == 0 or n == 0 is a no-op.
 *  - A failing HIP call returns GEMM_EHIP with the HIP error text.
 *  - Loading the library makes no HIP call; functions may be called from
 *    several host threads (the tuning table is lock-protected, and each
 *    (device, stream) workspace is locked from its growth to the enqueue of
 *    the work that uses it, so threads may share a stream).
 */
#ifndef MI355GEMM_H
#define MI355GEMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GEMM_OK = 0,
    GEMM_PENDING = 1,        /* informational: serving request not done yet */
    GEMM_EINVAL = -1,        /* bad argument */
    GEMM_EUNSUPPORTED = -2,  /* valid but not supported by this entry point */
    GEMM_ENOMEM = -3,        /* allocation failed or over the serving budget */
    GEMM_EHIP = -4,          /* a HIP runtime call failed */
    GEMM_EBUSY = -5,         /* serving queue full: retry later */
    GEMM_ENOTFOUND = -6,     /* unknown ticket / file */
    GEMM_EINTERNAL = -7
} gemm_status_t;

/* Arithmetic form of one product.  All forms accumulate in float32 and write
 * float32 C.  Element type of A and B:
 *   F32              float32  -- the paper's float product, on FP32 MFMA
 *   BF16, F16        bfloat16 / binary16 codes (uint16)
 *   F8E4M3           OCP FP8 E4M3 codes (uint8); C = scale_a*scale_b*(qA qB)
 *   F32_SPLIT_BF16X3 float32; each operand is split into
 *                    hi = RNE_bf16(x), lo = RNE_bf16(x - hi) and
 *                    C = hiA hiB + hiA loB + loA hiB (compensated BF16),
 *                    the three products summed per 16 k in the order
 *                    loA hiB, hiA loB, hiA hiB.  The split happens at
 *                    tile staging, or (n a multiple of 8) once per operand
 *                    into a library workspace of 6*k16*(m + n) bytes,
 *                    k16 = k rounded up to 16; both give the same bits. */
typedef enum {
    GEMM_MODE_F32 = 0,
    GEMM_MODE_BF16 = 1,
    GEMM_MODE_F16 = 2,
    GEMM_MODE_F8E4M3 = 3,
    GEMM_MODE_F32_SPLIT_BF16X3 = 4,
    /* Kernel families with entry points of their own (gemm_plain_f64,
     * gemm_plain_c32); they name configurations in gemm_num_configs /
     * gemm_config_info and are not valid in a gemm_problem_t. */
    GEMM_MODE_F64 = 5,
    GEMM_MODE_C32 = 6
} gemm_mode_t;

#define GEMM_NUM_MODES 5            /* modes a gemm_problem_t may carry */
#define GEMM_NUM_KERNEL_FAMILIES 7  /* modes gemm_num_configs accepts */

/* One product problem (row-major; C = A*B, C overwritten). */
typedef struct gemm_problem {
    int32_t mode;          /* gemm_mode_t */
    int32_t flags;         /* reserved, must be 0 */
    int64_t m, n, k;
    const void *A;         /* m x k, element type by mode */
    int64_t lda;
    const void *B;         /* k x n, same element type as A */
    int64_t ldb;
    float *C;              /* m x n float32 */
    int64_t ldc;
    float scale_a;         /* F8E4M3 only: dequantisation factors, C = */
    float scale_b;         /* scale_a*scale_b*sum(qa*qb); ignored otherwise */
} gemm_problem_t;

/* ---------------------------------------------------------------------- */
/* Plain product (method steps: tile decomposition, LDS staging, MFMA      */
/* inner product, split-K partial reduction, epilogue).                    */

/* C = A*B for one problem, enqueued on `stream`.  The tile configuration
 * and split-K factor come from the tuning table (shape-keyed); split-K
 * partial sums go to a library-owned workspace and are summed in a fixed
 * order, so a given (mode, m, n, k) always produces the same bits.  The
 * workspace (one per device and stream, grown on demand, kept until the
 * process ends) also holds the split-BF16x3 operand copies. */
int gemm_plain(const gemm_problem_t *p, void *stream);

/* As gemm_plain with an explicit tile configuration (index into
 * gemm_config_info) and split-K factor (>= 1).  For tuning and tests.
 * Configurations whose k-tile is copied straight into LDS in 16-byte chunks
 * need k and n multiples of the chunk (16 bytes of elements), lda and ldb
 * likewise and 16-byte aligned A and B; for any other problem the
 * register-staged configuration of the same tile size runs instead.  Split-K
 * cuts k into ranges of whole grains (32 k for FP32 and split-BF16x3, 64 for
 * BF16 and F16, 128 for FP8), each a whole number of every configuration's
 * k-tiles, so for a given split factor every configuration of a mode gives
 * the same bits. */
int gemm_plain_cfg(const gemm_problem_t *p, int32_t cfg, int32_t split_k, void *stream);

/* Device workspace bytes gemm_plain uses for this problem (split-K partial
 * slabs of split*m*n float32, plus the split-BF16x3 operand copies when the
 * pre-split path runs), rounded up to 256 bytes; 0 when the chosen
 * configuration needs none.  Same validation as gemm_plain (no memory is
 * touched); the configuration lookup may read the device's compute-unit
 * count. */
int gemm_plain_workspace_bytes(const gemm_problem_t *p, uint64_t *bytes_out);

/* Allocation-free plain product, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same tile configuration, split-K factor and bits as
 * gemm_plain; the workspace gemm_plain_workspace_bytes reports comes from a
 * fixed device array of GEMM_NOALLOC_SCRATCH_BYTES that each GPU holds from
 * the library's load until the process ends, instead of the per-stream
 * workspace.  No call allocates or frees device memory (the first call on a
 * device looks the array's address up once).  Errors: as gemm_plain, plus
 * GEMM_EINVAL when the product needs more workspace than the array holds
 * (gemm_plain serves it).  Every call on one GPU shares that GPU's array:
 * calls whose work overlaps on the device (different streams, or several
 * host threads without ordering) race and give undefined results; calls on
 * one stream are ordered by it.  Nothing in the array needs to start at
 * zero (every slab element is written before it is read). */
#define GEMM_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
int gemm_plain_noalloc(const gemm_problem_t *p, void *stream);

/* The paper's own GPU kernels on gfx950, float32 only, as a baseline for the
 * matrix-core path: variant 0 = one thread per c_ij reading A and B from
 * global memory (Implementation section, Listing 3); variant 1 = 16x16
 * blocks staging 16x16 tiles of A and B in LDS (Listing 4).  Bounds-checked
 * for any shape; same conventions and errors as gemm_plain
 * (GEMM_EUNSUPPORTED for other modes). */
int gemm_ablation(const gemm_problem_t *p, int32_t variant, void *stream);

/* Number of tile configurations compiled for `mode` (any of the
 * GEMM_NUM_KERNEL_FAMILIES), and their geometry:
 * info[0..5] = {BM, BN, BK, waves, lds_bytes, mfma_k}. */
int gemm_num_configs(int32_t mode);
int gemm_config_info(int32_t mode, int32_t cfg, int32_t info[6]);

/* The chunk a configuration copies straight into LDS, in elements (16 bytes
 * of the mode's element type), or 0 for a register-staged configuration that
 * takes any shape; GEMM_EINVAL for an unknown mode or configuration.  A
 * chunked configuration runs only where k, n, lda and ldb are multiples of
 * the chunk and A, B are 16-byte aligned (else see gemm_plain_cfg). */
int gemm_config_chunk(int32_t mode, int32_t cfg);

/* ---------------------------------------------------------------------- */
/* Double and complex-float products, matrix addition (the paper times the */
/* product for float, double and complex float matrices, Results section,  */
/* Table 2, and analyses matrix addition/subtraction beside it, Fig. 9).    */

/* C = A*B in binary64: A (m x k), B (k x n), C (m x n) are double, row-major,
 * strides in elements.  Products and sums are binary64 operations on the
 * matrix cores (v_mfma_f64_16x16x4_f64); summation order is unspecified, so
 * each c_ij is within (k+2) 2^-53 (|A||B|)_ij of the exact value.  The tile
 * configuration is chosen from the shape; there is no split-K.  Same
 * validation and errors as gemm_plain (C must not overlap A or B); k == 0
 * zeroes C. */
int gemm_plain_f64(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B, int64_t ldb,
                   double *C, int64_t ldc, void *stream);
/* As gemm_plain_f64 with an explicit configuration (gemm_config_info of
 * GEMM_MODE_F64; chunked configurations fall back as for gemm_plain_cfg, and
 * every configuration gives the same bits).  For tests. */
int gemm_plain_f64_cfg(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B,
                       int64_t ldb, double *C, int64_t ldc, int32_t cfg, void *stream);

/* C = A*B over complex float: every element is an interleaved (re, im) pair
 * of float32 (8 bytes; C99 float _Complex layout), strides count COMPLEX
 * elements.  Each complex multiply-add is four real float32 MFMA products
 * (Re += ar br - ai bi, Im += ar bi + ai br) accumulated in float32.  No
 * split-K; same validation and errors as gemm_plain_f64. */
int gemm_plain_c32(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda, const float *B, int64_t ldb,
                   float *C, int64_t ldc, void *stream);
int gemm_plain_c32_cfg(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda, const float *B,
                       int64_t ldb, float *C, int64_t ldc, int32_t cfg, void *stream);

/* c_ij = a_ij + b_ij (subtract == 0) or a_ij - b_ij (subtract != 0), one
 * IEEE operation per element.  `dtype` is GEMM_MODE_F32 (float) or
 * GEMM_MODE_F64 (double); A, B, C are m x n with strides in elements
 * (>= max(1, n)).  C may be A or B itself (same stride: in place); any other
 * overlap is GEMM_EINVAL.  m == 0 or n == 0 is a no-op. */
int gemm_add(int32_t dtype, int32_t subtract, int64_t m, int64_t n, const void *A, int64_t lda, const void *B,
             int64_t ldb, void *C, int64_t ldc, void *stream);

/* ---------------------------------------------------------------------- */
/* Operand preparation (the reduced-precision forms' input conversion).    */

/* out[i] = RNE(x[i]) in bfloat16 (to_mode = BF16) or binary16 (F16);
 * `out` holds `count` uint16 codes.  Device pointers. */
int gemm_convert_f32(const float *x, int64_t count, int32_t to_mode, void *out, void *stream);

/* Per-tensor E4M3 quantisation: amax = max|x| (exact), s = amax/448 in
 * float32 (1 for an all-zero tensor), q[i] = E4M3(RNE_sat(x[i]/s)) with the
 * quotient rounded to float32.  `scale_out` is one float of DEVICE memory;
 * `q` holds `count` uint8 codes. */
int gemm_quantize_e4m3(const float *x, int64_t count, uint8_t *q, float *scale_out, void *stream);

/* ---------------------------------------------------------------------- */
/* Comparison reduction (normwise error against a binary64 reference).    */

/* out3 (DEVICE, 3 doubles) = { sum (C-R)^2, sum R^2, max |C-R| } over the
 * m x n matrices C (float32, ldc) and R (binary64, ldr), in binary64.
 * The relative error is sqrt(out3[0] / out3[1]). */
int gemm_errnorm(const float *C, int64_t ldc, const double *R, int64_t ldr,
                 int64_t m, int64_t n, double *out3, void *stream);

/* ---------------------------------------------------------------------- */
/* Grouped product: many independent problems in one persistent launch.   */
/* Each problem is the product of the Implementation section; running many */
/* of them in one launch is not in the paper: it carries the paper's block */
/* decomposition (one thread block per output tile, Fig. 5) across         */
/* problems, with one queue of tiles over all of them.                     */

/* All problems must share one mode (F32 or BF16/F16/F8E4M3/split).  The
 * mode's grouped kernel is the variant the autotuner measured fastest on a
 * mixed batch (gemm_tune_grouped_mix; variant 0 when not measured): variant
 * 0 runs every problem on one 128 x 128 tile, variant 1 on 128 x 128 or
 * 64 x 64 by the cost model (all on the smaller one when the launch would
 * not fill the chip).  Every tile of a mode gives the same bits, so a
 * problem's result does not depend on the other problems or the variant,
 * and equals gemm_plain's with split_k = 1.  The host builds a static schedule (gemm_grouped_schedule)
 * and uploads it with the descriptors into the (device, stream) pair's
 * workspace, so calls on different streams run independently, and calls on
 * one stream are ordered by it. */
int gemm_grouped(const gemm_problem_t *ps, int32_t count, void *stream);

/* The grouped kernel of `mode` in use: info[0..6] = {first and second tile
 * configuration of its stream (indices into gemm_config_info; equal when it
 * runs one), resident workgroups per CU, LDS bytes per workgroup, the larger
 * and the smaller configuration a problem launched on its own may take, the
 * variant (0 or 1)}. */
int gemm_grouped_info(int32_t mode, int32_t info[7]);

/* The tile configuration a problem of this shape gets in a grouped launch
 * (out[0]: the stream's tile, or for a two-tile stream the cost model's
 * choice with the mode's calibrated small-tile efficiency) and as a launch
 * of its own in the server (out[1]: the bucket's measured choice between the
 * two configurations of gemm_grouped_info's info[4..5], else the model),
 * and out[2] = 1 when both come from measurements (0: the model's defaults).
 * A two-tile launch whose problems would not fill every resident-workgroup
 * slot runs all of them on the smaller tile instead (see gemm_grouped_plan). */
int gemm_grouped_lookup(int32_t mode, int64_t m, int64_t n, int64_t k, int32_t out[3]);

/* The tile configuration each problem of this list gets in gemm_grouped
 * (cfg_out[i], -1 for an empty output); validates like gemm_grouped and
 * enqueues nothing. */
int gemm_grouped_plan(const gemm_problem_t *ps, int32_t count, int32_t *cfg_out);

/* The static schedule gemm_grouped builds for this list (validates like
 * gemm_grouped; host only, no device call): *nwg_out workgroups (workgroup w
 * runs on XCD w mod 8) and *ntiles_out output tiles; when the arrays are not
 * NULL, wg_first[0..nwg] (workgroup w runs tiles wg_first[w] ..
 * wg_first[w+1]-1, in order) and, per tile, the index of its problem in
 * `ps` and its first output row and column.  Call once with NULL arrays
 * for the sizes. */
int gemm_grouped_schedule(const gemm_problem_t *ps, int32_t count, int32_t *nwg_out, int32_t *ntiles_out,
                          int32_t *wg_first, int32_t *tile_problem, int32_t *tile_m0, int32_t *tile_n0);

/* Build a graph that replays the grouped launch for this problem list
 * (descriptors are uploaded once, into graph-owned device memory).  The
 * problems' pointers must stay valid for the graph's lifetime. */
int gemm_grouped_graph_create(const gemm_problem_t *ps, int32_t count, void **graph_out);
int gemm_graph_launch(void *graph, void *stream);
int gemm_graph_destroy(void *graph);

/* ---------------------------------------------------------------------- */
/* Tuning table (project autotuner).  Not in the paper, whose kernels use */
/* one fixed 16x16 block: here the tile configuration and split-K factor   */
/* of each shape are measured on the device.                               */

/* Time every legal configuration and split-K factor for this shape on the
 * current device and record the fastest in the table (synchronises).  The
 * library allocates the operands and fills them with non-zero pseudo-random
 * values of the mode's type (the clock under load depends on the data); each
 * choice is the median of five launches, and the choices within 3 % of the
 * fastest are timed three more times in turn before the fastest is kept.
 * Errors: GEMM_EINVAL (unknown mode, an empty product), GEMM_ENOMEM (the
 * operands do not fit), GEMM_EHIP. */
int gemm_tune(int32_t mode, int64_t m, int64_t n, int64_t k, void *stream);
/* As gemm_tune, but the choice is recorded for the shape's bucket
 * (floor(log2) of m, n and k), which gemm_plain consults for any shape
 * without an exact entry; the split factor is kept as requested, and each
 * shape of the bucket normalises it to its own k. */
int gemm_tune_bucket(int32_t mode, int64_t m, int64_t n, int64_t k, void *stream);
/* Measure the two configurations a problem launched alone may take
 * (gemm_grouped_info's info[4..5]) on a problem of this shape (medians of seven event-timed launches on non-zero operands the
 * library allocates) and record the faster for the shape's bucket: the tile
 * a serving batch of one gets.  Synchronises.  Dimensions up to 65536.
 * Errors: GEMM_EINVAL, GEMM_EUNSUPPORTED, GEMM_ENOMEM, GEMM_EHIP. */
int gemm_tune_grouped(int32_t mode, int64_t m, int64_t n, int64_t k, void *stream);
/* Choose, on the caller's mixed problem list (one mode, device operands the
 * caller owns; C is overwritten), the mode's grouped kernel variant and the
 * cost model that picks each problem's tile in variant 1: variant 0, and
 * variant 1 with the small tile's efficiency relative to the large one
 * varied over a grid, are each planned and timed (median of seven launches,
 * two passes), and the fastest is recorded for the mode; variant 0 (with
 * the default efficiency 0.6) is kept unless another is more than 1 %
 * faster.  Synchronises.  Errors: as gemm_grouped, plus GEMM_EHIP. */
int gemm_tune_grouped_mix(const gemm_problem_t *ps, int32_t count, void *stream);
/* The (cfg, split_k) gemm_plain would use for this shape: the exact entry,
 * else the bucket entry, else the cost model. */
int gemm_tuner_lookup(int32_t mode, int64_t m, int64_t n, int64_t k, int32_t *cfg, int32_t *split_k);
int gemm_tuner_load(const char *path);
int gemm_tuner_save(const char *path);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of arriving products.  Not in the paper   */
/* (whose host launches one product at a time, Implementation section):    */
/* every request is the same product, admitted by the device memory it     */
/* holds and batched into grouped launches on several streams.             */

typedef struct gemm_serve_config {
    uint64_t hbm_budget_bytes;  /* admission limit on the sum of in-flight footprints */
    int32_t max_inflight;       /* maximum admitted, unfinished requests */
    int32_t num_streams;        /* device streams batches are spread over */
    int32_t max_batch;          /* maximum requests in one launch */
    int32_t queue_capacity;     /* maximum queued (not yet admitted) requests */
    int32_t executor;           /* 0 = GPU grouped batches, 1 = host fake executor (tests),
                                   2 = GPU plain launches, one per request, FIFO on one stream */
    int32_t fake_fail_every;    /* fake executor: fail every Nth batch (0 = never) */
} gemm_serve_config_t;

typedef struct gemm_serve_result {
    int32_t status;             /* GEMM_OK when done, < 0 on failure */
    int32_t batch_size;         /* requests in the launch that ran it */
    uint64_t t_arrival_ns, t_admit_ns, t_launch_ns, t_done_ns;  /* steady clock */
} gemm_serve_result_t;

typedef struct gemm_serve_stats {
    uint64_t submitted, completed, failed, batches;
    uint64_t inflight_bytes, peak_inflight_bytes;
    int32_t queued, inflight;
} gemm_serve_stats_t;

/* Admission footprint of a request under the batched executors (0, 1):
 * bytes(A) + bytes(B) + 4*m*n (grouped launches and a batch of one use no
 * workspace).  The plain-launch executor (2) admits each request by that
 * plus gemm_plain_workspace_bytes(p), the workspace of its plain launch. */
int gemm_serve_footprint(const gemm_problem_t *p, uint64_t *bytes_out);
int gemm_serve_create(const gemm_serve_config_t *cfg, void **server_out);
/* Enqueue one request (copied); returns a monotonic ticket.  GEMM_ENOMEM if
 * its footprint exceeds the budget, GEMM_EBUSY if the queue is full.
 * t_arrival_ns = 0 stamps the current steady-clock time. */
int gemm_serve_submit(void *server, const gemm_problem_t *p, uint64_t t_arrival_ns, uint64_t *ticket_out);
/* GEMM_OK (done, result filled), GEMM_PENDING, or < 0. */
int gemm_serve_poll(void *server, uint64_t ticket, gemm_serve_result_t *out);
/* Block until every submitted request has finished. */
int gemm_serve_drain(void *server);
int gemm_serve_stats(void *server, gemm_serve_stats_t *out);
/* Drains, then frees the server. */
int gemm_serve_destroy(void *server);
/* Open-loop load generator: submit ps[i] when the steady clock reaches
 * t0 + offsets_ns[i] (t0 = the call time) with that scheduled time as its
 * arrival stamp, retrying while the queue is full; tickets_out[i] receives
 * its ticket.  Returns once every request is submitted. */
int gemm_serve_replay(void *server, const gemm_problem_t *ps, const uint64_t *offsets_ns, int32_t count,
                      uint64_t *tickets_out);
/* Current steady-clock time in ns (the clock of the serving timestamps). */
uint64_t gemm_now_ns(void);

/* ---------------------------------------------------------------------- */
/* Diagnostics.                                                            */

/* Thread-local text of the last failure (static storage; valid until the
 * calling thread's next library call). */
const char *gemm_last_error(void);
int gemm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MI355GEMM_H */
