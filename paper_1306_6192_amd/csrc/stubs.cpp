// Entry points not built yet.
#include "host.hpp"

using namespace mg;

extern "C" {
int gemm_grouped(const gemm_problem_t *, int32_t, void *) { return fail(GEMM_EUNSUPPORTED, "not built"); }
int gemm_grouped_graph_create(const gemm_problem_t *, int32_t, void **) { return fail(GEMM_EUNSUPPORTED, "not built"); }
int gemm_graph_launch(void *, void *) { return fail(GEMM_EUNSUPPORTED, "not built"); }
int gemm_graph_destroy(void *) { return fail(GEMM_EUNSUPPORTED, "not built"); }
int gemm_serve_footprint(const gemm_problem_t *, uint64_t *) { return fail(GEMM_EUNSUPPORTED, "not built"); }
int gemm_serve_create(const gemm_serve_config_t *, void **) { return fail(GEMM_EUNSUPPORTED, "not built"); }
int gemm_serve_submit(void *, const gemm_problem_t *, uint64_t, uint64_t *) { return fail(GEMM_EUNSUPPORTED, "not built"); }
int gemm_serve_poll(void *, uint64_t, gemm_serve_result_t *) { return fail(GEMM_EUNSUPPORTED, "not built"); }
int gemm_serve_drain(void *) { return fail(GEMM_EUNSUPPORTED, "not built"); }
int gemm_serve_stats(void *, gemm_serve_stats_t *) { return fail(GEMM_EUNSUPPORTED, "not built"); }
int gemm_serve_destroy(void *) { return fail(GEMM_EUNSUPPORTED, "not built"); }
}
