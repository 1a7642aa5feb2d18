// Batched ST-HOSVD of many small 3-way blocks in one persistent launch.
#include "atc_internal.hpp"

extern "C" {

atc_status atc_batch_plan_create(const int32_t* dims, int64_t nblocks, const atc_sthosvd_opts* opts,
                                 atc_batch_plan** plan) {
    (void)dims;
    (void)nblocks;
    (void)opts;
    if (plan) *plan = nullptr;
    return ATC_ERR_UNSUPPORTED;
}

void atc_batch_plan_destroy(atc_batch_plan* plan) { (void)plan; }

atc_status atc_batch_plan_info(const atc_batch_plan* plan, int64_t* input_elems, int64_t* core_elems,
                               int64_t* factor_elems, size_t* workspace_bytes) {
    (void)plan;
    (void)input_elems;
    (void)core_elems;
    (void)factor_elems;
    (void)workspace_bytes;
    return ATC_ERR_UNSUPPORTED;
}

atc_status atc_batch_plan_offsets(const atc_batch_plan* plan, int64_t* input_off, int64_t* core_off,
                                  int64_t* factor_off) {
    (void)plan;
    (void)input_off;
    (void)core_off;
    (void)factor_off;
    return ATC_ERR_UNSUPPORTED;
}

atc_status atc_sthosvd_batched(atc_batch_plan* plan, const float* arena, float* core_arena, float* factor_arena,
                               atc_block_result* results, void* workspace, size_t workspace_bytes, void* stream) {
    (void)plan;
    (void)arena;
    (void)core_arena;
    (void)factor_arena;
    (void)results;
    (void)workspace;
    (void)workspace_bytes;
    (void)stream;
    return ATC_ERR_UNSUPPORTED;
}

atc_status atc_batch_autotune(atc_batch_plan* plan, const float* arena, float* core_arena, float* factor_arena,
                              atc_block_result* results, void* workspace, size_t workspace_bytes, void* stream,
                              int32_t reps, const char* cache_path, int32_t* out_choice) {
    (void)plan;
    (void)arena;
    (void)core_arena;
    (void)factor_arena;
    (void)results;
    (void)workspace;
    (void)workspace_bytes;
    (void)stream;
    (void)reps;
    (void)cache_path;
    (void)out_choice;
    return ATC_ERR_UNSUPPORTED;
}

atc_status atc_batch_graph_create(atc_batch_plan* plan, const float* arena, float* core_arena, float* factor_arena,
                                  atc_block_result* results, void* workspace, size_t workspace_bytes, void* stream,
                                  atc_graph** graph) {
    (void)plan;
    (void)arena;
    (void)core_arena;
    (void)factor_arena;
    (void)results;
    (void)workspace;
    (void)workspace_bytes;
    (void)stream;
    if (graph) *graph = nullptr;
    return ATC_ERR_UNSUPPORTED;
}

atc_status atc_graph_launch(atc_graph* graph, void* stream) {
    (void)graph;
    (void)stream;
    return ATC_ERR_UNSUPPORTED;
}

void atc_graph_destroy(atc_graph* graph) { (void)graph; }

}  // extern "C"
