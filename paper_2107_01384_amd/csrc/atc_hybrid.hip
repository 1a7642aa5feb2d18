// The quantization half of the hybrid truncation (Section 4.1.3) as one C
// call on the caller's stream: Householder form and signs of every factor
// (supplement S.2), the core quantized and decoded (Sections 3.3, 4.2, 4.3),
// its slice norms, then every factor weighted, quantized, decoded, rebuilt and
// its error term taken (eq. total_error_approximation).  The factors share
// each launch (one workgroup or grid slice per factor), so the d chains of
// small kernels cost one chain of launches; every buffer comes from the
// caller (outputs) or from one caller workspace.
#include <algorithm>
#include <cmath>

#include "atc_internal.hpp"

namespace atc {
namespace {

size_t align_ws(size_t b) { return (b + 255) & ~(size_t)255; }

struct WsCarve {
    char* base = nullptr;
    size_t off = 0;
    void* take(size_t bytes) {
        void* p = base ? base + off : nullptr;
        off += align_ws(bytes);
        return p;
    }
};

int64_t entries_of(int64_t n, int64_t r) { return n * r - r * (r + 1) / 2; }

// dst = src (bytes, 4-byte multiple) and *flag = 0, as one small kernel on the stream
__global__ void k_hy_copy(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, int64_t words,
                          int32_t* __restrict__ flag) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) *flag = 0;
    for (int64_t i = i0; i < words; i += (int64_t)gridDim.x * blockDim.x) dst[i] = src[i];
}

// workspace layout: the signed core, the core's quantization and decoding
// workspaces, then per factor its Householder, quantization and decoding
// workspaces and its decoded entries
struct HybridWs {
    void* signed_core;
    void* qws_core;
    size_t qws_core_b;
    void* dqws_core;
    size_t dqws_core_b;
    void* hws[ATC_MAX_DIMS];
    size_t hws_b[ATC_MAX_DIMS];
    void* qws[ATC_MAX_DIMS];
    size_t qws_b[ATC_MAX_DIMS];
    void* dqws[ATC_MAX_DIMS];
    size_t dqws_b[ATC_MAX_DIMS];
    double* cq[ATC_MAX_DIMS];
};

size_t carve_hybrid(const atc_shape* cs, const int64_t* n, int32_t block_len, char* base, HybridWs* w) {
    WsCarve c;
    c.base = base;
    const int d = cs->ndim;
    int64_t total = 1;
    for (int k = 0; k < d; ++k) total *= cs->dims[k];
    const size_t esz = cs->dtype == ATC_F64 ? 8 : 4;
    HybridWs h{};
    h.signed_core = c.take((size_t)total * esz);
    h.qws_core_b = atc_quantize_workspace_size(total, block_len);
    h.qws_core = c.take(h.qws_core_b);
    h.dqws_core_b = atc_dequantize_workspace_size(total, block_len);
    h.dqws_core = c.take(h.dqws_core_b);
    for (int k = 0; k < d; ++k) {
        const int64_t r = cs->dims[k], e = entries_of(n[k], r);
        h.hws_b[k] = atc_householder_workspace_size(n[k], r);
        h.hws[k] = c.take(h.hws_b[k]);
        h.qws_b[k] = e > 0 ? atc_quantize_workspace_size(e, block_len) : 0;
        h.qws[k] = c.take(h.qws_b[k]);
        h.dqws_b[k] = e > 0 ? atc_dequantize_workspace_size(e, block_len) : 0;
        h.dqws[k] = c.take(h.dqws_b[k]);
        h.cq[k] = (double*)c.take((size_t)(e > 0 ? e : 1) * sizeof(double));
    }
    if (w) *w = h;
    return c.off;
}

atc_status hy_fail(atc_status s, const char* msg) {
    set_last_error(msg);
    return s;
}

atc_status check_hybrid(const atc_shape* cs, const int64_t* n, int32_t block_len) {
    if (!cs || !n) return hy_fail(ATC_ERR_INVALID_ARGUMENT, "core_shape and n must be non-NULL");
    if (cs->ndim < 1 || cs->ndim > ATC_MAX_DIMS) return hy_fail(ATC_ERR_INVALID_ARGUMENT, "bad ndim");
    if (cs->dtype != ATC_F32 && cs->dtype != ATC_F64) return hy_fail(ATC_ERR_INVALID_ARGUMENT, "unknown dtype");
    if (block_len < 1 || block_len > ATC_QUANT_MAX_BLOCK) return hy_fail(ATC_ERR_INVALID_ARGUMENT, "block_len out of range");
    for (int k = 0; k < cs->ndim; ++k) {
        if (cs->dims[k] < 1 || n[k] < cs->dims[k]) return hy_fail(ATC_ERR_INVALID_ARGUMENT, "need 1 <= r_k <= n_k");
        if (atc_householder_workspace_size(n[k], cs->dims[k]) == 0)
            return hy_fail(ATC_ERR_UNSUPPORTED, "factor larger than 4096 x 256");
    }
    return ATC_OK;
}

}  // namespace
}  // namespace atc

using namespace atc;

extern "C" {

size_t atc_hybrid_workspace_size(const atc_shape* core_shape, const int64_t* n, int32_t block_len) {
    if (check_hybrid(core_shape, n, block_len) != ATC_OK) return 0;
    return carve_hybrid(core_shape, n, block_len, nullptr, nullptr);
}

atc_status atc_hybrid_quantize(const void* core, const atc_shape* core_shape, const void* const* factors,
                               const int64_t* n, double core_target_sse, double factor_target_sse,
                               int32_t block_len, const atc_hybrid_out* out, void* workspace,
                               size_t workspace_bytes, void* stream) {
    atc_status s = check_hybrid(core_shape, n, block_len);
    if (s != ATC_OK) return s;
    if (!core || !factors || !out || !workspace)
        return hy_fail(ATC_ERR_INVALID_ARGUMENT, "core, factors, out and workspace must be non-NULL");
    if (std::isnan(core_target_sse) || std::isinf(core_target_sse) || std::isnan(factor_target_sse) ||
        std::isinf(factor_target_sse))
        return hy_fail(ATC_ERR_INVALID_ARGUMENT, "the targets must be finite");
    const int d = core_shape->ndim;
    if (!out->core_enc || !out->core_info || !out->core_q || !out->sigma2 || !out->signs || !out->factor_term ||
        !out->status)
        return hy_fail(ATC_ERR_INVALID_ARGUMENT, "an output buffer is NULL");
    for (int k = 0; k < d; ++k) {
        if (!factors[k] || !out->factor_signed[k] || !out->factor_coef[k] || !out->factor_q[k])
            return hy_fail(ATC_ERR_INVALID_ARGUMENT, "a factor buffer is NULL");
        if (entries_of(n[k], core_shape->dims[k]) > 0 && (!out->factor_enc[k] || !out->factor_info[k]))
            return hy_fail(ATC_ERR_INVALID_ARGUMENT, "a factor stream buffer is NULL");
    }
    const size_t need = carve_hybrid(core_shape, n, block_len, nullptr, nullptr);
    if (workspace_bytes < need) return hy_fail(ATC_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
    HybridWs w;
    carve_hybrid(core_shape, n, block_len, (char*)workspace, &w);
    hipStream_t st = (hipStream_t)stream;
    const int32_t dt = core_shape->dtype;
    const int f64 = dt == ATC_F64;
    const size_t esz = f64 ? 8 : 4;
    int64_t total = 1, off[ATC_MAX_DIMS];
    for (int k = 0; k < d; ++k) {
        off[k] = k == 0 ? 0 : off[k - 1] + core_shape->dims[k - 1];
        total *= core_shape->dims[k];
    }
#define HY_HIP(x, what)                                              \
    do {                                                             \
        if ((x) != hipSuccess) return hy_fail(ATC_ERR_DEVICE, what); \
    } while (0)
    // reflectors and column signs of every factor (supplement S.2), unweighted
    FactorTask ft[ATC_MAX_DIMS] = {};
    for (int k = 0; k < d; ++k) {
        ft[k].n = n[k];
        ft[k].r = (int)core_shape->dims[k];
        ft[k].U = factors[k];
        ft[k].coef = out->factor_coef[k];
        ft[k].signs = out->signs + off[k];
        ft[k].Uprime = out->factor_signed[k];
        ft[k].ws = (double*)w.hws[k];
    }
    HY_HIP(householder_encode_batch(ft, d, f64, st), "Householder form of the factors failed");
    // the core with its slices flipped by the signs, quantized and decoded; its slice norms
    {
        const int64_t words = (int64_t)(total * esz / 4);
        const unsigned g = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, ceil_div(words, 256)));
        hipLaunchKernelGGL(k_hy_copy, dim3(g), dim3(256), 0, st, (const uint32_t*)core, (uint32_t*)w.signed_core,
                           words, out->status);
        HY_HIP(hipGetLastError(), "copy of the core failed");
    }
    if ((s = atc_core_apply_signs(w.signed_core, core_shape, out->signs, st)) != ATC_OK) return s;
    const QuantTask qc{w.signed_core, total, core_target_sse, out->core_enc, atc_quantize_max_words(total, block_len),
                       out->core_info, w.qws_core};
    HY_HIP(quantize_batch(&qc, 1, f64, block_len, st), "quantization of the core failed");
    const DequantTask dc{out->core_enc, total, out->core_q, out->status, w.dqws_core};
    HY_HIP(dequantize_batch(&dc, 1, f64, block_len, st), "decoding of the core failed");
    if ((s = atc_core_slice_norms(out->core_q, core_shape, out->sigma2, st)) != ATC_OK) return s;
    // every factor: entries weighted in place, quantized, decoded, the factor
    // rebuilt from them, its error term
    QuantTask qf[ATC_MAX_DIMS];
    DequantTask df[ATC_MAX_DIMS];
    int nq = 0;
    for (int k = 0; k < d; ++k) {
        const int64_t e = entries_of(n[k], core_shape->dims[k]);
        ft[k].s2 = out->sigma2 + off[k];
        ft[k].entries = out->factor_coef[k];
        if (e > 0) {
            qf[nq] = QuantTask{out->factor_coef[k], e, factor_target_sse, out->factor_enc[k],
                               atc_quantize_max_words(e, block_len), out->factor_info[k], w.qws[k]};
            df[nq] = DequantTask{out->factor_enc[k], e, w.cq[k], out->status, w.dqws[k]};
            ft[k].entries = w.cq[k];
            ++nq;
        }
        ft[k].U = out->factor_signed[k];
        ft[k].Uq = out->factor_q[k];
        ft[k].err = out->factor_term + k;
    }
    HY_HIP(householder_weight_batch(ft, d, st), "weighting of the factors failed");
    if (nq > 0) {
        HY_HIP(quantize_batch(qf, nq, 1, block_len, st), "quantization of the factors failed");
        HY_HIP(dequantize_batch(df, nq, 1, block_len, st), "decoding of the factors failed");
    }
    HY_HIP(householder_decode_batch(ft, d, f64, st), "rebuilding the factors failed");
    HY_HIP(factor_error_batch(ft, d, f64, st), "factor error terms failed");
#undef HY_HIP
    return ATC_OK;
}

}  // extern "C"
