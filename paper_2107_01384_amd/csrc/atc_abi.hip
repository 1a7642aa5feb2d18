// C ABI of libatc: argument checks, workspace carving and the host-side
// sequencing of the per-mode kernels.  No exception leaves this file.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "atc_internal.hpp"

using namespace atc;

namespace {

thread_local std::string g_last_error;

atc_status fail(atc_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define HIP_TRY(expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(ATC_ERR_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                     \
    } while (0)

constexpr int MAX_MODE = 4096;       // longest mode the eigensolvers accept
constexpr int SUBSPACE_M = 64;       // subspace size of the leading-eigenpair path
constexpr int SUBSPACE_ITERS = 2;    // power steps before the Rayleigh-Ritz projection
constexpr int SUBSPACE_GUARD = 8;    // Ritz pairs the chosen rank must leave unused
constexpr int S32_RANKS = 32;        // Ritz pairs of the m = 32 subspace path
constexpr int DEFAULT_SWEEPS = 60;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Carver {
    size_t off = 0;
    char* base = nullptr;
    void* take(size_t bytes) {
        void* p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    }
};

int64_t prod(const int64_t* d, int a, int b) {
    int64_t p = 1;
    for (int i = a; i < b; ++i) p *= d[i];
    return p;
}

atc_status check_shape(const atc_shape* s) {
    if (!s) return fail(ATC_ERR_INVALID_ARGUMENT, "shape is NULL");
    if (s->ndim < 1 || s->ndim > ATC_MAX_DIMS)
        return fail(ATC_ERR_INVALID_ARGUMENT, "ndim %d outside [1, %d]", s->ndim, ATC_MAX_DIMS);
    if (s->dtype != ATC_F32 && s->dtype != ATC_F64) return fail(ATC_ERR_INVALID_ARGUMENT, "unknown dtype %d", s->dtype);
    double total = 1.0;
    for (int k = 0; k < s->ndim; ++k) {
        if (s->dims[k] < 1) return fail(ATC_ERR_INVALID_ARGUMENT, "dims[%d] = %lld < 1", k, (long long)s->dims[k]);
        total *= (double)s->dims[k];
    }
    if (total > 9.0e15) return fail(ATC_ERR_UNSUPPORTED, "tensor too large");
    return ATC_OK;
}

atc_status check_opts(const atc_shape* s, const atc_sthosvd_opts* o) {
    if (!o) return fail(ATC_ERR_INVALID_ARGUMENT, "opts is NULL");
    if (!(o->rel_error >= 0.0) || !std::isfinite(o->rel_error))
        return fail(ATC_ERR_INVALID_ARGUMENT, "rel_error must be finite and >= 0");
    if (!(o->rtmss >= 0.0 && o->rtmss <= 1.0)) return fail(ATC_ERR_INVALID_ARGUMENT, "rtmss must lie in [0, 1]");
    if (o->precision != ATC_PREC_NATIVE && o->precision != ATC_PREC_BF16X3 && o->precision != ATC_PREC_F64ACC)
        return fail(ATC_ERR_INVALID_ARGUMENT, "unknown precision %d", o->precision);
    if (o->precision == ATC_PREC_BF16X3 && s->dtype != ATC_F32)
        return fail(ATC_ERR_UNSUPPORTED, "BF16X3 precision needs float32 input");
    if (o->precision == ATC_PREC_F64ACC && s->dtype != ATC_F32)
        return fail(ATC_ERR_UNSUPPORTED, "F64ACC precision needs float32 input (float64 input is FP64 throughout)");
    if (o->rank_rule != ATC_RANK_ADAPTIVE && o->rank_rule != ATC_RANK_EQUAL)
        return fail(ATC_ERR_INVALID_ARGUMENT, "unknown rank rule %d", o->rank_rule);
    if (o->max_sweeps < 0) return fail(ATC_ERR_INVALID_ARGUMENT, "max_sweeps < 0");
    if (o->eig_path < 0 || o->eig_path > 2) return fail(ATC_ERR_INVALID_ARGUMENT, "eig_path must be 0, 1 or 2");
    if (o->has_order) {
        int seen[ATC_MAX_DIMS] = {0};
        for (int i = 0; i < s->ndim; ++i) {
            const int k = o->mode_order[i];
            if (k < 0 || k >= s->ndim || seen[k]) return fail(ATC_ERR_INVALID_ARGUMENT, "mode_order is not a permutation");
            seen[k] = 1;
        }
    }
    if (o->has_fixed_ranks) {
        for (int k = 0; k < s->ndim; ++k)
            if (o->fixed_ranks[k] < 1 || o->fixed_ranks[k] > s->dims[k])
                return fail(ATC_ERR_INVALID_ARGUMENT, "fixed_ranks[%d] outside [1, n_k]", k);
    }
    for (int k = 0; k < s->ndim; ++k)
        if (s->dims[k] > MAX_MODE) return fail(ATC_ERR_UNSUPPORTED, "mode %d longer than %d", k, MAX_MODE);
    if (o->no_host_wait && (!o->has_fixed_ranks || o->profile))
        return fail(ATC_ERR_INVALID_ARGUMENT, "no_host_wait needs fixed ranks and no profiling");
    if (o->no_host_wait && o->eig_path == 2)
        for (int k = 0; k < s->ndim; ++k)
            if (s->dims[k] > 64 && o->fixed_ranks[k] > SUBSPACE_M - SUBSPACE_GUARD)
                return fail(ATC_ERR_UNSUPPORTED, "mode %d: rank needs more than %d Ritz pairs", k,
                            SUBSPACE_M - SUBSPACE_GUARD);
    return ATC_OK;
}

void processing_order(const atc_shape* s, const atc_sthosvd_opts* o, int* order) {
    const int d = s->ndim;
    for (int i = 0; i < d; ++i) order[i] = o->has_order ? o->mode_order[i] : i;
    if (!o->has_order)  // Section 4.1.1: increasing mode length, stable
        std::stable_sort(order, order + d, [&](int a, int b) { return s->dims[a] < s->dims[b]; });
}

// Arithmetic of the Gram matrices
int prec_of(const atc_shape* s, const atc_sthosvd_opts* o) {
    if (s->dtype == ATC_F64) return PREC_F64;
    if (o->precision == ATC_PREC_F64ACC) return PREC_F64ACC;
    return o->precision == ATC_PREC_BF16X3 ? PREC_BF16X3 : PREC_F32;
}

// Arithmetic of the mode products (projections): F64ACC projects in FP32
int ttm_prec_of(int gram_prec) { return gram_prec == PREC_F64ACC ? PREC_F32 : gram_prec; }

// Precision guard of the Gram matrix.  A Gram matrix accumulated from FP32
// (or bf16x3) products carries rounding of a small multiple of
// u32 = 2^-24 times the energy of the tensor it is formed from.  That rounding
// has both signs, and in the trailing eigenvalues (true values far below it)
// the negative part is clamped away, so the discarded-energy sums the rank
// choice compares with the mode's budget come out biased upwards.  Measured on
// smooth fields the bias stays near 0.2 u32 |Y|^2 for contractions of a few
// thousand terms or more, and reaches several u32 |Y|^2 for short ones (the
// last modes of strongly truncated tensors, small blocks).  So a mode's Gram
// matrix is formed with FP64 accumulation instead (the 64-bit internal
// arithmetic of Section 5) when
//   * its budget share is below 2 u32 |Y|^2 (a tail error above a tenth of the
//     share), or
//   * its contraction is shorter than GUARD_MIN_TERMS terms (then n^2 K is
//     small and the FP64 matrix cores cost little).
// The projections keep the requested arithmetic.
constexpr double GUARD_RATIO = 0x1p-23;
constexpr int64_t GUARD_MIN_TERMS = 2048;

bool guard_upgrades(int gprec, double budget, double energy, int64_t terms) {
    if (gprec != PREC_F32 && gprec != PREC_BF16X3) return false;
    return !(budget >= GUARD_RATIO * energy) || terms < GUARD_MIN_TERMS;
}

int32_t abi_prec(int p) {
    return p == PREC_F64ACC ? ATC_PREC_F64ACC : p == PREC_BF16X3 ? ATC_PREC_BF16X3 : ATC_PREC_NATIVE;
}

size_t part_capacity(int nmax) {
    const size_t t = (size_t)ceil_div(nmax, TILE);
    const size_t one_split = t * t * TILE * TILE * sizeof(double);  // cross Gram: all tile pairs
    return std::max<size_t>((size_t)64 << 20, one_split);
}

struct SthosvdWs {
    void* buf[2];
    double* part;
    size_t part_cap;
    double* dpart;   // exact-diagonal partials of the tiled Gram kernel
    size_t dpart_cap;
    double* G;
    double* lam;
    double* V;
    double* jac;     // global Jacobi scratch
    double* sub;     // subspace scratch
    double* Mt64;
    float* Mt32;
    __bf16* Mth;
    __bf16* Mtl;
    QtOut qt;        // Q^T of the m = 32 basis (32 x n), mode-product operand
    SelectArgs wt;   // only its Wt* fields: the Ritz rotation operand (32 x 32)
    DevBook* book;
};

size_t carve_sthosvd(const atc_shape* s, char* base, SthosvdWs* w) {
    const int d = s->ndim;
    int64_t N = prod(s->dims, 0, d);
    int nmax = 1;
    for (int k = 0; k < d; ++k) nmax = std::max<int>(nmax, (int)s->dims[k]);
    const size_t esz = s->dtype == ATC_F64 ? 8 : 4;
    const size_t n2 = (size_t)nmax * nmax;
    const int mpad = nmax + (nmax & 1);
    Carver c;
    c.base = base;
    SthosvdWs t{};
    t.buf[0] = c.take(d > 1 ? (size_t)N * esz : 0);
    t.buf[1] = c.take(d > 2 ? (size_t)N * esz : 0);
    t.part_cap = part_capacity(nmax);
    t.part = (double*)c.take(t.part_cap);
    t.dpart_cap = (size_t)512 * nmax * sizeof(double);
    t.dpart = (double*)c.take(t.dpart_cap);
    t.G = (double*)c.take(n2 * 8);
    t.lam = (double*)c.take((size_t)nmax * 8);
    t.V = (double*)c.take(n2 * 8);
    t.jac = (double*)c.take(nmax > 64 ? (size_t)2 * mpad * mpad * 8 : 0);
    t.sub = (double*)c.take(nmax > 64 ? std::max({subspace_ws_doubles(nmax, SUBSPACE_M),
                                                  subspace32_ws_doubles(std::min(nmax, 512)),
                                                  subspace64b_ws_doubles(std::min(nmax, 512))}) * 8
                                      : 0);
    t.Mt64 = (double*)c.take(s->dtype == ATC_F64 ? n2 * 8 : 0);
    t.Mt32 = (float*)c.take(s->dtype == ATC_F32 ? n2 * 4 : 0);
    t.Mth = (__bf16*)c.take(s->dtype == ATC_F32 ? n2 * 2 : 0);
    t.Mtl = (__bf16*)c.take(s->dtype == ATC_F32 ? n2 * 2 : 0);
    // the split m = 32 path (modes of 65 .. 512 rows): Q^T and the rotation
    const size_t qn = nmax > 64 ? (size_t)S32_RANKS * std::min(nmax, 512) : 0;
    const size_t wn = nmax > 64 ? (size_t)S32_RANKS * S32_RANKS : 0;
    const bool d64 = s->dtype == ATC_F64;
    t.qt.t64 = (double*)c.take(d64 ? qn * 8 : 0);
    t.qt.t32 = (float*)c.take(d64 ? 0 : qn * 4);
    t.qt.th = (__bf16*)c.take(d64 ? 0 : qn * 2);
    t.qt.tl = (__bf16*)c.take(d64 ? 0 : qn * 2);
    t.wt.Wt64 = (double*)c.take(d64 ? wn * 8 : 0);
    t.wt.Wt32 = (float*)c.take(d64 ? 0 : wn * 4);
    t.wt.Wth = (__bf16*)c.take(d64 ? 0 : wn * 2);
    t.wt.Wtl = (__bf16*)c.take(d64 ? 0 : wn * 2);
    // a region of size 0 still has an address: the unused dtype's pointers
    // are cleared, since the kernels write every non-null one
    if (qn == 0 || !d64) {
        t.qt.t64 = nullptr;
        t.wt.Wt64 = nullptr;
    }
    if (qn == 0 || d64) {
        t.qt.t32 = nullptr;
        t.qt.th = t.qt.tl = nullptr;
        t.wt.Wt32 = nullptr;
        t.wt.Wth = t.wt.Wtl = nullptr;
    }
    t.book = (DevBook*)c.take(sizeof(DevBook));
    if (w) *w = t;
    return c.off;
}

// Start / end events of one call (created once per thread).  stop() records
// the end event; elapsed() is valid once the stream has been synchronised.
struct StreamTimer {
    hipEvent_t a = nullptr, b = nullptr;
    bool ok = false;
    bool start(hipStream_t st) {
        if (!a && (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)) return ok = false;
        return ok = hipEventRecord(a, st) == hipSuccess;
    }
    void stop(hipStream_t st) { ok = ok && hipEventRecord(b, st) == hipSuccess; }
    void release() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        a = b = nullptr;
        ok = false;
    }
    double elapsed() const {
        float ms = 0.f;
        if (ok) (void)hipEventElapsedTime(&ms, a, b);
        return ms;
    }
};
thread_local StreamTimer g_timer;


// Per-mode phase events (Gram, reduction, eigensolver + rank choice, mode
// product), created once per thread and reused.
struct PhaseEvents {
    static constexpr int PER_MODE = 5;
    hipEvent_t ev[ATC_MAX_DIMS][PER_MODE];
    bool ready = false;
    bool init() {
        if (ready) return true;
        for (int i = 0; i < ATC_MAX_DIMS; ++i)
            for (int j = 0; j < PER_MODE; ++j)
                if (hipEventCreate(&ev[i][j]) != hipSuccess) return false;
        ready = true;
        return true;
    }
    void release() {
        if (!ready) return;
        for (int i = 0; i < ATC_MAX_DIMS; ++i)
            for (int j = 0; j < PER_MODE; ++j) (void)hipEventDestroy(ev[i][j]);
        ready = false;
    }
};
thread_local PhaseEvents g_phase;

// Pinned host word block the selection kernels report into, so that the host
// learns each mode's rank without draining the stream (see wait_selection).
struct PinnedFlags {
    HostFlags* h = nullptr;  // host view
    HostFlags* d = nullptr;  // device view
    int32_t seq = 0;
    bool init() {
        if (h) return true;
        void* p = nullptr;
        if (hipHostMalloc(&p, sizeof(HostFlags), hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) return false;
        void* dp = nullptr;
        if (hipHostGetDevicePointer(&dp, p, 0) != hipSuccess) {
            (void)hipHostFree(p);
            return false;
        }
        h = (HostFlags*)p;
        d = (HostFlags*)dp;
        memset(h, 0, sizeof(*h));
        return true;
    }
    void release() {
        if (h) (void)hipHostFree(h);
        h = d = nullptr;
    }
};
thread_local PinnedFlags g_flags;

// A second stream per device and two events, for the split m = 32 solver:
// the mode product by the basis runs there beside the Rayleigh-Ritz step on
// the caller's stream.  Made on first use (default priority), kept until
// atc_finalize.  (Giving the Rayleigh-Ritz step a stream of its own, on CUs
// that the product's stream masks off, was slower: it did not shorten that
// step, and each extra queue with a pending event wait delayed the next
// dispatches by tens of microseconds.)
struct SideQueue {
    static constexpr int MAXDEV = 16;
    struct Dev {
        hipStream_t ttm = nullptr;
        hipEvent_t basis = nullptr, proj = nullptr;
        bool tried = false, ok = false;
    };
    Dev dv[MAXDEV];
    Dev* get() {
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAXDEV) return nullptr;
        Dev& q = dv[dev];
        if (!q.tried) {
            q.tried = true;
            q.ok = hipStreamCreateWithPriority(&q.ttm, hipStreamNonBlocking, 0) == hipSuccess &&
                   hipEventCreateWithFlags(&q.basis, hipEventDisableTiming) == hipSuccess &&
                   hipEventCreateWithFlags(&q.proj, hipEventDisableTiming) == hipSuccess;
        }
        return q.ok ? &q : nullptr;
    }
    void release() {
        for (int i = 0; i < MAXDEV; ++i) {
            Dev& q = dv[i];
            if (q.basis) (void)hipEventDestroy(q.basis);
            if (q.proj) (void)hipEventDestroy(q.proj);
            if (q.ttm) (void)hipStreamDestroy(q.ttm);
            q = Dev{};
        }
    }
};
thread_local SideQueue g_side;

// Smallest tensor (bytes) whose mode product takes the split m = 32 solver;
// ATC_SPLIT_MIN_BYTES in the environment (read at every call) overrides it.
size_t split_min_bytes() {
    const char* e = getenv("ATC_SPLIT_MIN_BYTES");
    return e ? (size_t)strtoull(e, nullptr, 10) : ((size_t)64 << 20);
}

// ATC_NO_OVERLAP=1 in the environment (read at every call) keeps the m = 32
// solver in one launch (no side stream).
bool overlap_enabled() {
    const char* e = getenv("ATC_NO_OVERLAP");
    return !(e && e[0] == '1');
}

// Spins until the selection kernel reports sequence number `expect`; gives up
// with an error when the stream has drained without the report.
hipError_t wait_selection(const volatile HostFlags* f, int32_t expect, hipStream_t st) {
    for (uint64_t it = 0;; ++it) {
        if (__atomic_load_n(&f->seq, __ATOMIC_ACQUIRE) == expect) return hipSuccess;
        if ((it & 1023) == 1023) {
            const hipError_t q = hipStreamQuery(st);
            if (q == hipSuccess) return __atomic_load_n(&f->seq, __ATOMIC_ACQUIRE) == expect ? hipSuccess : hipErrorUnknown;
            if (q != hipErrorNotReady) return q;
        }
        __builtin_ia32_pause();
    }
}

// No-host-wait calls: the outcome of one mode's eigensolver and rank choice
// folded into the book's status (the first failure stays).
__global__ void k_book_check(DevBook* bk) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (bk->status != 0) return;
    if (bk->need_dense) bk->status = ATC_ERR_INTERNAL;
    else if (!bk->eig_ok) bk->status = ATC_ERR_NOT_CONVERGED;
}

double event_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1.0;
    return ms;
}

}  // namespace

namespace atc {
void set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }
}  // namespace atc

// The entry points below keep the C linkage of their declarations in atc.h.

void atc_default_opts(atc_sthosvd_opts* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->rel_error = 1e-3;
    o->rtmss = 1.0;
    o->precision = ATC_PREC_NATIVE;
    o->rank_rule = ATC_RANK_ADAPTIVE;
}

size_t atc_sthosvd_workspace_size(const atc_shape* shape, const atc_sthosvd_opts* opts) {
    if (check_shape(shape) != ATC_OK || check_opts(shape, opts) != ATC_OK) return 0;
    return carve_sthosvd(shape, nullptr, nullptr);
}

atc_status atc_sthosvd(const void* x, const atc_shape* shape, const atc_sthosvd_opts* opts, void* core,
                       void* const* factors, atc_result* result, void* workspace, size_t workspace_bytes,
                       void* stream) {
    atc_status s;
    if ((s = check_shape(shape)) != ATC_OK) return s;
    if ((s = check_opts(shape, opts)) != ATC_OK) return s;
    if (!x || !core || !factors) return fail(ATC_ERR_INVALID_ARGUMENT, "x, core and factors must be non-NULL");
    const int d = shape->ndim;
    for (int k = 0; k < d; ++k)
        if (!factors[k]) return fail(ATC_ERR_INVALID_ARGUMENT, "factors[%d] is NULL", k);
    const size_t need = carve_sthosvd(shape, nullptr, nullptr);
    if (!workspace || workspace_bytes < need)
        return fail(ATC_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", workspace_bytes, need);
    SthosvdWs w;
    carve_sthosvd(shape, (char*)workspace, &w);
    hipStream_t st = (hipStream_t)stream;
    const int gprec = prec_of(shape, opts);
    const int prec = ttm_prec_of(gprec);  // projections (and their operand copies)
    const bool f64 = shape->dtype == ATC_F64;
    const int max_sweeps = opts->max_sweeps > 0 ? opts->max_sweeps : DEFAULT_SWEEPS;
    int order[ATC_MAX_DIMS];
    processing_order(shape, opts, order);

    const bool prof = opts->profile != 0;
    if (prof && !g_phase.init()) return fail(ATC_ERR_DEVICE, "hipEventCreate failed");
    auto mark = [&](int i, int j) -> hipError_t { return prof ? hipEventRecord(g_phase.ev[i][j], st) : hipSuccess; };

    if (prof) g_timer.start(st);
    const bool nowait = opts->no_host_wait != 0;
    // no cooperative launch goes into a graph (its grid barriers need every
    // workgroup resident at once): under capture the eigensolvers run as
    // kernel chains, otherwise in their one-launch form
    bool coop_ok = true;
    if (nowait) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIP_TRY(hipStreamIsCapturing(st, &cs));
        coop_ok = cs == hipStreamCaptureStatusNone;
    }
    // cleared by a kernel (a memset node misbehaves in captured graphs)
    HIP_TRY(launch_zero(w.book, sizeof(DevBook), st));
    int64_t cur[ATC_MAX_DIMS];
    for (int k = 0; k < d; ++k) cur[k] = shape->dims[k];
    const void* src = x;
    HostFlags hf{};
    double rep_tail[ATC_MAX_DIMS] = {}, rep_budget[ATC_MAX_DIMS] = {}, rep_norm2 = 0.0, rep_used = 0.0;
    int32_t rep_sweeps[ATC_MAX_DIMS] = {};
    if (!g_flags.init()) return fail(ATC_ERR_DEVICE, "hipHostMalloc of the report block failed");
    int paths[ATC_MAX_DIMS] = {0};
    int lazy[ATC_MAX_DIMS], nlazy = 0;  // modes kept whole, rotated at the end
    bool wide_hint = false;             // the previous subspace mode needed m = 64
    int32_t gram_used[ATC_MAX_DIMS] = {};
    for (int i = 0; i < d; ++i) {
        const int k = order[i];
        const int64_t L = prod(cur, 0, k), R = prod(cur, k + 1, d);
        const int n = (int)cur[k];
        // this mode's budget share and the energy of the current tensor, both
        // relative to |A|^2 (known from the previous mode's report; the first
        // mode's share is S / d for either rule)
        int gprec_i = gprec;
        if (!opts->no_precision_guard && !opts->has_fixed_ranks) {
            const double S = opts->rtmss * opts->rel_error * opts->rel_error;
            double share = S / d, energy = 1.0;
            if (i > 0 && rep_norm2 > 0.0) {
                const double used = rep_used / rep_norm2;
                share = opts->rank_rule == ATC_RANK_EQUAL ? S / d : (S - used) / (d - i);
                energy = 1.0 - used;
            }
            if (guard_upgrades(gprec, share, energy, L * R)) gprec_i = PREC_F64ACC;
        }
        gram_used[k] = abi_prec(gprec_i);
        GramKcPlan kp{};
        if (gram_kc_applicable(gprec_i, R)) kp = gram_kc_plan(gprec_i, L, n, R, w.part_cap, w.dpart_cap);
        if (kp.ok) {
            HIP_TRY(mark(i, 0));
            HIP_TRY(launch_gram_kc(gprec_i, kp, (const float*)src, (float*)w.part, w.dpart, st));
            HIP_TRY(mark(i, 1));
            HIP_TRY(launch_gram_kc_reduce(kp, (const float*)w.part, w.dpart, w.G, st));
            HIP_TRY(mark(i, 2));
        } else if (gram_tall_applicable(gprec_i, n, R) && reinterpret_cast<uintptr_t>(src) % 16 == 0) {
            // short last mode: FP64 MFMA over rows streamed through LDS (reduction included)
            gram_used[k] = ATC_PREC_F64ACC;
            HIP_TRY(mark(i, 0));
            HIP_TRY(launch_gram_tall((const float*)src, n, L, w.part, w.part_cap, w.G, st));
            HIP_TRY(mark(i, 1));
            HIP_TRY(mark(i, 2));
        } else {
            const GramPlan gp = gram_plan(gprec_i, L, n, n, R, true, w.part_cap);
            HIP_TRY(mark(i, 0));
            HIP_TRY(launch_gram(gprec_i, gp, src, src, w.part, st));
            HIP_TRY(mark(i, 1));
            HIP_TRY(launch_gram_reduce(gp, w.part, w.G, st));
            HIP_TRY(mark(i, 2));
        }

        SelectArgs sa{};
        sa.G = w.G;
        sa.n = n;
        sa.lam = w.lam;
        sa.V = w.V;
        sa.pos = i;
        sa.d = d;
        sa.k = k;
        sa.rule = opts->rank_rule;
        sa.fixed_rank = opts->has_fixed_ranks ? opts->fixed_ranks[k] : -1;
        sa.rtmss = opts->rtmss;
        sa.eps2 = opts->rel_error * opts->rel_error;
        sa.book = w.book;
        sa.ufac = factors[k];
        sa.ufac_f64 = f64 ? 1 : 0;
        sa.Mt64 = f64 ? w.Mt64 : nullptr;
        sa.Mt32 = f64 ? nullptr : w.Mt32;
        sa.Mth = prec == PREC_BF16X3 ? w.Mth : nullptr;
        sa.Mtl = prec == PREC_BF16X3 ? w.Mtl : nullptr;
        sa.guard = SUBSPACE_GUARD;
        // a no-host-wait call reports nothing to the host: its kernels may
        // still run while a later call of this thread waits on the report block
        sa.hflags = nowait ? nullptr : g_flags.d;
        sa.publish_late = i == d - 1 ? 1 : 0;
        int32_t* sweeps_dev = &w.book->sweeps[k];
        int32_t* ok_dev = &w.book->eig_ok;

        // eigensolver ladder: n <= 64 dense in LDS; otherwise subspace m = 32,
        // then m = 64, then dense in global memory, each step taken only when the
        // chosen rank does not leave `guard` unused Ritz pairs.  FP64 input keeps
        // the dense solver (the subspace iteration is accurate to what an
        // FP32-grade Gram matrix carries, not to FP64) unless eig_path forces it.
        const int32_t zero = 0;
        const bool dense_first = n <= 64 || opts->eig_path == 1 || (f64 && opts->eig_path != 2);
        if (nowait) {
            // the eigensolver from the fixed rank, ordinary launches only; the
            // outcome goes to the book's status (atc_sthosvd_finish reads it)
            const int r = opts->fixed_ranks[k];
            sa.seq = ++g_flags.seq;
            void* const dst_nw = (i == d - 1) ? core : (src == w.buf[0] ? w.buf[1] : w.buf[0]);
            // the split form of the m = 32 solver, as below, with the rotation
            // queued at once (its rows come from the device-side rank, 0 when
            // the selection failed, which the record's status reports)
            const size_t esz_nw = f64 ? 8 : 4;
            const size_t qoff_nw = ((size_t)L * (S32_RANKS - SUBSPACE_GUARD) * R * esz_nw + 255) & ~(size_t)255;
            const bool split_nw = coop_ok && !dense_first && r <= S32_RANKS - SUBSPACE_GUARD && i + 1 < d &&
                                  (size_t)L * n * R * esz_nw >= split_min_bytes() && (w.qt.t64 || w.qt.t32) &&
                                  overlap_enabled() && dst_nw != core &&
                                  qoff_nw + (size_t)L * S32_RANKS * R * esz_nw <=
                                      (size_t)prod(shape->dims, 0, d) * esz_nw &&
                                  subspace32_split_available(n);
            SideQueue::Dev* sq_nw = split_nw ? g_side.get() : nullptr;
            if (sq_nw) {
                sa.ldv = 32;
                sa.ncand = 32;
                sa.subspace = 1;
                paths[k] = 2;
                HIP_TRY(run_subspace32_basis(w.G, n, SUBSPACE_ITERS, w.sub, sa, w.qt, st));
                void* yq = (char*)dst_nw + qoff_nw;
                const TtmPlan tq = ttm_plan(prec, L, n, R, S32_RANKS);
                HIP_TRY(hipEventRecord(sq_nw->basis, st));
                HIP_TRY(hipStreamWaitEvent(sq_nw->ttm, sq_nw->basis, 0));
                HIP_TRY(launch_ttm(prec, tq, src, f64 ? (const void*)w.qt.t64 : (const void*)w.qt.t32, w.qt.th,
                                   w.qt.tl, yq, sq_nw->ttm, split_rows_dev(w.sub, n)));
                HIP_TRY(hipEventRecord(sq_nw->proj, sq_nw->ttm));
                SelectArgs sr = sa;
                sr.Wt64 = w.wt.Wt64;
                sr.Wt32 = w.wt.Wt32;
                sr.Wth = prec == PREC_BF16X3 ? w.wt.Wth : nullptr;
                sr.Wtl = prec == PREC_BF16X3 ? w.wt.Wtl : nullptr;
                sr.Mt64 = nullptr;
                sr.Mt32 = nullptr;
                sr.Mth = sr.Mtl = nullptr;
                HIP_TRY(run_rr32_select(n, SUBSPACE_ITERS, max_sweeps, w.sub, sr, st));
                hipLaunchKernelGGL(k_book_check, dim3(1), dim3(64), 0, st, w.book);
                HIP_TRY(hipGetLastError());
                HIP_TRY(hipStreamWaitEvent(st, sq_nw->proj, 0));
                const TtmPlan tw = ttm_plan(prec, L, S32_RANKS, R, S32_RANKS - SUBSPACE_GUARD);
                HIP_TRY(launch_ttm(prec, tw, yq, f64 ? (const void*)w.wt.Wt64 : (const void*)w.wt.Wt32, sr.Wth,
                                   sr.Wtl, dst_nw, st, &w.book->rank[k], (float*)w.part, w.part_cap));
                cur[k] = r;
                src = dst_nw;
                continue;
            }
            if (!dense_first && r <= S32_RANKS - SUBSPACE_GUARD && subspace32_available(n)) {
                sa.ldv = 32;
                sa.ncand = 32;
                sa.subspace = 1;
                paths[k] = 2;
                HIP_TRY(run_subspace32_select(w.G, n, SUBSPACE_ITERS, max_sweeps, w.sub, sa, st, coop_ok));
            } else if (!dense_first && r <= SUBSPACE_M - SUBSPACE_GUARD && subspace32_available(n)) {
                sa.ldv = 64;
                sa.ncand = 64;
                sa.subspace = 1;
                sa.lam = w.lam;
                sa.V = w.V;
                paths[k] = 2;
                HIP_TRY(run_subspace64_select(w.G, n, max_sweeps, w.sub, w.lam, w.V, sweeps_dev, ok_dev, sa, st,
                                              coop_ok));
            } else {
                if (n <= 64) HIP_TRY(launch_eig_jacobi_lds(w.G, n, n, max_sweeps, w.lam, w.V, n, sweeps_dev, ok_dev, st));
                else HIP_TRY(launch_eig_jacobi_global(w.G, n, max_sweeps, w.jac, w.lam, w.V, sweeps_dev, ok_dev, st));
                sa.ldv = n;
                sa.ncand = n;
                sa.subspace = 0;
                paths[k] = 1;
                HIP_TRY(launch_select_factor(sa, st));
            }
            hipLaunchKernelGGL(k_book_check, dim3(1), dim3(64), 0, st, w.book);
            HIP_TRY(hipGetLastError());
            cur[k] = r;
            if (r == n && i + 1 < d) {
                lazy[nlazy++] = k;   // rotated on the final core, as below
                continue;
            }
            const TtmPlan tp = ttm_plan(prec, L, n, R, r);
            HIP_TRY(launch_ttm(prec, tp, src, f64 ? (const void*)w.Mt64 : (const void*)w.Mt32, w.Mth, w.Mtl, dst_nw,
                               st, nullptr, (float*)w.part, w.part_cap));
            src = dst_nw;
            continue;
        }
        // a mode after one whose rank needed the m = 64 subspace starts there
        // (ranks of neighbouring modes tend to be alike; m = 64 is never less
        // accurate, only slower when m = 32 would have done)
        int attempt = dense_first ? 2 : (wide_hint && subspace32_available(n) ? 1 : 0);
        const void* M = f64 ? (const void*)w.Mt64 : (const void*)w.Mt32;
        void* const dst = (i == d - 1) ? core : (src == w.buf[0] ? w.buf[1] : w.buf[0]);
        bool queued = false;  // mode product queued with the device-side rank
        // split form: the rotation, queued once the host knows the rank fits;
        // the side stream's product must end before anything else writes dst
        SideQueue::Dev* split_q = nullptr;
        void* split_yq = nullptr;
        SelectArgs split_sr{};
        for (;; ++attempt) {
            bool selected = false;
            sa.seq = ++g_flags.seq;
            // the split form: basis, then the mode product by Q^T on the side
            // stream beside the Rayleigh-Ritz step, then the rotation by W_r^T
            // into dst (the projection by Q^T sits after dst's rows in the same
            // buffer; a later mode of a wider rank than 24 never takes this path)
            const size_t esz_ = f64 ? 8 : 4;
            const size_t qoff = ((size_t)L * (S32_RANKS - SUBSPACE_GUARD) * R * esz_ + 255) & ~(size_t)255;
            // worth it when the mode product by the basis is long enough to hide
            // the Rayleigh-Ritz step behind it (splitting costs ~20 us: a second
            // launch, and the Rayleigh-Ritz products formed by one workgroup)
            const bool split_pays = (size_t)L * n * R * esz_ >= split_min_bytes();
            const bool split_fits = i + 1 < d && split_pays && (w.qt.t64 || w.qt.t32) && overlap_enabled() &&
                                    dst != core &&
                                    qoff + (size_t)L * S32_RANKS * R * esz_ <= (size_t)prod(shape->dims, 0, d) * esz_;
            SideQueue::Dev* sq = nullptr;
            if (attempt == 0 && split_fits && subspace32_split_available(n) && (sq = g_side.get()) != nullptr) {
                sa.ldv = 32;
                sa.ncand = 32;
                sa.subspace = 1;
                paths[k] = 2;
                HIP_TRY(run_subspace32_basis(w.G, n, SUBSPACE_ITERS, w.sub, sa, w.qt, st));
                void* yq = (char*)dst + qoff;
                const TtmPlan tq = ttm_plan(prec, L, n, R, S32_RANKS);
                HIP_TRY(hipEventRecord(sq->basis, st));
                HIP_TRY(hipStreamWaitEvent(sq->ttm, sq->basis, 0));
                HIP_TRY(launch_ttm(prec, tq, src, f64 ? (const void*)w.qt.t64 : (const void*)w.qt.t32, w.qt.th,
                                   w.qt.tl, yq, sq->ttm, split_rows_dev(w.sub, n)));
                HIP_TRY(hipEventRecord(sq->proj, sq->ttm));
                SelectArgs sr = sa;
                sr.Wt64 = w.wt.Wt64;
                sr.Wt32 = w.wt.Wt32;
                sr.Wth = prec == PREC_BF16X3 ? w.wt.Wth : nullptr;
                sr.Wtl = prec == PREC_BF16X3 ? w.wt.Wtl : nullptr;
                // U^T is not a mode-product operand on this path
                sr.Mt64 = nullptr;
                sr.Mt32 = nullptr;
                sr.Mth = sr.Mtl = nullptr;
                HIP_TRY(run_rr32_select(n, SUBSPACE_ITERS, max_sweeps, w.sub, sr, st));
                selected = true;
                HIP_TRY(mark(i, 3));
                split_q = sq;
                split_yq = yq;
                split_sr = sr;
            } else if (attempt == 0 && subspace32_available(n)) {
                sa.ldv = 32;
                sa.ncand = 32;
                sa.subspace = 1;
                paths[k] = 2;
                HIP_TRY(run_subspace32_select(w.G, n, SUBSPACE_ITERS, max_sweeps, w.sub, sa, st));
                selected = true;
                // the mode product with the rank the kernel chose, queued before the
                // host reads it (this path's ranks stay below 32 - guard < n, so
                // there is no deferred rotation); when the selection hands the
                // mode on, the rank slot holds 0 and the product writes nothing
                const TtmPlan tp = ttm_plan(prec, L, n, R, S32_RANKS - SUBSPACE_GUARD);
                HIP_TRY(mark(i, 3));
                HIP_TRY(launch_ttm(prec, tp, src, M, w.Mth, w.Mtl, dst, st, &w.book->rank[k], (float*)w.part,
                                   w.part_cap));
                HIP_TRY(mark(i, 4));
                queued = true;
            } else if (attempt == 1 && subspace32_available(n)) {
                sa.ldv = 64;
                sa.ncand = 64;
                sa.subspace = 1;
                sa.lam = w.lam;
                sa.V = w.V;
                paths[k] = 2;
                HIP_TRY(run_subspace64_select(w.G, n, max_sweeps, w.sub, w.lam, w.V, sweeps_dev, ok_dev, sa, st));
                selected = true;
            } else if (attempt < 2) {
                const int m = attempt == 0 ? std::min(SUBSPACE_M / 2, n) : std::min(SUBSPACE_M, n);
                HIP_TRY(run_subspace_eig(w.G, n, m, SUBSPACE_ITERS, max_sweeps, w.sub, w.lam, w.V, sweeps_dev, ok_dev,
                                         st));
                sa.ldv = m;
                sa.ncand = m;
                sa.subspace = 1;
                paths[k] = 2;
            } else if (n <= 64) {
                HIP_TRY(launch_eig_jacobi_lds(w.G, n, n, max_sweeps, w.lam, w.V, n, sweeps_dev, ok_dev, st));
                sa.ldv = n;
                sa.ncand = n;
                sa.subspace = 0;
                paths[k] = 1;
            } else {
                HIP_TRY(launch_eig_jacobi_global(w.G, n, max_sweeps, w.jac, w.lam, w.V, sweeps_dev, ok_dev, st));
                sa.ldv = n;
                sa.ncand = n;
                sa.subspace = 0;
                paths[k] = 1;
            }
            if (!selected) HIP_TRY(launch_select_factor(sa, st));
            HIP_TRY(wait_selection(g_flags.h, sa.seq, st));
            {
                const volatile HostFlags* f = g_flags.h;
                hf.rank = f->rank;
                hf.need_dense = f->need_dense;
                hf.eig_ok = f->eig_ok;
                hf.status = f->status;
                hf.sweeps = f->sweeps;
                hf.tail = f->tail;
                hf.budget = f->budget;
                hf.norm2 = f->norm2;
                hf.used = f->used;
            }
            if (hf.status != 0)
                return fail((atc_status)hf.status, hf.status == ATC_ERR_NONFINITE_INPUT
                                                       ? "input |A|^2 is not finite"
                                                       : "mode eigensolver: a grid barrier wait gave up");
            if (!hf.need_dense) break;
            queued = false;
            if (split_q && split_yq) {
                // handed on: the product by the basis is dropped, but it still
                // writes dst's tail until it ends
                split_yq = nullptr;
            }
            if (attempt >= 2) return fail(ATC_ERR_INTERNAL, "mode %d: dense eigensolver asked for more", k);
            if (attempt == 1 && opts->eig_path == 2)
                return fail(ATC_ERR_UNSUPPORTED, "mode %d: rank needs more than %d Ritz pairs", k,
                            SUBSPACE_M - SUBSPACE_GUARD);
            HIP_TRY(hipMemcpyAsync(&w.book->need_dense, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
        }
        if (!hf.eig_ok) return fail(ATC_ERR_NOT_CONVERGED, "mode %d: eigensolver hit %d sweeps", k, max_sweeps);
        if (n > 64) wide_hint = attempt >= 1;
        rep_tail[k] = hf.tail;
        rep_budget[k] = hf.budget;
        rep_sweeps[k] = hf.sweeps;
        rep_norm2 = hf.norm2;
        rep_used = hf.used;
        const int r = hf.rank;
        if (r < 1 || r > n) return fail(ATC_ERR_INTERNAL, "mode %d: rank %d outside [1, %d]", k, r, n);
        cur[k] = r;
        if (split_q) {
            // the side stream's product by the basis ends before dst is written
            // again; when the split selection stood, the rotation by W_r^T
            // takes it into dst (rows from the device-side rank, as above)
            HIP_TRY(hipStreamWaitEvent(st, split_q->proj, 0));
            if (split_yq) {
                const TtmPlan tw = ttm_plan(prec, L, S32_RANKS, R, S32_RANKS - SUBSPACE_GUARD);
                HIP_TRY(launch_ttm(prec, tw, split_yq, f64 ? (const void*)w.wt.Wt64 : (const void*)w.wt.Wt32,
                                   split_sr.Wth, split_sr.Wtl, dst, st, &w.book->rank[k], (float*)w.part, w.part_cap));
                HIP_TRY(mark(i, 4));
                queued = true;
            }
        }
        if (queued) {
            if (r >= n) return fail(ATC_ERR_INTERNAL, "mode %d: rank %d of the subspace path", k, r);
            src = dst;
            continue;
        }
        if (r == n && i + 1 < d) {
            // nothing discarded: the projection is a rotation of mode k, which
            // leaves every later Gram matrix unchanged, so it is applied to the
            // final core instead of the full tensor (Alg. 1 computes the same core)
            lazy[nlazy++] = k;
            HIP_TRY(mark(i, 3));
            HIP_TRY(mark(i, 4));
            continue;
        }
        const TtmPlan tp = ttm_plan(prec, L, n, R, r);
        HIP_TRY(mark(i, 3));
        HIP_TRY(launch_ttm(prec, tp, src, M, w.Mth, w.Mtl, dst, st, nullptr, (float*)w.part, w.part_cap));
        HIP_TRY(mark(i, 4));
        src = dst;
    }
    if (nlazy > 0) {
        // the deferred rotations, on the core (a copy of it in w.buf[1] first)
        const int64_t nc = prod(cur, 0, d);
        const size_t esz = f64 ? sizeof(double) : sizeof(float);
        HIP_TRY(hipMemcpyAsync(w.buf[1], core, (size_t)nc * esz, hipMemcpyDeviceToDevice, st));
        for (int j = 0; j < nlazy; ++j) {
            const int k = lazy[j];
            const int nk = (int)cur[k];
            HIP_TRY(launch_prepare_matrix(prec, factors[k], f64 ? 1 : 0, nk, nk, 1, f64 ? w.Mt64 : nullptr,
                                          f64 ? nullptr : w.Mt32, prec == PREC_BF16X3 ? w.Mth : nullptr,
                                          prec == PREC_BF16X3 ? w.Mtl : nullptr, st));
            const TtmPlan tp = ttm_plan(prec, prod(cur, 0, k), nk, prod(cur, k + 1, d), nk);
            const void* M = f64 ? (const void*)w.Mt64 : (const void*)w.Mt32;
            const void* in = w.buf[(j + 1) % 2];
            void* out = (j == nlazy - 1) ? core : w.buf[j % 2];
            HIP_TRY(launch_ttm(prec, tp, in, M, w.Mth, w.Mtl, out, st));
        }
    }
    // every figure of the result came with the host reports; only profiling
    // waits for the last mode product (the outputs are stream-ordered)
    double ms = 0.0;
    if (prof) {
        g_timer.stop(st);
        HIP_TRY(hipStreamSynchronize(st));
        ms = g_timer.elapsed();
    }
    if (result) {
        memset(result, 0, sizeof(*result));
        for (int i = 0; i < d; ++i) {
            const int k = order[i];
            result->ranks[k] = cur[k];
            result->order[i] = order[i];
            result->tail[k] = rep_tail[k];
            result->budget[k] = rep_budget[k];
            result->eig_path[k] = paths[k];
            result->eig_sweeps[k] = rep_sweeps[k];
            result->gram_prec[k] = gram_used[k];
            if (prof) {
                hipEvent_t* e = g_phase.ev[i];
                result->gram_ms[k] = event_ms(e[0], e[1]);
                result->reduce_ms[k] = event_ms(e[1], e[2]);
                result->eig_ms[k] = event_ms(e[2], e[3]);
                result->ttm_ms[k] = event_ms(e[3], e[4]);
            }
        }
        result->norm2 = rep_norm2;
        result->sse_pred = rep_used;
        result->elapsed_ms = ms;
    }
    return ATC_OK;
}

atc_status atc_sthosvd_finish(const atc_shape* shape, const atc_sthosvd_opts* opts, const void* workspace,
                              size_t workspace_bytes, atc_result* result, void* stream) {
    atc_status s;
    if ((s = check_shape(shape)) != ATC_OK) return s;
    if ((s = check_opts(shape, opts)) != ATC_OK) return s;
    if (!opts->no_host_wait) return fail(ATC_ERR_INVALID_ARGUMENT, "atc_sthosvd_finish follows a no_host_wait call");
    const size_t need = carve_sthosvd(shape, nullptr, nullptr);
    if (!workspace || workspace_bytes < need)
        return fail(ATC_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", workspace_bytes, need);
    SthosvdWs w;
    carve_sthosvd(shape, (char*)workspace, &w);
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    DevBook bk;
    HIP_TRY(hipMemcpy(&bk, w.book, sizeof(bk), hipMemcpyDeviceToHost));
    if (result) {
        const int d = shape->ndim;
        for (int k = 0; k < d; ++k) {
            result->tail[k] = bk.tail[k];
            result->budget[k] = bk.budget[k];
            result->eig_sweeps[k] = bk.sweeps[k];
        }
        result->norm2 = bk.norm2;
        result->sse_pred = bk.used;
    }
    switch (bk.status) {
        case 0: return ATC_OK;
        case ATC_ERR_NONFINITE_INPUT: return fail(ATC_ERR_NONFINITE_INPUT, "input |A|^2 is not finite");
        case ATC_ERR_NOT_CONVERGED: return fail(ATC_ERR_NOT_CONVERGED, "an eigensolver hit its sweep cap");
        default:
            return fail((atc_status)bk.status,
                        "a fixed rank the chosen eigensolver could not serve (or a grid wait gave up)");
    }
}

// ------------------------------------------------------------ reconstruction

namespace {

int64_t recon_cost(const int64_t* n, const int64_t* r, const int* p, int d) {
    int64_t total = 0;
    for (int i = 0; i < d; ++i) {
        int64_t t = 1;
        for (int j = 0; j <= i; ++j) t *= n[p[j]];
        for (int j = i; j < d; ++j) t *= r[p[j]];
        total += t;
    }
    return total;
}

// Section 4.1.1: exhaustive search, first permutation in lexicographic order on ties.
void best_order(const int64_t* n, const int64_t* r, int d, int* out) {
    int p[ATC_MAX_DIMS];
    for (int i = 0; i < d; ++i) p[i] = i;
    int64_t best = -1;
    do {
        const int64_t c = recon_cost(n, r, p, d);
        if (best < 0 || c < best) {
            best = c;
            for (int i = 0; i < d; ++i) out[i] = p[i];
        }
    } while (std::next_permutation(p, p + d));
}

atc_status check_ranks(const atc_shape* s, const int64_t* ranks) {
    if (!ranks) return fail(ATC_ERR_INVALID_ARGUMENT, "ranks is NULL");
    for (int k = 0; k < s->ndim; ++k)
        if (ranks[k] < 1 || ranks[k] > s->dims[k])
            return fail(ATC_ERR_INVALID_ARGUMENT, "ranks[%d] outside [1, n_k]", k);
    for (int k = 0; k < s->ndim; ++k)
        if (s->dims[k] > MAX_MODE) return fail(ATC_ERR_UNSUPPORTED, "mode %d longer than %d", k, MAX_MODE);
    return ATC_OK;
}

struct MatBufs {
    double* m64;
    float* m32;
};

// The two intermediates of the reconstruction, in the cheapest order; the
// factors serve as the mode-product matrices as they are.
size_t carve_recon(const atc_shape* s, const int64_t* ranks, char* base, void** buf) {
    const int d = s->ndim;
    const size_t esz = s->dtype == ATC_F64 ? 8 : 4;
    int order[ATC_MAX_DIMS];
    best_order(s->dims, ranks, d, order);
    int64_t cur[ATC_MAX_DIMS];
    for (int k = 0; k < d; ++k) cur[k] = ranks[k];
    int64_t big = 1;
    for (int i = 0; i + 1 < d; ++i) {
        cur[order[i]] = s->dims[order[i]];
        big = std::max<int64_t>(big, prod(cur, 0, d));
    }
    Carver c;
    c.base = base;
    void* b0 = c.take((size_t)big * esz);
    void* b1 = c.take((size_t)big * esz);
    if (buf) {
        buf[0] = b0;
        buf[1] = b1;
    }
    return c.off;
}

}  // namespace

namespace atc {
atc_status check_recon_args(const atc_shape* s, const int64_t* ranks) {
    atc_status st = check_shape(s);
    return st != ATC_OK ? st : check_ranks(s, ranks);
}
void recon_order(const atc_shape* s, const int64_t* ranks, int* order) { best_order(s->dims, ranks, s->ndim, order); }
}  // namespace atc

size_t atc_reconstruct_workspace_size(const atc_shape* shape, const int64_t* ranks) {
    if (check_shape(shape) != ATC_OK || check_ranks(shape, ranks) != ATC_OK) return 0;
    return carve_recon(shape, ranks, nullptr, nullptr);
}

namespace {

// Argument checks of the reconstruction entry points.
atc_status check_recon_call(const atc_shape* shape, const int64_t* ranks, const void* core, const void* const* factors,
                            const void* xhat) {
    atc_status s;
    if ((s = check_shape(shape)) != ATC_OK) return s;
    if ((s = check_ranks(shape, ranks)) != ATC_OK) return s;
    if (!core || !factors || !xhat) return fail(ATC_ERR_INVALID_ARGUMENT, "core, factors and xhat must be non-NULL");
    for (int k = 0; k < shape->ndim; ++k)
        if (!factors[k]) return fail(ATC_ERR_INVALID_ARGUMENT, "factors[%d] is NULL", k);
    return ATC_OK;
}

// The reconstruction proper: one mode product per mode in the cheapest
// order, the intermediates in `workspace` (carve_recon's layout, checked by
// the caller to be large enough).  Kernel launches only: no allocation, no
// memset, no host wait.
atc_status reconstruct_impl(const atc_shape* shape, const int64_t* ranks, const void* core, const void* const* factors,
                            void* xhat, void* workspace, hipStream_t st) {
    void* buf[2];
    carve_recon(shape, ranks, (char*)workspace, buf);
    const int d = shape->ndim;
    const bool f64 = shape->dtype == ATC_F64;
    // float32 mode products at FP32-equivalent accuracy (bf16 three-way splits where MFMA-bound)
    const int prec = f64 ? PREC_F64 : PREC_BF16X6;
    int order[ATC_MAX_DIMS];
    best_order(shape->dims, ranks, d, order);
    int64_t cur[ATC_MAX_DIMS];
    for (int k = 0; k < d; ++k) cur[k] = ranks[k];
    const void* src = core;
    // the last two products in one pass when they are the two trailing modes
    // (in either order) and their sizes fit the fused kernel (float32)
    const int64_t lead = d >= 2 ? prod(shape->dims, 0, d - 2) : 0;
    const bool fuse = !f64 && d >= 2 &&
                      ((order[d - 2] == d - 2 && order[d - 1] == d - 1) ||
                       (order[d - 2] == d - 1 && order[d - 1] == d - 2)) &&
                      ttm_fused_last2_fits(lead, (int)ranks[d - 2], (int)ranks[d - 1], (int)shape->dims[d - 2],
                                           (int)shape->dims[d - 1], xhat);
    const int steps = fuse ? d - 2 : d;
    for (int i = 0; i < steps; ++i) {
        const int k = order[i];
        const int64_t L = prod(cur, 0, k), R = prod(cur, k + 1, d);
        const int rk = (int)ranks[k], nk = (int)shape->dims[k];
        // M = U_k (n_k x r_k, row-major, the factor as given): expands mode k from r_k to n_k
        void* dst = (i == d - 1) ? xhat : buf[i % 2];
        const TtmPlan tp = ttm_plan(prec, L, rk, R, nk);
        HIP_TRY(launch_ttm(prec, tp, src, factors[k], nullptr, nullptr, dst, st));
        cur[k] = nk;
        src = dst;
    }
    if (fuse)
        HIP_TRY(launch_ttm_fused_last2((const float*)src, lead, (int)ranks[d - 2], (int)ranks[d - 1],
                                       (int)shape->dims[d - 2], (int)shape->dims[d - 1],
                                       (const float*)factors[d - 2], (const float*)factors[d - 1], (float*)xhat, st));
    return ATC_OK;
}

// Library-held scratch of atc_reconstruct_noalloc: one copy per device,
// alive until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host the name is a stand-in, not a device address); it uses
// the address hipGetSymbolAddress returns for the current device.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)ATC_NOALLOC_SCRATCH_MIB << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
atc_status noalloc_scratch(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(ATC_ERR_UNSUPPORTED, "device %d beyond the %d the scratch table holds", dev, NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(ATC_ERR_DEVICE, "hipGetSymbolAddress returned NULL for the scratch buffer");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ATC_OK;
}

}  // namespace

atc_status atc_reconstruct(const atc_shape* shape, const int64_t* ranks, const void* core, const void* const* factors,
                           void* xhat, void* workspace, size_t workspace_bytes, void* stream) {
    atc_status s = check_recon_call(shape, ranks, core, factors, xhat);
    if (s != ATC_OK) return s;
    const size_t need = carve_recon(shape, ranks, nullptr, nullptr);
    if (!workspace || workspace_bytes < need)
        return fail(ATC_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", workspace_bytes, need);
    return reconstruct_impl(shape, ranks, core, factors, xhat, workspace, (hipStream_t)stream);
}

atc_status atc_reconstruct_noalloc(const atc_shape* shape, const int64_t* ranks, const void* core,
                                   const void* const* factors, void* xhat, void* stream) {
    atc_status s = check_recon_call(shape, ranks, core, factors, xhat);
    if (s != ATC_OK) return s;
    const size_t need = carve_recon(shape, ranks, nullptr, nullptr);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(ATC_ERR_UNSUPPORTED, "reconstruction needs %zu bytes of scratch; the library's buffer holds %zu",
                    need, NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    if ((s = noalloc_scratch(&ws)) != ATC_OK) return s;
    return reconstruct_impl(shape, ranks, core, factors, xhat, ws, (hipStream_t)stream);
}

// ---------------------------------------------------- reconstruction adjoint
//
// dG = R x_0 U_0^T ... x_{d-1} U_{d-1}^T and dU_n = T_n(n) G_(n)^T with
// T_n = R x_{m != n} U_m^T: dL/dU_n = R_(n) (G x_{m != n} U_m)_(n)^T by the
// mode-product rules, and moving the U_m (m != n) to the other side of the
// contraction gives the T_n form, which only ever shrinks tensors.
// The T_n share work through a two-level tree: P = R x_a U_a^T is formed once
// (mode a shrinks first), every T_n with n != a is then shrunk from P, and
// T_a needs one more pass over R.

namespace {

struct BwdPlan {
    int a;                                // mode shrunk first: P = R x_a U_a^T
    std::vector<int> chain[ATC_MAX_DIMS];  // n != a: modes shrinking P into T_n, in order;
                                          // n == a: modes shrinking R into T_a
    int64_t big;                          // largest intermediate (elements)
};

// elements of the tensor after shrinking the modes in `mask`
int64_t shrunk_size(const atc_shape* s, const int64_t* ranks, unsigned mask) {
    int64_t t = 1;
    for (int k = 0; k < s->ndim; ++k) t *= (mask >> k & 1) ? ranks[k] : s->dims[k];
    return t;
}

// Work of shrinking, from the modes in `mask` already shrunk, the modes in
// `modes` in that order: the products' flops plus eight per byte moved (the
// FP32 mode products run at about eight flops per byte of HBM traffic).
double chain_cost(const atc_shape* s, const int64_t* ranks, unsigned mask, const std::vector<int>& modes) {
    const double esz = s->dtype == ATC_F64 ? 8.0 : 4.0;
    double c = 0.0;
    for (int k : modes) {
        const double in = (double)shrunk_size(s, ranks, mask);
        const double out = in / (double)s->dims[k] * (double)ranks[k];
        c += 2.0 * in * (double)ranks[k] + 8.0 * esz * (in + out);
        mask |= 1u << k;
    }
    return c;
}

// The cheapest order of `modes` (first in lexicographic order on ties).
std::vector<int> best_chain(const atc_shape* s, const int64_t* ranks, unsigned mask, std::vector<int> modes,
                            double* cost) {
    std::sort(modes.begin(), modes.end());
    std::vector<int> best = modes;
    double bc = chain_cost(s, ranks, mask, modes);
    while (std::next_permutation(modes.begin(), modes.end())) {
        const double c = chain_cost(s, ranks, mask, modes);
        if (c < bc) {
            bc = c;
            best = modes;
        }
    }
    if (cost) *cost = bc;
    return best;
}

// The first mode a and every chain order, by exhaustive search over a.
BwdPlan bwd_plan(const atc_shape* s, const int64_t* ranks) {
    const int d = s->ndim;
    BwdPlan p{};
    double best = -1.0;
    for (int a = 0; a < d; ++a) {
        BwdPlan q{};
        q.a = a;
        double c = chain_cost(s, ranks, 0u, std::vector<int>{a});
        for (int n = 0; n < d; ++n) {
            std::vector<int> modes;
            for (int k = 0; k < d; ++k)
                if (k != a && k != n) modes.push_back(k);
            double cc = 0.0;
            if (n == a) {
                modes.clear();
                for (int k = 0; k < d; ++k)
                    if (k != a) modes.push_back(k);
                q.chain[n] = best_chain(s, ranks, 0u, modes, &cc);
            } else {
                q.chain[n] = best_chain(s, ranks, 1u << a, modes, &cc);
            }
            c += cc;
        }
        if (best < 0.0 || c < best) {
            best = c;
            p = q;
        }
    }
    p.big = 1;
    for (int k = 0; k < d; ++k) p.big = std::max<int64_t>(p.big, shrunk_size(s, ranks, 1u << k));
    return p;
}

// bufs: P, the main chains' two scratch buffers, then the two of the mode-a
// chain (which may run on a second stream); part / cg: the main chains' Gram
// partials and FP64 product, then the mode-a chain's.
size_t carve_bwd(const atc_shape* s, const int64_t* ranks, char* base, void** bufs, double** part, size_t* part_cap,
                 double** cg, MatBufs* mb) {
    const int d = s->ndim;
    const size_t esz = s->dtype == ATC_F64 ? 8 : 4;
    const BwdPlan p = bwd_plan(s, ranks);
    int nmax = 1;
    size_t nr = 1;
    for (int k = 0; k < d; ++k) {
        nmax = std::max<int>(nmax, (int)s->dims[k]);
        nr = std::max<size_t>(nr, (size_t)s->dims[k] * ranks[k]);
    }
    Carver c;
    c.base = base;
    void* P = c.take((size_t)p.big * esz);     // R shrunk in one mode
    void* b0 = c.take((size_t)p.big * esz);    // chain scratch
    void* b1 = c.take((size_t)p.big * esz);
    void* b2 = c.take((size_t)p.big * esz);
    void* b3 = c.take((size_t)p.big * esz);
    const size_t pc = part_capacity(nmax);
    double* pt = (double*)c.take(pc);
    double* pt2 = (double*)c.take(pc);
    double* cgb = (double*)c.take(nr * 8);
    double* cgb2 = (double*)c.take(nr * 8);
    double* m64 = (double*)c.take((size_t)d * nr * 8);
    float* m32 = (float*)c.take(s->dtype == ATC_F32 ? (size_t)d * nr * 4 : 0);
    if (bufs) {
        bufs[0] = P;
        bufs[1] = b0;
        bufs[2] = b1;
        bufs[3] = b2;
        bufs[4] = b3;
    }
    if (part) {
        part[0] = pt;
        part[1] = pt2;
    }
    if (part_cap) *part_cap = pc;
    if (cg) {
        cg[0] = cgb;
        cg[1] = cgb2;
    }
    if (mb) {
        mb->m64 = m64;
        mb->m32 = m32;
    }
    return c.off;
}

__global__ void k_cast_out(const double* src, void* dst, int64_t count, int to_f64) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    if (to_f64) ((double*)dst)[i] = src[i];
    else ((float*)dst)[i] = (float)src[i];
}

}  // namespace

size_t atc_reconstruct_backward_workspace_size(const atc_shape* shape, const int64_t* ranks) {
    if (check_shape(shape) != ATC_OK || check_ranks(shape, ranks) != ATC_OK) return 0;
    return carve_bwd(shape, ranks, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
}

atc_status atc_reconstruct_backward(const atc_shape* shape, const int64_t* ranks, const void* core,
                                    const void* const* factors, const void* dxhat, void* dcore, void* const* dfactors,
                                    void* workspace, size_t workspace_bytes, void* stream) {
    atc_status s;
    if ((s = check_shape(shape)) != ATC_OK) return s;
    if ((s = check_ranks(shape, ranks)) != ATC_OK) return s;
    if (!core || !factors || !dxhat) return fail(ATC_ERR_INVALID_ARGUMENT, "core, factors and dxhat must be non-NULL");
    const int d = shape->ndim;
    for (int k = 0; k < d; ++k)
        if (!factors[k]) return fail(ATC_ERR_INVALID_ARGUMENT, "factors[%d] is NULL", k);
    const size_t need = carve_bwd(shape, ranks, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (!workspace || workspace_bytes < need)
        return fail(ATC_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", workspace_bytes, need);
    void* bufs[5];
    double* part[2];
    size_t part_cap;
    double* cg[2];
    MatBufs mb;
    carve_bwd(shape, ranks, (char*)workspace, bufs, part, &part_cap, cg, &mb);
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = shape->dtype == ATC_F64;
    const int prec = f64 ? PREC_F64 : PREC_F32;
    // float32 mode products at FP32-equivalent accuracy (bf16 three-way splits where MFMA-bound)
    const int tprec = f64 ? PREC_F64 : PREC_BF16X6;
    const size_t esz = f64 ? 8 : 4;
    size_t nr = 1;
    for (int k = 0; k < d; ++k) nr = std::max<size_t>(nr, (size_t)shape->dims[k] * ranks[k]);
    // U_k^T (r_k x n_k) for every mode
    std::vector<const void*> Mt(d);
    for (int k = 0; k < d; ++k) {
        double* m64 = mb.m64 + (size_t)k * nr;
        float* m32 = f64 ? nullptr : mb.m32 + (size_t)k * nr;
        HIP_TRY(launch_prepare_matrix(prec, factors[k], f64, (int)shape->dims[k], (int)ranks[k], 1, f64 ? m64 : nullptr,
                                      m32, nullptr, nullptr, st));
        Mt[k] = f64 ? (const void*)m64 : (const void*)m32;
    }
    const BwdPlan bp = bwd_plan(shape, ranks);

    // Shrinks `src` (current sizes cur) in every mode of `modes` (in order) and
    // leaves the result in *out (one of the scratch buffers or `final_dst`).
    // a chain's stream and buffers: the main chains, or the mode-a chain
    struct Lane {
        hipStream_t st;
        void* b[2];
        double* part;
        double* cg;
    };
    const Lane main_lane{st, {bufs[1], bufs[2]}, part[0], cg[0]};
    auto shrink_chain = [&](const Lane& ln, const void* src, int64_t* cur, const std::vector<int>& modes,
                            void* final_dst, const void** out) -> atc_status {
        const void* s_ = src;
        int flip = 0;
        for (size_t i = 0; i < modes.size(); ++i) {
            const int k = modes[i];
            const int64_t L = prod(cur, 0, k), R = prod(cur, k + 1, d);
            void* dst = (i + 1 == modes.size() && final_dst) ? final_dst : ln.b[flip];
            flip ^= 1;
            const TtmPlan tp = ttm_plan(tprec, L, (int)cur[k], R, (int)ranks[k]);
            HIP_TRY(launch_ttm(tprec, tp, s_, Mt[k], nullptr, nullptr, dst, ln.st));
            cur[k] = ranks[k];
            s_ = dst;
        }
        *out = s_;
        return ATC_OK;
    };
    // dU_n = T_n(n) G_(n)^T: cross Gram over the (L, ., R) view of mode n
    auto factor_grad = [&](const Lane& ln, const void* Tn, int n) -> atc_status {
        if (!dfactors || !dfactors[n]) return ATC_OK;
        int64_t rr[ATC_MAX_DIMS];
        for (int k = 0; k < d; ++k) rr[k] = ranks[k];
        const int64_t L = prod(rr, 0, n), R = prod(rr, n + 1, d);
        const GramPlan gp = gram_plan(prec, L, (int)shape->dims[n], (int)ranks[n], R, false, part_cap);
        HIP_TRY(launch_gram(prec, gp, Tn, core, ln.part, ln.st));
        HIP_TRY(launch_gram_reduce(gp, ln.part, ln.cg, ln.st));
        const int64_t cnt = shape->dims[n] * ranks[n];
        hipLaunchKernelGGL(k_cast_out, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, ln.st, ln.cg, dfactors[n],
                           cnt, f64 ? 1 : 0);
        HIP_TRY(hipGetLastError());
        return ATC_OK;
    };

    const int a = bp.a;
    // T_a (every mode but a shrunk): a second pass over R, independent of the
    // others; on the second stream with its own buffers, beside the pass that
    // makes P and the chains from P, and joined before the call returns
    SideQueue::Dev* sq = nullptr;
    if (dfactors && dfactors[a] && !bp.chain[a].empty() && overlap_enabled()) sq = g_side.get();
    const Lane a_lane{sq ? sq->ttm : st, {bufs[3], bufs[4]}, part[1], cg[1]};
    auto chain_a = [&]() -> atc_status {
        if (!dfactors || !dfactors[a]) return ATC_OK;
        const std::vector<int>& modes = bp.chain[a];
        int64_t cur[ATC_MAX_DIMS];
        for (int k = 0; k < d; ++k) cur[k] = shape->dims[k];
        const void* Ta = dxhat;
        if (!modes.empty()) {
            atc_status e = shrink_chain(a_lane, dxhat, cur, modes, nullptr, &Ta);
            if (e != ATC_OK) return e;
        }
        return factor_grad(a_lane, Ta, a);
    };
    if (sq) {
        HIP_TRY(hipEventRecord(sq->basis, st));  // the mode-product operands are ready
        HIP_TRY(hipStreamWaitEvent(sq->ttm, sq->basis, 0));
        atc_status e = chain_a();
        if (e != ATC_OK) return e;
        HIP_TRY(hipEventRecord(sq->proj, sq->ttm));
    }
    // P = R x_a U_a^T
    int64_t curP[ATC_MAX_DIMS];
    for (int k = 0; k < d; ++k) curP[k] = shape->dims[k];
    {
        const int64_t L = prod(curP, 0, a), R = prod(curP, a + 1, d);
        const TtmPlan tp = ttm_plan(tprec, L, (int)curP[a], R, (int)ranks[a]);
        HIP_TRY(launch_ttm(tprec, tp, dxhat, Mt[a], nullptr, nullptr, bufs[0], st));
        curP[a] = ranks[a];
    }
    // T_n for n != a from P (P itself stays intact in bufs[0])
    for (int n = 0; n < d; ++n) {
        if (n == a) continue;
        const std::vector<int>& modes = bp.chain[n];
        int64_t cur[ATC_MAX_DIMS];
        for (int k = 0; k < d; ++k) cur[k] = curP[k];
        const void* Tn = bufs[0];
        if (!modes.empty()) {
            atc_status e = shrink_chain(main_lane, bufs[0], cur, modes, nullptr, &Tn);
            if (e != ATC_OK) return e;
        }
        atc_status e = factor_grad(main_lane, Tn, n);
        if (e != ATC_OK) return e;
        // dG = T_n x_n U_n^T, once
        if (dcore && n == (a == 0 ? 1 : 0)) {
            std::vector<int> last{n};
            const void* outp;
            // shrink T_n in mode n straight into dcore
            e = shrink_chain(main_lane, Tn, cur, last, dcore, &outp);
            if (e != ATC_OK) return e;
        }
    }
    // T_a: joined from the second stream, or made here
    if (sq) {
        HIP_TRY(hipStreamWaitEvent(st, sq->proj, 0));
    } else {
        atc_status e = chain_a();
        if (e != ATC_OK) return e;
    }
    if (dcore && d == 1) {
        // d == 1: dG = R x_0 U_0^T is P itself
        HIP_TRY(hipMemcpyAsync(dcore, bufs[0], (size_t)ranks[0] * esz, hipMemcpyDeviceToDevice, st));
    }
    return ATC_OK;
}

// ------------------------------------------------------------------- misc

const char* atc_status_string(atc_status s) {
    switch (s) {
        case ATC_OK: return "ok";
        case ATC_ERR_INVALID_ARGUMENT: return "invalid argument";
        case ATC_ERR_UNSUPPORTED: return "unsupported";
        case ATC_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case ATC_ERR_DEVICE: return "device error";
        case ATC_ERR_NOT_CONVERGED: return "eigensolver did not converge";
        case ATC_ERR_NONFINITE_INPUT: return "non-finite input";
        case ATC_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char* atc_last_error(void) { return g_last_error.c_str(); }

void atc_finalize(void) {
    g_flags.release();
    g_side.release();
    g_phase.release();
    g_timer.release();
}

const char* atc_version(void) { return "atc-mi355x 0.1 gfx950"; }

