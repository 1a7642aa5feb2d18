/*
 * atc.h -- C ABI of the MI355X (gfx950) ST-HOSVD library.
 *
 * The library computes the sequentially truncated higher-order SVD (ST-HOSVD)
 * of a dense tensor, the first phase of the ATC Tucker compressor
 * (arXiv 2107.01384, Section 3.2, Algorithm 1; Section 4.1), and the Tucker
 * reconstruction (U_1, ..., U_d) . B (Section 3.2) with its adjoint.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Tensors are dense, row-major (C order, last index fastest), as the
 *    paper's flattened binary format (Section 5, "Supported types and I/O").
 *  * Every data pointer is a DEVICE pointer on the current HIP device unless
 *    the comment says "host".  `stream` is a hipStream_t passed as void*;
 *    NULL means the default stream.  All work is enqueued on that stream.
 *  * The caller allocates every buffer (inputs, outputs and the workspace
 *    whose size the matching *_workspace_size call returns).  The library
 *    never frees caller memory and keeps no pointer past the call, except
 *    the explicit plan / graph objects below, which own their own memory
 *    until destroyed.
 *  * Errors: every entry point returns an atc_status.  Arguments are checked
 *    before anything is enqueued; on error nothing is enqueued (except for
 *    ATC_ERR_DEVICE / ATC_ERR_NOT_CONVERGED / ATC_ERR_NONFINITE_INPUT /
 *    ATC_ERR_UNSUPPORTED raised mid-computation, after which output buffers
 *    hold unspecified values).  atc_last_error() returns a thread-local
 *    message describing the last failure of the calling thread.  No C++
 *    exception and no abort crosses this boundary.
 *  * Environment switches, read at every call (for tests and measurement; the
 *    results stay within each path's bounds): ATC_SUB32_KERNELS=1 runs the
 *    subspace eigensolvers as kernel chains instead of one cooperative
 *    launch; ATC_NO_OVERLAP=1 keeps a long mode's m = 32 solver in one launch
 *    and the reconstruction adjoint's first-mode chain on the caller's
 *    stream (no second stream); ATC_SPLIT_MIN_BYTES=<bytes> sets the smallest
 *    tensor that takes the split solver (default 64 MiB);
 *    ATC_GRID_SPIN_LIMIT=<polls> bounds each grid-barrier wait of the
 *    one-launch eigensolvers (default 2^20; a wait that gives up makes the
 *    call return ATC_ERR_INTERNAL).
 *  * Calls are re-entrant across host threads (each on its own stream with its
 *    own workspace).  atc_sthosvd returns only once the calling thread has
 *    learnt every rank, so one host thread runs its single-tensor calls one
 *    after another, except those with opts.no_host_wait, which never wait
 *    and write nothing to host memory; the batched and reconstruction calls
 *    never wait.
 */
#ifndef ATC_H_
#define ATC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ATC_MAX_DIMS 8

typedef enum {
    ATC_OK = 0,
    ATC_ERR_INVALID_ARGUMENT = -1,   /* NULL pointer, bad size, bad option value */
    ATC_ERR_UNSUPPORTED = -2,        /* valid request outside what is built (e.g. mode too long) */
    ATC_ERR_WORKSPACE_TOO_SMALL = -3,
    ATC_ERR_DEVICE = -4,             /* a HIP runtime call failed */
    ATC_ERR_NOT_CONVERGED = -5,      /* eigensolver hit its sweep cap */
    ATC_ERR_NONFINITE_INPUT = -6,    /* |A|^2 of the input is NaN or Inf */
    ATC_ERR_INTERNAL = -7
} atc_status;

typedef enum { ATC_F32 = 0, ATC_F64 = 1 } atc_dtype;

/* Arithmetic of the Gram matrix and the projection (mode product).
 *  NATIVE : FP64 MFMA for float64 input, FP32 MFMA for float32 input
 *           (FP32 products accumulated in FP32 over chunks of 128 terms,
 *           chunks summed in FP64).
 *  BF16X3 : float32 input only.  Each operand a is split into
 *           a_hi = bf16(a), a_lo = bf16(a - a_hi); a*b is formed on the bf16
 *           matrix cores as hi*hi + hi*lo + lo*hi with FP32 accumulation
 *           (chunks summed in FP64 as above).  The dropped lo*lo term would
 *           always be positive on the Gram diagonal: the tiled kernels of
 *           modes with a contiguous trailing extent and the batched kernel
 *           replace the diagonal by the exact FP64 sum of squares of the
 *           loaded floats (in both precisions); the generic-layout kernel adds
 *           lo*lo on its diagonal tiles instead.
 *  F64ACC : float32 input only: the 64-bit internal arithmetic option
 *           (Section 5) for the Gram matrix, where the error target asks for
 *           more than an FP32-accumulated Gram matrix holds (eps <= 1e-4):
 *           operands widened to FP64, exact products, FP64 accumulation on
 *           the FP64 matrix cores.  Projections stay FP32.
 * The eigensolver, rank choice and every tail sum are FP64 in all cases. */
typedef enum { ATC_PREC_NATIVE = 0, ATC_PREC_BF16X3 = 1, ATC_PREC_F64ACC = 2 } atc_precision;

/* Per-mode share of the SSE budget S = rtmss * (rel_error * |A|)^2
 * (Section 4.1.3; the paper defers the rule to the ST-HOSVD literature).
 *  ADAPTIVE : mode i (0-based in processing order) gets (S - used) / (d - i)
 *  EQUAL    : every mode gets S / d
 * r_k is the smallest r >= 1 whose discarded eigenvalue sum fits the share. */
typedef enum { ATC_RANK_ADAPTIVE = 0, ATC_RANK_EQUAL = 1 } atc_rank_rule;

typedef struct {
    int32_t ndim;                /* order d, 1 <= d <= ATC_MAX_DIMS */
    int32_t dtype;               /* atc_dtype */
    int64_t dims[ATC_MAX_DIMS];  /* n_0 .. n_{d-1}, each >= 1 */
} atc_shape;

typedef struct {
    double rel_error;            /* target |A - A~| / |A| (Section 2.1, "relative error"); >= 0 */
    double rtmss;                /* rank_truncation_max_sse_share (Section 4.1.3), in [0, 1]; default 1 */
    int32_t precision;           /* atc_precision; default NATIVE */
    int32_t rank_rule;           /* atc_rank_rule; default ADAPTIVE */
    int32_t has_order;           /* nonzero: use mode_order (Section 4.1.1, user order) */
    int32_t mode_order[ATC_MAX_DIMS]; /* permutation of 0..d-1 */
    int32_t has_fixed_ranks;     /* nonzero: use fixed_ranks instead of the budget rule */
    int32_t fixed_ranks[ATC_MAX_DIMS]; /* 1 <= r_k <= n_k */
    int32_t max_sweeps;          /* eigensolver sweep cap; 0 = default (60) */
    int32_t eig_path;            /* 0 = automatic, 1 = force dense Jacobi, 2 = force subspace (n > 64) */
    int32_t profile;             /* nonzero: time each phase with stream events (atc_result.*_ms) */
    /* Precision guard (NATIVE and BF16X3 on float32 input).  The rounding of
     * an FP32-accumulated Gram matrix has both signs; in the trailing
     * eigenvalues its negative part is clamped away, which biases the
     * discarded-energy sums upwards.  A mode gets an F64ACC Gram matrix when
     *  - its budget share is below 2^-23 times the energy of the tensor the
     *    Gram matrix is formed from (for d = 3 and rtmss = 1: rel_error below
     *    about 6e-4), or
     *  - its contraction (product of the other current mode sizes) has fewer
     *    than 2048 terms, where that bias grows to a sizeable part of a
     *    budget share (and FP64 costs little).
     * Nonzero turns the guard off.  atc_result.gram_prec reports what each
     * mode used. */
    int32_t no_precision_guard;
    /* Nonzero (needs has_fixed_ranks, profile = 0): every step is enqueued on
     * `stream` with no host wait and no host-side decision from device
     * results, so the call can be captured in a HIP graph.  The eigensolver of
     * each mode is picked from its fixed rank (n <= 64, FP64 data or
     * eig_path 1: dense; r <= 24: the m = 32 subspace path; r <= 56: m = 64;
     * else the dense solver in global memory); on a capturing stream the
     * subspace solvers run as kernel chains (the library records no
     * cooperative launch into a graph: the one-launch form's grid barriers
     * need all of its workgroups resident at once), otherwise in their
     * one-launch form.  atc_result gets the ranks, order, paths and Gram
     * precisions only; atc_sthosvd_finish reads the rest and the status once
     * the stream has run.  A subspace mode whose data has fewer than r_k
     * positive Ritz values is reported by atc_sthosvd_finish, not handed on
     * to the dense solver.  The host-side state of the library (the report
     * block, the per-device flags) is set up by the first call of a process:
     * make one ordinary call before capturing. */
    int32_t no_host_wait;
    int32_t reserved[3];
} atc_sthosvd_opts;

/* Host-side record of one ST-HOSVD call. */
typedef struct {
    int64_t ranks[ATC_MAX_DIMS];   /* chosen r_k (natural mode index) */
    int32_t order[ATC_MAX_DIMS];   /* processing order used */
    double norm2;                  /* |A|^2 (trace of the first Gram matrix) */
    double sse_pred;               /* sum over modes of the discarded eigenvalues (Section 4.1.3) */
    double tail[ATC_MAX_DIMS];     /* discarded energy per mode */
    double budget[ATC_MAX_DIMS];   /* budget share per mode */
    int32_t eig_path[ATC_MAX_DIMS];/* 1 = dense Jacobi, 2 = subspace iteration */
    int32_t eig_sweeps[ATC_MAX_DIMS];
    double elapsed_ms;             /* with opts.profile: device time of the call (stream events), else 0 */
    /* with opts.profile, per processed mode (natural index): Gram kernel,
     * split-K reduction, eigensolver + rank choice, mode-product kernel */
    double gram_ms[ATC_MAX_DIMS];
    double reduce_ms[ATC_MAX_DIMS];
    double eig_ms[ATC_MAX_DIMS];
    double ttm_ms[ATC_MAX_DIMS];
    int32_t gram_prec[ATC_MAX_DIMS]; /* atc_precision of each mode's Gram matrix (natural index) */
} atc_result;

/* Fills *o with the defaults documented above (rel_error = 1e-3). */
void atc_default_opts(atc_sthosvd_opts* o);

/* Bytes of device workspace atc_sthosvd needs for this shape and options
 * (0 on invalid arguments). */
size_t atc_sthosvd_workspace_size(const atc_shape* shape, const atc_sthosvd_opts* opts);

/*
 * ST-HOSVD (Section 3.2, Algorithm 1; mode order and error control of
 * Section 4.1): for each mode k in processing order, form the Gram matrix of
 * the mode-k unfolding of the current tensor, eigendecompose it in FP64,
 * keep the r_k leading eigenvectors (largest-magnitude entry of each made
 * positive) and project mode k onto them.
 *
 *  x        input tensor, dtype shape->dtype, prod(dims) elements.
 *  core     output core, same dtype, row-major r_0 x ... x r_{d-1} in natural
 *           mode order; capacity prod(dims) elements (worst case r = n).
 *  factors  host array of d device pointers; factors[k] receives U_k as a
 *           row-major n_k x r_k matrix of the input dtype; capacity n_k^2.
 *  result   host pointer, filled on success.
 * The call returns once every r_k is known (the selection kernels report each
 * rank and the result figures through pinned host memory, and the host sizes
 * the next step from them); the last mode product may still be running on
 * `stream`.  core and factors are complete in stream order, like the output
 * of a kernel launch: synchronise the stream, or keep later work on it,
 * before reading them, and keep workspace alive until then.  With
 * opts.profile the call waits for the stream (the phase times need it).
 */
atc_status atc_sthosvd(const void* x, const atc_shape* shape, const atc_sthosvd_opts* opts,
                       void* core, void* const* factors, atc_result* result,
                       void* workspace, size_t workspace_bytes, void* stream);

/*
 * After an opts.no_host_wait call (or the replay of a graph that captured
 * one): waits for `stream`, reads the call's device record from `workspace`
 * (the same buffer, shape and opts) and fills result's norm2, sse_pred, tail,
 * budget and eig_sweeps.  Returns the call's status: ATC_ERR_NONFINITE_INPUT,
 * ATC_ERR_NOT_CONVERGED (an eigensolver hit max_sweeps), ATC_ERR_INTERNAL (a
 * fixed rank left the subspace fewer than 8 unused Ritz pairs, or a Ritz value
 * at the rank was not positive), else ATC_OK.
 */
atc_status atc_sthosvd_finish(const atc_shape* shape, const atc_sthosvd_opts* opts, const void* workspace,
                              size_t workspace_bytes, atc_result* result, void* stream);

/* ---------------------------------------------------------------- batched */

/* Device-side record of one block of a batched call. */
typedef struct {
    int32_t ranks[3];
    int32_t status;       /* 0 ok, else an atc_status value */
    double norm2;
    double sse_pred;
    double tail[3];
} atc_block_result;

typedef struct atc_batch_plan atc_batch_plan;

/*
 * Plans the ST-HOSVD of many independent 3-way float32 blocks in one
 * persistent launch (each block treated exactly as atc_sthosvd would with
 * precision BF16X3 or NATIVE, mode order by increasing length).
 *  dims           host array, nblocks x 3 mode sizes, each in [1, 64].
 *  input_offsets  host array of nblocks element offsets (>= 0) of each block
 *                 in the caller's input arena (row-major block, prod(dims)
 *                 floats from there), or NULL for blocks packed back to back
 *                 in block order.
 *  The plan fixes: the input offsets, core slots (prod(dims) floats per
 *  block) and factor slots (n_k^2 floats per mode), the longest-first
 *  processing order and the launch configuration.
 *  opts->precision (BF16X3 or NATIVE) is the arithmetic of the mode
 *  products; the blocks' Gram matrices are always FP64-accumulated (their
 *  contractions have at most 4096 terms: the short-contraction case of the
 *  precision guard of atc_sthosvd_opts).
 * The plan owns device memory until atc_batch_plan_destroy.
 */
atc_status atc_batch_plan_create(const int32_t* dims, const int64_t* input_offsets, int64_t nblocks,
                                 const atc_sthosvd_opts* opts, atc_batch_plan** plan);
void atc_batch_plan_destroy(atc_batch_plan* plan);

/* Sizes in elements (float32) of the input arena (the end of the last block),
 * core arena and factor arena, and the workspace bytes; any pointer may be
 * NULL. */
atc_status atc_batch_plan_info(const atc_batch_plan* plan, int64_t* input_elems, int64_t* core_elems,
                               int64_t* factor_elems, size_t* workspace_bytes);

/* Host arrays of nblocks entries each (any may be NULL): element offsets of
 * block b in the input, core and factor arenas (factor k of block b starts at
 * factor_off[b] + sum_{j<k} n_j^2). */
atc_status atc_batch_plan_offsets(const atc_batch_plan* plan, int64_t* input_off, int64_t* core_off,
                                  int64_t* factor_off);

/* Runs the plan: no host synchronisation, no allocation, capturable in a
 * HIP graph.  results: device array of nblocks atc_block_result. */
atc_status atc_sthosvd_batched(atc_batch_plan* plan, const float* arena, float* core_arena,
                               float* factor_arena, atc_block_result* results,
                               void* workspace, size_t workspace_bytes, void* stream);

/* Times every candidate launch configuration of the persistent kernel on
 * these buffers (median of `reps` runs each) and stores the fastest in the
 * plan.  If cache_path is non-NULL the choice is read from / appended to that
 * JSON-lines file, keyed by architecture, precision and block-size histogram.
 * out_choice (host, may be NULL) receives the chosen candidate index. */
atc_status atc_batch_autotune(atc_batch_plan* plan, const float* arena, float* core_arena,
                              float* factor_arena, atc_block_result* results,
                              void* workspace, size_t workspace_bytes, void* stream,
                              int32_t reps, const char* cache_path, int32_t* out_choice);

typedef struct atc_graph atc_graph;

/* Captures one atc_sthosvd_batched call (all its launches) into a HIP graph
 * on `stream` and instantiates it; replays run the same buffers. */
atc_status atc_batch_graph_create(atc_batch_plan* plan, const float* arena, float* core_arena,
                                  float* factor_arena, atc_block_result* results,
                                  void* workspace, size_t workspace_bytes, void* stream,
                                  atc_graph** graph);
atc_status atc_graph_launch(atc_graph* graph, void* stream);
void atc_graph_destroy(atc_graph* graph);

/* ---------------------------------------------------------- reconstruction */

/* Workspace for atc_reconstruct (shape: the full n_k; ranks: r_k). */
size_t atc_reconstruct_workspace_size(const atc_shape* shape, const int64_t* ranks);

/*
 * Tucker reconstruction X~ = (U_0, ..., U_{d-1}) . G (Section 3.2): every mode
 * of the core G (r_0 x ... x r_{d-1}) is expanded by its factor U_k (n_k x r_k,
 * row-major).  The mode order minimises sum_i n_{p1}..n_{pi} r_{pi}..r_{pd}
 * (Section 4.1.1, exhaustive search, first lexicographic order on ties).
 *  ranks    host array of d ranks, 1 <= r_k <= n_k.
 *  factors  host array of d device pointers.
 *  xhat     output, prod(n) elements, dtype shape->dtype.
 * Arithmetic: FP32 MFMA for float32, FP64 MFMA for float64.
 */
atc_status atc_reconstruct(const atc_shape* shape, const int64_t* ranks, const void* core,
                           const void* const* factors, void* xhat,
                           void* workspace, size_t workspace_bytes, void* stream);

/* Size of the device scratch buffer the library holds for
 * atc_reconstruct_noalloc (per device, for the life of the process). */
#define ATC_NOALLOC_SCRATCH_MIB 64

/*
 * atc_reconstruct for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same reconstruction, its intermediates in a library-held device buffer of
 * ATC_NOALLOC_SCRATCH_MIB MiB instead of a caller workspace.  The call
 * allocates nothing (no hipMalloc, no allocating library routine); on its
 * first use on a device it looks up that device's copy of the buffer.
 *  Returns ATC_ERR_UNSUPPORTED when the reconstruction needs more scratch than
 *  the buffer holds (atc_reconstruct_workspace_size tells the need).
 *  Every call on one device shares that device's buffer: calls that overlap
 *  on one device (different streams, or host threads, without ordering) race
 *  and give undefined results.  Nothing in the buffer needs to start at zero
 *  (every intermediate is written before it is read).
 */
atc_status atc_reconstruct_noalloc(const atc_shape* shape, const int64_t* ranks, const void* core,
                                   const void* const* factors, void* xhat, void* stream);

size_t atc_reconstruct_backward_workspace_size(const atc_shape* shape, const int64_t* ranks);

/*
 * Adjoint of atc_reconstruct: given R = dL/dX~ (same shape as X~), writes
 *   dcore      = R x_0 U_0^T x_1 U_1^T ... x_{d-1} U_{d-1}^T     (r_0 x ... x r_{d-1})
 *   dfactors[n] = R_(n) W_(n)^T, W = G x_{m != n} U_m              (n_n x r_n)
 * (the mode-product rules of Section 3.1).  Partial products are recomputed
 * from G and the U_k, not read from the forward pass.  dfactors: host array of
 * d device pointers; any of dcore / dfactors[n] may be NULL to skip it.  The
 * chain of one mode (its own pass over R) may run on a second stream of the
 * library, ordered after the call's earlier work on `stream` and joined back
 * into `stream` before the call returns: the outputs are complete in the
 * order of `stream` like those of any kernel launch.
 */
atc_status atc_reconstruct_backward(const atc_shape* shape, const int64_t* ranks, const void* core,
                                    const void* const* factors, const void* dxhat, void* dcore,
                                    void* const* dfactors, void* workspace, size_t workspace_bytes,
                                    void* stream);

/* ------------------------------------------------------- core quantization */

/* Stream record of one quantized core (device memory, written by the call). */
typedef struct {
    int32_t status;     /* ATC_OK; ATC_ERR_NONFINITE_INPUT (core not finite:
                           nothing encoded); ATC_ERR_WORKSPACE_TOO_SMALL (the
                           stream did not fit: cannot happen with enc_words >=
                           atc_quantize_max_words) */
    int32_t k;          /* scale exponent: 2^63 <= 2^k max|b| < 2^64;
                           ATC_QUANT_KZERO for an all-zero core */
    int32_t plane;      /* breakpoint plane P: planes 63 .. P+1 encoded for every
                           coefficient, plane P for the first `count`; 64 =
                           nothing encoded */
    int32_t block_len;
    int64_t n;
    int64_t count;      /* coefficients encoded on plane P */
    int64_t nblocks;
    int64_t words;      /* stream length in 32-bit words */
    double sse;         /* |B - B~|^2 at the breakpoint in the core's units: the
                           exact integer error times 2^-2k, rounded */
    int64_t pad;
} atc_quant_info;

#define ATC_QUANT_KZERO INT32_MIN
#define ATC_QUANT_MAX_BLOCK 4096

/* Capacity in 32-bit words a stream of n coefficients in blocks of block_len
 * can need (0 on invalid arguments). */
size_t atc_quantize_max_words(int64_t n, int32_t block_len);
size_t atc_quantize_workspace_size(int64_t n, int32_t block_len);

/*
 * Bit-plane quantization and encoding of a core (Section 3.3, TTHRESH bit-plane
 * truncation, Table 2; Section 4.2, blocks encoded independently with their
 * sizes and a breakpoint each; Section 4.3, the dequantization correction
 * inside the error tracking).
 *  core        n coefficients (dtype ATC_F32 / ATC_F64), the core vectorised in
 *              C order (lexicographic, last index fastest).
 *  target_sse  quantization error allowed, |B - B~|^2 in the core's units
 *              (e.g. the total SSE target minus the ST-HOSVD's, Section
 *              4.1.3); below zero encodes every bit.
 *  block_len   coefficients per block, 1 .. ATC_QUANT_MAX_BLOCK.
 *  enc         output stream, at least atc_quantize_max_words words.
 *  info        DEVICE pointer to one atc_quant_info, written by the call.
 * Magnitudes q_i = rint(2^k |b_i|) (ties to even) are walked plane by plane
 * from bit 63; the error of encoding every bit so far is tracked exactly
 * (integers), each magnitude known down to plane p counting as its known bits
 * plus 2^(p-1) (zero while none of its one-bits is known).  The breakpoint is
 * the first position, on the first plane whose end reaches the target, at
 * which the error is at most target_sse; blocks before it encode that plane
 * in full, blocks after it not at all.
 * Stream (32-bit words): magic 0x51435441, k, P, block_len, n (2 words), count
 * (2), nblocks (2), nblocks block sizes in words (2 each), then the blocks.  A
 * block: run bytes, sign bits, trailing bits (3 words), the zero-run lengths of
 * its leading bits as LEB128 bytes (per plane from 63 down: the zeros before
 * each one-bit of a coefficient not yet significant, then the zeros after the
 * last; nothing for a plane without such coefficients), the signs of the
 * coefficients as they become significant, and the bits of the coefficients
 * already significant; bit fields packed least significant bit first, each
 * field padded to whole words.  No entropy coder is applied.
 * Nothing is allocated; no host wait; capturable in a HIP graph.
 */
atc_status atc_quantize_core(const void* core, int32_t dtype, int64_t n, double target_sse, int32_t block_len,
                             uint32_t* enc, size_t enc_words, atc_quant_info* info, void* workspace,
                             size_t workspace_bytes, void* stream);

size_t atc_dequantize_workspace_size(int64_t n, int32_t block_len);

/*
 * Decoding of an atc_quantize_core stream (n and block_len as recorded in its
 * atc_quant_info): every coefficient becomes sign * (known bits + 2^(p-1)) *
 * 2^-k, p its lowest encoded plane (nothing added when p = 0; zero when none of
 * its one-bits is encoded), written as dtype to core_out (n values).
 *  status  optional DEVICE int32: OR-ed with 2 when the stream's header does
 *          not match n / block_len (every value is then written as zero), with
 *          1 when a block's fields do not match its planes (a damaged stream;
 *          that block's values are then undefined).  The caller guarantees
 *          that `enc` holds the whole stream its header describes.
 */
atc_status atc_dequantize_core(const uint32_t* enc, int64_t n, int32_t block_len, int32_t dtype, void* core_out,
                               int32_t* status, void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------ factor representation, error model */

/* Device workspace of atc_factor_householder / atc_factor_from_householder
 * (0 unless 1 <= r <= n <= 4096, r <= 256). */
size_t atc_householder_workspace_size(int64_t n, int64_t r);

/*
 * Householder representation of a factor (supplement S.2): U (n x r,
 * row-major, dtype, orthonormal columns) = H_1 ... H_r [I_r; 0] diag(signs)
 * with H_j = I - 2 v_j v_j^T, v_j of unit norm, zero above row j, v_jj > 0.
 *  sigma2   optional DEVICE array of r squared slice norms of the quantized
 *           core in this factor's mode: each stored entry of v_j is then
 *           scaled by sqrt(2 alpha_j) (alpha_j as in supplement S.2, n_j =
 *           n - j + 1, 1-based j); NULL stores the entries unscaled.
 *  coef     DEVICE output, n r - r (r + 1) / 2 doubles: the entries of v_j
 *           below its diagonal, column by column (v_jj follows from |v_j| = 1).
 *  signs    DEVICE output, r int32: +1 / -1, the sign of R_jj in the
 *           Householder QR of U; U' = U diag(signs) is what the reflectors
 *           rebuild (apply the same signs to the core's slices,
 *           atc_core_apply_signs, to keep the decomposition).
 *  Uprime   optional DEVICE output (n x r, dtype): U diag(signs).
 * One workgroup, FP64.  No allocation, no host wait.
 */
atc_status atc_factor_householder(const void* U, int32_t dtype, int64_t n, int64_t r, const double* sigma2,
                                  double* coef, int32_t* signs, void* Uprime, void* workspace, size_t workspace_bytes,
                                  void* stream);

/* Scales stored reflector entries in place by the weights of supplement S.2:
 * the entries of column j (coef as written by atc_factor_householder with
 * sigma2 NULL, n r - r (r + 1) / 2 DEVICE doubles) are multiplied by
 * sqrt(2 alpha_j), alpha_j from the r squared slice norms sigma2 (DEVICE) and
 * n_j = n - j + 1 (1-based j); the result equals atc_factor_householder's
 * output with the same sigma2.  The reflectors of U diag(s) for any signs s
 * are those of U, so entries computed before the core is quantized serve
 * after it.  Grid of (rows, columns) workgroups; no allocation, no host wait. */
atc_status atc_factor_weight_coefficients(double* coef, const double* sigma2, int64_t n, int64_t r, void* stream);

/* The factor U' = H_1 ... H_r [I_r; 0] from the stored entries (weighted as
 * given to atc_factor_householder when sigma2 is non-NULL; a column whose
 * weight is zero, which happens only when it and every later slice norm are
 * zero, decodes with v_j = e_j).  U_out: DEVICE, n x r, dtype. */
atc_status atc_factor_from_householder(const double* coef, const double* sigma2, int64_t n, int64_t r, int32_t dtype,
                                       void* U_out, void* workspace, size_t workspace_bytes, void* stream);

/* Number of slice norms of a core: dims[0] + ... + dims[d-1]. */
size_t atc_core_slice_norms_count(const atc_shape* shape);

/* Squared slice norms of a core in every mode (eq. total_error_approximation,
 * Section 4.1.3): out (DEVICE, atc_core_slice_norms_count doubles) holds, mode
 * after mode, sum over the other indices of B[..., i_k, ...]^2.  shape->dims
 * are the core's sizes; dtype F32 or F64. */
atc_status atc_core_slice_norms(const void* core, const atc_shape* shape, double* out, void* stream);

/* Flips the core's slices: B[i_0, .., i_{d-1}] *= prod_k signs_k[i_k], signs
 * (DEVICE int32) laid out mode after mode as the slice norms. */
atc_status atc_core_apply_signs(void* core, const atc_shape* shape, const int32_t* signs, void* stream);

/* |dU Sigma|_F^2 = sum_j sigma2[j] sum_i (Uq[i][j] - U[i][j])^2 for one factor
 * (the factor term of eq. total_error_approximation); U, Uq DEVICE n x r
 * (dtype), sigma2 DEVICE r doubles, out DEVICE one double. */
atc_status atc_factor_error_term(const void* U, const void* Uq, int32_t dtype, int64_t n, int64_t r,
                                 const double* sigma2, double* out, void* stream);

/* ------------------------------------------------------- hybrid compressor */

/* Outputs of atc_hybrid_quantize: DEVICE buffers the caller owns (d = the
 * core's order, r_k its sizes, n_k the factors' rows, e_k = n_k r_k - r_k
 * (r_k + 1) / 2 the stored reflector entries of factor k). */
typedef struct {
    uint32_t* core_enc;                 /* atc_quantize_max_words(prod r_k, block_len) words */
    atc_quant_info* core_info;          /* one record */
    void* core_q;                       /* the dequantized core (core dtype, prod r_k values) */
    double* sigma2;                     /* squared slice norms of core_q, mode after mode (sum r_k) */
    int32_t* signs;                     /* the factors' column signs, mode after mode (sum r_k) */
    void* factor_signed[ATC_MAX_DIMS];  /* U_k diag(signs_k), n_k x r_k (core dtype) */
    double* factor_coef[ATC_MAX_DIMS];  /* weighted reflector entries, max(1, e_k) doubles */
    uint32_t* factor_enc[ATC_MAX_DIMS]; /* atc_quantize_max_words(e_k, block_len) words (unused when e_k = 0) */
    atc_quant_info* factor_info[ATC_MAX_DIMS];  /* one record each (not written when e_k = 0) */
    void* factor_q[ATC_MAX_DIMS];       /* factors rebuilt from the quantized entries, n_k x r_k */
    double* factor_term;                /* d doubles: |dU_k Sigma_k|_F^2 */
    int32_t* status;                    /* one int32: the decoders' damage flags OR-ed (0 expected) */
} atc_hybrid_out;

/* Workspace of atc_hybrid_quantize (0 on invalid arguments).  core_shape:
 * the core (r_k, dtype); n: the factors' rows n_k. */
size_t atc_hybrid_workspace_size(const atc_shape* core_shape, const int64_t* n, int32_t block_len);

/*
 * The quantization half of the hybrid truncation (Section 4.1.3) after an
 * ST-HOSVD, in one call: the Householder form of every factor and its column
 * signs (supplement S.2), the core's slices flipped by them, the core
 * quantized to core_target_sse and decoded (Sections 3.3, 4.2, 4.3), its
 * slice norms, then per factor the stored entries weighted by sqrt(2 alpha_j),
 * quantized to factor_target_sse, decoded, the factor rebuilt from them and
 * its error term |dU Sigma|_F^2 (eq. total_error_approximation).  The error
 * predicted by that equation is the ST-HOSVD's discarded energy plus
 * core_info->sse plus the sum of factor_term.
 *  core      DEVICE, the ST-HOSVD core (row-major r_0 x ... x r_{d-1}).
 *  factors   host array of d DEVICE pointers, U_k (n_k x r_k, row-major,
 *            orthonormal columns, the core's dtype).
 *  n         host array of the d row counts n_k (<= 4096; r_k <= 256).
 * Every step runs on `stream`, the d factors sharing each launch; no
 * allocation of device memory, no host wait.  Targets must be finite (a
 * negative target keeps every bit).  Errors: ATC_ERR_INVALID_ARGUMENT (NULL
 * buffer, bad shape, r_k > n_k), ATC_ERR_UNSUPPORTED (n_k > 4096 or r_k > 256),
 * ATC_ERR_WORKSPACE_TOO_SMALL, ATC_ERR_DEVICE (a launch failed).
 */
atc_status atc_hybrid_quantize(const void* core, const atc_shape* core_shape, const void* const* factors,
                               const int64_t* n, double core_target_sse, double factor_target_sse,
                               int32_t block_len, const atc_hybrid_out* out, void* workspace,
                               size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------ misc */
const char* atc_status_string(atc_status s);
const char* atc_last_error(void);
/* Library version string, e.g. "atc-mi355x 0.1 gfx950". */
const char* atc_version(void);

/* Releases what the library holds for the calling thread outside plans and
 * graphs: the pinned host block atc_sthosvd's selection kernels report ranks
 * into and the HIP events of opts.profile.  Call once the thread's work on
 * its streams has completed (e.g. before the process exits, while the HIP
 * runtime is still up); a later call re-creates them.  Idempotent. */
void atc_finalize(void);

#ifdef __cplusplus
}
#endif
#endif /* ATC_H_ */
