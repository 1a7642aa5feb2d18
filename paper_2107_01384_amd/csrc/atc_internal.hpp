// Internal declarations shared by the HIP translation units of libatc.
// Everything here is gfx950 (CDNA4) code: 64-wide wavefronts, MFMA matrix
// cores, 160 KB of LDS per compute unit.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/atc.h"

namespace atc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Arithmetic of a contraction (Gram matrix or mode product).
//  PREC_F64ACC: float32 operands widened to FP64 on their way to LDS, FP64
//  MFMA products and accumulation (the Gram matrix of float32 data to FP64
//  accuracy); the mode products of that path run as PREC_F32.
//  PREC_BF16X6: float32 operands split into three bf16 pieces (8 + 8 + 8
//              significant bits, exact), the six products of order <= 2 on
//              bf16 MFMA with FP32 accumulation: FP32-equivalent products (the
//              dropped terms are below 2^-23 of |a b|).  Mode products of the
//              reconstruction and its adjoint only; everything else treats it
//              as PREC_F32.
enum Prec : int { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16X3 = 2, PREC_F64ACC = 3, PREC_BF16X6 = 4 };

// Jacobi couplings left alone in the eigenproblems of float32 data (the
// Rayleigh-Ritz problems of the subspace paths and the batched blocks'
// Gram matrices): entries at or below JACOBI_FLOOR_F32 times the trace.  The
// input's own float32 rounding already moves every Gram entry of the data it
// stands for by about 2^-24 of the trace; couplings 64 times smaller resolve
// nothing of the data, and leaving them changes a discarded-energy sum only at
// second order, or not at all when both indices lie in the discarded block
// (rotations inside it keep its trace).  FP64 input keeps 2^-53.
constexpr double JACOBI_FLOOR_F32 = 0x1p-30;

// How the contracted index of an (L, n, R) view is walked:
//  KC: R large, the R index is contiguous -> tiles step along R inside one l.
//  NC: R == 1, the n index is contiguous -> tiles step along l.
//  SR: 1 < R < tile depth -> a tile covers whole (n x R) planes of several l.
enum Layout : int { LAYOUT_KC = 0, LAYOUT_NC = 1, LAYOUT_SR = 2 };

template <int P> struct ElemOf { typedef float T; };
template <> struct ElemOf<PREC_F64> { typedef double T; };

// Device-side bookkeeping of one ST-HOSVD call (Section 4.1.3 error control).
struct DevBook {
    double norm2;        // |A|^2, trace of the first Gram matrix
    double S;            // SSE budget rtmss * eps^2 * |A|^2
    double used;         // discarded energy so far
    double tail[ATC_MAX_DIMS];
    double budget[ATC_MAX_DIMS];
    double trace[ATC_MAX_DIMS];
    int32_t rank[ATC_MAX_DIMS];
    int32_t sweeps[ATC_MAX_DIMS];
    int32_t status;      // 0, or a negative atc_status
    int32_t need_dense;  // subspace basis too small for the chosen rank
    int32_t eig_ok;      // last eigensolve converged
    int32_t pad;
    // words of the cooperative subspace kernel: barrier arrivals, rank,
    // need_dense, a wait that gave up, workgroups done; zero between launches
    // (the book is cleared per call and the kernel's last workgroup resets them)
    uint32_t grid[8];
};

// ------------------------------------------------------------ small helpers
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Tile geometry of the Gram and mode-product kernels.
constexpr int TILE = 64;          // output tile edge
constexpr int NTHREADS = 256;     // 4 waves
constexpr int FLUSH_TERMS = 128;  // FP32 accumulation chunk before the FP64 add

template <int P> struct KDepth { static constexpr int value = 32; };
template <> struct KDepth<PREC_F64> { static constexpr int value = 16; };
template <> struct KDepth<PREC_F64ACC> { static constexpr int value = 16; };

// FP64 MFMA arithmetic (FP64 input, or float32 input widened)
__host__ __device__ constexpr bool prec_f64_mfma(int p) { return p == PREC_F64 || p == PREC_F64ACC; }

// The Jacobi rotation of a symmetric pair (p, q), rotated when |a_pq| > tol
// sqrt(|a_pp a_qq|), by the smaller angle, with two
// reciprocal square roots instead of two divisions and two square roots:
// d = a_qq - a_pp, g = 2 a_pq, h = hypot(d, g), u = (1 + |d| / h) / 2,
// c = sqrt(u), s = sign(d) g / (2 h c), t = s / c.

// 1 / sqrt(z) for positive, normal, finite z: the hardware estimate y0
// (v_rsq_f64) and one correction from the series (1 - e)^(-1/2) = 1 + e/2 +
// 3e^2/8 + ..., e = 1 - z y0^2, whose truncation error is O(e^3).
__device__ inline double rsqrt_pos(double z) {
    const double y0 = __builtin_amdgcn_rsq(z);
    const double e = fma(-z * y0, y0, 1.0);
    return fma(y0 * e, fma(e, 0.375, 0.5), y0);
}
__device__ inline bool schur2_rs(double app, double aqq, double apq, double tol, double& c, double& s, double& dp,
                                 double& dq) {
    c = 1.0;
    s = 0.0;
    dp = app;
    dq = aqq;
    if (!(apq * apq > tol * tol * fabs(app * aqq))) return false;
    const double d = aqq - app, g = 2.0 * apq;
    const double hh = d * d + g * g;
    if (!(hh >= 0x1p-1022) || !(hh < INFINITY)) return false;  // squares out of range: leave the pair
    const double rh = rsqrt_pos(hh);
    const double u = 0.5 + 0.5 * fabs(d) * rh;
    const double rc = rsqrt_pos(u);
    c = u * rc;
    s = (d >= 0.0 ? 0.5 : -0.5) * g * rh * rc;
    const double t = s * rc;
    dp = app - t * apq;
    dq = aqq + t * apq;
    return true;
}

// Output row held in register v by `lane` for the 16 x 16 MFMA blocks (the
// column is lane % 16): the FP32-accumulating f32 / bf16 forms hold rows
// 4*(lane/16) + v, the f64 form holds rows lane/16 + 4*v (measured on gfx950).
template <int P>
__device__ inline int mfma16_row(int lane, int v) {
    return prec_f64_mfma(P) ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
}

// ------------------------------------------------------------ launchers
// All launchers enqueue on `st` and return hipGetLastError().

// Gram / cross-Gram partials: part[split][pair][64*64] in FP64.
//   X: (L, nx, R) view, Y: (L, ny, R) view (Y == X and sym for a Gram matrix).
struct GramPlan {
    int layout;
    int64_t L, R;
    int nx, ny;
    int sym;
    int tiles_x, tiles_y, npairs;
    int64_t steps;   // K steps of depth KDepth
    int nsplit;
    int planes;      // SR: planes of R per step
    size_t part_bytes, part_capacity;
};
GramPlan gram_plan(int prec, int64_t L, int nx, int ny, int64_t R, bool sym, size_t part_capacity_bytes);
hipError_t launch_gram(int prec, const GramPlan& g, const void* X, const void* Y, double* part,
                       hipStream_t st);
// Sums the split partials in fixed order into C (nx x ny, row-major, FP64);
// symmetric plans write both triangles from the upper one.
hipError_t launch_gram_reduce(const GramPlan& g, const double* part, double* C, hipStream_t st);

// Gram matrix of a float32 (L, n, 1) view with n <= 16 (rows of n floats back
// to back, X 16-byte aligned) into G (n x n FP64): FP64 MFMA with exact
// products, partials (one n x n per workgroup) in part.
bool gram_tall_applicable(int prec, int n, int64_t R);
hipError_t launch_gram_tall(const float* X, int n, int64_t L, double* part, size_t part_capacity_bytes, double* G,
                            hipStream_t st);

// Gram matrix of a float32 (L, n, R) view with contiguous R (R >= 32, R % 4 == 0):
// 128 x 128 MFMA tiles, split-K, FP32 partial tiles + FP64 exact diagonal.
struct GramKcPlan {
    int64_t L, R;
    int n;
    int tiles, npairs;
    int64_t steps;
    int nsplit;      // multiple of 8 (one group per XCD)
    size_t part_bytes, dpart_bytes;
    bool ok;
};
bool gram_kc_applicable(int prec, int64_t R);
GramKcPlan gram_kc_plan(int prec, int64_t L, int n, int64_t R, size_t part_capacity_bytes,
                        size_t dpart_capacity_bytes);
hipError_t launch_gram_kc(int prec, const GramKcPlan& g, const float* X, float* part, double* dpart,
                          hipStream_t st);
hipError_t launch_gram_kc_reduce(const GramKcPlan& g, const float* part, const double* dpart, double* G,
                                 hipStream_t st);

// Mode product Z = M x_k Y on the (L, n, R) view: Z[l, j, r] = sum_i M[j, i] Y[l, i, r].
// M is m_out x n row-major: FP64 for PREC_F64, FP32 for PREC_F32, and for
// PREC_BF16X3 two bf16 arrays (Mh, Ml) holding hi/lo of the FP32 matrix.
struct TtmPlan {
    int layout;
    int64_t L, R;
    int n, m_out;
    int64_t ctiles;  // column tiles
    int jtiles;
    int planes;
    int64_t tiles_per_l;
};
TtmPlan ttm_plan(int prec, int64_t L, int n, int64_t R, int m_out);
// m_dev (optional): the output rows are min(t.m_out, *m_dev), read on the
// device (a rank chosen by a kernel earlier on the stream); none when < 1.
// kpart (optional, kpart_bytes of device scratch): lets a product over few
// output tiles and a long mode split its K range across workgroups into
// partial outputs that a second kernel sums in a fixed order.
hipError_t launch_ttm(int prec, const TtmPlan& t, const void* Y, const void* M, const void* Mh,
                      const void* Ml, void* Z, hipStream_t st, const int32_t* m_dev = nullptr,
                      float* kpart = nullptr, size_t kpart_bytes = 0);
// The last two mode products of a reconstruction in one pass (float32): Y is
// (L, r_a, r_b) row-major, U_a n_a x r_a and U_b n_b x r_b (the factors as
// given), X (L, n_a, n_b) = Y x_a U_a x_b U_b.  For r_a <= 32, r_b <= 16,
// n_a <= 128, n_b <= 64 (and X 16-byte aligned when n_b % 4 == 0): the fits
// test, then the launch (hipErrorInvalidValue when it does not fit).
bool ttm_fused_last2_fits(int64_t L, int ra, int rb, int na, int nb, const void* X);
hipError_t launch_ttm_fused_last2(const float* Y, int64_t L, int ra, int rb, int na, int nb, const float* Ua,
                                  const float* Ub, float* X, hipStream_t st);

// Symmetric eigensolvers (FP64).  Outputs lam (descending; not clamped, so a
// tail sum over rounding-level eigenvalues of an FP32-accurate Gram matrix
// averages their errors instead of keeping only the positive ones) and
// V (row-major n x ncols, column j is the eigenvector of lam[j]).
// Dense one-workgroup Jacobi with the matrix in LDS, n <= 64.
hipError_t launch_eig_jacobi_lds(const double* G, int n, int ldg, int max_sweeps, double* lam,
                                 double* V, int ldv, int32_t* sweeps_out, int32_t* ok_out,
                                 hipStream_t st, double floor_rel = 0.0);
// Dense one-workgroup Jacobi in global memory, any n (slow; fallback).
hipError_t launch_eig_jacobi_global(const double* G, int n, int max_sweeps, double* A_ws, double* lam,
                                    double* V, int32_t* sweeps_out, int32_t* ok_out, hipStream_t st);

// Subspace iteration with Rayleigh-Ritz for the leading m eigenpairs of an
// n x n PSD matrix (n > 64, m <= 64).  ws must hold subspace_ws_doubles(n, m).
size_t subspace_ws_doubles(int n, int m);
hipError_t run_subspace_eig(const double* G, int n, int m, int iters, int max_sweeps, double* ws,
                            double* lam, double* V, int32_t* sweeps_out, int32_t* ok_out,
                            hipStream_t st);

// Rank choice, sign rule and factor output for mode position i (of d) on mode k.
// Outcome of a selection kernel that the host polls for: pinned host memory,
// written by the kernel with seq last (after a system-scope fence).
struct HostFlags {
    int32_t seq;
    int32_t rank, need_dense, eig_ok, status, sweeps;
    int32_t pad[2];
    double tail, budget, norm2, used;  // this mode's book entries, |A|^2, discarded energy so far
};

struct SelectArgs {
    const double* lam;    // descending eigenvalues (ncand of them)
    const double* V;      // n x ncand, column j <-> lam[j]
    int ldv;
    const double* G;      // the Gram matrix (trace), ldg = n
    int n;
    int ncand;            // n (dense) or m (subspace)
    int subspace;         // 1: tails are trace - prefix sums, rank must leave a guard
    int guard;
    int pos, d, k;
    int rule;             // atc_rank_rule
    int fixed_rank;       // -1: budget rule
    double rtmss, eps2;
    DevBook* book;
    void* ufac;           // user factor n x r row-major (dtype)
    int ufac_f64;
    double* Mt64;         // U^T, r x n, FP64 (mode product of the FP64 path)
    float* Mt32;          // U^T, r x n, FP32
    __bf16* Mth;          // hi/lo split of Mt32
    __bf16* Mtl;
    HostFlags* hflags;    // null: no host report
    int32_t seq;          // value written to hflags->seq
    int32_t publish_late; // one-launch m = 32 path: report after the last grid barrier
                          // (the last processed mode: nothing waits on it, and a
                          // barrier wait that gave up is then still reported)
    // optional (null: not written): (W_r diag(signs))^T, r x 32, the Ritz
    // rotation that takes the projection onto the basis Q to the projection
    // onto U = Q W_r diag(signs) (split path of the m = 32 solver)
    double* Wt64;
    float* Wt32;
    __bf16* Wth;
    __bf16* Wtl;
};
hipError_t launch_select_factor(const SelectArgs& a, hipStream_t st);

// Subspace path with m = 32 for 64 <= n <= 512: power steps whose bases are
// orthonormalised by one-sided Jacobi in LDS, then a fused Rayleigh-Ritz step
// that also runs the rank choice and factor output of launch_select_factor.
// sa must have ncand = ldv = 32 and subspace = 1; its lam and V (n x 32) are
// written.  ws holds subspace32_ws_doubles(n) doubles.
bool subspace32_available(int n);
size_t subspace32_ws_doubles(int n);
// The m = 32 solver in two launches, so that the mode product by the basis can
// run beside the Rayleigh-Ritz step: run_subspace32_basis leaves the
// orthonormal basis Q (n x 32) and G Q in ws and writes Q^T (32 x n) into the
// mode-product operand buffers of qt (FP64, or FP32 with its bf16 hi / lo
// split; null pointers are skipped); run_rr32_select then takes the
// Rayleigh-Ritz step, rank choice and factor output (sa as for
// run_subspace32_select, with sa.Wt* set for the rotation operand; iters as
// given to the basis launch).  When the
// basis fails, the first launch reports the hand-over and the second does
// nothing.  split_rows_dev(ws, n): a device int, 32 once the basis stands and
// 0 when the mode is handed on (set by either launch); the product by the
// basis takes it as its device-side row count, so that its workgroups stop
// early when the result will not be used.
struct QtOut {
    double* t64;
    float* t32;
    __bf16* th;
    __bf16* tl;
};
bool subspace32_split_available(int n);  // the basis launch is cooperative
hipError_t run_subspace32_basis(const double* G, int n, int iters, double* ws, const SelectArgs& sa, const QtOut& qt,
                                hipStream_t st);
hipError_t run_rr32_select(int n, int iters, int max_sweeps, double* ws, const SelectArgs& sa, hipStream_t st);
const int32_t* split_rows_dev(const double* ws, int n);
hipError_t run_subspace32_select(const double* G, int n, int iters, int max_sweeps, double* ws, const SelectArgs& sa,
                                 hipStream_t st, bool allow_coop = true);
// m = 64 for 64 <= n <= 512 from the m = 32 kernels: the block as two
// orthonormalised 32-column halves, the 64 x 64 Rayleigh-Ritz problem on the
// LDS Jacobi, then launch_select_factor (sa: ncand = ldv = 64, subspace = 1,
// V = the n x 64 Ritz vectors written here, lam likewise).  ws holds
// subspace64b_ws_doubles(n) doubles.
size_t subspace64b_ws_doubles(int n);
hipError_t run_subspace64_select(const double* G, int n, int max_sweeps, double* ws, double* lam, double* V,
                                 int32_t* sweeps_dev, int32_t* ok_dev, const SelectArgs& sa, hipStream_t st,
                                 bool allow_coop = true);

// Prepares the mode-product matrix for reconstruction: M = U (n x r, dtype)
// converted to FP64 / FP32 / bf16 hi-lo.  transpose != 0 gives U^T (r x n).
hipError_t launch_prepare_matrix(int prec, const void* U, int src_f64, int rows, int cols, int transpose,
                                 double* M64, float* M32, __bf16* Mh, __bf16* Ml, hipStream_t st);

// Message returned by atc_last_error() on the calling thread.
void set_last_error(const char* msg);

// Reconstruction helpers of the C ABI: argument checks (shape, then ranks
// 1 <= r_k <= n_k; the last error is set on failure) and the decompression
// order of Section 4.1.1 (exhaustive search, first lexicographic on ties).
atc_status check_recon_args(const atc_shape* s, const int64_t* ranks);
void recon_order(const atc_shape* s, const int64_t* ranks, int* order);

// Zeroes n bytes with a kernel (capturable in a graph, unlike memset nodes).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);

// Batched forms of atc_quantize_core and atc_dequantize_core: `count` arrays
// (1 .. ATC_MAX_DIMS) of one dtype and block length share every launch, grid
// slice z working on task z.  Fields as in the C entry points, checked by the
// caller; ws sized by atc_quantize_workspace_size / atc_dequantize_workspace_size
// for the task's n.
struct QuantTask {
    const void* x;
    int64_t n;
    double target;
    uint32_t* enc;
    size_t enc_words;
    atc_quant_info* info;
    void* ws;
};
hipError_t quantize_batch(const QuantTask* tasks, int count, int f64, int len, hipStream_t st);
struct DequantTask {
    const uint32_t* enc;
    int64_t n;
    void* out;
    int32_t* status;
    void* ws;
};
hipError_t dequantize_batch(const DequantTask* tasks, int count, int f64, int len, hipStream_t st);

// Batched forms of the factor steps of the hybrid compressor (supplement S.2,
// eq. (total_error_approximation)): one workgroup (or grid slice) per factor,
// `count` factors (1 .. ATC_MAX_DIMS) of one dtype per launch, each n x r
// with 1 <= r <= n <= 4096, r <= 256 (checked by the caller).  A step reads
// and writes the fields that its C entry point takes.
struct FactorTask {
    int64_t n;
    int r;
    const void* U;          // the factor (encode, error term)
    const double* s2;       // squared slice norms of the quantized core (NULL: unweighted encode)
    double* coef;           // reflector entries (written by encode, weighted in place)
    int32_t* signs;         // column signs (encode)
    void* Uprime;           // the signed factor (encode; may be NULL)
    const double* entries;  // the entries a factor is rebuilt from (decode)
    void* Uq;               // the rebuilt factor (decode, error term)
    double* err;            // |dU Sigma|_F^2 (error term)
    double* ws;             // atc_householder_workspace_size(n, r) bytes (encode, decode)
};
hipError_t householder_encode_batch(const FactorTask* t, int count, int f64, hipStream_t st);
hipError_t householder_weight_batch(const FactorTask* t, int count, hipStream_t st);
hipError_t householder_decode_batch(const FactorTask* t, int count, int f64, hipStream_t st);
hipError_t factor_error_batch(const FactorTask* t, int count, int f64, hipStream_t st);

}  // namespace atc
