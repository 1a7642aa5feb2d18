// FP64 symmetric eigensolvers, rank choice and factor extraction.
//
// Algorithm 1 (Section 3.2) needs, per mode, the left singular vectors of the
// unfolding and its singular values; they are the eigenvectors of the Gram
// matrix G and the square roots of its eigenvalues.  Everything here is FP64:
// the Gram matrix squares the conditioning of the unfolding, so the
// eigenvalues that decide the rank (Section 4.1.3: discarded SSE = sum of the
// discarded squared singular values) need the extra precision.
//
// Dense path: cyclic two-sided Jacobi with the round-robin parallel ordering
// (m/2 disjoint rotations per round, m-1 rounds per sweep).  A rotation is
// skipped when |a_pq| <= tol * sqrt(|a_pp a_qq|), tol = n * 2^-53; a rotated
// pair is annihilated exactly and its diagonal set from the 2 x 2 formulas;
// a sweep with no rotation ends the iteration.  For m <= 64 one workgroup
// holds the matrix and the eigenvectors in LDS and thread (k, l) owns the
// 2 x 2 block (pair k, pair l), so a round is one read-modify-write pass.
// Larger n use the same iteration in global memory (slow; a fallback).
//
// Subspace path (n > 64): the ranks this method keeps are small next to n, so
// only the leading m (32 or 64) eigenpairs are needed: power steps with CGS2
// re-orthonormalisation, Q_0 = orth(G Omega), Q_t = orth(G Q_{t-1}), then a
// Rayleigh-Ritz projection B = Q^T G Q = W diag(theta) W^T, U = Q W, the
// m x m problem solved by the LDS Jacobi.  Ritz values never exceed the true
// eigenvalues, so the tail trace(G) - sum(kept Ritz values) over-estimates the
// discarded energy and the error bound still holds; a rank that reaches into
// the last `guard` Ritz pairs sends the mode to a larger m or the dense path.
#include <math.h>
#include <stdlib.h>

#include "atc_internal.hpp"
#include "atc_jacobi64.hpp"

namespace atc {
namespace {

__device__ inline void round_robin_pair(int round, int k, int m, int& p, int& q) {
    // circle method: player 0 fixed, players 1..m-1 rotate
    if (k == 0) {
        p = 0;
        q = 1 + round % (m - 1);
    } else {
        p = 1 + (round + k) % (m - 1);
        q = 1 + (round + (m - 1) - k) % (m - 1);
    }
    if (p > q) {
        const int t = p;
        p = q;
        q = t;
    }
}

// Symmetric 2x2 Schur rotation: [c s; -s c]^T [app apq; apq aqq] [c s; -s c] is
// diagonal, with new diagonal (app - t apq, aqq + t apq), t = s / c.
__device__ inline bool schur2(double app, double aqq, double apq, double tol, double& c, double& s, double& dp,
                              double& dq) {
    c = 1.0;
    s = 0.0;
    dp = app;
    dq = aqq;
    if (apq == 0.0) return false;
    if (fabs(apq) <= tol * sqrt(fabs(app)) * sqrt(fabs(aqq))) return false;
    const double tau = (aqq - app) / (2.0 * apq);
    double t;
    if (fabs(tau) > 1e150) t = 0.5 / tau;
    else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    c = 1.0 / sqrt(1.0 + t * t);
    s = t * c;
    dp = app - t * apq;
    dq = aqq + t * apq;
    return true;
}

// deterministic pseudo-random value in [-1, 1) (splitmix64 of the key)
__device__ inline double hash_unit(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (double)(x >> 11) * 0x1p-52 - 1.0;
}

// Sum over the workgroup in a fixed order (wave shuffles, then waves in order).
__device__ inline double block_sum(double s, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += red[w];
        red[16] = t;
    }
    __syncthreads();
    const double r = red[16];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------- LDS Jacobi (m <= 64)
template <int MAXM>
__global__ __launch_bounds__((MAXM / 2) * (MAXM / 2)) void k_eig_jacobi_lds(
    const double* __restrict__ G, int n, int ldg, int max_sweeps, double* __restrict__ lam, double* __restrict__ V,
    int ldv, int32_t* __restrict__ sweeps_out, int32_t* __restrict__ ok_out, double floor_rel) {
    constexpr int H = MAXM / 2;
    __shared__ double A[MAXM][MAXM + 1];
    __shared__ double Vs[MAXM][MAXM + 1];
    __shared__ int pp[H], qq[H];
    __shared__ double cs[H], sn[H], dpp[H], dqq[H];
    __shared__ int rotated;
    __shared__ int rank_of[MAXM];
    const int tid = threadIdx.x;
    const int m = n + (n & 1);
    const int h = m / 2;
    const int kb = tid / H, lb = tid % H;  // row pair, column pair of this thread's block
    for (int idx = tid; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m;
        A[i][j] = (i < n && j < n) ? G[(int64_t)i * ldg + j] : 0.0;
        Vs[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const double tol = (double)n * 0x1p-53;
    // with floor_rel > 0 an entry at or below floor_rel |trace| is left alone
    double trace = 0.0;
    for (int i = 0; i < n; ++i) trace += A[i][i];
    const double floor = floor_rel * fabs(trace);
    int sweeps = 0;
    bool converged = (m < 2);
    while (!converged && sweeps < max_sweeps) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int round = 0; round < m - 1; ++round) {
            if (tid < h) {
                int p, q;
                round_robin_pair(round, tid, m, p, q);
                double c = 1.0, s = 0.0, dp = A[p][p], dq = A[q][q];
                if (fabs(A[p][q]) > floor && schur2_rs(A[p][p], A[q][q], A[p][q], tol, c, s, dp, dq)) rotated = 1;
                pp[tid] = p;
                qq[tid] = q;
                cs[tid] = c;
                sn[tid] = s;
                dpp[tid] = dp;
                dqq[tid] = dq;
            }
            __syncthreads();
            if (kb < h && lb < h) {
                const int p = pp[kb], q = qq[kb];
                const double c1 = cs[kb], s1 = sn[kb];
                if (kb == lb) {
                    if (s1 != 0.0) {
                        A[p][p] = dpp[kb];
                        A[q][q] = dqq[kb];
                        A[p][q] = 0.0;
                        A[q][p] = 0.0;
                    }
                } else if (kb < lb) {
                    // block (rows p,q ; cols p2,q2) <- J_k^T block J_l, mirrored into (l, k)
                    const int p2 = pp[lb], q2 = qq[lb];
                    const double c2 = cs[lb], s2 = sn[lb];
                    if (s1 != 0.0 || s2 != 0.0) {
                        const double a = A[p][p2], b = A[p][q2], c = A[q][p2], d = A[q][q2];
                        const double ra = c1 * a - s1 * c, rb = c1 * b - s1 * d;
                        const double rc = s1 * a + c1 * c, rd = s1 * b + c1 * d;
                        const double na = c2 * ra - s2 * rb, nb = s2 * ra + c2 * rb;
                        const double nc = c2 * rc - s2 * rd, nd = s2 * rc + c2 * rd;
                        A[p][p2] = na;
                        A[p][q2] = nb;
                        A[q][p2] = nc;
                        A[q][q2] = nd;
                        A[p2][p] = na;
                        A[q2][p] = nb;
                        A[p2][q] = nc;
                        A[q2][q] = nd;
                    }
                }
                // eigenvector rows 2 lb and 2 lb + 1, columns of pair k: V <- V J_k
                if (s1 != 0.0) {
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const int i = 2 * lb + t;
                        const double x = Vs[i][p], y = Vs[i][q];
                        Vs[i][p] = c1 * x - s1 * y;
                        Vs[i][q] = s1 * x + c1 * y;
                    }
                }
            }
            __syncthreads();
        }
        ++sweeps;
        converged = (rotated == 0);
        __syncthreads();
    }
    // eigenvalues = diagonal; order descending, equal values by index
    for (int i = tid; i < n; i += blockDim.x) {
        const double li = A[i][i];
        int r = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = A[j][j];
            r += (lj > li) || (lj == li && j < i);
        }
        rank_of[i] = r;
    }
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) lam[rank_of[i]] = A[i][i];  // unclamped (see select)
    for (int idx = tid; idx < n * n; idx += blockDim.x) {
        const int row = idx / n, i = idx % n;
        V[(int64_t)row * ldv + rank_of[i]] = Vs[row][i];
    }
    if (tid == 0) {
        if (sweeps_out) *sweeps_out = sweeps;
        if (ok_out) *ok_out = converged ? 1 : 0;
    }
}

// --------------------------------------------------------------- global Jacobi
// Same iteration with A (m x m) and V in global memory; one workgroup.
__global__ __launch_bounds__(1024) void k_eig_jacobi_global(const double* __restrict__ G, int n, int max_sweeps,
                                                            double* __restrict__ A, double* __restrict__ lam,
                                                            double* __restrict__ V, double* __restrict__ Vw,
                                                            int32_t* __restrict__ sweeps_out,
                                                            int32_t* __restrict__ ok_out) {
    extern __shared__ double dyn[];
    const int m = n + (n & 1);
    int* pp = reinterpret_cast<int*>(dyn);
    int* qq = pp + m / 2;
    double* cs = reinterpret_cast<double*>(pp + m);  // 4*m bytes: 8-aligned for even m
    double* sn = cs + m / 2;
    double* dpp = sn + m / 2;
    double* dqq = dpp + m / 2;
    __shared__ int rotated;
    const int tid = threadIdx.x;
    for (int64_t idx = tid; idx < (int64_t)m * m; idx += blockDim.x) {
        const int i = (int)(idx / m), j = (int)(idx % m);
        A[idx] = (i < n && j < n) ? G[(int64_t)i * n + j] : 0.0;
        Vw[idx] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const double tol = (double)n * 0x1p-53;
    int sweeps = 0;
    bool converged = (m < 2);
    while (!converged && sweeps < max_sweeps) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int round = 0; round < m - 1; ++round) {
            for (int k = tid; k < m / 2; k += blockDim.x) {
                int p, q;
                round_robin_pair(round, k, m, p, q);
                double c, s, dp, dq;
                if (schur2(A[(int64_t)p * m + p], A[(int64_t)q * m + q], A[(int64_t)p * m + q], tol, c, s, dp, dq))
                    rotated = 1;
                pp[k] = p;
                qq[k] = q;
                cs[k] = c;
                sn[k] = s;
                dpp[k] = dp;
                dqq[k] = dq;
            }
            __syncthreads();
            for (int64_t idx = tid; idx < (int64_t)(m / 2) * m; idx += blockDim.x) {
                const int k = (int)(idx / m), j = (int)(idx % m);
                const double c = cs[k], s = sn[k];
                if (s == 0.0) continue;
                const int64_t p = pp[k], q = qq[k];
                const double x = A[p * m + j], y = A[q * m + j];
                A[p * m + j] = c * x - s * y;
                A[q * m + j] = s * x + c * y;
            }
            __syncthreads();
            for (int64_t idx = tid; idx < (int64_t)m * (m / 2); idx += blockDim.x) {
                const int64_t i = idx / (m / 2);
                const int k = (int)(idx % (m / 2));
                const double c = cs[k], s = sn[k];
                if (s == 0.0) continue;
                const int p = pp[k], q = qq[k];
                const double x = A[i * m + p], y = A[i * m + q];
                A[i * m + p] = c * x - s * y;
                A[i * m + q] = s * x + c * y;
                const double vx = Vw[i * m + p], vy = Vw[i * m + q];
                Vw[i * m + p] = c * vx - s * vy;
                Vw[i * m + q] = s * vx + c * vy;
            }
            __syncthreads();
            for (int k = tid; k < m / 2; k += blockDim.x) {
                if (sn[k] == 0.0) continue;
                const int64_t p = pp[k], q = qq[k];
                A[p * m + q] = 0.0;
                A[q * m + p] = 0.0;
                A[p * m + p] = dpp[k];
                A[q * m + q] = dqq[k];
            }
            __syncthreads();
        }
        ++sweeps;
        converged = (rotated == 0);
        __syncthreads();
    }
    for (int i = tid; i < n; i += blockDim.x) {
        const double li = A[(int64_t)i * m + i];
        int r = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = A[(int64_t)j * m + j];
            r += (lj > li) || (lj == li && j < i);
        }
        lam[r] = li;
        for (int row = 0; row < n; ++row) V[(int64_t)row * n + r] = Vw[(int64_t)row * m + i];
    }
    if (tid == 0) {
        *sweeps_out = sweeps;
        *ok_out = converged ? 1 : 0;
    }
}

// ------------------------------------------------------- small FP64 products
// C (n x m) = A (n x n, row-major) * B (n x m, row-major), m <= 64.
// A workgroup stages 4 rows of A (in chunks of 512) and computes 4 x m outputs.
constexpr int GR_ROWS = 4;
constexpr int GR_KC = 512;
__global__ __launch_bounds__(256) void k_gemm_rows(const double* __restrict__ A, const double* __restrict__ B,
                                                   double* __restrict__ C, int n, int m) {
    __shared__ double As[GR_ROWS][GR_KC];
    const int tid = threadIdx.x;
    const int r = tid >> 6, j = tid & 63;
    const int row = blockIdx.x * GR_ROWS + r;
    double acc = 0.0;
    for (int k0 = 0; k0 < n; k0 += GR_KC) {
        const int kc = min(GR_KC, n - k0);
        for (int idx = tid; idx < GR_ROWS * GR_KC; idx += blockDim.x) {
            const int rr = idx / GR_KC, kk = idx % GR_KC;
            const int grow = blockIdx.x * GR_ROWS + rr;
            As[rr][kk] = (grow < n && kk < kc) ? A[(int64_t)grow * n + k0 + kk] : 0.0;
        }
        __syncthreads();
        if (j < m)
            for (int kk = 0; kk < kc; ++kk) acc += As[r][kk] * B[(int64_t)(k0 + kk) * m + j];
        __syncthreads();
    }
    if (row < n && j < m) C[(int64_t)row * m + j] = acc;
}

// Partial C_c = A_c^T B_c over row chunk c of 64 rows (A: n x ma, B: n x mb).
constexpr int TN_ROWS = 64;
__global__ __launch_bounds__(256) void k_gemm_tn_partial(const double* __restrict__ A, const double* __restrict__ B,
                                                         double* __restrict__ part, int n, int ma, int mb) {
    __shared__ double As[TN_ROWS][65];
    __shared__ double Bs[TN_ROWS][65];
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * TN_ROWS;
    for (int idx = tid; idx < TN_ROWS * 64; idx += blockDim.x) {
        const int rr = idx / 64, c = idx % 64;
        const int row = r0 + rr;
        As[rr][c] = (row < n && c < ma) ? A[(int64_t)row * ma + c] : 0.0;
        Bs[rr][c] = (row < n && c < mb) ? B[(int64_t)row * mb + c] : 0.0;
    }
    __syncthreads();
    double* out = part + (int64_t)blockIdx.x * ma * mb;
    for (int o = tid; o < ma * mb; o += blockDim.x) {
        const int i = o / mb, j = o % mb;
        double s = 0.0;
        for (int rr = 0; rr < TN_ROWS; ++rr) s += As[rr][i] * Bs[rr][j];
        out[o] = s;
    }
}

__global__ void k_sum_partials(const double* __restrict__ part, int nparts, int count, double* __restrict__ C) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= count) return;
    double s = 0.0;
    for (int c = 0; c < nparts; ++c) s += part[(int64_t)c * count + o];
    C[o] = s;
}

// C (n x mb) = A (n x ma) * W (ma x mb), everything row-major, ma, mb <= 64.
__global__ __launch_bounds__(256) void k_gemm_small(const double* __restrict__ A, const double* __restrict__ W,
                                                    double* __restrict__ C, int n, int ma, int mb) {
    __shared__ double Ws[64][65];
    const int tid = threadIdx.x;
    for (int idx = tid; idx < ma * mb; idx += blockDim.x) Ws[idx / mb][idx % mb] = W[idx];
    __syncthreads();
    const int r = tid >> 6, j = tid & 63;
    const int row = blockIdx.x * 4 + r;
    if (row >= n || j >= mb) return;
    double s = 0.0;
    for (int c = 0; c < ma; ++c) s += A[(int64_t)row * ma + c] * Ws[c][j];
    C[(int64_t)row * mb + j] = s;
}

__global__ void k_fill_random(double* Q, int n, int m, uint64_t salt) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < (int64_t)n * m) Q[idx] = hash_unit((uint64_t)idx * 0x2545F4914F6CDD1Dull + salt);
}

// Orthonormalises the columns of X (n x m, row-major, in place) by classical
// Gram-Schmidt applied twice per column (CGS2); a column that loses all but
// 1e-10 of its norm is numerically dependent and is replaced by a
// pseudo-random vector (then orthogonalised again), or zeroed if that fails.
// One workgroup; the whole basis sits column-major in LDS (n * m doubles).
__global__ __launch_bounds__(1024) void k_cgs2_lds(double* __restrict__ X, int n, int m, uint64_t salt) {
    extern __shared__ double Xs[];  // column c at Xs + c * n
    __shared__ double h[64];
    __shared__ double red[17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    for (int idx = tid; idx < n * m; idx += blockDim.x) {
        const int i = idx / m, c = idx % m;
        Xs[c * n + i] = X[idx];
    }
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        double* xj = Xs + j * n;
        for (int attempt = 0; attempt < 2; ++attempt) {
            double s = 0.0;
            for (int i = tid; i < n; i += blockDim.x) s += xj[i] * xj[i];
            const double norm0 = sqrt(block_sum(s, red));
            for (int pass = 0; pass < 2 && j > 0; ++pass) {
                for (int c = wave; c < j; c += nw) {
                    const double* xc = Xs + c * n;
                    double d = 0.0;
                    for (int i = lane; i < n; i += 64) d += xc[i] * xj[i];
                    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
                    if (lane == 0) h[c] = d;
                }
                __syncthreads();
                for (int i = tid; i < n; i += blockDim.x) {
                    double v = xj[i];
                    for (int c = 0; c < j; ++c) v -= Xs[c * n + i] * h[c];
                    xj[i] = v;
                }
                __syncthreads();
            }
            s = 0.0;
            for (int i = tid; i < n; i += blockDim.x) s += xj[i] * xj[i];
            const double nrm = sqrt(block_sum(s, red));
            if (nrm > 1e-10 * norm0 && nrm > 0.0 && isfinite(nrm)) {
                for (int i = tid; i < n; i += blockDim.x) xj[i] /= nrm;
                __syncthreads();
                break;
            }
            for (int i = tid; i < n; i += blockDim.x)
                xj[i] = attempt == 0 ? hash_unit(((uint64_t)i * 977 + j) * 0x2545F4914F6CDD1Dull + salt) : 0.0;
            __syncthreads();
        }
    }
    for (int idx = tid; idx < n * m; idx += blockDim.x) {
        const int i = idx / m, c = idx % m;
        X[idx] = Xs[c * n + i];
    }
}

// The same with the basis in global memory (n * m too large for LDS).
__global__ __launch_bounds__(1024) void k_cgs2_global(double* __restrict__ X, int n, int m, uint64_t salt) {
    extern __shared__ double col[];  // n doubles
    __shared__ double h[64];
    __shared__ double red[17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    for (int j = 0; j < m; ++j) {
        for (int i = tid; i < n; i += blockDim.x) col[i] = X[(int64_t)i * m + j];
        __syncthreads();
        for (int attempt = 0; attempt < 2; ++attempt) {
            double s = 0.0;
            for (int i = tid; i < n; i += blockDim.x) s += col[i] * col[i];
            const double norm0 = sqrt(block_sum(s, red));
            for (int pass = 0; pass < 2 && j > 0; ++pass) {
                for (int c = wave; c < j; c += nw) {
                    double d = 0.0;
                    for (int i = lane; i < n; i += 64) d += X[(int64_t)i * m + c] * col[i];
                    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
                    if (lane == 0) h[c] = d;
                }
                __syncthreads();
                for (int i = tid; i < n; i += blockDim.x) {
                    double v = col[i];
                    const double* xr = X + (int64_t)i * m;
                    for (int c = 0; c < j; ++c) v -= xr[c] * h[c];
                    col[i] = v;
                }
                __syncthreads();
            }
            s = 0.0;
            for (int i = tid; i < n; i += blockDim.x) s += col[i] * col[i];
            const double nrm = sqrt(block_sum(s, red));
            if (nrm > 1e-10 * norm0 && nrm > 0.0 && isfinite(nrm)) {
                for (int i = tid; i < n; i += blockDim.x) col[i] /= nrm;
                __syncthreads();
                break;
            }
            for (int i = tid; i < n; i += blockDim.x)
                col[i] = attempt == 0 ? hash_unit(((uint64_t)i * 977 + j) * 0x2545F4914F6CDD1Dull + salt) : 0.0;
            __syncthreads();
        }
        for (int i = tid; i < n; i += blockDim.x) X[(int64_t)i * m + j] = col[i];
        __syncthreads();
    }
}

constexpr size_t CGS2_LDS_MAX = 128 * 1024;  // bytes of basis kept in LDS

bool cgs2_lds_ready() {
    static int state = 0;  // 0 unknown, 1 ok, -1 not available
    if (state == 0) {
        state = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cgs2_lds),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)CGS2_LDS_MAX) == hipSuccess
                    ? 1
                    : -1;
    }
    return state == 1;
}

hipError_t orthonormalise(double* X, int n, int m, uint64_t salt, hipStream_t st) {
    const size_t bytes = sizeof(double) * (size_t)n * m;
    if (bytes <= CGS2_LDS_MAX && cgs2_lds_ready()) {
        hipLaunchKernelGGL(k_cgs2_lds, dim3(1), dim3(1024), bytes, st, X, n, m, salt);
    } else {
        hipLaunchKernelGGL(k_cgs2_global, dim3(1), dim3(1024), sizeof(double) * (size_t)n, st, X, n, m, salt);
    }
    return hipGetLastError();
}

// The 64 x 64 Jacobi in slot order (defined with the m = 64 subspace path).
__global__ __launch_bounds__(J64_THREADS) void k_jacobi64_slots(const double* __restrict__ G, int n, int ldg,
                                                                int max_sweeps, double* __restrict__ lam,
                                                                double* __restrict__ V, int ldv,
                                                                int32_t* __restrict__ sweeps_out,
                                                                int32_t* __restrict__ ok_out, double floor_rel);

}  // namespace

hipError_t launch_eig_jacobi_lds(const double* G, int n, int ldg, int max_sweeps, double* lam, double* V, int ldv,
                                 int32_t* sweeps_out, int32_t* ok_out, hipStream_t st, double floor_rel) {
    if (n < 1 || n > 64) return hipErrorInvalidValue;
    if (n <= 32)
        hipLaunchKernelGGL((k_eig_jacobi_lds<32>), dim3(1), dim3(256), 0, st, G, n, ldg, max_sweeps, lam, V, ldv,
                           sweeps_out, ok_out, floor_rel);
    else
        hipLaunchKernelGGL(k_jacobi64_slots, dim3(1), dim3(J64_THREADS), 0, st, G, n, ldg, max_sweeps, lam, V, ldv,
                           sweeps_out, ok_out, floor_rel);
    return hipGetLastError();
}

hipError_t launch_eig_jacobi_global(const double* G, int n, int max_sweeps, double* A_ws, double* lam, double* V,
                                    int32_t* sweeps_out, int32_t* ok_out, hipStream_t st) {
    const int m = n + (n & 1);
    // pair indices (2 x m/2 ints) then c, s and the two new diagonals (4 x m/2 doubles);
    // A_ws holds 2 * m * m doubles: the working matrix, then the eigenvector accumulator
    const size_t shm = (size_t)m * sizeof(int) + (size_t)2 * m * sizeof(double) + 64;
    if (shm > 64 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_eig_jacobi_global, dim3(1), dim3(1024), shm, st, G, n, max_sweeps, A_ws, lam, V,
                       A_ws + (size_t)m * m, sweeps_out, ok_out);
    return hipGetLastError();
}

size_t subspace_ws_doubles(int n, int m) {
    const size_t chunks = (size_t)ceil_div(n, TN_ROWS);
    return (size_t)3 * n * m + (size_t)2 * m * m + chunks * (size_t)m * m + 64;
}

// Leading m eigenpairs of the PSD matrix G (n x n): power steps with CGS2
// re-orthonormalisation, Q_0 = orth(G Omega), Q_t = orth(G Q_{t-1}), then the
// Rayleigh-Ritz projection B = Q^T G Q = W diag(theta) W^T, V = Q W (n x m).
hipError_t run_subspace_eig(const double* G, int n, int m, int iters, int max_sweeps, double* ws, double* lam,
                            double* V, int32_t* sweeps_out, int32_t* ok_out, hipStream_t st) {
    if (m > 64 || m < 2 || n < m || n > 4096) return hipErrorInvalidValue;
    double* Q = ws;                       // n x m
    double* Z = Q + (size_t)n * m;        // n x m
    double* Y = Z + (size_t)n * m;        // n x m
    double* B = Y + (size_t)n * m;        // m x m
    double* W = B + (size_t)m * m;        // m x m
    double* part = W + (size_t)m * m;     // chunks x m x m
    const int chunks = (int)ceil_div(n, TN_ROWS);
    hipError_t e;
    const unsigned gr = (unsigned)ceil_div(n, GR_ROWS);
    hipLaunchKernelGGL(k_fill_random, dim3((unsigned)ceil_div((int64_t)n * m, 256)), dim3(256), 0, st, Y, n, m,
                       (uint64_t)0x5eed);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int steps = iters < 1 ? 1 : iters;
    for (int it = 0; it < steps; ++it) {
        hipLaunchKernelGGL(k_gemm_rows, dim3(gr), dim3(256), 0, st, G, it == 0 ? Y : Z, Q, n, m);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = orthonormalise(Q, n, m, (uint64_t)(it + 1), st)) != hipSuccess) return e;
        if (it + 1 < steps) {
            if ((e = hipMemcpyAsync(Z, Q, sizeof(double) * n * m, hipMemcpyDeviceToDevice, st)) != hipSuccess)
                return e;
        }
    }
    hipLaunchKernelGGL(k_gemm_rows, dim3(gr), dim3(256), 0, st, G, Q, Z, n, m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gemm_tn_partial, dim3(chunks), dim3(256), 0, st, Q, Z, part, n, m, m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)ceil_div(m * m, 256)), dim3(256), 0, st, part, chunks, m * m, B);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_eig_jacobi_lds(B, m, m, max_sweeps, lam, W, m, sweeps_out, ok_out, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gemm_small, dim3(gr), dim3(256), 0, st, Q, W, V, n, m, m);
    return hipGetLastError();
}

// ------------------------------------------------------- rank select + factor
namespace {

// Reports the selection outcome to the host (one thread): the fields, a
// system-scope fence, then the sequence number the host waits for.
__device__ inline void publish_selection(const SelectArgs& a, int rank) {
    if (!a.hflags) return;
    volatile HostFlags* h = a.hflags;
    const DevBook* bk = a.book;
    h->rank = rank;
    h->need_dense = bk->need_dense;
    h->eig_ok = bk->eig_ok;
    h->status = bk->status;
    h->sweeps = bk->sweeps[a.k];
    h->tail = bk->tail[a.k];
    h->budget = bk->budget[a.k];
    h->norm2 = bk->norm2;
    h->used = bk->used;
    __threadfence_system();
    h->seq = a.seq;
}

// Rank choice (Section 4.1.3), sign rule and factor output for one mode, run
// by a whole workgroup (any multiple of 64 threads).  The pieces: gram_trace
// (every thread), choose_rank (thread 0: budget, rank, book, host flags),
// store_factor (one entry of the user factor and of the mode-product operand)
// and sign_factor_from_v (sign rule and factor output from V in global memory).

// trace of G (fixed-order block sum); red: 17 doubles of LDS
__device__ __forceinline__ double gram_trace(const SelectArgs& a, double* red) {
    double part = 0.0;
    for (int i = threadIdx.x; i < a.n; i += blockDim.x) part += a.G[(int64_t)i * a.n + i];
    return block_sum(part, red);
}

// Thread 0 only: the rank from the eigenvalues (or Ritz values) a.lam and the
// trace; the book entries, the host flags.  r_s <- rank, dense_s <- 1 when the
// subspace does not hold enough Ritz pairs (the caller then stops: the host
// moves to a larger eigensolver).
__device__ __forceinline__ void choose_rank(const SelectArgs& a, double tr, int& r_s, int& dense_s,
                                            bool publish = true) {
    DevBook* bk = a.book;
    if (a.pos == 0) {
        bk->norm2 = tr;
        bk->S = a.rtmss * a.eps2 * tr;
        bk->used = 0.0;
        if (!isfinite(tr)) bk->status = ATC_ERR_NONFINITE_INPUT;
    }
    bk->trace[a.k] = tr;
    const double b = (a.rule == ATC_RANK_EQUAL) ? bk->S / a.d : (bk->S - bk->used) / (a.d - a.pos);
    int r = a.n;
    double tail_r = 0.0;
    if (!a.subspace) {
        // tail(r) = sum_{j >= r} lam_j, added from the smallest upward; the
        // eigenvalues are not clamped, so rounding-level negative values of
        // an FP32-accurate Gram matrix offset the positive ones
        double acc = 0.0;
        int best = a.n;
        double best_tail = 0.0;
        for (int j = a.n - 1; j >= 0; --j) {
            if (acc <= b) {  // acc = tail at r = j + 1
                best = j + 1;
                best_tail = acc;
            }
            acc += a.lam[j];
        }
        r = best;
        tail_r = best_tail;
        if (a.fixed_rank > 0) {
            r = a.fixed_rank;
            double t = 0.0;
            for (int j = a.n - 1; j >= r; --j) t += a.lam[j];
            tail_r = t;
        }
    } else {
        // tail(r) = trace - sum_{j < r} theta_j (an upper bound of the true tail)
        double pre = 0.0;
        int found = -1;
        for (int j = 0; j < a.ncand; ++j) {
            pre += a.lam[j];
            const double t = tr - pre;
            if (found < 0 && t <= b) {
                found = j + 1;
                tail_r = t > 0.0 ? t : 0.0;
            }
            if (a.fixed_rank > 0 && j + 1 == a.fixed_rank) {
                found = a.fixed_rank;
                tail_r = t > 0.0 ? t : 0.0;
                break;
            }
        }
        if (found < 0 || found > a.ncand - a.guard || !(a.lam[found - 1] > 0.0)) {
            bk->need_dense = 1;
            found = a.ncand < a.n ? a.ncand : a.n;
        }
        r = found;
    }
    const int dense = bk->need_dense;
    if (dense == 0) {
        bk->used += tail_r;
        bk->tail[a.k] = tail_r;
        bk->budget[a.k] = b;
        bk->rank[a.k] = r;
    }
    r_s = r;
    dense_s = dense;
    if (publish) publish_selection(a, r);
}

// Entry (i, j) of the factor, u with its sign applied: the user factor is
// row-major n x r, the mode-product operand U^T is r x n (FP64, or FP32 with
// its bf16 hi / lo split).
__device__ __forceinline__ void store_factor(const SelectArgs& a, int i, int j, int r, double u) {
    const int64_t idx = (int64_t)i * r + j;
    if (a.ufac_f64) ((double*)a.ufac)[idx] = u;
    else ((float*)a.ufac)[idx] = (float)u;
    const int64_t t = (int64_t)j * a.n + i;
    if (a.Mt64) a.Mt64[t] = u;
    if (a.Mt32) {
        const float f = (float)u;
        a.Mt32[t] = f;
        if (a.Mth) {
            const __bf16 hh = (__bf16)f;
            a.Mth[t] = hh;
            a.Mtl[t] = (__bf16)(f - (float)hh);
        }
    }
}

// Sign rule (largest-magnitude entry of each kept column positive, first row
// on ties) and factor output for the leading r columns of V (global, n x ldv).
// sign_s: r ints of LDS.
__device__ __forceinline__ void sign_factor_from_v(const SelectArgs& a, int r, int* sign_s) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    // one wave per column, lanes scan rows, then a fixed-order shuffle reduction
    for (int j = wave; j < r; j += nw) {
        double best = -1.0;
        int bi = 0x7fffffff;
        double val = 0.0;
        for (int i0 = lane; i0 < a.n; i0 += 8 * 64) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + 64 * u;
                v[u] = a.V[(int64_t)(i < a.n ? i : a.n - 1) * a.ldv + j];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + 64 * u;
                if (i < a.n && fabs(v[u]) > best) {
                    best = fabs(v[u]);
                    bi = i;
                    val = v[u];
                }
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o);
            const int oi = __shfl_xor(bi, o);
            const double ov = __shfl_xor(val, o);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
                val = ov;
            }
        }
        if (lane == 0) sign_s[j] = val < 0.0 ? -1 : 1;
    }
    __syncthreads();
    // 32-lane column groups (no division per element)
    const int lanes_per_row = 32;
    const int rows_per_pass = blockDim.x / lanes_per_row;
    const int jl = tid % lanes_per_row;
    constexpr int RB = 8;  // rows whose loads go out together
    for (int i0 = tid / lanes_per_row; i0 < a.n; i0 += RB * rows_per_pass) {
        for (int j = jl; j < r; j += lanes_per_row) {
            double vv[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int i = i0 + q * rows_per_pass;
                vv[q] = a.V[(int64_t)(i < a.n ? i : a.n - 1) * a.ldv + j];
            }
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int i = i0 + q * rows_per_pass;
                if (i >= a.n) break;
                store_factor(a, i, j, r, sign_s[j] * vv[q]);
            }
        }
    }
}

// red: 17 doubles, sign_s: n ints, r_s: 1 int, all in LDS.
__device__ __forceinline__ void select_factor_body(const SelectArgs& a, double* red, int* sign_s, int& r_s) {
    __shared__ int dense_s;
    const double tr = gram_trace(a, red);
    if (threadIdx.x == 0) choose_rank(a, tr, r_s, dense_s);
    __syncthreads();
    if (dense_s) return;
    sign_factor_from_v(a, r_s, sign_s);
}

// 512 threads: the sign rule takes one wavefront per column (8 in flight)
__global__ __launch_bounds__(512) void k_select_factor(SelectArgs a) {
    __shared__ int r_s;
    __shared__ double red[17];
    __shared__ int sign_s[4096];
    select_factor_body(a, red, sign_s, r_s);
}

// ------------------------------------------- subspace path, m = 32, n <= 512
// Orthogonal iteration with a Rayleigh-Ritz finish:
//   Y0 = G Omega          split-K FP64 product on many workgroups (Omega is a
//                         counter-based pseudo-random matrix made in the kernel)
//   Q0 = orth(Y0)         a shifted Cholesky QR pass, then a plain one, in one
//                         workgroup (the columns of Y0 spread like the
//                         eigenvalues of G, far beyond what plain Cholesky QR
//                         can orthonormalise)
//   Q1 = orth(G Q0)       the same two passes, then the series C^{-1/2} = I - E/2
//                         + 3 E^2 / 8 of C = Q^T Q = I + E, which also checks |E|
//   Z = G Q1
//   B = Q1^T Z = W diag(theta) W^T (one-wavefront Jacobi), the rank choice
//   from theta, then V = Q1 W in registers, its sign rule and the factor output.
constexpr int S32 = 32;
constexpr int GX_ROWS = 16;   // rows of G per workgroup of k_gemm_gx
constexpr int GX_SPLIT = 4;   // K chunks; the consumer adds the partial products
constexpr int OT = 512;       // threads of the orthonormalisation workgroup
constexpr int OW = OT / 64;   // its wavefronts
constexpr int RT = 512;       // threads of the Rayleigh-Ritz workgroup
constexpr int RW = RT / 64;
constexpr size_t ORTH_LDS = (size_t)(OW * S32 * S32 + 2 * S32 * (S32 + 1)) * sizeof(double);
constexpr size_t RR_LDS = (size_t)(RW * S32 * S32 + 2 * S32 * (S32 + 1)) * sizeof(double);

// Rows r0 .. r0 + 15 of G X over the s-th of GX_SPLIT K chunks into red (16 x
// 33, LDS), one wavefront, on v_mfma_f64_16x16x4f64 (eight K steps' loads in
// flight).  X == nullptr: X[k][j] = hash_unit((32 k + j) * C + salt).  Rows
// past n repeat row n - 1 (their results are not stored).
__device__ __forceinline__ void gx_partial(const double* __restrict__ G, const double* __restrict__ X, int n,
                                           uint64_t salt, int r0, int s, double (*red)[S32 + 1]) {
    const int lane = threadIdx.x & 63;
    const int kr = lane >> 4, cl = lane & 15;
    const int chunk = (int)ceil_div(ceil_div(n, GX_SPLIT), 4) * 4;
    const int k0 = min(n, s * chunk), k1 = min(n, k0 + chunk);
    const int ra = min(r0 + cl, n - 1);
    const double* grow = G + (int64_t)ra * n;
    f64x4 acc0 = f64x4{0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    for (int kb = k0; kb < k1; kb += 32) {
        double av[8], b0[8], b1[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int k = kb + 4 * t + kr;
            const bool in = k < k1;
            const int kk = in ? k : k0;
            const double m = in ? 1.0 : 0.0;
            av[t] = m * grow[kk];
            if (X) {
                b0[t] = X[(int64_t)kk * S32 + cl];
                b1[t] = X[(int64_t)kk * S32 + 16 + cl];
            } else {
                const uint64_t key = (uint64_t)kk * S32 + cl;
                b0[t] = hash_unit(key * 0x2545F4914F6CDD1Dull + salt);
                b1[t] = hash_unit((key + 16) * 0x2545F4914F6CDD1Dull + salt);
            }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], b0[t], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], b1[t], acc1, 0, 0, 0);
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = mfma16_row<PREC_F64>(lane, e);
        red[r][cl] = acc0[e];
        red[r][16 + cl] = acc1[e];
    }
}

// Y (n x 32) = G X (gx_partial).  One workgroup of GX_SPLIT wavefronts per
// 16-row tile; wavefront w takes the w-th K chunk and the partial tiles are
// added in LDS in wavefront order.
__global__ __launch_bounds__(64 * GX_SPLIT) void k_gemm_gx(const double* __restrict__ G, const double* __restrict__ X,
                                                           double* __restrict__ Y, int n, uint64_t salt) {
    __shared__ double red[GX_SPLIT][GX_ROWS][S32 + 1];
    const int s = threadIdx.x >> 6;
    const int r0 = blockIdx.x * GX_ROWS;
    gx_partial(G, X, n, salt, r0, s, red[s]);
    __syncthreads();
    for (int e = threadIdx.x; e < GX_ROWS * S32; e += 64 * GX_SPLIT) {
        const int r = e / S32, c = e % S32;
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < GX_SPLIT; ++w) t += red[w][r][c];
        if (r0 + r < n) Y[(int64_t)(r0 + r) * S32 + c] = t;
    }
}

// Orders LDS accesses between the lanes of one wavefront (a wavefront's LDS
// operations complete in issue order; this keeps the compiler from moving them).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The value of v held by lane `src` (uniform), for every lane.
__device__ inline double lane_bcast(double v, int src) {
    const uint64_t u = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, src);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), src);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}


// Row r of an n x 32 matrix held as NP partial arrays spaced n x 32 apart
// (their sum), element c.
template <int NP>
__device__ __forceinline__ double parts_at(const double* __restrict__ X, int64_t ps, int64_t off) {
    double v = X[off];
#pragma unroll
    for (int s = 1; s < NP; ++s) v += X[s * ps + off];
    return v;
}

// C[32][33] (LDS) = P^T Y for n x 32 row-major P and Y (global; P the sum of
// NPP partial arrays, Y of NPY, spaced n x 32 apart), FP64, fixed summation
// order; P == Y with NPP == NPY gives a Gram matrix from one set of loads.
// Each wavefront accumulates the four 16 x 16 blocks of C with
// v_mfma_f64_16x16x4f64 over groups of four rows (rows 4w, 4w + 4 NW, ...; four
// groups' loads in flight), every element loaded once per wavefront; the NW
// partial products pass through part_lds and are added in wavefront order.
template <int NW, int NPP, int NPY, int UNR_ = 0>
__device__ __forceinline__ void cross32(const double* __restrict__ P, const double* __restrict__ Y, int n,
                                        double* part_lds, double (*C)[S32 + 1]) {
    // row groups whose loads go out together (1 for a 32-row slab)
    constexpr int UNR = UNR_ ? UNR_ : ((NW >= 8) ? 16 : 8);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kr = lane >> 4, cl = lane & 15;
    const int64_t ps = (int64_t)n * S32;
    const bool gram = (P == Y) && NPP == NPY;
    f64x4 acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int g0 = 4 * wave; g0 < n; g0 += 4 * NW * UNR) {
        double pa[UNR][2], yb[UNR][2];
#pragma unroll
        for (int t = 0; t < UNR; ++t) {
            const int r = g0 + 4 * NW * t + kr;
            const double m = r < n ? 1.0 : 0.0;
            const int64_t off = (int64_t)(r < n ? r : n - 1) * S32 + cl;
            pa[t][0] = m * parts_at<NPP>(P, ps, off);
            pa[t][1] = m * parts_at<NPP>(P, ps, off + 16);
            if (gram) {
                yb[t][0] = pa[t][0];
                yb[t][1] = pa[t][1];
            } else {
                yb[t][0] = m * parts_at<NPY>(Y, ps, off);
                yb[t][1] = m * parts_at<NPY>(Y, ps, off + 16);
            }
        }
#pragma unroll
        for (int t = 0; t < UNR; ++t)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v)
                    acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[t][u], yb[t][v], acc[u][v], 0, 0, 0);
    }
    double* mine = part_lds + wave * (S32 * S32);
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                mine[(16 * u + mfma16_row<PREC_F64>(lane, e)) * S32 + 16 * v + cl] = acc[u][v][e];
    __syncthreads();
    for (int e = tid; e < S32 * S32; e += NW * 64) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += part_lds[w * (S32 * S32) + e];
        C[e >> 5][e & 31] = t;
    }
    __syncthreads();
}

// R^{-1} for the upper Cholesky factor R of C (32 x 32, LDS, symmetric), by one
// wavefront, without forming R: the row operations that reduce C to the
// identity (right-looking Cholesky, R^T R = C) are applied to the identity as
// well, which leaves R^{-T} = L^{-1} (column-oriented forward substitution).
// Lanes 0-31 keep column b = lane of the trailing matrix in registers, lanes
// 32-63 column b = lane - 32 of the identity being transformed.  Every lane
// publishes its v[J] in rowbuf (64 doubles, LDS; the upper half is never read)
// and all lanes read row J of the trailing matrix back as uniform loads; at
// step J, d = C'[J][J] gives r = d^{-1/2} and each lane subtracts
// rowbuf[a] v[J] / d from v[a], a > J, v[J + 1] first so that row J + 1 is
// published while the rest are updated.  v[J] r of an identity lane is final
// (entry J of row b of R^{-1}, exact zero below the diagonal) and goes to
// Rinv at once; the other lanes store into the padding column of Rinv.  No
// branches: the steps are unrolled through templates so every register index
// is static.  Returns false (on every lane) when a pivot is not positive and
// finite.
template <int J>
__device__ __forceinline__ void cinv_step(double (&v)[S32], const double (&rb)[S32 - J], double* rowbuf,
                                          double (*Rinv)[S32 + 1], bool idl, int b, bool& ok) {
    const int lane = threadIdx.x & 63;
    const double d = rb[0];
    ok = ok && (d >= 0x1p-1022) && (d < INFINITY);  // a positive normal pivot
    double r = rsqrt_pos(d);
    r = ok ? r : 0.0;
    const double s = v[J] * (r * r);
    *(idl ? &Rinv[b][J] : &Rinv[b][S32]) = v[J] * r;
    if constexpr (J + 1 < S32) {
        // v[J + 1] first: the next row goes out through LDS while the other
        // entries of this step are updated
        v[J + 1] -= rb[1] * s;
        rowbuf[lane] = v[J + 1];  // read back below in issue order (one wavefront)
        double nb[S32 - J - 1];
#pragma unroll
        for (int a = J + 1; a < S32; ++a) nb[a - J - 1] = rowbuf[a];
#pragma unroll
        for (int a = J + 2; a < S32; ++a) v[a] -= rb[a - J] * s;
        cinv_step<J + 1>(v, nb, rowbuf, Rinv, idl, b, ok);
    }
}

// Not inlined: a call site of its own keeps its unrolled steps from raising the
// register pressure of the caller.
__device__ __attribute__((noinline)) bool chol_inv32_wave(const double (*C)[S32 + 1], double (*Rinv)[S32 + 1],
                                                double* rowbuf) {
    const int lane = threadIdx.x & 63, b = lane & 31;
    const bool idl = lane >= S32;
    double v[S32];
#pragma unroll
    for (int a = 0; a < S32; ++a) {
        const double c = C[a][b];
        v[a] = idl ? (a == b ? 1.0 : 0.0) : c;
    }
    bool ok = true;
    rowbuf[lane] = v[0];
    wave_sync();
    double rb[S32];
#pragma unroll
    for (int a = 0; a < S32; ++a) rb[a] = rowbuf[a];
    cinv_step<0>(v, rb, rowbuf, Rinv, idl, b, ok);
    return ok;
}

// Out[r][j] = sum_k X[r][k] B[k][col(j)] for an n x 32 X (the sum of NP partial
// arrays spaced n x 32 apart) and B 32 x 32 in LDS; col(j) = colmap[j] or j.
// v_mfma_f64_16x16x4f64 on 16-row tiles, wavefront w of NW taking tiles w,
// w + NW, ...; B in registers.  Out may be the first array of X: a tile's
// rows are all loaded before any of them is stored.  With Sub (n x 32,
// global; may be Out) Out receives Sub - X B instead.
template <int NP, int NW, int TPW = 4>  // TPW: tiles per wavefront whose loads go out together
__device__ __forceinline__ void apply32(const double* X, double* Out, int n, const double (*B)[S32 + 1],
                                        const int* colmap, const double* Sub = nullptr) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kr = lane >> 4, cl = lane & 15;
    const int64_t ps = (int64_t)n * S32;
    const int c0 = colmap ? colmap[cl] : cl, c1 = colmap ? colmap[16 + cl] : 16 + cl;
    double bop[8][2];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
        bop[ks][0] = B[4 * ks + kr][c0];
        bop[ks][1] = B[4 * ks + kr][c1];
    }
    for (int rb = 16 * wave; rb < n; rb += 16 * NW * TPW) {
        double aop[TPW][8];
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int ra = rb + 16 * NW * t + cl;
            const int64_t rowoff = (int64_t)(ra < n ? ra : n - 1) * S32;
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) aop[t][ks] = parts_at<NP>(X, ps, rowoff + 4 * ks + kr);
        }
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int r0 = rb + 16 * NW * t;
            f64x4 acc0 = f64x4{0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[t][ks], bop[ks][0], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[t][ks], bop[ks][1], acc1, 0, 0, 0);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = r0 + mfma16_row<PREC_F64>(lane, e);
                if (r < n) {
                    const int64_t o = (int64_t)r * S32 + cl;
                    Out[o] = Sub ? Sub[o] - acc0[e] : acc0[e];
                    Out[o + 16] = Sub ? Sub[o + 16] - acc1[e] : acc1[e];
                }
            }
        }
    }
}

// One Cholesky QR pass: Y <- X R^{-1}, R^T R = X^T X (+ shift I), X the sum of
// NP partial arrays of which Y is the first (in place).  Returns false,
// uniformly, on a failed pivot.  The product X R^{-1} runs on
// v_mfma_f64_16x16x4f64, 16-row tiles per wavefront, R^{-1} held in registers.
template <int NP>
__device__ __forceinline__ bool cholqr_pass(double* __restrict__ Y, int n, bool shifted, double* part_lds,
                                            double (*C)[S32 + 1], double (*Rinv)[S32 + 1], double* rowbuf,
                                            int* ok_s) {
    const int tid = threadIdx.x;
    cross32<OW, NP, NP>(Y, Y, n, part_lds, C);
    if (tid < 64) {
        if (shifted) {
            // shift 11 (n m + m (m + 1)) u |Y|_F^2, an upper bound of the
            // shifted Cholesky QR choice (it takes |Y|_2^2)
            double fro = 0.0;
            for (int j = 0; j < S32; ++j) fro += C[j][j];
            const double sh = 11.0 * ((double)n * S32 + (double)S32 * (S32 + 1)) * 0x1p-53 * fro;
            wave_sync();
            if (tid < S32) C[tid][tid] += sh;
            wave_sync();
        }
        const bool ok = chol_inv32_wave(C, Rinv, rowbuf);
        if (tid == 0) *ok_s = ok ? 1 : 0;
    }
    __syncthreads();
    if (!*ok_s) return false;
    apply32<NP, OW>(Y, Y, n, Rinv, nullptr);
    __syncthreads();
    return true;
}

// Final orthonormalisation of an almost orthonormal Y (n x 32, global, in
// place): C = Y^T Y = I + E, Y <- Y (I - E/2 + 3 E^2 / 8), the series of
// C^{-1/2} to second order (error about |E|^3).  Returns false, uniformly,
// without touching Y, when max |E_ij| > 1e-4 (the caller then runs a
// Cholesky QR pass instead).
__device__ __forceinline__ bool series_pass(double* __restrict__ Y, int n, double* part_lds, double (*C)[S32 + 1],
                                            double (*X)[S32 + 1], int* ok_s) {
    const int tid = threadIdx.x;
    cross32<OW, 1, 1>(Y, Y, n, part_lds, C);
    // E = C - I in place; max |E| by wavefront 0
    for (int e = tid; e < S32 * S32; e += OT) {
        const int i = e >> 5, j = e & 31;
        if (i == j) C[i][j] -= 1.0;
    }
    __syncthreads();
    if (tid < 64) {
        double m = 0.0;
        for (int e = tid; e < S32 * S32; e += 64) m = fmax(m, fabs(C[e >> 5][e & 31]));
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
        if (tid == 0) *ok_s = (m <= 1e-4) ? 1 : 0;
    }
    __syncthreads();
    if (!*ok_s) return false;
    // X = I - E/2 + 3/8 E^2 (E symmetric)
    for (int e = tid; e < S32 * S32; e += OT) {
        const int i = e >> 5, j = e & 31;
        double t = 0.0;
#pragma unroll 8
        for (int k = 0; k < S32; ++k) t += C[i][k] * C[k][j];
        X[i][j] = (i == j ? 1.0 : 0.0) - 0.5 * C[i][j] + 0.375 * t;
    }
    __syncthreads();
    apply32<1, OW>(Y, Y, n, X, nullptr);
    __syncthreads();
    return true;
}

// Orthonormal basis of the columns of Y (n x 32, global), in place: a shifted
// Cholesky QR pass and a plain one; with full != 0 (the Rayleigh-Ritz basis) also the
// verified series correction.  *ok = 1 on success (first != 0) or *ok &=
// success (first == 0).
__global__ __launch_bounds__(OT) void k_orth32(double* __restrict__ Y, int n, int full, int first,
                                               int32_t* __restrict__ ok) {
    extern __shared__ double lds[];
    double* part_lds = lds;
    double(*C)[S32 + 1] = reinterpret_cast<double(*)[S32 + 1]>(lds + OW * S32 * S32);
    double(*Rinv)[S32 + 1] = reinterpret_cast<double(*)[S32 + 1]>(lds + OW * S32 * S32 + S32 * (S32 + 1));
    __shared__ double rowbuf[64];
    __shared__ int ok_s;
    const int tid = threadIdx.x;
    // pass 0 shifted (condition number down to about 5e-6 of the input's), pass
    // 1 plain (orthonormal to about u cond^2); for the final basis the series
    // correction, which also verifies |Y^T Y - I|, and if that is not yet small
    // a pass 2 and the series again.  One call site each keeps one inlined copy.
    bool good = true, done = false;
    for (int pass = 0; pass < 3 && good && !done; ++pass) {
        good = cholqr_pass<1>(Y, n, pass == 0, part_lds, C, Rinv, rowbuf, &ok_s);
        if (!good || pass == 0) continue;
        if (!full) done = true;
        else if (series_pass(Y, n, part_lds, C, Rinv, &ok_s)) done = true;
        else if (pass == 2) good = false;
    }
    good = good && done;
    if (tid == 0) *ok = first ? (good ? 1 : 0) : ((*ok && good) ? 1 : 0);
}

// Cyclic Jacobi on the symmetric A (32 x 32, LDS; only the upper triangle is
// read or written), rotations accumulated in W (32 x 32, LDS).  Called by
// every thread of a workgroup of at least 6 wavefronts.  Wavefront 0 runs the
// sweeps over the round-robin ordering.  A sweep starts with a test of all 496
// pairs (rot2_needed); when none needs a rotation the matrix has converged and
// the sweep is not run.  Otherwise in each round lanes 0-15 compute the
// rotation of pair `lane` into the rotation log and write that pair's 2 x 2
// diagonal block exactly (new diagonal, zero coupling), while every lane
// holds two of the 120 off-diagonal blocks (pair k, pair l), k < l, whose
// LDS offsets come from a per-round table, so their loads go out before the
// rotations are computed; after one wavefront sync the lanes read the two
// rotations each block needs and store it.  A round with no rotation is
// skipped.  Wavefronts 1, 2, 3 and 5 (off wavefront 0's SIMD) meanwhile
// apply the previous sweep's log to 8 rows of W each; one workgroup barrier
// per sweep.  Besides the relative test, an off-diagonal entry at or below
// JACOBI_FLOOR_F32 trace(A) is left alone: it is under what the float32 data
// behind A = Q^T G Q resolves, and rotating it away costs sweeps without
// changing the result at that accuracy.  log: 2 x 31 x 16 double2
// (c, s); ptab: 31 x 16 ints; btab:
// 31 x 128 uint4 (62 KB); flag: 1 int; all LDS.  Unused block slots point at
// the padding column of A, which nothing reads.
__device__ __forceinline__ void jacobi32(double (*A)[S32 + 1], double (*W)[S32 + 1], int max_sweeps, double2* log,
                                         int* ptab, uint4* btab, int* flag, int& sweeps_out, bool& conv_out) {
    constexpr int H = S32 / 2;             // pairs per round
    constexpr int NR = S32 - 1;            // rounds per sweep
    constexpr int NOFF = H * (H - 1) / 2;  // off-diagonal blocks per round
    constexpr int SL = 128;                // block slots per round, two per lane
    constexpr int LOGR = NR * H;           // rotation records per sweep
    static_assert(NOFF <= SL && SL - NOFF <= S32, "block slots");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double tol = (double)S32 * 0x1p-53;
    const double tol2 = tol * tol;
    double trace = 0.0;
    for (int i = 0; i < S32; ++i) trace += A[i][i];
    const double floor = JACOBI_FLOOR_F32 * fabs(trace);
    const double floor2 = floor * floor;
    char* const abase = reinterpret_cast<char*>(&A[0][0]);
    for (int e = tid; e < LOGR; e += blockDim.x) {
        int p, q;
        round_robin_pair(e / H, e % H, S32, p, q);
        ptab[e] = p | (q << 8);
    }
    // block slot b < NOFF -> (k, l), k < l, in row-major order of the strict upper triangle
    auto block_kl = [](int b, int& k, int& l) {
        k = 0;
        while (b >= H - 1 - k) {
            b -= H - 1 - k;
            ++k;
        }
        l = k + 1 + b;
    };
    __syncthreads();
    for (int e = tid; e < NR * SL; e += blockDim.x) {
        const int r = e / SL, b = e % SL;
        uint4 o;
        if (b < NOFF) {
            int k, l;
            block_kl(b, k, l);
            const int c1 = ptab[r * H + k], c2 = ptab[r * H + l];
            const int p = c1 & 255, q = c1 >> 8, p2 = c2 & 255, q2 = c2 >> 8;
            auto off = [](int x, int y) -> unsigned {
                return (unsigned)((x < y ? x * (S32 + 1) + y : y * (S32 + 1) + x) * (int)sizeof(double));
            };
            o = make_uint4(off(p, p2), off(p, q2), off(q, p2), off(q, q2));
        } else {
            const unsigned pad = (unsigned)(((b - NOFF) * (S32 + 1) + S32) * (int)sizeof(double));
            o = make_uint4(pad, pad, pad, pad);
        }
        btab[e] = o;
    }
    int kt[2], lt[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int b = lane + 64 * t;
        if (b < NOFF) {
            block_kl(b, kt[t], lt[t]);
        } else {
            kt[t] = 0;
            lt[t] = 0;
        }
    }
    __syncthreads();
    auto at = [&](unsigned off) -> double& { return *reinterpret_cast<double*>(abase + off); };
    // wavefronts 1, 2, 3, 5: rows 8 j + lane / 8 (j = 0..3), pairs lane % 8 and lane % 8 + 8
    const bool w_apply = wave == 1 || wave == 2 || wave == 3 || wave == 5;
    auto apply_log = [&](const double2* lg) {
        const int j = wave == 5 ? 3 : wave - 1;
        const int i = 8 * j + (lane >> 3);
        const int k0 = lane & 7;
        for (int round = 0; round < NR; ++round) {
            const int c0 = ptab[round * H + k0], c1 = ptab[round * H + k0 + 8];
            const int p0 = c0 & 255, q0 = c0 >> 8, p1 = c1 & 255, q1 = c1 >> 8;
            const double2 r0 = lg[round * H + k0], r1 = lg[round * H + k0 + 8];
            const double x0 = W[i][p0], y0 = W[i][q0], x1 = W[i][p1], y1 = W[i][q1];
            // (c, s) = (1, 0) for a pair that did not rotate: the same values back
            W[i][p0] = r0.x * x0 - r0.y * y0;
            W[i][q0] = r0.y * x0 + r0.x * y0;
            W[i][p1] = r1.x * x1 - r1.y * y1;
            W[i][q1] = r1.y * x1 + r1.x * y1;
        }
    };
    int sweeps = 0;
    bool conv = false;
    while (!conv && sweeps < max_sweeps) {
        double2* lg = log + (sweeps & 1) * LOGR;
        if (wave == 0) {
            bool need = false;
            for (int e = lane; e < LOGR; e += 64) {
                const int c = ptab[e], p = c & 255, q = c >> 8;
                need = need || rot2_needed(A[p][p], A[q][q], A[p][q], tol2, floor2);
            }
            bool any = false;
            uint4 ad[2] = {btab[lane], btab[64 + lane]};
            int me = ptab[lane & (H - 1)];
            for (int round = 0; round < NR && __ballot(need) != 0; ++round) {
                // the rotation's inputs go out first (LDS serves a wavefront's
                // accesses in issue order), then the block loads and next-round
                // tables, whose latency the rotation hides.  Every lane computes
                // the rotation of pair lane % 16 (no branch to sink the loads
                // into); lanes 0-15 store it.
                const int mp = me & 255, mq = me >> 8;
                const double app = A[mp][mp], aqq = A[mq][mq], apq = A[mp][mq];
                double x[2][4];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    x[t][0] = at(ad[t].x);
                    x[t][1] = at(ad[t].y);
                    x[t][2] = at(ad[t].z);
                    x[t][3] = at(ad[t].w);
                }
                const int rn = round + 1 < NR ? round + 1 : 0;
                const uint4 nad0 = btab[rn * SL + lane], nad1 = btab[rn * SL + 64 + lane];
                const int nme = ptab[rn * H + (lane & (H - 1))];
                double c, s, dp, dq;
                const bool rr = rot2(app, aqq, apq, tol2, floor2, c, s, dp, dq);
                const bool r = rr && lane < H;
                if (lane < H) {
                    lg[round * H + lane] = double2{c, s};
                    A[mp][mp] = dp;
                    A[mq][mq] = dq;
                    A[mp][mq] = rr ? 0.0 : apq;
                }
                if (__ballot(r) != 0) {
                    any = true;
                    // no wait: a wavefront's LDS accesses complete in issue order,
                    // so these loads see the log and blocks stored above
                    double2 ck[2], cl[2];
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        ck[t] = lg[round * H + kt[t]];
                        cl[t] = lg[round * H + lt[t]];
                    }
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const double c1 = ck[t].x, s1 = ck[t].y, c2 = cl[t].x, s2 = cl[t].y;
                        const double ra = c1 * x[t][0] - s1 * x[t][2], rb = c1 * x[t][1] - s1 * x[t][3];
                        const double rc = s1 * x[t][0] + c1 * x[t][2], rd = s1 * x[t][1] + c1 * x[t][3];
                        at(ad[t].x) = c2 * ra - s2 * rb;
                        at(ad[t].y) = s2 * ra + c2 * rb;
                        at(ad[t].z) = c2 * rc - s2 * rd;
                        at(ad[t].w) = s2 * rc + c2 * rd;
                    }
                }
                ad[0] = nad0;
                ad[1] = nad1;
                me = nme;
            }
            if (lane == 0) *flag = any ? 1 : 0;
        } else if (w_apply && sweeps > 0) {
            apply_log(log + ((sweeps - 1) & 1) * LOGR);
        }
        __syncthreads();
        conv = (*flag == 0);
        ++sweeps;
        __syncthreads();
    }
    // the last sweep's log: applied already when that sweep was followed by
    // the converged one (whose log is unused: not written, or all (1, 0))
    if (!conv && w_apply && sweeps > 0) apply_log(log + ((sweeps - 1) & 1) * LOGR);
    __syncthreads();
    sweeps_out = sweeps;
    conv_out = conv;
}

// Best-|v| candidate of one column for the sign rule.
struct SignCand {
    double best, val;
    int row, pad;
};

// Merges candidate (ob, oi, ov) into (best, bi, val): larger |v| wins, the
// smaller row on ties (the first row, whatever the order of the merges).
__device__ __forceinline__ void sign_merge(double& best, int& bi, double& val, double ob, int oi, double ov) {
    if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
        val = ov;
    }
}

// V = Q W[:, colmap] for n <= 16 RW TPW rows, on v_mfma_f64_16x16x4f64 as in
// apply32, kept in the accumulators: the sign rule over the leading r columns
// (per-wavefront candidates in LDS, merged in wavefront order) and the factor
// output come straight from registers, so V never goes to memory.  cand: RW x
// 32 records, sign_s: 32 ints, both LDS.
__device__ __forceinline__ void rr_factor_out(const SelectArgs& a, const double* __restrict__ Q, int n,
                                              const double (*B)[S32 + 1], const int* colmap, int r, SignCand* cand,
                                              int* sign_s) {
    constexpr int TPW = 4;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kr = lane >> 4, cl = lane & 15;
    const int c0 = colmap[cl], c1 = colmap[16 + cl];
    double bop[8][2];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
        bop[ks][0] = B[4 * ks + kr][c0];
        bop[ks][1] = B[4 * ks + kr][c1];
    }
    double aop[TPW][8];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int ra = 16 * wave + 16 * RW * t + cl;
        const int64_t rowoff = (int64_t)(ra < n ? ra : n - 1) * S32;
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) aop[t][ks] = Q[rowoff + 4 * ks + kr];
    }
    f64x4 acc[TPW][2];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        acc[t][0] = f64x4{0.0, 0.0, 0.0, 0.0};
        acc[t][1] = acc[t][0];
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            acc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[t][ks], bop[ks][0], acc[t][0], 0, 0, 0);
            acc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[t][ks], bop[ks][1], acc[t][1], 0, 0, 0);
        }
    }
    // sign candidates of columns cl (h = 0) and 16 + cl (h = 1)
    double best[2] = {-1.0, -1.0}, val[2] = {0.0, 0.0};
    int bi[2] = {0x7fffffff, 0x7fffffff};
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = 16 * wave + 16 * RW * t + mfma16_row<PREC_F64>(lane, e);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const double v = acc[t][h][e];
                if (row < n) sign_merge(best[h], bi[h], val[h], fabs(v), row, v);
            }
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        for (int o = 16; o < 64; o <<= 1) {
            const double ob = __shfl_xor(best[h], o);
            const int oi = __shfl_xor(bi[h], o);
            const double ov = __shfl_xor(val[h], o);
            sign_merge(best[h], bi[h], val[h], ob, oi, ov);
        }
        if (lane < 16) cand[wave * S32 + 16 * h + cl] = SignCand{best[h], val[h], bi[h], 0};
    }
    __syncthreads();
    if (tid < S32) {
        SignCand c = cand[tid];
        for (int w = 1; w < RW; ++w) {
            const SignCand o = cand[w * S32 + tid];
            sign_merge(c.best, c.row, c.val, o.best, o.row, o.val);
        }
        sign_s[tid] = c.val < 0.0 ? -1 : 1;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = 16 * wave + 16 * RW * t + mfma16_row<PREC_F64>(lane, e);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int j = 16 * h + cl;
                if (row < n && j < r) store_factor(a, row, j, r, sign_s[j] * acc[t][h][e]);
            }
        }
    }
}

// Rayleigh-Ritz on span(Q) (Q n x 32 orthonormal, Z = G Q), then rank choice
// and factor output: B = Q^T Z = W diag(theta) W^T, the rank from theta and
// trace(G), and V = Q W straight into the factor (rr_factor_out).  When either
// orthonormalisation failed the mode is handed to the next eigensolver.
__global__ __launch_bounds__(RT) void k_rr32_select(const double* __restrict__ Q, const double* __restrict__ Z,
                                                    int n, int max_sweeps,
                                                    const int32_t* __restrict__ orth_ok, int quiet,
                                                    const double* __restrict__ bsym, SelectArgs a) {
    extern __shared__ double lds[];
    double* part_lds = lds;
    double(*Bm)[S32 + 1] = reinterpret_cast<double(*)[S32 + 1]>(lds + RW * S32 * S32);
    double(*Wm)[S32 + 1] = reinterpret_cast<double(*)[S32 + 1]>(lds + RW * S32 * S32 + S32 * (S32 + 1));
    __shared__ double2 jlog[2 * (S32 - 1) * (S32 / 2)];
    __shared__ int jptab[(S32 - 1) * (S32 / 2)];
    __shared__ int jflag;
    __shared__ int col_of[S32];
    __shared__ double lam_s[S32];
    __shared__ double red[17];
    __shared__ int sign_s[S32];
    __shared__ int r_s, dense_s;
    __shared__ int sweeps_s, conv_s;
    const int tid = threadIdx.x;
    DevBook* bk = a.book;
    if (!*orth_ok) {
        // quiet: the basis launch has reported the hand-over already
        if (tid == 0 && !quiet) {
            bk->need_dense = 1;
            publish_selection(a, 0);
        }
        return;
    }
    double tr;
    if (bsym) {
        // B (symmetrised) and trace(G) from the basis launch
        for (int e = tid; e < S32 * S32; e += RT) {
            const int i = e >> 5, j = e & 31;
            Bm[i][j] = bsym[e];
            Wm[i][j] = (i == j) ? 1.0 : 0.0;
        }
        tr = bsym[S32 * S32];
        __syncthreads();
    } else {
        tr = gram_trace(a, red);
        cross32<RW, 1, 1>(Q, Z, n, part_lds, Bm);
        for (int e = tid; e < S32 * S32; e += RT) {
            const int i = e >> 5, j = e & 31;
            Wm[i][j] = 0.5 * (Bm[i][j] + Bm[j][i]);
        }
        __syncthreads();
        for (int e = tid; e < S32 * S32; e += RT) {
            const int i = e >> 5, j = e & 31;
            Bm[i][j] = Wm[i][j];
            Wm[i][j] = (i == j) ? 1.0 : 0.0;
        }
        __syncthreads();
    }
    {
        int sw;
        bool cv;
        // the cross-product partials are dead here: their space holds the block table
        static_assert(RW * S32 * S32 * sizeof(double) >= (S32 - 1) * 128 * sizeof(uint4), "block table");
        jacobi32(Bm, Wm, max_sweeps, jlog, jptab, reinterpret_cast<uint4*>(part_lds), &jflag, sw, cv);
        if (tid == 0) {
            sweeps_s = sw;
            conv_s = cv ? 1 : 0;
        }
    }
    __syncthreads();
    double* lam = const_cast<double*>(a.lam);
    // every slot of col_of a valid column even when NaN Ritz values tie
    if (tid < S32) col_of[tid] = tid;
    __syncthreads();
    if (tid < S32) {
        const double li = Bm[tid][tid];
        int r = 0;
        for (int j = 0; j < S32; ++j) {
            const double lj = Bm[j][j];
            r += (lj > li) || (lj == li && j < tid);
        }
        col_of[r] = tid;
        lam[r] = li;
        lam_s[r] = li;
    }
    if (tid == 0) {
        bk->sweeps[a.k] = sweeps_s;
        bk->eig_ok = conv_s;
    }
    __syncthreads();
    SelectArgs al = a;
    al.lam = lam_s;  // the Ritz values from LDS
    if (tid == 0) choose_rank(al, tr, r_s, dense_s);
    __syncthreads();
    if (dense_s) {
        // split form: the mode product by the basis, running beside this
        // launch, is of no use now; its workgroups that start from here on
        // read 0 rows and return
        if (tid == 0 && quiet)
            __hip_atomic_store(const_cast<int32_t*>(orth_ok) + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    // V = Q W[:, col_of], sign rule and factor output (the partials' space is free again)
    static_assert(RW * S32 * S32 * sizeof(double) >= RW * S32 * sizeof(SignCand), "sign candidates");
    rr_factor_out(al, Q, n, Wm, col_of, r_s, reinterpret_cast<SignCand*>(part_lds), sign_s);
    // the rotation operand (W_r diag(signs))^T, r x 32 (sign_s is final after
    // the barriers inside rr_factor_out)
    if (a.Wt64 || a.Wt32) {
        const int r = r_s;
        for (int e = tid; e < r * S32; e += RT) {
            const int j = e >> 5, c = e & 31;
            const double u = sign_s[j] * Wm[c][col_of[j]];
            if (a.Wt64) a.Wt64[e] = u;
            if (a.Wt32) {
                const float f = (float)u;
                a.Wt32[e] = f;
                if (a.Wth) {
                    const __bf16 hh = (__bf16)f;
                    a.Wth[e] = hh;
                    a.Wtl[e] = (__bf16)(f - (float)hh);
                }
            }
        }
    }
}

// ------------------------------- subspace path, m = 32, one cooperative launch
// The orthogonal iteration and Rayleigh-Ritz step of k_gemm_gx / k_orth32 /
// k_rr32_select in one launch of ceil(n / 32) workgroups, workgroup b owning
// rows 32 b .. 32 b + 31 of the n x 32 blocks.  The 32 x 32 products Y^T Y and
// Q^T Z are formed per slab and summed over the workgroups through global
// partial arrays in workgroup order, so every workgroup holds the same matrix
// bit for bit and computes the same Cholesky factor, series correction and
// Jacobi eigenvectors by itself (no broadcast step).  Only the products G X
// read every row of X and wait for all workgroups.  The launch is cooperative
// (all workgroups resident), which the grid barrier relies on.

constexpr int GRID_ROWS = 32;                 // rows per workgroup
constexpr int GRID_MAXB = 512 / GRID_ROWS;    // workgroups for n <= 512
constexpr unsigned GRID_SPIN_LIMIT = 1u << 20;  // polls before a wait gives up (default)

// Global scratch of the cooperative path (inside the subspace workspace).
struct Sub32Grid {
    double* P1;       // n x 32
    double* P2;       // n x 32
    double* part;     // 2 x GRID_MAXB x 1024: per-workgroup 32 x 32 products, two alternating sets
    double* cand;     // GRID_MAXB x 32 x 3: sign candidates (|v|, v, row)
    unsigned* sync;   // DevBook::grid: [0] arrivals, [1] rank, [2] need_dense, [3] a wait gave up, [4] exits
    unsigned spin_limit;  // polls before a wait gives up
    int32_t* basis_ok;    // basis-only launch: 1 when Q was formed (null otherwise)
    double* bsym;         // basis-only launch: B = Q^T G Q symmetrised (32 x 32), then trace(G)
};

// Grid barrier: every wavefront drains its stores, thread 0 makes the
// workgroup's stores visible at device scope (release), adds its arrival and
// polls until `target` arrivals, then makes the other workgroups' stores
// visible (acquire).  The wait is bounded: a workgroup that gives up records
// it and goes on, so every wavefront still reaches the end of the kernel.
// Returns true in every thread of a workgroup whose wait gave up.
__device__ __forceinline__ bool grid_sync(unsigned* sync, unsigned target, unsigned spin_limit) {
    __shared__ int gave;
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    if (threadIdx.x == 0) {
        gave = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(&sync[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        // a limit of 0 gives up without looking (forces the failure path)
        while (spin_limit == 0 || __hip_atomic_load(&sync[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > spin_limit) {
                __hip_atomic_store(&sync[3], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                gave = 1;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return gave != 0;
}

// End of a cooperative launch: the last workgroup to finish clears the
// barrier words for the next launch (every workgroup has passed its last wait).
__device__ __forceinline__ void grid_exit(unsigned* sync) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned done = __hip_atomic_fetch_add(&sync[4], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done + 1 == gridDim.x) {
            // the rank words too: a workgroup that reads them after a wait that
            // gave up then finds 0 (nothing to write), never a previous mode's
            for (int w = 0; w < 5; ++w) __hip_atomic_store(&sync[w], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Per-workgroup state of the cooperative path.
struct GridCtx {
    Sub32Grid g;
    int n, b, nb, row0, nr;
    unsigned arrivals;  // barriers passed so far times nb
    int parity;         // partial set of the next exchange
    bool gave_up;       // one of this workgroup's waits gave up
    __device__ void sync() {
        arrivals += (unsigned)nb;
        gave_up = grid_sync(g.sync, arrivals, g.spin_limit) || gave_up;
    }
};

// C (LDS) = sum over workgroups, in workgroup order, of P_b^T Z_b (each
// workgroup's nr rows of P and Z); the same value in every workgroup.
__device__ __forceinline__ void cross_grid(GridCtx& x, const double* P, const double* Z, double* part_lds,
                                           double (*C)[S32 + 1]) {
    const int tid = threadIdx.x;
    cross32<RW, 1, 1, 1>(P, Z, x.nr, part_lds, C);
    double* slot = x.g.part + (size_t)x.parity * GRID_MAXB * (S32 * S32);
    x.parity ^= 1;
    for (int e = tid; e < S32 * S32; e += RT) slot[(size_t)x.b * (S32 * S32) + e] = C[e >> 5][e & 31];
    x.sync();
    for (int e = tid; e < S32 * S32; e += RT) {
        double v[GRID_MAXB];
#pragma unroll
        for (int o = 0; o < GRID_MAXB; ++o) v[o] = slot[(size_t)(o < x.nb ? o : 0) * (S32 * S32) + e];
        double t = 0.0;
#pragma unroll
        for (int o = 0; o < GRID_MAXB; ++o)
            if (o < x.nb) t += v[o];
        C[e >> 5][e & 31] = t;
    }
    __syncthreads();
}

// Rows row0 .. row0 + 31 of G X into Y (X == nullptr: the hash matrix of
// salt, as in gx_partial, when HASH): wavefront w takes the w-th of RW K
// chunks for all 32 rows and columns, in batches of eight K steps whose loads
// go out together (two memory latencies per product for n = 512), then the
// chunks are added in order through LDS.  red_lds: RW x 32 x 32 doubles.
template <bool HASH>
__device__ __forceinline__ void gx_rows32(const GridCtx& x, const double* __restrict__ G, const double* X,
                                          uint64_t salt, double* Y, double* red_lds) {
    constexpr int KB = 16;  // K steps of four per batch
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kr = lane >> 4, cl = lane & 15;
    const int n = x.n;
    const int chunk = (int)ceil_div(ceil_div(n, RW), 4) * 4;
    const int k0 = min(n, wave * chunk), k1 = min(n, k0 + chunk);
    const double* g0 = G + (int64_t)min(x.row0 + cl, n - 1) * n;
    const double* g1 = G + (int64_t)min(x.row0 + 16 + cl, n - 1) * n;
    f64x4 acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int kb = k0; kb < k1; kb += 4 * KB) {
        double a0[KB], a1[KB], b0[KB], b1[KB];
#pragma unroll
        for (int t = 0; t < KB; ++t) {
            const int k = kb + 4 * t + kr;
            const bool in = k < k1;
            const int kk = in ? k : k0;
            const double m = in ? 1.0 : 0.0;
            a0[t] = m * g0[kk];
            a1[t] = m * g1[kk];
            if constexpr (HASH) {
                const uint64_t key = (uint64_t)kk * S32 + cl;
                b0[t] = hash_unit(key * 0x2545F4914F6CDD1Dull + salt);
                b1[t] = hash_unit((key + 16) * 0x2545F4914F6CDD1Dull + salt);
            } else {
                b0[t] = X[(int64_t)kk * S32 + cl];
                b1[t] = X[(int64_t)kk * S32 + 16 + cl];
            }
        }
#pragma unroll
        for (int t = 0; t < KB; ++t) {
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[t], b0[t], acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[t], b1[t], acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[t], b0[t], acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[t], b1[t], acc[1][1], 0, 0, 0);
        }
    }
    double* mine = red_lds + wave * (S32 * S32);
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                mine[(16 * u + mfma16_row<PREC_F64>(lane, e)) * S32 + 16 * v + cl] = acc[u][v][e];
    __syncthreads();
    for (int e = tid; e < S32 * S32; e += RT) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < RW; ++w) t += red_lds[w * (S32 * S32) + e];
        const int row = x.row0 + (e >> 5);
        if (row < n) Y[(int64_t)row * S32 + (e & 31)] = t;
    }
    __syncthreads();
}

// One Cholesky QR pass on the workgroup's rows Y (in place), as cholqr_pass.
__device__ __forceinline__ bool cholqr_grid(GridCtx& x, double* Y, bool shifted, double* part_lds,
                                            double (*C)[S32 + 1], double (*Rinv)[S32 + 1], double* rowbuf,
                                            int* ok_s) {
    const int tid = threadIdx.x;
    cross_grid(x, Y, Y, part_lds, C);
    if (tid < 64) {
        if (shifted) {
            double fro = 0.0;
            for (int j = 0; j < S32; ++j) fro += C[j][j];
            const double sh = 11.0 * ((double)x.n * S32 + (double)S32 * (S32 + 1)) * 0x1p-53 * fro;
            wave_sync();
            if (tid < S32) C[tid][tid] += sh;
            wave_sync();
        }
        const bool ok = chol_inv32_wave(C, Rinv, rowbuf);
        if (tid == 0) *ok_s = ok ? 1 : 0;
    }
    __syncthreads();
    if (!*ok_s) return false;
    apply32<1, RW, 1>(Y, Y, x.nr, Rinv, nullptr);
    __syncthreads();
    return true;
}

// The series correction of series_pass on the workgroup's rows.
__device__ __forceinline__ bool series_grid(GridCtx& x, double* Y, double* part_lds, double (*C)[S32 + 1],
                                            double (*X)[S32 + 1], int* ok_s) {
    const int tid = threadIdx.x;
    cross_grid(x, Y, Y, part_lds, C);
    for (int e = tid; e < S32 * S32; e += RT) {
        const int i = e >> 5, j = e & 31;
        if (i == j) C[i][j] -= 1.0;
    }
    __syncthreads();
    if (tid < 64) {
        double m = 0.0;
        for (int e = tid; e < S32 * S32; e += 64) m = fmax(m, fabs(C[e >> 5][e & 31]));
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
        if (tid == 0) *ok_s = (m <= 1e-4) ? 1 : 0;
    }
    __syncthreads();
    if (!*ok_s) return false;
    for (int e = tid; e < S32 * S32; e += RT) {
        const int i = e >> 5, j = e & 31;
        double t = 0.0;
#pragma unroll 8
        for (int k = 0; k < S32; ++k) t += C[i][k] * C[k][j];
        X[i][j] = (i == j ? 1.0 : 0.0) - 0.5 * C[i][j] + 0.375 * t;
    }
    __syncthreads();
    apply32<1, RW, 1>(Y, Y, x.nr, X, nullptr);
    __syncthreads();
    return true;
}

// The orthonormalisation of k_orth32 on the workgroup's rows of Y.
__device__ __forceinline__ bool orth_grid(GridCtx& x, double* Y, bool full, double* part_lds, double (*C)[S32 + 1],
                                          double (*R)[S32 + 1], double* rowbuf, int* ok_s) {
    bool good = true, done = false;
    for (int pass = 0; pass < 3 && good && !done; ++pass) {
        good = cholqr_grid(x, Y, pass == 0, part_lds, C, R, rowbuf, ok_s);
        if (!good || pass == 0) continue;
        if (!full) done = true;
        else if (series_grid(x, Y, part_lds, C, R, ok_s)) done = true;
        else if (pass == 2) good = false;
    }
    return good && done;
}

__device__ __forceinline__ void sub32_grid_body(const double* __restrict__ G, int n, int steps, int max_sweeps,
                                                const Sub32Grid& g, const SelectArgs& a, const QtOut& qt) {
    extern __shared__ double lds[];
    double* part_lds = lds;
    double(*Bm)[S32 + 1] = reinterpret_cast<double(*)[S32 + 1]>(lds + RW * S32 * S32);
    double(*Wm)[S32 + 1] = reinterpret_cast<double(*)[S32 + 1]>(lds + RW * S32 * S32 + S32 * (S32 + 1));
    __shared__ double2 jlog[2 * (S32 - 1) * (S32 / 2)];
    __shared__ int jptab[(S32 - 1) * (S32 / 2)];
    __shared__ int jflag;
    __shared__ double rowbuf[64];
    __shared__ int col_of[S32];
    __shared__ double lam_s[S32];
    __shared__ double red[17];
    __shared__ int sign_s[S32];
    __shared__ SignCand wcand[2][S32];
    __shared__ int ok_s, r_s, dense_s;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    GridCtx x;
    x.g = g;
    x.n = n;
    x.b = blockIdx.x;
    x.nb = gridDim.x;
    x.row0 = GRID_ROWS * x.b;
    x.nr = min(GRID_ROWS, n - x.row0);
    x.arrivals = 0;
    x.parity = 0;
    x.gave_up = false;
    DevBook* bk = a.book;
    double tr = 0.0;
    if (x.b == 0) tr = gram_trace(a, red);
    // power steps: P1 <- orth(P1), P2 <- G P1, swap
    double* P1 = g.P1;
    double* P2 = g.P2;
    gx_rows32<true>(x, G, nullptr, 0x5eed, P1, part_lds);
    bool good = true;
    for (int it = 0; it < steps && good; ++it) {
        double* Yb = P1 + (int64_t)x.row0 * S32;
        good = orth_grid(x, Yb, it + 1 == steps, part_lds, Bm, Wm, rowbuf, &ok_s);
        if (!good) break;
        x.sync();
        gx_rows32<false>(x, G, P1, 0, P2, part_lds);
        double* t = P1;
        P1 = P2;
        P2 = t;
    }
    if (!good) {
        // the same outcome in every workgroup: hand the mode to the next eigensolver
        if (x.b == 0 && tid == 0) {
            if (g.basis_ok) {
                g.basis_ok[0] = 0;
                g.basis_ok[1] = 0;
            }
            bk->need_dense = 1;
            if (__hip_atomic_load(&g.sync[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                bk->status = ATC_ERR_INTERNAL;  // not a failed basis: a wait gave up
            publish_selection(a, 0);
        }
        return;
    }
    if (qt.t64 || qt.t32) {
        // basis only: Q^T for the mode product by the basis; the Rayleigh-Ritz
        // step follows in its own launch
        for (int e = tid; e < x.nr * S32; e += RT) {
            const int i = e >> 5, j = e & 31;
            const int row = x.row0 + i;
            const double q = P2[(int64_t)row * S32 + j];
            const int64_t t = (int64_t)j * n + row;
            if (qt.t64) qt.t64[t] = q;
            if (qt.t32) {
                const float f = (float)q;
                qt.t32[t] = f;
                if (qt.th) {
                    const __bf16 hh = (__bf16)f;
                    qt.th[t] = hh;
                    qt.tl[t] = (__bf16)(f - (float)hh);
                }
            }
        }
        // B = Q^T Z from the slabs (every workgroup), stored symmetrised with
        // trace(G) by workgroup 0 for the Rayleigh-Ritz launch
        cross_grid(x, P2 + (int64_t)x.row0 * S32, P1 + (int64_t)x.row0 * S32, part_lds, Bm);
        if (x.b == 0) {
            for (int e = tid; e < S32 * S32; e += RT) {
                const int i = e >> 5, j = e & 31;
                g.bsym[e] = 0.5 * (Bm[i][j] + Bm[j][i]);
            }
            if (tid == 0) {
                g.bsym[S32 * S32] = tr;
                *g.basis_ok = 1;
                g.basis_ok[1] = S32;  // rows of the product by the basis (0 once handed on)
            }
        }
        return;
    }
    // P2: the basis Q, P1 = G Q.  B = Q^T Z, symmetrised; Jacobi in every workgroup
    const double* Qb = P2 + (int64_t)x.row0 * S32;
    cross_grid(x, Qb, P1 + (int64_t)x.row0 * S32, part_lds, Bm);
    for (int e = tid; e < S32 * S32; e += RT) {
        const int i = e >> 5, j = e & 31;
        Wm[i][j] = 0.5 * (Bm[i][j] + Bm[j][i]);
    }
    __syncthreads();
    for (int e = tid; e < S32 * S32; e += RT) {
        const int i = e >> 5, j = e & 31;
        Bm[i][j] = Wm[i][j];
        Wm[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    int sw;
    bool cv;
    static_assert(RW * S32 * S32 * sizeof(double) >= (S32 - 1) * 128 * sizeof(uint4), "block table");
    jacobi32(Bm, Wm, max_sweeps, jlog, jptab, reinterpret_cast<uint4*>(part_lds), &jflag, sw, cv);
    // every slot of col_of a valid column even when NaN Ritz values tie
    if (tid < S32) col_of[tid] = tid;
    __syncthreads();
    if (tid < S32) {
        const double li = Bm[tid][tid];
        int r = 0;
        for (int j = 0; j < S32; ++j) {
            const double lj = Bm[j][j];
            r += (lj > li) || (lj == li && j < tid);
        }
        col_of[r] = tid;
        lam_s[r] = li;
        if (x.b == 0) const_cast<double*>(a.lam)[r] = li;
    }
    __syncthreads();
    SelectArgs al = a;
    al.lam = lam_s;
    if (x.b == 0 && tid == RT - 64) {
        // the rank choice and host report by the last wavefront of workgroup 0,
        // while wavefronts 0 and 1 form V_b; the host can queue the mode
        // product while this kernel finishes
        bk->sweeps[a.k] = sw;
        bk->eig_ok = cv ? 1 : 0;
        if (__hip_atomic_load(&g.sync[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) bk->status = ATC_ERR_INTERNAL;
        choose_rank(al, tr, r_s, dense_s, !a.publish_late);
        __hip_atomic_store(&g.sync[1], (unsigned)r_s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&g.sync[2], (unsigned)dense_s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // V_b = Q_b W[:, col_of] in the accumulators of wavefronts 0 and 1 (16 rows each)
    const int kr = lane >> 4, cl = lane & 15;
    const bool vw = wave < 2;
    f64x4 acc0 = f64x4{0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    const int rbase = x.row0 + 16 * (wave & 1);
    if (vw) {
        const int c0 = col_of[cl], c1 = col_of[16 + cl];
        const int ra = min(rbase + cl, n - 1);
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const double av = P2[(int64_t)ra * S32 + 4 * ks + kr];
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Wm[4 * ks + kr][c0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Wm[4 * ks + kr][c1], acc1, 0, 0, 0);
        }
        double best[2] = {-1.0, -1.0}, val[2] = {0.0, 0.0};
        int bi[2] = {0x7fffffff, 0x7fffffff};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = rbase + mfma16_row<PREC_F64>(lane, e);
            if (row < n) {
                sign_merge(best[0], bi[0], val[0], fabs(acc0[e]), row, acc0[e]);
                sign_merge(best[1], bi[1], val[1], fabs(acc1[e]), row, acc1[e]);
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            for (int o = 16; o < 64; o <<= 1) {
                const double ob = __shfl_xor(best[h], o);
                const int oi = __shfl_xor(bi[h], o);
                const double ov = __shfl_xor(val[h], o);
                sign_merge(best[h], bi[h], val[h], ob, oi, ov);
            }
            if (lane < 16) wcand[wave][16 * h + cl] = SignCand{best[h], val[h], bi[h], 0};
        }
    }
    __syncthreads();
    if (tid < S32) {
        SignCand c = wcand[0][tid];
        const SignCand o = wcand[1][tid];
        sign_merge(c.best, c.row, c.val, o.best, o.row, o.val);
        double* gc = g.cand + ((size_t)x.b * S32 + tid) * 3;
        gc[0] = c.best;
        gc[1] = c.val;
        gc[2] = (double)c.row;
    }
    x.sync();
    if (x.gave_up) {
        // this workgroup may hold a stale rank and the other workgroups'
        // candidates may be missing: write nothing, record the failure (the
        // host reads it with the next report, or below for the last mode)
        if (tid == 0) bk->status = ATC_ERR_INTERNAL;
    }
    if (a.publish_late && x.b == 0 && tid == 0) {
        if (x.gave_up || __hip_atomic_load(&g.sync[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            bk->status = ATC_ERR_INTERNAL;
        publish_selection(al, r_s);
    }
    if (x.gave_up) return;
    const int r = (int)__hip_atomic_load(&g.sync[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int dense = (int)__hip_atomic_load(&g.sync[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (dense) return;
    if (tid < S32) {
        double cb[GRID_MAXB], cv_[GRID_MAXB], cr[GRID_MAXB];
#pragma unroll
        for (int o = 0; o < GRID_MAXB; ++o) {
            const double* gc = g.cand + ((size_t)(o < x.nb ? o : 0) * S32 + tid) * 3;
            cb[o] = gc[0];
            cv_[o] = gc[1];
            cr[o] = gc[2];
        }
        double best = -1.0, val = 0.0;
        int bi = 0x7fffffff;
#pragma unroll
        for (int o = 0; o < GRID_MAXB; ++o)
            if (o < x.nb) sign_merge(best, bi, val, cb[o], (int)cr[o], cv_[o]);
        sign_s[tid] = val < 0.0 ? -1 : 1;
    }
    __syncthreads();
    if (vw) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = rbase + mfma16_row<PREC_F64>(lane, e);
            if (row < n) {
                if (cl < r) store_factor(al, row, cl, r, sign_s[cl] * acc0[e]);
                if (16 + cl < r) store_factor(al, row, 16 + cl, r, sign_s[16 + cl] * acc1[e]);
            }
        }
    }
}

// The body above, then the last workgroup to finish clears the barrier words
// for the next launch (every workgroup has passed its last wait by then).
__global__ __launch_bounds__(RT) void k_sub32_grid(const double* __restrict__ G, int n, int steps, int max_sweeps,
                                                   Sub32Grid g, SelectArgs a, QtOut qt) {
    sub32_grid_body(G, n, steps, max_sweeps, g, a, qt);
    grid_exit(g.sync);
}

// The cooperative path needs cooperative launches and its LDS (checked once);
// ATC_SUB32_KERNELS=1 in the environment (read at every call) selects the
// kernel-per-step path.
bool sub32_grid_supported() {
    static int state = 0;
    if (state == 0) {
        int dev = 0, coop = 0;
        const bool a = hipGetDevice(&dev) == hipSuccess &&
                       hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess && coop;
        const bool b = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sub32_grid),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)RR_LDS) == hipSuccess;
        state = (a && b) ? 1 : -1;
    }
    return state == 1;
}

bool kernel_chain_forced() {
    const char* env = getenv("ATC_SUB32_KERNELS");
    return env && env[0] == '1';
}

bool sub32_grid_ready() { return sub32_grid_supported() && !kernel_chain_forced(); }

bool sub32_ready() {
    static int state = 0;
    if (state == 0) {
        const bool a = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_orth32),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)ORTH_LDS) == hipSuccess;
        const bool b = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rr32_select),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)RR_LDS) == hipSuccess;
        state = (a && b) ? 1 : -1;
    }
    return state == 1;
}

__global__ void k_prepare_matrix(const void* U, int src_f64, int rows, int cols, int transpose, double* M64,
                                 float* M32, __bf16* Mh, __bf16* Ml) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)rows * cols) return;
    const int i = (int)(idx / cols), j = (int)(idx % cols);
    const double u = src_f64 ? ((const double*)U)[idx] : (double)((const float*)U)[idx];
    const int64_t t = transpose ? (int64_t)j * rows + i : idx;
    if (M64) M64[t] = u;
    if (M32) {
        const float f = (float)u;
        M32[t] = f;
        if (Mh) {
            const __bf16 h = (__bf16)f;
            Mh[t] = h;
            Ml[t] = (__bf16)(f - (float)h);
        }
    }
}

__global__ void k_zero(uint32_t* p, size_t words) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < words) p[idx] = 0u;
}

}  // namespace

hipError_t launch_select_factor(const SelectArgs& a, hipStream_t st) {
    if (a.n > 4096) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_select_factor, dim3(1), dim3(512), 0, st, a);
    return hipGetLastError();
}

namespace {

// ------------------------------------------- subspace path, m = 64, n <= 512
// The same orthogonal iteration with a 64-column block kept as two 32-column
// halves Pa, Pb (each n x 32): every power step orthonormalises Pa (k_orth32),
// removes its span from Pb twice (k_proj32: Pb -= Pa (Pa^T Pb)), then
// orthonormalises Pb, so [Pa Pb] is orthonormal; the Rayleigh-Ritz matrix B =
// [Pa Pb]^T G [Pa Pb] (k_rr64_prep) goes to the 64-wide LDS Jacobi, V =
// [Pa Pb] W (k_combine64), and launch_select_factor takes the rank.

// Pb -= Pa (Pa^T Pb), twice (classical Gram-Schmidt of the block, repeated).
__global__ __launch_bounds__(OT) void k_proj32(const double* __restrict__ Pa, double* __restrict__ Pb, int n) {
    extern __shared__ double lds[];
    double* part_lds = lds;
    double(*C)[S32 + 1] = reinterpret_cast<double(*)[S32 + 1]>(lds + OW * S32 * S32);
    for (int pass = 0; pass < 2; ++pass) {
        cross32<OW, 1, 1>(Pa, Pb, n, part_lds, C);
        apply32<1, OW>(Pa, Pb, n, C, nullptr, Pb);
        __syncthreads();
    }
}

// B (64 x 64, row-major, symmetrised) = [Qa Qb]^T [Za Zb]; when either
// orthonormalisation failed, the mode is handed to the next eigensolver.
__global__ __launch_bounds__(RT) void k_rr64_prep(const double* __restrict__ Qa, const double* __restrict__ Qb,
                                                  const double* __restrict__ Za, const double* __restrict__ Zb,
                                                  int n, const int32_t* __restrict__ orth_ok,
                                                  DevBook* __restrict__ book, double* __restrict__ B) {
    extern __shared__ double lds[];
    double* part_lds = lds;
    double(*C)[S32 + 1] = reinterpret_cast<double(*)[S32 + 1]>(lds + RW * S32 * S32);
    __shared__ double full[2 * S32][2 * S32 + 1];
    const int tid = threadIdx.x;
    if (!*orth_ok) {
        if (tid == 0) book->need_dense = 1;
        return;
    }
    for (int blk = 0; blk < 4; ++blk) {
        const double* P = (blk >> 1) ? Qb : Qa;
        const double* Z = (blk & 1) ? Zb : Za;
        cross32<RW, 1, 1>(P, Z, n, part_lds, C);
        for (int e = tid; e < S32 * S32; e += RT) {
            const int i = e >> 5, j = e & 31;
            full[32 * (blk >> 1) + i][32 * (blk & 1) + j] = C[i][j];
        }
        __syncthreads();
    }
    for (int e = tid; e < 4 * S32 * S32; e += RT) {
        const int i = e >> 6, j = e & 63;
        B[e] = 0.5 * (full[i][j] + full[j][i]);
    }
}

// The 64 x 64 Jacobi in slot order (jacobi64_slots) on one matrix: G (n x n,
// row stride ldg, 33 <= n <= 64) in, eigenvalues descending in lam (equal
// values by index), eigenvectors in the matching columns of V (row stride ldv).
__global__ __launch_bounds__(J64_THREADS) void k_jacobi64_slots(const double* __restrict__ G, int n, int ldg,
                                                                int max_sweeps, double* __restrict__ lam,
                                                                double* __restrict__ V, int ldv,
                                                                int32_t* __restrict__ sweeps_out,
                                                                int32_t* __restrict__ ok_out, double floor_rel) {
    __shared__ double Ab[2][J64_ROWS][J64_LD];
    __shared__ J64Shared sh;
    __shared__ int rank_of[64];
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += J64_THREADS) {
        const int i = e / n, j = e % n;
        Ab[0][i][j] = G[(int64_t)i * ldg + j];
    }
    __syncthreads();
    int sweeps = 0;
    const bool conv = jacobi64_slots(n, max_sweeps, floor_rel, Ab[0], Ab[1], sh, Ab[0], sweeps);
    for (int i = tid; i < n; i += J64_THREADS) {
        const double li = sh.diag[i];
        int r = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = sh.diag[j];
            r += (lj > li) || (lj == li && j < i);
        }
        rank_of[i] = r;
    }
    __syncthreads();
    for (int i = tid; i < n; i += J64_THREADS) lam[rank_of[i]] = sh.diag[i];  // unclamped (see select)
    for (int idx = tid; idx < n * n; idx += J64_THREADS) {
        const int row = idx / n, i = idx % n;
        V[(int64_t)row * ldv + rank_of[i]] = Ab[0][row][i];
    }
    if (tid == 0) {
        if (sweeps_out) *sweeps_out = sweeps;
        if (ok_out) *ok_out = conv ? 1 : 0;
    }
}

// V[i][j] = sum_c Qa[i][c] W[c][j] + Qb[i][c] W[32 + c][j]  (n x 64, W 64 x 64).
__global__ __launch_bounds__(256) void k_combine64(const double* __restrict__ Qa, const double* __restrict__ Qb,
                                                   const double* __restrict__ W, double* __restrict__ V, int n) {
    __shared__ double w[2 * S32][2 * S32];
    for (int e = threadIdx.x; e < 4 * S32 * S32; e += 256) w[e >> 6][e & 63] = W[e];
    __syncthreads();
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)n * 64) return;
    const int i = (int)(idx >> 6), j = (int)(idx & 63);
    const double* qa = Qa + (int64_t)i * S32;
    const double* qb = Qb + (int64_t)i * S32;
    double t = 0.0;
#pragma unroll 8
    for (int c = 0; c < S32; ++c) t += qa[c] * w[c][j];
#pragma unroll 8
    for (int c = 0; c < S32; ++c) t += qb[c] * w[S32 + c][j];
    V[idx] = t;
}

// The power steps and the 64 x 64 Rayleigh-Ritz matrix of the m = 64 path in
// one cooperative launch (the kernels k_gemm_gx, k_orth32, k_proj32 and
// k_rr64_prep of the kernel chain, with the slab decomposition and fixed-order
// exchanges of k_sub32_grid): on return B (64 x 64, row-major, symmetrised)
// and the basis halves are in global memory and *ok says whether both
// orthonormalisations succeeded (else book->need_dense is set).  With two
// power steps the basis ends in the buffers passed as Za, Zb.
__device__ __forceinline__ void sub64_grid_body(const double* __restrict__ G, int n, double* Pa, double* Pb,
                                                double* Za, double* Zb, const Sub32Grid& g,
                                                DevBook* __restrict__ book, double* __restrict__ B,
                                                int32_t* __restrict__ ok) {
    extern __shared__ double lds[];
    double* part_lds = lds;
    double(*C)[S32 + 1] = reinterpret_cast<double(*)[S32 + 1]>(lds + RW * S32 * S32);
    double(*R)[S32 + 1] = reinterpret_cast<double(*)[S32 + 1]>(lds + RW * S32 * S32 + S32 * (S32 + 1));
    __shared__ double full[2 * S32][2 * S32 + 1];
    __shared__ double rowbuf[64];
    __shared__ int ok_s;
    const int tid = threadIdx.x;
    GridCtx x;
    x.g = g;
    x.n = n;
    x.b = blockIdx.x;
    x.nb = gridDim.x;
    x.row0 = GRID_ROWS * x.b;
    x.nr = min(GRID_ROWS, n - x.row0);
    x.arrivals = 0;
    x.parity = 0;
    x.gave_up = false;
    const int64_t ro = (int64_t)x.row0 * S32;
    gx_rows32<true>(x, G, nullptr, 0x5eed, Pa, part_lds);
    gx_rows32<true>(x, G, nullptr, 0x64b5eed, Pb, part_lds);
    constexpr int steps = 2;
    bool good = true;
    for (int it = 0; it < steps && good; ++it) {
        const bool fin = it + 1 == steps;
        good = orth_grid(x, Pa + ro, fin, part_lds, C, R, rowbuf, &ok_s);
        if (!good) break;
        for (int pass = 0; pass < 2; ++pass) {  // Pb -= Pa (Pa^T Pb), twice
            cross_grid(x, Pa + ro, Pb + ro, part_lds, C);
            apply32<1, RW, 1>(Pa + ro, Pb + ro, x.nr, C, nullptr, Pb + ro);
            __syncthreads();
        }
        good = orth_grid(x, Pb + ro, fin, part_lds, C, R, rowbuf, &ok_s);
        if (!good) break;
        x.sync();
        gx_rows32<false>(x, G, Pa, 0, Za, part_lds);
        gx_rows32<false>(x, G, Pb, 0, Zb, part_lds);
        if (!fin) {
            double* t = Pa;
            Pa = Za;
            Za = t;
            t = Pb;
            Pb = Zb;
            Zb = t;
        }
    }
    if (!good) {
        // the same outcome in every workgroup: hand the mode to the next eigensolver
        if (x.b == 0 && tid == 0) {
            book->need_dense = 1;
            if (__hip_atomic_load(&g.sync[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                book->status = ATC_ERR_INTERNAL;  // not a failed basis: a wait gave up
            *ok = 0;
        }
        return;
    }
    // B = [Pa Pb]^T [Za Zb], block by block, symmetrised by workgroup 0
    for (int blk = 0; blk < 4; ++blk) {
        const double* P = (blk >> 1) ? Pb : Pa;
        const double* Z = (blk & 1) ? Zb : Za;
        cross_grid(x, P + ro, Z + ro, part_lds, C);
        for (int e = tid; e < S32 * S32; e += RT) {
            const int i = e >> 5, j = e & 31;
            full[32 * (blk >> 1) + i][32 * (blk & 1) + j] = C[i][j];
        }
        __syncthreads();
    }
    if (x.b == 0) {
        for (int e = tid; e < 4 * S32 * S32; e += RT) {
            const int i = e >> 6, j = e & 63;
            B[e] = 0.5 * (full[i][j] + full[j][i]);
        }
        if (tid == 0) {
            if (__hip_atomic_load(&g.sync[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                book->status = ATC_ERR_INTERNAL;
            *ok = 1;
        }
    }
}

__global__ __launch_bounds__(RT) void k_sub64_grid(const double* __restrict__ G, int n, double* Pa, double* Pb,
                                                   double* Za, double* Zb, Sub32Grid g, DevBook* __restrict__ book,
                                                   double* __restrict__ B, int32_t* __restrict__ ok) {
    sub64_grid_body(G, n, Pa, Pb, Za, Zb, g, book, B, ok);
    grid_exit(g.sync);
}

bool sub64_ready() {
    static int state = 0;
    if (state == 0) {
        const bool a = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_proj32),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)ORTH_LDS) == hipSuccess;
        const bool b = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rr64_prep),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)RR_LDS) == hipSuccess;
        state = (a && b) ? 1 : -1;
    }
    return state == 1;
}

bool sub64_grid_ready() {
    static int state = 0;
    if (state == 0)
        state = sub32_grid_supported() && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sub64_grid),
                                                              hipFuncAttributeMaxDynamicSharedMemorySize,
                                                              (int)RR_LDS) == hipSuccess
                    ? 1
                    : -1;
    return state == 1 && !kernel_chain_forced();
}

}  // namespace

bool subspace32_available(int n) { return n >= 2 * S32 && n <= 512 && sub32_ready(); }

bool subspace32_split_available(int n) { return subspace32_available(n) && sub32_grid_ready(); }

// P1, P2 (n x 32 each), 8 doubles of flags, then the cooperative path's
// partial products and sign candidates, then B and trace(G) of the split form.
size_t subspace32_ws_doubles(int n) {
    return (size_t)2 * n * S32 + 8 + (size_t)2 * GRID_MAXB * S32 * S32 + (size_t)GRID_MAXB * S32 * 3 + S32 * S32 + 8;
}

namespace {
Sub32Grid sub32_grid_args(double* ws, int n, const SelectArgs& sa) {
    Sub32Grid g;
    g.P1 = ws;
    g.P2 = ws + (size_t)n * S32;
    g.part = g.P2 + (size_t)n * S32 + 8;
    g.cand = g.part + (size_t)2 * GRID_MAXB * S32 * S32;
    g.sync = &sa.book->grid[0];
    // ATC_GRID_SPIN_LIMIT (tests): a small limit makes the waits give up,
    // which the mode must report as an error without hanging
    const char* lim = getenv("ATC_GRID_SPIN_LIMIT");
    g.spin_limit = lim ? (unsigned)strtoul(lim, nullptr, 10) : GRID_SPIN_LIMIT;
    g.basis_ok = nullptr;
    g.bsym = nullptr;
    return g;
}
}  // namespace

hipError_t run_subspace32_select(const double* G, int n, int iters, int max_sweeps, double* ws, const SelectArgs& sa,
                                 hipStream_t st, bool allow_coop) {
    if (!subspace32_available(n)) return hipErrorInvalidValue;
    if (sa.ncand != S32 || sa.ldv != S32 || !sa.subspace) return hipErrorInvalidValue;
    double* P1 = ws;                   // n x 32
    double* P2 = P1 + (size_t)n * S32;  // n x 32
    int32_t* ok = reinterpret_cast<int32_t*>(P2 + (size_t)n * S32);
    const int steps = iters < 1 ? 1 : iters;
    hipError_t e;
    if (allow_coop && sub32_grid_ready()) {
        Sub32Grid g = sub32_grid_args(ws, n, sa);
        const int nb = (int)ceil_div(n, GRID_ROWS);
        int n_ = n, steps_ = steps, sweeps_ = max_sweeps;
        SelectArgs sa_ = sa;
        QtOut qt{};
        void* args[] = {(void*)&G, (void*)&n_, (void*)&steps_, (void*)&sweeps_, (void*)&g, (void*)&sa_, (void*)&qt};
        e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_sub32_grid), dim3(nb), dim3(RT), args,
                                       (unsigned)RR_LDS, st);
        if (e == hipSuccess) return hipSuccess;
        (void)hipGetLastError();  // not launched: the kernel-per-step path below
    }
    const dim3 gg((unsigned)ceil_div(n, GX_ROWS));
    const dim3 gb(64 * GX_SPLIT);
    hipLaunchKernelGGL(k_gemm_gx, gg, gb, 0, st, G, (const double*)nullptr, P1, n, (uint64_t)0x5eed);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int it = 0; it < steps; ++it) {
        // P1 <- orthonormal basis of its columns, then P2 <- G P1; the last basis
        // (the Rayleigh-Ritz one) gets the verified final correction
        hipLaunchKernelGGL(k_orth32, dim3(1), dim3(OT), ORTH_LDS, st, P1, n, it + 1 == steps ? 1 : 0,
                           it == 0 ? 1 : 0, ok);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_gemm_gx, gg, gb, 0, st, G, (const double*)P1, P2, n, (uint64_t)0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        std::swap(P1, P2);
    }
    // P2 holds the basis, P1 = G times it
    hipLaunchKernelGGL(k_rr32_select, dim3(1), dim3(RT), RR_LDS, st, (const double*)P2, (const double*)P1, n,
                       max_sweeps, (const int32_t*)ok, 0, (const double*)nullptr, sa);
    return hipGetLastError();
}

hipError_t run_subspace32_basis(const double* G, int n, int iters, double* ws, const SelectArgs& sa, const QtOut& qt,
                                hipStream_t st) {
    if (!subspace32_available(n) || !sub32_grid_ready()) return hipErrorInvalidValue;
    if (sa.ncand != S32 || sa.ldv != S32 || !sa.subspace || (!qt.t64 && !qt.t32)) return hipErrorInvalidValue;
    Sub32Grid g = sub32_grid_args(ws, n, sa);
    g.basis_ok = reinterpret_cast<int32_t*>(g.P2 + (size_t)n * S32);
    g.bsym = g.cand + (size_t)GRID_MAXB * S32 * 3;
    const int nb = (int)ceil_div(n, GRID_ROWS);
    const double* G_ = G;
    int n_ = n, steps_ = iters < 1 ? 1 : iters, sweeps_ = 0;
    SelectArgs sa_ = sa;
    QtOut qt_ = qt;
    void* args[] = {(void*)&G_, (void*)&n_, (void*)&steps_, (void*)&sweeps_, (void*)&g, (void*)&sa_, (void*)&qt_};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_sub32_grid), dim3(nb), dim3(RT), args,
                                      (unsigned)RR_LDS, st);
}

const int32_t* split_rows_dev(const double* ws, int n) {
    return reinterpret_cast<const int32_t*>(ws + (size_t)2 * n * S32) + 1;
}

hipError_t run_rr32_select(int n, int iters, int max_sweeps, double* ws, const SelectArgs& sa, hipStream_t st) {
    if (!subspace32_available(n)) return hipErrorInvalidValue;
    // the power steps swap the two n x 32 blocks once each: after an odd
    // number of steps the basis is in the first block
    const int steps = iters < 1 ? 1 : iters;
    const double* Q = ws + ((steps & 1) ? 0 : (size_t)n * S32);
    const double* Z = ws + ((steps & 1) ? (size_t)n * S32 : 0);  // G Q
    const int32_t* ok = reinterpret_cast<const int32_t*>(ws + (size_t)2 * n * S32);
    const double* bsym = ws + (size_t)2 * n * S32 + 8 + (size_t)2 * GRID_MAXB * S32 * S32 + (size_t)GRID_MAXB * S32 * 3;
    hipLaunchKernelGGL(k_rr32_select, dim3(1), dim3(RT), RR_LDS, st, Q, Z, n, max_sweeps, ok, 1, bsym, sa);
    return hipGetLastError();
}

// Pa, Pb, Za, Zb (n x 32 each), B and W (64 x 64), 8 doubles of flags, then
// the cooperative path's partial products.
size_t subspace64b_ws_doubles(int n) {
    return (size_t)4 * n * S32 + 2 * 64 * 64 + 8 + (size_t)2 * GRID_MAXB * S32 * S32;
}

hipError_t run_subspace64_select(const double* G, int n, int max_sweeps, double* ws, double* lam, double* V,
                                 int32_t* sweeps_dev, int32_t* ok_dev, const SelectArgs& sa, hipStream_t st, bool allow_coop) {
    if (!subspace32_available(n) || !sub64_ready()) return hipErrorInvalidValue;
    if (sa.ncand != 64 || sa.ldv != 64 || !sa.subspace) return hipErrorInvalidValue;
    double* Pa = ws;
    double* Pb = Pa + (size_t)n * S32;
    double* Za = Pb + (size_t)n * S32;
    double* Zb = Za + (size_t)n * S32;
    double* B = Zb + (size_t)n * S32;     // 64 x 64
    double* W = B + 64 * 64;              // 64 x 64
    int32_t* ok = reinterpret_cast<int32_t*>(W + 64 * 64);
    const dim3 gg((unsigned)ceil_div(n, GX_ROWS));
    const dim3 gb(64 * GX_SPLIT);
    hipError_t e;
    bool prepared = false;
    if (allow_coop && sub64_grid_ready()) {
        Sub32Grid g;
        g.P1 = nullptr;
        g.P2 = nullptr;
        g.part = W + 64 * 64 + 8;
        g.cand = nullptr;
        g.sync = &sa.book->grid[0];
        g.basis_ok = nullptr;
        g.bsym = nullptr;
        const char* lim = getenv("ATC_GRID_SPIN_LIMIT");
        g.spin_limit = lim ? (unsigned)strtoul(lim, nullptr, 10) : GRID_SPIN_LIMIT;
        const int nb = (int)ceil_div(n, GRID_ROWS);
        int n_ = n;
        DevBook* book = sa.book;
        void* args[] = {(void*)&G, (void*)&n_, (void*)&Pa, (void*)&Pb, (void*)&Za,
                        (void*)&Zb, (void*)&g,  (void*)&book, (void*)&B, (void*)&ok};
        e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_sub64_grid), dim3(nb), dim3(RT), args,
                                       (unsigned)RR_LDS, st);
        if (e == hipSuccess) {
            prepared = true;
            // two power steps: the basis ends in the buffers passed as Za, Zb
            std::swap(Pa, Za);
            std::swap(Pb, Zb);
        } else {
            (void)hipGetLastError();  // not launched: the kernel-per-step path below
        }
    }
    if (!prepared) {
        hipLaunchKernelGGL(k_gemm_gx, gg, gb, 0, st, G, (const double*)nullptr, Pa, n, (uint64_t)0x5eed);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_gemm_gx, gg, gb, 0, st, G, (const double*)nullptr, Pb, n, (uint64_t)0x64b5eed);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        constexpr int steps = 2;
        for (int it = 0; it < steps; ++it) {
            const int full = it + 1 == steps ? 1 : 0;
            hipLaunchKernelGGL(k_orth32, dim3(1), dim3(OT), ORTH_LDS, st, Pa, n, full, 1, ok);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_proj32, dim3(1), dim3(OT), ORTH_LDS, st, (const double*)Pa, Pb, n);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_orth32, dim3(1), dim3(OT), ORTH_LDS, st, Pb, n, full, 0, ok);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_gemm_gx, gg, gb, 0, st, G, (const double*)Pa, Za, n, (uint64_t)0);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_gemm_gx, gg, gb, 0, st, G, (const double*)Pb, Zb, n, (uint64_t)0);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if (it + 1 < steps) {
                std::swap(Pa, Za);
                std::swap(Pb, Zb);
            }
        }
        hipLaunchKernelGGL(k_rr64_prep, dim3(1), dim3(RT), RR_LDS, st, (const double*)Pa, (const double*)Pb,
                           (const double*)Za, (const double*)Zb, n, (const int32_t*)ok, sa.book, B);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // the Ritz problem of float32 data: couplings under JACOBI_FLOOR_F32 trace(B) left alone, as in jacobi32
    if ((e = launch_eig_jacobi_lds(B, 64, 64, max_sweeps, lam, W, 64, sweeps_dev, ok_dev, st, JACOBI_FLOOR_F32)) !=
        hipSuccess)
        return e;
    hipLaunchKernelGGL(k_combine64, dim3((unsigned)ceil_div((int64_t)n * 64, 256)), dim3(256), 0, st,
                       (const double*)Pa, (const double*)Pb, (const double*)W, V, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_select_factor(sa, st);
}

hipError_t launch_prepare_matrix(int prec, const void* U, int src_f64, int rows, int cols, int transpose,
                                 double* M64, float* M32, __bf16* Mh, __bf16* Ml, hipStream_t st) {
    (void)prec;
    const int64_t total = (int64_t)rows * cols;
    hipLaunchKernelGGL(k_prepare_matrix, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, U, src_f64, rows,
                       cols, transpose, M64, M32, Mh, Ml);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
    const size_t words = bytes / 4;
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)ceil_div((int64_t)words, 256)), dim3(256), 0, st, (uint32_t*)p, words);
    return hipGetLastError();
}

}  // namespace atc
