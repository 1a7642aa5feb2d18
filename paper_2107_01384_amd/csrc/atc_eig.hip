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
// (n/2 disjoint rotations per round, n-1 rounds per sweep), one workgroup,
// matrix and eigenvectors in LDS for n <= 64, or in global memory (any n,
// slow) as the fallback.  A rotation is skipped when
// |a_pq| <= tol * sqrt(|a_pp a_qq|), tol = n * 2^-53; a sweep with no rotation
// ends the iteration.
//
// Subspace path (n > 64): the ranks this method keeps are small next to n, so
// only the leading m (<= 64) eigenpairs are needed: subspace iteration with a
// Rayleigh-Ritz projection at every step, the small m x m problems solved by
// the LDS Jacobi.  Ritz values never exceed the true eigenvalues, so the tail
// trace(G) - sum(kept Ritz values) over-estimates the discarded energy and
// the error bound still holds; a rank that reaches into the last `guard`
// Ritz pairs sends the mode to the dense path instead.
#include <math.h>

#include "atc_internal.hpp"

namespace atc {
namespace {

constexpr int JMAX = 64;

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

// ------------------------------------------------------------------ LDS Jacobi
__global__ __launch_bounds__(256) void k_eig_jacobi_lds(const double* __restrict__ G, int n, int ldg,
                                                        int max_sweeps, double* __restrict__ lam,
                                                        double* __restrict__ V, int ldv,
                                                        int32_t* __restrict__ sweeps_out,
                                                        int32_t* __restrict__ ok_out) {
    __shared__ double A[JMAX][JMAX + 1];
    __shared__ double Vs[JMAX][JMAX + 1];
    __shared__ int pp[JMAX / 2], qq[JMAX / 2];
    __shared__ double cs[JMAX / 2], sn[JMAX / 2], dpp[JMAX / 2], dqq[JMAX / 2];
    __shared__ int rotated;
    const int tid = threadIdx.x;
    const int m = n + (n & 1);
    for (int idx = tid; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx % m;
        A[i][j] = (i < n && j < n) ? G[(int64_t)i * ldg + j] : 0.0;
        Vs[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const double tol = (double)n * 0x1p-53;
    int sweeps = 0;
    bool converged = (m < 2);
    while (!converged && sweeps < max_sweeps) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int round = 0; round < m - 1; ++round) {
            if (tid < m / 2) {
                int p, q;
                round_robin_pair(round, tid, m, p, q);
                double c, s, dp, dq;
                if (schur2(A[p][p], A[q][q], A[p][q], tol, c, s, dp, dq)) rotated = 1;
                pp[tid] = p;
                qq[tid] = q;
                cs[tid] = c;
                sn[tid] = s;
                dpp[tid] = dp;
                dqq[tid] = dq;
            }
            __syncthreads();
            for (int idx = tid; idx < (m / 2) * m; idx += blockDim.x) {
                const int k = idx / m, j = idx % m;
                const double c = cs[k], s = sn[k];
                if (s == 0.0) continue;
                const int p = pp[k], q = qq[k];
                const double x = A[p][j], y = A[q][j];
                A[p][j] = c * x - s * y;
                A[q][j] = s * x + c * y;
            }
            __syncthreads();
            for (int idx = tid; idx < m * (m / 2); idx += blockDim.x) {
                const int i = idx / (m / 2), k = idx % (m / 2);
                const double c = cs[k], s = sn[k];
                if (s == 0.0) continue;
                const int p = pp[k], q = qq[k];
                const double x = A[i][p], y = A[i][q];
                A[i][p] = c * x - s * y;
                A[i][q] = s * x + c * y;
                const double vx = Vs[i][p], vy = Vs[i][q];
                Vs[i][p] = c * vx - s * vy;
                Vs[i][q] = s * vx + c * vy;
            }
            __syncthreads();
            // the rotated pair is annihilated exactly and its diagonal set from the
            // 2x2 formulas (the row and column passes leave rounding residue there)
            if (tid < m / 2 && sn[tid] != 0.0) {
                const int p = pp[tid], q = qq[tid];
                A[p][q] = 0.0;
                A[q][p] = 0.0;
                A[p][p] = dpp[tid];
                A[q][q] = dqq[tid];
            }
            __syncthreads();
        }
        ++sweeps;
        converged = (rotated == 0);
        __syncthreads();
    }
    // eigenvalues = diagonal; order descending, equal values by index
    __shared__ int rank_of[JMAX];
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
    for (int i = tid; i < n; i += blockDim.x) {
        const double li = A[i][i];
        lam[rank_of[i]] = li;  // unclamped: tail sums keep the sign of rounding-level values
    }
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

// ------------------------------------------------------------ small FP64 GEMM
// C[i, j] = alpha * sum_k A(i, k) B(k, j) (+ beta * C), with A(i, k) = A[i*sa0 + k*sa1],
// B(k, j) = B[k*sb0 + j*sb1]; optional column scale of B: B(k, j) * bscale[j].
__global__ __launch_bounds__(256) void k_gemm64(int M, int N, int K, const double* __restrict__ A, int64_t sa0,
                                                int64_t sa1, const double* __restrict__ B, int64_t sb0, int64_t sb1,
                                                const double* __restrict__ bscale, double* __restrict__ C,
                                                int64_t ldc) {
    __shared__ double As[32][33];
    __shared__ double Bs[32][33];
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
    double acc[2][2] = {{0, 0}, {0, 0}};
    for (int k0 = 0; k0 < K; k0 += 32) {
        for (int idx = tid; idx < 32 * 32; idx += 256) {
            const int r = idx / 32, c = idx % 32;
            const int gi = i0 + r, gk = k0 + c;
            As[r][c] = (gi < M && gk < K) ? A[gi * sa0 + gk * sa1] : 0.0;
            const int bk = k0 + r, bj = j0 + c;
            double bv = (bk < K && bj < N) ? B[bk * sb0 + bj * sb1] : 0.0;
            if (bscale && bj < N) bv *= bscale[bj];
            Bs[r][c] = bv;
        }
        __syncthreads();
#pragma unroll 8
        for (int k = 0; k < 32; ++k) {
            const double a0 = As[ty * 2][k], a1 = As[ty * 2 + 1][k];
            const double b0 = Bs[k][tx * 2], b1 = Bs[k][tx * 2 + 1];
            acc[0][0] += a0 * b0;
            acc[0][1] += a0 * b1;
            acc[1][0] += a1 * b0;
            acc[1][1] += a1 * b1;
        }
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int gi = i0 + ty * 2 + a, gj = j0 + tx * 2 + b;
            if (gi < M && gj < N) C[gi * ldc + gj] = acc[a][b];
        }
}

hipError_t gemm64(int M, int N, int K, const double* A, int64_t sa0, int64_t sa1, const double* B, int64_t sb0,
                  int64_t sb1, const double* bscale, double* C, int64_t ldc, hipStream_t st) {
    dim3 grid((unsigned)ceil_div(N, 32), (unsigned)ceil_div(M, 32));
    hipLaunchKernelGGL(k_gemm64, grid, dim3(256), 0, st, M, N, K, A, sa0, sa1, B, sb0, sb1, bscale, C, ldc);
    return hipGetLastError();
}

// deterministic pseudo-random fill in [-1, 1) (splitmix64 of the index)
__device__ inline double hash_unit(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (double)(x >> 11) * 0x1p-52 - 1.0;
}

__global__ void k_fill_random(double* Q, int n, int m, uint64_t salt) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < (int64_t)n * m) Q[idx] = hash_unit((uint64_t)idx * 0x2545F4914F6CDD1Dull + salt);
}

// Orthonormalises the columns of X (n x m, row-major, in place) by classical
// Gram-Schmidt applied twice per column (CGS2); a column that loses all but
// 1e-10 of its norm is numerically dependent and is replaced by a
// pseudo-random vector (then orthogonalised again), or zeroed if that fails.
// One workgroup; the current column is staged in LDS.
__device__ inline double block_sum(double s, double* red, int lane, int wave, int nw) {
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

__global__ __launch_bounds__(1024) void k_cgs2(double* __restrict__ X, int n, int m, uint64_t salt) {
    extern __shared__ double col[];     // n doubles
    __shared__ double h[64];
    __shared__ double red[17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    for (int j = 0; j < m; ++j) {
        for (int i = tid; i < n; i += blockDim.x) col[i] = X[(int64_t)i * m + j];
        __syncthreads();
        for (int attempt = 0; attempt < 2; ++attempt) {
            double s = 0.0;
            for (int i = tid; i < n; i += blockDim.x) s += col[i] * col[i];
            const double norm0 = sqrt(block_sum(s, red, lane, wave, nw));
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
            const double nrm = sqrt(block_sum(s, red, lane, wave, nw));
            if (nrm > 1e-10 * norm0 && nrm > 0.0 && isfinite(nrm)) {
                for (int i = tid; i < n; i += blockDim.x) col[i] /= nrm;
                __syncthreads();
                break;
            }
            // dependent column: retry once with a pseudo-random vector, else zero it
            for (int i = tid; i < n; i += blockDim.x)
                col[i] = attempt == 0 ? hash_unit(((uint64_t)i * 977 + j) * 0x2545F4914F6CDD1Dull + salt) : 0.0;
            __syncthreads();
        }
        for (int i = tid; i < n; i += blockDim.x) X[(int64_t)i * m + j] = col[i];
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_eig_jacobi_lds(const double* G, int n, int ldg, int max_sweeps, double* lam, double* V, int ldv,
                                 int32_t* sweeps_out, int32_t* ok_out, hipStream_t st) {
    if (n > JMAX || n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_eig_jacobi_lds, dim3(1), dim3(256), 0, st, G, n, ldg, max_sweeps, lam, V, ldv,
                       sweeps_out, ok_out);
    return hipGetLastError();
}

hipError_t launch_eig_jacobi_global(const double* G, int n, int max_sweeps, double* A_ws, double* lam, double* V,
                                    int32_t* sweeps_out, int32_t* ok_out, hipStream_t st) {
    const int m = n + (n & 1);
    // A_ws holds 2 * m * m doubles: the working matrix, then the eigenvector accumulator
    // pair indices (2 x m/2 ints) then c, s and the two new diagonals (4 x m/2 doubles)
    const size_t shm = (size_t)m * sizeof(int) + (size_t)2 * m * sizeof(double) + 64;
    if (shm > 64 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_eig_jacobi_global, dim3(1), dim3(1024), shm, st, G, n, max_sweeps, A_ws, lam, V,
                       A_ws + (size_t)m * m, sweeps_out, ok_out);
    return hipGetLastError();
}

size_t subspace_ws_doubles(int n, int m) {
    return (size_t)3 * n * m + (size_t)2 * m * m + (size_t)m + 64;
}

// Leading m eigenpairs of the PSD matrix G (n x n): power steps with
// re-orthonormalisation, Q_0 = orth(G Omega), Q_t = orth(G Q_{t-1}), then the
// Rayleigh-Ritz projection B = Q^T G Q = W diag(theta) W^T, U = Q W.
hipError_t run_subspace_eig(const double* G, int n, int m, int iters, int max_sweeps, double* ws, double* lam,
                            double* V, int32_t* sweeps_out, int32_t* ok_out, hipStream_t st) {
    if (m > JMAX || m < 2 || n < m || n > 4096) return hipErrorInvalidValue;
    double* Q = ws;                       // n x m
    double* Z = Q + (size_t)n * m;        // n x m
    double* Y = Z + (size_t)n * m;        // n x m
    double* B = Y + (size_t)n * m;        // m x m
    double* W = B + (size_t)m * m;        // m x m
    hipError_t e;
    const int nb = (int)ceil_div((int64_t)n * m, 256);
    const size_t shm = sizeof(double) * (size_t)n;
    hipLaunchKernelGGL(k_fill_random, dim3(nb), dim3(256), 0, st, Y, n, m, (uint64_t)0x5eed);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int steps = iters < 1 ? 1 : iters;
    for (int it = 0; it < steps; ++it) {
        if ((e = gemm64(n, m, n, G, n, 1, it == 0 ? Y : Z, m, 1, nullptr, Q, m, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_cgs2, dim3(1), dim3(1024), shm, st, Q, n, m, (uint64_t)(it + 1));
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (it + 1 < steps) {
            if ((e = hipMemcpyAsync(Z, Q, sizeof(double) * n * m, hipMemcpyDeviceToDevice, st)) != hipSuccess)
                return e;
        }
    }
    if ((e = gemm64(n, m, n, G, n, 1, Q, m, 1, nullptr, Z, m, st)) != hipSuccess) return e;
    if ((e = gemm64(m, m, n, Q, 1, m, Z, m, 1, nullptr, B, m, st)) != hipSuccess) return e;
    if ((e = launch_eig_jacobi_lds(B, m, m, max_sweeps, lam, W, m, sweeps_out, ok_out, st)) != hipSuccess) return e;
    return gemm64(n, m, m, Q, m, 1, W, m, 1, nullptr, V, m, st);
}

// ------------------------------------------------------- rank select + factor
namespace {

__global__ __launch_bounds__(256) void k_select_factor(SelectArgs a) {
    __shared__ int r_s;
    __shared__ int sign_s[4096];
    const int tid = threadIdx.x;
    DevBook* bk = a.book;
    if (tid == 0) {
        // trace of G in a fixed order
        double tr = 0.0;
        for (int i = 0; i < a.n; ++i) tr += a.G[(int64_t)i * a.n + i];
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
            // tail(r) = sum_{j >= r} lam_j, added from the smallest upward
            double acc = 0.0;
            int best = a.n;
            double best_tail = 0.0;
            for (int j = a.n - 1; j >= 0; --j) {
                // acc = tail at r = j + 1
                if (j + 1 >= 1 && acc <= b) {
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
        if (bk->need_dense == 0) {
            bk->used += tail_r;
            bk->tail[a.k] = tail_r;
            bk->budget[a.k] = b;
            bk->rank[a.k] = r;
        }
        r_s = r;
    }
    __syncthreads();
    if (bk->need_dense) return;
    const int r = r_s;
    // sign rule: largest-magnitude entry of each kept column positive (first row on ties)
    for (int j = tid; j < r; j += blockDim.x) {
        double best = -1.0;
        double val = 0.0;
        for (int i = 0; i < a.n; ++i) {
            const double v = a.V[(int64_t)i * a.ldv + j];
            if (fabs(v) > best) {
                best = fabs(v);
                val = v;
            }
        }
        sign_s[j] = val < 0.0 ? -1 : 1;
    }
    __syncthreads();
    for (int64_t idx = tid; idx < (int64_t)a.n * r; idx += blockDim.x) {
        const int i = (int)(idx / r), j = (int)(idx % r);
        const double u = sign_s[j] * a.V[(int64_t)i * a.ldv + j];
        if (a.ufac_f64) ((double*)a.ufac)[idx] = u;
        else ((float*)a.ufac)[idx] = (float)u;
        const int64_t t = (int64_t)j * a.n + i;  // U^T, r x n
        if (a.Mt64) a.Mt64[t] = u;
        if (a.Mt32) {
            const float f = (float)u;
            a.Mt32[t] = f;
            if (a.Mth) {
                const __bf16 h = (__bf16)f;
                a.Mth[t] = h;
                a.Mtl[t] = (__bf16)(f - (float)h);
            }
        }
    }
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
    hipLaunchKernelGGL(k_select_factor, dim3(1), dim3(256), 0, st, a);
    return hipGetLastError();
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
