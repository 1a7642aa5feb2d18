// Batched ST-HOSVD: many independent small 3-way float32 blocks (every mode
// <= 64) in one persistent launch.
//
// Each workgroup loops: take the next block from an atomic work counter (blocks
// pre-sorted longest first), then run the whole ST-HOSVD of that block
// (Algorithm 1, Section 3.2; modes by increasing length, Section 4.1.1; error
// budget split as in atc_sthosvd, Section 4.1.3):
//   Gram matrix of the current unfolding  -> LDS, FP64 (the staged floats
//                                            widened, FP64 MFMA)
//   FP64 cyclic Jacobi eigensolver         -> in LDS (round-robin pairs,
//                                            exact annihilation)
//   rank choice (FP64 tail sums) and sign rule
//   factor -> its slot of the factor arena
//   mode product Z = U^T x_k Y (MFMA)      -> a per-workgroup scratch block or
//                                            the block's core slot
// Nothing is allocated and the host is not consulted, so the launch (plus the
// kernel that zeroes the counter) can be captured in a HIP graph.  A plan
// object fixes offsets, order and the launch configuration; a small
// autotuner times the candidate configurations on the caller's data.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "atc_internal.hpp"
#include "atc_jacobi64.hpp"

namespace atc {
namespace {

constexpr int BMAX = 64;       // longest mode of a block
constexpr int BT = 256;        // threads per workgroup
constexpr int APAD = BMAX + 1;

struct BlockDesc {
    int64_t in_off;
    int64_t core_off;
    int64_t fac_off;
    int32_t dims[3];
    int32_t pad;
};

template <int BK>
struct BatchSmem {
    union {
        struct {
            // Gram matrix, then the Jacobi iterate; V the eigenvectors.  The
            // slot-order Jacobi (n > 16) uses both as its two buffers of
            // J64_ROWS rows and leaves the eigenvectors in V.
            double A[J64_ROWS][APAD];
            double V[J64_ROWS][APAD];
        } e;
        struct {                   // Gram staging (aliases A; V unused then)
            __bf16 xh[BMAX][BK + 8];
            __bf16 xl[BMAX][BK + 8];
            float xf[BMAX][BK + 1];
        } g;
        union {                    // mode-product staging of Y (aliases A, dead
            struct {               // after the eigensolve; V stays intact)
                __bf16 yh[BMAX][BK + 8];
                __bf16 yl[BMAX][BK + 8];
            } b;
            float yf[BMAX][BK + 1];
        } t;
    } u;
    J64Shared j64;
    double lam[BMAX];
    int col_of[BMAX];   // eigenvector column of the j-th largest eigenvalue
    int sgn[BMAX];
    int pp[BMAX / 2], qq[BMAX / 2];
    double cs[BMAX / 2], sn[BMAX / 2], dpp[BMAX / 2], dqq[BMAX / 2];
    double red[8];
    int flag;
    int next;
    int rank;
    int status;
};

// ---- Gram of one (L, n, R) view (n <= 64) into sm.u.e.A ------------------
template <int P, int LAYOUT, int BK>
__device__ void blk_gram(const float* __restrict__ Y, int n, int64_t L, int64_t R, BatchSmem<BK>& sm) {
    constexpr int E = BMAX * BK / BT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    int srow[E], skk[E], sp[E], sr[E];
    bool sok[E];
    const int planes = (LAYOUT == LAYOUT_SR) ? BK / (int)R : 1;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        sp[e] = 0;
        sr[e] = 0;
        sok[e] = true;
        if (LAYOUT == LAYOUT_KC) {
            srow[e] = tid / BK + (BT / BK) * e;
            skk[e] = tid % BK;
        } else if (LAYOUT == LAYOUT_NC) {
            srow[e] = tid % BMAX;
            skk[e] = tid / BMAX + (BT / BMAX) * e;
        } else {
            const int Ri = (int)R;
            const int q = tid + BT * e;
            sr[e] = q % Ri;
            srow[e] = (q / Ri) % BMAX;
            sp[e] = q / (BMAX * Ri);
            sok[e] = sp[e] < planes;
            skk[e] = sp[e] * Ri + sr[e];
        }
    }
    int64_t steps, spl = 1;
    if (LAYOUT == LAYOUT_KC) {
        spl = ceil_div(R, BK);
        steps = L * spl;
    } else if (LAYOUT == LAYOUT_NC) {
        steps = ceil_div(L, BK);
    } else {
        steps = ceil_div(L, planes);
    }
    // unwritten slab columns (SR) stay zero
    for (int idx = tid; idx < BMAX * BK; idx += BT) {
        const int rr = idx / BK, kk = idx % BK;
        if (P == PREC_BF16X3) {
            sm.u.g.xh[rr][kk] = (__bf16)0.0f;
            sm.u.g.xl[rr][kk] = (__bf16)0.0f;
        } else {
            sm.u.g.xf[rr][kk] = 0.0f;
        }
    }
    f32x4 acc[2][2];
    f64x4 acc64[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            acc[a][b] = f32x4{0, 0, 0, 0};
            acc64[a][b] = f64x4{0, 0, 0, 0};
        }
    // exact diagonal: FP64 sums of squares of the loaded floats, one per
    // staging slot (row, kk) this thread fills (the same slots every step)
    double dsq[E];
#pragma unroll
    for (int e = 0; e < E; ++e) dsq[e] = 0.0;
    constexpr int FLUSH_STEPS = FLUSH_TERMS / BK;
    int since = 0;
    // the slab of step s into registers (zeros outside the tensor)
    float vreg[E];
    auto load = [&](int64_t s) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int row = srow[e];
            bool in = sok[e] && row < n;
            int64_t off = 0;
            if (LAYOUT == LAYOUT_KC) {
                const int64_t l = s / spl;
                const int64_t r = (s - l * spl) * BK + skk[e];
                in = in && r < R;
                off = (l * n + row) * R + r;
            } else if (LAYOUT == LAYOUT_NC) {
                const int64_t k = s * BK + skk[e];
                in = in && k < L;
                off = k * n + row;
            } else {
                const int64_t l = s * planes + sp[e];
                in = in && l < L;
                off = (l * n + row) * R + sr[e];
            }
            vreg[e] = in ? Y[off] : 0.f;
        }
    };
    if (steps > 0) load(0);
    for (int64_t s = 0; s < steps; ++s) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int row = srow[e];
            const float v = vreg[e];
            dsq[e] = fma((double)v, (double)v, dsq[e]);
            if (sok[e]) {
                if (P == PREC_BF16X3) {
                    const __bf16 h = (__bf16)v;
                    sm.u.g.xh[row][skk[e]] = h;
                    sm.u.g.xl[row][skk[e]] = (__bf16)(v - (float)h);
                } else {
                    sm.u.g.xf[row][skk[e]] = v;
                }
            }
        }
        __syncthreads();
        if (s + 1 < steps) load(s + 1);  // in flight while this slab is multiplied
        if (P == PREC_BF16X3) {
#pragma unroll
            for (int k0 = 0; k0 < BK; k0 += 32) {
                const int kq = k0 + 8 * (lane >> 4);
                bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    ah[a] = *reinterpret_cast<const bf16x8*>(&sm.u.g.xh[wr + a * 16 + (lane & 15)][kq]);
                    al[a] = *reinterpret_cast<const bf16x8*>(&sm.u.g.xl[wr + a * 16 + (lane & 15)][kq]);
                    bh[a] = *reinterpret_cast<const bf16x8*>(&sm.u.g.xh[wc + a * 16 + (lane & 15)][kq]);
                    bl[a] = *reinterpret_cast<const bf16x8*>(&sm.u.g.xl[wc + a * 16 + (lane & 15)][kq]);
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
                    }
            }
        } else if (P == PREC_F64ACC) {
            // the staged floats widened to FP64: exact products, FP64 sums
#pragma unroll
            for (int k4 = 0; k4 < BK; k4 += 4) {
                const int kk = k4 + (lane >> 4);
                double av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    av[a] = (double)sm.u.g.xf[wr + a * 16 + (lane & 15)][kk];
                    bv[a] = (double)sm.u.g.xf[wc + a * 16 + (lane & 15)][kk];
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc64[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc64[a][b], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int k4 = 0; k4 < BK; k4 += 4) {
                const int kk = k4 + (lane >> 4);
                float av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    av[a] = sm.u.g.xf[wr + a * 16 + (lane & 15)][kk];
                    bv[a] = sm.u.g.xf[wc + a * 16 + (lane & 15)][kk];
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
            }
        }
        if (P != PREC_F64ACC && ++since == FLUSH_STEPS) {
            since = 0;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc64[a][b][v] += (double)acc[a][b][v];
                    acc[a][b] = f32x4{0, 0, 0, 0};
                }
        }
    }
    __syncthreads();  // staging (aliasing A) no longer read
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = wr + a * 16 + mfma16_row<P>(lane, v);
                const int j = wc + b * 16 + (lane & 15);
                sm.u.e.A[i][j] = acc64[a][b][v] + (double)acc[a][b][v];
            }
    // per-slot squares into V (free until the eigensolver), laid out as the
    // staging slots: row i's are D[i * BK + kk]
    double* D = &sm.u.e.V[0][0];
    static_assert(BMAX * BK <= J64_ROWS * APAD, "diagonal partials fit in V");
#pragma unroll
    for (int e = 0; e < E; ++e)
        if (sok[e]) D[srow[e] * BK + skk[e]] = dsq[e];
    __syncthreads();
    // exact symmetry: the upper triangle wins; the diagonal is the exact sum
    // of squares (the products' rounding and the dropped lo*lo term of the
    // split would otherwise bias every discarded-energy sum by the trace error)
    const int kmax = LAYOUT == LAYOUT_SR ? planes * (int)R : BK;  // SR slots past the planes stay unwritten
    for (int idx = tid; idx < n * n; idx += BT) {
        const int i = idx / n, j = idx % n;
        if (i > j) sm.u.e.A[i][j] = sm.u.e.A[j][i];
    }
    if (tid < n) {
        double d = 0.0;
        for (int kk = 0; kk < kmax; ++kk) d += D[tid * BK + kk];
        sm.u.e.A[tid][tid] = d;
    }
    __syncthreads();
}

// ---- cyclic Jacobi on sm.u.e.A (n <= 64) --------------------------------
// The slot-order Jacobi inlined into the persistent kernel: a call would
// keep the kernel off the accumulation registers, whose 256 extra registers
// per lane then take what the Gram and mode-product loops would otherwise
// spill to scratch memory (133 -> 16 spilled registers).
template <int M>
__device__ __attribute__((always_inline)) inline bool blk_jacobi_slots(int n, int max_sweeps, double (*A)[APAD],
                                                           double (*V)[APAD], J64Shared* sh, int* sweeps) {
    return jacobi_slots<M>(n, max_sweeps, JACOBI_FLOOR_F32, A, V, *sh, V, *sweeps);
}

template <int BK>
__device__ bool blk_jacobi(int n, int max_sweeps, BatchSmem<BK>& sm) {
    const int tid = threadIdx.x;
    static_assert(APAD == J64_LD && BT == J64_THREADS, "slot-order Jacobi layout");
    if (n > 16) {
        // 17 <= n <= 64: the slot-order Jacobi (zero-padded to 32 or 64), same tests
        int sweeps = 0;
        const bool conv = n > 32 ? blk_jacobi_slots<64>(n, max_sweeps, sm.u.e.A, sm.u.e.V, &sm.j64, &sweeps)
                                 : blk_jacobi_slots<32>(n, max_sweeps, sm.u.e.A, sm.u.e.V, &sm.j64, &sweeps);
        for (int i = tid; i < n; i += BT) {
            const double li = sm.j64.diag[i];
            int r = 0;
            for (int j = 0; j < n; ++j) {
                const double lj = sm.j64.diag[j];
                r += (lj > li) || (lj == li && j < i);
            }
            sm.lam[r] = li;
            sm.col_of[r] = i;
        }
        __syncthreads();
        return conv;
    }
    const int m = n + (n & 1), h = m / 2;
    double (*A)[APAD] = sm.u.e.A;
    double (*Vm)[APAD] = sm.u.e.V;
    for (int idx = tid; idx < m * m; idx += BT) {
        const int i = idx / m, j = idx % m;
        if (i >= n || j >= n) A[i][j] = 0.0;
        Vm[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const double tol = (double)n * 0x1p-53;
    // couplings at or below JACOBI_FLOOR_F32 |trace| are left alone: below
    // what the float32 input resolves, and rotating them away costs sweeps
    // without changing the result at that accuracy
    double trace = 0.0;
    for (int i = 0; i < n; ++i) trace += A[i][i];
    const double floor = JACOBI_FLOOR_F32 * fabs(trace);
    // this thread's share of the round's work, fixed for the whole solve: up
    // to 3 of the h (h + 1) / 2 blocks (k, l), k <= l, and up to 8 of the m h
    // (row, pair) entries of the eigenvector update (codes k | l << 8 and
    // i | k << 8, -1 for none), so the rounds need no division
    constexpr int NBK = (BMAX / 2) * (BMAX / 2 + 1) / 2 / BT + 1;
    constexpr int NVR = BMAX * (BMAX / 2) / BT;
    int blk[NBK], vrk[NVR];
    {
        int b = 0, k = 0, l = 0;  // enumerate the upper triangle in order
        for (int j = 0; j < NBK; ++j) {
            const int want = tid + BT * j;
            while (b < want && k < h) {
                ++b;
                if (++l == h) {
                    ++k;
                    l = k;
                }
            }
            blk[j] = (want < h * (h + 1) / 2 && k < h) ? (k | (l << 8)) : -1;
        }
#pragma unroll
        for (int j = 0; j < NVR; ++j) {
            const int idx = tid + BT * j;
            vrk[j] = idx < m * h ? ((idx / h) | ((idx % h) << 8)) : -1;
        }
    }
    int sweeps = 0;
    bool converged = m < 2;
    while (!converged && sweeps < max_sweeps) {
        // a sweep is run only when some pair passes the rotation test
        if (tid == 0) sm.flag = 0;
        __syncthreads();
        for (int e = tid; e < m * m; e += BT) {
            const int p = e / m, q = e % m;
            if (p < q && fabs(A[p][q]) > floor && A[p][q] * A[p][q] > tol * tol * fabs(A[p][p] * A[q][q]))
                sm.flag = 1;
        }
        __syncthreads();
        if (sm.flag == 0) {
            converged = true;
            break;
        }
        __syncthreads();
        if (tid == 0) sm.flag = 0;
        __syncthreads();
        for (int round = 0; round < m - 1; ++round) {
            if (tid < h) {
                int p, q;
                if (tid == 0) {
                    p = 0;
                    q = 1 + round % (m - 1);
                } else {
                    p = 1 + (round + tid) % (m - 1);
                    q = 1 + (round + (m - 1) - tid) % (m - 1);
                }
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                double c = 1.0, s = 0.0, dp = A[p][p], dq = A[q][q];
                if (fabs(A[p][q]) > floor && schur2_rs(A[p][p], A[q][q], A[p][q], tol, c, s, dp, dq)) sm.flag = 1;
                sm.pp[tid] = p;
                sm.qq[tid] = q;
                sm.cs[tid] = c;
                sm.sn[tid] = s;
                sm.dpp[tid] = dp;
                sm.dqq[tid] = dq;
            }
            __syncthreads();
            // 2x2 blocks (k <= l) of the rotation pairs, mirrored
#pragma unroll
            for (int j = 0; j < NBK; ++j) {
                if (blk[j] < 0) continue;
                const int k = blk[j] & 255, l = blk[j] >> 8;
                const int p = sm.pp[k], q = sm.qq[k];
                const double c1 = sm.cs[k], s1 = sm.sn[k];
                if (k == l) {
                    if (s1 != 0.0) {
                        A[p][p] = sm.dpp[k];
                        A[q][q] = sm.dqq[k];
                        A[p][q] = 0.0;
                        A[q][p] = 0.0;
                    }
                    continue;
                }
                const int p2 = sm.pp[l], q2 = sm.qq[l];
                const double c2 = sm.cs[l], s2 = sm.sn[l];
                if (s1 == 0.0 && s2 == 0.0) continue;
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
#pragma unroll
            for (int j = 0; j < NVR; ++j) {
                if (vrk[j] < 0) continue;
                const int i = vrk[j] & 255, k = vrk[j] >> 8;
                const double s1 = sm.sn[k];
                if (s1 == 0.0) continue;
                const double c1 = sm.cs[k];
                const int p = sm.pp[k], q = sm.qq[k];
                const double x = Vm[i][p], y = Vm[i][q];
                Vm[i][p] = c1 * x - s1 * y;
                Vm[i][q] = s1 * x + c1 * y;
            }
            __syncthreads();
        }
        ++sweeps;
        converged = sm.flag == 0;
        __syncthreads();
    }
    // descending order, equal values by index
    for (int i = tid; i < n; i += BT) {
        const double li = A[i][i];
        int r = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = A[j][j];
            r += (lj > li) || (lj == li && j < i);
        }
        sm.lam[r] = li;
        sm.col_of[r] = i;
    }
    __syncthreads();
    return converged;
}

// ---- mode product Z = U^T x_k Y, U = sign * V[:, col_of[:r]] --------------
template <int P, int LAYOUT, int BK>
__device__ void blk_ttm(const float* __restrict__ Y, int n, int64_t L, int64_t R, int r, float* __restrict__ Z,
                        BatchSmem<BK>& sm) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    constexpr int CT = 64;  // columns per tile
    constexpr int E = CT * BK / BT;
    int64_t ctiles, tpl = 1;
    int planes = 1;
    if (LAYOUT == LAYOUT_KC) {
        tpl = ceil_div(R, CT);
        ctiles = L * tpl;
    } else if (LAYOUT == LAYOUT_NC) {
        ctiles = ceil_div(L, CT);
    } else {
        planes = CT / (int)R;
        ctiles = ceil_div(L, planes);
    }
    auto colmap = [&](int64_t ct, int cc, int64_t& l, int64_t& rr) -> bool {
        if (LAYOUT == LAYOUT_KC) {
            l = ct / tpl;
            rr = (ct - l * tpl) * CT + cc;
            return rr < R;
        } else if (LAYOUT == LAYOUT_NC) {
            l = ct * CT + cc;
            rr = 0;
            return l < L;
        } else {
            const int Ri = (int)R;
            const int p = cc / Ri;
            l = ct * planes + p;
            rr = cc % Ri;
            return p < planes && l < L;
        }
    };
    // (column tile, slab) steps in one sequence, the next step's loads in
    // flight while the current slab is multiplied
    const int nks = (n + BK - 1) / BK;
    const int64_t total = ctiles * nks;
    auto slot = [&](int e, int& cc, int& kk) {
        if (LAYOUT == LAYOUT_NC) {
            kk = tid % BK;
            cc = tid / BK + (BT / BK) * e;
        } else {
            cc = tid % CT;
            kk = tid / CT + (BT / CT) * e;
        }
    };
    float vreg[E];
    auto load = [&](int64_t step) {
        const int64_t ct = step / nks;
        const int i0 = (int)(step - ct * nks) * BK;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            int cc, kk;
            slot(e, cc, kk);
            int64_t l, rr;
            const bool ok = colmap(ct, cc, l, rr) && i0 + kk < n;
            vreg[e] = ok ? Y[(l * n + i0 + kk) * R + rr] : 0.f;
        }
    };
    if (total > 0) load(0);
    f32x4 acc[2][2];
    for (int64_t step = 0; step < total; ++step) {
        const int64_t ct = step / nks;
        const int i0 = (int)(step - ct * nks) * BK;
        if (i0 == 0) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0, 0, 0, 0};
        }
        {
            __syncthreads();
#pragma unroll
            for (int e = 0; e < E; ++e) {
                int cc, kk;
                slot(e, cc, kk);
                const float v = vreg[e];
                if (P == PREC_BF16X3) {
                    const __bf16 hh = (__bf16)v;
                    sm.u.t.b.yh[cc][kk] = hh;
                    sm.u.t.b.yl[cc][kk] = (__bf16)(v - (float)hh);
                } else {
                    sm.u.t.yf[cc][kk] = v;
                }
            }
            __syncthreads();
            if (step + 1 < total) load(step + 1);
            if (P == PREC_BF16X3) {
#pragma unroll
                for (int k0 = 0; k0 < BK; k0 += 32) {
                    const int kq = k0 + 8 * (lane >> 4);
                    bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        // A operand: rows j of U^T, 8 consecutive i from the FP64 eigenvectors
                        const int j = wr + a * 16 + (lane & 15);
                        const bool jok = j < r;
                        const int col = jok ? sm.col_of[j] : 0;
                        const double sg = jok ? (double)sm.sgn[j] : 0.0;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const int i = i0 + kq + e;
                            const float f = (jok && i < n) ? (float)(sg * sm.u.e.V[i][col]) : 0.f;
                            const __bf16 hh = (__bf16)f;
                            ah[a][e] = hh;
                            al[a][e] = (__bf16)(f - (float)hh);
                        }
                        bh[a] = *reinterpret_cast<const bf16x8*>(&sm.u.t.b.yh[wc + a * 16 + (lane & 15)][kq]);
                        bl[a] = *reinterpret_cast<const bf16x8*>(&sm.u.t.b.yl[wc + a * 16 + (lane & 15)][kq]);
                    }
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 2; ++b) {
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
                        }
                }
            } else {
#pragma unroll
                for (int k4 = 0; k4 < BK; k4 += 4) {
                    const int kk = k4 + (lane >> 4);
                    float av[2], bv[2];
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        const int j = wr + a * 16 + (lane & 15);
                        const int i = i0 + kk;
                        av[a] = (j < r && i < n) ? (float)(sm.sgn[j] * sm.u.e.V[i][sm.col_of[j]]) : 0.f;
                        bv[a] = sm.u.t.yf[wc + a * 16 + (lane & 15)][kk];
                    }
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 2; ++b)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
                }
            }
        }
        if (i0 + BK >= n) {
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int cc = wc + b * 16 + (lane & 15);
                int64_t l, rr;
                if (!colmap(ct, cc, l, rr)) continue;
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int j = wr + a * 16 + mfma16_row<PREC_F32>(lane, v);
                        if (j < r) Z[(l * r + j) * R + rr] = acc[a][b][v];
                    }
            }
        }
    }
    __syncthreads();
}

template <int P, int BK>
__global__ __launch_bounds__(BT) void k_sthosvd_batched(const BlockDesc* __restrict__ descs,
                                                        const int32_t* __restrict__ order, int nblocks,
                                                        const float* __restrict__ arena, float* __restrict__ core,
                                                        float* __restrict__ fac, atc_block_result* __restrict__ res,
                                                        float* __restrict__ scratch, int64_t scratch_elems,
                                                        int* __restrict__ counter, double eps2, double rtmss,
                                                        int rule, int max_sweeps) {
    __shared__ BatchSmem<BK> sm;
    const int tid = threadIdx.x;
    float* my_scratch = scratch + (int64_t)blockIdx.x * scratch_elems;
    for (;;) {
        if (tid == 0) sm.next = atomicAdd(counter, 1);
        __syncthreads();
        const int item = sm.next;
        __syncthreads();
        if (item >= nblocks) break;  // every wave of the workgroup leaves together
        const int b = order[item];
        const BlockDesc d = descs[b];
        int64_t cur[3] = {d.dims[0], d.dims[1], d.dims[2]};
        int ord[3] = {0, 1, 2};
        // Section 4.1.1: increasing mode length, stable
        for (int i = 1; i < 3; ++i)
            for (int j = i; j > 0 && cur[ord[j]] < cur[ord[j - 1]]; --j) {
                const int t = ord[j];
                ord[j] = ord[j - 1];
                ord[j - 1] = t;
            }
        const float* src = arena + d.in_off;
        float* core_slot = core + d.core_off;
        double norm2 = 0.0, S = 0.0, used = 0.0;
        double tails[3] = {0, 0, 0};
        int ranks[3] = {(int)cur[0], (int)cur[1], (int)cur[2]};
        int status = 0;
        bool in_scratch = false;
        for (int i = 0; i < 3; ++i) {
            const int k = ord[i];
            const int n = (int)cur[k];
            const int64_t L = (k > 0 ? cur[0] : 1) * (k > 1 ? cur[1] : 1);
            const int64_t R = (k < 2 ? cur[2] : 1) * (k < 1 ? cur[1] : 1);
            // Gram matrices FP64-accumulated in both precisions: the
            // contractions of these blocks are short (at most 4096 terms), and
            // the rounding of an FP32- or bf16x3-accumulated Gram matrix of a
            // short contraction lands in the small trailing eigenvalues (its
            // negative part is clamped away), which biases the discarded-energy
            // sums by a sizeable part of a mode budget at eps = 1e-3
            if (R >= BK) blk_gram<PREC_F64ACC, LAYOUT_KC, BK>(src, n, L, R, sm);
            else if (R == 1) blk_gram<PREC_F64ACC, LAYOUT_NC, BK>(src, n, L, R, sm);
            else blk_gram<PREC_F64ACC, LAYOUT_SR, BK>(src, n, L, R, sm);
            // trace (fixed order) and budget
            if (tid == 0) {
                double tr = 0.0;
                for (int a = 0; a < n; ++a) tr += sm.u.e.A[a][a];
                sm.red[0] = tr;
            }
            __syncthreads();
            const double tr = sm.red[0];
            if (i == 0) {
                norm2 = tr;
                S = rtmss * eps2 * tr;
                if (!isfinite(tr)) status = ATC_ERR_NONFINITE_INPUT;
            }
            const bool conv = blk_jacobi<BK>(n, max_sweeps, sm);
            if (!conv) status = ATC_ERR_NOT_CONVERGED;
            if (tid == 0) {
                const double bud = (rule == ATC_RANK_EQUAL) ? S / 3.0 : (S - used) / (3 - i);
                double acc = 0.0, best_tail = 0.0;
                int best = n;
                for (int j = n - 1; j >= 0; --j) {
                    if (acc <= bud) {
                        best = j + 1;
                        best_tail = acc;
                    }
                    acc += sm.lam[j];
                }
                sm.rank = best;
                sm.red[1] = best_tail;
            }
            __syncthreads();
            const int r = sm.rank;
            used += sm.red[1];
            tails[k] = sm.red[1];
            ranks[k] = r;
            // sign rule, then the factor into its slot (row-major n x r)
            for (int j = tid; j < r; j += BT) {
                const int col = sm.col_of[j];
                double best = -1.0, val = 0.0;
                for (int a = 0; a < n; ++a) {
                    const double v = sm.u.e.V[a][col];
                    if (fabs(v) > best) {
                        best = fabs(v);
                        val = v;
                    }
                }
                sm.sgn[j] = val < 0.0 ? -1 : 1;
            }
            __syncthreads();
            float* fk = fac + d.fac_off;
            for (int j = 0; j < k; ++j) fk += (int64_t)d.dims[j] * d.dims[j];
            for (int idx = tid; idx < n * r; idx += BT) {
                const int a = idx / r, j = idx % r;
                fk[idx] = (float)(sm.sgn[j] * sm.u.e.V[a][sm.col_of[j]]);
            }
            // projection: ping-pong between the scratch block and the core slot
            float* dst = in_scratch ? core_slot : my_scratch;
            if (R >= 32) blk_ttm<P, LAYOUT_KC, BK>(src, n, L, R, r, dst, sm);
            else if (R == 1) blk_ttm<P, LAYOUT_NC, BK>(src, n, L, R, r, dst, sm);
            else blk_ttm<P, LAYOUT_SR, BK>(src, n, L, R, r, dst, sm);
            cur[k] = r;
            src = dst;
            in_scratch = !in_scratch;
        }
        // the core ends in the scratch block after an odd number of modes
        if (in_scratch) {
            const int64_t cnt = cur[0] * cur[1] * cur[2];
            __threadfence_block();
            __syncthreads();
            for (int64_t idx = tid; idx < cnt; idx += BT) core_slot[idx] = my_scratch[idx];
        }
        if (tid == 0) {
            atc_block_result o;
            o.ranks[0] = ranks[0];
            o.ranks[1] = ranks[1];
            o.ranks[2] = ranks[2];
            o.status = status;
            o.norm2 = norm2;
            o.sse_pred = used;
            o.tail[0] = tails[0];
            o.tail[1] = tails[1];
            o.tail[2] = tails[2];
            res[b] = o;
        }
        __syncthreads();
    }
}

__global__ void k_zero_counter(int* c) {
    if (threadIdx.x == 0) *c = 0;
}

}  // namespace
}  // namespace atc

// ------------------------------------------------------------------ host side
using namespace atc;

struct atc_batch_plan {
    int64_t nblocks;
    int prec;
    double eps2, rtmss;
    int rule, max_sweeps;
    std::vector<int32_t> dims;      // nblocks x 3
    std::vector<int64_t> in_off, core_off, fac_off;
    int64_t in_elems, core_elems, fac_elems;
    int64_t scratch_elems;          // per workgroup
    BlockDesc* d_desc;
    int32_t* d_order;
    int cus;
    int choice;                     // autotuned candidate
};

struct atc_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {


struct Candidate {
    int bk;
    int wg_per_cu;
};
const Candidate kCandidates[] = {{32, 1}, {32, 2}, {64, 1}, {64, 2}};
constexpr int kNumCandidates = 4;
constexpr int kDefaultCandidate = 1;

int max_grid(const atc_batch_plan* p) { return p->cus * 2; }

size_t batch_ws_bytes(const atc_batch_plan* p) {
    return 256 + (size_t)max_grid(p) * (size_t)p->scratch_elems * sizeof(float);
}

template <int P, int BK>
hipError_t launch_batched_t(const atc_batch_plan* p, int grid, const float* arena, float* core, float* fac,
                            atc_block_result* res, void* ws, hipStream_t st) {
    int* counter = reinterpret_cast<int*>(ws);
    float* scratch = reinterpret_cast<float*>(reinterpret_cast<char*>(ws) + 256);
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, st, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sthosvd_batched<P, BK>), dim3(grid), dim3(BT), 0, st, p->d_desc, p->d_order,
                       (int)p->nblocks, arena, core, fac, res, scratch, p->scratch_elems, counter, p->eps2, p->rtmss,
                       p->rule, p->max_sweeps);
    return hipGetLastError();
}

hipError_t launch_batched(const atc_batch_plan* p, int cand, const float* arena, float* core, float* fac,
                          atc_block_result* res, void* ws, hipStream_t st) {
    const Candidate c = kCandidates[cand];
    const int grid = (int)std::min<int64_t>(p->nblocks, (int64_t)p->cus * c.wg_per_cu);
    if (grid < 1) return hipSuccess;
    if (p->prec == PREC_BF16X3)
        return c.bk == 32 ? launch_batched_t<PREC_BF16X3, 32>(p, grid, arena, core, fac, res, ws, st)
                          : launch_batched_t<PREC_BF16X3, 64>(p, grid, arena, core, fac, res, ws, st);
    return c.bk == 32 ? launch_batched_t<PREC_F32, 32>(p, grid, arena, core, fac, res, ws, st)
                      : launch_batched_t<PREC_F32, 64>(p, grid, arena, core, fac, res, ws, st);
}

atc_status bfail(atc_status s, const char* msg) {
    set_last_error(msg);  // read back through atc_last_error()
    return s;
}

std::string tune_key(const atc_batch_plan* p) {
    // architecture, precision and the histogram of block sizes
    int hist[65] = {0};
    for (int64_t b = 0; b < p->nblocks; ++b)
        for (int k = 0; k < 3; ++k) hist[p->dims[3 * b + k]]++;
    std::ostringstream os;
    os << "gfx950|prec" << p->prec << "|n" << p->nblocks << "|";
    for (int i = 1; i <= 64; ++i)
        if (hist[i]) os << i << ":" << hist[i] << ",";
    return os.str();
}

}  // namespace

extern "C" {

atc_status atc_batch_plan_create(const int32_t* dims, const int64_t* input_offsets, int64_t nblocks,
                                 const atc_sthosvd_opts* opts, atc_batch_plan** plan) {
    if (!plan) return bfail(ATC_ERR_INVALID_ARGUMENT, "plan is NULL");
    *plan = nullptr;
    if (!dims || nblocks < 1 || !opts) return bfail(ATC_ERR_INVALID_ARGUMENT, "dims, nblocks and opts required");
    if (!(opts->rel_error >= 0.0) || !(opts->rtmss >= 0.0 && opts->rtmss <= 1.0))
        return bfail(ATC_ERR_INVALID_ARGUMENT, "bad rel_error or rtmss");
    if (opts->precision != ATC_PREC_NATIVE && opts->precision != ATC_PREC_BF16X3)
        return bfail(ATC_ERR_INVALID_ARGUMENT, "unknown precision");
    if (opts->rank_rule != ATC_RANK_ADAPTIVE && opts->rank_rule != ATC_RANK_EQUAL)
        return bfail(ATC_ERR_INVALID_ARGUMENT, "unknown rank rule");
    if (opts->has_order || opts->has_fixed_ranks)
        return bfail(ATC_ERR_UNSUPPORTED, "batched blocks use the default order and the budget rule");
    for (int64_t i = 0; i < 3 * nblocks; ++i)
        if (dims[i] < 1 || dims[i] > BMAX) return bfail(ATC_ERR_UNSUPPORTED, "block modes must lie in [1, 64]");
    if (input_offsets)
        for (int64_t b = 0; b < nblocks; ++b)
            if (input_offsets[b] < 0) return bfail(ATC_ERR_INVALID_ARGUMENT, "negative input offset");
    atc_batch_plan* p = new (std::nothrow) atc_batch_plan();
    if (!p) return bfail(ATC_ERR_INTERNAL, "out of host memory");
    p->nblocks = nblocks;
    p->prec = opts->precision == ATC_PREC_BF16X3 ? PREC_BF16X3 : PREC_F32;
    p->eps2 = opts->rel_error * opts->rel_error;
    p->rtmss = opts->rtmss;
    p->rule = opts->rank_rule;
    p->max_sweeps = opts->max_sweeps > 0 ? opts->max_sweeps : 60;
    p->dims.assign(dims, dims + 3 * nblocks);
    p->in_off.resize(nblocks);
    p->core_off.resize(nblocks);
    p->fac_off.resize(nblocks);
    std::vector<BlockDesc> desc(nblocks);
    int64_t io = 0, co = 0, fo = 0, maxsize = 1, in_end = 0;
    for (int64_t b = 0; b < nblocks; ++b) {
        const int64_t n0 = dims[3 * b], n1 = dims[3 * b + 1], n2 = dims[3 * b + 2];
        const int64_t sz = n0 * n1 * n2;
        const int64_t ib = input_offsets ? input_offsets[b] : io;  // caller's placement, else back to back
        p->in_off[b] = ib;
        p->core_off[b] = co;
        p->fac_off[b] = fo;
        desc[b].in_off = ib;
        desc[b].core_off = co;
        desc[b].fac_off = fo;
        desc[b].dims[0] = (int32_t)n0;
        desc[b].dims[1] = (int32_t)n1;
        desc[b].dims[2] = (int32_t)n2;
        desc[b].pad = 0;
        io += sz;
        co += sz;
        fo += n0 * n0 + n1 * n1 + n2 * n2;
        maxsize = std::max(maxsize, sz);
        in_end = std::max(in_end, ib + sz);
    }
    p->in_elems = in_end;
    p->core_elems = co;
    p->fac_elems = fo;
    p->scratch_elems = (maxsize + 63) / 64 * 64;
    // longest processing time first
    std::vector<int32_t> ord(nblocks);
    for (int64_t b = 0; b < nblocks; ++b) ord[b] = (int32_t)b;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        const int64_t sa = (int64_t)dims[3 * a] * dims[3 * a + 1] * dims[3 * a + 2];
        const int64_t sb = (int64_t)dims[3 * b] * dims[3 * b + 1] * dims[3 * b + 2];
        return sa > sb;
    });
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete p;
        return bfail(ATC_ERR_DEVICE, "no HIP device");
    }
    p->cus = prop.multiProcessorCount;
    p->choice = kDefaultCandidate;
    if (hipMalloc(&p->d_desc, sizeof(BlockDesc) * nblocks) != hipSuccess ||
        hipMalloc(&p->d_order, sizeof(int32_t) * nblocks) != hipSuccess) {
        delete p;
        return bfail(ATC_ERR_DEVICE, "plan tables: hipMalloc failed");
    }
    if (hipMemcpy(p->d_desc, desc.data(), sizeof(BlockDesc) * nblocks, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_order, ord.data(), sizeof(int32_t) * nblocks, hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(p->d_desc);
        hipFree(p->d_order);
        delete p;
        return bfail(ATC_ERR_DEVICE, "plan tables: upload failed");
    }
    *plan = p;
    return ATC_OK;
}

void atc_batch_plan_destroy(atc_batch_plan* plan) {
    if (!plan) return;
    hipFree(plan->d_desc);
    hipFree(plan->d_order);
    delete plan;
}

atc_status atc_batch_plan_info(const atc_batch_plan* plan, int64_t* input_elems, int64_t* core_elems,
                               int64_t* factor_elems, size_t* workspace_bytes) {
    if (!plan) return bfail(ATC_ERR_INVALID_ARGUMENT, "plan is NULL");
    if (input_elems) *input_elems = plan->in_elems;
    if (core_elems) *core_elems = plan->core_elems;
    if (factor_elems) *factor_elems = plan->fac_elems;
    if (workspace_bytes) *workspace_bytes = batch_ws_bytes(plan);
    return ATC_OK;
}

atc_status atc_batch_plan_offsets(const atc_batch_plan* plan, int64_t* input_off, int64_t* core_off,
                                  int64_t* factor_off) {
    if (!plan) return bfail(ATC_ERR_INVALID_ARGUMENT, "plan is NULL");
    const size_t bytes = sizeof(int64_t) * plan->nblocks;
    if (input_off) memcpy(input_off, plan->in_off.data(), bytes);
    if (core_off) memcpy(core_off, plan->core_off.data(), bytes);
    if (factor_off) memcpy(factor_off, plan->fac_off.data(), bytes);
    return ATC_OK;
}

atc_status atc_sthosvd_batched(atc_batch_plan* plan, const float* arena, float* core_arena, float* factor_arena,
                               atc_block_result* results, void* workspace, size_t workspace_bytes, void* stream) {
    if (!plan || !arena || !core_arena || !factor_arena || !results || !workspace)
        return bfail(ATC_ERR_INVALID_ARGUMENT, "plan, arenas, results and workspace must be non-NULL");
    if (workspace_bytes < batch_ws_bytes(plan)) return bfail(ATC_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
    const hipError_t e = launch_batched(plan, plan->choice, arena, core_arena, factor_arena, results, workspace,
                                        (hipStream_t)stream);
    if (e != hipSuccess) return bfail(ATC_ERR_DEVICE, hipGetErrorString(e));
    return ATC_OK;
}

atc_status atc_batch_autotune(atc_batch_plan* plan, const float* arena, float* core_arena, float* factor_arena,
                              atc_block_result* results, void* workspace, size_t workspace_bytes, void* stream,
                              int32_t reps, const char* cache_path, int32_t* out_choice) {
    if (!plan || !arena || !core_arena || !factor_arena || !results || !workspace)
        return bfail(ATC_ERR_INVALID_ARGUMENT, "plan, arenas, results and workspace must be non-NULL");
    if (workspace_bytes < batch_ws_bytes(plan)) return bfail(ATC_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
    if (reps < 1) reps = 3;
    const std::string key = tune_key(plan);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            const std::string tag = "{\"key\": \"" + key + "\", \"choice\": ";
            if (line.compare(0, tag.size(), tag) == 0) {
                const int c = atoi(line.c_str() + tag.size());
                if (c >= 0 && c < kNumCandidates) {
                    plan->choice = c;
                    if (out_choice) *out_choice = c;
                    return ATC_OK;
                }
            }
        }
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return bfail(ATC_ERR_DEVICE, "hipEventCreate failed");
    double best = 1e300;
    int best_c = kDefaultCandidate;
    double times[kNumCandidates];
    for (int c = 0; c < kNumCandidates; ++c) {
        std::vector<float> t;
        for (int r = 0; r < reps + 1; ++r) {  // first run warms up
            hipEventRecord(a, st);
            if (launch_batched(plan, c, arena, core_arena, factor_arena, results, workspace, st) != hipSuccess) {
                hipEventDestroy(a);
                hipEventDestroy(b);
                return bfail(ATC_ERR_DEVICE, "candidate launch failed");
            }
            hipEventRecord(b, st);
            hipEventSynchronize(b);
            float ms = 0.f;
            hipEventElapsedTime(&ms, a, b);
            if (r > 0) t.push_back(ms);
        }
        std::sort(t.begin(), t.end());
        times[c] = t[t.size() / 2];
        if (times[c] < best) {  // ties keep the lower index
            best = times[c];
            best_c = c;
        }
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    plan->choice = best_c;
    if (out_choice) *out_choice = best_c;
    if (cache_path) {
        std::ofstream out(cache_path, std::ios::app);
        out << "{\"key\": \"" << key << "\", \"choice\": " << best_c << ", \"bk\": " << kCandidates[best_c].bk
            << ", \"wg_per_cu\": " << kCandidates[best_c].wg_per_cu << ", \"median_ms\": [";
        for (int c = 0; c < kNumCandidates; ++c) out << (c ? ", " : "") << times[c];
        out << "]}\n";
    }
    return ATC_OK;
}

atc_status atc_batch_graph_create(atc_batch_plan* plan, const float* arena, float* core_arena, float* factor_arena,
                                  atc_block_result* results, void* workspace, size_t workspace_bytes, void* stream,
                                  atc_graph** graph) {
    if (!graph) return bfail(ATC_ERR_INVALID_ARGUMENT, "graph is NULL");
    *graph = nullptr;
    if (!plan || !arena || !core_arena || !factor_arena || !results || !workspace)
        return bfail(ATC_ERR_INVALID_ARGUMENT, "plan, arenas, results and workspace must be non-NULL");
    if (workspace_bytes < batch_ws_bytes(plan)) return bfail(ATC_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    if (st == nullptr) return bfail(ATC_ERR_INVALID_ARGUMENT, "graph capture needs a non-default stream");
    atc_graph* g = new (std::nothrow) atc_graph();
    if (!g) return bfail(ATC_ERR_INTERNAL, "out of host memory");
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        delete g;
        return bfail(ATC_ERR_DEVICE, "hipStreamBeginCapture failed");
    }
    const hipError_t le = launch_batched(plan, plan->choice, arena, core_arena, factor_arena, results, workspace, st);
    const hipError_t ce = hipStreamEndCapture(st, &g->graph);
    if (le != hipSuccess || ce != hipSuccess) {
        if (ce == hipSuccess) hipGraphDestroy(g->graph);
        delete g;
        return bfail(ATC_ERR_DEVICE, "graph capture failed");
    }
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
        hipGraphDestroy(g->graph);
        delete g;
        return bfail(ATC_ERR_DEVICE, "hipGraphInstantiate failed");
    }
    *graph = g;
    return ATC_OK;
}

atc_status atc_graph_launch(atc_graph* graph, void* stream) {
    if (!graph) return bfail(ATC_ERR_INVALID_ARGUMENT, "graph is NULL");
    if (hipGraphLaunch(graph->exec, (hipStream_t)stream) != hipSuccess)
        return bfail(ATC_ERR_DEVICE, "hipGraphLaunch failed");
    return ATC_OK;
}

void atc_graph_destroy(atc_graph* graph) {
    if (!graph) return;
    hipGraphExecDestroy(graph->exec);
    hipGraphDestroy(graph->graph);
    delete graph;
}

}  // extern "C"
