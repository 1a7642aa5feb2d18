// Jacobi rotations and the slot-order Jacobi eigensolver (32 x 32, 64 x 64), shared by
// the single-matrix eigensolvers (atc_eig.hip) and the batched kernel
// (atc_batched.hip).  The eigenvalues of the symmetric Gram matrix are those
// of Algorithm 1 (Section 3.2); Jacobi is one way to reach them in FP64.
#pragma once

#include "atc_internal.hpp"

namespace atc {

// Whether the pair (p, q) is rotated: |a_pq| > tol sqrt(|a_pp a_qq|) (the
// relative test of schur2, squared) and |a_pq| > floor.
__device__ __forceinline__ bool rot2_needed(double app, double aqq, double apq, double tol2, double floor2) {
    const double a2 = apq * apq;
    return a2 > tol2 * fabs(app * aqq) && a2 > floor2;
}

// Jacobi rotation for the pair (p, q) as in schur2, with fewer long-latency
// operations: with d = a_qq - a_pp, g = 2 a_pq, h = hypot(d, g), u = (1 + |d|
// / h) / 2: c = sqrt(u), s = sign(d) g / (2 h c), t = s / c (the smaller
// angle).  Pairs that fail rot2_needed keep (c, s) = (1, 0).
__device__ inline bool rot2(double app, double aqq, double apq, double tol2, double floor2, double& c, double& s,
                            double& dp, double& dq) {
    c = 1.0;
    s = 0.0;
    dp = app;
    dq = aqq;
    if (!rot2_needed(app, aqq, apq, tol2, floor2)) return false;
    const double d = aqq - app, g = 2.0 * apq;
    const double hh = d * d + g * g;
    if (!(hh >= 0x1p-1022) || !(hh < INFINITY)) return false;  // squares out of range: leave the pair
    const double rh = rsqrt_pos(hh);  // 1 / h
    const double u = 0.5 + 0.5 * fabs(d) * rh;   // cos^2 of the angle
    const double rc = rsqrt_pos(u);              // 1 / c
    c = u * rc;
    s = (d >= 0.0 ? 0.5 : -0.5) * g * rh * rc;
    const double t = s * rc;
    dp = app - t * apq;
    dq = aqq + t * apq;
    return true;
}

// ------------------------------------- M x M Jacobi (M = 32, 64), slot order
// Cyclic Jacobi for n <= M (zero-padded to M) with the pairs of the circle
// method: index 0 stays in slot 0, the other M - 1 indices move one step along
// a fixed cycle of slots after every round, and the pairs of a round are the
// slot pairs (2k, 2k + 1).  A is kept in slot order, so every lane reads its
// 2 x 2 blocks at fixed offsets and writes the rotated block to the slots its
// rows and columns move to (the fixed permutation j64_sigma); after M - 1
// rounds every index is back in its own slot.  A round reads one buffer and writes
// the other (every upper-triangle entry is written once), so a round needs
// one workgroup barrier.  The block wavefronts (3 for M = 64, 2 for M = 32)
// each compute all M / 2 rotations of a round (lane k and its copies take
// pair k) and rotate their share of the off-diagonal blocks (3 of 496 per
// lane for M = 64, 1 of 120 for M = 32) into their new slots; wavefront 0
// writes the diagonal blocks (new diagonal, zero coupling).  Wavefront 3
// holds the eigenvector matrix in registers, lane i its row i in slot order,
// so a rotation and the move to the next slots use only compile-time
// register indices; it applies a round's rotations (double-buffered in LDS)
// while the other wavefronts compute the next round.  A sweep starts with
// the test of all pairs; none passing ends the iteration.  Only the upper
// triangle of A (in slot order) is read or written.
constexpr int J64_LD = 65;    // row stride of the buffers (doubles)
constexpr int J64_ROWS = 69;  // unused block slots write rows M.. (64-68 for M = 64, 32 for M = 32)
constexpr int J64_THREADS = 256;

// slot of cycle position j, cycle position of slot s != 0, next slot of s
template <int M>
__host__ __device__ constexpr int j64_cyc(int j) { return j < M / 2 - 1 ? 2 * (j + 1) : 2 * (M - 2 - j) + 1; }
template <int M>
__host__ __device__ constexpr int j64_pos(int s) { return (s & 1) ? M - 2 - (s >> 1) : (s >> 1) - 1; }
template <int M>
__host__ __device__ constexpr int j64_sigma(int s) { return s == 0 ? 0 : j64_cyc<M>((j64_pos<M>(s) + 1) % (M - 1)); }
__device__ __forceinline__ unsigned j64_up(int x, int y) {
    return (unsigned)((x < y ? x * J64_LD + y : y * J64_LD + x) * (int)sizeof(double));
}

struct J64Shared {
    double2 xch[3][32];   // the round's rotations, one copy per block wavefront
    double2 rlog[2][32];  // the same for the eigenvector wavefront, by round parity
    double diag[64];      // the eigenvalues on return, by index
    int need_s[3];
};

// Called by every thread of a workgroup of J64_THREADS threads, n <= M.  A0, A1: J64_ROWS
// x J64_LD doubles each; on entry A0 holds the symmetric n x n matrix (upper
// triangle read; entries of the leading M x M outside n x n are cleared
// here).  On return sh.diag[i] is the eigenvalue of index i, Wout (J64_LD
// stride, rows 0..63 written, may alias A0 or A1) row r column i the r-th
// component of its eigenvector; A0 and A1 are overwritten.  Entries at or
// below floor_rel |trace| are left alone.
template <int M>
__device__ __forceinline__ bool jacobi_slots(int n, int max_sweeps, double floor_rel, double (*A0)[J64_LD],
                                             double (*A1)[J64_LD], J64Shared& sh, double (*Wout)[J64_LD],
                                             int& sweeps_out) {
    static_assert(M == 32 || M == 64, "slot-order Jacobi sizes");
    constexpr int H = M / 2, NR = M - 1, NOFF = H * (H - 1) / 2;
    constexpr int BW = M == 64 ? 3 : 2;    // block wavefronts
    constexpr int SPL = M == 64 ? 3 : 1;   // block slots per lane
    constexpr int NSLOT = 64 * BW * SPL;   // 576 for 496 blocks, 128 for 120
    constexpr int UNR = M == 64 ? 7 : 31;  // eigenvector rounds per loop body (divides NR)
    static_assert(NSLOT >= NOFF && 4 * (NSLOT - NOFF) <= (J64_ROWS - M) * J64_LD, "unused slots fit the spare rows");
    static_assert(NR % UNR == 0 && H % 8 == 0, "loop shapes");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < M * M; e += J64_THREADS) {
        const int i = e / M, j = e % M;
        if (i >= n || j >= n) A0[i][j] = 0.0;
    }
    __syncthreads();
    const double tol = (double)n * 0x1p-53;
    const double tol2 = tol * tol;
    double trace = 0.0;
    for (int i = 0; i < n; ++i) trace += A0[i][i];
    const double floor = floor_rel * fabs(trace);
    const double floor2 = floor * floor;
    char* const base[2] = {reinterpret_cast<char*>(&A0[0][0]), reinterpret_cast<char*>(&A1[0][0])};
    int cur = 0;  // the buffer that holds A
    // block wavefronts: slots b = 64 wave + lane + 64 BW t; b < NOFF is block (k, l), k < l, in
    // row-major order of the strict upper triangle, the rest read and write the spare rows
    unsigned ld[SPL][4], st[SPL][4];
    int kt[SPL], lt[SPL];
#pragma unroll
    for (int t = 0; t < SPL; ++t) {
        int b = 64 * (wave < BW ? wave : 0) + lane + 64 * BW * t;
        if (b < NOFF) {
            int k = 0;
            while (b >= H - 1 - k) {
                b -= H - 1 - k;
                ++k;
            }
            const int l = k + 1 + b;
            kt[t] = k;
            lt[t] = l;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = 2 * k + (e >> 1), y = 2 * l + (e & 1);
                ld[t][e] = j64_up(x, y);
                st[t][e] = j64_up(j64_sigma<M>(x), j64_sigma<M>(y));
            }
        } else {
            kt[t] = 0;
            lt[t] = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const unsigned spare = (unsigned)(M * J64_LD + 4 * (b - NOFF) + e) * (unsigned)sizeof(double);
                ld[t][e] = spare;
                st[t][e] = spare;
            }
        }
    }
    const int kp = lane & (H - 1);
    const unsigned o_pp = j64_up(2 * kp, 2 * kp), o_qq = j64_up(2 * kp + 1, 2 * kp + 1), o_pq = j64_up(2 * kp, 2 * kp + 1);
    const int sp = j64_sigma<M>(2 * kp), sq = j64_sigma<M>(2 * kp + 1);
    const unsigned s_pp = j64_up(sp, sp), s_qq = j64_up(sq, sq), s_pq = j64_up(sp, sq);
    int sweeps = 0;
    bool conv = false;
    // after a sweep's test: the same decision in every wavefront (true: stop)
    auto decide = [&]() -> bool {
        __syncthreads();
        bool need = false;
#pragma unroll
        for (int v = 0; v < BW; ++v) need = need || sh.need_s[v] != 0;
        if (!need) conv = true;
        return !need || sweeps >= max_sweeps;
    };
    // Each role runs its own sweep loop (the same barriers in the same order),
    // so the eigenvector registers are not live in the block wavefronts' loop.
    if (wave < BW) {
        while (true) {
            // at a sweep's start every index is in its own slot
            const double(*A)[J64_LD] = reinterpret_cast<const double(*)[J64_LD]>(base[cur]);
            bool need = false;
            for (int e = 64 * wave + lane; e < M * M; e += 64 * BW) {
                const int p = e / M, q = e % M;
                need = need || (p < q && rot2_needed(A[p][p], A[q][q], A[p][q], tol2, floor2));
            }
            const bool any = __ballot(need) != 0;
            if (lane == 0) sh.need_s[wave] = any ? 1 : 0;
            if (decide()) break;
            for (int round = 0; round < NR; ++round) {
                char* const src = base[cur];
                char* const dst = base[cur ^ 1];
                auto at = [&](unsigned off) -> double& { return *reinterpret_cast<double*>(src + off); };
                auto to = [&](unsigned off) -> double& { return *reinterpret_cast<double*>(dst + off); };
                const double app = at(o_pp), aqq = at(o_qq), apq = at(o_pq);
                double x[SPL][4];
#pragma unroll
                for (int t = 0; t < SPL; ++t)
#pragma unroll
                    for (int e = 0; e < 4; ++e) x[t][e] = at(ld[t][e]);
                double c, s, dp, dq;
                const bool rr = rot2(app, aqq, apq, tol2, floor2, c, s, dp, dq);
                if (lane < H) {
                    sh.xch[wave][lane] = double2{c, s};
                    if (wave == 0) sh.rlog[round & 1][lane] = double2{c, s};
                }
                // no wait: a wavefront's LDS accesses complete in issue order
                double y[SPL][4];
#pragma unroll
                for (int t = 0; t < SPL; ++t) {
                    const double2 ck = sh.xch[wave][kt[t]], cl = sh.xch[wave][lt[t]];
                    const double c1 = ck.x, s1 = ck.y, c2 = cl.x, s2 = cl.y;
                    const double ra = c1 * x[t][0] - s1 * x[t][2], rb = c1 * x[t][1] - s1 * x[t][3];
                    const double rc = s1 * x[t][0] + c1 * x[t][2], rd = s1 * x[t][1] + c1 * x[t][3];
                    y[t][0] = c2 * ra - s2 * rb;
                    y[t][1] = s2 * ra + c2 * rb;
                    y[t][2] = c2 * rc - s2 * rd;
                    y[t][3] = s2 * rc + c2 * rd;
                }
#pragma unroll
                for (int t = 0; t < SPL; ++t)
#pragma unroll
                    for (int e = 0; e < 4; ++e) to(st[t][e]) = y[t][e];
                if (wave == 0 && lane < H) {
                    to(s_pp) = dp;
                    to(s_qq) = dq;
                    to(s_pq) = rr ? 0.0 : apq;
                }
                __syncthreads();  // the next buffer is complete; this one is free
                cur ^= 1;
            }
            ++sweeps;
        }
        // every index back in its own slot: the diagonal, before the
        // eigenvectors are stored (Wout may alias either buffer)
        if (tid < M) sh.diag[tid] = reinterpret_cast<const double*>(base[cur])[tid * (J64_LD + 1)];
        __syncthreads();
        __syncthreads();
    } else if (wave == 3) {
        // row `lane` of W in slot order (slot = index at a sweep's start); for
        // M = 32 lanes 32-63 carry zero rows
        double w[M];
#pragma unroll
        for (int j = 0; j < M; ++j) w[j] = (j == lane) ? 1.0 : 0.0;
        while (true) {
            if (decide()) break;
            // unrolled by UNR rounds (7 of 63, all 31): the register moves that bring
            // the permuted columns back to the loop's registers come once per body
            for (int r7 = 0; r7 < NR; r7 += UNR) {
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int round = r7 + u;
                    // this round's rotations: written before the round's barrier, rewritten
                    // two rounds later, after this wavefront has passed the next barrier
                    __syncthreads();
                    const double2* lg = sh.rlog[round & 1];
                    double2 ca[8], cb[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        ca[j] = lg[j];
                        cb[j] = lg[8 + j];
                    }
                    double wn[M];
                    auto rotate8 = [&](const double2(&cs)[8], int kb) {
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            const int k = kb + j;
                            const double xv = w[2 * k], yv = w[2 * k + 1];
                            wn[j64_sigma<M>(2 * k)] = cs[j].x * xv - cs[j].y * yv;
                            wn[j64_sigma<M>(2 * k + 1)] = cs[j].y * xv + cs[j].x * yv;
                        }
                    };
                    rotate8(ca, 0);
                    if constexpr (H == 32) {
#pragma unroll
                        for (int j = 0; j < 8; ++j) ca[j] = lg[16 + j];
                        rotate8(cb, 8);
#pragma unroll
                        for (int j = 0; j < 8; ++j) cb[j] = lg[24 + j];
                        rotate8(ca, 16);
                        rotate8(cb, 24);
                    } else {
                        rotate8(cb, 8);
                    }
#pragma unroll
                    for (int j = 0; j < M; ++j) w[j] = wn[j];
                }
            }
            ++sweeps;
        }
        __syncthreads();  // the diagonal is saved: both buffers are free
#pragma unroll
        for (int j = 0; j < M; ++j) Wout[lane][j] = w[j];
        __syncthreads();
    } else {
        // idle wavefront (M = 32): the same barriers
        while (true) {
            if (decide()) break;
            for (int round = 0; round < NR; ++round) __syncthreads();
            ++sweeps;
        }
        __syncthreads();
        __syncthreads();
    }
    sweeps_out = sweeps;
    return conv;
}

__device__ __forceinline__ bool jacobi64_slots(int n, int max_sweeps, double floor_rel, double (*A0)[J64_LD],
                                               double (*A1)[J64_LD], J64Shared& sh, double (*Wout)[J64_LD],
                                               int& sweeps_out) {
    return jacobi_slots<64>(n, max_sweeps, floor_rel, A0, A1, sh, Wout, sweeps_out);
}

}  // namespace atc
