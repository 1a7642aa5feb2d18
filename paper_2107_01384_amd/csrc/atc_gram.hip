// Gram matrix (SYRK) and cross-Gram kernels on MFMA.
//
// For the mode-k step of Algorithm 1 (Section 3.2) the left singular vectors of
// the unfolding B_(k) are the eigenvectors of G = B_(k) B_(k)^T.  The current
// tensor is read in place through its (L, n, R) view (Section 3.1: fiber order
// inside the unfolding does not change G), so no transpose is ever made:
//   G[a, b] = sum_{l, r} X[l, a, r] * Y[l, b, r]         (Y == X for G)
//
// One workgroup (4 waves) owns a 64 x 64 output tile and a contiguous range
// of K steps (split-K).  Each step stages a 64 x BK slab of both operands in
// LDS; each wave computes a 32 x 32 quarter with 16 x 16 MFMA blocks.
//   PREC_F64   : v_mfma_f64_16x16x4f64, FP64 accumulation.
//   PREC_F64ACC: float32 input widened to FP64 in LDS, then as PREC_F64
//                (every product exact, FP64 accumulation).
//   PREC_F32   : v_mfma_f32_16x16x4f32, FP32 accumulation flushed into FP64
//                registers every FLUSH_TERMS contracted terms.
//   PREC_BF16X3: operands split on load into bf16 hi + lo; products
//                hi*hi + hi*lo + lo*hi (and lo*lo on diagonal tiles, so the
//                diagonal, whose dropped lo*lo would always be positive, is
//                unbiased) with v_mfma_f32_16x16x32_bf16, flushed to FP64
//                like PREC_F32.
// Each workgroup writes its FP64 partial tile; a second kernel sums the splits
// in a fixed order, so the result is bit-reproducible.
#include "atc_internal.hpp"

#include <type_traits>

namespace atc {
namespace {

__device__ inline void decode_upper_pair(int pair, int tiles, int& ti, int& tj) {
    int p = pair, i = 0;
    while (p >= tiles - i) {
        p -= tiles - i;
        ++i;
    }
    ti = i;
    tj = i + p;
}

__host__ __device__ inline int upper_pair_index(int ti, int tj, int tiles) {
    return ti * tiles - ti * (ti - 1) / 2 + (tj - ti);
}

template <int P> struct GramSmem;
template <> struct GramSmem<PREC_F64> {
    double x[TILE][KDepth<PREC_F64>::value + 1];
    double y[TILE][KDepth<PREC_F64>::value + 1];
};
template <> struct GramSmem<PREC_F64ACC> : GramSmem<PREC_F64> {};
template <> struct GramSmem<PREC_F32> {
    float x[TILE][KDepth<PREC_F32>::value + 1];
    float y[TILE][KDepth<PREC_F32>::value + 1];
};
template <> struct GramSmem<PREC_BF16X3> {
    // row stride 40 bf16 = 80 bytes keeps every 8-element read 16-byte aligned
    __bf16 xh[TILE][KDepth<PREC_BF16X3>::value + 8];
    __bf16 xl[TILE][KDepth<PREC_BF16X3>::value + 8];
    __bf16 yh[TILE][KDepth<PREC_BF16X3>::value + 8];
    __bf16 yl[TILE][KDepth<PREC_BF16X3>::value + 8];
};

// Element slot of the per-step operand slab owned by this thread.
struct Slot {
    int row;   // row inside the 64-row tile
    int kk;    // column inside the step (contracted index)
    int p, r;  // SR: plane and r of the slot
    bool ok;   // slot maps into the slab
};

template <int LAYOUT, int BK>
__device__ inline Slot make_slot(int tid, int e, int64_t R, int planes) {
    Slot s;
    s.p = 0;
    s.r = 0;
    s.ok = true;
    if (LAYOUT == LAYOUT_KC) {
        s.row = tid / BK + (NTHREADS / BK) * e;
        s.kk = tid % BK;
    } else if (LAYOUT == LAYOUT_NC) {
        s.row = tid % TILE;
        s.kk = tid / TILE + (NTHREADS / TILE) * e;
    } else {
        const int Ri = (int)R;
        const int q = tid + NTHREADS * e;
        s.r = q % Ri;
        s.row = (q / Ri) % TILE;
        s.p = q / (TILE * Ri);
        s.ok = s.p < planes;
        s.kk = s.p * Ri + s.r;
    }
    return s;
}

// Global offset of slot `s` at step `step` for rows of an (L, nrows, R) view,
// or -1 if the element lies outside the tensor.
template <int LAYOUT, int BK>
__device__ inline int64_t slot_offset(const Slot& s, int64_t step, int64_t spl, int rowg, int nrows,
                                      int64_t L, int64_t R, int planes) {
    if (!s.ok || rowg >= nrows) return -1;
    if (LAYOUT == LAYOUT_KC) {
        const int64_t l = step / spl;
        const int64_t r0 = (step - l * spl) * BK;
        if (r0 + s.kk >= R) return -1;
        return (l * nrows + rowg) * R + r0 + s.kk;
    } else if (LAYOUT == LAYOUT_NC) {
        const int64_t k = step * BK + s.kk;
        if (k >= L) return -1;
        return k * nrows + rowg;
    } else {
        const int64_t l = step * planes + s.p;
        if (l >= L) return -1;
        return (l * nrows + rowg) * R + s.r;
    }
}

template <int P, int LAYOUT, bool SYM>
__global__ __launch_bounds__(NTHREADS) void k_gram(const typename ElemOf<P>::T* __restrict__ X,
                                                   const typename ElemOf<P>::T* __restrict__ Y, int nx,
                                                   int ny, int64_t L, int64_t R, int64_t steps, int nsplit,
                                                   int tiles_x, int tiles_y, int npairs, int planes,
                                                   double* __restrict__ part) {
    using T = typename ElemOf<P>::T;                                   // input element
    using S = typename std::conditional<prec_f64_mfma(P), double, T>::type;  // LDS / MFMA operand
    constexpr int BK = KDepth<P>::value;
    constexpr int E = TILE * BK / NTHREADS;
    __shared__ GramSmem<P> sm;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int pair = blockIdx.x;
    const int split = blockIdx.y;
    int ti, tj;
    if (SYM) {
        decode_upper_pair(pair, tiles_x, ti, tj);
    } else {
        ti = pair / tiles_y;
        tj = pair % tiles_y;
    }
    const bool diag = SYM && ti == tj;
    const int row0 = ti * TILE, col0 = tj * TILE;
    const int64_t s0 = steps * split / nsplit;
    const int64_t s1 = steps * (split + 1) / nsplit;
    const int64_t spl = ceil_div(R, BK);

    Slot sl[E];
#pragma unroll
    for (int e = 0; e < E; ++e) sl[e] = make_slot<LAYOUT, BK>(tid, e, R, planes);

    if (LAYOUT == LAYOUT_SR) {
        // columns no slot writes stay zero for the whole kernel
        for (int idx = tid; idx < TILE * BK; idx += NTHREADS) {
            const int rr = idx / BK, kk = idx % BK;
            if constexpr (P == PREC_BF16X3) {
                sm.xh[rr][kk] = (__bf16)0.0f; sm.xl[rr][kk] = (__bf16)0.0f;
                sm.yh[rr][kk] = (__bf16)0.0f; sm.yl[rr][kk] = (__bf16)0.0f;
            } else {
                sm.x[rr][kk] = (S)0; sm.y[rr][kk] = (S)0;
            }
        }
    }

    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    f64x4 acc64[2][2];
    f32x4 acc32[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            acc64[a][b] = f64x4{0, 0, 0, 0};
            acc32[a][b] = f32x4{0, 0, 0, 0};
        }
    constexpr int FLUSH_STEPS = FLUSH_TERMS / BK;
    int since_flush = 0;

    for (int64_t s = s0; s < s1; ++s) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const Slot& q = sl[e];
            const int64_t ox = slot_offset<LAYOUT, BK>(q, s, spl, row0 + q.row, nx, L, R, planes);
            const T vx = ox >= 0 ? X[ox] : (T)0;
            T vy = (T)0;
            if (!diag) {
                const int64_t oy = slot_offset<LAYOUT, BK>(q, s, spl, col0 + q.row, ny, L, R, planes);
                vy = oy >= 0 ? Y[oy] : (T)0;
            }
            if (q.ok) {
                if constexpr (P == PREC_BF16X3) {
                    const __bf16 xh = (__bf16)vx;
                    sm.xh[q.row][q.kk] = xh;
                    sm.xl[q.row][q.kk] = (__bf16)(vx - (float)xh);
                    if (!diag) {
                        const __bf16 yh = (__bf16)vy;
                        sm.yh[q.row][q.kk] = yh;
                        sm.yl[q.row][q.kk] = (__bf16)(vy - (float)yh);
                    }
                } else {
                    sm.x[q.row][q.kk] = (S)vx;
                    if (!diag) sm.y[q.row][q.kk] = (S)vy;
                }
            }
        }
        __syncthreads();

        if constexpr (P == PREC_BF16X3) {
            const int kq = 8 * (lane >> 4);
            bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int rr = wr + a * 16 + (lane & 15);
                ah[a] = *reinterpret_cast<const bf16x8*>(&sm.xh[rr][kq]);
                al[a] = *reinterpret_cast<const bf16x8*>(&sm.xl[rr][kq]);
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int cc = wc + b * 16 + (lane & 15);
                if (diag) {
                    bh[b] = *reinterpret_cast<const bf16x8*>(&sm.xh[cc][kq]);
                    bl[b] = *reinterpret_cast<const bf16x8*>(&sm.xl[cc][kq]);
                } else {
                    bh[b] = *reinterpret_cast<const bf16x8*>(&sm.yh[cc][kq]);
                    bl[b] = *reinterpret_cast<const bf16x8*>(&sm.yl[cc][kq]);
                }
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc32[a][b], 0, 0, 0);
                    acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc32[a][b], 0, 0, 0);
                    acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc32[a][b], 0, 0, 0);
                    if (diag)
                        acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bl[b], acc32[a][b], 0, 0, 0);
                }
        } else {
#pragma unroll
            for (int k4 = 0; k4 < BK; k4 += 4) {
                const int kk = k4 + (lane >> 4);
                S av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) av[a] = sm.x[wr + a * 16 + (lane & 15)][kk];
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    bv[b] = diag ? sm.x[wc + b * 16 + (lane & 15)][kk] : sm.y[wc + b * 16 + (lane & 15)][kk];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        if constexpr (prec_f64_mfma(P))
                            acc64[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc64[a][b], 0, 0, 0);
                        else
                            acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc32[a][b], 0, 0, 0);
                    }
            }
        }
        if constexpr (!prec_f64_mfma(P)) {
            if (++since_flush == FLUSH_STEPS) {
                since_flush = 0;
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc64[a][b][v] += (double)acc32[a][b][v];
                        acc32[a][b] = f32x4{0, 0, 0, 0};
                    }
            }
        }
    }
    if constexpr (!prec_f64_mfma(P)) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc64[a][b][v] += (double)acc32[a][b][v];
    }
    // 16x16 MFMA result layout: column lane%16, row mfma16_row(lane, v)
    double* out = part + ((int64_t)split * npairs + pair) * (TILE * TILE);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = wr + a * 16 + mfma16_row<P>(lane, v);
                const int j = wc + b * 16 + (lane & 15);
                out[i * TILE + j] = acc64[a][b][v];
            }
}

// Sum of the split partials: a workgroup takes 64 consecutive outputs
// (row-major over nx x ny) and four groups of splits (group q: splits q, q +
// 4, ..., four loads in flight each), whose sums are added in group order.
constexpr int RED_OUT = 64;
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ part, int nsplit, int npairs,
                                                     int tiles_x, int tiles_y, int nx, int ny, int sym,
                                                     double* __restrict__ C) {
    __shared__ double red[4][RED_OUT];
    const int o = threadIdx.x & (RED_OUT - 1), q = threadIdx.x / RED_OUT;
    const int64_t idx = (int64_t)blockIdx.x * RED_OUT + o;
    const bool ok = idx < (int64_t)nx * ny;
    const int a = ok ? (int)(idx / ny) : 0, b = ok ? (int)(idx % ny) : 0;
    const bool want = ok && !(sym && a > b);
    double s = 0.0;
    if (want) {
        const int ti = a / TILE, tj = b / TILE;
        const int pair = sym ? upper_pair_index(ti, tj, tiles_x) : ti * tiles_y + tj;
        const double* p = part + (int64_t)pair * (TILE * TILE) + (a % TILE) * TILE + (b % TILE);
        const int64_t stride = (int64_t)npairs * TILE * TILE;
        int sp = q;
        for (; sp + 12 < nsplit; sp += 16) {
            const double v0 = p[sp * stride], v1 = p[(sp + 4) * stride], v2 = p[(sp + 8) * stride],
                         v3 = p[(sp + 12) * stride];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; sp < nsplit; sp += 4) s += p[sp * stride];
    }
    red[q][o] = s;
    __syncthreads();
    if (q == 0 && want) {
        const double t = ((red[0][o] + red[1][o]) + red[2][o]) + red[3][o];
        C[(int64_t)a * ny + b] = t;
        if (sym) C[(int64_t)b * ny + a] = t;
    }
}

template <int P, int LAYOUT, bool SYM>
hipError_t launch_gram_t(const GramPlan& g, const void* X, const void* Y, double* part, hipStream_t st) {
    using T = typename ElemOf<P>::T;
    dim3 grid(g.npairs, g.nsplit);
    hipLaunchKernelGGL((k_gram<P, LAYOUT, SYM>), grid, dim3(NTHREADS), 0, st, (const T*)X, (const T*)Y, g.nx,
                       g.ny, g.L, g.R, g.steps, g.nsplit, g.tiles_x, g.tiles_y, g.npairs, g.planes, part);
    return hipGetLastError();
}

template <int P, bool SYM>
hipError_t launch_gram_l(const GramPlan& g, const void* X, const void* Y, double* part, hipStream_t st) {
    switch (g.layout) {
        case LAYOUT_KC: return launch_gram_t<P, LAYOUT_KC, SYM>(g, X, Y, part, st);
        case LAYOUT_NC: return launch_gram_t<P, LAYOUT_NC, SYM>(g, X, Y, part, st);
        default: return launch_gram_t<P, LAYOUT_SR, SYM>(g, X, Y, part, st);
    }
}

template <int P>
hipError_t launch_gram_p(const GramPlan& g, const void* X, const void* Y, double* part, hipStream_t st) {
    return g.sym ? launch_gram_l<P, true>(g, X, Y, part, st) : launch_gram_l<P, false>(g, X, Y, part, st);
}

}  // namespace

GramPlan gram_plan(int prec, int64_t L, int nx, int ny, int64_t R, bool sym, size_t part_capacity_bytes) {
    GramPlan g{};
    const int BK = prec_f64_mfma(prec) ? KDepth<PREC_F64>::value : KDepth<PREC_F32>::value;
    g.L = L;
    g.R = R;
    g.nx = nx;
    g.ny = ny;
    g.sym = sym ? 1 : 0;
    g.planes = 1;
    if (R >= BK) {
        g.layout = LAYOUT_KC;
        g.steps = L * ceil_div(R, BK);
    } else if (R == 1) {
        g.layout = LAYOUT_NC;
        g.steps = ceil_div(L, BK);
    } else {
        g.layout = LAYOUT_SR;
        g.planes = BK / (int)R;
        g.steps = ceil_div(L, g.planes);
    }
    g.tiles_x = (int)ceil_div(nx, TILE);
    g.tiles_y = (int)ceil_div(ny, TILE);
    g.npairs = sym ? g.tiles_x * (g.tiles_x + 1) / 2 : g.tiles_x * g.tiles_y;
    // enough workgroups to cover 256 CUs several times, at least 8 steps each
    // (2 for short products, whose time is one memory latency per step, and
    // for products of a few tile pairs, which need the splits to fill the chip)
    int64_t want = ceil_div(2048, g.npairs);
    const int64_t min_steps = (g.steps < 64 || g.npairs <= 4) ? 2 : 8;
    int64_t max_by_steps = g.steps / min_steps > 0 ? g.steps / min_steps : 1;
    int64_t max_by_mem = (int64_t)(part_capacity_bytes / ((size_t)g.npairs * TILE * TILE * sizeof(double)));
    int64_t ns = want;
    if (ns > max_by_steps) ns = max_by_steps;
    if (ns > max_by_mem) ns = max_by_mem;
    if (ns > 65535) ns = 65535;
    if (ns < 1) ns = 1;
    g.nsplit = (int)ns;
    g.part_capacity = part_capacity_bytes;
    g.part_bytes = (size_t)g.nsplit * g.npairs * TILE * TILE * sizeof(double);
    return g;
}

hipError_t launch_gram(int prec, const GramPlan& g, const void* X, const void* Y, double* part, hipStream_t st) {
    if (g.part_bytes > g.part_capacity) return hipErrorInvalidValue;  // partials would not fit
    switch (prec) {
        case PREC_F64: return launch_gram_p<PREC_F64>(g, X, Y, part, st);
        case PREC_F32: return launch_gram_p<PREC_F32>(g, X, Y, part, st);
        case PREC_F64ACC: return launch_gram_p<PREC_F64ACC>(g, X, Y, part, st);
        default: return launch_gram_p<PREC_BF16X3>(g, X, Y, part, st);
    }
}

hipError_t launch_gram_reduce(const GramPlan& g, const double* part, double* C, hipStream_t st) {
    const int64_t total = (int64_t)g.nx * g.ny;
    const int64_t blocks = ceil_div(total, (int64_t)RED_OUT);
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)blocks), dim3(256), 0, st, part, g.nsplit, g.npairs,
                       g.tiles_x, g.tiles_y, g.nx, g.ny, g.sym, C);
    return hipGetLastError();
}


// ------------------------------------------------------------ tall and narrow
// Gram matrix of an (L, n, 1) view with n <= 16: L rows of n floats back to
// back (the last mode of a row-major tensor when it is short, e.g. the 13
// variables of a 4-way field).  The generic tiles would be almost all padding
// here; instead each workgroup streams a contiguous range of rows through LDS
// (chunks of TALL_ROWS rows, float4 loads of the contiguous floats) and every
// wave runs v_mfma_f64_16x16x4f64 over 4 rows per instruction: lane l feeds
// X[row + l / 16][l % 16] (0 beyond n) as both operands (A = X^T, B = X).
// FP32 products are exact in FP64 and accumulate in FP64, so this mode's Gram
// matrix (and |A|^2 when it is processed first) carries no rounding bias.
// Each workgroup writes its n x n partial; k_gram_tall_reduce adds them in
// workgroup order.
constexpr int TALL_ROWS = 256;

namespace {

__global__ __launch_bounds__(256) void k_gram_tall(const float* __restrict__ X, int n, int64_t L,
                                                   int64_t rows_per_wg, double* __restrict__ part) {
    __shared__ float4 buf4[TALL_ROWS * 16 / 4];
    __shared__ double red[4][16][17];
    float* const buf = reinterpret_cast<float*>(buf4);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t r1 = r0 + rows_per_wg < L ? r0 + rows_per_wg : L;
    const int col = lane & 15, rsub = lane >> 4;
    const int colc = col < n ? col : n - 1;
    // four independent accumulators (rows 4 wave + 16 u + 64 m, u = 0..3)
    // keep several MFMAs in flight; the workgroups resident on a CU overlap
    // one another's loads.  No branches around loads: masked lanes read a
    // clamped address and select zero.
    f64x4 acc0 = f64x4{0.0, 0.0, 0.0, 0.0}, acc1 = acc0, acc2 = acc0, acc3 = acc0;
    for (int64_t c0 = r0; c0 < r1; c0 += TALL_ROWS) {
        const int cnt = (int)(r1 - c0 < TALL_ROWS ? r1 - c0 : TALL_ROWS);
        const int nf = cnt * n, nf4 = nf >> 2;
        const float4* src4 = reinterpret_cast<const float4*>(X + c0 * n);  // c0 % 4 == 0: 16-byte aligned
        for (int e = tid; e < nf4; e += 256) buf4[e] = src4[e];
        const int et = (nf4 << 2) + tid;
        if (et < nf) buf[et] = X[c0 * n + et];
        __syncthreads();
        for (int q = 4 * wave; q < cnt; q += 64) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int row = q + 16 * u + rsub;
                const float raw = buf[(row < cnt ? row : cnt - 1) * n + colc];
                v[u] = (row < cnt && col < n) ? (double)raw : 0.0;
            }
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(v[0], v[0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(v[1], v[1], acc1, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(v[2], v[2], acc2, 0, 0, 0);
            acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(v[3], v[3], acc3, 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
        red[wave][mfma16_row<PREC_F64>(lane, e)][col] = ((acc0[e] + acc1[e]) + acc2[e]) + acc3[e];
    __syncthreads();
    for (int e = tid; e < n * n; e += 256) {
        const int i = e / n, j = e % n;
        part[(int64_t)blockIdx.x * n * n + e] = ((red[0][i][j] + red[1][i][j]) + red[2][i][j]) + red[3][i][j];
    }
}

// G[e] = sum of the nblocks partials of entry e: one workgroup per entry, each
// thread a strided subset, then a fixed-order tree in LDS.
__global__ __launch_bounds__(256) void k_gram_tall_reduce(const double* __restrict__ part, int nblocks, int n,
                                                          double* __restrict__ G) {
    __shared__ double sred[256];
    const int e = blockIdx.x, tid = threadIdx.x;
    const int nn = n * n;
    double s = 0.0;
    for (int b = tid; b < nblocks; b += 256) s += part[(int64_t)b * nn + e];
    sred[tid] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) sred[tid] += sred[tid + w];
        __syncthreads();
    }
    if (tid == 0) G[e] = sred[0];
}

}  // namespace

bool gram_tall_applicable(int prec, int n, int64_t R) { return prec != PREC_F64 && R == 1 && n >= 1 && n <= 16; }

int gram_tall_blocks(int64_t L) {
    const int64_t want = 1536;  // six workgroups per CU
    return (int)(L < want * TALL_ROWS / 8 ? ceil_div(L, (int64_t)TALL_ROWS / 8) : want);
}

hipError_t launch_gram_tall(const float* X, int n, int64_t L, double* part, size_t part_capacity_bytes, double* G,
                            hipStream_t st) {
    if (n < 1 || n > 16 || L < 1) return hipErrorInvalidValue;
    if (reinterpret_cast<uintptr_t>(X) % 16 != 0) return hipErrorInvalidValue;
    const int nb = gram_tall_blocks(L);
    int64_t per = ceil_div(L, (int64_t)nb);
    per = ceil_div(per, (int64_t)4) * 4;  // chunk starts stay 16-byte aligned
    const int blocks = (int)ceil_div(L, per);
    if ((size_t)blocks * n * n * sizeof(double) > part_capacity_bytes) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gram_tall, dim3(blocks), dim3(256), 0, st, X, n, L, per, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_tall_reduce, dim3((unsigned)(n * n)), dim3(256), 0, st, (const double*)part, blocks, n,
                       G);
    return hipGetLastError();
}

}  // namespace atc
