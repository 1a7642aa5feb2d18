// Mode product (TTM) kernels on MFMA.
//
// Z = M x_k Y (Section 3.1: Z_(k) = M Y_(k)) on the in-place (L, n, R) view:
//   Z[l, j, r] = sum_i M[j, i] * Y[l, i, r]
// With M = U_k^T this is the projection step of Algorithm 1 (Section 3.2):
// mode k shrinks from n_k to r_k while every other mode stays where it is, so
// the tensor keeps its natural mode order and needs no transposition.  With
// M = U_k it expands a mode (reconstruction, Section 3.2 Tucker format).
//
// Treated as the matrix product (m_out x n) * (n x cols) with cols = L*R
// columns (l, r).  A workgroup owns 64 output rows j and 64 columns; it steps
// through the contracted index i in slabs of BK, staging M (64 x BK) and a
// (BK x 64) slab of Y in LDS (Y stored column-major so each lane reads its
// MFMA operand contiguously).  The kernel reads the tensor exactly once and
// is bound by HBM bandwidth for small m_out.
#include "atc_internal.hpp"

namespace atc {
namespace {

template <int P> struct TtmSmem;
template <> struct TtmSmem<PREC_F64> {
    double m[TILE][KDepth<PREC_F64>::value + 1];
    double y[TILE][KDepth<PREC_F64>::value + 1];  // [column][i]
};
template <> struct TtmSmem<PREC_F32> {
    float m[TILE][KDepth<PREC_F32>::value + 1];
    float y[TILE][KDepth<PREC_F32>::value + 1];
};
template <> struct TtmSmem<PREC_BF16X3> {
    __bf16 mh[TILE][KDepth<PREC_BF16X3>::value + 8];
    __bf16 ml[TILE][KDepth<PREC_BF16X3>::value + 8];
    __bf16 yh[TILE][KDepth<PREC_BF16X3>::value + 8];
    __bf16 yl[TILE][KDepth<PREC_BF16X3>::value + 8];
};

// Column cc of column tile `ct`: returns the (L, ., R) base offset parts.
struct ColMap {
    int64_t l;   // slice index
    int64_t r;   // position along R
    bool ok;
};

template <int LAYOUT>
__device__ inline ColMap col_map(int64_t ct, int cc, int64_t L, int64_t R, int64_t tpl, int planes) {
    ColMap c;
    if (LAYOUT == LAYOUT_KC) {
        c.l = ct / tpl;
        c.r = (ct - c.l * tpl) * TILE + cc;
        c.ok = c.r < R;
    } else if (LAYOUT == LAYOUT_NC) {
        c.l = ct * TILE + cc;
        c.r = 0;
        c.ok = c.l < L;
    } else {
        const int Ri = (int)R;
        const int p = cc / Ri;
        c.l = ct * planes + p;
        c.r = cc % Ri;
        c.ok = p < planes && c.l < L;
    }
    return c;
}

template <int P, int LAYOUT>
__global__ __launch_bounds__(NTHREADS) void k_ttm(const typename ElemOf<P>::T* __restrict__ Y, int64_t L, int n,
                                                  int64_t R, int m_out, int64_t tpl, int planes,
                                                  const double* __restrict__ M64, const float* __restrict__ M32,
                                                  const __bf16* __restrict__ Mh, const __bf16* __restrict__ Ml,
                                                  typename ElemOf<P>::T* __restrict__ Z) {
    using T = typename ElemOf<P>::T;
    constexpr int BK = KDepth<P>::value;
    constexpr int E = TILE * BK / NTHREADS;
    __shared__ TtmSmem<P> sm;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t ct = blockIdx.x;
    const int j0 = blockIdx.y * TILE;

    // Y slab slots: columns fastest when columns are contiguous (KC, SR),
    // contracted index fastest when it is (NC).
    int ycol[E], yk[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (LAYOUT == LAYOUT_NC) {
            yk[e] = tid % BK;
            ycol[e] = tid / BK + (NTHREADS / BK) * e;
        } else {
            ycol[e] = tid % TILE;
            yk[e] = tid / TILE + (NTHREADS / TILE) * e;
        }
    }
    ColMap cm[E];
#pragma unroll
    for (int e = 0; e < E; ++e) cm[e] = col_map<LAYOUT>(ct, ycol[e], L, R, tpl, planes);
    // M slab slots: contracted index fastest (M is row-major m_out x n)
    int mrow[E], mk[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        mk[e] = tid % BK;
        mrow[e] = tid / BK + (NTHREADS / BK) * e;
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

    for (int i0 = 0; i0 < n; i0 += BK) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = i0 + yk[e];
            T v = (T)0;
            if (cm[e].ok && i < n) v = Y[(cm[e].l * n + i) * R + cm[e].r];
            if constexpr (P == PREC_BF16X3) {
                const __bf16 h = (__bf16)v;
                sm.yh[ycol[e]][yk[e]] = h;
                sm.yl[ycol[e]][yk[e]] = (__bf16)(v - (float)h);
            } else {
                sm.y[ycol[e]][yk[e]] = v;
            }
            const int j = j0 + mrow[e], im = i0 + mk[e];
            const bool mok = j < m_out && im < n;
            const int64_t mo = (int64_t)j * n + im;
            if constexpr (P == PREC_BF16X3) {
                sm.mh[mrow[e]][mk[e]] = mok ? Mh[mo] : (__bf16)0.0f;
                sm.ml[mrow[e]][mk[e]] = mok ? Ml[mo] : (__bf16)0.0f;
            } else if constexpr (P == PREC_F64) {
                sm.m[mrow[e]][mk[e]] = mok ? M64[mo] : 0.0;
            } else {
                sm.m[mrow[e]][mk[e]] = mok ? M32[mo] : 0.0f;
            }
        }
        __syncthreads();
        if constexpr (P == PREC_BF16X3) {
            const int kq = 8 * (lane >> 4);
            bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                ah[a] = *reinterpret_cast<const bf16x8*>(&sm.mh[wr + a * 16 + (lane & 15)][kq]);
                al[a] = *reinterpret_cast<const bf16x8*>(&sm.ml[wr + a * 16 + (lane & 15)][kq]);
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                bh[b] = *reinterpret_cast<const bf16x8*>(&sm.yh[wc + b * 16 + (lane & 15)][kq]);
                bl[b] = *reinterpret_cast<const bf16x8*>(&sm.yl[wc + b * 16 + (lane & 15)][kq]);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc32[a][b], 0, 0, 0);
                    acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc32[a][b], 0, 0, 0);
                    acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc32[a][b], 0, 0, 0);
                }
        } else {
#pragma unroll
            for (int k4 = 0; k4 < BK; k4 += 4) {
                const int kk = k4 + (lane >> 4);
                T av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) av[a] = sm.m[wr + a * 16 + (lane & 15)][kk];
#pragma unroll
                for (int b = 0; b < 2; ++b) bv[b] = sm.y[wc + b * 16 + (lane & 15)][kk];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        if constexpr (P == PREC_F64)
                            acc64[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc64[a][b], 0, 0, 0);
                        else
                            acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc32[a][b], 0, 0, 0);
                    }
            }
        }
    }
    // write: column lane%16, row mfma16_row(lane, v) of each 16x16 block
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int cc = wc + b * 16 + (lane & 15);
        const ColMap c = col_map<LAYOUT>(ct, cc, L, R, tpl, planes);
        if (!c.ok) continue;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = j0 + wr + a * 16 + mfma16_row<P>(lane, v);
                if (j >= m_out) continue;
                const T val = (P == PREC_F64) ? (T)acc64[a][b][v] : (T)acc32[a][b][v];
                Z[(c.l * m_out + j) * R + c.r] = val;
            }
    }
}

template <int P, int LAYOUT>
hipError_t launch_ttm_t(const TtmPlan& t, const void* Y, const void* M, const void* Mh, const void* Ml, void* Z,
                        hipStream_t st) {
    using T = typename ElemOf<P>::T;
    dim3 grid((unsigned)t.ctiles, t.jtiles);
    hipLaunchKernelGGL((k_ttm<P, LAYOUT>), grid, dim3(NTHREADS), 0, st, (const T*)Y, t.L, t.n, t.R, t.m_out,
                       t.tiles_per_l, t.planes, (const double*)M, (const float*)M, (const __bf16*)Mh,
                       (const __bf16*)Ml, (T*)Z);
    return hipGetLastError();
}

template <int P>
hipError_t launch_ttm_p(const TtmPlan& t, const void* Y, const void* M, const void* Mh, const void* Ml, void* Z,
                        hipStream_t st) {
    switch (t.layout) {
        case LAYOUT_KC: return launch_ttm_t<P, LAYOUT_KC>(t, Y, M, Mh, Ml, Z, st);
        case LAYOUT_NC: return launch_ttm_t<P, LAYOUT_NC>(t, Y, M, Mh, Ml, Z, st);
        default: return launch_ttm_t<P, LAYOUT_SR>(t, Y, M, Mh, Ml, Z, st);
    }
}

}  // namespace

TtmPlan ttm_plan(int prec, int64_t L, int n, int64_t R, int m_out) {
    (void)prec;
    TtmPlan t{};
    t.L = L;
    t.R = R;
    t.n = n;
    t.m_out = m_out;
    t.planes = 1;
    t.tiles_per_l = 1;
    if (R >= 32) {
        t.layout = LAYOUT_KC;
        t.tiles_per_l = ceil_div(R, TILE);
        t.ctiles = L * t.tiles_per_l;
    } else if (R == 1) {
        t.layout = LAYOUT_NC;
        t.ctiles = ceil_div(L, TILE);
    } else {
        t.layout = LAYOUT_SR;
        t.planes = TILE / (int)R;
        t.ctiles = ceil_div(L, t.planes);
    }
    t.jtiles = (int)ceil_div(m_out, TILE);
    return t;
}

hipError_t launch_ttm(int prec, const TtmPlan& t, const void* Y, const void* M, const void* Mh, const void* Ml,
                      void* Z, hipStream_t st) {
    switch (prec) {
        case PREC_F64: return launch_ttm_p<PREC_F64>(t, Y, M, Mh, Ml, Z, st);
        case PREC_F32: return launch_ttm_p<PREC_F32>(t, Y, M, Mh, Ml, Z, st);
        default: return launch_ttm_p<PREC_BF16X3>(t, Y, M, Mh, Ml, Z, st);
    }
}

}  // namespace atc
