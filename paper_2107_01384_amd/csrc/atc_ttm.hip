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
#include <algorithm>
#include <type_traits>

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
                                                  typename ElemOf<P>::T* __restrict__ Z,
                                                  const int32_t* __restrict__ m_dev) {
    using T = typename ElemOf<P>::T;
    constexpr int BK = KDepth<P>::value;
    if (m_dev) m_out = min(m_out, *m_dev);  // the rank chosen on the device
    if (m_out < 1) return;
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

// Wide variant for the contiguous-R layout (R % 4 == 0) and small m_out (<=
// 16 MT): a workgroup owns 256 consecutive columns of one slice (R >= 256,
// pl = 1) or pl = 256 / R whole slices of R columns each (R < 256), and every
// output row, so the tensor is read once, in coalesced float4 rows.  The
// next 32-row slab of Y (and of M, split into bf16 hi/lo on the fly for the
// bf16x3 form) is loaded into registers while the current one is multiplied;
// Y is staged in LDS column-major, eight rows of a column per 16-byte store.
template <int P, int MT>
__global__ __launch_bounds__(NTHREADS) void k_ttm_wide(const float* __restrict__ Y, int64_t L, int n, int64_t R,
                                                       int m_out, int64_t tpl, int pl, const float* __restrict__ M32,
                                                       float* __restrict__ Z, const int32_t* __restrict__ m_dev,
                                                       int kchunk) {
    constexpr int W = 256, BK = 32, MR = 16 * MT;
    if (m_dev) m_out = min(m_out, *m_dev);  // the rank chosen on the device
    if (m_out < 1) return;
    // split K (gridDim.y > 1): slice blockIdx.y of K (kchunk terms, a multiple
    // of BK) into its own partial output, Z + blockIdx.y * L m_out R
    const int k_lo = (int)blockIdx.y * kchunk, k_hi = min(n, k_lo + kchunk);
    Z += (int64_t)blockIdx.y * L * m_out * R;
    constexpr int YP = (P == PREC_BF16X3) ? BK : BK + 4;  // row of a staged column
    // bf16 columns staged without padding (37 KB of LDS: four workgroups per
    // CU): the 16-byte chunk c of row r sits at c ^ ((r >> 1) ^ (r >> 3)) & 3,
    // so the 16 consecutive rows an MFMA operand load reads hit distinct banks
    struct SmB {
        __bf16 yh[W][BK], yl[W][BK], mh[MR][BK + 8], ml[MR][BK + 8];
    };
    struct SmF {
        float yf[W][BK + 4], mf[MR][BK + 4];
    };
    struct SmB6 {
        __bf16 yh[W][BK], ym[W][BK], yl[W][BK], mh[MR][BK + 8], mm[MR][BK + 8], ml[MR][BK + 8];
    };
    typedef typename std::conditional<
        P == PREC_BF16X3, SmB, typename std::conditional<P == PREC_BF16X6, SmB6, SmF>::type>::type Sm;
    __shared__ Sm sm;
    (void)YP;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t ct = blockIdx.x;
    // column c of the tile: slice l0 + c / R, position c0 + c % R (pl > 1: c0 = 0)
    const int64_t l0 = pl > 1 ? ct * pl : ct / tpl;
    const int64_t c0 = pl > 1 ? 0 : (ct - l0 * tpl) * W;
    const int cg = tid & 63, rg = tid >> 6;  // columns 4 cg .. + 3, slab rows 8 rg .. + 7
    const int pc = pl > 1 ? (4 * cg) / (int)R : 0;
    const int64_t rc = pl > 1 ? 4 * cg - (int64_t)pc * R : c0 + 4 * cg;
    const bool colok = pc < pl && l0 + pc < L && rc < R;
    const float* ybase = Y + (l0 + pc) * (int64_t)n * R + rc;
    float4 yv[8];
    float mv[MT][8];
    auto load = [&](int i0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int i = i0 + 8 * rg + e;
            yv[e] = (colok && i < k_hi) ? *reinterpret_cast<const float4*>(ybase + (int64_t)i * R)
                                        : float4{0.f, 0.f, 0.f, 0.f};
        }
        // M: MR rows x 32 k, eight consecutive k per (thread, row block)
#pragma unroll
        for (int q = 0; q < MT; ++q) {
            const int idx = tid + NTHREADS * q;  // < MR * 4 = 64 MT
            const int mr = idx >> 2, kq = (idx & 3) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int i = i0 + kq + e;
                mv[q][e] = (idx < MR * 4 && mr < m_out && i < k_hi) ? M32[(int64_t)mr * n + i] : 0.f;
            }
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float f[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) f[e] = q == 0 ? yv[e].x : q == 1 ? yv[e].y : q == 2 ? yv[e].z : yv[e].w;
            if constexpr (P == PREC_BF16X3) {
                bf16x8 hv, lv;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const __bf16 h = (__bf16)f[e];
                    hv[e] = h;
                    lv[e] = (__bf16)(f[e] - (float)h);
                }
                const int row = 4 * cg + q;
                const int ch = rg ^ (((row >> 1) ^ (row >> 3)) & 3);
                *reinterpret_cast<bf16x8*>(&sm.yh[row][8 * ch]) = hv;
                *reinterpret_cast<bf16x8*>(&sm.yl[row][8 * ch]) = lv;
            } else if constexpr (P == PREC_BF16X6) {
                bf16x8 hv, mv_, lv;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const __bf16 h = (__bf16)f[e];
                    const float r1 = f[e] - (float)h;
                    const __bf16 m = (__bf16)r1;
                    hv[e] = h;
                    mv_[e] = m;
                    lv[e] = (__bf16)(r1 - (float)m);
                }
                const int row = 4 * cg + q;
                const int ch = rg ^ (((row >> 1) ^ (row >> 3)) & 3);
                *reinterpret_cast<bf16x8*>(&sm.yh[row][8 * ch]) = hv;
                *reinterpret_cast<bf16x8*>(&sm.ym[row][8 * ch]) = mv_;
                *reinterpret_cast<bf16x8*>(&sm.yl[row][8 * ch]) = lv;
            } else {
                *reinterpret_cast<float4*>(&sm.yf[4 * cg + q][8 * rg]) = float4{f[0], f[1], f[2], f[3]};
                *reinterpret_cast<float4*>(&sm.yf[4 * cg + q][8 * rg + 4]) = float4{f[4], f[5], f[6], f[7]};
            }
        }
#pragma unroll
        for (int q = 0; q < MT; ++q) {
            const int idx = tid + NTHREADS * q;
            if (idx >= MR * 4) continue;
            const int mr = idx >> 2, kq = (idx & 3) * 8;
            if constexpr (P == PREC_BF16X3) {
                bf16x8 hv, lv;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const __bf16 h = (__bf16)mv[q][e];
                    hv[e] = h;
                    lv[e] = (__bf16)(mv[q][e] - (float)h);
                }
                *reinterpret_cast<bf16x8*>(&sm.mh[mr][kq]) = hv;
                *reinterpret_cast<bf16x8*>(&sm.ml[mr][kq]) = lv;
            } else if constexpr (P == PREC_BF16X6) {
                bf16x8 hv, mv_, lv;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const __bf16 h = (__bf16)mv[q][e];
                    const float r1 = mv[q][e] - (float)h;
                    const __bf16 m = (__bf16)r1;
                    hv[e] = h;
                    mv_[e] = m;
                    lv[e] = (__bf16)(r1 - (float)m);
                }
                *reinterpret_cast<bf16x8*>(&sm.mh[mr][kq]) = hv;
                *reinterpret_cast<bf16x8*>(&sm.mm[mr][kq]) = mv_;
                *reinterpret_cast<bf16x8*>(&sm.ml[mr][kq]) = lv;
            } else {
                *reinterpret_cast<float4*>(&sm.mf[mr][kq]) = float4{mv[q][0], mv[q][1], mv[q][2], mv[q][3]};
                *reinterpret_cast<float4*>(&sm.mf[mr][kq + 4]) = float4{mv[q][4], mv[q][5], mv[q][6], mv[q][7]};
            }
        }
    };
    const int wc = wave * 64;  // this wavefront's 64 columns
    f32x4 acc[MT][4];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    load(k_lo);
    for (int i0 = k_lo; i0 < k_hi; i0 += BK) {
        __syncthreads();
        stage();
        __syncthreads();
        if (i0 + BK < k_hi) load(i0 + BK);
        if constexpr (P == PREC_BF16X3) {
            const int kq = 8 * (lane >> 4);
            bf16x8 bh[4], bl[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int row = wc + 16 * b + (lane & 15);
                const int yq = 8 * ((lane >> 4) ^ (((row >> 1) ^ (row >> 3)) & 3));
                bh[b] = *reinterpret_cast<const bf16x8*>(&sm.yh[row][yq]);
                bl[b] = *reinterpret_cast<const bf16x8*>(&sm.yl[row][yq]);
            }
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&sm.mh[16 * a + (lane & 15)][kq]);
                const bf16x8 al = *reinterpret_cast<const bf16x8*>(&sm.ml[16 * a + (lane & 15)][kq]);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[b], acc[a][b], 0, 0, 0);
                }
            }
        } else if constexpr (P == PREC_BF16X6) {
            const int kq = 8 * (lane >> 4);
            bf16x8 bh[4], bm[4], bl[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int row = wc + 16 * b + (lane & 15);
                const int yq = 8 * ((lane >> 4) ^ (((row >> 1) ^ (row >> 3)) & 3));
                bh[b] = *reinterpret_cast<const bf16x8*>(&sm.yh[row][yq]);
                bm[b] = *reinterpret_cast<const bf16x8*>(&sm.ym[row][yq]);
                bl[b] = *reinterpret_cast<const bf16x8*>(&sm.yl[row][yq]);
            }
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                const int mrow = 16 * a + (lane & 15);
                const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&sm.mh[mrow][kq]);
                const bf16x8 am = *reinterpret_cast<const bf16x8*>(&sm.mm[mrow][kq]);
                const bf16x8 al = *reinterpret_cast<const bf16x8*>(&sm.ml[mrow][kq]);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    // the terms of order 2, then 1, then 0 (smallest first)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[b], acc[a][b], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int k4 = 0; k4 < BK; k4 += 4) {
                const int kk = k4 + (lane >> 4);
                float bv[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) bv[b] = sm.yf[wc + 16 * b + (lane & 15)][kk];
#pragma unroll
                for (int a = 0; a < MT; ++a) {
                    const float av = sm.mf[16 * a + (lane & 15)][kk];
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[b], acc[a][b], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int c = wc + 16 * b + (lane & 15);
        const int p = pl > 1 ? c / (int)R : 0;
        const int64_t r = pl > 1 ? c - (int64_t)p * R : c0 + c;
        if (p >= pl || l0 + p >= L || r >= R) continue;
        float* zbase = Z + (l0 + p) * (int64_t)m_out * R + r;
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = 16 * a + mfma16_row<PREC_F32>(lane, v);
                if (j < m_out) zbase[(int64_t)j * R] = acc[a][b][v];
            }
    }
}

// Mode product for a last, contiguous mode (R == 1) and m_out <= 32: Z[l][j] =
// sum_i Y[l][i] M[j][i] (M = U^T, m_out x n, FP32).  One workgroup per 16 rows
// l; wavefront w takes the w-th quarter of i in batches of 128 whose loads go
// out together (one memory latency per batch instead of one per 32 rows of a
// tile loop), v_mfma_f32_16x16x4f32 (FP32 products and sums), and the
// quarters are added in wavefront order through LDS.
__global__ __launch_bounds__(NTHREADS) void k_ttm_rows(const float* __restrict__ Y, int64_t L, int n, int m_out,
                                                       const float* __restrict__ M32, float* __restrict__ Z,
                                                       const int32_t* __restrict__ m_dev) {
    if (m_dev) m_out = min(m_out, *m_dev);  // the rank chosen on the device
    if (m_out < 1) return;
    constexpr int KB = 32;  // K steps of four per batch
    __shared__ float red[4][16][33];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t l0 = (int64_t)blockIdx.x * 16;
    const int c = lane & 15, kr = lane >> 4;
    const int chunk = ((n + 3) / 4 + 3) / 4 * 4;
    const int k0 = min(n, wave * chunk), k1 = min(n, k0 + chunk);
    const float* yrow = Y + min(l0 + c, L - 1) * (int64_t)n;
    const float* m0 = M32 + (int64_t)min(c, m_out - 1) * n;
    const float* m1 = M32 + (int64_t)min(16 + c, m_out - 1) * n;
    const float w0 = c < m_out ? 1.f : 0.f, w1 = 16 + c < m_out ? 1.f : 0.f;
    f32x4 acc0 = f32x4{0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
    for (int kb = k0; kb < k1; kb += 4 * KB) {
        float a[KB], b0[KB], b1[KB];
#pragma unroll
        for (int t = 0; t < KB; ++t) {
            const int k = kb + 4 * t + kr;
            const bool in = k < k1;
            const int kk = in ? k : k0;
            const float m = in ? 1.f : 0.f;
            a[t] = m * yrow[kk];
            b0[t] = w0 * m0[kk];
            b1[t] = w1 * m1[kk];
        }
#pragma unroll
        for (int t = 0; t < KB; ++t) {
            acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], b0[t], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], b1[t], acc1, 0, 0, 0);
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = mfma16_row<PREC_F32>(lane, e);
        red[wave][r][c] = acc0[e];
        red[wave][r][16 + c] = acc1[e];
    }
    __syncthreads();
    for (int e = tid; e < 16 * 32; e += NTHREADS) {
        const int r = e >> 5, j = e & 31;
        const float t = ((red[0][r][j] + red[1][r][j]) + red[2][r][j]) + red[3][r][j];
        if (l0 + r < L && j < m_out) Z[(l0 + r) * m_out + j] = t;
    }
}

// Expansion of a last, contiguous mode (R == 1) in FP32: Z[l][j] = sum_i
// Y[l][i] M[j][i] with n <= 4 KC contracted entries and m_out <= 16 JT
// outputs per row (m_out % 4 == 0), the reconstruction's final step.  A
// workgroup takes tiles of EXP_ROWS consecutive rows of Y (one contiguous
// block, coalesced loads) into LDS rows padded to an odd stride; each
// wavefront then forms 16 rows at a time as Z^T tiles on
// v_mfma_f32_16x16x4f32 (FP32 products and sums): A = M (16 outputs j x 4
// entries i, held in registers for the whole kernel), B = the rows' entries
// from LDS, so lane (c, q) ends with Z[l0 + c][16 t + 4 q .. 16 t + 4 q + 3]
// and writes it with one 16-byte store.
constexpr int EXP_ROWS = 256;

template <int KC, int JT>
__global__ __launch_bounds__(NTHREADS) void k_ttm_expand_last(const float* __restrict__ Y, int64_t L, int n,
                                                              int m_out, const float* __restrict__ M32,
                                                              float* __restrict__ Z) {
    constexpr int NS = 4 * KC + 1;
    __shared__ float ys[EXP_ROWS * NS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = lane & 15, q = lane >> 4;
    float a[JT][KC];
#pragma unroll
    for (int t = 0; t < JT; ++t)
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int j = 16 * t + c, i = 4 * k + q;
            a[t][k] = (j < m_out && i < n) ? M32[(int64_t)j * n + i] : 0.f;
        }
    const bool vec = (n & 3) == 0;
    for (int64_t tile = blockIdx.x; tile * EXP_ROWS < L; tile += gridDim.x) {
        const int64_t l0 = tile * EXP_ROWS;
        const int rows = (int)min<int64_t>(EXP_ROWS, L - l0);
        // rows' entries in groups of four (zeros past n), all loads issued first
        float v[KC][4];
#pragma unroll
        for (int x = 0; x < KC; ++x) {
            const int e = tid + x * NTHREADS;
            const int rr = e / KC, k4 = 4 * (e % KC);
            const float* src = Y + (l0 + min(rr, rows - 1)) * n + k4;
            if (vec && k4 < n) {
                const float4 w = rr < rows ? *reinterpret_cast<const float4*>(src) : float4{0.f, 0.f, 0.f, 0.f};
                v[x][0] = w.x;
                v[x][1] = w.y;
                v[x][2] = w.z;
                v[x][3] = w.w;
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) v[x][u] = (rr < rows && k4 + u < n) ? src[u] : 0.f;
            }
        }
#pragma unroll
        for (int x = 0; x < KC; ++x) {
            const int e = tid + x * NTHREADS;
            const int rr = e / KC, k4 = 4 * (e % KC);
            if (rr < rows)
#pragma unroll
                for (int u = 0; u < 4; ++u) ys[rr * NS + k4 + u] = v[x][u];
        }
        __syncthreads();
        for (int rb = 16 * wave; rb < rows; rb += 16 * (NTHREADS / 64)) {
            const int r = min(rb + c, rows - 1);
            f32x4 acc[JT];
#pragma unroll
            for (int t = 0; t < JT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const float b = ys[r * NS + 4 * k + q];
#pragma unroll
                for (int t = 0; t < JT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][k], b, acc[t], 0, 0, 0);
            }
            if (rb + c < rows) {
                float* zr = Z + (l0 + rb + c) * m_out;
#pragma unroll
                for (int t = 0; t < JT; ++t) {
                    const int j = 16 * t + 4 * q;
                    if (j < m_out) *reinterpret_cast<float4*>(zr + j) = float4{acc[t][0], acc[t][1], acc[t][2], acc[t][3]};
                }
            }
        }
        __syncthreads();
    }
}

// Z = sum over the ks partial outputs of a split-K mode product, in split
// order (rows min(m_out, *m_dev) of the device-side rank, as the product).
__global__ __launch_bounds__(NTHREADS) void k_ttm_ksum(const float* __restrict__ part, int ks, int64_t L, int m_out,
                                                       int64_t R, const int32_t* __restrict__ m_dev,
                                                       float* __restrict__ Z) {
    if (m_dev) m_out = min(m_out, *m_dev);
    if (m_out < 1) return;
    const int64_t total = L * m_out * R;
    for (int64_t i = (int64_t)blockIdx.x * NTHREADS + threadIdx.x; i < total; i += (int64_t)gridDim.x * NTHREADS) {
        float s = part[i];
        for (int k = 1; k < ks; ++k) s += part[(int64_t)k * total + i];
        Z[i] = s;
    }
}

// The last two mode products of a reconstruction in one pass (float32):
// for every l of the leading modes, X[l] = U_a Y[l] U_b^T with Y[l] the
// r_a x r_b slab of the input (r_a <= 32, r_b <= 16), U_a n_a x r_a (n_a <=
// 128) and U_b n_b x r_b (n_b <= 64), so the n_a x r_b intermediate never
// goes to memory.  Wavefront w owns rows 32 w .. 32 w + 31 of T and X for
// every slab, so the wavefronts never wait for each other: T = U_a Y[l]
// (K = r_a in steps of 4, U_a rows in registers, Y[l] loaded one slab
// ahead), T through the wavefront's LDS rows (read back whole), X = T U_b^T
// (U_b in registers), X staged in the same LDS rows and written as one
// contiguous block of 32 rows with 16-byte stores.  FP32 products and sums
// on v_mfma_f32_16x16x4f32.
constexpr int F2_RA = 32, F2_RB = 16, F2_NA = 128, F2_NB = 64;
constexpr int F2_TS = F2_RB + 1;   // T row stride (floats)
constexpr int F2_XS = F2_NB + 4;   // staged X row stride (floats): rows 4 apart in distinct banks

__global__ __launch_bounds__(NTHREADS) void k_ttm_fused_last2(const float* __restrict__ Y, int64_t L, int ra, int rb,
                                                              int na, int nb, const float* __restrict__ Ua,
                                                              const float* __restrict__ Ub, float* __restrict__ X) {
    static_assert(32 * F2_TS <= 32 * F2_XS, "T fits in the staging rows");
    __shared__ float xs_all[F2_NA * F2_XS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = lane & 15, q = lane >> 4;
    float* xs = xs_all + 32 * wave * F2_XS;   // this wavefront's 32 rows
    float* ts = xs;                           // T goes through the same rows first
    const int row0 = 32 * wave;
    const int rows = max(0, min(32, na - row0));
    // A operands of T = U_a Y: rows 32 w + 16 h + c of U_a, K = 4 s + q
    float ua[2][F2_RA / 4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int st = 0; st < F2_RA / 4; ++st) {
            const int row = row0 + 16 * h + c, k = 4 * st + q;
            ua[h][st] = (row < na && k < ra) ? Ua[(int64_t)row * ra + k] : 0.f;
        }
    // B operands of X = T U_b^T: B[k][col] = U_b[16 t + col][k], K = 4 s + q
    float ub[F2_NB / 16][F2_RB / 4];
#pragma unroll
    for (int t = 0; t < F2_NB / 16; ++t)
#pragma unroll
        for (int st = 0; st < F2_RB / 4; ++st) {
            const int d = 16 * t + c, k = 4 * st + q;
            ub[t][st] = (d < nb && k < rb) ? Ub[(int64_t)d * rb + k] : 0.f;
        }
    const int xsz = na * nb;   // <= 8192
    const bool vec = (nb & 3) == 0;
    // B operands of T = U_a Y[l]: Y[l][4 s + q][c], loaded one slab ahead
    float yv[F2_RA / 4];
    auto load_y = [&](int64_t l) {
        const float* yl = Y + min(l, L - 1) * (int64_t)ra * rb;
#pragma unroll
        for (int st = 0; st < F2_RA / 4; ++st) {
            const int k = 4 * st + q;
            yv[st] = (k < ra && c < rb) ? yl[k * rb + c] : 0.f;
        }
    };
    load_y(blockIdx.x);
    for (int64_t l = blockIdx.x; l < L; l += gridDim.x) {
        // T rows 32 w + 16 h + (4 q + e), column c
        f32x4 tacc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int st = 0; st < F2_RA / 4; ++st)
#pragma unroll
            for (int h = 0; h < 2; ++h) tacc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(ua[h][st], yv[st], tacc[h], 0, 0, 0);
        load_y(l + gridDim.x);   // the next slab's loads in flight over the rest
        // (LDS accesses of one wavefront take effect in issue order)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < 4; ++e) ts[(16 * h + 4 * q + e) * F2_TS + c] = tacc[h][e];
        __builtin_amdgcn_wave_barrier();
        // T back as A operands (all of it before X overwrites the rows)
        float tv[2][F2_RB / 4];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int st = 0; st < F2_RB / 4; ++st) tv[h][st] = ts[(16 * h + c) * F2_TS + 4 * st + q];
        __builtin_amdgcn_wave_barrier();
        // X rows 32 w + 16 h + (4 q + e), columns 16 t + c
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            f32x4 xacc[F2_NB / 16];
#pragma unroll
            for (int t = 0; t < F2_NB / 16; ++t) xacc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < F2_RB / 4; ++st)
#pragma unroll
                for (int t = 0; t < F2_NB / 16; ++t)
                    xacc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(tv[h][st], ub[t][st], xacc[t], 0, 0, 0);
#pragma unroll
            for (int t = 0; t < F2_NB / 16; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = 16 * h + 4 * q + e, col = 16 * t + c;
                    if (r < rows && col < nb) xs[r * F2_XS + col] = xacc[t][e];
                }
        }
        __builtin_amdgcn_wave_barrier();
        // this wavefront's rows of X[l]: rows * n_b consecutive floats
        float* xl = X + l * (int64_t)xsz + (int64_t)row0 * nb;
        const int wsz = rows * nb;
        if (vec) {
            for (int e4 = 4 * lane; e4 < wsz; e4 += 256) {
                const int r = e4 / nb, col = e4 - r * nb;
                const float4 v = *reinterpret_cast<const float4*>(&xs[r * F2_XS + col]);
                *reinterpret_cast<float4*>(xl + e4) = v;
            }
        } else {
            for (int e = lane; e < wsz; e += 64) {
                const int r = e / nb, col = e - r * nb;
                xl[e] = xs[r * F2_XS + col];
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

template <int KC>
void launch_expand_last_k(int jt, unsigned grid, hipStream_t st, const float* Y, int64_t L, int n, int m_out,
                          const float* M, float* Z) {
    if (jt <= 2) hipLaunchKernelGGL((k_ttm_expand_last<KC, 2>), dim3(grid), dim3(NTHREADS), 0, st, Y, L, n, m_out, M, Z);
    else if (jt <= 4) hipLaunchKernelGGL((k_ttm_expand_last<KC, 4>), dim3(grid), dim3(NTHREADS), 0, st, Y, L, n, m_out, M, Z);
    else hipLaunchKernelGGL((k_ttm_expand_last<KC, 8>), dim3(grid), dim3(NTHREADS), 0, st, Y, L, n, m_out, M, Z);
}

// Shrinking of a last, contiguous mode (R == 1) in FP32: Z[l][j] = sum_i
// Y[l][i] M[j][i] with n <= 4 KC entries per row and m_out <= 16 JT outputs
// (the reconstruction adjoint's projections of the last mode).  Tiles of
// SHR_ROWS consecutive rows of Y (one contiguous block, coalesced loads) are
// staged in LDS rows of odd stride; each wavefront then forms 16 rows at a
// time on v_mfma_f32_16x16x4f32 with A = the rows' entries (16 rows x 4
// entries, from LDS) and B = M^T (4 entries x 16 outputs, in registers for
// the whole kernel): lane (c, q) ends with Z[l0 + 4 q + v][16 t + c], v < 4.
constexpr int SHR_ROWS = 128;

template <int KC, int JT>
__global__ __launch_bounds__(NTHREADS) void k_ttm_shrink_last(const float* __restrict__ Y, int64_t L, int n,
                                                              int m_out, const float* __restrict__ M32,
                                                              float* __restrict__ Z) {
    constexpr int NS = 4 * KC + 1;
    __shared__ float ys[SHR_ROWS * NS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = lane & 15, q = lane >> 4;
    float bm[JT][KC];
#pragma unroll
    for (int t = 0; t < JT; ++t)
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int j = 16 * t + c, i = 4 * k + q;
            bm[t][k] = (j < m_out && i < n) ? M32[(int64_t)j * n + i] : 0.f;
        }
    const bool vec = (n & 3) == 0;
    for (int64_t tile = blockIdx.x; tile * SHR_ROWS < L; tile += gridDim.x) {
        const int64_t l0 = tile * SHR_ROWS;
        const int rows = (int)min<int64_t>(SHR_ROWS, L - l0);
        // the tile's entries in groups of four (zeros past n), loads first
        constexpr int PER = SHR_ROWS * KC / NTHREADS;
        static_assert(PER * NTHREADS == SHR_ROWS * KC, "tile split");
        float v[PER][4];
#pragma unroll
        for (int x = 0; x < PER; ++x) {
            const int e = tid + x * NTHREADS;
            const int rr = e / KC, k4 = 4 * (e % KC);
            const float* src = Y + (l0 + min(rr, rows - 1)) * n + k4;
            if (vec && k4 < n) {
                const float4 w = rr < rows ? *reinterpret_cast<const float4*>(src) : float4{0.f, 0.f, 0.f, 0.f};
                v[x][0] = w.x;
                v[x][1] = w.y;
                v[x][2] = w.z;
                v[x][3] = w.w;
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) v[x][u] = (rr < rows && k4 + u < n) ? src[u] : 0.f;
            }
        }
#pragma unroll
        for (int x = 0; x < PER; ++x) {
            const int e = tid + x * NTHREADS;
            const int rr = e / KC, k4 = 4 * (e % KC);
#pragma unroll
            for (int u = 0; u < 4; ++u) ys[rr * NS + k4 + u] = v[x][u];
        }
        __syncthreads();
        for (int rb = 16 * wave; rb < rows; rb += 16 * (NTHREADS / 64)) {
            const int r = min(rb + c, rows - 1);
            f32x4 acc[JT];
#pragma unroll
            for (int t = 0; t < JT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const float av = ys[r * NS + 4 * k + q];
#pragma unroll
                for (int t = 0; t < JT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bm[t][k], acc[t], 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < JT; ++t) {
                const int j = 16 * t + c;
                if (j >= m_out) continue;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int row = rb + mfma16_row<PREC_F32>(lane, u);
                    if (row < rows) Z[(l0 + row) * m_out + j] = acc[t][u];
                }
            }
        }
        __syncthreads();
    }
}

template <int KC>
void launch_shrink_last_k(int jt, unsigned grid, hipStream_t st, const float* Y, int64_t L, int n, int m_out,
                          const float* M, float* Z) {
    if (jt <= 1) hipLaunchKernelGGL((k_ttm_shrink_last<KC, 1>), dim3(grid), dim3(NTHREADS), 0, st, Y, L, n, m_out, M, Z);
    else hipLaunchKernelGGL((k_ttm_shrink_last<KC, 2>), dim3(grid), dim3(NTHREADS), 0, st, Y, L, n, m_out, M, Z);
}

template <int P, int LAYOUT>
hipError_t launch_ttm_t(const TtmPlan& t, const void* Y, const void* M, const void* Mh, const void* Ml, void* Z,
                        const int32_t* m_dev, hipStream_t st) {
    using T = typename ElemOf<P>::T;
    dim3 grid((unsigned)t.ctiles, t.jtiles);
    hipLaunchKernelGGL((k_ttm<P, LAYOUT>), grid, dim3(NTHREADS), 0, st, (const T*)Y, t.L, t.n, t.R, t.m_out,
                       t.tiles_per_l, t.planes, (const double*)M, (const float*)M, (const __bf16*)Mh,
                       (const __bf16*)Ml, (T*)Z, m_dev);
    return hipGetLastError();
}

template <int P>
hipError_t launch_ttm_p(const TtmPlan& t, const void* Y, const void* M, const void* Mh, const void* Ml, void* Z,
                        const int32_t* m_dev, hipStream_t st) {
    switch (t.layout) {
        case LAYOUT_KC: return launch_ttm_t<P, LAYOUT_KC>(t, Y, M, Mh, Ml, Z, m_dev, st);
        case LAYOUT_NC: return launch_ttm_t<P, LAYOUT_NC>(t, Y, M, Mh, Ml, Z, m_dev, st);
        default: return launch_ttm_t<P, LAYOUT_SR>(t, Y, M, Mh, Ml, Z, m_dev, st);
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

bool ttm_fused_last2_fits(int64_t L, int ra, int rb, int na, int nb, const void* X) {
    // float4 stores (n_b % 4 == 0) need 16-byte aligned slabs
    const bool aligned = (nb & 3) != 0 || reinterpret_cast<uintptr_t>(X) % 16 == 0;
    return L >= 1 && ra >= 1 && ra <= F2_RA && rb >= 1 && rb <= F2_RB && na >= 1 && na <= F2_NA && nb >= 1 &&
           nb <= F2_NB && aligned;
}

hipError_t launch_ttm_fused_last2(const float* Y, int64_t L, int ra, int rb, int na, int nb, const float* Ua,
                                  const float* Ub, float* X, hipStream_t st) {
    if (!ttm_fused_last2_fits(L, ra, rb, na, nb, X)) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)std::min<int64_t>(L, 2048);
    hipLaunchKernelGGL(k_ttm_fused_last2, dim3(grid), dim3(NTHREADS), 0, st, Y, L, ra, rb, na, nb, Ua, Ub, X);
    return hipGetLastError();
}

hipError_t launch_ttm(int prec, const TtmPlan& t, const void* Y, const void* M, const void* Mh, const void* Ml,
                      void* Z, hipStream_t st, const int32_t* m_dev, float* kpart, size_t kpart_bytes) {
    if (prec != PREC_F64 && t.layout == LAYOUT_KC && t.R >= 32 && t.R % 4 == 0 && t.m_out <= 64 &&
        reinterpret_cast<uintptr_t>(Y) % 16 == 0) {
        // R >= 256: 256-column chunks of one slice; R < 256: 256 / R whole slices per workgroup
        const int pl = t.R >= 256 ? 1 : (int)(256 / t.R);
        const int64_t tpl = t.R >= 256 ? ceil_div(t.R, (int64_t)256) : 1;
        const int64_t tiles = pl > 1 ? ceil_div(t.L, (int64_t)pl) : t.L * tpl;
        // few tiles over a long K: K split over grid.y into partial outputs,
        // summed in split order by k_ttm_ksum (each workgroup otherwise walks
        // all of K, one memory latency per 32 terms)
        int ks = 1;
        if (kpart && tiles < 128 && t.n >= 256) {
            ks = (int)std::min<int64_t>(8, std::max<int64_t>(1, 256 / tiles));
            while (ks > 1 && (size_t)ks * t.L * t.m_out * t.R * sizeof(float) > kpart_bytes) --ks;
        }
        const int kchunk = (int)(ceil_div(ceil_div((int64_t)t.n, (int64_t)ks), (int64_t)32) * 32);
        ks = (int)ceil_div((int64_t)t.n, (int64_t)kchunk);
        const dim3 grid((unsigned)tiles, (unsigned)ks);
        const float* y = (const float*)Y;
        const float* m = (const float*)M;
        float* z = ks > 1 ? kpart : (float*)Z;
        if (prec == PREC_BF16X3) {
            if (t.m_out <= 32) hipLaunchKernelGGL((k_ttm_wide<PREC_BF16X3, 2>), grid, dim3(NTHREADS), 0, st, y, t.L, t.n, t.R, t.m_out, tpl, pl, m, z, m_dev, kchunk);
            else hipLaunchKernelGGL((k_ttm_wide<PREC_BF16X3, 4>), grid, dim3(NTHREADS), 0, st, y, t.L, t.n, t.R, t.m_out, tpl, pl, m, z, m_dev, kchunk);
        } else if (prec == PREC_BF16X6) {
            if (t.m_out <= 32) hipLaunchKernelGGL((k_ttm_wide<PREC_BF16X6, 2>), grid, dim3(NTHREADS), 0, st, y, t.L, t.n, t.R, t.m_out, tpl, pl, m, z, m_dev, kchunk);
            else hipLaunchKernelGGL((k_ttm_wide<PREC_BF16X6, 4>), grid, dim3(NTHREADS), 0, st, y, t.L, t.n, t.R, t.m_out, tpl, pl, m, z, m_dev, kchunk);
        } else {
            if (t.m_out <= 32) hipLaunchKernelGGL((k_ttm_wide<PREC_F32, 2>), grid, dim3(NTHREADS), 0, st, y, t.L, t.n, t.R, t.m_out, tpl, pl, m, z, m_dev, kchunk);
            else hipLaunchKernelGGL((k_ttm_wide<PREC_F32, 4>), grid, dim3(NTHREADS), 0, st, y, t.L, t.n, t.R, t.m_out, tpl, pl, m, z, m_dev, kchunk);
        }
        if (ks > 1) {
            const unsigned g = (unsigned)std::min<int64_t>(2048, std::max<int64_t>(1, ceil_div(t.L * t.m_out * t.R, (int64_t)1024)));
            hipLaunchKernelGGL(k_ttm_ksum, dim3(g), dim3(NTHREADS), 0, st, (const float*)kpart, ks, t.L, t.m_out, t.R, m_dev,
                               (float*)Z);
        }
        return hipGetLastError();
    }
    // expansion of a last, contiguous mode in FP32 (the reconstruction's last step)
    const bool f32ish = prec == PREC_F32 || prec == PREC_BF16X6;
    if (f32ish && t.layout == LAYOUT_NC && t.R == 1 && !m_dev && t.n <= 32 && t.m_out > t.n &&
        t.m_out % 4 == 0 && t.m_out <= 128 && reinterpret_cast<uintptr_t>(Y) % 16 == 0 &&
        reinterpret_cast<uintptr_t>(Z) % 16 == 0) {
        const unsigned grid = (unsigned)std::min<int64_t>(std::max<int64_t>(1, ceil_div(t.L, (int64_t)EXP_ROWS)), 4096);
        const int jt = (int)ceil_div(t.m_out, 16);
        const float* y = (const float*)Y;
        const float* m = (const float*)M;
        float* z = (float*)Z;
        if (t.n <= 8) launch_expand_last_k<2>(jt, grid, st, y, t.L, t.n, t.m_out, m, z);
        else if (t.n <= 16) launch_expand_last_k<4>(jt, grid, st, y, t.L, t.n, t.m_out, m, z);
        else launch_expand_last_k<8>(jt, grid, st, y, t.L, t.n, t.m_out, m, z);
        return hipGetLastError();
    }
    // shrinking of a last, contiguous mode in FP32 over many rows
    if (f32ish && t.layout == LAYOUT_NC && t.R == 1 && !m_dev && t.n <= 128 && t.m_out < t.n &&
        t.m_out <= 32 && t.L >= 8192 && reinterpret_cast<uintptr_t>(Y) % 16 == 0) {
        const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(t.L, (int64_t)SHR_ROWS), 4096);
        const int jt = (int)ceil_div(t.m_out, 16);
        const float* y = (const float*)Y;
        const float* m = (const float*)M;
        float* z = (float*)Z;
        if (t.n <= 16) launch_shrink_last_k<4>(jt, grid, st, y, t.L, t.n, t.m_out, m, z);
        else if (t.n <= 32) launch_shrink_last_k<8>(jt, grid, st, y, t.L, t.n, t.m_out, m, z);
        else if (t.n <= 64) launch_shrink_last_k<16>(jt, grid, st, y, t.L, t.n, t.m_out, m, z);
        else launch_shrink_last_k<32>(jt, grid, st, y, t.L, t.n, t.m_out, m, z);
        return hipGetLastError();
    }
    // short slabs (few 64-row tiles for the tile kernel, latency-bound): rows kernel
    if (prec != PREC_F64 && t.layout == LAYOUT_NC && t.R == 1 && t.m_out <= 32 && t.L < 8192) {
        hipLaunchKernelGGL(k_ttm_rows, dim3((unsigned)ceil_div(t.L, 16)), dim3(NTHREADS), 0, st, (const float*)Y, t.L,
                           t.n, t.m_out, (const float*)M, (float*)Z, m_dev);
        return hipGetLastError();
    }
    switch (prec) {
        case PREC_F64: return launch_ttm_p<PREC_F64>(t, Y, M, Mh, Ml, Z, m_dev, st);
        case PREC_F32:
        case PREC_BF16X6: return launch_ttm_p<PREC_F32>(t, Y, M, Mh, Ml, Z, m_dev, st);
        default: return launch_ttm_p<PREC_BF16X3>(t, Y, M, Mh, Ml, Z, m_dev, st);
    }
}

}  // namespace atc
