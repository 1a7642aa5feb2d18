// Gram matrix (SYRK) of an (L, n, R) view whose R index is contiguous and a
// multiple of 4 -- the layout of every mode but the last of a row-major
// tensor, and where almost all of the Gram work of an ST-HOSVD is done (the
// first mode sees the whole input).
//
//   G[a, b] = sum_{l, r} X[l, a, r] X[l, b, r]      (Section 3.2, Algorithm 1)
//
// Work decomposition: 128 x 128 output tiles of the upper triangle times
// split-K ranges.  Block b runs on XCD b % 8; the tiles of one split are
// given consecutive slots of the same XCD, so the rows of one K slab are
// fetched from HBM once and served to the other tiles of that split from
// that XCD's L2.  Each workgroup: 4 waves, each owning a 64 x 64 quarter made
// of 2 x 2 blocks of 32 x 32 MFMAs; K advances in steps of 32 with the next
// step's global loads (float4, coalesced along R) held in registers while the
// current step is multiplied out of LDS.
//   PREC_BF16X3: every loaded float is split into bf16 hi + lo on the way to
//     LDS; three v_mfma_f32_32x32x16_bf16 per 32 x 32 x 16 (hi*hi, hi*lo,
//     lo*hi); the diagonal is replaced by the exact sum of squares of the
//     loaded floats accumulated in FP64 (the dropped lo*lo would bias it).
//   PREC_F32: v_mfma_f32_32x32x2f32, same diagonal treatment.
// A workgroup accumulates one split (a few thousand terms) in FP32 and
// writes an FP32 partial tile; the reduction adds the splits in FP64 in a
// fixed order.
#include "atc_internal.hpp"

#include <type_traits>

namespace atc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int KC_BM = 128;
constexpr int KC_BK = 32;
constexpr int KC_PAD_BF = 8;   // bf16 row stride 40 (80 bytes: 16-byte aligned fragment reads)
constexpr int KC_PAD_F = 1;

__device__ inline void kc_decode_pair(int pair, int tiles, int& ti, int& tj) {
    int p = pair, i = 0;
    while (p >= tiles - i) {
        p -= tiles - i;
        ++i;
    }
    ti = i;
    tj = i + p;
}

__host__ __device__ inline int kc_pair_index(int ti, int tj, int tiles) {
    return ti * tiles - ti * (ti - 1) / 2 + (tj - ti);
}

template <int P> struct KcSmem;
template <> struct KcSmem<PREC_BF16X3> {
    __bf16 ah[KC_BM][KC_BK + KC_PAD_BF];
    __bf16 al[KC_BM][KC_BK + KC_PAD_BF];
    __bf16 bh[KC_BM][KC_BK + KC_PAD_BF];
    __bf16 bl[KC_BM][KC_BK + KC_PAD_BF];
};
template <> struct KcSmem<PREC_F32> {
    float a[KC_BM][KC_BK + KC_PAD_F];
    float b[KC_BM][KC_BK + KC_PAD_F];
};

// 32 x 32 MFMA result layout: register v of lane l holds column l % 32 of
// row 8 * (v / 4) + 4 * (l / 32) + v % 4.
__device__ inline int mfma32_row(int lane, int v) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

template <int P>
__device__ inline void kc_store(KcSmem<P>& sm, bool second, int row, int col, const float4& v) {
    if constexpr (P == PREC_BF16X3) {
        const float x[4] = {v.x, v.y, v.z, v.w};
        union {
            __bf16 h[4];
            uint2 u;
        } hi, lo;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            hi.h[e] = (__bf16)x[e];
            lo.h[e] = (__bf16)(x[e] - (float)hi.h[e]);
        }
        *reinterpret_cast<uint2*>(second ? &sm.bh[row][col] : &sm.ah[row][col]) = hi.u;
        *reinterpret_cast<uint2*>(second ? &sm.bl[row][col] : &sm.al[row][col]) = lo.u;
    } else {
        float* p = second ? &sm.b[row][col] : &sm.a[row][col];
        p[0] = v.x;
        p[1] = v.y;
        p[2] = v.z;
        p[3] = v.w;
    }
}

template <int P>
__global__ __launch_bounds__(256, 2) void k_gram_kc(const float* __restrict__ X, int n, int64_t L, int64_t R,
                                                 int64_t steps, int nsplit, int tiles, int npairs,
                                                 float* __restrict__ part, double* __restrict__ dpart) {
    __shared__ KcSmem<P> sm;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    // XCD-aware block -> (pair, split): the pairs of one split share an XCD
    const int b = blockIdx.x;
    const int xcd = b & 7, slot = b >> 3;
    const int pair = slot % npairs;
    const int split = (slot / npairs) * 8 + xcd;
    if (split >= nsplit) return;
    int ti, tj;
    kc_decode_pair(pair, tiles, ti, tj);
    const bool diag = ti == tj;
    const int row0 = ti * KC_BM, col0 = tj * KC_BM;
    const int64_t s0 = steps * split / nsplit, s1 = steps * (split + 1) / nsplit;
    const int64_t spl = ceil_div(R, KC_BK);

    // load slots: 8 threads per row (4 floats each), rows lr + 32 i.  The K
    // position (slice l, offset r) advances incrementally (no division per step).
    const int lr = tid >> 3, lc = (tid & 7) * 4;
    float4 ra[4], rb[4];
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    int64_t ld_l = s0 / spl;
    int64_t ld_r = (s0 - ld_l * spl) * KC_BK + lc;
    bool rowa_ok[4], rowb_ok[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        rowa_ok[i] = row0 + lr + 32 * i < n;
        rowb_ok[i] = col0 + lr + 32 * i < n;
    }
    const int64_t rowstep = (int64_t)32 * R;  // 32 rows apart
    // global address space made explicit: a flat load would also count
    // against lgkmcnt and stall every LDS wait behind the prefetch
    typedef float v4f __attribute__((ext_vector_type(4)));
    typedef const v4f __attribute__((address_space(1)))* gf4;
    auto gload = [](const float* p) -> float4 {
        const v4f v = *(gf4)p;
        return make_float4(v.x, v.y, v.z, v.w);
    };
    auto load = [&]() {
        const bool rok = ld_r < R;
        const float* pa = X + (ld_l * n + row0 + lr) * R + ld_r;
        const float* pb = X + (ld_l * n + col0 + lr) * R + ld_r;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ra[i] = zero4;
            if (rok && rowa_ok[i]) ra[i] = gload(pa + i * rowstep);
            if (!diag) {
                rb[i] = zero4;
                if (rok && rowb_ok[i]) rb[i] = gload(pb + i * rowstep);
            }
        }
        ld_r += KC_BK;
        if (ld_r - lc >= spl * KC_BK) {
            ld_r -= spl * KC_BK;
            ++ld_l;
        }
    };

    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    // two-level FP32 accumulation: the MFMA accumulators hold a chunk of
    // FLUSH_TERMS terms, chunk sums are added into `tot` (fewer, larger
    // roundings than one long MFMA accumulation; half the registers of FP64)
    f32x16 acc[2][2], tot[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                acc[a][c][v] = 0.f;
                tot[a][c][v] = 0.f;
            }
    double dsq[4] = {0.0, 0.0, 0.0, 0.0};
    constexpr int FLUSH_STEPS = FLUSH_TERMS / KC_BK;
    int since_flush = 0;
    auto flush = [&]() {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                tot[a][c] += acc[a][c];
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[a][c][v] = 0.f;
            }
    };

    if (s0 < s1) load();
    for (int64_t s = s0; s < s1; ++s) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            kc_store<P>(sm, false, lr + 32 * i, lc, ra[i]);
            if (!diag) kc_store<P>(sm, true, lr + 32 * i, lc, rb[i]);
            if (diag) {
                const double x0 = ra[i].x, x1 = ra[i].y, x2 = ra[i].z, x3 = ra[i].w;
                dsq[i] += x0 * x0 + x1 * x1 + x2 * x2 + x3 * x3;
            }
        }
        __syncthreads();
        if (s + 1 < s1) load();
#pragma unroll
        for (int sl = 0; sl < KC_BK / 16; ++sl) {
            if constexpr (P == PREC_BF16X3) {
                const int kq = sl * 16 + 8 * (lane >> 5);
                bf16x8 ah[2], al[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const int rr = wr + a * 32 + (lane & 31);
                    ah[a] = *reinterpret_cast<const bf16x8*>(&sm.ah[rr][kq]);
                    al[a] = *reinterpret_cast<const bf16x8*>(&sm.al[rr][kq]);
                }
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int cc = wc + c * 32 + (lane & 31);
                    const bf16x8 bh = diag ? *reinterpret_cast<const bf16x8*>(&sm.ah[cc][kq])
                                           : *reinterpret_cast<const bf16x8*>(&sm.bh[cc][kq]);
                    const bf16x8 bl = diag ? *reinterpret_cast<const bf16x8*>(&sm.al[cc][kq])
                                           : *reinterpret_cast<const bf16x8*>(&sm.bl[cc][kq]);
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh, acc[a][c], 0, 0, 0);
                        acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl, acc[a][c], 0, 0, 0);
                        acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh, acc[a][c], 0, 0, 0);
                    }
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < 16; kk += 2) {
                    const int k = sl * 16 + kk + (lane >> 5);
                    float av[2], bv[2];
#pragma unroll
                    for (int a = 0; a < 2; ++a) av[a] = sm.a[wr + a * 32 + (lane & 31)][k];
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        bv[c] = diag ? sm.a[wc + c * 32 + (lane & 31)][k] : sm.b[wc + c * 32 + (lane & 31)][k];
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int c = 0; c < 2; ++c)
                            acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a], bv[c], acc[a][c], 0, 0, 0);
                }
            }
        }
        if (++since_flush == FLUSH_STEPS) {
            since_flush = 0;
            flush();
        }
        __syncthreads();
    }
    flush();
    float* out = part + ((int64_t)split * npairs + pair) * (KC_BM * KC_BM);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = wr + a * 32 + mfma32_row(lane, v);
                const int j = wc + c * 32 + (lane & 31);
                out[i * KC_BM + j] = tot[a][c][v];
            }
    if (diag) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double s = dsq[i];
            s += __shfl_xor(s, 1);
            s += __shfl_xor(s, 2);
            s += __shfl_xor(s, 4);
            const int row = row0 + lr + 32 * i;
            if ((tid & 7) == 0 && row < n) dpart[(int64_t)split * n + row] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// bf16x3 variant for full tiles (n % 128 == 0, R % 32 == 0): the same work
// decomposition and accumulation as k_gram_kc, with
//   * LDS rows of 32 bf16 (64 bytes) without padding; the four 16-byte chunks
//     of row r sit at chunk ^ ((r >> 2) & 3), so the 16 rows one ds_read_b128
//     group touches cover all 64 banks;
//   * two LDS stages: step s+1 is stored into the other stage while step s is
//     multiplied, one workgroup barrier per step;
//   * the split x = hi + lo from one packed conversion per pair (hi), the
//     exact difference, and one packed conversion per pair (lo);
//   * no row or K masking, and the chunk's first products take a zero
//     accumulator instead of clearing it;
//   * a diagonal tile loads and splits its second panel like every other tile
//     (the same rows as the first), so the tiles of one split advance at one
//     pace and the slab one of them fetches is still in L2 for the others
//     (L2 hit rate 72% against 48% when diagonal tiles ran ahead); only the
//     products of its strictly lower quarter, never read, are skipped.
struct K3Stage {
    uint4 ah[KC_BM][4], al[KC_BM][4], bh[KC_BM][4], bl[KC_BM][4];
};

__device__ __forceinline__ int k3_chunk(int row, int c) { return c ^ ((row >> 2) & 3); }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// hi / lo bf16 pairs of (x, y): hi = bf16(x), lo = bf16(x - hi)
__device__ __forceinline__ void k3_split2(float x, float y, uint32_t& hi, uint32_t& lo) {
    const bf16x2 h = {(__bf16)x, (__bf16)y};
    uint32_t hu = __builtin_bit_cast(uint32_t, h);
    asm("" : "+v"(hu));  // keeps the compiler from converting x a second time for hx
    const float hx = __uint_as_float(hu << 16), hy = __uint_as_float(hu & 0xffff0000u);
    const bf16x2 l = {(__bf16)(x - hx), (__bf16)(y - hy)};
    hi = hu;
    lo = __builtin_bit_cast(uint32_t, l);
}

__global__ __launch_bounds__(256, 2) void k_gram_kc3(const float* __restrict__ X, int n, int64_t L, int64_t R,
                                                  int64_t steps, int nsplit, int tiles, int npairs,
                                                  float* __restrict__ part, double* __restrict__ dpart) {
    __shared__ K3Stage sm[2];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int b = blockIdx.x;
    const int xcd = b & 7, slot = b >> 3;
    const int pair = slot % npairs;
    const int split = (slot / npairs) * 8 + xcd;
    if (split >= nsplit) return;
    int ti, tj;
    kc_decode_pair(pair, tiles, ti, tj);
    const bool diag = ti == tj;
    const int row0 = ti * KC_BM, col0 = tj * KC_BM;
    const int64_t s0 = steps * split / nsplit, s1 = steps * (split + 1) / nsplit;
    const int64_t spl = R / KC_BK;  // K steps per slice l

    // loader: 8 threads per row (4 floats each), rows lr + 32 i
    const int lr = tid >> 3, lc = (tid & 7) * 4;
    typedef float v4f __attribute__((ext_vector_type(4)));
    typedef const v4f __attribute__((address_space(1)))* gf4;
    const int64_t rowstep = (int64_t)32 * R;
    int64_t l0 = s0 / spl, kpos = (s0 - l0 * spl) * KC_BK;  // slice and K offset of the next load
    const float* pa = X + (l0 * n + row0 + lr) * R + kpos + lc;
    const float* pb = X + (l0 * n + col0 + lr) * R + kpos + lc;
    const int64_t wrap = (int64_t)(n - 1) * R;  // from one slice's row end to the next slice's row start
    v4f ra[4], rb[4];
    auto load = [&]() {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ra[i] = *(gf4)(pa + i * rowstep);
            rb[i] = *(gf4)(pb + i * rowstep);
        }
        pa += KC_BK;
        pb += KC_BK;
        kpos += KC_BK;
        if (kpos == R) {
            kpos = 0;
            pa += wrap;
            pb += wrap;
        }
    };
    // store of the loaded rows into stage st (hi / lo), diagonal sums of squares
    double dsq[4] = {0.0, 0.0, 0.0, 0.0};
    const int cst = lc >> 3, half = (lc >> 2) & 1;
    auto store = [&](K3Stage& S) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = lr + 32 * i;
            const int ch = k3_chunk(row, cst);
            uint2 h, l;
            k3_split2(ra[i].x, ra[i].y, h.x, l.x);
            k3_split2(ra[i].z, ra[i].w, h.y, l.y);
            reinterpret_cast<uint2*>(&S.ah[row][ch])[half] = h;
            reinterpret_cast<uint2*>(&S.al[row][ch])[half] = l;
            k3_split2(rb[i].x, rb[i].y, h.x, l.x);
            k3_split2(rb[i].z, rb[i].w, h.y, l.y);
            reinterpret_cast<uint2*>(&S.bh[row][ch])[half] = h;
            reinterpret_cast<uint2*>(&S.bl[row][ch])[half] = l;
            if (diag) {
                const double x0 = ra[i].x, x1 = ra[i].y, x2 = ra[i].z, x3 = ra[i].w;
                dsq[i] += x0 * x0 + x1 * x1 + x2 * x2 + x3 * x3;
            }
        }
    };

    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    const bool lower = diag && wr > wc;
    f32x16 acc[2][2], tot[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 16; ++v) tot[a][c][v] = 0.f;
    const f32x16 zero16 = {};
    // products of one K step from stage S; ZC: the first slice starts from zero
    auto mma = [&](const K3Stage& S, auto zc) {
        constexpr bool ZC = decltype(zc)::value;
#pragma unroll
        for (int sl = 0; sl < KC_BK / 16; ++sl) {
            const int cq = 2 * sl + (lane >> 5);
            bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int rr = wr + a * 32 + (lane & 31);
                ah[a] = __builtin_bit_cast(bf16x8, S.ah[rr][k3_chunk(rr, cq)]);
                al[a] = __builtin_bit_cast(bf16x8, S.al[rr][k3_chunk(rr, cq)]);
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int cc = wc + c * 32 + (lane & 31);
                const int ch = k3_chunk(cc, cq);
                bh[c] = __builtin_bit_cast(bf16x8, S.bh[cc][ch]);
                bl[c] = __builtin_bit_cast(bf16x8, S.bl[cc][ch]);
            }
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const f32x16 c0 = (ZC && sl == 0) ? zero16 : acc[a][c];
                    acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[c], c0, 0, 0, 0);
                    acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[c], acc[a][c], 0, 0, 0);
                    acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[c], acc[a][c], 0, 0, 0);
                }
        }
    };
    constexpr int FLUSH_STEPS = FLUSH_TERMS / KC_BK;
    int since = 0;
    if (s0 < s1) {
        load();
        store(sm[0]);
    }
    __syncthreads();
    for (int64_t s = s0; s < s1; ++s) {
        const int cur = (int)((s - s0) & 1);
        const bool more = s + 1 < s1;
        if (more) load();
        if (lower) {
            // the strictly lower quarter of a diagonal tile is never read
        } else if (since == 0) {
            mma(sm[cur], std::true_type{});
        } else {
            mma(sm[cur], std::false_type{});
        }
        if (++since == FLUSH_STEPS || !more) {
            since = 0;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) tot[a][c] += acc[a][c];
        }
        if (more) store(sm[cur ^ 1]);
        __syncthreads();
    }
    float* out = part + ((int64_t)split * npairs + pair) * (KC_BM * KC_BM);
#pragma unroll
    for (int a = 0; a < 2 && !lower; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = wr + a * 32 + mfma32_row(lane, v);
                const int j = wc + c * 32 + (lane & 31);
                out[i * KC_BM + j] = tot[a][c][v];
            }
    if (diag) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double sq = dsq[i];
            sq += __shfl_xor(sq, 1);
            sq += __shfl_xor(sq, 2);
            sq += __shfl_xor(sq, 4);
            const int row = row0 + lr + 32 * i;
            if ((tid & 7) == 0) dpart[(int64_t)split * n + row] = sq;
        }
    }
}

// G (n x n, FP64, both triangles) from the split partials: one workgroup of
// 256 threads per 32 x 32 block of the upper triangle of blocks, a thread four
// consecutive entries of one row.  It loads those entries' partials of 16
// splits at once (one 16-byte load per split) and adds them in split order;
// diagonal entries take the exact FP64 sums of squares instead.  The block is
// stored, and through LDS its transpose, both with 32-byte row pieces.
constexpr int RDB = 32;   // reduction block edge
constexpr int RDS = 16;   // splits loaded together
__global__ __launch_bounds__(256) void k_gram_kc_reduce(const float* __restrict__ part,
                                                        const double* __restrict__ dpart, int nsplit, int npairs,
                                                        int tiles, int n, double* __restrict__ G) {
    __shared__ double tb[RDB][RDB + 1];
    const int nbk = (n + RDB - 1) / RDB;
    int t = blockIdx.x, bi = 0;
    while (t >= nbk - bi) {  // block (bi, bj), bi <= bj, in row-major order of the upper triangle
        t -= nbk - bi;
        ++bi;
    }
    const int bj = bi + t;
    const int ty = threadIdx.x >> 3, tx = threadIdx.x & 7;
    const int a = bi * RDB + ty, b0 = bj * RDB + 4 * tx;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (a < n && b0 < n) {
        const int ti = a / KC_BM, tj = b0 / KC_BM;
        const int pair = kc_pair_index(ti, tj, tiles);
        const int64_t off = (int64_t)(a % KC_BM) * KC_BM + b0 % KC_BM;  // four entries in one tile row
        for (int sp0 = 0; sp0 < nsplit; sp0 += RDS) {
            float4 v[RDS];
#pragma unroll
            for (int u = 0; u < RDS; ++u) {
                const int sp = min(sp0 + u, nsplit - 1);
                v[u] = *reinterpret_cast<const float4*>(part + ((int64_t)sp * npairs + pair) * (KC_BM * KC_BM) + off);
            }
#pragma unroll
            for (int u = 0; u < RDS; ++u) {
                if (sp0 + u < nsplit) {
                    s[0] += (double)v[u].x;
                    s[1] += (double)v[u].y;
                    s[2] += (double)v[u].z;
                    s[3] += (double)v[u].w;
                }
            }
        }
        const int e = a - b0;  // the diagonal entry of this row piece, if any
        if (e >= 0 && e < 4) {
            double d = 0.0;
            for (int sp0 = 0; sp0 < nsplit; sp0 += RDS) {
                double w[RDS];
#pragma unroll
                for (int u = 0; u < RDS; ++u) w[u] = dpart[(int64_t)min(sp0 + u, nsplit - 1) * n + a];
#pragma unroll
                for (int u = 0; u < RDS; ++u)
                    if (sp0 + u < nsplit) d += w[u];
            }
            s[e] = d;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (b0 + q < n && a <= b0 + q) G[(int64_t)a * n + b0 + q] = s[q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) tb[ty][4 * tx + q] = s[q];
    __syncthreads();
    // mirror: row bj*32 + ty, columns bi*32 + 4 tx .. + 3 <- entries (column, row) of the block
    const int ra = bj * RDB + ty, cb0 = bi * RDB + 4 * tx;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int cb = cb0 + q;
        if (ra < n && cb < n && ra > cb) G[(int64_t)ra * n + cb] = tb[4 * tx + q][ty];
    }
}

}  // namespace

bool gram_kc_applicable(int prec, int64_t R) {
    return (prec == PREC_F32 || prec == PREC_BF16X3) && R >= KC_BK && R % 4 == 0;
}

GramKcPlan gram_kc_plan(int prec, int64_t L, int n, int64_t R, size_t part_capacity_bytes,
                        size_t dpart_capacity_bytes) {
    (void)prec;
    GramKcPlan g{};
    g.L = L;
    g.R = R;
    g.n = n;
    g.tiles = (int)ceil_div(n, KC_BM);
    g.npairs = g.tiles * (g.tiles + 1) / 2;
    g.steps = L * ceil_div(R, KC_BK);
    // about two workgroups per CU in one wave of dispatch, a multiple of 8 splits
    int64_t ns = (512 / g.npairs) / 8 * 8;
    if (ns < 8) ns = 8;
    const int64_t by_steps = (g.steps / 16) / 8 * 8;  // at least 16 steps per split
    if (ns > by_steps) ns = by_steps < 8 ? 8 : by_steps;
    const size_t tile_bytes = (size_t)KC_BM * KC_BM * sizeof(float);
    while (ns > 8 && ((size_t)ns * g.npairs * tile_bytes > part_capacity_bytes ||
                      (size_t)ns * n * sizeof(double) > dpart_capacity_bytes))
        ns -= 8;
    g.nsplit = (int)ns;
    g.part_bytes = (size_t)ns * g.npairs * tile_bytes;
    g.dpart_bytes = (size_t)ns * n * sizeof(double);
    g.ok = g.part_bytes <= part_capacity_bytes && g.dpart_bytes <= dpart_capacity_bytes;
    return g;
}

hipError_t launch_gram_kc(int prec, const GramKcPlan& g, const float* X, float* part, double* dpart,
                          hipStream_t st) {
    if (!g.ok) return hipErrorInvalidValue;
    const int blocks = g.nsplit * g.npairs;  // nsplit is a multiple of 8
    if (prec == PREC_BF16X3 && g.n % KC_BM == 0 && g.R % KC_BK == 0)
        hipLaunchKernelGGL(k_gram_kc3, dim3(blocks), dim3(256), 0, st, X, g.n, g.L, g.R, g.steps, g.nsplit, g.tiles,
                           g.npairs, part, dpart);
    else if (prec == PREC_BF16X3)
        hipLaunchKernelGGL(k_gram_kc<PREC_BF16X3>, dim3(blocks), dim3(256), 0, st, X, g.n, g.L, g.R, g.steps,
                           g.nsplit, g.tiles, g.npairs, part, dpart);
    else
        hipLaunchKernelGGL(k_gram_kc<PREC_F32>, dim3(blocks), dim3(256), 0, st, X, g.n, g.L, g.R, g.steps, g.nsplit,
                           g.tiles, g.npairs, part, dpart);
    return hipGetLastError();
}

hipError_t launch_gram_kc_reduce(const GramKcPlan& g, const float* part, const double* dpart, double* G,
                                 hipStream_t st) {
    const int64_t nbk = ceil_div(g.n, RDB);
    hipLaunchKernelGGL(k_gram_kc_reduce, dim3((unsigned)(nbk * (nbk + 1) / 2)), dim3(256), 0, st, part, dpart,
                       g.nsplit, g.npairs, g.tiles, g.n, G);
    return hipGetLastError();
}

}  // namespace atc
