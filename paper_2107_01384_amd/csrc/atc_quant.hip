// Core quantization and encoding on the GPU: TTHRESH bit-plane truncation
// (Section 3.3), cut into blocks that are encoded independently with a
// breakpoint per block (Section 4.2), with the dequantization correction inside
// the error tracking (Section 4.3).
//
// The error tracking is exact.  Magnitudes q_i = rint(2^k |b_i|) are 64-bit
// integers (2^63 <= 2^k max|b| < 2^64); the squared error of one magnitude
// known down to plane p is a 128-bit integer; sums over the core are 192-bit.
// The target T (in the core's units) is compared as S <= floor(T 2^(2k)),
// which is the exact comparison for an integer S.
//
// Kernels, in launch order (n coefficients, B blocks of `len` coefficients):
//   k_q_init       state words cleared
//   k_q_max        max |b| (bit pattern of the double, atomicMax) + non-finite
//   k_q_planes     per block: q_i (kept in the workspace), and for every plane
//                  p in 0..64 the block's error with all its planes >= p known
//                  (15 partial sums per plane, 1024 threads)
//   k_q_plane_sums one workgroup per plane: the core's error at its end
//   k_q_plane_pick the breakpoint plane P (the first whose end reaches T)
//   k_q_run_start  one workgroup: the error at the start of every block on
//                  plane P (a scan over blocks)
//   k_q_cross      per block: walk of plane P with exact prefix sums, first
//                  position where the running error reaches T (atomicMin)
//   k_q_block_sse  per block: coefficients encoded on plane P, exact error
//   k_q_segment<0> per (block, plane >= P) wavefront: run bytes, sign bits and
//                  trailing bits of that plane's segment of the block
//   k_q_seg_offsets one wavefront per block: segment offsets (scan over planes)
//   k_q_layout     one workgroup: block offsets (scan over blocks), stream
//                  header, final error at the breakpoint, the info record
//   k_q_fill       the stream body cleared (its words are OR-ed into), then
//                  k_q_block_headers
//   k_q_segment<1> per (block, plane) wavefront: the segment's bits and bytes
// Decoding: k_dq_offsets (block offsets from the sizes) and k_dq_decode (one
// wavefront per block: the runs parsed in parallel, then planes in order with
// every coefficient of the block on its own lane, magnitudes in LDS).
#include <cmath>

#include "atc_internal.hpp"

namespace atc {
namespace {

constexpr int QPLANES = 64;
constexpr int32_t QKZERO = INT32_MIN;
constexpr uint32_t QMAGIC = 0x51435441u;   // 'ATCQ'
constexpr int QHEADER = 10;                // stream header words
constexpr int QBLK_HDR = 3;                // block header words
constexpr int QMAX_BLOCK = 4096;           // longest block (decoder keeps it in LDS)
// run bytes of a block of QMAX_BLOCK coefficients: one run per coefficient plus
// a final one per plane, at most 2 bytes each
constexpr int QMAX_RUN_WORDS = (2 * (QMAX_BLOCK + 64) + 3) / 4;

// ------------------------------------------------------------ 192-bit integers
struct U192 {
    uint64_t w0, w1, w2;
};

__device__ __forceinline__ U192 u192_zero() { return U192{0, 0, 0}; }

__device__ __forceinline__ void u192_add(U192& a, const U192& b) {
    const uint64_t s0 = a.w0 + b.w0;
    const uint64_t c0 = s0 < b.w0;
    const uint64_t s1 = a.w1 + b.w1;
    uint64_t c1 = s1 < b.w1;
    const uint64_t s1c = s1 + c0;
    c1 += s1c < c0;
    a.w0 = s0;
    a.w1 = s1c;
    a.w2 = a.w2 + b.w2 + c1;
}

// a - b modulo 2^192
__device__ __forceinline__ void u192_sub(U192& a, const U192& b) {
    const uint64_t d0 = a.w0 - b.w0;
    const uint64_t br0 = a.w0 < b.w0;
    const uint64_t d1 = a.w1 - b.w1;
    uint64_t br1 = a.w1 < b.w1;
    const uint64_t d1b = d1 - br0;
    br1 += d1 < br0;
    a.w0 = d0;
    a.w1 = d1b;
    a.w2 = a.w2 - b.w2 - br1;
}

__device__ __forceinline__ bool u192_le(const U192& a, const U192& b) {
    if (a.w2 != b.w2) return a.w2 < b.w2;
    if (a.w1 != b.w1) return a.w1 < b.w1;
    return a.w0 <= b.w0;
}

__device__ __forceinline__ double u192_to_double(const U192& a) {
    return ldexp((double)a.w2, 128) + ldexp((double)a.w1, 64) + (double)a.w0;
}

// ------------------------------------------------------------ bit-plane values
// Magnitude decoded from the bits of planes >= p (Section 4.3): zero while no
// one-bit is known, else the known bits plus 2^(p-1); nothing is added once
// every bit is known (p = 0).
__device__ __forceinline__ uint64_t dec_mag(uint64_t q, int p) {
    if (p >= QPLANES) return 0;
    const uint64_t hi = p == 0 ? q : (q >> p) << p;
    if (hi == 0) return 0;
    return p >= 1 ? hi + (1ull << (p - 1)) : hi;
}

// Squared error of one magnitude known down to plane p, as a 128-bit value
__device__ __forceinline__ U192 err128(uint64_t q, int p) {
    const uint64_t d = dec_mag(q, p);
    const uint64_t a = q >= d ? q - d : d - q;
    return U192{a * a, __umul64hi(a, a), 0};
}

__device__ __forceinline__ int varint_len(uint32_t v) {
    return v < (1u << 7) ? 1 : v < (1u << 14) ? 2 : v < (1u << 21) ? 3 : v < (1u << 28) ? 4 : 5;
}

__device__ __forceinline__ uint64_t lanemask_lt(int lane) { return lane == 0 ? 0ull : (~0ull >> (64 - lane)); }

// ------------------------------------------------------------ shared state
struct QState {
    unsigned long long maxbits;   // bit pattern of max |b| (positive doubles order as integers)
    unsigned long long first;     // first crossing position on plane P (atomicMin)
    int32_t nonfinite;
    int32_t k;
    int32_t plane;
    int32_t all_bits;             // the target is below zero: every bit is encoded
    int64_t count;
    U192 T;                       // floor(target 2^(2k)) (saturated)
    U192 sse_bp;                  // exact error at the breakpoint
    int64_t total_words;
    int32_t pad[6];
    U192 S[65];                   // the core's error with every plane >= p known, p = 0..64
};

struct QBlk {
    int64_t word_off;             // block start in the stream
    uint32_t nrb, nsb, ntb;       // run bytes, sign bits, trailing bits
    uint32_t count;               // coefficients encoded on plane P
};

struct QWs {
    QState* st;
    uint64_t* q;
    uint8_t* neg;
    U192* part;        // [B][65]
    U192* run_start;   // [B]
    U192* sse_part;    // [B]
    uint32_t* cnt;     // [B][64][3]
    uint32_t* off;     // [B][64][3]
    QBlk* blk;         // [B]
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t carve_quant(int64_t n, int64_t nb, char* base, QWs* w) {
    size_t o = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + o : nullptr;
        o = align256(o + bytes);
        return p;
    };
    QWs t{};
    t.st = (QState*)take(sizeof(QState));
    t.q = (uint64_t*)take((size_t)n * 8);
    t.neg = (uint8_t*)take((size_t)n);
    t.part = (U192*)take((size_t)nb * 65 * sizeof(U192));
    t.run_start = (U192*)take((size_t)nb * sizeof(U192));
    t.sse_part = (U192*)take((size_t)nb * sizeof(U192));
    t.cnt = (uint32_t*)take((size_t)nb * QPLANES * 3 * 4);
    t.off = (uint32_t*)take((size_t)nb * QPLANES * 3 * 4);
    t.blk = (QBlk*)take((size_t)nb * sizeof(QBlk));
    if (w) *w = t;
    return o;
}

// worst case words of one block of m coefficients: header, runs (one per
// coefficient plus a final one per plane, at most 2 bytes each for m <= 4096),
// signs, trailing bits (63 planes at most after the first one-bit)
size_t block_max_words(int64_t m) {
    const size_t run_bytes = (size_t)2 * (m + QPLANES);
    return QBLK_HDR + (run_bytes + 3) / 4 + ((size_t)m + 31) / 32 + ((size_t)QPLANES * m + 31) / 32;
}

// One array of a batch quantized by the same launches: grid slice z of every
// kernel works on job z (arrays of one dtype and block length).
constexpr int QMAX_JOBS = ATC_MAX_DIMS;
struct QJob {
    const void* x;
    int64_t n, nb;
    double target;
    uint32_t* out;
    size_t out_words;
    atc_quant_info* info;
    QWs w;
};
struct QJobs {
    QJob j[QMAX_JOBS];
};

// ------------------------------------------------------------ kernels
__global__ void k_q_init(const QJobs B) {
    QState* st = B.j[blockIdx.z].w.st;
    if (threadIdx.x == 0) {
        st->maxbits = 0;
        st->first = ~0ull;
        st->nonfinite = 0;
        st->k = QKZERO;
        st->plane = QPLANES;
        st->all_bits = 0;
        st->count = 0;
        st->T = u192_zero();
        st->sse_bp = u192_zero();
        st->total_words = 0;
    }
}

template <typename T>
__global__ void k_q_max(const QJobs B) {
    const QJob& J = B.j[blockIdx.z];
    const T* __restrict__ x = (const T*)J.x;
    const int64_t n = J.n;
    QState* st = J.w.st;
    unsigned long long m = 0;
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = fabs((double)x[i]);
        if (!(v <= 1.7976931348623157e308)) bad = 1;
        else m = max(m, (unsigned long long)__double_as_longlong(v));
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long t = __shfl_xor(m, o);
        m = max(m, t);
    }
    // one atomic per workgroup (per-wavefront atomics on the one word
    // serialised at L2: ~80 us for a 2M-coefficient core)
    __shared__ unsigned long long wm[4];
    __shared__ int wb[4];
    const int wave = threadIdx.x >> 6;
    const bool anybad = __ballot(bad) != 0;
    if ((threadIdx.x & 63) == 0) {
        wm[wave] = m;
        wb[wave] = anybad ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long bm = 0;
        int bb = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            bm = max(bm, wm[w]);
            bb |= wb[w];
        }
        if (bm) atomicMax(&st->maxbits, bm);
        if (bb) atomicOr(&st->nonfinite, 1);
    }
}

// k with 2^63 <= 2^k m < 2^64 for the maximum m > 0 (Section 3.3)
__device__ __forceinline__ int32_t scale_of(unsigned long long maxbits) {
    if (maxbits == 0) return QKZERO;
    int e = 0;
    (void)frexp(__longlong_as_double((long long)maxbits), &e);  // m = f 2^e, 1/2 <= f < 1
    return 64 - e;
}

constexpr int PLANES_J = 15;          // partial sums per plane
constexpr int PLANES_THREADS = 1024;  // 65 planes x 15 partial sums (975 threads), 16 wavefronts

template <typename T>
__global__ void __launch_bounds__(PLANES_THREADS) k_q_planes(const QJobs B, int len) {
    __shared__ uint64_t sq[QMAX_BLOCK];
    __shared__ U192 red[PLANES_THREADS];
    const QJob& J = B.j[blockIdx.z];
    const T* __restrict__ x = (const T*)J.x;
    const int64_t n = J.n;
    const QWs w = J.w;
    const int b = blockIdx.x;
    if (b >= J.nb) return;
    const int64_t lo = (int64_t)b * len;
    const int m = (int)min<int64_t>(len, n - lo);
    const int32_t k = scale_of(w.st->maxbits);
    for (int i = threadIdx.x; i < m; i += PLANES_THREADS) {
        const double v = (double)x[lo + i];
        uint64_t q = 0;
        if (k != QKZERO) {
            const double s = rint(ldexp(fabs(v), k));
            q = (uint64_t)s;
        }
        sq[i] = q;
        w.q[lo + i] = q;
        w.neg[lo + i] = v < 0.0 ? 1 : 0;
    }
    __syncthreads();
    // thread (p, j): plane p = tid / PLANES_J, every PLANES_J-th coefficient
    // from j (exact integer sums: the order does not matter)
    const int tid = threadIdx.x;
    U192 acc = u192_zero();
    if (tid < 65 * PLANES_J) {
        const int p = tid / PLANES_J, j = tid - p * PLANES_J;
        for (int i = j; i < m; i += PLANES_J) u192_add(acc, err128(sq[i], p));
    }
    red[tid] = acc;
    __syncthreads();
    if (tid < 65) {
        U192 s = red[PLANES_J * tid];
        for (int j = 1; j < PLANES_J; ++j) u192_add(s, red[PLANES_J * tid + j]);
        w.part[(size_t)b * 65 + tid] = s;
    }
}

// floor(t 2^(2k)) as a saturated 192-bit integer (t >= 0, finite)
__device__ U192 scaled_target(double t, int32_t k) {
    U192 r = u192_zero();
    if (!(t > 0.0)) return r;
    int e = 0;
    const double f = frexp(t, &e);                            // t = f 2^e
    const uint64_t M = (uint64_t)ldexp(f, 53);                // t = M 2^(e - 53)
    const int64_t s = (int64_t)e - 53 + 2 * (int64_t)(k == QKZERO ? 0 : k);
    if (s >= 0) {
        if (s > 192 - 53) return U192{~0ull, ~0ull, ~0ull};   // above every error there is
        const int sh = (int)s;
        if (sh < 64) {
            r.w0 = M << sh;
            r.w1 = sh ? (M >> (64 - sh)) : 0;
        } else if (sh < 128) {
            r.w1 = M << (sh - 64);
            r.w2 = (sh - 64) ? (M >> (128 - sh)) : 0;
        } else {
            r.w2 = M << (sh - 128);
        }
    } else if (s > -64) {
        r.w0 = M >> (int)(-s);
    }
    return r;
}

// Block-wide sum of one U192 per thread in a fixed order (LDS tree).
__device__ U192 block_sum_u192(U192 v, U192* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) u192_add(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    const U192 t = red[0];
    __syncthreads();
    return t;
}

// Workgroup p: the core's error with every plane >= p known, summed over the
// blocks' partials.
__global__ void __launch_bounds__(256) k_q_plane_sums(const QJobs B) {
    __shared__ U192 red[256];
    const int64_t nb = B.j[blockIdx.z].nb;
    const QWs w = B.j[blockIdx.z].w;
    const int p = blockIdx.x;
    U192 s = u192_zero();
    for (int64_t b = threadIdx.x; b < nb; b += 256) u192_add(s, w.part[(size_t)b * 65 + p]);
    const U192 t = block_sum_u192(s, red);
    if (threadIdx.x == 0) w.st->S[p] = t;
}

// One thread: scale, target, breakpoint plane.
__global__ void k_q_plane_pick(const QJobs B) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double target = B.j[blockIdx.z].target;
    QState* st = B.j[blockIdx.z].w.st;
    const int32_t k = scale_of(st->maxbits);
    st->k = k;
    if (st->nonfinite || k == QKZERO) {   // nothing to encode
        st->plane = QPLANES;
        st->count = 0;
        return;
    }
    if (target < 0.0) {                   // every bit
        st->all_bits = 1;
        st->plane = 0;
        return;
    }
    const U192 T = scaled_target(target, k);
    st->T = T;
    if (u192_le(st->S[64], T)) {
        st->plane = QPLANES;
        st->count = 0;
        return;
    }
    for (int p = QPLANES - 1; p >= 0; --p)
        if (u192_le(st->S[p], T)) {
            st->plane = p;
            return;
        }
    st->all_bits = 1;  // cannot happen for T >= 0 (plane 0 ends with no error)
    st->plane = 0;
}

// The error at the start of every block on plane P: S[P + 1] plus the
// exclusive prefix over blocks of (block error at P - block error at P + 1).
// Each thread scans a contiguous run of blocks; the runs' sums are scanned in LDS.
__global__ void __launch_bounds__(256) k_q_run_start(const QJobs B) {
    __shared__ U192 sums[256];
    const int64_t nb = B.j[blockIdx.z].nb;
    const QWs w = B.j[blockIdx.z].w;
    const QState* st = w.st;
    if (st->all_bits || st->plane >= QPLANES) return;
    const int P = st->plane;
    const int64_t per = (nb + 255) / 256;
    const int64_t b0 = min(nb, (int64_t)threadIdx.x * per), b1 = min(nb, b0 + per);
    U192 s = u192_zero();
    for (int64_t b = b0; b < b1; ++b) {
        u192_add(s, w.part[(size_t)b * 65 + P]);
        u192_sub(s, w.part[(size_t)b * 65 + P + 1]);
    }
    sums[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        U192 v = sums[threadIdx.x];
        if ((int)threadIdx.x >= o) u192_add(v, sums[threadIdx.x - o]);
        __syncthreads();
        sums[threadIdx.x] = v;
        __syncthreads();
    }
    U192 run = st->S[P + 1];
    if (threadIdx.x > 0) u192_add(run, sums[threadIdx.x - 1]);
    for (int64_t b = b0; b < b1; ++b) {
        w.run_start[b] = run;
        u192_add(run, w.part[(size_t)b * 65 + P]);
        u192_sub(run, w.part[(size_t)b * 65 + P + 1]);
    }
}

constexpr int CROSS_THREADS = 256;

// First position of plane P where the running error reaches T: every thread
// walks a contiguous piece of its block, the pieces' sums scanned in LDS.
__global__ void __launch_bounds__(CROSS_THREADS) k_q_cross(const QJobs B, int len) {
    __shared__ U192 sums[CROSS_THREADS];
    const QJob& J = B.j[blockIdx.z];
    const int64_t n = J.n;
    const QWs w = J.w;
    const int b = blockIdx.x;
    if (b >= J.nb) return;
    const QState* st = w.st;
    if (st->all_bits || st->plane >= QPLANES) return;
    const int P = st->plane;
    const U192 T = st->T;
    const int64_t lo = (int64_t)b * len;
    const int m = (int)min<int64_t>(len, n - lo);
    const int per = (m + CROSS_THREADS - 1) / CROSS_THREADS;
    const int a0 = min(m, threadIdx.x * per), a1 = min(m, a0 + per);
    U192 s = u192_zero();
    for (int i = a0; i < a1; ++i) {
        const uint64_t q = w.q[lo + i];
        u192_add(s, err128(q, P));
        u192_sub(s, err128(q, P + 1));
    }
    sums[threadIdx.x] = s;
    __syncthreads();
    // inclusive scan (Hillis-Steele), then exclusive by shifting
    for (int o = 1; o < CROSS_THREADS; o <<= 1) {
        U192 v = sums[threadIdx.x];
        if (threadIdx.x >= o) u192_add(v, sums[threadIdx.x - o]);
        __syncthreads();
        sums[threadIdx.x] = v;
        __syncthreads();
    }
    U192 run = w.run_start[b];
    if (threadIdx.x > 0) u192_add(run, sums[threadIdx.x - 1]);
    for (int i = a0; i < a1; ++i) {
        const uint64_t q = w.q[lo + i];
        u192_add(run, err128(q, P));
        u192_sub(run, err128(q, P + 1));
        if (u192_le(run, T)) {
            atomicMin(&w.st->first, (unsigned long long)(lo + i));
            break;
        }
    }
}

// Per block: coefficients encoded on plane P, and the exact error there.
__global__ void __launch_bounds__(256) k_q_block_sse(const QJobs B, int len) {
    __shared__ U192 red[256];
    const QJob& J = B.j[blockIdx.z];
    const int64_t n = J.n;
    const QWs w = J.w;
    const QState* st = w.st;
    const int b = blockIdx.x;
    if (b >= J.nb) return;
    const int64_t lo = (int64_t)b * len;
    const int m = (int)min<int64_t>(len, n - lo);
    const int P = st->plane;
    int64_t count;
    if (st->all_bits) count = n;
    else if (P >= QPLANES) count = 0;
    else count = (int64_t)st->first + 1;
    const int cb = (int)min<int64_t>(max<int64_t>(count - lo, 0), m);
    U192 s = u192_zero();
    for (int i = threadIdx.x; i < m; i += 256) u192_add(s, err128(w.q[lo + i], i < cb ? P : P + 1));
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) u192_add(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        w.sse_part[b] = red[0];
        w.blk[b].count = (uint32_t)cb;
    }
}

// One wavefront per (block, plane): the plane's segment of the block.
// WRITE = false counts run bytes / sign bits / trailing bits; WRITE = true
// ORs them into the stream at the offsets k_q_layout computed.
template <bool WRITE>
__global__ void __launch_bounds__(64) k_q_segment(const QJobs B, int len) {
    const QJob& J = B.j[blockIdx.z];
    const int64_t n = J.n;
    const QWs w = J.w;
    uint32_t* __restrict__ out = J.out;
    const QState* st = w.st;
    const int b = blockIdx.x;
    if (b >= J.nb) return;
    if (WRITE && (size_t)st->total_words > J.out_words) return;
    const int p = QPLANES - 1 - (int)blockIdx.y;
    const int P = st->plane;
    const int lane = threadIdx.x;
    uint32_t* c = w.cnt + ((size_t)b * QPLANES + p) * 3;
    if (p < P || P >= QPLANES) {
        if (!WRITE && lane == 0) c[0] = c[1] = c[2] = 0;
        return;
    }
    const int64_t lo = (int64_t)b * len;
    const int m = (int)min<int64_t>(len, n - lo);
    const int upto = p == P ? (int)w.blk[b].count : m;
    uint32_t run_pos = 0, sign_pos = 0, trail_pos = 0;   // within this segment
    uint32_t* runs = nullptr;
    uint32_t* signs = nullptr;
    uint32_t* trail = nullptr;
    uint32_t rbase = 0, sbase = 0, tbase = 0;
    if (WRITE) {
        const QBlk bk = w.blk[b];
        const uint32_t* o = w.off + ((size_t)b * QPLANES + p) * 3;
        uint32_t* blk = out + bk.word_off;
        runs = blk + QBLK_HDR;
        signs = runs + (bk.nrb + 3) / 4;
        trail = signs + (bk.nsb + 31) / 32;
        rbase = o[0];
        sbase = o[1];
        tbase = o[2];
    }
    uint32_t zeros = 0;
    bool any_lead = false;
    for (int c0 = 0; c0 < upto; c0 += 64) {
        const int i = c0 + lane;
        const bool valid = i < upto;
        const uint64_t q = valid ? w.q[lo + i] : 0;
        const bool sig = p < QPLANES - 1 && (q >> (p + 1)) != 0;
        const bool bit = (q >> p) & 1;
        const bool lead = valid && !sig;
        const bool one = lead && bit;
        const bool tr = valid && sig;
        const uint64_t lmask = __ballot(lead), omask = __ballot(one), tmask = __ballot(tr);
        const uint64_t lt = lanemask_lt(lane);
        // run ending at this lane's one-bit: zeros since the previous one-bit
        uint32_t run = 0;
        if (one) {
            const uint32_t my_rank = __popcll(lmask & lt);
            const uint64_t prev = omask & lt;
            if (prev) {
                const int pl = 63 - __clzll(prev);
                run = my_rank - (uint32_t)__popcll(lmask & lanemask_lt(pl)) - 1;
            } else {
                run = zeros + my_rank;
            }
        }
        const int vl = one ? varint_len(run) : 0;
        const uint64_t m2 = __ballot(vl >= 2), m3 = __ballot(vl >= 3), m4 = __ballot(vl >= 4), m5 = __ballot(vl >= 5);
        const uint32_t chunk_bytes = __popcll(omask) + __popcll(m2) + __popcll(m3) + __popcll(m4) + __popcll(m5);
        if (WRITE) {
            if (one) {
                uint32_t pos = rbase + run_pos + __popcll(omask & lt) + __popcll(m2 & lt) + __popcll(m3 & lt) +
                               __popcll(m4 & lt) + __popcll(m5 & lt);
                uint32_t v = run;
                for (int j = 0; j < vl; ++j, ++pos) {
                    const uint32_t byte = (v & 0x7Fu) | (j + 1 < vl ? 0x80u : 0u);
                    v >>= 7;
                    if (byte) atomicOr(&runs[pos >> 2], byte << (8 * (pos & 3)));
                }
                if (w.neg[lo + i]) {
                    const uint32_t sp = sbase + sign_pos + __popcll(omask & lt);
                    atomicOr(&signs[sp >> 5], 1u << (sp & 31));
                }
            }
            if (tr && bit) {
                const uint32_t tp = tbase + trail_pos + __popcll(tmask & lt);
                atomicOr(&trail[tp >> 5], 1u << (tp & 31));
            }
        }
        run_pos += chunk_bytes;
        sign_pos += __popcll(omask);
        trail_pos += __popcll(tmask);
        if (lmask) any_lead = true;
        if (omask) {
            const int last = 63 - __clzll(omask);
            zeros = __popcll(lmask) - __popcll(lmask & lanemask_lt(last)) - 1;
        } else {
            zeros += __popcll(lmask);
        }
    }
    if (any_lead) {   // the zeros after the last one-bit of the plane
        const int vl = varint_len(zeros);
        if (WRITE && lane == 0) {
            uint32_t pos = rbase + run_pos;
            uint32_t v = zeros;
            for (int j = 0; j < vl; ++j, ++pos) {
                const uint32_t byte = (v & 0x7Fu) | (j + 1 < vl ? 0x80u : 0u);
                v >>= 7;
                if (byte) atomicOr(&runs[pos >> 2], byte << (8 * (pos & 3)));
            }
        }
        run_pos += vl;
    }
    if (!WRITE && lane == 0) {
        c[0] = run_pos;
        c[1] = sign_pos;
        c[2] = trail_pos;
    }
}

// One wavefront per block: segment offsets within the block's three fields,
// planes 63 .. P in that order (lane l holds plane 63 - l), and the block's
// field sizes.
__global__ void __launch_bounds__(64) k_q_seg_offsets(const QJobs B) {
    const QWs w = B.j[blockIdx.z].w;
    const int P = w.st->plane;
    const int b = blockIdx.x;
    if (b >= B.j[blockIdx.z].nb) return;
    const int lane = threadIdx.x;
    const int p = QPLANES - 1 - lane;
    const uint32_t* c = w.cnt + ((size_t)b * QPLANES + p) * 3;
    uint32_t v[3] = {0, 0, 0};
    if (p >= P) {
        v[0] = c[0];
        v[1] = c[1];
        v[2] = c[2];
    }
    uint32_t* o = w.off + ((size_t)b * QPLANES + p) * 3;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        // inclusive scan over lanes (planes from the top)
        uint32_t x = v[f];
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d);
            if (lane >= d) x += y;
        }
        o[f] = x - v[f];
        const uint32_t tot = __shfl(x, 63);
        if (lane == 0) {
            if (f == 0) w.blk[b].nrb = tot;
            if (f == 1) w.blk[b].nsb = tot;
            if (f == 2) w.blk[b].ntb = tot;
        }
    }
}

__device__ __forceinline__ int64_t block_words(const QBlk& bk) {
    return QBLK_HDR + (bk.nrb + 3) / 4 + (bk.nsb + 31) / 32 + (bk.ntb + 31) / 32;
}

// One workgroup: block word offsets (scan over blocks), the exact error at
// the breakpoint (sum over blocks), the stream header and block sizes, the
// caller's info record.
__global__ void __launch_bounds__(256) k_q_layout(const QJobs B, int len) {
    __shared__ int64_t wsum[256];
    __shared__ U192 red[256];
    const QJob& J = B.j[blockIdx.z];
    const int64_t n = J.n, nb = J.nb;
    const QWs w = J.w;
    uint32_t* __restrict__ out = J.out;
    const size_t out_words = J.out_words;
    atc_quant_info* info = J.info;
    const QState* st = w.st;
    const int P = st->plane;
    const int64_t per = (nb + 255) / 256;
    const int64_t b0 = min(nb, (int64_t)threadIdx.x * per), b1 = min(nb, b0 + per);
    int64_t mine = 0;
    U192 sse = u192_zero();
    for (int64_t b = b0; b < b1; ++b) {
        mine += block_words(w.blk[b]);
        u192_add(sse, w.sse_part[b]);
    }
    wsum[threadIdx.x] = mine;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int64_t v = wsum[threadIdx.x] + ((int)threadIdx.x >= o ? wsum[threadIdx.x - o] : 0);
        __syncthreads();
        wsum[threadIdx.x] = v;
        __syncthreads();
    }
    const int64_t total = QHEADER + 2 * nb + wsum[255];
    int64_t pos = QHEADER + 2 * nb + (threadIdx.x > 0 ? wsum[threadIdx.x - 1] : 0);
    const bool fits = (size_t)total <= out_words;
    for (int64_t b = b0; b < b1; ++b) {
        QBlk& bk = w.blk[b];
        const int64_t words = block_words(bk);
        bk.word_off = pos;
        pos += words;
        if (fits) {
            out[QHEADER + 2 * b] = (uint32_t)(uint64_t)words;
            out[QHEADER + 2 * b + 1] = (uint32_t)((uint64_t)words >> 32);
        }
    }
    const U192 sse_all = block_sum_u192(sse, red);
    if (threadIdx.x != 0) return;
    QState* stw = w.st;
    int64_t count;
    if (st->all_bits) count = n;
    else if (P >= QPLANES) count = 0;
    else count = (int64_t)st->first + 1;
    stw->count = count;
    stw->sse_bp = sse_all;
    stw->total_words = total;
    const int32_t k = st->k;
    if (fits) {
        out[0] = QMAGIC;
        out[1] = (uint32_t)k;
        out[2] = (uint32_t)P;
        out[3] = (uint32_t)len;
        out[4] = (uint32_t)(uint64_t)n;
        out[5] = (uint32_t)((uint64_t)n >> 32);
        out[6] = (uint32_t)(uint64_t)count;
        out[7] = (uint32_t)((uint64_t)count >> 32);
        out[8] = (uint32_t)(uint64_t)nb;
        out[9] = (uint32_t)((uint64_t)nb >> 32);
    }
    if (info) {
        info->status = st->nonfinite ? ATC_ERR_NONFINITE_INPUT : fits ? ATC_OK : ATC_ERR_WORKSPACE_TOO_SMALL;
        info->k = k;
        info->plane = P;
        info->block_len = len;
        info->n = n;
        info->count = count;
        info->nblocks = nb;
        info->words = total;
        const double s_units = u192_to_double(sse_all);
        info->sse = (k == QKZERO || st->nonfinite) ? 0.0 : ldexp(s_units, -2 * k);
        info->pad = 0;
    }
}

// Clears the block area of the stream; the block headers are written here.
__global__ void k_q_fill(const QJobs B) {
    const QJob& J = B.j[blockIdx.z];
    uint32_t* __restrict__ out = J.out;
    const int64_t total = J.w.st->total_words;
    if ((size_t)total > J.out_words) return;
    const int64_t start = QHEADER + 2 * J.nb;
    for (int64_t i = start + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = 0;
}

__global__ void k_q_block_headers(const QJobs B) {
    const QJob& J = B.j[blockIdx.z];
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= J.nb || (size_t)J.w.st->total_words > J.out_words) return;
    const QBlk bk = J.w.blk[b];
    uint32_t* h = J.out + bk.word_off;
    h[0] = bk.nrb;
    h[1] = bk.nsb;
    h[2] = bk.ntb;
}

// ------------------------------------------------------------ decoding
// One stream of a batch decoded by the same launches (grid slice z = job z).
struct DJob {
    const uint32_t* in;
    int64_t n, nb;
    int64_t* boff;
    void* out;
    int32_t* status;
};
struct DJobs {
    DJob j[QMAX_JOBS];
};

// Block offsets from the recorded sizes (scan over blocks in one workgroup),
// after checking the header against the caller's n and block length (a
// mismatch marks every block unreadable).
__global__ void __launch_bounds__(256) k_dq_offsets(const DJobs B, int len) {
    __shared__ int64_t wsum[256];
    const DJob& J = B.j[blockIdx.z];
    const uint32_t* __restrict__ in = J.in;
    const int64_t n = J.n, nb = J.nb;
    int64_t* boff = J.boff;
    int32_t* status = J.status;
    const uint64_t hn = (uint64_t)in[4] | ((uint64_t)in[5] << 32);
    const uint64_t hnb = (uint64_t)in[8] | ((uint64_t)in[9] << 32);
    const bool ok = in[0] == QMAGIC && in[3] == (uint32_t)len && hn == (uint64_t)n && hnb == (uint64_t)nb &&
                    in[2] <= (uint32_t)QPLANES;
    const int64_t per = (nb + 255) / 256;
    const int64_t b0 = min(nb, (int64_t)threadIdx.x * per), b1 = min(nb, b0 + per);
    int64_t mine = 0;
    if (ok)
        for (int64_t b = b0; b < b1; ++b)
            mine += (int64_t)((uint64_t)in[QHEADER + 2 * b] | ((uint64_t)in[QHEADER + 2 * b + 1] << 32));
    wsum[threadIdx.x] = mine;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int64_t v = wsum[threadIdx.x] + ((int)threadIdx.x >= o ? wsum[threadIdx.x - o] : 0);
        __syncthreads();
        wsum[threadIdx.x] = v;
        __syncthreads();
    }
    int64_t pos = QHEADER + 2 * nb + (threadIdx.x > 0 ? wsum[threadIdx.x - 1] : 0);
    for (int64_t b = b0; b < b1; ++b) {
        boff[b] = ok ? pos : -1;
        if (ok) pos += (int64_t)((uint64_t)in[QHEADER + 2 * b] | ((uint64_t)in[QHEADER + 2 * b + 1] << 32));
    }
    if (!ok && threadIdx.x == 0 && status) atomicOr(status, 2);
}

__device__ __forceinline__ uint32_t read_byte(const uint32_t* __restrict__ w, uint32_t i) {
    return (w[i >> 2] >> (8 * (i & 3))) & 0xFFu;
}
__device__ __forceinline__ uint32_t read_bit(const uint32_t* __restrict__ w, uint32_t i) {
    return (w[i >> 5] >> (i & 31)) & 1u;
}

// Inclusive sum over lanes 0 .. lane of a wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

constexpr int QMAX_WORDS = QMAX_BLOCK / 64;        // significance words of the longest block
constexpr int QMAX_RUNS = QMAX_BLOCK + QPLANES;    // a run per one-bit of a leading position, a final one per plane

// One wavefront per block, every step parallel over the block:
//  * the run bytes are parsed at once: lane j looks at byte j of a 64-byte
//    window, a byte with its top bit clear ends a run, whose value is read
//    back from the bytes after the previous end; the prefix sums B_k of
//    (run_k + 1) go to LDS, so the k-th run of a plane ends at leading rank
//    B_k - B_(start - 1) - 1, a one-bit when below the plane's count of
//    leading positions and the plane's last run when equal to it;
//  * per plane, lane w takes significance word w (coefficients 64 w ..
//    64 w + 63) for the counts and their prefix over words; the plane's
//    one-bits, as ranks among its leading positions, become a bit mask;
//    then lane l takes coefficient 64 w + l of every word w: a significant
//    one reads its trailing bit at (bits so far) + (its rank among the
//    significant), a leading one looks its rank up in the mask, and a
//    one-bit there also takes the next sign bits in rank order.
// The magnitudes stay in registers (MAXW 64-bit words per lane: coefficient
// 64 w + lane in word w, MAXW >= len / 64), and so do the per-word state
// (lane w holds word w's significance and sign masks, read by every lane with
// readlane), so the words of a plane carry no LDS dependence on each other;
// the values (Section 4.3) are scaled by 2^-k at the end.
constexpr int DQ_WAVES = 4;   // wavefronts per decoded block

template <typename T, int MAXW>
__global__ void __launch_bounds__(64 * DQ_WAVES) k_dq_decode(const DJobs B, int len) {
    constexpr int MW = MAXW / DQ_WAVES;             // words per wavefront (word w = DQ_WAVES j + wave)
    __shared__ uint32_t runs_lds[QMAX_RUN_WORDS];   // the block's run bytes
    __shared__ uint32_t signs_lds[QMAX_BLOCK / 32];  // its sign bits (one per coefficient at most)
    __shared__ uint32_t bsum[QMAX_RUNS];             // B_k = sum over runs i <= k of (run_i + 1)
    __shared__ uint64_t onew[QMAX_WORDS];            // this plane's one-bits by leading rank
    __shared__ uint64_t sigw[QMAX_WORDS];            // coefficients with a decoded one-bit, by word
    __shared__ uint32_t tplane[QMAX_BLOCK / 32 + 2];  // this plane's trailing bits, from bit tpos & ~31
    __shared__ uint32_t sh_nruns, sh_rk, sh_nones;
    __shared__ int sh_bad;
    const DJob& J = B.j[blockIdx.z];
    const uint32_t* __restrict__ in = J.in;
    const int64_t n = J.n;
    const int64_t* __restrict__ boff = J.boff;
    T* __restrict__ out = (T*)J.out;
    int32_t* status = J.status;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int b = blockIdx.x;
    if (b >= J.nb) return;
    if (boff[b] < 0) {   // header did not match: zeros
        for (int64_t i = (int64_t)b * len + tid; i < min<int64_t>(n, (int64_t)(b + 1) * len); i += 64 * DQ_WAVES)
            out[i] = (T)0;
        return;
    }
    const int32_t k = (int32_t)in[1];
    const int P = (int)in[2];
    const int64_t count = (int64_t)((uint64_t)in[6] | ((uint64_t)in[7] << 32));
    const int64_t lo = (int64_t)b * len;
    const int m = (int)min<int64_t>(len, n - lo);
    const int cb = (int)min<int64_t>(max<int64_t>(count - lo, 0), m);
    const int nw = (m + 63) / 64;   // <= MAXW (the launch picks MAXW from len)
    // registers: mag[j] = magnitude of coefficient 64 w + lane of word
    // w = DQ_WAVES j + wave; ng_l (lane w of w's wavefront) its sign mask
    uint64_t mag[MW];
#pragma unroll
    for (int j = 0; j < MW; ++j) mag[j] = 0;
    uint64_t ng_l = 0;
    const uint64_t bwords = (uint64_t)in[QHEADER + 2 * b] | ((uint64_t)in[QHEADER + 2 * b + 1] << 32);
    const uint32_t* blk = in + boff[b];
    const uint32_t nrb = blk[0], nsb = blk[1], ntb = blk[2];
    const uint32_t* runs_g = blk + QBLK_HDR;
    const uint32_t* signs = runs_g + (nrb + 3) / 4;
    const uint32_t* trail = signs + (nsb + 31) / 32;
    bool bad = (nrb + 3) / 4 > (uint32_t)QMAX_RUN_WORDS || (nsb + 31) / 32 > (uint32_t)(QMAX_BLOCK / 32) ||
               (uint64_t)QBLK_HDR + (nrb + 3) / 4 + (nsb + 31) / 32 + ((uint64_t)ntb + 31) / 32 > bwords;
    if (!bad) {
        for (uint32_t i = tid; i < (nrb + 3) / 4; i += 64 * DQ_WAVES) runs_lds[i] = runs_g[i];
        for (uint32_t i = tid; i < (nsb + 31) / 32; i += 64 * DQ_WAVES) signs_lds[i] = signs[i];
    }
    if (tid < QMAX_WORDS) sigw[tid] = 0;
    __syncthreads();
    // the runs (wavefront 0): B_k for k < nruns
    if (wave == 0) {
        uint32_t nruns = 0, carry = 0;
        int prev_end = -1;
        for (uint32_t c0 = 0; c0 < nrb && !bad; c0 += 64) {
            const uint32_t j = c0 + lane;
            const bool inb = j < nrb;
            const uint32_t byte = inb ? read_byte(runs_lds, j) : 0u;
            const bool end = inb && !(byte & 0x80u);
            const uint64_t em = __ballot(end);
            const uint64_t below = em & lanemask_lt(lane);
            const int start = below ? (int)(c0 + 63 - __clzll(below)) + 1 : prev_end + 1;
            uint32_t v = 0;
            bool over = false;
            if (end) {
                const int L = (int)j - start + 1;
                if (L > 5) over = true;
                else
                    for (int t = 0; t < L; ++t) v |= (read_byte(runs_lds, (uint32_t)(start + t)) & 0x7Fu) << (7 * t);
            }
            const uint32_t kk = nruns + (uint32_t)__popcll(below);
            if (end && kk >= (uint32_t)QMAX_RUNS) over = true;
            if (__ballot(over)) {
                bad = true;
                break;
            }
            const uint32_t x = wave_incl_scan(end ? v + 1 : 0u, lane);
            if (end) bsum[kk] = carry + x;
            carry += __shfl(x, 63);
            nruns += (uint32_t)__popcll(em);
            if (em) prev_end = (int)(c0 + 63 - __clzll(em));
        }
        if (nrb > 0 && prev_end != (int)nrb - 1) bad = true;   // an unterminated last run
        if (lane == 0) {
            sh_nruns = nruns;
            sh_bad = bad ? 1 : 0;
        }
    }
    __syncthreads();
    const uint32_t nruns = sh_nruns;
    bad = sh_bad != 0;
    uint32_t rk = 0, spos = 0, tpos = 0;
    const uint64_t me = 1ull << lane, lt = me - 1;
    for (int p = QPLANES - 1; p >= P && k != QKZERO && !bad; --p) {
        const int upto = p == P ? cb : m;
        // every wavefront: word `lane`'s significant and leading positions
        // below upto and their prefix counts over the words before it
        const uint64_t sw_l = lane < nw ? sigw[lane] : 0ull;
        uint64_t sw = 0, lw = 0;
        if (lane < nw) {
            const int c = min(64, max(0, upto - 64 * lane));
            const uint64_t vm = c >= 64 ? ~0ull : ((1ull << c) - 1);
            sw = sw_l & vm;
            lw = ~sw_l & vm;
        }
        const uint32_t cs = (uint32_t)__popcll(sw), cl = (uint32_t)__popcll(lw);
        const uint32_t isig = wave_incl_scan(cs, lane), ilead = wave_incl_scan(cl, lane);
        const uint32_t nsig = __shfl(isig, 63), nlead = __shfl(ilead, 63);
        const uint32_t sigpre_l = isig - cs, leadpre_l = ilead - cl;
        if (tpos + nsig > ntb) {
            bad = true;   // the same in every wavefront
            break;
        }
        if (tid < nw) onew[tid] = 0;
        {
            const uint32_t tw = ((tpos & 31u) + nsig + 31u) >> 5;   // at most QMAX_BLOCK / 32 + 1
            for (uint32_t i = tid; i < tw; i += 64 * DQ_WAVES) tplane[i] = trail[(tpos >> 5) + i];
        }
        __syncthreads();
        // this plane's runs (wavefront 0): one-bits at the leading ranks below
        // nlead, then the final run
        if (wave == 0) {
            uint32_t nones = 0;
            bool wbad = false;
            if (nlead > 0) {
                const uint32_t base = rk > 0 ? bsum[rk - 1] : 0u;
                bool found = false;
                for (uint32_t c0 = rk; !found; c0 += 64) {
                    if (c0 >= nruns) {
                        wbad = true;
                        break;
                    }
                    const uint32_t kk = c0 + lane;
                    const bool inr = kk < nruns;
                    const uint32_t val = inr ? bsum[kk] - base - 1u : 0u;
                    const uint64_t endm = __ballot(inr && val == nlead);
                    const uint64_t overm = __ballot(inr && val > nlead);
                    const int le = endm ? __ffsll((long long)endm) - 1 : 64;
                    const int lov = overm ? __ffsll((long long)overm) - 1 : 64;
                    if (lov < le) {
                        wbad = true;
                        break;
                    }
                    const bool one = inr && lane < le && val < nlead;
                    if (one) atomicOr((unsigned long long*)&onew[val >> 6], 1ull << (val & 63));
                    nones += (uint32_t)__popcll(__ballot(one));
                    if (endm) {
                        found = true;
                        rk = c0 + (uint32_t)le + 1;
                    }
                }
                if (!wbad && spos + nones > nsb) wbad = true;
            }
            if (lane == 0) {
                sh_nones = nones;
                sh_rk = rk;
                sh_bad = wbad ? 1 : 0;
            }
        }
        __syncthreads();
        const uint32_t nones = sh_nones;
        rk = sh_rk;
        if (sh_bad) {
            bad = true;
            break;
        }
        // one-bits of the words before each word of onew (lane w: word w)
        const uint64_t onew_l = lane < nw ? onew[lane] : 0ull;
        const uint32_t co = (uint32_t)__popcll(onew_l);
        const uint32_t onepre_l = wave_incl_scan(co, lane) - co;
        const uint32_t tb0 = tpos & 31u;
        // this wavefront's words; lane l, word w: coefficient 64 w + l.  A
        // significant one reads its trailing bit at (bits so far) + (its rank
        // among the significant); a leading one looks its rank a up in onew,
        // and a one-bit there takes the next sign bit in rank order.
        uint64_t sw_own = sw_l;   // lane w of word w's wavefront: its updated mask
#pragma unroll
        for (int j = 0; j < MW; ++j) {
            const int w = DQ_WAVES * j + wave;
            if (w < nw) {
                const int c = min(64, max(0, upto - 64 * w));
                const uint64_t vm = c >= 64 ? ~0ull : ((1ull << c) - 1);
                const uint64_t sg = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(sw_l >> 32), w) << 32) |
                                    (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)sw_l, w);
                const uint32_t sp = (uint32_t)__builtin_amdgcn_readlane((int)sigpre_l, w);
                const uint32_t lp = (uint32_t)__builtin_amdgcn_readlane((int)leadpre_l, w);
                const bool valid = (vm & me) != 0;
                const bool is_sig = (sg & me) != 0;
                const uint32_t a = lp + (uint32_t)__popcll(~sg & vm & lt);
                const uint32_t ai = min(a >> 6, (uint32_t)(QMAX_WORDS - 1));
                const uint32_t op = (uint32_t)__shfl((int)onepre_l, (int)ai);   // every lane takes part
                bool setbit = false, becomes = false, negative = false;
                if (valid && is_sig) {
                    const uint32_t rho = sp + (uint32_t)__popcll(sg & vm & lt);
                    setbit = read_bit(tplane, tb0 + rho) != 0;
                } else if (valid) {
                    const uint64_t ow = onew[ai];
                    if ((ow >> (a & 63)) & 1ull) {
                        setbit = true;
                        becomes = true;
                        const uint32_t si = spos + op + (uint32_t)__popcll(ow & ((1ull << (a & 63)) - 1));
                        negative = read_bit(signs_lds, si) != 0;
                    }
                }
                if (setbit) mag[j] |= 1ull << p;
                const uint64_t nbm = __ballot(becomes), ngm = __ballot(negative);
                if (lane == w) {
                    sw_own |= nbm;
                    ng_l |= ngm;
                }
            }
        }
        // the new significance masks of this wavefront's words, for the next plane
        if (lane < nw && (lane % DQ_WAVES) == wave) sigw[lane] = sw_own;
        tpos += nsig;
        spos += nones;
        __syncthreads();
    }
    if (!bad && k != QKZERO && P < QPLANES && (rk != nruns || spos != nsb || tpos != ntb)) bad = true;
    if (bad && tid == 0 && status) atomicOr(status, 1);
#pragma unroll
    for (int j = 0; j < MW; ++j) {
        const int w = DQ_WAVES * j + wave;
        const int i = 64 * w + lane;
        const uint64_t ngw = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(ng_l >> 32), w) << 32) |
                             (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)ng_l, w);
        if (w < nw && i < m) {
            double v = 0.0;
            if (k != QKZERO) {
                const int lowp = i < cb ? P : P + 1;
                const uint64_t d = dec_mag(mag[j], lowp);
                if (d) {
                    v = ldexp((double)d, -k);
                    if ((ngw >> lane) & 1ull) v = -v;
                }
            }
            out[lo + i] = (T)v;
        }
    }
}

// ------------------------------------------------------------ host side
int64_t quant_nblocks(int64_t n, int len) { return (n + len - 1) / len; }

size_t quant_workspace_bytes(int64_t n, int len) { return carve_quant(n, quant_nblocks(n, len), nullptr, nullptr); }

size_t quant_max_words(int64_t n, int len) {
    const int64_t nb = quant_nblocks(n, len);
    return (size_t)QHEADER + 2 * (size_t)nb + (size_t)nb * block_max_words(len);
}

// The kernels over jobs 0 .. count - 1 (one dtype, one block length); the
// x extent of every grid is the largest job's, the surplus workgroups of the
// smaller jobs return at once.
hipError_t launch_quantize_jobs(const QJobs& B, int count, int f64, int len, hipStream_t st) {
    int64_t maxn = 1, maxnb = 1;
    size_t maxout = 1;
    for (int z = 0; z < count; ++z) {
        maxn = std::max(maxn, B.j[z].n);
        maxnb = std::max(maxnb, B.j[z].nb);
        maxout = std::max(maxout, B.j[z].out_words);
    }
    const unsigned Z = (unsigned)count, nb = (unsigned)maxnb;
    hipLaunchKernelGGL(k_q_init, dim3(1, 1, Z), dim3(64), 0, st, B);
    const unsigned gmax = (unsigned)std::min<int64_t>(256, std::max<int64_t>(1, ceil_div(maxn, 256)));
    if (f64) hipLaunchKernelGGL(k_q_max<double>, dim3(gmax, 1, Z), dim3(256), 0, st, B);
    else hipLaunchKernelGGL(k_q_max<float>, dim3(gmax, 1, Z), dim3(256), 0, st, B);
    if (f64) hipLaunchKernelGGL(k_q_planes<double>, dim3(nb, 1, Z), dim3(PLANES_THREADS), 0, st, B, len);
    else hipLaunchKernelGGL(k_q_planes<float>, dim3(nb, 1, Z), dim3(PLANES_THREADS), 0, st, B, len);
    hipLaunchKernelGGL(k_q_plane_sums, dim3(65, 1, Z), dim3(256), 0, st, B);
    hipLaunchKernelGGL(k_q_plane_pick, dim3(1, 1, Z), dim3(64), 0, st, B);
    hipLaunchKernelGGL(k_q_run_start, dim3(1, 1, Z), dim3(256), 0, st, B);
    hipLaunchKernelGGL(k_q_cross, dim3(nb, 1, Z), dim3(CROSS_THREADS), 0, st, B, len);
    hipLaunchKernelGGL(k_q_block_sse, dim3(nb, 1, Z), dim3(256), 0, st, B, len);
    hipLaunchKernelGGL(k_q_segment<false>, dim3(nb, QPLANES, Z), dim3(64), 0, st, B, len);
    hipLaunchKernelGGL(k_q_seg_offsets, dim3(nb, 1, Z), dim3(64), 0, st, B);
    hipLaunchKernelGGL(k_q_layout, dim3(1, 1, Z), dim3(256), 0, st, B, len);
    const unsigned gfill = (unsigned)std::min<size_t>(4096, std::max<size_t>(1, (maxout + 255) / 256));
    hipLaunchKernelGGL(k_q_fill, dim3(gfill, 1, Z), dim3(256), 0, st, B);
    hipLaunchKernelGGL(k_q_block_headers, dim3((unsigned)ceil_div(maxnb, 256), 1, Z), dim3(256), 0, st, B);
    hipLaunchKernelGGL(k_q_segment<true>, dim3(nb, QPLANES, Z), dim3(64), 0, st, B, len);
    return hipGetLastError();
}

size_t dequant_workspace_bytes(int64_t n, int len) { return align256((size_t)quant_nblocks(n, len) * 8); }

hipError_t launch_dequantize_jobs(const DJobs& B, int count, int f64, int len, hipStream_t st) {
    int64_t maxnb = 1;
    for (int z = 0; z < count; ++z) maxnb = std::max(maxnb, B.j[z].nb);
    const unsigned Z = (unsigned)count;
    hipLaunchKernelGGL(k_dq_offsets, dim3(1, 1, Z), dim3(256), 0, st, B, len);
    const dim3 grid((unsigned)maxnb, 1, Z);
    if (len <= 1024) {
        if (f64) hipLaunchKernelGGL((k_dq_decode<double, 16>), grid, dim3(64 * DQ_WAVES), 0, st, B, len);
        else hipLaunchKernelGGL((k_dq_decode<float, 16>), grid, dim3(64 * DQ_WAVES), 0, st, B, len);
    } else {
        if (f64) hipLaunchKernelGGL((k_dq_decode<double, QMAX_WORDS>), grid, dim3(64 * DQ_WAVES), 0, st, B, len);
        else hipLaunchKernelGGL((k_dq_decode<float, QMAX_WORDS>), grid, dim3(64 * DQ_WAVES), 0, st, B, len);
    }
    return hipGetLastError();
}

QJob quant_job(const QuantTask& t, int len) {
    QJob j{};
    j.x = t.x;
    j.n = t.n;
    j.nb = quant_nblocks(t.n, len);
    j.target = t.target;
    j.out = t.enc;
    j.out_words = t.enc_words;
    j.info = t.info;
    carve_quant(t.n, j.nb, (char*)t.ws, &j.w);
    return j;
}

DJob dequant_job(const DequantTask& t, int len) {
    return DJob{t.enc, t.n, quant_nblocks(t.n, len), (int64_t*)t.ws, t.out, t.status};
}

}  // namespace

hipError_t quantize_batch(const QuantTask* tasks, int count, int f64, int len, hipStream_t st) {
    if (count < 1 || count > QMAX_JOBS) return hipErrorInvalidValue;
    QJobs B{};
    for (int z = 0; z < count; ++z) B.j[z] = quant_job(tasks[z], len);
    return launch_quantize_jobs(B, count, f64, len, st);
}

hipError_t dequantize_batch(const DequantTask* tasks, int count, int f64, int len, hipStream_t st) {
    if (count < 1 || count > QMAX_JOBS) return hipErrorInvalidValue;
    DJobs B{};
    for (int z = 0; z < count; ++z) B.j[z] = dequant_job(tasks[z], len);
    return launch_dequantize_jobs(B, count, f64, len, st);
}

}  // namespace atc

// ------------------------------------------------------------ C ABI
using namespace atc;

namespace {
atc_status qfail(atc_status s, const char* msg) {
    set_last_error(msg);
    return s;
}
atc_status check_quant_args(int64_t n, int32_t block_len) {
    if (n < 1) return qfail(ATC_ERR_INVALID_ARGUMENT, "n must be >= 1");
    if (block_len < 1 || block_len > QMAX_BLOCK) return qfail(ATC_ERR_UNSUPPORTED, "block_len must lie in [1, 4096]");
    if (quant_nblocks(n, block_len) > (int64_t)UINT32_MAX) return qfail(ATC_ERR_UNSUPPORTED, "too many blocks");
    return ATC_OK;
}
}  // namespace

extern "C" {

size_t atc_quantize_max_words(int64_t n, int32_t block_len) {
    if (n < 1 || block_len < 1 || block_len > QMAX_BLOCK) return 0;
    return quant_max_words(n, block_len);
}

size_t atc_quantize_workspace_size(int64_t n, int32_t block_len) {
    if (n < 1 || block_len < 1 || block_len > QMAX_BLOCK) return 0;
    return quant_workspace_bytes(n, block_len);
}

atc_status atc_quantize_core(const void* core, int32_t dtype, int64_t n, double target_sse, int32_t block_len,
                             uint32_t* enc, size_t enc_words, atc_quant_info* info, void* workspace,
                             size_t workspace_bytes, void* stream) {
    atc_status s = check_quant_args(n, block_len);
    if (s != ATC_OK) return s;
    if (!core || !enc || !info || !workspace) return qfail(ATC_ERR_INVALID_ARGUMENT, "core, enc, info and workspace must be non-NULL");
    if (dtype != ATC_F32 && dtype != ATC_F64) return qfail(ATC_ERR_INVALID_ARGUMENT, "unknown dtype");
    if (std::isnan(target_sse) || std::isinf(target_sse)) return qfail(ATC_ERR_INVALID_ARGUMENT, "target_sse must be finite");
    if (enc_words < quant_max_words(n, block_len))
        return qfail(ATC_ERR_WORKSPACE_TOO_SMALL, "enc holds fewer words than atc_quantize_max_words");
    if (workspace_bytes < quant_workspace_bytes(n, block_len))
        return qfail(ATC_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than atc_quantize_workspace_size");
    const QuantTask t{core, n, target_sse, enc, enc_words, info, workspace};
    const hipError_t e = quantize_batch(&t, 1, dtype == ATC_F64, block_len, (hipStream_t)stream);
    if (e != hipSuccess) return qfail(ATC_ERR_DEVICE, hipGetErrorString(e));
    return ATC_OK;
}

size_t atc_dequantize_workspace_size(int64_t n, int32_t block_len) {
    if (n < 1 || block_len < 1 || block_len > QMAX_BLOCK) return 0;
    return dequant_workspace_bytes(n, block_len);
}

atc_status atc_dequantize_core(const uint32_t* enc, int64_t n, int32_t block_len, int32_t dtype, void* core_out,
                               int32_t* status, void* workspace, size_t workspace_bytes, void* stream) {
    atc_status s = check_quant_args(n, block_len);
    if (s != ATC_OK) return s;
    if (!enc || !core_out || !workspace) return qfail(ATC_ERR_INVALID_ARGUMENT, "enc, core_out and workspace must be non-NULL");
    if (dtype != ATC_F32 && dtype != ATC_F64) return qfail(ATC_ERR_INVALID_ARGUMENT, "unknown dtype");
    if (workspace_bytes < dequant_workspace_bytes(n, block_len))
        return qfail(ATC_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than atc_dequantize_workspace_size");
    const DequantTask t{enc, n, core_out, status, workspace};
    const hipError_t e = dequantize_batch(&t, 1, dtype == ATC_F64, block_len, (hipStream_t)stream);
    if (e != hipSuccess) return qfail(ATC_ERR_DEVICE, hipGetErrorString(e));
    return ATC_OK;
}

}  // extern "C"
