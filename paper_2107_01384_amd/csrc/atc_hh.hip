// Householder representation of the factors and the terms of the hybrid
// error model.
//
// Supplement S.2: a factor U (n x r, orthonormal columns) is the product of r
// Householder reflectors H_j = I - 2 v_j v_j^T (v_j of unit norm, zero above
// row j) applied to the first r columns of the identity, once the columns
// whose R_jj came out negative in the Householder QR are flipped.  Only the
// entries of v_j below its diagonal are kept (v_jj > 0 follows from the unit
// norm): n r - r (r + 1) / 2 numbers, each scaled by sqrt(2 alpha_j) (alpha_j
// from the slice norms of the quantized core) before quantization.
// Section 4.1.3, eq. (total_error_approximation): the slice norms of the
// quantized core per mode and |dU Sigma|_F^2 per factor.
//
// One workgroup per factor (n <= 4096 rows, r <= 256 columns); the working
// matrix sits in the caller's workspace (FP64, column-major, L2-resident at
// these sizes).  Reductions run in a fixed order (per-thread sums, then
// wavefront shuffles, then wavefronts in order).
#include <algorithm>
#include <cmath>

#include "atc_internal.hpp"

namespace atc {
namespace {

constexpr int HT = 256;          // threads of the slice-norm and factor-error workgroups
constexpr int HW = HT / 64;
constexpr int64_t HH_MAX_N = 4096;
constexpr int64_t HH_MAX_R = 256;

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sum over the workgroup in a fixed order; every thread gets the result.
__device__ double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < HW; ++w) t += red[w];
    __syncthreads();
    return t;
}

template <typename T>
__device__ __forceinline__ double ld(const T* p, int64_t i) {
    return (double)p[i];
}

// alpha_j of supplement S.2 (j 0-based here, n_j = n - j), from the squared
// slice norms s2[0..r-1]; `rest` = sum_{k > j} s2[k].
__device__ __forceinline__ double alpha_of(int64_t n, int j, int r, double s2j, double rest) {
    const double nj = (double)(n - j);
    const double rt = sqrt(nj);
    const double own = (1.0 + (nj + 5.0 * rt + 2.0) / ((rt + 1.0) * (rt + 1.0) * rt)) * s2j;
    double later = 0.0;
    if (j + 1 < r) later = (2.0 / (nj - 1.0) + (nj + 2.0 * rt + 2.0) / ((rt + 1.0) * (rt + 1.0) * (rt + 1.0) * rt)) * rest;
    return own + later;
}

// weight sqrt(2 alpha_j) of every column into w[0..r-1] (1 when s2 == nullptr)
__device__ void column_weights(int64_t n, int r, const double* __restrict__ s2, double* w) {
    if (threadIdx.x != 0) return;
    double rest = 0.0;
    for (int j = r - 1; j >= 0; --j) {
        w[j] = s2 ? sqrt(2.0 * alpha_of(n, j, r, s2[j], rest)) : 1.0;
        if (s2) rest += s2[j];
    }
}

// Work split of the Householder kernels: HHT threads, thread t < S r takes
// column c = t % r and row slice s = t / r (S = HHT / r slices of
// consecutive rows), so every dot product of a step is a thread-local sum
// over its slice, and the S slice partials of a column are summed in order
// from LDS: two barriers per reflector, no cross-lane shuffles.  The working
// matrix (row-major, odd row stride) lives in LDS when it fits, else in the
// workspace.
constexpr int HHT = 512;
constexpr size_t HH_LDS_CAP = 128 * 1024;  // bytes of LDS for the working matrix

__host__ __device__ inline int hh_ld(int r) { return r | 1; }
__host__ __device__ inline int64_t hh_coef_base(int64_t n, int j) { return (int64_t)j * (n - 1) - (int64_t)j * (j - 1) / 2; }
// whether the working matrix (plus `extra` doubles) fits the LDS budget
inline bool hh_in_lds(int64_t n, int r, int64_t extra) {
    return ((size_t)n * hh_ld(r) + (size_t)extra) * sizeof(double) <= HH_LDS_CAP;
}

// The factors of one launch, indexed by the workgroup's factor slot.
struct FJobs {
    FactorTask j[ATC_MAX_DIMS];
};

struct HhSlice {
    int c, s, S, i0, i1;  // column, slice, slices, rows [i0, i1)
    bool on;
};
__device__ __forceinline__ HhSlice hh_slice(int64_t n, int r) {
    HhSlice h;
    const int t = threadIdx.x;
    h.S = HHT / r;
    h.on = t < h.S * r;
    h.c = t % r;
    h.s = t / r;
    const int L = (int)((n + h.S - 1) / h.S);
    h.i0 = h.on ? min((int64_t)h.s * L, n) : 0;
    h.i1 = h.on ? min((int64_t)(h.s + 1) * L, n) : 0;
    return h;
}

// The sums over the S slice partials, once per column: thread c in [j, r)
// forms out[c] = sum_s part[s * r + c], and with pv non-null thread r forms
// out[r] = sum_s pv[s]; each in slice order, eight LDS loads in flight.
// (Every slice thread summing its column itself read each partial S times
// over and took 1.4 us of each 3.7 us reflector step for 512 x 19.)
__device__ __forceinline__ void column_sums(const double* part, const double* pv, int r, int S, int j, double* out) {
    const int t = threadIdx.x;
    const double* src;
    int stride;
    if (t >= j && t < r) {
        src = part + t;
        stride = r;
    } else if (pv && t == r) {
        src = pv;
        stride = 1;
    } else {
        return;
    }
    double acc = 0.0;
    for (int s = 0; s < S; s += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = s + u < S ? src[(s + u) * stride] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    out[t] = acc;
}

// Rows i in [a, b) of one column: z[i * ld] -= g * y[i * ld] (z, y two
// different columns, or y a vector with stride 1 when ld_y == 1), eight rows
// at a time with every load of a batch issued before its stores (the
// compiler cannot tell the two columns apart, so a plain loop waits for each
// row's loads after the previous row's store).
__device__ __forceinline__ void axpy_rows(double* z, int ldz, const double* y, int ldy, double g, int a, int b) {
    int i = a;
    for (; i + 8 <= b; i += 8) {
        double zv[8], yv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            zv[u] = z[(int64_t)(i + u) * ldz];
            yv[u] = y[(int64_t)(i + u) * ldy];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) z[(int64_t)(i + u) * ldz] = zv[u] - g * yv[u];
    }
    for (; i < b; ++i) z[(int64_t)i * ldz] -= g * y[(int64_t)i * ldy];
}

// Householder QR of U (n x r), column by column (supplement S.2).  Step j
// takes x = R[j:, j], |v|^2 = 2 |x| (|x| + |x_0|) for v = x + sgn(x_0) |x| e_1,
// and w_c = v^T R[j:, c] = x^T R[j:, c] + sgn(x_0) |x| R[j][c] for the later
// columns, then R[j:, c] -= 2 v w_c / |v|^2.  Column j itself is not
// rewritten: v_j / |v| (sign so that v_jj > 0), weighted, goes straight to the
// coefficients.  R[j][c] and x_0 are read before the first barrier, since
// the thread of row j updates them after it.
template <typename T, bool LDS>
__global__ void __launch_bounds__(HHT) k_hh_encode(const FJobs B) {
    extern __shared__ double hh_lds[];
    __shared__ double part[HHT];
    __shared__ double wcol[HH_MAX_R];
    __shared__ double colsum[HH_MAX_R + 1];
    __shared__ int32_t sg[HH_MAX_R];
    const FactorTask& J = B.j[blockIdx.x];
    const T* __restrict__ U = (const T*)J.U;
    const int64_t n = J.n;
    const int r = J.r;
    const double* __restrict__ s2 = J.s2;
    double* __restrict__ coef = J.coef;
    int32_t* __restrict__ signs = J.signs;
    T* __restrict__ Uprime = (T*)J.Uprime;
    double* __restrict__ Rg = J.ws;
    const int ld = hh_ld(r);
    double* R = LDS ? hh_lds : Rg;
    const HhSlice h = hh_slice(n, r);
    const int nr = (int)n * r;  // at most 4096 x 256
    for (int e = threadIdx.x; e < nr; e += HHT) {
        const int i = e / r;
        R[(int64_t)i * ld + (e - i * r)] = (double)U[e];
    }
    column_weights(n, r, s2, wcol);
    __syncthreads();
    for (int j = 0; j < r; ++j) {
        // phase A: slice partials of |x|^2 (column j) or x^T R[:, c] (c > j)
        const bool act = h.on && h.c >= j;
        double p = 0.0, rjc = 0.0, x0 = 0.0;
        if (act) {
            rjc = R[(int64_t)j * ld + h.c];
            x0 = R[(int64_t)j * ld + j];
#pragma unroll 4
            for (int i = max(h.i0, j); i < h.i1; ++i) p += R[(int64_t)i * ld + j] * R[(int64_t)i * ld + h.c];
            part[h.s * r + h.c] = p;
        }
        __syncthreads();
        column_sums(part, nullptr, r, HHT / r, j, colsum);
        __syncthreads();
        // phase B: the reflector, then the owned slice of column c
        if (act) {
            const double xx = colsum[j], wsum = colsum[h.c];
            const double nx = sqrt(xx);
            const double sgn = x0 >= 0.0 ? 1.0 : -1.0;
            const double v0 = x0 + sgn * nx;
            const double nv2 = 2.0 * nx * (nx + fabs(x0));
            const bool zero = !(nv2 > 0.0);
            if (h.c == j) {
                // v_j / |v| below the diagonal, weighted
                const double sc = zero ? 0.0 : (v0 >= 0.0 ? 1.0 : -1.0) / sqrt(nv2) * wcol[j];
                const int64_t base = hh_coef_base(n, j) - j - 1;
                int i = max(h.i0, j + 1);
                for (; i + 8 <= h.i1; i += 8) {   // a batch's loads before its stores
                    double rv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) rv[u] = R[(int64_t)(i + u) * ld + j];
#pragma unroll
                    for (int u = 0; u < 8; ++u) coef[base + i + u] = sc * rv[u];
                }
                for (; i < h.i1; ++i) coef[base + i] = sc * R[(int64_t)i * ld + j];
                if (h.s == 0) sg[j] = zero ? 1 : (x0 >= 0.0 ? -1 : 1);
            } else {
                const double w = zero ? rjc : wsum + sgn * nx * rjc;
                const double gw = (zero ? 2.0 : 2.0 / nv2) * w;
                const double vj = zero ? 1.0 : v0;
                if (h.i0 <= j && j < h.i1) R[(int64_t)j * ld + h.c] -= gw * vj;
                if (!zero)
                    axpy_rows(R + h.c, ld, R + j, ld, gw, max(h.i0, j + 1), h.i1);
            }
        }
        __syncthreads();
    }
    if (Uprime)
        for (int e = threadIdx.x; e < nr; e += HHT) Uprime[e] = (T)((double)U[e] * (double)sg[e % r]);
    for (int j = threadIdx.x; j < r; j += HHT) signs[j] = sg[j];
}

// U' = H_1 ... H_r [I_r; 0] from the weighted coefficients, the reflectors
// applied from H_r down to H_1.  Before H_j is applied, row j and the columns
// before j are still those of the identity, so step j only touches columns
// j .. r - 1 and y_c = v_j^T X[:, c] = (sum over rows below j) + v_jj [c == j];
// v_jj = sqrt(max(0, 1 - sum of the stored entries' squares)) comes from the
// slice partials of column j's threads.  v_j (unweighted) is staged in LDS,
// the next reflector's while the current one is applied.
template <typename T, bool LDS>
__global__ void __launch_bounds__(HHT) k_hh_decode(const FJobs B) {
    extern __shared__ double hh_lds[];
    __shared__ double part[HHT];
    __shared__ double partv[HHT];
    __shared__ double wcol[HH_MAX_R];
    __shared__ double colsum[HH_MAX_R + 1];
    const FactorTask& J = B.j[blockIdx.x];
    const double* __restrict__ coef = J.entries;
    const double* __restrict__ s2 = J.s2;
    const int64_t n = J.n;
    const int r = J.r;
    T* __restrict__ Uout = (T*)J.Uq;
    double* __restrict__ Xg = J.ws;
    const int ld = hh_ld(r);
    double* vbuf = hh_lds;                     // 2 x n
    double* X = LDS ? hh_lds + 2 * n : Xg;    // n x ld
    const HhSlice h = hh_slice(n, r);
    column_weights(n, r, s2, wcol);
    const int nr = (int)n * r;  // at most 4096 x 256
    for (int e = threadIdx.x; e < nr; e += HHT) {
        const int i = e / r, c = e - i * r;
        X[(int64_t)i * ld + c] = (i == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    // a zero weight only ends the factor: every later slice norm is zero too,
    // so those columns multiply nothing and their reflectors are e_j
    auto stage = [&](int j, double* vb) {
        const double wj = wcol[j];
        const int64_t base = hh_coef_base(n, j) - j - 1;
        for (int64_t i = threadIdx.x; i < n; i += HHT) vb[i] = (i > j && wj > 0.0) ? coef[base + i] / wj : 0.0;
    };
    stage(r - 1, vbuf + ((r - 1) & 1) * n);
    __syncthreads();
    for (int j = r - 1; j >= 0; --j) {
        const double* v = vbuf + (j & 1) * n;
        const bool act = h.on && h.c >= j;
        if (act) {
            double p = 0.0, q = 0.0;
#pragma unroll 4
            for (int i = max(h.i0, j + 1); i < h.i1; ++i) {
                const double vi = v[i];
                p += vi * X[(int64_t)i * ld + h.c];
                q += vi * vi;
            }
            part[h.s * r + h.c] = p;
            if (h.c == j) partv[h.s] = q;
        }
        __syncthreads();
        if (j > 0) stage(j - 1, vbuf + ((j - 1) & 1) * n);
        column_sums(part, partv, r, HHT / r, j, colsum);
        __syncthreads();
        if (act) {
            const double vv = colsum[r];
            double y = colsum[h.c];
            const double vjj = sqrt(fmax(0.0, 1.0 - vv));
            if (h.c == j) y += vjj;
            const double y2 = 2.0 * y;
            if (h.i0 <= j && j < h.i1) X[(int64_t)j * ld + h.c] -= y2 * vjj;
            axpy_rows(X + h.c, ld, v, 1, y2, max(h.i0, j + 1), h.i1);
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < nr; e += HHT) {
        const int i = e / r;
        Uout[e] = (T)X[(int64_t)i * ld + (e - i * r)];
    }
}

// coef of column j (blockIdx.y) of factor blockIdx.z times sqrt(2 alpha_j);
// each workgroup forms its column's weight from the slice norms after it.
__global__ void __launch_bounds__(256) k_hh_weight(const FJobs B) {
    __shared__ double wj;
    const FactorTask& J = B.j[blockIdx.z];
    double* __restrict__ coef = J.coef;
    const double* __restrict__ s2 = J.s2;
    const int64_t n = J.n;
    const int r = J.r;
    const int j = blockIdx.y;
    if (j >= r) return;
    if (threadIdx.x == 0) {
        double rest = 0.0;
        for (int k = r - 1; k > j; --k) rest += s2[k];
        wj = sqrt(2.0 * alpha_of(n, j, r, s2[j], rest));
    }
    __syncthreads();
    const int64_t m = n - j - 1;
    const int64_t base = hh_coef_base(n, j);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) coef[base + i] *= wj;
}

// Squared slice norms of the core in every mode: one workgroup per (mode,
// slice), the slice's elements visited in row-major order of the others.
struct Dims8 {
    int64_t v[ATC_MAX_DIMS];
};

template <typename T>
__global__ void __launch_bounds__(HT) k_slice_norms(const T* __restrict__ core, int d, Dims8 dm, double* __restrict__ out) {
    const int64_t* dims_d = dm.v;
    __shared__ double red[HW];
    // slot -> (mode k, slice s)
    int64_t slot = blockIdx.x;
    int k = 0;
    while (k < d && slot >= dims_d[k]) {
        slot -= dims_d[k];
        ++k;
    }
    int64_t L = 1, R = 1;
    for (int a = 0; a < k; ++a) L *= dims_d[a];
    for (int a = k + 1; a < d; ++a) R *= dims_d[a];
    const int64_t nk = dims_d[k];
    double p = 0.0;
    for (int64_t e = threadIdx.x; e < L * R; e += HT) {
        const int64_t l = e / R, rr = e % R;
        const double v = (double)core[(l * nk + slot) * R + rr];
        p += v * v;
    }
    const double t = block_sum(p, red);
    int64_t off = 0;
    for (int a = 0; a < k; ++a) off += dims_d[a];
    if (threadIdx.x == 0) out[off + slot] = t;
}

template <typename T>
__global__ void k_apply_signs(T* __restrict__ core, int d, Dims8 dm, int64_t total, const int32_t* __restrict__ signs) {
    const int64_t* dims_d = dm.v;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t rem = e;
        int s = 1;
        int64_t off = 0;
        int64_t stride = total;
        for (int k = 0; k < d; ++k) {
            stride /= dims_d[k];
            const int64_t ik = rem / stride;
            rem -= ik * stride;
            s *= signs[off + ik];
            off += dims_d[k];
        }
        if (s < 0) core[e] = -core[e];
    }
}

template <typename T>
__global__ void __launch_bounds__(HT) k_factor_error(const FJobs B) {
    __shared__ double red[HW];
    const FactorTask& J = B.j[blockIdx.x];
    const T* __restrict__ U = (const T*)J.U;
    const T* __restrict__ Uq = (const T*)J.Uq;
    const int64_t n = J.n;
    const int r = J.r;
    const double* __restrict__ s2 = J.s2;
    double* __restrict__ out = J.err;
    double p = 0.0;
    for (int64_t e = threadIdx.x; e < n * r; e += HT) {
        const double dlt = (double)Uq[e] - (double)U[e];
        p += dlt * dlt * s2[e % r];
    }
    const double t = block_sum(p, red);
    if (threadIdx.x == 0) *out = t;
}

// Dynamic LDS beyond the default limit for the eight kernel instances, once.
bool hh_lds_ready() {
    static int state = 0;
    if (state == 0) {
        const int cap = (int)HH_LDS_CAP;  // also covers the decoder's 2 n staged entries (n <= 4096)
        const void* ks[] = {reinterpret_cast<const void*>(&k_hh_encode<float, true>),
                            reinterpret_cast<const void*>(&k_hh_encode<float, false>),
                            reinterpret_cast<const void*>(&k_hh_encode<double, true>),
                            reinterpret_cast<const void*>(&k_hh_encode<double, false>),
                            reinterpret_cast<const void*>(&k_hh_decode<float, true>),
                            reinterpret_cast<const void*>(&k_hh_decode<float, false>),
                            reinterpret_cast<const void*>(&k_hh_decode<double, true>),
                            reinterpret_cast<const void*>(&k_hh_decode<double, false>)};
        bool ok = true;
        for (const void* k : ks) ok = ok && hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, cap) == hipSuccess;
        state = ok ? 1 : -1;
    }
    return state == 1;
}

// Factors whose working matrix fits the LDS budget go in one launch, the
// others in a second one (the kernel variant is per launch).
template <typename Kt, typename Kg>
hipError_t launch_hh_groups(const FactorTask* t, int count, int64_t extra_per_n, Kt k_lds, Kg k_ws, hipStream_t st) {
    FJobs in{}, out{};
    int ni = 0, no = 0;
    size_t shm_in = 0, shm_out = 0;
    for (int z = 0; z < count; ++z) {
        const int64_t n = t[z].n;
        const int r = t[z].r;
        const int64_t extra = extra_per_n * n;
        if (hh_in_lds(n, r, extra)) {
            in.j[ni++] = t[z];
            shm_in = std::max(shm_in, ((size_t)n * hh_ld(r) + (size_t)extra) * sizeof(double));
        } else {
            out.j[no++] = t[z];
            shm_out = std::max(shm_out, (size_t)extra * sizeof(double));
        }
    }
    if (ni) hipLaunchKernelGGL(k_lds, dim3((unsigned)ni), dim3(HHT), shm_in, st, in);
    if (no) hipLaunchKernelGGL(k_ws, dim3((unsigned)no), dim3(HHT), shm_out, st, out);
    return hipGetLastError();
}

atc_status hfail(atc_status s, const char* msg) {
    set_last_error(msg);
    return s;
}

atc_status check_nr(int64_t n, int64_t r) {
    if (n < 1 || r < 1 || r > n) return hfail(ATC_ERR_INVALID_ARGUMENT, "need 1 <= r <= n");
    if (n > HH_MAX_N || r > HH_MAX_R) return hfail(ATC_ERR_UNSUPPORTED, "factor larger than 4096 x 256");
    return ATC_OK;
}

}  // namespace

hipError_t householder_encode_batch(const FactorTask* t, int count, int f64, hipStream_t st) {
    if (count < 1 || count > ATC_MAX_DIMS || !hh_lds_ready()) return hipErrorInvalidValue;
    return f64 ? launch_hh_groups(t, count, 0, k_hh_encode<double, true>, k_hh_encode<double, false>, st)
               : launch_hh_groups(t, count, 0, k_hh_encode<float, true>, k_hh_encode<float, false>, st);
}

hipError_t householder_decode_batch(const FactorTask* t, int count, int f64, hipStream_t st) {
    if (count < 1 || count > ATC_MAX_DIMS || !hh_lds_ready()) return hipErrorInvalidValue;
    return f64 ? launch_hh_groups(t, count, 2, k_hh_decode<double, true>, k_hh_decode<double, false>, st)
               : launch_hh_groups(t, count, 2, k_hh_decode<float, true>, k_hh_decode<float, false>, st);
}

hipError_t householder_weight_batch(const FactorTask* t, int count, hipStream_t st) {
    if (count < 1 || count > ATC_MAX_DIMS) return hipErrorInvalidValue;
    FJobs B{};
    int64_t maxn = 1;
    int maxr = 1;
    for (int z = 0; z < count; ++z) {
        B.j[z] = t[z];
        maxn = std::max(maxn, t[z].n);
        maxr = std::max(maxr, t[z].r);
    }
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(16, ceil_div(maxn - 1, 256)));
    hipLaunchKernelGGL(k_hh_weight, dim3(gx, (unsigned)maxr, (unsigned)count), dim3(256), 0, st, B);
    return hipGetLastError();
}

hipError_t factor_error_batch(const FactorTask* t, int count, int f64, hipStream_t st) {
    if (count < 1 || count > ATC_MAX_DIMS) return hipErrorInvalidValue;
    FJobs B{};
    for (int z = 0; z < count; ++z) B.j[z] = t[z];
    if (f64) hipLaunchKernelGGL(k_factor_error<double>, dim3((unsigned)count), dim3(HT), 0, st, B);
    else hipLaunchKernelGGL(k_factor_error<float>, dim3((unsigned)count), dim3(HT), 0, st, B);
    return hipGetLastError();
}

}  // namespace atc

using namespace atc;

extern "C" {

size_t atc_householder_workspace_size(int64_t n, int64_t r) {
    if (check_nr(n, r) != ATC_OK) return 0;
    return (size_t)2 * n * r * sizeof(double) + 256;
}

atc_status atc_factor_householder(const void* U, int32_t dtype, int64_t n, int64_t r, const double* sigma2,
                                  double* coef, int32_t* signs, void* Uprime, void* workspace, size_t workspace_bytes,
                                  void* stream) {
    atc_status s = check_nr(n, r);
    if (s != ATC_OK) return s;
    if (!U || !coef || !signs || !workspace) return hfail(ATC_ERR_INVALID_ARGUMENT, "U, coef, signs and workspace must be non-NULL");
    if (dtype != ATC_F32 && dtype != ATC_F64) return hfail(ATC_ERR_INVALID_ARGUMENT, "unknown dtype");
    if (workspace_bytes < atc_householder_workspace_size(n, r)) return hfail(ATC_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
    if (!hh_lds_ready()) return hfail(ATC_ERR_DEVICE, "could not raise the LDS limit of the Householder kernels");
    FactorTask t{};
    t.n = n;
    t.r = (int)r;
    t.U = U;
    t.s2 = sigma2;
    t.coef = coef;
    t.signs = signs;
    t.Uprime = Uprime;
    t.ws = (double*)workspace;
    const hipError_t e = householder_encode_batch(&t, 1, dtype == ATC_F64, (hipStream_t)stream);
    return e == hipSuccess ? ATC_OK : hfail(ATC_ERR_DEVICE, hipGetErrorString(e));
}

atc_status atc_factor_from_householder(const double* coef, const double* sigma2, int64_t n, int64_t r, int32_t dtype,
                                       void* U_out, void* workspace, size_t workspace_bytes, void* stream) {
    atc_status s = check_nr(n, r);
    if (s != ATC_OK) return s;
    if (!coef || !U_out || !workspace) return hfail(ATC_ERR_INVALID_ARGUMENT, "coef, U_out and workspace must be non-NULL");
    if (dtype != ATC_F32 && dtype != ATC_F64) return hfail(ATC_ERR_INVALID_ARGUMENT, "unknown dtype");
    if (workspace_bytes < atc_householder_workspace_size(n, r)) return hfail(ATC_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
    if (!hh_lds_ready()) return hfail(ATC_ERR_DEVICE, "could not raise the LDS limit of the Householder kernels");
    FactorTask t{};
    t.n = n;
    t.r = (int)r;
    t.s2 = sigma2;
    t.entries = coef;
    t.Uq = U_out;
    t.ws = (double*)workspace;
    const hipError_t e = householder_decode_batch(&t, 1, dtype == ATC_F64, (hipStream_t)stream);
    return e == hipSuccess ? ATC_OK : hfail(ATC_ERR_DEVICE, hipGetErrorString(e));
}

atc_status atc_factor_weight_coefficients(double* coef, const double* sigma2, int64_t n, int64_t r, void* stream) {
    atc_status s = check_nr(n, r);
    if (s != ATC_OK) return s;
    if (!coef || !sigma2) return hfail(ATC_ERR_INVALID_ARGUMENT, "coef and sigma2 must be non-NULL");
    if (n == 1) return ATC_OK;  // r = 1: nothing stored
    FactorTask t{};
    t.n = n;
    t.r = (int)r;
    t.s2 = sigma2;
    t.coef = coef;
    const hipError_t e = householder_weight_batch(&t, 1, (hipStream_t)stream);
    return e == hipSuccess ? ATC_OK : hfail(ATC_ERR_DEVICE, hipGetErrorString(e));
}

size_t atc_core_slice_norms_count(const atc_shape* shape) {
    if (!shape || shape->ndim < 1 || shape->ndim > ATC_MAX_DIMS) return 0;
    size_t t = 0;
    for (int k = 0; k < shape->ndim; ++k) t += (size_t)shape->dims[k];
    return t;
}

atc_status atc_core_slice_norms(const void* core, const atc_shape* shape, double* out, void* stream) {
    if (!core || !shape || !out) return hfail(ATC_ERR_INVALID_ARGUMENT, "core, shape and out must be non-NULL");
    if (shape->ndim < 1 || shape->ndim > ATC_MAX_DIMS) return hfail(ATC_ERR_INVALID_ARGUMENT, "bad ndim");
    if (shape->dtype != ATC_F32 && shape->dtype != ATC_F64) return hfail(ATC_ERR_INVALID_ARGUMENT, "unknown dtype");
    Dims8 dm{};
    int64_t slots = 0;
    for (int k = 0; k < shape->ndim; ++k) {
        if (shape->dims[k] < 1) return hfail(ATC_ERR_INVALID_ARGUMENT, "dims must be >= 1");
        dm.v[k] = shape->dims[k];
        slots += shape->dims[k];
    }
    hipStream_t st = (hipStream_t)stream;
    if (shape->dtype == ATC_F64)
        hipLaunchKernelGGL(k_slice_norms<double>, dim3((unsigned)slots), dim3(HT), 0, st, (const double*)core,
                           shape->ndim, dm, out);
    else
        hipLaunchKernelGGL(k_slice_norms<float>, dim3((unsigned)slots), dim3(HT), 0, st, (const float*)core,
                           shape->ndim, dm, out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ATC_OK : hfail(ATC_ERR_DEVICE, hipGetErrorString(e));
}

atc_status atc_core_apply_signs(void* core, const atc_shape* shape, const int32_t* signs, void* stream) {
    if (!core || !shape || !signs) return hfail(ATC_ERR_INVALID_ARGUMENT, "core, shape and signs must be non-NULL");
    if (shape->ndim < 1 || shape->ndim > ATC_MAX_DIMS) return hfail(ATC_ERR_INVALID_ARGUMENT, "bad ndim");
    if (shape->dtype != ATC_F32 && shape->dtype != ATC_F64) return hfail(ATC_ERR_INVALID_ARGUMENT, "unknown dtype");
    Dims8 dm{};
    int64_t total = 1;
    for (int k = 0; k < shape->ndim; ++k) {
        if (shape->dims[k] < 1) return hfail(ATC_ERR_INVALID_ARGUMENT, "dims must be >= 1");
        dm.v[k] = shape->dims[k];
        total *= shape->dims[k];
    }
    hipStream_t st = (hipStream_t)stream;
    const unsigned g = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, ceil_div(total, 256)));
    if (shape->dtype == ATC_F64)
        hipLaunchKernelGGL(k_apply_signs<double>, dim3(g), dim3(256), 0, st, (double*)core, shape->ndim, dm, total,
                           signs);
    else
        hipLaunchKernelGGL(k_apply_signs<float>, dim3(g), dim3(256), 0, st, (float*)core, shape->ndim, dm, total,
                           signs);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ATC_OK : hfail(ATC_ERR_DEVICE, hipGetErrorString(e));
}

atc_status atc_factor_error_term(const void* U, const void* Uq, int32_t dtype, int64_t n, int64_t r,
                                 const double* sigma2, double* out, void* stream) {
    if (!U || !Uq || !sigma2 || !out) return hfail(ATC_ERR_INVALID_ARGUMENT, "U, Uq, sigma2 and out must be non-NULL");
    if (n < 1 || r < 1) return hfail(ATC_ERR_INVALID_ARGUMENT, "n and r must be >= 1");
    if (dtype != ATC_F32 && dtype != ATC_F64) return hfail(ATC_ERR_INVALID_ARGUMENT, "unknown dtype");
    FactorTask t{};
    t.n = n;
    t.r = (int)r;
    t.U = U;
    t.Uq = const_cast<void*>(Uq);  // read only by the error-term kernel
    t.s2 = sigma2;
    t.err = out;
    const hipError_t e = factor_error_batch(&t, 1, dtype == ATC_F64, (hipStream_t)stream);
    return e == hipSuccess ? ATC_OK : hfail(ATC_ERR_DEVICE, hipGetErrorString(e));
}

}  // extern "C"
