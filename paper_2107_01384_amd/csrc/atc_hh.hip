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
// matrix R sits in the caller's workspace (FP64, L2-resident at these sizes).
// Reductions run in a fixed order (per-thread strided sums, then wavefront
// shuffles, then wavefronts in order).
#include <algorithm>
#include <cmath>

#include "atc_internal.hpp"

namespace atc {
namespace {

constexpr int HT = 256;          // threads of the Householder workgroup
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

template <typename T>
__global__ void __launch_bounds__(HT) k_hh_encode(const T* __restrict__ U, int64_t n, int r,
                                                  const double* __restrict__ s2, double* __restrict__ coef,
                                                  int32_t* __restrict__ signs, T* __restrict__ Uprime,
                                                  double* __restrict__ R) {
    __shared__ double red[HW];
    __shared__ double wcol[HH_MAX_R];   // v^T R[:, c], then the column weights
    __shared__ int32_t sg[HH_MAX_R];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int64_t e = tid; e < n * r; e += HT) R[e] = ld(U, e);
    __syncthreads();
    double* vcol = R;  // v_j is kept in column j of R below the diagonal once the column is done
    for (int j = 0; j < r; ++j) {
        // x = R[j:, j]; |x|^2
        double p = 0.0;
        for (int64_t i = j + tid; i < n; i += HT) {
            const double x = R[i * r + j];
            p += x * x;
        }
        const double nx = sqrt(block_sum(p, red));
        const double x0 = R[(int64_t)j * r + j];
        const double v0 = x0 + (x0 >= 0.0 ? nx : -nx);
        // |v|^2 = v0^2 + |x[1:]|^2
        double q = 0.0;
        for (int64_t i = j + 1 + tid; i < n; i += HT) {
            const double x = R[i * r + j];
            q += x * x;
        }
        const double nv = sqrt(v0 * v0 + block_sum(q, red));
        const bool zero = !(nv > 0.0);
        const double inv = zero ? 0.0 : 1.0 / nv;
        // w_c = v^T R[j:, c] for c > j, one wavefront per column (strided)
        for (int c = j + 1 + wave; c < r; c += HW) {
            double s = 0.0;
            for (int64_t i = j + lane; i < n; i += 64) {
                const double v = zero ? (i == j ? 1.0 : 0.0) : (i == j ? v0 : R[i * r + j]) * inv;
                s += v * R[i * r + c];
            }
            s = wave_sum(s);
            if (lane == 0) wcol[c] = s;
        }
        __syncthreads();
        // R[j:, c] -= 2 v w_c (c > j); column j becomes (R_jj, 0, ..., 0)
        for (int64_t e = tid; e < (n - j) * (int64_t)(r - j - 1); e += HT) {
            const int64_t i = j + e / (r - j - 1);
            const int c = j + 1 + (int)(e % (r - j - 1));
            const double v = zero ? (i == j ? 1.0 : 0.0) : (i == j ? v0 : R[i * r + j]) * inv;
            R[i * r + c] -= 2.0 * v * wcol[c];
        }
        __syncthreads();
        // H_j x = -sgn(x0) |x| e_1 for the column itself: R_jj = -sgn(x0) nx
        if (tid == 0) sg[j] = zero ? 1 : (x0 >= 0.0 ? -1 : 1);
        // v_j into column j (v_jj > 0: H_j does not change with the sign of v)
        const double flip = (zero || v0 >= 0.0) ? 1.0 : -1.0;
        for (int64_t i = j + 1 + tid; i < n; i += HT) vcol[i * r + j] = zero ? 0.0 : flip * R[i * r + j] * inv;
        __syncthreads();
    }
    // weights, coefficients (column by column, rows below the diagonal)
    column_weights(n, r, s2, wcol);
    __syncthreads();
    int64_t base = 0;
    for (int j = 0; j < r; ++j) {
        const int64_t m = n - j - 1;
        for (int64_t i = tid; i < m; i += HT) coef[base + i] = vcol[(j + 1 + i) * r + j] * wcol[j];
        base += m;
    }
    for (int j = tid; j < r; j += HT) signs[j] = sg[j];
    if (Uprime)
        for (int64_t e = tid; e < n * r; e += HT) Uprime[e] = (T)(ld(U, e) * (double)sg[e % r]);
}

template <typename T>
__global__ void __launch_bounds__(HT) k_hh_decode(const double* __restrict__ coef, const double* __restrict__ s2,
                                                  int64_t n, int r, T* __restrict__ Uout,
                                                  double* __restrict__ V, double* __restrict__ X) {
    __shared__ double red[HW];
    __shared__ double wcol[HH_MAX_R];
    __shared__ double ycol[HH_MAX_R];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    column_weights(n, r, s2, wcol);
    __syncthreads();
    // V: unweighted coefficients, v_jj from the unit norm
    int64_t base = 0;
    for (int j = 0; j < r; ++j) {
        const int64_t m = n - j - 1;
        double p = 0.0;
        for (int64_t i = tid; i < m; i += HT) {
            // a zero weight only ends the factor: every later slice norm is zero
            // too, so those columns multiply nothing and their reflectors are e_j
            const double v = wcol[j] > 0.0 ? coef[base + i] / wcol[j] : 0.0;
            V[(j + 1 + i) * r + j] = v;
            p += v * v;
        }
        const double t = block_sum(p, red);
        if (tid == 0) V[(int64_t)j * r + j] = sqrt(fmax(0.0, 1.0 - t));
        for (int64_t i = tid; i < j; i += HT) V[i * r + j] = 0.0;
        base += m;
    }
    // X = first r columns of the identity, then H_r .. H_1 applied in turn
    for (int64_t e = tid; e < n * r; e += HT) X[e] = (e / r == e % r) ? 1.0 : 0.0;
    __syncthreads();
    for (int j = r - 1; j >= 0; --j) {
        for (int c = wave; c < r; c += HW) {
            double s = 0.0;
            for (int64_t i = j + lane; i < n; i += 64) s += V[i * r + j] * X[i * r + c];
            s = wave_sum(s);
            if (lane == 0) ycol[c] = s;
        }
        __syncthreads();
        for (int64_t e = tid; e < (n - j) * (int64_t)r; e += HT) {
            const int64_t i = j + e / r;
            const int c = (int)(e % r);
            X[i * r + c] -= 2.0 * V[i * r + j] * ycol[c];
        }
        __syncthreads();
    }
    for (int64_t e = tid; e < n * r; e += HT) Uout[e] = (T)X[e];
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
__global__ void __launch_bounds__(HT) k_factor_error(const T* __restrict__ U, const T* __restrict__ Uq, int64_t n, int r,
                                                     const double* __restrict__ s2, double* __restrict__ out) {
    __shared__ double red[HW];
    double p = 0.0;
    for (int64_t e = threadIdx.x; e < n * r; e += HT) {
        const double dlt = (double)Uq[e] - (double)U[e];
        p += dlt * dlt * s2[e % r];
    }
    const double t = block_sum(p, red);
    if (threadIdx.x == 0) *out = t;
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
    hipStream_t st = (hipStream_t)stream;
    double* R = (double*)workspace;
    if (dtype == ATC_F64)
        hipLaunchKernelGGL(k_hh_encode<double>, dim3(1), dim3(HT), 0, st, (const double*)U, n, (int)r, sigma2, coef,
                           signs, (double*)Uprime, R);
    else
        hipLaunchKernelGGL(k_hh_encode<float>, dim3(1), dim3(HT), 0, st, (const float*)U, n, (int)r, sigma2, coef,
                           signs, (float*)Uprime, R);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ATC_OK : hfail(ATC_ERR_DEVICE, hipGetErrorString(e));
}

atc_status atc_factor_from_householder(const double* coef, const double* sigma2, int64_t n, int64_t r, int32_t dtype,
                                       void* U_out, void* workspace, size_t workspace_bytes, void* stream) {
    atc_status s = check_nr(n, r);
    if (s != ATC_OK) return s;
    if (!coef || !U_out || !workspace) return hfail(ATC_ERR_INVALID_ARGUMENT, "coef, U_out and workspace must be non-NULL");
    if (dtype != ATC_F32 && dtype != ATC_F64) return hfail(ATC_ERR_INVALID_ARGUMENT, "unknown dtype");
    if (workspace_bytes < atc_householder_workspace_size(n, r)) return hfail(ATC_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    double* V = (double*)workspace;
    double* X = V + n * r;
    if (dtype == ATC_F64)
        hipLaunchKernelGGL(k_hh_decode<double>, dim3(1), dim3(HT), 0, st, coef, sigma2, n, (int)r, (double*)U_out, V, X);
    else
        hipLaunchKernelGGL(k_hh_decode<float>, dim3(1), dim3(HT), 0, st, coef, sigma2, n, (int)r, (float*)U_out, V, X);
    const hipError_t e = hipGetLastError();
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
    hipStream_t st = (hipStream_t)stream;
    if (dtype == ATC_F64)
        hipLaunchKernelGGL(k_factor_error<double>, dim3(1), dim3(HT), 0, st, (const double*)U, (const double*)Uq, n,
                           (int)r, sigma2, out);
    else
        hipLaunchKernelGGL(k_factor_error<float>, dim3(1), dim3(HT), 0, st, (const float*)U, (const float*)Uq, n,
                           (int)r, sigma2, out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ATC_OK : hfail(ATC_ERR_DEVICE, hipGetErrorString(e));
}

}  // extern "C"
