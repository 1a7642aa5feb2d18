/*
 * Plain FP64 CPU reference ("oracle") for the ST-HOSVD hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no source, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * Everything here is float64, row-major, single-pass loops in a fixed order.
 * A tensor that is being worked on along mode k is viewed as a 3-index array
 * (L, n, R): L = product of the sizes before mode k, n = size of mode k,
 * R = product of the sizes after mode k.  Element (l, i, r) sits at
 * (l * n + i) * R + r.  This view is exact for a row-major tensor and needs no
 * data movement (Section 3.1: the matricization may order the fibers in any
 * consistent manner, and neither the Gram matrix nor the mode product depends
 * on that order).
 *
 * Summation order: dot products over long index ranges use eight interleaved
 * partial sums (element m goes to partial m mod 8) that are then added
 * pairwise; the order is fixed, so results are reproducible bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_LANES 8

static double orc_combine(const double s[ORC_LANES]) {
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

/* Sum of x[m] * y[m] for m in [0, len), strides sx and sy. */
static double orc_dot(const double* x, int64_t sx, const double* y, int64_t sy, int64_t len) {
    double s[ORC_LANES] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t m = 0;
    if (sx == 1 && sy == 1) {
        for (; m + ORC_LANES <= len; m += ORC_LANES)
            for (int j = 0; j < ORC_LANES; ++j) s[j] += x[m + j] * y[m + j];
    }
    for (; m < len; ++m) s[m % ORC_LANES] += x[m * sx] * y[m * sy];
    return orc_combine(s);
}

/* Squared Euclidean norm (Section 3.1: inner product of a tensor with itself),
 * by pairwise (recursive halving) summation of the squares. */
static double orc_sumsq(const double* x, int64_t n) {
    if (n <= 64) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += x[i] * x[i];
        return s;
    }
    int64_t h = n / 2;
    return orc_sumsq(x, h) + orc_sumsq(x + h, n - h);
}

double oracle_norm2(const double* x, int64_t n) { return orc_sumsq(x, n); }

/*
 * Cross Gram of two tensors that share the (L, ., R) view:
 *   C[a * nw + b] = sum_{l, r} X[l, a, r] * W[l, b, r],   X: (L, nx, R), W: (L, nw, R).
 * With W = X this is the Gram matrix B_(k) B_(k)^T of the mode-k unfolding,
 * i.e. U Sigma^2 U^T of the SVD that Algorithm 1 asks for.
 */
void oracle_cross_gram(const double* X, int64_t nx, const double* W, int64_t nw,
                       int64_t L, int64_t R, double* C) {
#pragma omp parallel for schedule(dynamic) collapse(2)
    for (int64_t a = 0; a < nx; ++a) {
        for (int64_t b = 0; b < nw; ++b) {
            double s[ORC_LANES] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int64_t l = 0; l < L; ++l) {
                const double* xa = X + (l * nx + a) * R;
                const double* wb = W + (l * nw + b) * R;
                /* each l-row contributes one fixed-order partial dot */
                s[l % ORC_LANES] += orc_dot(xa, 1, wb, 1, R);
            }
            C[a * nw + b] = orc_combine(s);
        }
    }
}

/* Gram matrix G = B_(k) B_(k)^T of the (L, n, R) view; the upper triangle is
 * computed and mirrored so that G is exactly symmetric. */
void oracle_gram(const double* Y, int64_t L, int64_t n, int64_t R, double* G) {
#pragma omp parallel for schedule(dynamic)
    for (int64_t a = 0; a < n; ++a) {
        for (int64_t b = a; b < n; ++b) {
            double s[ORC_LANES] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int64_t l = 0; l < L; ++l) {
                const double* ya = Y + (l * n + a) * R;
                const double* yb = Y + (l * n + b) * R;
                s[l % ORC_LANES] += orc_dot(ya, 1, yb, 1, R);
            }
            double g = orc_combine(s);
            G[a * n + b] = g;
            G[b * n + a] = g;
        }
    }
}

/*
 * Mode product (Section 3.1): Z = M x_k Y, i.e. Z_(k) = M Y_(k).
 *   Z[l, j, r] = sum_i M[j, i] * Y[l, i, r],  M: (m, n) row-major, Y: (L, n, R), Z: (L, m, R).
 * The truncating projection of Algorithm 1 is M = U^T (m = r_k < n); the
 * expansion used by reconstruction is M = U (the core's r_k grows to n_k).
 * Each output element is summed over i in ascending order.
 */
void oracle_mode_product(const double* Y, int64_t L, int64_t n, int64_t R,
                         const double* M, int64_t m, double* Z) {
#pragma omp parallel for schedule(static) collapse(2)
    for (int64_t l = 0; l < L; ++l) {
        for (int64_t j = 0; j < m; ++j) {
            double* z = Z + (l * m + j) * R;
            for (int64_t r = 0; r < R; ++r) z[r] = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                const double mji = M[j * n + i];
                const double* y = Y + (l * n + i) * R;
                for (int64_t r = 0; r < R; ++r) z[r] += mji * y[r];
            }
        }
    }
}

/*
 * Symmetric eigendecomposition of a positive semidefinite G (n x n, row-major)
 * by one-sided (Hestenes) Jacobi.
 *
 * Start from W = G and V = I and apply plane rotations to column pairs (p, q),
 * p < q, in cyclic row order, each one chosen to make columns p and q of W
 * orthogonal; V receives the same rotations, so W = G V throughout.  A pair is
 * rotated only when |w_p . w_q| > tol * |w_p| |w_q| with tol = n * 2^-53.
 * When a whole sweep rotates nothing, the columns of G V are mutually
 * orthogonal, so V^T G^2 V is diagonal and V holds eigenvectors of G^2, which
 * for a positive semidefinite G are eigenvectors of G.  Eigenvalues are the
 * Rayleigh quotients lambda_j = v_j^T G v_j, sorted in descending order (equal
 * values keep ascending column index), with negative rounding values clamped
 * to zero.
 *
 * Outputs: lam[n] descending; V row-major with V[i * n + j] = component i of
 * eigenvector j (so V[:, :r] is the leading factor).  Returns the number of
 * sweeps performed, or -(sweeps) if the cap was reached without a quiet sweep.
 */
typedef struct { double val; int64_t idx; } orc_pair;

static int orc_desc(const void* a, const void* b) {
    const orc_pair* x = (const orc_pair*)a;
    const orc_pair* y = (const orc_pair*)b;
    if (x->val > y->val) return -1;
    if (x->val < y->val) return 1;
    return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

int oracle_eig_jacobi(const double* G, int64_t n, int max_sweeps, double* lam, double* V) {
    double* W = (double*)malloc(sizeof(double) * n * n); /* column j at W + j * n */
    double* Q = (double*)malloc(sizeof(double) * n * n); /* column j at Q + j * n */
    orc_pair* ord = (orc_pair*)malloc(sizeof(orc_pair) * (n > 0 ? n : 1));
    if (!W || !Q || !ord) { free(W); free(Q); free(ord); return -1000000; }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
            W[j * n + i] = G[i * n + j];
            Q[j * n + i] = (i == j) ? 1.0 : 0.0;
        }
    const double tol = (double)n * ldexp(1.0, -53);
    int sweeps = 0, quiet = 0;
    while (sweeps < max_sweeps && !quiet) {
        ++sweeps;
        int64_t rotations = 0;
        for (int64_t p = 0; p + 1 < n; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                double* wp = W + p * n;
                double* wq = W + q * n;
                const double alpha = orc_dot(wp, 1, wp, 1, n);
                const double beta = orc_dot(wq, 1, wq, 1, n);
                const double gamma = orc_dot(wp, 1, wq, 1, n);
                if (alpha == 0.0 || beta == 0.0) continue;
                if (fabs(gamma) <= tol * sqrt(alpha) * sqrt(beta)) continue;
                ++rotations;
                /* t = tan(theta) is the smaller root of t^2 + 2 zeta t - 1 = 0 */
                const double zeta = (beta - alpha) / (2.0 * gamma);
                double t;
                if (fabs(zeta) > 1e150) t = 0.5 / zeta;
                else t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = c * t;
                double* qp = Q + p * n;
                double* qq = Q + q * n;
                for (int64_t i = 0; i < n; ++i) {
                    const double a = wp[i], b = wq[i];
                    wp[i] = c * a - s * b;
                    wq[i] = s * a + c * b;
                }
                for (int64_t i = 0; i < n; ++i) {
                    const double a = qp[i], b = qq[i];
                    qp[i] = c * a - s * b;
                    qq[i] = s * a + c * b;
                }
            }
        }
        if (rotations == 0) quiet = 1;
    }
    /* Rayleigh quotients lambda_j = q_j^T G q_j */
    double* gq = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int64_t j = 0; j < n; ++j) {
        const double* qj = Q + j * n;
        for (int64_t i = 0; i < n; ++i) gq[i] = orc_dot(G + i * n, 1, qj, 1, n);
        ord[j].val = orc_dot(qj, 1, gq, 1, n);
        ord[j].idx = j;
    }
    free(gq);
    qsort(ord, (size_t)n, sizeof(orc_pair), orc_desc);
    for (int64_t j = 0; j < n; ++j) {
        lam[j] = ord[j].val > 0.0 ? ord[j].val : 0.0;
        const double* qj = Q + ord[j].idx * n;
        for (int64_t i = 0; i < n; ++i) V[i * n + j] = qj[i];
    }
    free(W);
    free(Q);
    free(ord);
    return quiet ? sweeps : -sweeps;
}
