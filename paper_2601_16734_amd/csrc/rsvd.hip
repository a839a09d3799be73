// Device pieces of the randomized two-site factorization: the Gaussian
// sketch (Philox4x64-10 + Box-Muller), the rank-predictor features, the
// acceptance test and the identity warm-start basis.  The host sequence that
// strings them together with the GEMM and Jacobi kernels is in sweep.hip.
//
// Sketch stream: entry n of the row-major rows x nvec matrix takes block
// n / 4 of Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11) with counter
// (n / 4, step, 0, 0) and key (SKETCH_KEY0, SKETCH_KEY1).  The four 64-bit
// words give uniforms u = ((x >> 11) + 1/2) 2^-53 in (0, 1) and two
// Box-Muller pairs: (u0, u1) -> rho0 (cos, sin)(2 pi u1), rho0 = sqrt(-2 ln u0),
// and likewise (u2, u3).  Lane n % 4 selects the value.

#include <cmath>

#include "common.h"

namespace smps {

constexpr unsigned long long SKETCH_KEY0 = 0x0260116734000001ULL;
constexpr unsigned long long SKETCH_KEY1 = 0x00000000005EE95DULL;

__device__ __forceinline__ void philox4x64_10(unsigned long long x[4], unsigned long long k0,
                                              unsigned long long k1) {
    const unsigned long long M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const unsigned long long W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const unsigned long long hi0 = __umul64hi(M0, x[0]), lo0 = M0 * x[0];
        const unsigned long long hi1 = __umul64hi(M1, x[2]), lo1 = M1 * x[2];
        const unsigned long long y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
        x[0] = y0;
        x[1] = lo1;
        x[2] = y2;
        x[3] = lo0;
    }
}

__device__ __forceinline__ double unit_open(unsigned long long x) {
    return ((double)(x >> 11) + 0.5) * 0x1.0p-53;
}

__global__ void sketch_kernel(double* G, long long n, unsigned long long step) {
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (4 * b >= n) return;
    unsigned long long x[4] = {(unsigned long long)b, step, 0ULL, 0ULL};
    philox4x64_10(x, SKETCH_KEY0, SKETCH_KEY1);
    const double u0 = unit_open(x[0]), u1 = unit_open(x[1]), u2 = unit_open(x[2]), u3 = unit_open(x[3]);
    const double two_pi = 6.283185307179586476925286766559;
    const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
    double z[4];
    z[0] = r0 * cos(two_pi * u1);
    z[1] = r0 * sin(two_pi * u1);
    z[2] = r1 * cos(two_pi * u3);
    z[3] = r1 * sin(two_pi * u3);
    for (int l = 0; l < 4; ++l)
        if (4 * b + l < n) G[4 * b + l] = z[l];
}

// rows x nvec Gaussian matrix of factorization step `step`
hipError_t launch_sketch(double* G, int rows, int nvec, unsigned long long step, hipStream_t s) {
    const long long n = (long long)rows * nvec;
    if (n <= 0) return hipSuccess;
    const long long blocks = (n + 3) / 4;
    hipLaunchKernelGGL(sketch_kernel, dim3((unsigned)((blocks + 255) / 256)), dim3(256), 0, s, G, n, step);
    return hipGetLastError();
}

// Predictor input of bond i (i < count): the 32 leading log(s_j / s_0) of the
// spectrum logged at step first + stride * i, floored at log(1e-30).
__global__ void rank_features_kernel(const double* lspec, int first, int stride, int count, float* feats) {
    const int i = blockIdx.x, j = threadIdx.x;
    if (i >= count || j >= 32) return;
    const double* sp = lspec + 32 * (size_t)(first + stride * i);
    const double floor_ratio = 1e-30;
    const double s0 = sp[0];
    double v = log(floor_ratio);
    if (s0 > 0.0) {
        const double r = sp[j] / s0;
        if (r > floor_ratio) v = log(r);
    }
    feats[32 * i + j] = (float)v;
}

hipError_t launch_rank_features(const double* lspec, int first, int stride, int count, float* feats, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(rank_features_kernel, dim3(count), dim3(32), 0, s, lspec, first, stride, count, feats);
    return hipGetLastError();
}

// accepted = r <= k - p/2, the last kept value is nonzero (a zero one would
// leave a zero row in the isometry) and (relative-norm rule) discarded <= tol * total
__global__ void rsvd_accept_kernel(const int* dims, int rank_idx, const double* delta, const double* total,
                                   const double* sigma, int ksketch, int oversample, double tol, int mode,
                                   const int* status, int* flag) {
    const int r = dims[rank_idx];
    bool ok = r <= ksketch - oversample / 2 && sigma[r - 1] > 0.0;
    if (mode == SMPS_TRUNC_REL_NORM2) ok = ok && *delta <= tol * *total;
    if (status && *status) ok = false;
    *flag = ok ? 1 : 0;
}

hipError_t launch_rsvd_accept(const int* dims, int rank_idx, const double* delta, const double* total,
                              const double* sigma, int ksketch, int oversample, double tol, int mode,
                              const int* status, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(rsvd_accept_kernel, dim3(1), dim3(1), 0, s, dims, rank_idx, delta, total, sigma, ksketch,
                       oversample, tol, mode, status, flag);
    return hipGetLastError();
}

// W[j][i] /= s_j for j < rows, i < cols (row-major, ld = cols); zero s_j gives a zero row
__global__ void scale_rows_kernel(double* W, const double* sigma, const int* dims, DimExpr rows_e, DimExpr cols_e) {
    const int rows = eval_dim(dims, rows_e), cols = eval_dim(dims, cols_e);
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)rows * cols) return;
    const double sj = sigma[e / cols];
    W[e] = sj > 0.0 ? W[e] / sj : 0.0;
}

hipError_t launch_scale_rows(double* W, const double* sigma, const int* dims, DimExpr rows, DimExpr cols, int cap,
                             hipStream_t s) {
    if (cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_rows_kernel, dim3((cap + 255) / 256), dim3(256), 0, s, W, sigma, dims, rows, cols);
    return hipGetLastError();
}

// n x n identity, n = eval(nexpr) (<= cap)
__global__ void identity_kernel(double* B, const int* dims, DimExpr nexpr) {
    const int n = eval_dim(dims, nexpr);
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * n) return;
    B[e] = (e / n == e % n) ? 1.0 : 0.0;
}

hipError_t launch_identity(double* B, const int* dims, DimExpr n, int cap, hipStream_t s) {
    const long long tot = (long long)cap * cap;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(identity_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, B, dims, n);
    return hipGetLastError();
}

}  // namespace smps
