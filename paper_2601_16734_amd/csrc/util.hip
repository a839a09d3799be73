// Small device utilities: copies sized by device-resident dimensions, fills,
// FP64 sum of squares (the Frobenius norm of a centre tensor) and checks.

#include <algorithm>
#include <cfloat>

#include "common.h"

namespace smps {

__global__ __launch_bounds__(256) void copy_kernel(const double* src, double* dst, const int* dims, DimExpr a,
                                                  DimExpr b) {
    const size_t n = (size_t)eval_dim(dims, a) * eval_dim(dims, b);
    for (size_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

hipError_t launch_copy(const double* src, double* dst, const int* dims, DimExpr a, DimExpr b, int cap,
                       hipStream_t s) {
    if (cap <= 0) return hipSuccess;
    int blocks = (cap + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, s, src, dst, dims, a, b);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_kernel(double* dst, double v, size_t n) {
    for (size_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = v;
}

hipError_t launch_fill(double* dst, double value, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dst, value, n);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_f32_kernel(float* dst, float v, size_t n) {
    for (size_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = v;
}

hipError_t launch_fill_typed(void* dst, int type, double value, size_t n, hipStream_t s) {
    if (type == T_F64) return launch_fill((double*)dst, value, n, s);
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (float*)dst, (float)value, n);
    return hipGetLastError();
}

__global__ void copy_int_kernel(int* dims, int from, int to) { dims[to] = dims[from]; }

hipError_t launch_copy_int(int* dims, int from, int to, hipStream_t s) {
    hipLaunchKernelGGL(copy_int_kernel, dim3(1), dim3(1), 0, s, dims, from, to);
    return hipGetLastError();
}

__global__ void zero_ints_kernel(int* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

struct DimsArg {
    int v[64];
};

__global__ void set_dims_kernel(int* dims, DimsArg a, int n) {
    const int i = threadIdx.x;
    if (i < n) dims[i] = a.v[i];
}

hipError_t launch_set_dims(int* dims, const int* host_vals, int n, hipStream_t s) {
    // values travel as kernel arguments (no host buffer has to outlive the call)
    for (int off = 0; off < n; off += 64) {
        DimsArg a;
        const int m = (n - off) < 64 ? (n - off) : 64;
        for (int i = 0; i < m; ++i) a.v[i] = host_vals[off + i];
        hipLaunchKernelGGL(set_dims_kernel, dim3(1), dim3(64), 0, s, dims + off, a, m);
    }
    return hipGetLastError();
}

// Sum of squares in FP64: per-thread partials, wavefront shuffles, then LDS.
__global__ __launch_bounds__(1024) void sumsq_kernel(const double* x, const int* dims, DimExpr nexpr, double* out) {
    const int n = eval_dim(dims, nexpr);
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) a = fma(x[i], x[i], a);
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    __shared__ double part[16];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += part[w];
        *out = t;
    }
}

hipError_t launch_sumsq(const double* x, const int* dims, DimExpr n, int n_cap, double* out, hipStream_t s) {
    (void)n_cap;
    hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(1024), 0, s, x, dims, n, out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void check_finite_kernel(const double* x, const int* dims, DimExpr nexpr,
                                                          int* status) {
    const int n = eval_dim(dims, nexpr);
    int bad = 0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) bad |= !isfinite(x[i]);
    if (bad) atomicOr(status, 1);
}

hipError_t launch_check_finite(const double* x, const int* dims, DimExpr n, int n_cap, int* status,
                               hipStream_t s) {
    if (n_cap <= 0) return hipSuccess;
    int blocks = (n_cap + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(check_finite_kernel, dim3(blocks), dim3(256), 0, s, x, dims, n, status);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void convert_kernel(const float* src, double* dst, size_t n) {
    for (size_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = (double)src[i];
}

hipError_t launch_convert_f32_f64(const float* src, double* dst, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(convert_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace smps

namespace smps {

__global__ __launch_bounds__(256) void copy_batched_kernel(const CopyDesc* arr) {
    const CopyDesc d = arr[blockIdx.y];
    const size_t n = (size_t)eval_dim(d.dims, d.a) * eval_dim(d.dims, d.b);
    for (size_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) d.dst[i] = d.src[i];
}

hipError_t launch_copy_batched(const CopyDesc* arr, int count, int cap, hipStream_t s) {
    if (count <= 0 || cap <= 0) return hipSuccess;
    int blocks = (cap + 255) / 256;
    if (blocks > 512) blocks = 512;
    hipLaunchKernelGGL(copy_batched_kernel, dim3(blocks, count), dim3(256), 0, s, arr);
    return hipGetLastError();
}

__global__ void copy_int_batched_kernel(const IntCopyDesc* arr, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        arr[i].dims[arr[i].to] = arr[i].dims[arr[i].from];
}

hipError_t launch_copy_int_batched(const IntCopyDesc* arr, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_int_batched_kernel, dim3(1), dim3(256), 0, s, arr, count);
    return hipGetLastError();
}

// One workgroup per descriptor: FP64 sum of squares (wavefront shuffles, then
// LDS) and a finiteness check.
__global__ __launch_bounds__(1024) void norm_check_batched_kernel(const NormDesc* arr) {
    const NormDesc d = arr[blockIdx.x];
    const int n = eval_dim(d.dims, d.n);
    double a = 0.0;
    int bad = 0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        const double x = d.x[i];
        bad |= !isfinite(x);
        a = fma(x, x, a);
    }
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    __shared__ double part[16];
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = a;
    if (bad) s_bad = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += part[w];
        *d.out = t;
        if (s_bad) *d.status = 1;
    }
}

hipError_t launch_norm_check_batched(const NormDesc* arr, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(norm_check_batched_kernel, dim3(count), dim3(1024), 0, s, arr);
    return hipGetLastError();
}

__global__ void axpby_kernel(double* y, const double* x, double a, double b, const int* dims, DimExpr me,
                             DimExpr ne) {
    const long long n = (long long)eval_dim(dims, me) * eval_dim(dims, ne);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        y[i] = a * x[i] + b * y[i];
}

hipError_t launch_axpby(double* y, const double* x, double a, double b, const int* dims, DimExpr m, DimExpr n,
                        int cap, hipStream_t s) {
    if (cap <= 0) return hipSuccess;
    const int blocks = std::min(1024, (cap + 255) / 256);
    hipLaunchKernelGGL(axpby_kernel, dim3(blocks), dim3(256), 0, s, y, x, a, b, dims, m, n);
    return hipGetLastError();
}

// dst[b][i][o][b'] = src[b][o][i][b'] (one MPO site, Dl x o x i x Dr)
__global__ void mpo_site_transpose_kernel(const double* src, double* dst, int Dl, int o, int i, int Dr) {
    const long long n = (long long)Dl * o * i * Dr;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        long long r = e;
        const int br = (int)(r % Dr);
        r /= Dr;
        const int ii = (int)(r % i);
        r /= i;
        const int oo = (int)(r % o);
        const int bl = (int)(r / o);
        dst[(((long long)bl * i + ii) * o + oo) * Dr + br] = src[e];
    }
}

hipError_t launch_mpo_site_transpose(const double* src, double* dst, int Dl, int o, int i, int Dr, hipStream_t s) {
    const long long n = (long long)Dl * o * i * Dr;
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<long long>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(mpo_site_transpose_kernel, dim3(blocks), dim3(256), 0, s, src, dst, Dl, o, i, Dr);
    return hipGetLastError();
}

}  // namespace smps
