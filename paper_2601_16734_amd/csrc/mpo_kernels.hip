// Contractions with one MPO site tensor B[b][t][q][b'] (Sec. 2.2 layout:
// left bond, output index, input index, right bond).
//
// These contract over (D_l or D_r) x d <= a few tens of entries, so they are
// bandwidth-bound streams: one thread per output column, coalesced along the
// fastest (rightmost) index, with the MPO tensor staged in LDS.

#include "common.h"

namespace smps {

template <typename T>
__device__ __forceinline__ double ldx(const void* p, size_t i) {
    return (double)((const T*)p)[i];
}

// Y[a][t][b'][y] = sum_{b,q} X[a][b][q][y] * B[b][t][q][b']
// X holds (environment x v-site) with rows (a, b) and columns (q, y).
template <typename TX, typename TY>
__global__ __launch_bounds__(128) void left_mpo_kernel(LeftMpoDesc d0, const LeftMpoDesc* arr) {
    extern __shared__ double Bs[];
    const LeftMpoDesc d = arr ? arr[blockIdx.z] : d0;
    const int nB = d.Dl * d.e * d.d * d.Dr;
    for (int i = threadIdx.x; i < nB; i += blockDim.x) Bs[i] = d.B[i];
    __syncthreads();
    const int A = eval_dim(d.dims, d.a);
    const int a = blockIdx.y;
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= A || y >= d.ny) return;
    const int ny = d.ny;
    const void* xa = (const char*)d.X + (size_t)a * d.Dl * d.d * ny * sizeof(TX);
    TY* ya = (TY*)d.Y + (size_t)a * d.e * d.Dr * ny;
    for (int t = 0; t < d.e; ++t)
        for (int bp = 0; bp < d.Dr; ++bp) {
            double acc = 0.0;
            for (int b = 0; b < d.Dl; ++b)
                for (int q = 0; q < d.d; ++q)
                    acc += ldx<TX>(xa, (size_t)(b * d.d + q) * ny + y) * Bs[((b * d.e + t) * d.d + q) * d.Dr + bp];
            ya[(size_t)(t * d.Dr + bp) * ny + y] = (TY)acc;
        }
}

// Y[b][x][t][c] = sum_{q,b'} B[b][t][q][b'] * X[x][q][c][b']
// X holds (v-site x environment) with rows (x, q) and columns (c, b').
template <typename TX, typename TY>
__global__ __launch_bounds__(128) void right_mpo_kernel(RightMpoDesc d0, const RightMpoDesc* arr) {
    extern __shared__ double Bs[];
    const RightMpoDesc d = arr ? arr[blockIdx.z] : d0;
    const int nB = d.Dl * d.e * d.d * d.Dr;
    for (int i = threadIdx.x; i < nB; i += blockDim.x) Bs[i] = d.B[i];
    __syncthreads();
    const int C = eval_dim(d.dims, d.c);
    const int x = blockIdx.y;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= d.nx || c >= C) return;
    const size_t xrow = (size_t)C * d.Dr;  // elements per (x, q)
    for (int b = 0; b < d.Dl; ++b)
        for (int t = 0; t < d.e; ++t) {
            double acc = 0.0;
            for (int q = 0; q < d.d; ++q)
                for (int bp = 0; bp < d.Dr; ++bp)
                    acc += Bs[((b * d.e + t) * d.d + q) * d.Dr + bp] *
                           ldx<TX>(d.X, ((size_t)x * d.d + q) * xrow + (size_t)c * d.Dr + bp);
            ((TY*)d.Y)[(((size_t)b * d.nx + x) * d.e + t) * C + c] = (TY)acc;
        }
}

static hipError_t left_any(const LeftMpoDesc& d, const LeftMpoDesc* arr, int count, int a_cap, int ny_cap,
                           size_t shm, hipStream_t s) {
    if (a_cap <= 0 || ny_cap <= 0 || count <= 0) return hipSuccess;
    dim3 grid((ny_cap + 127) / 128, a_cap, count);
    if (d.x_type == T_F64 && d.y_type == T_F64)
        hipLaunchKernelGGL((left_mpo_kernel<double, double>), grid, dim3(128), shm, s, d, arr);
    else if (d.x_type == T_F32 && d.y_type == T_F32)
        hipLaunchKernelGGL((left_mpo_kernel<float, float>), grid, dim3(128), shm, s, d, arr);
    else if (d.x_type == T_F64)
        hipLaunchKernelGGL((left_mpo_kernel<double, float>), grid, dim3(128), shm, s, d, arr);
    else
        hipLaunchKernelGGL((left_mpo_kernel<float, double>), grid, dim3(128), shm, s, d, arr);
    return hipGetLastError();
}

hipError_t launch_left_mpo(const LeftMpoDesc& d, int a_cap, hipStream_t s) {
    return left_any(d, nullptr, 1, a_cap, d.ny, sizeof(double) * d.Dl * d.e * d.d * d.Dr, s);
}

// `types` supplies x_type / y_type; caps are maxima over the descriptors
hipError_t launch_left_mpo_batched(const LeftMpoDesc* arr, int count, const LeftMpoDesc& types, int a_cap,
                                   int ny_cap, int nB_max, hipStream_t s) {
    return left_any(types, arr, count, a_cap, ny_cap, sizeof(double) * nB_max, s);
}

static hipError_t right_any(const RightMpoDesc& d, const RightMpoDesc* arr, int count, int c_cap, int nx_cap,
                            size_t shm, hipStream_t s) {
    if (c_cap <= 0 || nx_cap <= 0 || count <= 0) return hipSuccess;
    dim3 grid((c_cap + 127) / 128, nx_cap, count);
    if (d.x_type == T_F64 && d.y_type == T_F64)
        hipLaunchKernelGGL((right_mpo_kernel<double, double>), grid, dim3(128), shm, s, d, arr);
    else if (d.x_type == T_F32 && d.y_type == T_F32)
        hipLaunchKernelGGL((right_mpo_kernel<float, float>), grid, dim3(128), shm, s, d, arr);
    else if (d.x_type == T_F64)
        hipLaunchKernelGGL((right_mpo_kernel<double, float>), grid, dim3(128), shm, s, d, arr);
    else
        hipLaunchKernelGGL((right_mpo_kernel<float, double>), grid, dim3(128), shm, s, d, arr);
    return hipGetLastError();
}

hipError_t launch_right_mpo(const RightMpoDesc& d, int c_cap, hipStream_t s) {
    return right_any(d, nullptr, 1, c_cap, d.nx, sizeof(double) * d.Dl * d.e * d.d * d.Dr, s);
}

hipError_t launch_right_mpo_batched(const RightMpoDesc* arr, int count, const RightMpoDesc& types, int c_cap,
                                    int nx_cap, int nB_max, hipStream_t s) {
    return right_any(types, arr, count, c_cap, nx_cap, sizeof(double) * nB_max, s);
}

}  // namespace smps
