// Contractions with one MPO site tensor B[b][t][q][b'] (Sec. 2.2 layout:
// left bond, output index, input index, right bond).
//
// These contract over (D_l or D_r) x d <= a few tens of entries, so they are
// bandwidth-bound streams: one thread per output column, coalesced along the
// fastest (rightmost) index, with the MPO tensor staged in LDS and each
// thread's inputs held in registers across all its outputs.

#include "common.h"

namespace smps {

template <typename T>
__device__ __forceinline__ double ldx(const void* p, size_t i) {
    return (double)((const T*)p)[i];
}

// Contraction depth cached in registers per thread (D d <= 32 covers D <= 16
// at d = 2); deeper contractions take the generic loop.
constexpr int MPO_KMAX = 32;

// Y[a][t][b'][y] = sum_{b,q} X[a][b][q][y] * B[b][t][q][b']
// X holds (environment x v-site) with rows (a, b) and columns (q, y).  A
// thread owns one (a, y): its K = Dl d inputs are loaded once into registers
// (independent loads, issued together) and B is staged in LDS transposed to
// [t][b'][k] so that every output reads K consecutive broadcast entries; the
// sum runs over k = b d + q in increasing order.
template <typename TX, typename TY>
__global__ __launch_bounds__(64) void left_mpo_kernel(LeftMpoDesc d0, const LeftMpoDesc* arr) {
    extern __shared__ double Bs[];
    const LeftMpoDesc d = arr ? arr[blockIdx.z] : d0;
    const int K = d.Dl * d.d, nO = d.e * d.Dr, nB = K * nO;
    for (int i = threadIdx.x; i < nB; i += blockDim.x) {
        // i = ((b e + t) d + q) Dr + b'  ->  Bs[(t Dr + b') K + b d + q]
        const int bp = i % d.Dr, r1 = i / d.Dr, q = r1 % d.d, r2 = r1 / d.d, t = r2 % d.e, b = r2 / d.e;
        Bs[(t * d.Dr + bp) * K + b * d.d + q] = d.B[i];
    }
    __syncthreads();
    const int A = eval_dim(d.dims, d.a);
    const int a = blockIdx.y;
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= A || y >= d.ny) return;
    const int ny = d.ny;
    const TX* xa = (const TX*)d.X + (size_t)a * K * ny;
    TY* ya = (TY*)d.Y + (size_t)a * nO * ny;
    if (K <= MPO_KMAX) {
        double xv[MPO_KMAX];
#pragma unroll
        for (int k = 0; k < MPO_KMAX; ++k) xv[k] = k < K ? (double)xa[(size_t)k * ny + y] : 0.0;
        for (int o = 0; o < nO; ++o) {
            const double* bo = Bs + o * K;
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < MPO_KMAX; ++k)
                if (k < K) acc += xv[k] * bo[k];
            ya[(size_t)o * ny + y] = (TY)acc;
        }
        return;
    }
    for (int o = 0; o < nO; ++o) {
        const double* bo = Bs + o * K;
        double acc = 0.0;
        for (int k = 0; k < K; ++k) acc += (double)xa[(size_t)k * ny + y] * bo[k];
        ya[(size_t)o * ny + y] = (TY)acc;
    }
}

// Y[b][x][t][c] = sum_{q,b'} B[b][t][q][b'] * X[x][q][c][b']
// X holds (v-site x environment) with rows (x, q) and columns (c, b').  A
// thread owns one (x, c): its K = d Dr inputs (Dr consecutive per q) are
// loaded once into registers; B in LDS is already [b][t][k] with
// k = q Dr + b', the order of the sum.
template <typename TX, typename TY>
__global__ __launch_bounds__(64) void right_mpo_kernel(RightMpoDesc d0, const RightMpoDesc* arr) {
    extern __shared__ double Bs[];
    const RightMpoDesc d = arr ? arr[blockIdx.z] : d0;
    const int K = d.d * d.Dr, nO = d.Dl * d.e, nB = K * nO;
    for (int i = threadIdx.x; i < nB; i += blockDim.x) Bs[i] = d.B[i];
    __syncthreads();
    const int C = eval_dim(d.dims, d.c);
    const int x = blockIdx.y;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= d.nx || c >= C) return;
    const size_t xrow = (size_t)C * d.Dr;  // elements per (x, q)
    const TX* xc = (const TX*)d.X + (size_t)x * d.d * xrow + (size_t)c * d.Dr;
    TY* Y = (TY*)d.Y;
    if (K <= MPO_KMAX) {
        double xv[MPO_KMAX];
#pragma unroll
        for (int k = 0; k < MPO_KMAX; ++k) {
            const int q = k / d.Dr, bp = k - q * d.Dr;
            xv[k] = k < K ? (double)xc[(size_t)q * xrow + bp] : 0.0;
        }
        for (int o = 0; o < nO; ++o) {  // o = b e + t
            const double* bo = Bs + o * K;
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < MPO_KMAX; ++k)
                if (k < K) acc += bo[k] * xv[k];
            const int b = o / d.e, t = o - b * d.e;
            Y[(((size_t)b * d.nx + x) * d.e + t) * C + c] = (TY)acc;
        }
        return;
    }
    for (int o = 0; o < nO; ++o) {
        const double* bo = Bs + o * K;
        double acc = 0.0;
        for (int k = 0; k < K; ++k) {
            const int q = k / d.Dr, bp = k - q * d.Dr;
            acc += bo[k] * (double)xc[(size_t)q * xrow + bp];
        }
        const int b = o / d.e, t = o - b * d.e;
        Y[(((size_t)b * d.nx + x) * d.e + t) * C + c] = (TY)acc;
    }
}

static hipError_t left_any(const LeftMpoDesc& d, const LeftMpoDesc* arr, int count, int a_cap, int ny_cap,
                           size_t shm, hipStream_t s) {
    if (a_cap <= 0 || ny_cap <= 0 || count <= 0) return hipSuccess;
    dim3 grid((ny_cap + 63) / 64, a_cap, count);
    if (d.x_type == T_F64 && d.y_type == T_F64)
        hipLaunchKernelGGL((left_mpo_kernel<double, double>), grid, dim3(64), shm, s, d, arr);
    else if (d.x_type == T_F32 && d.y_type == T_F32)
        hipLaunchKernelGGL((left_mpo_kernel<float, float>), grid, dim3(64), shm, s, d, arr);
    else if (d.x_type == T_F64)
        hipLaunchKernelGGL((left_mpo_kernel<double, float>), grid, dim3(64), shm, s, d, arr);
    else
        hipLaunchKernelGGL((left_mpo_kernel<float, double>), grid, dim3(64), shm, s, d, arr);
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
    dim3 grid((c_cap + 63) / 64, nx_cap, count);
    if (d.x_type == T_F64 && d.y_type == T_F64)
        hipLaunchKernelGGL((right_mpo_kernel<double, double>), grid, dim3(64), shm, s, d, arr);
    else if (d.x_type == T_F32 && d.y_type == T_F32)
        hipLaunchKernelGGL((right_mpo_kernel<float, float>), grid, dim3(64), shm, s, d, arr);
    else if (d.x_type == T_F64)
        hipLaunchKernelGGL((right_mpo_kernel<double, float>), grid, dim3(64), shm, s, d, arr);
    else
        hipLaunchKernelGGL((right_mpo_kernel<float, double>), grid, dim3(64), shm, s, d, arr);
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
