// Dense contractions on the CDNA4 matrix cores.
//
// Every contraction of the sweep (environment growth, the two-site tensor, the
// environment update, the scalar-product transfer step) is a product of two
// compact row-major matrices once the tensor indices are grouped, so one
// tiled MFMA kernel serves them all.  Dimensions may be device-resident
// (bond ranks chosen by truncation), so the launch grid is sized for the
// allocation cap and tiles outside the live extent exit at once.
//
// Precisions: FP64 (v_mfma_f64_16x16x4, FP64 accumulation), FP32
// (v_mfma_f32_16x16x4_f32), BF16 (v_mfma_f32_16x16x32_bf16) and split BF16x3
// (x = hi + lo, product hi*hi + hi*lo + lo*hi, all with FP32 accumulation).
// Operands are converted from their storage type while being staged in LDS.
//
// Workgroup: 256 threads = 4 wave64s arranged 2 x 2 over a TM x TN output
// tile (TM, TN in {32, 64}); each wave owns a (TM/2) x (TN/2) block of
// 16 x 16 MFMA outputs.  K is consumed in deep chunks whose global loads are
// issued one chunk ahead, into registers.  Small products (few tiles) run
// faster on the smaller tiles, larger ones on 64 x 64; the tile of each
// product shape is chosen by the autotuner (autotune.hip) when a table entry
// exists, else 64 x 64.

#include "common.h"

namespace smps {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));


__device__ __forceinline__ unsigned short f2bf(float x) {
    // round to nearest even (inputs are finite)
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

// Staging geometry.  Element i (of a chunk) of thread tid sits at
// (outer0 + i d_outer, inner0 + i d_inner) of the operand tile, lanes running
// along the operand's contiguous index: A (M x K row-major) rows tid / BK +
// i 256 / BK at k = tid % BK; A^T (K x M row-major) k = tid / BM + i 256 / BM at
// m = tid % BM; B likewise with BN.  So every element is one base address plus
// a constant stride, in global memory and in LDS.
struct StageAxis {
    int mn0, k0, dmn, dk;  // tile coordinates of element 0 and per-element steps
};
template <int BMN, int BK>
__device__ __forceinline__ StageAxis stage_axis(int tid, bool k_contiguous) {
    static_assert(256 % BK == 0 && 256 % BMN == 0, "staging needs tile sides dividing 256");
    if (k_contiguous) return StageAxis{tid / BK, tid % BK, 256 / BK, 0};
    return StageAxis{tid % BMN, tid / BMN, 0, 256 / BMN};
}

// ---------------------------------------------------------------------------
// FP64 / FP32 path: LDS holds A as [k][m] and B as [k][n].  The K loop is
// latency-bound at these sizes (a few to a few tens of workgroups, the next
// chunk cannot start before its loads return), so chunks are deep (BK = 32
// for 64 x 64 tiles, 64 otherwise) and the next chunk's global loads are
// issued into registers before the current chunk's MFMAs.  The MFMA sequence
// over k is k = 0, 4, 8, ... in every configuration; k steps beyond K are
// skipped (they would add exact zeros).
// ---------------------------------------------------------------------------
template <int BM, int BN>
__host__ __device__ constexpr int gemm_bk_f() { return (BM == 64 && BN == 64) ? 32 : 64; }

template <int PREC, typename TA, typename TB, typename TC, int BM, int BN>
__global__ __launch_bounds__(256) void gemm_kernel_f(GemmDesc g0, const GemmDesc* garr) {
    // one descriptor, or one per blockIdx.z (batched launch over independent problems)
    const GemmDesc g = garr ? garr[blockIdx.z] : g0;
    using CT = typename std::conditional<PREC == P_F64, double, float>::type;
    constexpr int BK = gemm_bk_f<BM, BN>();
    constexpr int NA = BM * BK / 256, NB = BN * BK / 256;  // elements per thread per chunk
    const int M = eval_dim(g.dims, g.M), N = eval_dim(g.dims, g.N), K = eval_dim(g.dims, g.K);
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    if (m0 >= M || n0 >= N) return;
    const void* A = g.A;
    const void* B = g.B;
    void* C = g.C;
    const int ta = g.ta, tb = g.tb;

    __shared__ CT As[BK][BM + 1];
    __shared__ CT Bs[BK][BN + 1];
    constexpr int FM = BM / 32, FN = BN / 32;  // 16 x 16 fragments per wave
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
    const int li = lane & 15, lk = lane >> 4;

    typedef typename std::conditional<PREC == P_F64, v4d, v4f>::type acc_t;
    acc_t acc[FM][FN];
    for (int i = 0; i < FM; ++i)
        for (int j = 0; j < FN; ++j)
            for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;

    // operand tiles: A as (m, k) with k contiguous unless transposed, B as
    // (n, k) with n contiguous unless transposed
    const StageAxis sa = stage_axis<BM, BK>(tid, !ta), sb = stage_axis<BN, BK>(tid, tb);
    const size_t a_step = ta ? (size_t)sa.dk * M : (size_t)sa.dmn * K;
    const size_t b_step = tb ? (size_t)sb.dmn * K : (size_t)sb.dk * N;
    CT* const as0 = &As[sa.k0][sa.mn0];
    CT* const bs0 = &Bs[sb.k0][sb.mn0];
    const int as_step = sa.dk * (BM + 1) + sa.dmn, bs_step = sb.dk * (BN + 1) + sb.dmn;
    TA ra[NA];
    TB rb[NB];
    auto fetch = [&](int k0) {
        const int gm0 = m0 + sa.mn0, ga0 = k0 + sa.k0;
        const TA* pa = (const TA*)A + (ta ? (size_t)ga0 * M + gm0 : (size_t)gm0 * K + ga0);
#pragma unroll
        for (int i = 0; i < NA; ++i)
            ra[i] = (gm0 + i * sa.dmn < M && ga0 + i * sa.dk < K) ? pa[i * a_step] : (TA)0;
        const int gn0 = n0 + sb.mn0, gb0 = k0 + sb.k0;
        const TB* pb = (const TB*)B + (tb ? (size_t)gn0 * K + gb0 : (size_t)gb0 * N + gn0);
#pragma unroll
        for (int i = 0; i < NB; ++i)
            rb[i] = (gn0 + i * sb.dmn < N && gb0 + i * sb.dk < K) ? pb[i * b_step] : (TB)0;
    };
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int i = 0; i < NA; ++i) as0[i * as_step] = (CT)ra[i];
#pragma unroll
        for (int i = 0; i < NB; ++i) bs0[i * bs_step] = (CT)rb[i];
        __syncthreads();
        if (k0 + BK < K) fetch(k0 + BK);  // in flight during this chunk's MFMAs
        const int kend = min(BK, K - k0);
        for (int kk = 0; kk < kend; kk += 4) {
            CT a[FM], b[FN];
            for (int i = 0; i < FM; ++i) a[i] = As[kk + lk][wm + i * 16 + li];
            for (int j = 0; j < FN; ++j) b[j] = Bs[kk + lk][wn + j * 16 + li];
            for (int i = 0; i < FM; ++i)
                for (int j = 0; j < FN; ++j) {
                    if constexpr (PREC == P_F64)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
                    else
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    const CT alpha = (CT)g.alpha;
    const double beta = g.beta;
    for (int i = 0; i < FM; ++i)
        for (int j = 0; j < FN; ++j)
            for (int v = 0; v < 4; ++v) {
                // v_mfma_f64_16x16x4 returns rows lk + 4v; the f32 forms return rows 4lk + v
                const int row = m0 + wm + i * 16 + (PREC == P_F64 ? lk + 4 * v : lk * 4 + v);
                const int col = n0 + wn + j * 16 + li;
                if (row < M && col < N) {
                    const size_t o = g.tc ? (size_t)col * M + row : (size_t)row * N + col;
                    if (beta != 0.0)
                        ((TC*)C)[o] = (TC)((double)(alpha * acc[i][j][v]) + beta * (double)((TC*)C)[o]);
                    else
                        ((TC*)C)[o] = (TC)(alpha * acc[i][j][v]);
                }
            }
}

// ---------------------------------------------------------------------------
// BF16 / BF16x3 path: LDS holds A as [m][k] and B as [n][k] so that a lane's
// eight consecutive k values are one 16-byte read.  Chunks of BK = 64 (two
// MFMA k steps of 32), the next chunk's loads issued before this chunk's
// MFMAs; operands are rounded (and split) while being stored to LDS.
// ---------------------------------------------------------------------------
template <int PREC, typename TA, typename TB, typename TC, int BM, int BN>
__global__ __launch_bounds__(256) void gemm_kernel_bf(GemmDesc g0, const GemmDesc* garr) {
    // one descriptor, or one per blockIdx.z (batched launch over independent problems)
    const GemmDesc g = garr ? garr[blockIdx.z] : g0;
    constexpr int BK = 64, LD = BK + 8;
    constexpr int NA = BM * BK / 256, NB = BN * BK / 256;
    constexpr bool SPLIT = (PREC == P_BF16X3);
    const int M = eval_dim(g.dims, g.M), N = eval_dim(g.dims, g.N), K = eval_dim(g.dims, g.K);
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    if (m0 >= M || n0 >= N) return;
    const void* A = g.A;
    const void* B = g.B;
    void* C = g.C;
    const int ta = g.ta, tb = g.tb;

    __shared__ __attribute__((aligned(16))) unsigned short Ah[BM][LD];
    __shared__ __attribute__((aligned(16))) unsigned short Bh[BN][LD];
    __shared__ __attribute__((aligned(16))) unsigned short Al[SPLIT ? BM : 1][LD];
    __shared__ __attribute__((aligned(16))) unsigned short Bl[SPLIT ? BN : 1][LD];
    constexpr int FM = BM / 32, FN = BN / 32;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
    const int li = lane & 15, lk = lane >> 4;

    v4f acc[FM][FN];
    for (int i = 0; i < FM; ++i)
        for (int j = 0; j < FN; ++j)
            for (int v = 0; v < 4; ++v) acc[i][j][v] = 0.f;

    const StageAxis sa = stage_axis<BM, BK>(tid, !ta), sb = stage_axis<BN, BK>(tid, tb);
    const size_t a_step = ta ? (size_t)sa.dk * M : (size_t)sa.dmn * K;
    const size_t b_step = tb ? (size_t)sb.dmn * K : (size_t)sb.dk * N;
    const int a_off = sa.mn0 * LD + sa.k0, as_step = sa.dmn * LD + sa.dk;
    const int b_off = sb.mn0 * LD + sb.k0, bs_step = sb.dmn * LD + sb.dk;
    TA ra[NA];
    TB rb[NB];
    auto fetch = [&](int k0) {
        const int gm0 = m0 + sa.mn0, ga0 = k0 + sa.k0;
        const TA* pa = (const TA*)A + (ta ? (size_t)ga0 * M + gm0 : (size_t)gm0 * K + ga0);
#pragma unroll
        for (int i = 0; i < NA; ++i)
            ra[i] = (gm0 + i * sa.dmn < M && ga0 + i * sa.dk < K) ? pa[i * a_step] : (TA)0;
        const int gn0 = n0 + sb.mn0, gb0 = k0 + sb.k0;
        const TB* pb = (const TB*)B + (tb ? (size_t)gn0 * K + gb0 : (size_t)gb0 * N + gn0);
#pragma unroll
        for (int i = 0; i < NB; ++i)
            rb[i] = (gn0 + i * sb.dmn < N && gb0 + i * sb.dk < K) ? pb[i * b_step] : (TB)0;
    };
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const float v = (float)ra[i];
            const unsigned short h = f2bf(v);
            (&Ah[0][0])[a_off + i * as_step] = h;
            if constexpr (SPLIT) (&Al[0][0])[a_off + i * as_step] = f2bf(v - bf2f(h));
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const float v = (float)rb[i];
            const unsigned short h = f2bf(v);
            (&Bh[0][0])[b_off + i * bs_step] = h;
            if constexpr (SPLIT) (&Bl[0][0])[b_off + i * bs_step] = f2bf(v - bf2f(h));
        }
        __syncthreads();
        if (k0 + BK < K) fetch(k0 + BK);  // in flight during this chunk's MFMAs
        const int kend = min(BK, K - k0);
        for (int ks = 0; ks < kend; ks += 32) {
            v8bf ah[FM], bh[FN], al[FM], bl[FN];
            for (int i = 0; i < FM; ++i) {
                ah[i] = __builtin_bit_cast(v8bf, *(const uint4*)&Ah[wm + i * 16 + li][ks + lk * 8]);
                if constexpr (SPLIT)
                    al[i] = __builtin_bit_cast(v8bf, *(const uint4*)&Al[wm + i * 16 + li][ks + lk * 8]);
            }
            for (int j = 0; j < FN; ++j) {
                bh[j] = __builtin_bit_cast(v8bf, *(const uint4*)&Bh[wn + j * 16 + li][ks + lk * 8]);
                if constexpr (SPLIT)
                    bl[j] = __builtin_bit_cast(v8bf, *(const uint4*)&Bl[wn + j * 16 + li][ks + lk * 8]);
            }
            for (int i = 0; i < FM; ++i)
                for (int j = 0; j < FN; ++j) {
                    if constexpr (SPLIT) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                    }
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    const float alpha = (float)g.alpha;
    const double beta = g.beta;
    for (int i = 0; i < FM; ++i)
        for (int j = 0; j < FN; ++j)
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm + i * 16 + lk * 4 + v;
                const int col = n0 + wn + j * 16 + li;
                if (row < M && col < N) {
                    const size_t o = g.tc ? (size_t)col * M + row : (size_t)row * N + col;
                    if (beta != 0.0)
                        ((TC*)C)[o] = (TC)((double)(alpha * acc[i][j][v]) + beta * (double)((TC*)C)[o]);
                    else
                        ((TC*)C)[o] = (TC)(alpha * acc[i][j][v]);
                }
            }
}

template <int PREC, typename TA, typename TB, typename TC, int BM, int BN>
static void launch_t(const GemmDesc& g, const GemmDesc* arr, dim3 grid, hipStream_t s) {
    if constexpr (PREC == P_F64 || PREC == P_F32)
        hipLaunchKernelGGL((gemm_kernel_f<PREC, TA, TB, TC, BM, BN>), grid, dim3(256), 0, s, g, arr);
    else
        hipLaunchKernelGGL((gemm_kernel_bf<PREC, TA, TB, TC, BM, BN>), grid, dim3(256), 0, s, g, arr);
}

template <int PREC, int BM, int BN>
static void launch_types(const GemmDesc& g, const GemmDesc* arr, dim3 grid, hipStream_t s) {
    const int code = (g.a_type << 2) | (g.b_type << 1) | g.c_type;
    switch (code) {
        case 0: launch_t<PREC, double, double, double, BM, BN>(g, arr, grid, s); break;
        case 1: launch_t<PREC, double, double, float, BM, BN>(g, arr, grid, s); break;
        case 2: launch_t<PREC, double, float, double, BM, BN>(g, arr, grid, s); break;
        case 3: launch_t<PREC, double, float, float, BM, BN>(g, arr, grid, s); break;
        case 4: launch_t<PREC, float, double, double, BM, BN>(g, arr, grid, s); break;
        case 5: launch_t<PREC, float, double, float, BM, BN>(g, arr, grid, s); break;
        case 6: launch_t<PREC, float, float, double, BM, BN>(g, arr, grid, s); break;
        default: launch_t<PREC, float, float, float, BM, BN>(g, arr, grid, s); break;
    }
}

template <int PREC>
static void launch_prec(const GemmDesc& g, const GemmDesc* arr, int tile, int M_cap, int N_cap, int count,
                        hipStream_t s) {
    const int bm = gemm_tile_m(tile), bn = gemm_tile_n(tile);
    const dim3 grid((N_cap + bn - 1) / bn, (M_cap + bm - 1) / bm, count);
    switch (tile) {
        case 1: launch_types<PREC, 64, 32>(g, arr, grid, s); break;
        case 2: launch_types<PREC, 32, 64>(g, arr, grid, s); break;
        case 3: launch_types<PREC, 32, 32>(g, arr, grid, s); break;
        default: launch_types<PREC, 64, 64>(g, arr, grid, s); break;
    }
}

hipError_t launch_gemm_tile(const GemmDesc& g, const GemmDesc* arr, int M_cap, int N_cap, int count, hipStream_t s,
                            int prec, int tile) {
    if (M_cap <= 0 || N_cap <= 0 || count <= 0) return hipSuccess;
    switch (prec) {
        case P_F64: launch_prec<P_F64>(g, arr, tile, M_cap, N_cap, count, s); break;
        case P_F32: launch_prec<P_F32>(g, arr, tile, M_cap, N_cap, count, s); break;
        case P_BF16X3: launch_prec<P_BF16X3>(g, arr, tile, M_cap, N_cap, count, s); break;
        default: launch_prec<P_BF16>(g, arr, tile, M_cap, N_cap, count, s); break;
    }
    return hipGetLastError();
}

static hipError_t launch_any(const GemmDesc& g, const GemmDesc* arr, int M_cap, int N_cap, int count, hipStream_t s,
                             int prec) {
    return launch_gemm_tile(g, arr, M_cap, N_cap, count, s, prec, gemm_tile_for(g, M_cap, N_cap, prec));
}

hipError_t launch_gemm(const GemmDesc& g, int M_cap, int N_cap, int batch, hipStream_t s, int prec) {
    (void)batch;
    return launch_any(g, nullptr, M_cap, N_cap, 1, s, prec);
}

// `types` carries a_type, b_type, c_type (shared by every descriptor of the launch)
hipError_t launch_gemm_batched(const GemmDesc* d_descs, int count, const GemmDesc& types, int M_cap, int N_cap,
                               hipStream_t s, int prec) {
    return launch_any(types, d_descs, M_cap, N_cap, count, s, prec);
}

}  // namespace smps
