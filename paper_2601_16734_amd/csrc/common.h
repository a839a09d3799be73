// Internal definitions shared by the kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "seemps_hip.h"

namespace smps {

// A dimension known only on the device: value = mul * dims[idx] (idx < 0: value = mul).
// Bond dimensions chosen by truncation live in a device array so that the
// whole sweep can be enqueued (and captured) without reading ranks back.
struct DimExpr {
    int idx;
    int mul;
};

__host__ __device__ inline DimExpr dconst(int v) { return DimExpr{-1, v}; }
__host__ __device__ inline DimExpr ddyn(int idx, int mul = 1) { return DimExpr{idx, mul}; }

__device__ __forceinline__ int eval_dim(const int* dims, DimExpr e) {
    return e.idx < 0 ? e.mul : e.mul * dims[e.idx];
}

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16X3 = 2, P_BF16 = 3 };
enum DType { T_F64 = 0, T_F32 = 1 };

// C[M x N] = alpha * op(A) op(B); A is M x K (K x M stored if ta), B is K x N
// (N x K stored if tb), all compact row-major; C written N x M if tc.
struct GemmDesc {
    const void* A;
    const void* B;
    void* C;
    const int* dims;
    DimExpr M, N, K;
    int ta, tb, tc;
    int a_type, b_type, c_type;  // DType
    double alpha;
    double beta;  // C = alpha op(A) op(B) + beta C (beta = 0: C is not read)
    // batching: pointer strides in elements per blockIdx.z (0 for unbatched)
    long long sA, sB, sC;
};

// Small-K contraction with an MPO site tensor B[Dl][e][d][Dr] (see mpo_kernels).
struct LeftMpoDesc {   // Y[a][t][b'][y] = sum_{b,q} X[a][b][q][y] * B[b][t][q][b']
    const void* X;
    void* Y;
    const double* B;
    const int* dims;
    DimExpr a;   // chi_psi (rows)
    int Dl, e, d, Dr, ny;  // ny = chi_v (right bond of v)
    int x_type, y_type;
};
struct RightMpoDesc {  // Y[b][x][t][c] = sum_{q,b'} B[b][t][q][b'] * X[x][q][c][b']
    const void* X;
    void* Y;
    const double* B;
    const int* dims;
    DimExpr c;   // chi_psi (right)
    int Dl, e, d, Dr, nx;  // nx = chi_v (left bond of v)
    int x_type, y_type;
};

// One-sided Jacobi on nvec vectors of length len (row-major X), producing the
// orthonormal leading vectors Q (r x len), descending singular values, the
// kept rank (written to dims[rank_idx]) and the discarded weight.
struct JacobiDesc {
    double* X;           // nvec x len, overwritten by the rotated vectors
    double* Q;           // r x len output (may alias nothing else)
    double* sigma;       // nvec output, descending
    int* perm;           // nvec scratch
    const int* dims_in;  // dims used to evaluate nvec/len
    int* dims_out;       // rank written to dims_out[rank_idx] (may equal dims_in)
    DimExpr nvec, len;
    int rank_idx;
    int max_rank;        // max_bond (and allocation cap)
    double tol;
    int mode;            // truncation rule
    double* log_delta;   // discarded weight of this step (nullable)
    int* log_rank;       // kept rank of this step (nullable)
    double* log_spec;    // 32 leading singular values (nullable)
    double* log_norm2;   // sum of kept s_j^2 (nullable)
    int* log_sweeps;     // Jacobi sweeps that rotated (nullable)
    int* status;         // set to nonzero on non-finite input (nullable)
    int* conv;           // blocked path: set to 1 when a rotation was applied (nullable)
    double* fro2;        // blocked path: ||X||_F^2 (device scalar, filled by the launcher)
    double* basis;       // len x len: all normalised vectors when they span R^len, else the
                         // identity; pre-rotates the next factorization at this bond (nullable)
    double floor_eps;    // unit roundoff used by the numerical rank floor (FP64: 2^-52)
    int bs, nblk;        // blocked path: vectors per block, number of blocks (even)
    int* done;           // blocked path, batched: set once a sweep rotated nothing
    int gram;            // X is a symmetric PSD Gram matrix B B^T: a converged row has norm
                         // s_j^2, so s_j = sqrt(row norm) and Q rows are divided by s_j^2
    const double* total_ext;  // nullable: exact total weight ||B||_F^2; the weight that the
                              // computed s_j miss is then counted in every tail
    int accumulate;      // LDS kernel only: rotate an nvec x nvec matrix J (the identity at the
                         // start) with the vectors; Q then receives the rows of J of the kept
                         // values (the singular vectors on the nvec side, r x nvec) and basis,
                         // when given, the whole J (nvec x nvec)
    // Warm start of an accumulated factorization (nullable acc_tag: none).  acc_basis is the
    // nvec x nvec J that the last accumulated factorization at this bond in the same
    // orientation left, valid when *acc_tag == 2 nvec + acc_dir + 1.  Valid: X holds
    // acc_basis times the raw vectors and J starts from acc_basis; otherwise the raw
    // vectors are read from X_raw and J starts from the identity.  The final J is saved
    // back to acc_basis with its tag.
    const double* X_raw;
    double* acc_basis;
    int* acc_tag;
    int acc_dir;
};

}  // namespace smps

// ---- host-side launch helpers (defined in the kernel translation units) ----
namespace smps {
hipError_t launch_gemm(const GemmDesc& g, int M_cap, int N_cap, int batch, hipStream_t s, int prec);
// GEMM output tiles: 0 = 64 x 64, 1 = 64 x 32, 2 = 32 x 64, 3 = 32 x 32
constexpr int GEMM_TILES = 4;
__host__ __device__ constexpr int gemm_tile_m(int t) { return t == 2 || t == 3 ? 32 : 64; }
__host__ __device__ constexpr int gemm_tile_n(int t) { return t == 1 || t == 3 ? 32 : 64; }
hipError_t launch_gemm_tile(const GemmDesc& g, const GemmDesc* arr, int M_cap, int N_cap, int count, hipStream_t s,
                            int prec, int tile);
// tile from the autotuner's table for this product shape (64 x 64 without an entry)
int gemm_tile_for(const GemmDesc& g, int M_cap, int N_cap, int prec);
hipError_t launch_left_mpo(const LeftMpoDesc& d, int a_cap, hipStream_t s);
hipError_t launch_right_mpo(const RightMpoDesc& d, int c_cap, hipStream_t s);

size_t jacobi_work_doubles(int nvec_cap, int len_cap);
// Gram / tridiagonal / divide-and-conquer split (gtd.hip): rows of at most
// 128 elements (and at most 1024 rows); `work` holds gtd_work_doubles doubles.
bool gtd_supported(int nvec_cap, int len_cap);
size_t gtd_work_doubles(int nvec_cap, int len_cap);
hipError_t gtd_init();
hipError_t launch_gtd(const JacobiDesc& d, int nvec_cap, int len_cap, double* work, hipStream_t s);
hipError_t jacobi_init(int device);
int jacobi_lds_limit();
int jacobi_lds_class(int len_cap);
size_t jacobi_lds_bytes(int nvec_cap, int len_cap, bool accumulate = false);
void jacobi_panel_params(int nvec_cap, int len_cap, int* bs, int* nblk);
size_t jacobi_panel_bytes(int len_cap, int bs);
// every descriptor of one launch has the same `accumulate` setting (acc)
hipError_t launch_jacobi_lds_batched(const JacobiDesc* arr, int count, int E, size_t shm, hipStream_t s,
                                     bool acc = false);
// Queue state of one persistent batched blocked launch: the queue head and,
// per team of workgroups, its barrier count, current factorization, a
// give-up flag and the rotation flags of sweeps s mod 3 (one 128-byte line
// each).  The launch zeroes it before the persistent kernel starts.
struct PanelTeamState {
    int bar, prob, abort, rot[3];
    int pad[26];
};
constexpr int PANEL_MAX_TEAMS = 256;
struct PanelQueueState {
    int head;
    int pad[31];
    PanelTeamState team[PANEL_MAX_TEAMS];
};
constexpr size_t PANEL_QUEUE_BYTES = sizeof(PanelQueueState);
// teams of a persistent launch of `count` factorizations of at most
// max_pairs block pairs (grid = teams x max_pairs workgroups)
int jacobi_panel_teams(int count, int max_pairs);
hipError_t launch_jacobi_panel_batched(const JacobiDesc* arr, int count, int max_pairs, int max_rows, int len_cap,
                                       size_t shm, PanelQueueState* q, hipStream_t s);
// Exact factorization.  Chooses the LDS-resident kernel when nvec_cap*len_cap
// fits (or the Gram split when `work` is given and the size allows),
// otherwise the blocked multi-workgroup path, one launch per round with the
// sweeps driven from the host (`flags`: one device int).
hipError_t launch_jacobi(const JacobiDesc& d, int nvec_cap, int len_cap, double* work, int* flags, hipStream_t s);
hipError_t launch_gemm_batched(const GemmDesc* d_descs, int count, const GemmDesc& types, int M_cap, int N_cap,
                               hipStream_t s, int prec);
hipError_t launch_left_mpo_batched(const LeftMpoDesc* arr, int count, const LeftMpoDesc& types, int a_cap,
                                   int ny_cap, int nB_max, hipStream_t s);
hipError_t launch_right_mpo_batched(const RightMpoDesc* arr, int count, const RightMpoDesc& types, int c_cap,
                                    int nx_cap, int nB_max, hipStream_t s);
// copies of count = a * b doubles per descriptor (dims from each descriptor's array)
struct CopyDesc {
    const double* src;
    double* dst;
    const int* dims;
    DimExpr a, b;
};
hipError_t launch_copy_batched(const CopyDesc* arr, int count, int cap, hipStream_t s);
// small per-problem scalar work: dims[to] = dims[from]
struct IntCopyDesc {
    int* dims;
    int from, to;
};
hipError_t launch_copy_int_batched(const IntCopyDesc* arr, int count, hipStream_t s);
// sum of squares of n = eval(nexpr) doubles into out, and a finiteness check into status
struct NormDesc {
    const double* x;
    const int* dims;
    DimExpr n;
    double* out;
    int* status;
};
hipError_t launch_norm_check_batched(const NormDesc* arr, int count, hipStream_t s);
bool jacobi_fits_lds(int nvec_cap, int len_cap, bool accumulate = false);
hipError_t launch_copy(const double* src, double* dst, const int* dims, DimExpr a, DimExpr b, int cap,
                       hipStream_t s);
hipError_t launch_fill(double* dst, double value, size_t n, hipStream_t s);
hipError_t launch_fill_typed(void* dst, int type, double value, size_t n, hipStream_t s);
hipError_t launch_copy_int(int* dims, int from, int to, hipStream_t s);
hipError_t launch_zero_ints(int* p, int n, hipStream_t s);
hipError_t launch_set_dims(int* dims, const int* host_vals, int n, hipStream_t s);
hipError_t launch_sumsq(const double* x, const int* dims, DimExpr n, int n_cap, double* out, hipStream_t s);
hipError_t launch_check_finite(const double* x, const int* dims, DimExpr n, int n_cap, int* status,
                               hipStream_t s);
hipError_t launch_convert_f32_f64(const float* src, double* dst, size_t n, hipStream_t s);
hipError_t launch_mpo_site_transpose(const double* src, double* dst, int Dl, int o, int i, int Dr, hipStream_t s);
// y = a x + b y over m * n doubles (m, n from dims)
hipError_t launch_axpby(double* y, const double* x, double a, double b, const int* dims, DimExpr m, DimExpr n,
                        int cap, hipStream_t s);
// randomized factorization pieces (rsvd.hip)
hipError_t launch_sketch(double* G, int rows, int nvec, unsigned long long step, hipStream_t s);
hipError_t launch_rank_features(const double* lspec, int first, int stride, int count, float* feats, hipStream_t s);
hipError_t launch_rsvd_accept(const int* dims, int rank_idx, const double* delta, const double* total,
                              const double* sigma, int ksketch, int oversample, double tol, int mode,
                              const int* status, int* flag, hipStream_t s);
hipError_t launch_scale_rows(double* W, const double* sigma, const int* dims, DimExpr rows, DimExpr cols, int cap,
                             hipStream_t s);
hipError_t launch_identity(double* B, const int* dims, DimExpr n, int cap, hipStream_t s);
constexpr int RSVD_OVERSAMPLE = 16;
// factor on the rank predicted by the learned model before oversampling
constexpr double RSVD_PREDICT_MARGIN = 1.25;
}  // namespace smps
