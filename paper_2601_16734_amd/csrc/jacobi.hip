// FP64 factorization of the two-site tensor and the truncation step.
//
// The split of Sec. 2.3 needs, for the side the isometry centre leaves, an
// orthonormal basis of the leading singular subspace, the singular values
// (for the truncation rule and the discarded weight) and nothing else: the
// other factor is recomputed as an exact projection by a matrix product.
// One-sided (Hestenes) Jacobi gives exactly that without accumulating a
// rotation matrix: rotating pairs of vectors until all are mutually
// orthogonal leaves W = Q diag(s), so the kept rows of Q are W_j / s_j.
//
// * jacobi_lds_kernel: the whole matrix resides in LDS (up to ~19k doubles on
//   gfx950's 160 KB); one workgroup of 1024 threads; disjoint vector pairs of a
//   round-robin tournament are rotated in parallel, each by a group of lanes
//   that reduce their three dot products with cross-lane shuffles.
// * blocked path (larger matrices): the vectors are cut into blocks; in each
//   round every workgroup takes one pair of blocks into LDS and orthogonalises
//   the union completely (same device routine), and rounds follow the same
//   tournament over blocks until a whole sweep changes nothing.
// * select / write: norms, descending order, the truncation rule and the
//   discarded weight in FP64 (tail summed from the smallest value up), then
//   the kept rows normalised.

#include <cfloat>

#include "common.h"

namespace smps {

constexpr int JT = 1024;               // threads per Jacobi workgroup
constexpr int LDS_BYTES = 160 * 1024;  // gfx950 LDS per workgroup
constexpr int JAC_MAX_SWEEPS = 40;
constexpr int SEL_MAX = 2048;          // vectors handled by the select kernel

__device__ __forceinline__ int tourney(int pos, int rd, int n2) {
    // player at position pos in round rd of a round-robin over n2 (even) players
    return pos == 0 ? 0 : ((pos - 1 + rd) % (n2 - 1)) + 1;
}

// Orthogonalise nv vectors (row j at W + j*ld, length len) held in LDS.
// Returns (block-uniform) whether any rotation was applied.
__device__ bool jacobi_orthogonalize(double* W, int nv, int len, int ld, int* s_flag) {
    const int tid = threadIdx.x;
    if (nv < 2) return false;
    const double tol = 2.0 * DBL_EPSILON * sqrt((double)len);
    const double tiny = DBL_MIN * 1.0e4;
    const int P = (nv + 1) / 2, n2 = 2 * P;
    int g = 64;
    while (g > 1 && g * P > JT) g >>= 1;
    const int gl = tid & (g - 1), gi = tid / g, ngroups = JT / g;
    bool any = false;
    for (int sweep = 0; sweep < JAC_MAX_SWEEPS; ++sweep) {
        if (tid == 0) *s_flag = 0;
        __syncthreads();
        for (int rd = 0; rd < n2 - 1; ++rd) {
            for (int pi = gi; pi < P; pi += ngroups) {
                const int p = tourney(pi, rd, n2), q = tourney(n2 - 1 - pi, rd, n2);
                if (p >= nv || q >= nv) continue;
                double* wp = W + (size_t)p * ld;
                double* wq = W + (size_t)q * ld;
                double a = 0.0, b = 0.0, c = 0.0;
                for (int i = gl; i < len; i += g) {
                    const double x = wp[i], y = wq[i];
                    a = fma(x, x, a);
                    b = fma(y, y, b);
                    c = fma(x, y, c);
                }
                for (int off = g >> 1; off > 0; off >>= 1) {
                    a += __shfl_xor(a, off, g);
                    b += __shfl_xor(b, off, g);
                    c += __shfl_xor(c, off, g);
                }
                if (a > tiny && b > tiny && fabs(c) > tol * sqrt(a) * sqrt(b)) {
                    const double zeta = (b - a) / (2.0 * c);
                    const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                    for (int i = gl; i < len; i += g) {
                        const double x = wp[i], y = wq[i];
                        wp[i] = cs * x - sn * y;
                        wq[i] = sn * x + cs * y;
                    }
                    if (gl == 0) *s_flag = 1;
                }
            }
            __syncthreads();
        }
        const int rot = *s_flag;
        __syncthreads();
        if (!rot) break;
        any = true;
    }
    return any;
}

// Norms, order, rank rule and discarded weight for nv vectors; results in
// LDS arrays sig (sorted order), perm, and the returned rank.  W may be in
// LDS or global memory.  Must be called by all JT threads.
__device__ int jacobi_select(const double* W, int nv, int len, int ld, double* sig_raw, double* sig_sorted,
                             int* perm, const JacobiDesc& d, double* s_delta) {
    const int tid = threadIdx.x;
    // norms: a group of 16 lanes per vector
    const int g = 16, gl = tid & (g - 1), gi = tid / g, ngroups = JT / g;
    for (int j = gi; j < nv; j += ngroups) {
        const double* w = W + (size_t)j * ld;
        double a = 0.0;
        for (int i = gl; i < len; i += g) a = fma(w[i], w[i], a);
        for (int off = g >> 1; off > 0; off >>= 1) a += __shfl_xor(a, off, g);
        if (gl == 0) sig_raw[j] = sqrt(a);
    }
    __syncthreads();
    // descending order with ties broken by index
    for (int j = tid; j < nv; j += JT) {
        const double sj = sig_raw[j];
        int pos = 0;
        for (int k = 0; k < nv; ++k) {
            const double sk = sig_raw[k];
            pos += (sk > sj) || (sk == sj && k < j);
        }
        perm[pos] = j;
        sig_sorted[pos] = sj;
    }
    __syncthreads();
    __shared__ int s_r;
    if (tid == 0) {
        int r;
        double delta;
        if (d.mode == SMPS_TRUNC_REL_SV) {
            r = 0;
            const double thr = d.tol * sig_sorted[0];
            for (int j = 0; j < nv; ++j) r += sig_sorted[j] > thr;
            if (r < 1) r = 1;
            if (r > d.max_rank) r = d.max_rank;
            if (r > nv) r = nv;
            if (r > len) r = len;
            delta = 0.0;
            for (int j = nv - 1; j >= r; --j) delta += sig_sorted[j] * sig_sorted[j];
        } else {
            // t[j] = sum_{i>=j} s_i^2 accumulated from the smallest value upwards
            double total = 0.0;
            for (int j = nv - 1; j >= 0; --j) total += sig_sorted[j] * sig_sorted[j];
            const double thr = d.tol * total;
            // smallest r >= 1 with t[r] <= thr: scan the tail upwards
            double t = 0.0;
            r = nv;
            int cand = nv;
            // t at cand = nv is 0 (<= thr always); walk down while the tail still fits
            while (cand > 1) {
                const double tn = t + sig_sorted[cand - 1] * sig_sorted[cand - 1];
                if (tn <= thr) {
                    t = tn;
                    --cand;
                } else {
                    break;
                }
            }
            r = cand;
            if (r > d.max_rank) r = d.max_rank;
            if (r > len) r = len;
            delta = 0.0;
            for (int j = nv - 1; j >= r; --j) delta += sig_sorted[j] * sig_sorted[j];
        }
        s_r = r;
        *s_delta = delta;
        if (d.log_delta) *d.log_delta = delta;
        if (d.log_rank) *d.log_rank = r;
        if (d.log_norm2) {
            double kept = 0.0;
            for (int j = r - 1; j >= 0; --j) kept += sig_sorted[j] * sig_sorted[j];
            *d.log_norm2 = kept;
        }
        d.dims_out[d.rank_idx] = r;
    }
    __syncthreads();
    if (d.log_spec)
        for (int j = tid; j < 32; j += JT) d.log_spec[j] = j < nv ? sig_sorted[j] : 0.0;
    for (int j = tid; j < nv; j += JT) d.sigma[j] = sig_sorted[j];
    const int r = s_r;
    __syncthreads();
    return r;
}

// Kept rows: Q[i] = W[perm[i]] / s_i (a zero vector only occurs when the
// whole matrix is zero and one row is kept: it becomes the first unit vector).
__device__ void jacobi_write_rows(const double* W, int len, int ld, const double* sig_sorted, const int* perm,
                                  int r, double* Q) {
    for (size_t e = threadIdx.x; e < (size_t)r * len; e += JT) {
        const int i = (int)(e / len), l = (int)(e % len);
        const double s = sig_sorted[i];
        Q[e] = s > 0.0 ? W[(size_t)perm[i] * ld + l] / s : (l == i ? 1.0 : 0.0);
    }
}

__global__ __launch_bounds__(JT) void jacobi_lds_kernel(JacobiDesc d) {
    extern __shared__ double sm[];
    __shared__ int s_flag, s_bad;
    __shared__ double s_delta;
    const int nv = eval_dim(d.dims_in, d.nvec), len = eval_dim(d.dims_in, d.len);
    const int tid = threadIdx.x;
    double* W = sm;
    double* sig_raw = sm + (size_t)nv * len;
    double* sig_sorted = sig_raw + nv;
    int* perm = (int*)(sig_sorted + nv);
    if (tid == 0) s_bad = 0;
    __syncthreads();
    int bad = 0;
    for (size_t i = tid; i < (size_t)nv * len; i += JT) {
        const double x = d.X[i];
        bad |= !isfinite(x);
        W[i] = x;
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (s_bad) {
        for (size_t i = tid; i < (size_t)nv * len; i += JT) W[i] = 0.0;
        if (tid == 0 && d.status) *d.status = 1;
        __syncthreads();
    }
    jacobi_orthogonalize(W, nv, len, len, &s_flag);
    const int r = jacobi_select(W, nv, len, len, sig_raw, sig_sorted, perm, d, &s_delta);
    jacobi_write_rows(W, len, len, sig_sorted, perm, r, d.Q);
}

// One round of the blocked path: workgroup i takes the block pair of
// tournament position i, orthogonalises the union in LDS, writes it back.
__global__ __launch_bounds__(JT) void jacobi_panel_kernel(JacobiDesc d, int bs, int nblk2, int rd) {
    extern __shared__ double sm[];
    __shared__ int s_flag, s_bad;
    const int nv = eval_dim(d.dims_in, d.nvec), len = eval_dim(d.dims_in, d.len);
    const int bp = tourney(blockIdx.x, rd, nblk2), bq = tourney(nblk2 - 1 - blockIdx.x, rd, nblk2);
    // vectors of the two blocks that exist
    int idx[2], cnt[2];
    idx[0] = bp * bs;
    idx[1] = bq * bs;
    cnt[0] = min(bs, max(0, nv - idx[0]));
    cnt[1] = min(bs, max(0, nv - idx[1]));
    const int nloc = cnt[0] + cnt[1];
    if (nloc < 2) return;
    const int tid = threadIdx.x;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    int bad = 0;
    for (size_t e = tid; e < (size_t)nloc * len; e += JT) {
        const int j = (int)(e / len), l = (int)(e % len);
        const int gj = j < cnt[0] ? idx[0] + j : idx[1] + (j - cnt[0]);
        const double x = d.X[(size_t)gj * len + l];
        bad |= !isfinite(x);
        sm[e] = x;
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (s_bad) {
        if (tid == 0 && d.status) *d.status = 1;
        return;
    }
    const bool any = jacobi_orthogonalize(sm, nloc, len, len, &s_flag);
    if (!any) return;
    for (size_t e = tid; e < (size_t)nloc * len; e += JT) {
        const int j = (int)(e / len), l = (int)(e % len);
        const int gj = j < cnt[0] ? idx[0] + j : idx[1] + (j - cnt[0]);
        d.X[(size_t)gj * len + l] = sm[e];
    }
    if (tid == 0 && d.conv) atomicOr(d.conv, 1);
}

// Blocked path finish: select on the vectors in global memory.
__global__ __launch_bounds__(JT) void jacobi_select_kernel(JacobiDesc d) {
    __shared__ double sig_raw[SEL_MAX];
    __shared__ double sig_sorted[SEL_MAX];
    __shared__ int perm_s[SEL_MAX];
    __shared__ double s_delta;
    const int nv = eval_dim(d.dims_in, d.nvec), len = eval_dim(d.dims_in, d.len);
    jacobi_select(d.X, nv, len, len, sig_raw, sig_sorted, perm_s, d, &s_delta);
    for (int j = threadIdx.x; j < nv; j += JT) d.perm[j] = perm_s[j];
}

__global__ __launch_bounds__(256) void jacobi_write_kernel(JacobiDesc d) {
    const int len = eval_dim(d.dims_in, d.len);
    const int r = d.dims_out[d.rank_idx];
    const int i = blockIdx.y;
    if (i >= r) return;
    const double s = d.sigma[i];
    const double* w = d.X + (size_t)d.perm[i] * len;
    for (int l = blockIdx.x * 256 + threadIdx.x; l < len; l += gridDim.x * 256)
        d.Q[(size_t)i * len + l] = s > 0.0 ? w[l] / s : (l == i ? 1.0 : 0.0);
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

// LDS a Jacobi workgroup may use: the device limit, capped at 160 KB.
static int g_lds_bytes = 64 * 1024;

hipError_t jacobi_init(int device) {
    int lim = 0;
    hipError_t e = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (e != hipSuccess) return e;
    lim = lim < LDS_BYTES ? lim : LDS_BYTES;
    // the dynamic part may use what the kernels' static LDS leaves free
    size_t stat = 0;
    for (const void* f : {(const void*)jacobi_lds_kernel, (const void*)jacobi_panel_kernel}) {
        hipFuncAttributes a{};
        if (hipFuncGetAttributes(&a, f) == hipSuccess && a.sharedSizeBytes > stat) stat = a.sharedSizeBytes;
    }
    int dyn = lim - (int)((stat + 255) / 256 * 256);
    bool ok = true;
    for (const void* f : {(const void*)jacobi_lds_kernel, (const void*)jacobi_panel_kernel})
        ok = ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();  // keep the default limit
        dyn = 64 * 1024 - (int)((stat + 255) / 256 * 256);
    }
    g_lds_bytes = dyn;
    return hipSuccess;
}

int jacobi_lds_limit() { return g_lds_bytes; }

static size_t lds_need(int nvec, int len) {
    return sizeof(double) * ((size_t)nvec * len + 2 * (size_t)nvec) + sizeof(int) * (size_t)nvec + 64;
}

bool jacobi_fits_lds(int nvec_cap, int len_cap) { return lds_need(nvec_cap, len_cap) <= (size_t)g_lds_bytes - 1024; }

static int panel_bs(int len_cap) {
    int bs = (int)((g_lds_bytes - 4096) / (2 * sizeof(double) * (size_t)len_cap));
    if (bs > 32) bs = 32;
    if (bs < 1) bs = 1;
    return bs;
}

size_t jacobi_work_doubles(int nvec_cap, int len_cap) { return 0; }

hipError_t launch_jacobi(const JacobiDesc& d, int nvec_cap, int len_cap, double* work, int* flags, hipStream_t s) {
    (void)work;
    if (nvec_cap <= 0 || len_cap <= 0) return hipSuccess;
    if (jacobi_fits_lds(nvec_cap, len_cap)) {
        hipLaunchKernelGGL(jacobi_lds_kernel, dim3(1), dim3(JT), lds_need(nvec_cap, len_cap), s, d);
        return hipGetLastError();
    }
    if (nvec_cap > SEL_MAX) return hipErrorInvalidValue;
    // blocked path; `flags` is one device int used as the "rotated" flag
    const int bs = panel_bs(len_cap);
    int nblk = (nvec_cap + bs - 1) / bs;
    if (nblk & 1) ++nblk;
    const size_t shm = sizeof(double) * 2 * (size_t)bs * len_cap;
    JacobiDesc dd = d;
    dd.conv = flags;
    for (int sweep = 0; sweep < JAC_MAX_SWEEPS; ++sweep) {
        hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, s, flags);
        for (int rd = 0; rd < nblk - 1; ++rd)
            hipLaunchKernelGGL(jacobi_panel_kernel, dim3(nblk / 2), dim3(JT), shm, s, dd, bs, nblk, rd);
        int h = 0;
        hipError_t e = hipMemcpyAsync(&h, flags, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (!h) break;
    }
    hipLaunchKernelGGL(jacobi_select_kernel, dim3(1), dim3(JT), 0, s, dd);
    hipLaunchKernelGGL(jacobi_write_kernel, dim3((len_cap + 255) / 256, nvec_cap), dim3(256), 0, s, dd);
    return hipGetLastError();
}

}  // namespace smps
