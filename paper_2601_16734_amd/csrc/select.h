// Device helpers shared by the factorization kernels: DPP row sums, the
// numerical rank floor, and the selection step of a split (norms of the
// orthogonalised vectors, descending order, the truncation rule of Sec. 2.3
// and the discarded weight).
#pragma once

#include <cfloat>

#include "common.h"
#include "rules.h"

namespace smps {

// Cross-lane move inside a row of 16 lanes (DPP), for a double.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of a row; every lane ends with the identical value
// (each step adds a disjoint partner, and addition is commutative).
__device__ __forceinline__ double row_sum16(double x) {
    x += dpp_mov<0xB1>(x);   // quad_perm [1,0,3,2]: partner lane ^ 1
    x += dpp_mov<0x4E>(x);   // quad_perm [2,3,0,1]: partner lane ^ 2
    x += dpp_mov<0x141>(x);  // row_half_mirror: quad 0 <-> quad 1, quad 2 <-> quad 3
    x += dpp_mov<0x140>(x);  // row_mirror: lanes 0-7 <-> lanes 8-15
    return x;
}

// Norms, order, rank rule and discarded weight for nv vectors; results in
// LDS arrays sig (sorted order), perm, and the returned rank.  W may be in
// LDS or global memory.  Must be called by all threads of the workgroup.
static __device__ int jacobi_select(const double* W, int nv, int len, int ld, double* sig_raw, double* sig_sorted,
                             int* perm, const JacobiDesc& d, double* s_delta) {
    const int tid = threadIdx.x;
    // norms: a group of 16 lanes per vector
    const int nt = blockDim.x;
    const int g = 16, gl = tid & (g - 1), gi = tid / g, ngroups = nt / g;
    for (int j = gi; j < nv; j += ngroups) {
        const double* w = W + (size_t)j * ld;
        double a = 0.0;
        for (int i = gl; i < len; i += g) a = fma(w[i], w[i], a);
        a = row_sum16(a);
        if (gl == 0) sig_raw[j] = a;
    }
    __syncthreads();
    // squared norms -> singular values, with the numerical rank floor
    __shared__ double s_floor2;
    if (tid == 0) {
        double t2 = 0.0;
        for (int j = 0; j < nv; ++j) t2 += sig_raw[j];
        s_floor2 = zero_floor2(t2, nv, len, d.floor_eps);
    }
    __syncthreads();
    for (int j = tid; j < nv; j += nt) {
        const double a = sig_raw[j];
        sig_raw[j] = a > s_floor2 ? (d.gram ? sqrt(sqrt(a)) : sqrt(a)) : 0.0;
    }
    __syncthreads();
    // descending order with ties broken by index
    for (int j = tid; j < nv; j += nt) {
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
        // rank rule and weights (rules.h); with an exact total supplied, the
        // weight the computed values miss is counted in every tail
        const TruncResult tr = trunc_rule(sig_sorted, nv, len, d.mode, d.tol, d.max_rank, d.total_ext);
        const int r = tr.r;
        s_r = r;
        *s_delta = tr.delta;
        if (d.log_delta) *d.log_delta = tr.delta;
        if (d.log_rank) *d.log_rank = r;
        if (d.log_norm2) *d.log_norm2 = tr.kept;
        d.dims_out[d.rank_idx] = r;
    }
    __syncthreads();
    if (d.log_spec)
        for (int j = tid; j < 32; j += nt) d.log_spec[j] = j < nv ? sig_sorted[j] : 0.0;
    for (int j = tid; j < nv; j += nt) d.sigma[j] = sig_sorted[j];
    const int r = s_r;
    __syncthreads();
    return r;
}

}  // namespace smps
