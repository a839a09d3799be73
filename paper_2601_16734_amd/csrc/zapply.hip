// Complex FP64 apply + compression (Sec. 2.3 Eq. simplification, Sec. 2.4.2,
// Sec. 2.5) for complex MPS and MPO.
//
// The method is the two-site variational sweep of the real path with the bra
// conjugated in the environments: L and R contract conj(psi), U and v, the
// pair's minimiser is theta = X_L[k] X_R[k+1], and theta is split by a complex
// one-sided Jacobi SVD.  For a pair (x, y) with squared norms a, b and
// c = <x, y> = sum conj(x) y, the row y is first multiplied by the phase
// conj(c)/|c|, which makes the pair's inner product the real |c|; the real
// Jacobi rotation for (a, b, |c|) then orthogonalises them.
//
// This path is host-driven (the bond dimensions are read back after every
// split, so every launch has host-known sizes), FP64 only, single problem;
// its kernels are plain tiled / elementwise ones, not the MFMA and register-
// resident kernels of the real path.  Complex numbers are stored interleaved
// (re, im), tensors in C order with the real path's index orders.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime.h"

struct smps_zmps {
    smps_ctx* ctx = nullptr;
    int L = 0;
    std::vector<int> phys, bonds;
    double2* data = nullptr;
    size_t bytes = 0;
    std::vector<size_t> off;  // complex-element offsets
    size_t site_size(int k) const { return (size_t)bonds[k] * phys[k] * bonds[k + 1]; }
};

struct smps_zmpo {
    smps_ctx* ctx = nullptr;
    int L = 0;
    std::vector<int> pout, pin, bonds;
    double2* data = nullptr;
    size_t bytes = 0;
    std::vector<size_t> off;
    size_t site_size(int k) const { return (size_t)bonds[k] * pout[k] * pin[k] * bonds[k + 1]; }
};

namespace smps {

// complex handles, registered like the real ones (see runtime.h)
static int destroy_zmps_entry(void* h) { return smps_zmps_destroy((smps_zmps*)h); }
static int destroy_zmpo_entry(void* h) { return smps_zmpo_destroy((smps_zmpo*)h); }
static smps_zmps* new_zmps_handle(smps_ctx* c) {
    smps_zmps* m = new smps_zmps();
    m->ctx = c;
    handle_track(m, c, destroy_zmps_entry);
    return m;
}
static smps_zmpo* new_zmpo_handle(smps_ctx* c) {
    smps_zmpo* m = new smps_zmpo();
    m->ctx = c;
    handle_track(m, c, destroy_zmpo_entry);
    return m;
}
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {  // acc + a b
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// op codes of zgemm operands: N, T (transpose), H (conjugate transpose), K (conjugate)
enum ZOp { ZN = 0, ZT = 1, ZH = 2, ZK = 3 };

// C (M x N, row-major, batch stride sC) = alpha op(A) op(B) + beta C; A is M x K
// (K x M stored for T/H), B is K x N (N x K stored for T/H).  16 x 16 output
// tile per workgroup, K in steps of 16 through LDS; fixed summation order.
__global__ __launch_bounds__(256) void zgemm_kernel(const double2* A, const double2* B, double2* C, int M, int N,
                                                    int K, int opa, int opb, double2 alpha, double2 beta,
                                                    long long sA, long long sB, long long sC) {
    __shared__ double2 As[16][17], Bs[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int m = blockIdx.y * 16 + ty, n = blockIdx.x * 16 + tx;
    A += blockIdx.z * sA;
    B += blockIdx.z * sB;
    C += blockIdx.z * sC;
    double2 acc = make_double2(0.0, 0.0);
    for (int k0 = 0; k0 < K; k0 += 16) {
        {  // A tile: rows m0..m0+15, cols k0..k0+15 of op(A)
            const int mm = blockIdx.y * 16 + ty, kk = k0 + tx;
            double2 v = make_double2(0.0, 0.0);
            if (mm < M && kk < K) {
                v = (opa == ZN || opa == ZK) ? A[(size_t)mm * K + kk] : A[(size_t)kk * M + mm];
                if (opa == ZH || opa == ZK) v = cconj(v);
            }
            As[ty][tx] = v;
        }
        {  // B tile: rows k0..k0+15, cols n0..n0+15 of op(B)
            const int kk = k0 + ty, nn = blockIdx.x * 16 + tx;
            double2 v = make_double2(0.0, 0.0);
            if (kk < K && nn < N) {
                v = (opb == ZN || opb == ZK) ? B[(size_t)kk * N + nn] : B[(size_t)nn * K + kk];
                if (opb == ZH || opb == ZK) v = cconj(v);
            }
            Bs[ty][tx] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) acc = cfma(As[ty][q], Bs[q][tx], acc);
        __syncthreads();
    }
    if (m < M && n < N) {
        double2 r = cmul(alpha, acc);
        if (beta.x != 0.0 || beta.y != 0.0) r = cfma(beta, C[(size_t)m * N + n], r);
        C[(size_t)m * N + n] = r;
    }
}

// Y[a][t][b'][y] = sum_{b,q} X[a][b][q][y] W[b][t][q][b']
__global__ void zleft_mpo_kernel(const double2* X, const double2* W, double2* Y, int na, int Dl, int e, int d, int Dr,
                                 int ny) {
    const long long total = (long long)na * e * Dr * ny;
    for (long long o = blockIdx.x * (long long)blockDim.x + threadIdx.x; o < total;
         o += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(o % ny);
        long long r = o / ny;
        const int bp = (int)(r % Dr);
        r /= Dr;
        const int t = (int)(r % e);
        const int a = (int)(r / e);
        double2 acc = make_double2(0.0, 0.0);
        for (int b = 0; b < Dl; ++b)
            for (int q = 0; q < d; ++q)
                acc = cfma(X[(((size_t)a * Dl + b) * d + q) * ny + y], W[(((size_t)b * e + t) * d + q) * Dr + bp], acc);
        Y[o] = acc;
    }
}

// Y[b][x][t][c] = sum_{q,b'} W[b][t][q][b'] X[x][q][c][b']
__global__ void zright_mpo_kernel(const double2* X, const double2* W, double2* Y, int nx, int Dl, int e, int d,
                                  int Dr, int nc) {
    const long long total = (long long)Dl * nx * e * nc;
    for (long long o = blockIdx.x * (long long)blockDim.x + threadIdx.x; o < total;
         o += (long long)gridDim.x * blockDim.x) {
        const int cidx = (int)(o % nc);
        long long r = o / nc;
        const int t = (int)(r % e);
        r /= e;
        const int x = (int)(r % nx);
        const int b = (int)(r / nx);
        double2 acc = make_double2(0.0, 0.0);
        for (int q = 0; q < d; ++q)
            for (int bp = 0; bp < Dr; ++bp)
                acc = cfma(W[(((size_t)b * e + t) * d + q) * Dr + bp], X[(((size_t)x * d + q) * nc + cidx) * Dr + bp], acc);
        Y[o] = acc;
    }
}

// B (cols x rows) = A^T (no conjugation), A rows x cols
__global__ void ztranspose_kernel(const double2* A, double2* B, int rows, int cols) {
    const long long n = (long long)rows * cols;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(e / cols), c = (int)(e % cols);
        B[(long long)c * rows + r] = A[e];
    }
}

// out[0] = sum |x|^2, one workgroup, fixed order
__global__ __launch_bounds__(256) void znorm2_kernel(const double2* x, long long n, double* out) {
    __shared__ double part[256];
    double a = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256) a = fma(x[i].x, x[i].x, fma(x[i].y, x[i].y, a));
    part[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0];
}

constexpr int ZJ_NT = 1024;         // threads of the Jacobi workgroup (64 groups of 16 lanes)
constexpr int ZJ_MAX_SWEEPS = 60;

// Cross-lane move inside a row of 16 lanes (DPP) for a double, and the sum
// over the row's 16 lanes (every lane ends with the same value).
template <int CTRL>
__device__ __forceinline__ double zdpp(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double group_sum16(double x) {
    x += zdpp<0xB1>(x);   // lane ^ 1
    x += zdpp<0x4E>(x);   // lane ^ 2
    x += zdpp<0x141>(x);  // half-row mirror
    x += zdpp<0x140>(x);  // row mirror
    return x;
}

// Complex one-sided Jacobi SVD of nv rows of length len (X, row-major) in one
// workgroup: rows made orthogonal by unitary rotations (round-robin tournament
// per sweep, a 16-lane group per pair), then the singular values (row norms,
// with the numerical rank floor eps max(nv, len) ||X||_F), descending order,
// the rank rule (relative-norm tail summed from the smallest value, or
// relative singular value), the discarded weight, and the kept rows
// normalised into Q (r x len).  out_int = {rank, status}; out_dbl = {delta}.
// basis (nullable, len x len): every normalised row when the rows span C^len,
// else the identity -- the warm start of the next factorization of the bond.
__global__ __launch_bounds__(ZJ_NT) void zjacobi_kernel(const double2* X, int nv, int len, int max_rank, double tol,
                                                        int mode, double2* Q, double* sigma, int* out_int,
                                                        double* out_dbl, double2* basis) {
    extern __shared__ double2 zsm[];
    double2* W = zsm;                               // nv x len
    double* nrm = (double*)(W + (size_t)nv * len);  // nv
    double* sig = nrm + nv;                         // nv, sorted
    int* perm = (int*)(sig + nv);                   // nv
    __shared__ int s_flag, s_bad, s_r;
    __shared__ double s_total, s_delta;
    const int tid = threadIdx.x, gl = tid & 15, gi = tid >> 4, ng = ZJ_NT / 16;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    int bad = 0;
    for (int e = tid; e < nv * len; e += ZJ_NT) {
        const double2 v = X[e];
        bad |= !(isfinite(v.x) && isfinite(v.y));
        W[e] = v;
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (s_bad) {
        if (tid == 0) out_int[1] = 1;
        for (int e = tid; e < nv * len; e += ZJ_NT) W[e] = make_double2(0.0, 0.0);
        __syncthreads();
    }
    // exact squared norms, and the total for the rank floor
    for (int j = gi; j < nv; j += ng) {
        double a = 0.0;
        for (int i = gl; i < len; i += 16) a = fma(W[(size_t)j * len + i].x, W[(size_t)j * len + i].x,
                                                   fma(W[(size_t)j * len + i].y, W[(size_t)j * len + i].y, a));
        a = group_sum16(a);
        if (gl == 0) nrm[j] = a;
    }
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int j = 0; j < nv; ++j) t += nrm[j];
        s_total = t;
    }
    __syncthreads();
    const double f = 2.220446049250313e-16 * (double)(nv > len ? nv : len);
    const double floor2 = fmax(f * f * s_total, 1e-300);
    const double ctol = 2.220446049250313e-16 * (double)(len > 16 ? len : 16);
    const int P = (nv + 1) / 2, n2 = 2 * P;
    for (int sweep = 0; sweep < ZJ_MAX_SWEEPS && nv > 1; ++sweep) {
        if (tid == 0) s_flag = 0;
        __syncthreads();
        for (int rd = 0; rd < n2 - 1; ++rd) {
            for (int pi = gi; pi < P; pi += ng) {
                auto pos = [&](int x) {
                    if (x == 0) return 0;
                    int y = x - 1 + rd;
                    if (y >= n2 - 1) y -= n2 - 1;
                    return y + 1;
                };
                const int p = pos(pi), q = pos(n2 - 1 - pi);
                if (p >= nv || q >= nv) continue;
                const double a = nrm[p], b = nrm[q];
                if (!(a > floor2 && b > floor2)) continue;
                double2* wp = W + (size_t)p * len;
                double2* wq = W + (size_t)q * len;
                double cr = 0.0, ci = 0.0;  // c = sum conj(x_p) x_q
                for (int i = gl; i < len; i += 16) {
                    const double2 x = wp[i], y = wq[i];
                    cr = fma(x.x, y.x, fma(x.y, y.y, cr));
                    ci = fma(x.x, y.y, fma(-x.y, y.x, ci));
                }
                cr = group_sum16(cr);
                ci = group_sum16(ci);
                const double cabs = sqrt(fma(cr, cr, ci * ci));
                if (!(cabs > ctol * sqrt(a) * sqrt(b))) continue;
                // real rotation for (a, b, |c|) after multiplying row q by conj(c)/|c|
                const double dd = b - a;
                const double t = (dd >= 0.0 ? 1.0 : -1.0) * 2.0 * cabs / (fabs(dd) + sqrt(dd * dd + 4.0 * cabs * cabs));
                const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                const double2 ph = make_double2(cr / cabs, -ci / cabs);  // conj(c) / |c|
                for (int i = gl; i < len; i += 16) {
                    const double2 x = wp[i];
                    const double2 y = cmul(ph, wq[i]);
                    wp[i] = make_double2(cs * x.x - sn * y.x, cs * x.y - sn * y.y);
                    wq[i] = make_double2(sn * x.x + cs * y.x, sn * x.y + cs * y.y);
                }
                if (gl == 0) {
                    nrm[p] = fmax(a - t * cabs, 0.0);
                    nrm[q] = b + t * cabs;
                    s_flag = 1;
                }
            }
            __syncthreads();
        }
        // exact norms again for the next sweep (the 2 x 2 updates drift)
        for (int j = gi; j < nv; j += ng) {
            double a = 0.0;
            for (int i = gl; i < len; i += 16) a = fma(W[(size_t)j * len + i].x, W[(size_t)j * len + i].x,
                                                       fma(W[(size_t)j * len + i].y, W[(size_t)j * len + i].y, a));
            a = group_sum16(a);
            if (gl == 0) nrm[j] = a;
        }
        const int rot = s_flag;
        __syncthreads();
        if (!rot) break;
        if (sweep == ZJ_MAX_SWEEPS - 1 && tid == 0) out_int[1] |= 2;
    }
    // singular values, floor, descending order (ties by index)
    for (int j = tid; j < nv; j += ZJ_NT) nrm[j] = nrm[j] > floor2 ? sqrt(nrm[j]) : 0.0;
    __syncthreads();
    for (int j = tid; j < nv; j += ZJ_NT) {
        const double sj = nrm[j];
        int pos = 0;
        for (int k = 0; k < nv; ++k) pos += (nrm[k] > sj) || (nrm[k] == sj && k < j);
        perm[pos] = j;
        sig[pos] = sj;
    }
    __syncthreads();
    if (tid == 0) {
        int r;
        double total = 0.0;
        for (int j = nv - 1; j >= 0; --j) total += sig[j] * sig[j];
        if (mode == SMPS_TRUNC_REL_SV) {
            r = 0;
            for (int j = 0; j < nv; ++j) r += sig[j] > tol * sig[0];
        } else {
            const double thr = tol * total;
            double tl = 0.0;
            r = nv;
            while (r > 1) {
                const double tn = tl + sig[r - 1] * sig[r - 1];
                if (tn <= thr) {
                    tl = tn;
                    --r;
                } else {
                    break;
                }
            }
        }
        r = r < 1 ? 1 : r;
        r = r > max_rank ? max_rank : r;
        r = r > nv ? nv : r;
        r = r > len ? len : r;
        double delta = 0.0;
        for (int j = nv - 1; j >= r; --j) delta += sig[j] * sig[j];
        s_r = r;
        s_delta = delta;
        out_int[0] = r;
        out_dbl[0] = delta;
    }
    __syncthreads();
    const int r = s_r;
    for (int j = tid; j < nv; j += ZJ_NT) sigma[j] = sig[j];
    for (long long e = tid; e < (long long)r * len; e += ZJ_NT) {
        const int i = (int)(e / len), l = (int)(e % len);
        const double s = sig[i];
        const double2 w = W[(size_t)perm[i] * len + l];
        Q[e] = s > 0.0 ? make_double2(w.x / s, w.y / s) : make_double2(l == i ? 1.0 : 0.0, 0.0);
    }
    if (!basis) return;
    const bool full = nv >= len && sig[len - 1] > 0.0;
    for (long long e = tid; e < (long long)len * len; e += ZJ_NT) {
        const int i = (int)(e / len), l = (int)(e % len);
        if (full) {
            const double2 w = W[(size_t)perm[i] * len + l];
            basis[e] = make_double2(w.x / sig[i], w.y / sig[i]);
        } else {
            basis[e] = make_double2(i == l ? 1.0 : 0.0, 0.0);
        }
    }
}

int blocks_for(long long n) { return (int)std::max<long long>(1, std::min<long long>(2048, (n + 255) / 256)); }

size_t zjacobi_lds(int nv, int len) {
    return sizeof(double2) * (size_t)nv * len + 2 * sizeof(double) * nv + sizeof(int) * nv + 64;
}

struct ZApply {
    smps_ctx* c;
    hipStream_t s;
    const smps_zmpo* U;
    const smps_zmps* v;
    const smps_strategy& st;
    int L = 0;
    std::vector<int> d, D, cv, chi, cap;
    std::vector<double2*> psi, Lenv, Renv;
    double2 *theta = nullptr, *x1 = nullptr, *x2 = nullptr, *xl = nullptr, *xr = nullptr, *jx = nullptr, *Q = nullptr;
    double2* jx2 = nullptr;
    // per bond: the basis the last split there left (len x len of that split,
    // the identity when its rows did not span) and that len (0: none); the next
    // split at the bond, whose vectors are that len in number, is pre-rotated
    // by its conjugate
    std::vector<double2*> basis;
    std::vector<int> basis_dim;
    double *sigma = nullptr, *dbl = nullptr;
    int* ints = nullptr;
    int* host_ints = nullptr;
    double* host_dbl = nullptr;
    std::vector<void*> allocs;
    std::vector<double> deltas;
    int status_seen = 0;
    size_t lds_limit = 0;

    ZApply(smps_ctx* c_, const smps_zmpo* U_, const smps_zmps* v_, const smps_strategy& st_)
        : c(c_), s(c_->stream), U(U_), v(v_), st(st_) {}
    ~ZApply() {
        for (void* p : allocs) hipFree(p);
    }
    template <typename T>
    T* alloc(size_t n) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
        allocs.push_back(p);
        return (T*)p;
    }
    const double2* Wk(int k) const { return U->data + U->off[k]; }
    const double2* Ak(int k) const { return v->data + v->off[k]; }

    hipError_t mm(const double2* A, const double2* B, double2* C, int M, int N, int K, int opa, int opb,
                  double2 alpha = make_double2(1.0, 0.0), double2 beta = make_double2(0.0, 0.0)) {
        if (M <= 0 || N <= 0) return hipSuccess;
        hipLaunchKernelGGL(zgemm_kernel, dim3((N + 15) / 16, (M + 15) / 16, 1), dim3(256), 0, s, A, B, C, M, N, K,
                           opa, opb, alpha, beta, 0LL, 0LL, 0LL);
        return hipGetLastError();
    }
    hipError_t lmpo(const double2* X, double2* Y, int k, int na, int ny) {
        const long long n = (long long)na * d[k] * D[k + 1] * ny;
        hipLaunchKernelGGL(zleft_mpo_kernel, dim3(blocks_for(n)), dim3(256), 0, s, X, Wk(k), Y, na, D[k], d[k], d[k],
                           D[k + 1], ny);
        return hipGetLastError();
    }
    hipError_t rmpo(const double2* X, double2* Y, int k, int nx, int nc) {
        const long long n = (long long)D[k] * nx * d[k] * nc;
        hipLaunchKernelGGL(zright_mpo_kernel, dim3(blocks_for(n)), dim3(256), 0, s, X, Wk(k), Y, nx, D[k], d[k], d[k],
                           D[k + 1], nc);
        return hipGetLastError();
    }
    hipError_t transpose(const double2* A, double2* B, int rows, int cols) {
        const long long n = (long long)rows * cols;
        hipLaunchKernelGGL(ztranspose_kernel, dim3(blocks_for(n)), dim3(256), 0, s, A, B, rows, cols);
        return hipGetLastError();
    }

    // Rows of X (nv x ln) orthogonalised; Q receives the r kept normalised rows.
    hipError_t svd_rows(const double2* X, int nv, int ln, int max_rank, double tol, int mode, int* r_out,
                        double* delta_out, int bond = -1) {
        const size_t shm = zjacobi_lds(nv, ln);
        if (shm > lds_limit) return hipErrorInvalidValue;
        double2* bout = nullptr;
        if (bond >= 0) {
            if (basis_dim[bond] == nv) {  // warm start: conj(basis) X has nearly orthogonal rows
                hipError_t e = mm(basis[bond], X, jx2, nv, ln, nv, ZK, ZN);
                if (e != hipSuccess) return e;
                X = jx2;
            }
            bout = basis[bond];
            basis_dim[bond] = ln;
        }
        hipLaunchKernelGGL(zjacobi_kernel, dim3(1), dim3(ZJ_NT), shm, s, X, nv, ln, max_rank, tol, mode, Q, sigma,
                           ints, dbl, bout);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(host_ints, ints, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(host_dbl, dbl, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (host_ints[1]) {
            status_seen = host_ints[1];
            return hipErrorInvalidValue;
        }
        *r_out = host_ints[0];
        if (delta_out) *delta_out = host_dbl[0];
        return hipSuccess;
    }

    // R[k] from R[k+1] (bra psi_k conjugated)
    hipError_t env_R(int k) {
        const int x = cv[k], p = d[k], y = cv[k + 1], a = chi[k], cc = chi[k + 1];
        hipError_t e = mm(Ak(k), Renv[k + 1], x1, x * p, cc * D[k + 1], y, ZN, ZT);  // [x][p][c][d]
        if (e == hipSuccess) e = rmpo(x1, x2, k, x, cc);                               // [b][x][s][c]
        if (e == hipSuccess) e = mm(psi[k], x2, Renv[k], a, D[k] * x, p * cc, ZK, ZT);  // [a][b][x]
        return e;
    }
    // L[k+1] from L[k]
    hipError_t env_L(int k) {
        const int a = chi[k], p = d[k], x = cv[k], y = cv[k + 1], cc = chi[k + 1];
        hipError_t e = mm(Lenv[k], Ak(k), x1, a * D[k], p * y, x, ZN, ZN);                // [a][b][p][y]
        if (e == hipSuccess) e = lmpo(x1, x2, k, a, y);                                     // [a][s][d][y]
        if (e == hipSuccess) e = mm(psi[k], x2, Lenv[k + 1], cc, D[k + 1] * y, a * p, ZH, ZN);  // [c][d][y]
        return e;
    }
    // theta (a s) x (t c) for the pair (k, k+1)
    hipError_t build_theta(int k) {
        const int a = chi[k], s1 = d[k], t1 = d[k + 1], cc = chi[k + 2];
        const int x = cv[k], y = cv[k + 1], z = cv[k + 2];
        hipError_t e = mm(Lenv[k], Ak(k), x1, a * D[k], s1 * y, x, ZN, ZN);  // [a][b][p][y]
        if (e == hipSuccess) e = lmpo(x1, xl, k, a, y);                       // XL [a][s][e][y]
        if (e == hipSuccess) e = mm(Ak(k + 1), Renv[k + 2], x1, y * t1, cc * D[k + 2], z, ZN, ZT);  // [y][q][c][f]
        if (e == hipSuccess) e = rmpo(x1, xr, k + 1, y, cc);                  // XR [e][y][t][c]
        if (e == hipSuccess) e = mm(xl, xr, theta, a * s1, t1 * cc, D[k + 1] * y, ZN, ZN);
        return e;
    }

    hipError_t step(int k, bool ltr) {
        const int a = chi[k], s1 = d[k], t1 = d[k + 1], cc = chi[k + 2];
        hipError_t e = build_theta(k);
        if (e != hipSuccess) return e;
        const int mr = std::min(st.max_bond, cap[k + 1]);
        int r = 0;
        double delta = 0.0;
        if (ltr) {  // left isometry: rows of theta^T are u_j^T
            e = transpose(theta, jx, a * s1, t1 * cc);
            if (e == hipSuccess) e = svd_rows(jx, t1 * cc, a * s1, mr, st.tol, st.trunc_mode, &r, &delta, k);
            if (e == hipSuccess) e = transpose(Q, psi[k], r, a * s1);                         // psi_k = U
            if (e == hipSuccess) e = mm(Q, theta, psi[k + 1], r, t1 * cc, a * s1, ZK, ZN);  // U^H theta
            if (e != hipSuccess) return e;
            chi[k + 1] = r;
            deltas.push_back(delta);
            return env_L(k);
        }
        e = svd_rows(theta, a * s1, t1 * cc, mr, st.tol, st.trunc_mode, &r, &delta, k);  // rows v_j^H
        if (e == hipSuccess)
            e = hipMemcpyAsync(psi[k + 1], Q, sizeof(double2) * (size_t)r * t1 * cc, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = mm(theta, Q, psi[k], a * s1, r, t1 * cc, ZN, ZH);  // theta V
        if (e != hipSuccess) return e;
        chi[k + 1] = r;
        deltas.push_back(delta);
        return env_R(k + 1);
    }

    int step_error(hipError_t e) {
        if (status_seen & 1) return fail(c, SMPS_ENUMERIC, "complex apply: non-finite values in a two-site tensor");
        if (status_seen & 2) return fail(c, SMPS_ENUMERIC, "complex apply: factorization did not converge");
        if (e == hipErrorInvalidValue)
            return fail(c, SMPS_EUNSUPPORTED, "complex apply: a two-site tensor exceeds the factorization's LDS");
        return fail(c, SMPS_EHIP, std::string("complex apply: ") + hipGetErrorString(e));
    }

    int run(smps_zmps** out, double* trunc_err) {
        L = v->L;
        d = v->phys;
        D = U->bonds;
        cv = v->bonds;
        chi = v->bonds;
        {
            int dev = 0, lim = 0;
            SMPS_HIP(c, hipGetDevice(&dev));
            SMPS_HIP(c, hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
            lds_limit = (size_t)std::min(lim, 64 * 1024) - 1024;
            if (hipFuncSetAttribute((const void*)zjacobi_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    std::min(lim, 160 * 1024) - 4096) == hipSuccess)
                lds_limit = (size_t)std::min(lim, 160 * 1024) - 4096;
            else
                (void)hipGetLastError();
        }
        std::vector<long long> left(L + 1, 1), right(L + 1, 1);
        for (int k = 1; k <= L; ++k) left[k] = std::min<long long>(left[k - 1] * d[k - 1], 1LL << 40);
        for (int k = L - 1; k >= 0; --k) right[k] = std::min<long long>(right[k + 1] * d[k], 1LL << 40);
        cap.resize(L + 1);
        for (int k = 0; k <= L; ++k)
            cap[k] = (int)std::max<long long>(chi[k], std::min<long long>(st.max_bond, std::min(left[k], right[k])));
        int dmax = 1, Dmax = 1, cvmax = 1;
        for (int k = 0; k < L; ++k) dmax = std::max(dmax, d[k]);
        for (int k = 0; k <= L; ++k) Dmax = std::max(Dmax, D[k]), cvmax = std::max(cvmax, cv[k]);
        size_t nth = 1, nx = 1;
        for (int k = 0; k < L; ++k) {
            const size_t ck = std::max(cap[k], 1), ck1 = std::max(cap[k + 1], 1);
            nth = std::max(nth, ck * dmax * ck1);
            nx = std::max(nx, (size_t)std::max(ck, ck1) * Dmax * dmax * cvmax * Dmax);
            if (k + 1 < L) nth = std::max(nth, ck * d[k] * d[k + 1] * (size_t)cap[k + 2]);
        }
        psi.assign(L, nullptr);
        Lenv.assign(L + 1, nullptr);
        Renv.assign(L + 1, nullptr);
        bool ok = true;
        for (int k = 0; k < L; ++k) ok = ok && (psi[k] = alloc<double2>((size_t)cap[k] * d[k] * cap[k + 1]));
        for (int k = 0; k <= L; ++k) {
            ok = ok && (Lenv[k] = alloc<double2>((size_t)cap[k] * D[k] * cv[k]));
            ok = ok && (Renv[k] = alloc<double2>((size_t)cap[k] * D[k] * cv[k]));
        }
        basis.assign(std::max(0, L - 1), nullptr);
        basis_dim.assign(std::max(0, L - 1), 0);
        for (int k = 0; k + 1 < L; ++k) {
            const size_t nb = std::max((size_t)cap[k] * d[k], (size_t)d[k + 1] * cap[k + 2]);
            ok = ok && (basis[k] = alloc<double2>(nb * nb));
        }
        ok = ok && (theta = alloc<double2>(nth)) && (jx = alloc<double2>(nth)) && (jx2 = alloc<double2>(nth)) &&
             (Q = alloc<double2>(nth)) &&
             (x1 = alloc<double2>(nx)) && (x2 = alloc<double2>(nx)) && (xl = alloc<double2>(nx)) &&
             (xr = alloc<double2>(nx)) && (sigma = alloc<double>(nth)) && (dbl = alloc<double>(4)) &&
             (ints = alloc<int>(4));
        if (!ok) return fail(c, SMPS_ENOMEM, "complex apply: workspace allocation failed");
        int rc = ensure_pinned(c, 64);
        if (rc) return rc;
        host_ints = (int*)c->pinned;
        host_dbl = (double*)(c->pinned + 32);
        SMPS_HIP(c, hipMemsetAsync(ints, 0, 4 * sizeof(int), s));
        for (int k = 0; k < L; ++k)
            SMPS_HIP(c, hipMemcpyAsync(psi[k], Ak(k), sizeof(double2) * v->site_size(k), hipMemcpyDeviceToDevice, s));
        const double2 one = make_double2(1.0, 0.0);
        SMPS_HIP(c, hipMemcpyAsync(Lenv[0], &one, sizeof(double2), hipMemcpyHostToDevice, s));
        SMPS_HIP(c, hipMemcpyAsync(Renv[L], &one, sizeof(double2), hipMemcpyHostToDevice, s));
        // right-canonical guess (nothing truncated)
        for (int k = L - 1; k >= 1; --k) {
            const int rows = chi[k], len = d[k] * chi[k + 1];
            int r = 0;
            hipError_t e = svd_rows(psi[k], rows, len, rows, 0.0, SMPS_TRUNC_REL_NORM2, &r, nullptr);
            if (e != hipSuccess) return step_error(e);
            e = mm(psi[k], Q, x1, rows, r, len, ZN, ZH);  // carry psi_k Q^H
            if (e == hipSuccess) e = mm(psi[k - 1], x1, x2, chi[k - 1] * d[k - 1], r, rows, ZN, ZN);
            if (e == hipSuccess)
                e = hipMemcpyAsync(psi[k - 1], x2, sizeof(double2) * chi[k - 1] * d[k - 1] * r, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(psi[k], Q, sizeof(double2) * r * len, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return step_error(e);
            chi[k] = r;
        }
        for (int k = L - 1; k >= 1; --k) {
            hipError_t e = env_R(k);
            if (e != hipSuccess) return step_error(e);
        }
        if (L == 1) {  // the product of the single site: W_0 applied to A_0
            hipError_t e = mm(Lenv[0], Ak(0), x1, D[0], d[0] * cv[1], cv[0], ZN, ZN);
            if (e == hipSuccess) e = lmpo(x1, psi[0], 0, 1, cv[1]);
            if (e != hipSuccess) return step_error(e);
        }
        for (int sw = 0; sw < st.max_sweeps && L > 1; ++sw) {
            for (int k = 0; k + 1 < L; ++k) {
                hipError_t e = step(k, true);
                if (e != hipSuccess) return step_error(e);
            }
            for (int k = L - 2; k >= 0; --k) {
                hipError_t e = step(k, false);
                if (e != hipSuccess) return step_error(e);
            }
        }
        // result handle
        smps_zmps* res = new_zmps_handle(c);
        res->ctx = c;
        res->L = L;
        res->phys = d;
        res->bonds = chi;
        res->bonds[0] = res->bonds[L] = 1;
        res->off.resize(L);
        size_t tot = 0;
        for (int k = 0; k < L; ++k) {
            res->off[k] = tot;
            tot += res->site_size(k);
        }
        res->bytes = sizeof(double2) * std::max<size_t>(tot, 1);
        res->data = (double2*)dev_alloc(c, res->bytes);
        if (!res->data) {
            handle_untrack(res);
            delete res;
            return fail(c, SMPS_ENOMEM, "output allocation failed");
        }
        for (int k = 0; k < L; ++k)
            SMPS_HIP(c, hipMemcpyAsync(res->data + res->off[k], psi[k], sizeof(double2) * res->site_size(k),
                                       hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(znorm2_kernel, dim3(1), dim3(256), 0, s, res->data, (long long)res->site_size(0), dbl);
        SMPS_HIP(c, hipMemcpyAsync(host_dbl, dbl, sizeof(double), hipMemcpyDeviceToHost, s));
        SMPS_HIP(c, hipStreamSynchronize(s));
        c->info = smps_apply_info{};
        c->info.norm = std::sqrt(std::max(0.0, host_dbl[0]));
        c->info.sweeps_done = L > 1 ? st.max_sweeps : 0;
        c->info.steps = (int)deltas.size();
        double eb = 0.0, dsum = 0.0;
        for (double x : deltas) eb += std::sqrt(std::max(0.0, x)), dsum += x;
        c->info.error_bound = eb;
        c->info.discarded = dsum;
        if (trunc_err) *trunc_err = eb;
        *out = res;
        return SMPS_OK;
    }
};

}  // namespace
}  // namespace smps

using namespace smps;

extern "C" {

static int zcheck_chain(smps_ctx* c, int L, const int* phys, const int* bonds) {
    if (L < 1) return fail(c, SMPS_EINVAL, "L must be >= 1");
    if (!phys || !bonds) return fail(c, SMPS_EINVAL, "phys/bonds is NULL");
    if (bonds[0] != 1 || bonds[L] != 1) return fail(c, SMPS_EINVAL, "open boundary bonds must be 1");
    for (int k = 0; k < L; ++k)
        if (phys[k] < 1) return fail(c, SMPS_EINVAL, "physical dimensions must be >= 1");
    for (int k = 0; k <= L; ++k)
        if (bonds[k] < 1) return fail(c, SMPS_EINVAL, "bond dimensions must be >= 1");
    return SMPS_OK;
}

int smps_zmps_create(smps_ctx* c, int L, const int* phys, const int* bonds, const double* const* tensors,
                     smps_zmps** out) {
    if (!c) return SMPS_EINVAL;
    if (!out) return fail(c, SMPS_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = zcheck_chain(c, L, phys, bonds);
    if (rc) return rc;
    if (!tensors) return fail(c, SMPS_EINVAL, "tensors is NULL");
    rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipSetDevice(c->device));
    smps_zmps* m = new_zmps_handle(c);
    m->L = L;
    m->phys.assign(phys, phys + L);
    m->bonds.assign(bonds, bonds + L + 1);
    m->off.resize(L);
    size_t tot = 0;
    for (int k = 0; k < L; ++k) {
        m->off[k] = tot;
        tot += m->site_size(k);
    }
    m->bytes = sizeof(double2) * std::max<size_t>(tot, 1);
    m->data = (double2*)dev_alloc(c, m->bytes);
    if (!m->data) {
        handle_untrack(m);
        delete m;
        return fail(c, SMPS_ENOMEM, "allocation failed");
    }
    for (int k = 0; k < L; ++k) {
        if (!tensors[k]) {
            dev_release(c, m->data, m->bytes);
            handle_untrack(m);
            delete m;
            return fail(c, SMPS_EINVAL, "site tensor is NULL");
        }
        const hipError_t e = hipMemcpy(m->data + m->off[k], tensors[k], sizeof(double2) * m->site_size(k),
                                       hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            dev_release(c, m->data, m->bytes);
            handle_untrack(m);
            delete m;
            return fail(c, SMPS_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
        }
    }
    *out = m;
    return SMPS_OK;
}

int smps_zmps_destroy(smps_zmps* m) {
    if (!m) return SMPS_OK;
    if (!handle_untrack(m)) return SMPS_EINVAL;
    if (m->data) dev_release(m->ctx, m->data, m->bytes);
    delete m;
    return SMPS_OK;
}

int smps_zmps_shape(const smps_zmps* m, int* L, int* phys, int* bonds) {
    if (!m || !handle_live(m)) return SMPS_EINVAL;
    if (L) *L = m->L;
    if (phys) std::copy(m->phys.begin(), m->phys.end(), phys);
    if (bonds) std::copy(m->bonds.begin(), m->bonds.end(), bonds);
    return SMPS_OK;
}

int smps_zmps_read(smps_ctx* c, const smps_zmps* m, int site, double* host_out, size_t count) {
    if (!c) return SMPS_EINVAL;
    int rc = check_live(c, m, m && handle_live(m) ? m->ctx : nullptr, "complex MPS");
    if (rc) return rc;
    if (!host_out) return fail(c, SMPS_EINVAL, "NULL argument");
    if (site < 0 || site >= m->L) return fail(c, SMPS_EINVAL, "site out of range");
    if (count != m->site_size(site)) return fail(c, SMPS_EINVAL, "count does not match the site size");
    rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipSetDevice(c->device));
    SMPS_HIP(c, hipStreamSynchronize(c->stream));
    SMPS_HIP(c, hipMemcpy(host_out, m->data + m->off[site], sizeof(double2) * count, hipMemcpyDeviceToHost));
    return SMPS_OK;
}

int smps_zmpo_create(smps_ctx* c, int L, const int* pout, const int* pin, const int* bonds,
                     const double* const* tensors, smps_zmpo** out) {
    if (!c) return SMPS_EINVAL;
    if (!out) return fail(c, SMPS_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = zcheck_chain(c, L, pout, bonds);
    if (rc) return rc;
    rc = zcheck_chain(c, L, pin, bonds);
    if (rc) return rc;
    if (!tensors) return fail(c, SMPS_EINVAL, "tensors is NULL");
    rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipSetDevice(c->device));
    smps_zmpo* m = new_zmpo_handle(c);
    m->L = L;
    m->pout.assign(pout, pout + L);
    m->pin.assign(pin, pin + L);
    m->bonds.assign(bonds, bonds + L + 1);
    m->off.resize(L);
    size_t tot = 0;
    for (int k = 0; k < L; ++k) {
        m->off[k] = tot;
        tot += m->site_size(k);
    }
    m->bytes = sizeof(double2) * std::max<size_t>(tot, 1);
    m->data = (double2*)dev_alloc(c, m->bytes);
    if (!m->data) {
        handle_untrack(m);
        delete m;
        return fail(c, SMPS_ENOMEM, "allocation failed");
    }
    for (int k = 0; k < L; ++k) {
        if (!tensors[k]) {
            dev_release(c, m->data, m->bytes);
            handle_untrack(m);
            delete m;
            return fail(c, SMPS_EINVAL, "site tensor is NULL");
        }
        const hipError_t e = hipMemcpy(m->data + m->off[k], tensors[k], sizeof(double2) * m->site_size(k),
                                       hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            dev_release(c, m->data, m->bytes);
            handle_untrack(m);
            delete m;
            return fail(c, SMPS_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
        }
    }
    *out = m;
    return SMPS_OK;
}

int smps_zmpo_destroy(smps_zmpo* m) {
    if (!m) return SMPS_OK;
    if (!handle_untrack(m)) return SMPS_EINVAL;
    if (m->data) dev_release(m->ctx, m->data, m->bytes);
    delete m;
    return SMPS_OK;
}

int smps_zmpo_apply(smps_ctx* c, const smps_zmpo* U, const smps_zmps* v, const smps_strategy* st, smps_zmps** out,
                    double* trunc_err) {
    if (!c) return SMPS_EINVAL;
    if (!out) return fail(c, SMPS_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_live(c, U, U && handle_live(U) ? U->ctx : nullptr, "complex MPO");
    if (rc) return rc;
    rc = check_live(c, v, v && handle_live(v) ? v->ctx : nullptr, "complex MPS");
    if (rc) return rc;
    if (!st) return fail(c, SMPS_EINVAL, "strategy is NULL");
    if (st->max_bond < 1 || !(st->tol >= 0.0) || !std::isfinite(st->tol) || st->max_sweeps < 1)
        return fail(c, SMPS_EINVAL, "bad strategy");
    if (st->trunc_mode != SMPS_TRUNC_REL_NORM2 && st->trunc_mode != SMPS_TRUNC_REL_SV)
        return fail(c, SMPS_EINVAL, "unknown truncation mode");
    if (st->precision != SMPS_PREC_FP64 || st->factorization != SMPS_FACT_SVD)
        return fail(c, SMPS_EUNSUPPORTED, "complex apply runs in FP64 with the exact factorization");
    if (U->L != v->L) return fail(c, SMPS_EINVAL, "operator and state lengths differ");
    for (int k = 0; k < v->L; ++k)
        if (U->pin[k] != v->phys[k] || U->pout[k] != v->phys[k])
            return fail(c, SMPS_EUNSUPPORTED, "complex apply needs square operator sites matching the state");
    rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipSetDevice(c->device));
    ZApply za(c, U, v, *st);
    return za.run(out, trunc_err);
}

// <a, b> = sum conj(a) b by the transfer-matrix sweep (Sec. 2.4.4)
int smps_zscprod(smps_ctx* c, const smps_zmps* a, const smps_zmps* b, double* re, double* im) {
    if (!c) return SMPS_EINVAL;
    int rc = check_live(c, a, a && handle_live(a) ? a->ctx : nullptr, "complex MPS");
    if (rc) return rc;
    rc = check_live(c, b, b && handle_live(b) ? b->ctx : nullptr, "complex MPS");
    if (rc) return rc;
    if (a->L != b->L || a->phys != b->phys) return fail(c, SMPS_EINVAL, "shapes do not match");
    rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipSetDevice(c->device));
    const int L = a->L;
    size_t ne = 1, nt = 1;
    for (int k = 0; k <= L; ++k) ne = std::max(ne, (size_t)a->bonds[k] * b->bonds[k]);
    for (int k = 0; k < L; ++k) nt = std::max(nt, (size_t)a->bonds[k] * a->phys[k] * b->bonds[k + 1]);
    double2 *E = nullptr, *T = nullptr;
    SMPS_HIP(c, hipMalloc(&E, sizeof(double2) * ne));
    hipError_t e = hipMalloc(&T, sizeof(double2) * nt);
    if (e != hipSuccess) {
        hipFree(E);
        return fail(c, SMPS_ENOMEM, "allocation failed");
    }
    const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
    e = hipMemcpyAsync(E, &one, sizeof(double2), hipMemcpyHostToDevice, c->stream);
    for (int k = 0; k < L && e == hipSuccess; ++k) {
        const int ca = a->bonds[k], cb = b->bonds[k], s = a->phys[k], ca1 = a->bonds[k + 1], cb1 = b->bonds[k + 1];
        // T[a][s d] = E (ca x cb) B (cb x s cb1); E' = A^H (ca1 x ca s) T (ca s x cb1)
        hipLaunchKernelGGL(zgemm_kernel, dim3((s * cb1 + 15) / 16, (ca + 15) / 16, 1), dim3(256), 0, c->stream, E,
                           b->data + b->off[k], T, ca, s * cb1, cb, (int)ZN, (int)ZN, one, zero, 0LL, 0LL, 0LL);
        hipLaunchKernelGGL(zgemm_kernel, dim3((cb1 + 15) / 16, (ca1 + 15) / 16, 1), dim3(256), 0, c->stream,
                           a->data + a->off[k], T, E, ca1, cb1, ca * s, (int)ZH, (int)ZN, one, zero, 0LL, 0LL, 0LL);
        e = hipGetLastError();
    }
    double2 h = make_double2(0.0, 0.0);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, E, sizeof(double2), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    hipFree(E);
    hipFree(T);
    if (e != hipSuccess) return fail(c, SMPS_EHIP, std::string("complex scprod: ") + hipGetErrorString(e));
    if (re) *re = h.x;
    if (im) *im = h.y;
    return SMPS_OK;
}

}  // extern "C"
