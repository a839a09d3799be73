// Two-site DMRG (Sec. 3.1.1) on the device: the ground state of a real
// symmetric MPO H.
//
// With the state in mixed canonical form around the pair (k, k+1) the norm
// form of the pair is the identity, so the local problem is H_k a = E a with
// H_k a = L[k] W_k W_{k+1} R[k+2] a (three-layer environments of <psi|H|psi>).
// It is solved matrix-free by Lanczos: every product with H_k is two GEMMs
// and two MPO-site contractions on the device; the Krylov basis stays on the
// device and every new vector is re-orthogonalised against it twice (one
// workgroup per basis vector for the projections, one pass for the update);
// only the small tridiagonal eigenproblem (at most a few tens of rows) is
// solved on the host.  The pair
// is then split by the one-sided Jacobi SVD with the strategy's truncation and
// the environment on the side the centre leaves is extended.  Bond dimensions
// are read back after every split, so every launch here has host-known sizes.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime.h"

namespace smps {

namespace {

// out[0] = <x, y> over n doubles, one workgroup, fixed summation order
__global__ __launch_bounds__(1024) void dot_kernel(const double* x, const double* y, long long n, double* out) {
    __shared__ double part[1024];
    double a = 0.0;
    for (long long i = threadIdx.x; i < n; i += 1024) a = fma(x[i], y[i], a);
    part[threadIdx.x] = a;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0];
}

// B (cols x rows) = A^T, A rows x cols
__global__ void transpose_kernel(const double* A, double* B, int rows, int cols) {
    const long long n = (long long)rows * cols;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(e / cols), c = (int)(e % cols);
        B[(long long)c * rows + r] = A[e];
    }
}

// h[i] = <V_i, w> for the rows i < rows of V (row stride n): one workgroup per
// row, fixed summation order
__global__ __launch_bounds__(256) void multidot_kernel(const double* V, long long n, const double* w, double* h) {
    __shared__ double part[256];
    const double* v = V + (long long)blockIdx.x * n;
    double a = 0.0;
    for (long long x = threadIdx.x; x < n; x += 256) a = fma(v[x], w[x], a);
    part[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) h[blockIdx.x] = part[0];
}

// w -= sum_{i < rows} h[i] V_i (coalesced along the vector)
__global__ void project_out_kernel(const double* V, long long n, int rows, const double* h, double* w) {
    for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < n; x += (long long)gridDim.x * blockDim.x) {
        double a = w[x];
        for (int i = 0; i < rows; ++i) a = fma(-h[i], V[(long long)i * n + x], a);
        w[x] = a;
    }
}

// w = sum_{i < rows} y[i] V_i
__global__ void combine_rows_kernel(const double* V, long long n, int rows, const double* y, double* w) {
    for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < n; x += (long long)gridDim.x * blockDim.x) {
        double a = 0.0;
        for (int i = 0; i < rows; ++i) a = fma(y[i], V[(long long)i * n + x], a);
        w[x] = a;
    }
}

// dst = src / sqrt(*nrm2); zero when the norm is at most rel * |*ref| (ref
// non-NULL: Lanczos breakdown) or not positive
__global__ void normalize_kernel(const double* src, double* dst, long long n, const double* nrm2, const double* ref,
                                 double rel) {
    const double b = sqrt(fmax(*nrm2, 0.0));
    const bool zero = !(b > 1e-300) || (ref && !(b > rel * fabs(*ref)));
    const double inv = zero ? 0.0 : 1.0 / b;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = src[i] * inv;
}

__global__ void scale_kernel(double* x, double a, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] *= a;
}

int blocks_for(long long n) { return (int)std::max<long long>(1, std::min<long long>(1024, (n + 255) / 256)); }

// Lowest eigenpair of a small symmetric matrix (row-major, m x m) by cyclic
// Jacobi rotations (Golub & Van Loan, Alg. 8.5.3); returns the eigenvalue and
// writes the normalised eigenvector.
double smallest_eigenpair(std::vector<double> A, int m, std::vector<double>& vec) {
    std::vector<double> V((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                const double a = A[(size_t)i * m + j];
                tot += a * a;
                if (i != j) off += a * a;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = A[(size_t)p * m + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < m; ++k) {  // A <- J^T A J, columns p, q
                    const double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
                    A[(size_t)k * m + p] = c * akp - s * akq;
                    A[(size_t)k * m + q] = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {  // rows p, q
                    const double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
                    A[(size_t)p * m + k] = c * apk - s * aqk;
                    A[(size_t)q * m + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) {  // V <- V J
                    const double vkp = V[(size_t)k * m + p], vkq = V[(size_t)k * m + q];
                    V[(size_t)k * m + p] = c * vkp - s * vkq;
                    V[(size_t)k * m + q] = s * vkp + c * vkq;
                }
            }
    }
    int best = 0;
    for (int i = 1; i < m; ++i)
        if (A[(size_t)i * m + i] < A[(size_t)best * m + best]) best = i;
    vec.assign(m, 0.0);
    for (int k = 0; k < m; ++k) vec[k] = V[(size_t)k * m + best];
    return A[(size_t)best * m + best];
}

struct Dmrg {
    smps_ctx* c;
    hipStream_t s;
    const smps_mpo* H;
    const smps_strategy& st;
    int L, m;
    std::vector<int> d, D, chi, cap;
    std::vector<double*> psi, Lenv, Renv;
    // per bond: the singular basis the last split there left (len x len of that
    // factorization, the identity when its vectors did not span), and that len
    // (0: none yet).  The next split at the bond pre-rotates its vectors by it
    // when their count equals that len (the opposite visit's orientation).
    std::vector<double*> basis;
    std::vector<int> basis_dim;
    double* jx2 = nullptr;
    double *theta = nullptr, *V = nullptr, *w = nullptr, *x1 = nullptr, *x2 = nullptr, *x3 = nullptr;
    double *jx = nullptr, *Q = nullptr, *sigma = nullptr, *scal = nullptr, *fro2 = nullptr, *tmp = nullptr;
    int* ints = nullptr;  // [rank, status, flag, perm...]
    double* hc = nullptr;    // Lanczos coefficients: 2 (m+1)^2 projections, m+1 |w|^2, m+1 Ritz weights
    double* host = nullptr;  // pinned staging of hc
    int* host_ints = nullptr;  // pinned staging of the factorization's rank and status
    static constexpr double BREAKDOWN = 1e-12;  // beta <= BREAKDOWN |alpha|: invariant subspace found
    // stop once beta_j |y_j| <= RESIDUAL |E|: the Ritz value is then within
    // about (RESIDUAL |E|)^2 / gap of the local eigenvalue, far below the
    // truncation error, and the next visit of the pair refines the vector
    static constexpr double RESIDUAL = 1e-7;
    static constexpr int CHUNK = 4;  // Lanczos iterations between read-backs of the coefficients
    std::vector<void*> allocs;
    double energy = 0.0;
    int status_seen = 0;  // factorization status that stopped the run
    size_t nth = 0;  // largest two-site size

    Dmrg(smps_ctx* c_, const smps_mpo* H_, const smps_strategy& st_, int m_) : c(c_), s(c_->stream), H(H_), st(st_), m(m_) {}
    ~Dmrg() {
        for (void* p : allocs) hipFree(p);
    }

    template <typename T>
    T* alloc(size_t n) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
        allocs.push_back(p);
        return (T*)p;
    }

    const double* W(int k) const { return H->data + H->off[k]; }

    hipError_t mm(const double* A, const double* B, double* C, int M, int N, int K, int ta, int tb, double alpha = 1.0,
                  double beta = 0.0) {
        GemmDesc g{};
        g.A = A;
        g.B = B;
        g.C = C;
        g.dims = nullptr;
        g.M = dconst(M);
        g.N = dconst(N);
        g.K = dconst(K);
        g.ta = ta;
        g.tb = tb;
        g.tc = 0;
        g.a_type = g.b_type = g.c_type = T_F64;
        g.alpha = alpha;
        g.beta = beta;
        return launch_gemm(g, M, N, 1, s, P_F64);
    }

    // Y[a][t][b'][y] = sum_{b,q} X[a][b][q][y] W[b][t][q][b']
    hipError_t lmpo(const double* X, double* Y, int k, int a, int ny) {
        LeftMpoDesc dd{};
        dd.X = X;
        dd.Y = Y;
        dd.B = W(k);
        dd.dims = nullptr;
        dd.a = dconst(a);
        dd.Dl = D[k];
        dd.e = d[k];
        dd.d = d[k];
        dd.Dr = D[k + 1];
        dd.ny = ny;
        dd.x_type = dd.y_type = T_F64;
        return launch_left_mpo(dd, a, s);
    }

    // Y[b][x][t][c] = sum_{q,b'} W[b][t][q][b'] X[x][q][c][b']
    hipError_t rmpo(const double* X, double* Y, int k, int nx, int cc) {
        RightMpoDesc dd{};
        dd.X = X;
        dd.Y = Y;
        dd.B = W(k);
        dd.dims = nullptr;
        dd.c = dconst(cc);
        dd.Dl = D[k];
        dd.e = d[k];
        dd.d = d[k];
        dd.Dr = D[k + 1];
        dd.nx = nx;
        dd.x_type = dd.y_type = T_F64;
        return launch_right_mpo(dd, cc, s);
    }

    hipError_t dot(const double* x, const double* y, long long n, double* host) {
        hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(1024), 0, s, x, y, n, scal);
        hipError_t e = hipMemcpyAsync(host, scal, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);
    }

    hipError_t scale(double* x, double a, long long n) {
        hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(n)), dim3(256), 0, s, x, a, n);
        return hipGetLastError();
    }

    hipError_t transpose(const double* A, double* B, int rows, int cols) {
        const long long n = (long long)rows * cols;
        hipLaunchKernelGGL(transpose_kernel, dim3(blocks_for(n)), dim3(256), 0, s, A, B, rows, cols);
        return hipGetLastError();
    }

    // Rows of X (nv x ln) orthogonalised; the first r rows of Q are the kept
    // right singular vectors.  tol < 0: keep every nonzero value (no truncation).
    hipError_t svd_rows(double* X, int nv, int ln, int max_rank, double tol, int* r_out, int bond = -1) {
        if (bond >= 0 && basis_dim[bond] == nv) {  // warm start
            hipError_t e = mm(basis[bond], X, jx2, nv, ln, nv, 0, 0);
            if (e != hipSuccess) return e;
            X = jx2;
        }
        JacobiDesc jd{};
        if (bond >= 0) {
            jd.basis = basis[bond];
            basis_dim[bond] = ln;
        }
        jd.X = X;
        jd.Q = Q;
        jd.sigma = sigma;
        jd.perm = ints + 3;
        jd.dims_in = ints;
        jd.dims_out = ints;
        jd.nvec = dconst(nv);
        jd.len = dconst(ln);
        jd.rank_idx = 0;
        jd.max_rank = max_rank;
        jd.tol = tol < 0 ? 0.0 : tol;
        jd.mode = tol < 0 ? SMPS_TRUNC_REL_NORM2 : st.trunc_mode;
        jd.status = ints + 1;
        jd.fro2 = fro2;
        jd.conv = ints + 2;
        jd.floor_eps = 2.220446049250313e-16;
        hipError_t e = launch_jacobi(jd, nv, ln, nullptr, ints + 2, s);
        if (e != hipSuccess) return e;
        int* h = host_ints;
        e = hipMemcpyAsync(h, ints, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (h[1]) {  // bit 0: non-finite input, bit 1: no convergence
            status_seen = h[1];
            return hipErrorInvalidValue;
        }
        *r_out = h[0];
        return hipSuccess;
    }

    // R[k] from R[k+1] and psi_k (bra = ket): T = psi_k R[k+1]^T, Y = W_k . T, R[k] = psi_k Y^T
    hipError_t env_R(int k) {
        const int x = chi[k], q = d[k], cc = chi[k + 1];
        hipError_t e = mm(psi[k], Renv[k + 1], x1, x * q, cc * D[k + 1], cc, 0, 1);
        if (e != hipSuccess) return e;
        e = rmpo(x1, x2, k, x, cc);
        if (e != hipSuccess) return e;
        return mm(psi[k], x2, Renv[k], x, D[k] * x, q * cc, 0, 1);
    }

    // L[k+1] from L[k] and psi_k: T = L[k] psi_k, Y = T . W_k, L[k+1] = psi_k^T Y
    hipError_t env_L(int k) {
        const int a = chi[k], q = d[k], r = chi[k + 1];
        hipError_t e = mm(Lenv[k], psi[k], x1, a * D[k], q * r, a, 0, 0);
        if (e != hipSuccess) return e;
        e = lmpo(x1, x2, k, a, r);
        if (e != hipSuccess) return e;
        return mm(psi[k], x2, Lenv[k + 1], r, D[k + 1] * r, a * q, 1, 0);
    }

    // out = H_k in for the pair (k, k+1) with the current bonds
    hipError_t matvec(int k, const double* in, double* out) {
        const int a = chi[k], sd = d[k], td = d[k + 1], cc = chi[k + 2];
        hipError_t e = mm(Lenv[k], in, x1, a * D[k], sd * td * cc, a, 0, 0);
        if (e != hipSuccess) return e;
        e = lmpo(x1, x2, k, a, td * cc);
        if (e != hipSuccess) return e;
        e = lmpo(x2, x3, k + 1, a * sd, cc);
        if (e != hipSuccess) return e;
        return mm(x3, Renv[k + 2], out, a * sd * td, cc, D[k + 2] * cc, 0, 1);
    }

    // Lanczos with full re-orthogonalisation (two Gram-Schmidt passes by GEMMs)
    // on the pair tensor in theta; theta is replaced by the lowest Ritz vector.
    // The recurrence runs on the device: the projections of pass 1 and pass 2
    // of iteration j land in row j of hc[0] / hc[1], |w|^2 in bn[j], and the next
    // basis vector is normalised by a kernel reading bn[j] (zero on breakdown).
    // The host reads the coefficients once per chunk of iterations (pinned),
    // solves the small tridiagonal problem and stops when the Ritz residual
    // beta_j |y_j| is small or the Krylov space is exhausted.
    hipError_t lanczos(int k) {
        const long long n = (long long)chi[k] * d[k] * d[k + 1] * chi[k + 2];
        const int mmax = (int)std::min<long long>(m, n);
        const int ld = m + 1;
        double* hc0 = hc;
        double* hc1 = hc + (size_t)ld * ld;
        double* bn = hc + 2 * (size_t)ld * ld;
        hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(1024), 0, s, theta, theta, n, scal);
        hipLaunchKernelGGL(normalize_kernel, dim3(blocks_for(n)), dim3(256), 0, s, theta, V, n, scal,
                           (const double*)nullptr, 0.0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        int j = 0, mk = 0;
        std::vector<double> y;
        bool done = false;
        while (!done) {
            const int j1 = std::min(mmax, j + CHUNK);
            for (; j < j1; ++j) {
                const double* vj = V + (size_t)j * n;
                e = matvec(k, vj, w);
                if (e != hipSuccess) return e;
                for (int pass = 0; pass < 2; ++pass) {
                    double* h = (pass ? hc1 : hc0) + (size_t)j * ld;
                    hipLaunchKernelGGL(multidot_kernel, dim3(j + 1), dim3(256), 0, s, V, n, w, h);
                    hipLaunchKernelGGL(project_out_kernel, dim3(blocks_for(n)), dim3(256), 0, s, V, n, j + 1, h, w);
                    e = hipGetLastError();
                    if (e != hipSuccess) return e;
                }
                hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(1024), 0, s, w, w, n, bn + j);
                hipLaunchKernelGGL(normalize_kernel, dim3(blocks_for(n)), dim3(256), 0, s, w, V + (size_t)(j + 1) * n,
                                   n, bn + j, hc0 + (size_t)j * ld + j, BREAKDOWN);
                e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
            const size_t nb = (2 * (size_t)ld * ld + ld) * sizeof(double);
            e = hipMemcpyAsync(host, hc, nb, hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) return e;
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) return e;
            const double* h0 = host;
            const double* hb = host + 2 * (size_t)ld * ld;
            // Krylov size: up to the first breakdown (the same test as the kernel's)
            mk = j;
            for (int i = 0; i < j; ++i) {
                const double b = std::sqrt(std::max(0.0, hb[i]));
                if (!(b > BREAKDOWN * std::fabs(h0[(size_t)i * ld + i])) || !(b > 1e-300)) {
                    mk = i + 1;
                    done = true;
                    break;
                }
            }
            std::vector<double> T((size_t)mk * mk, 0.0);
            for (int i = 0; i < mk; ++i) {
                T[(size_t)i * mk + i] = h0[(size_t)i * ld + i];
                if (i + 1 < mk) T[(size_t)i * mk + i + 1] = T[(size_t)(i + 1) * mk + i] = std::sqrt(hb[i]);
            }
            energy = smallest_eigenpair(T, mk, y);
            const double resid = std::sqrt(std::max(0.0, hb[mk - 1])) * std::fabs(y[mk - 1]);
            if (j >= mmax || resid <= RESIDUAL * std::max(std::fabs(energy), 1e-300)) done = true;
        }
        // theta = V^T y, normalised
        double* yd = hc + 2 * (size_t)ld * ld + ld;
        std::memcpy(host, y.data(), sizeof(double) * mk);
        e = hipMemcpyAsync(yd, host, sizeof(double) * mk, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(combine_rows_kernel, dim3(blocks_for(n)), dim3(256), 0, s, V, n, mk, yd, w);
        hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(1024), 0, s, w, w, n, scal);
        hipLaunchKernelGGL(normalize_kernel, dim3(blocks_for(n)), dim3(256), 0, s, w, theta, n, scal,
                           (const double*)nullptr, 0.0);
        return hipGetLastError();
    }

    hipError_t step(int k, bool left_to_right) {
        const int a = chi[k], sd = d[k], td = d[k + 1], cc = chi[k + 2];
        // theta = psi_k psi_{k+1}
        hipError_t e = mm(psi[k], psi[k + 1], theta, a * sd, td * cc, chi[k + 1], 0, 0);
        if (e != hipSuccess) return e;
        e = lanczos(k);
        if (e != hipSuccess) return e;
        const int mr = std::min(st.max_bond, cap[k + 1]);
        int r = 0;
        if (left_to_right) {
            // left isometry: rows of theta^T are the columns of theta
            e = transpose(theta, jx, a * sd, td * cc);
            if (e != hipSuccess) return e;
            e = svd_rows(jx, td * cc, a * sd, mr, st.tol, &r, k);
            if (e != hipSuccess) return e;
            e = transpose(Q, psi[k], r, a * sd);  // psi_k = U (a s x r)
            if (e != hipSuccess) return e;
            e = mm(Q, theta, psi[k + 1], r, td * cc, a * sd, 0, 0);  // psi_{k+1} = U^T theta
            if (e != hipSuccess) return e;
            chi[k + 1] = r;
            return env_L(k);
        }
        e = hipMemcpyAsync(jx, theta, sizeof(double) * (size_t)a * sd * td * cc, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = svd_rows(jx, a * sd, td * cc, mr, st.tol, &r, k);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(psi[k + 1], Q, sizeof(double) * (size_t)r * td * cc, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = mm(theta, Q, psi[k], a * sd, r, td * cc, 0, 1);  // psi_k = theta V
        if (e != hipSuccess) return e;
        chi[k + 1] = r;
        return env_R(k + 1);
    }

    int step_error(hipError_t e) {
        if (status_seen & 1) return fail(c, SMPS_ENUMERIC, "DMRG: non-finite values in a two-site tensor");
        if (status_seen & 2) return fail(c, SMPS_ENUMERIC, "DMRG: factorization did not converge");
        return fail(c, SMPS_EHIP, std::string("DMRG step: ") + hipGetErrorString(e));
    }

    int run(const smps_mps* guess, smps_mps** out, double* energy_out) {
        L = guess->L;
        d = guess->phys;
        D = H->bonds;
        chi = guess->bonds;
        std::vector<long long> left(L + 1, 1), right(L + 1, 1);
        for (int k = 1; k <= L; ++k) left[k] = std::min<long long>(left[k - 1] * d[k - 1], 1LL << 40);
        for (int k = L - 1; k >= 0; --k) right[k] = std::min<long long>(right[k + 1] * d[k], 1LL << 40);
        cap.resize(L + 1);
        for (int k = 0; k <= L; ++k)
            cap[k] = (int)std::max<long long>(chi[k], std::min<long long>(st.max_bond, std::min(left[k], right[k])));
        int dmax = 1, Dmax = 1;
        for (int k = 0; k < L; ++k) dmax = std::max(dmax, d[k]);
        for (int k = 0; k <= L; ++k) Dmax = std::max(Dmax, D[k]);
        size_t nx = 1;
        for (int k = 0; k + 1 < L; ++k) {
            nth = std::max(nth, (size_t)cap[k] * d[k] * d[k + 1] * cap[k + 2]);
            nx = std::max(nx, (size_t)cap[k] * Dmax * d[k] * d[k + 1] * cap[k + 2] * Dmax);
        }
        for (int k = 0; k < L; ++k) {
            nth = std::max(nth, (size_t)cap[k] * d[k] * cap[k + 1]);
            nx = std::max(nx, (size_t)cap[k] * Dmax * dmax * cap[k + 1] * Dmax);
        }
        int nvmax = 1;
        for (int k = 0; k + 1 < L; ++k) nvmax = std::max({nvmax, cap[k] * d[k], d[k + 1] * cap[k + 2]});
        for (int k = 0; k <= L; ++k) nvmax = std::max(nvmax, cap[k]);
        if (nvmax > 2048)
            return fail(c, SMPS_EUNSUPPORTED, "two-site tensors with more than 2048 rows or columns are not supported");
        psi.assign(L, nullptr);
        Lenv.assign(L + 1, nullptr);
        Renv.assign(L + 1, nullptr);
        bool ok = true;
        for (int k = 0; k < L; ++k) ok = ok && (psi[k] = alloc<double>((size_t)cap[k] * d[k] * cap[k + 1]));
        for (int k = 0; k <= L; ++k) {
            ok = ok && (Lenv[k] = alloc<double>((size_t)cap[k] * D[k] * cap[k]));
            ok = ok && (Renv[k] = alloc<double>((size_t)cap[k] * D[k] * cap[k]));
        }
        ok = ok && (theta = alloc<double>(nth)) && (V = alloc<double>(nth * (size_t)(m + 1))) &&
             (w = alloc<double>(nth)) && (x1 = alloc<double>(nx)) && (x2 = alloc<double>(nx)) &&
             (x3 = alloc<double>(nx)) && (jx = alloc<double>(nth)) && (jx2 = alloc<double>(nth)) &&
             (Q = alloc<double>(nth)) &&
             (sigma = alloc<double>(nvmax)) && (scal = alloc<double>(1)) && (fro2 = alloc<double>(1)) &&
             (tmp = alloc<double>(std::max<size_t>(nth, (size_t)m + 1))) && (ints = alloc<int>(3 + (size_t)nvmax)) &&
             (hc = alloc<double>(2 * (size_t)(m + 1) * (m + 1) + 2 * (size_t)(m + 1)));
        basis.assign(std::max(0, L - 1), nullptr);
        basis_dim.assign(std::max(0, L - 1), 0);
        for (int k = 0; k + 1 < L; ++k) {
            const size_t nb = std::max((size_t)cap[k] * d[k], (size_t)d[k + 1] * cap[k + 2]);
            ok = ok && (basis[k] = alloc<double>(nb * nb));
        }
        if (!ok) return fail(c, SMPS_ENOMEM, "DMRG workspace allocation failed");
        {
            const size_t hb = (2 * (size_t)(m + 1) * (m + 1) + 2 * (size_t)(m + 1)) * sizeof(double);
            int rc = ensure_pinned(c, hb + 64);
            if (rc) return rc;
            host = (double*)c->pinned;
            host_ints = (int*)(c->pinned + hb);
        }
        for (int k = 0; k < L; ++k)
            SMPS_HIP(c, hipMemcpyAsync(psi[k], guess->data + guess->off[k], 8 * guess->site_size(k),
                                       hipMemcpyDeviceToDevice, s));
        SMPS_HIP(c, hipMemsetAsync(ints, 0, sizeof(int) * 3, s));
        const double one = 1.0;
        SMPS_HIP(c, hipMemcpyAsync(Lenv[0], &one, sizeof(double), hipMemcpyHostToDevice, s));
        SMPS_HIP(c, hipMemcpyAsync(Renv[L], &one, sizeof(double), hipMemcpyHostToDevice, s));
        // right-canonical form of the guess (nothing truncated), then a unit norm
        for (int k = L - 1; k >= 1; --k) {
            const int rows = chi[k], len = d[k] * chi[k + 1];
            SMPS_HIP(c, hipMemcpyAsync(jx, psi[k], sizeof(double) * rows * len, hipMemcpyDeviceToDevice, s));
            int r = 0;
            hipError_t e = svd_rows(jx, rows, len, rows, -1.0, &r);
            if (e != hipSuccess) return step_error(e);
            if (r == 0) return fail(c, SMPS_EINVAL, "the guess has zero norm");
            SMPS_HIP(c, mm(psi[k], Q, x1, rows, r, len, 0, 1));                   // carry = psi_k V
            SMPS_HIP(c, mm(psi[k - 1], x1, x2, chi[k - 1] * d[k - 1], r, rows, 0, 0));
            SMPS_HIP(c, hipMemcpyAsync(psi[k - 1], x2, sizeof(double) * chi[k - 1] * d[k - 1] * r,
                                       hipMemcpyDeviceToDevice, s));
            SMPS_HIP(c, hipMemcpyAsync(psi[k], Q, sizeof(double) * r * len, hipMemcpyDeviceToDevice, s));
            chi[k] = r;
        }
        {
            const long long n0 = (long long)d[0] * chi[1];
            double nn = 0.0;
            SMPS_HIP(c, dot(psi[0], psi[0], n0, &nn));
            if (!(nn > 0.0)) return fail(c, SMPS_EINVAL, "the guess has zero norm");
            SMPS_HIP(c, scale(psi[0], 1.0 / std::sqrt(nn), n0));
        }
        for (int k = L - 1; k >= 1; --k) SMPS_HIP(c, env_R(k));
        double prev = 0.0;
        int sweeps_done = 0;
        for (int sw = 0; sw < st.max_sweeps; ++sw) {
            for (int k = 0; k + 1 < L; ++k) {
                hipError_t e = step(k, true);
                if (e != hipSuccess) return step_error(e);
            }
            for (int k = L - 2; k >= 0; --k) {
                hipError_t e = step(k, false);
                if (e != hipSuccess) return step_error(e);
            }
            ++sweeps_done;
            if (st.sweep_tol > 0.0 && sw > 0 && std::fabs(energy - prev) <= st.sweep_tol * std::fabs(energy)) break;
            prev = energy;
        }
        SMPS_HIP(c, hipStreamSynchronize(s));
        std::vector<int> bonds = chi;
        bonds[0] = bonds[L] = 1;
        smps_mps* res = new_mps(c, L, d, bonds);
        if (!res) return fail(c, SMPS_ENOMEM, "output allocation failed");
        for (int k = 0; k < L; ++k)
            SMPS_HIP(c, hipMemcpyAsync(res->data + res->off[k], psi[k], 8 * res->site_size(k),
                                       hipMemcpyDeviceToDevice, s));
        SMPS_HIP(c, hipStreamSynchronize(s));
        res->center = 0;
        c->info = smps_apply_info{};
        c->info.sweeps_done = sweeps_done;
        c->info.steps = sweeps_done * 2 * (L - 1);
        c->info.norm = 1.0;
        *out = res;
        if (energy_out) *energy_out = energy;
        return SMPS_OK;
    }
};

}  // namespace

int run_dmrg(smps_ctx* c, const smps_mpo* H, const smps_mps* guess, const smps_strategy& st, int krylov,
             smps_mps** out, double* energy) {
    Dmrg dm(c, H, st, krylov);
    return dm.run(guess, out, energy);
}

}  // namespace smps
