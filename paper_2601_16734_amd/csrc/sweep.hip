// The apply + compression sweep (Sec. 2.3 Eq. simplification, Sec. 2.4.2,
// Sec. 2.5): host-side planning and the enqueue of every kernel.
//
// Layouts (compact, row-major, live bond dimensions):
//   psi[k]  (chi_k, e_k, chi_{k+1})                        FP64
//   Lenv[k] (chi_k, D_k, chiv_k)  contraction of sites < k     env type
//   Renv[k] (chi_k, D_k, chiv_k)  contraction of sites >= k    env type
//   XL[k]   (chi_k, e_k, D_{k+1}, chiv_{k+1}) = Lenv[k] A_k B_k
//   XR[k]   (D_k, chiv_k, e_k, chi_{k+1})     = B_k A_k Renv[k+1]
//   theta   (chi_k e_k) x (e_{k+1} chi_{k+2}) = XL[k] XR[k+1]   FP64
// psi's bond dimensions live in a device array so nothing waits on the host.
// XL[k] built in a left-to-right step is still valid when the right-to-left
// pass reaches bond k (and XR[k+1] likewise in the other direction), so each
// two-site update builds one new X tensor, one theta, one factorization and
// one environment.

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>

#include "runtime.h"

namespace smps {

namespace {

constexpr size_t ALIGN = 256;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
    size_t total = 0;
    size_t add(size_t bytes) {
        size_t o = total;
        total += align_up(bytes ? bytes : 1);
        return o;
    }
};

long long sat_mul(long long a, long long b) {
    if (a > INT_MAX / std::max(1LL, b)) return INT_MAX;
    return a * b;
}

}  // namespace

// Everything the enqueue needs about one problem: shapes, caps and offsets.
struct Plan {
    int L = 0;
    int prec = P_F64;
    int et = T_F64;     // storage type of environments / X tensors
    size_t es = 8;      // its size
    std::vector<int> e, dv, Dm, chiv, capb;
    // offsets into the workspace
    size_t o_dims, o_status, o_flag, o_norm2, o_fro2;
    std::vector<size_t> o_psi, o_L, o_R, o_XL, o_XR, o_basis;
    size_t o_tmp, o_theta, o_theta2, o_Q, o_carry, o_tmpB, o_sigma, o_perm;
    size_t o_ldelta, o_lrank, o_lspec, o_lnorm2, o_lsweeps;
    size_t o_R64a, o_R64b, o_XR64, o_Y64;
    int steps = 0;
    size_t max_theta = 0, max_tmp = 0, max_env = 0, max_xr = 0;
    int max_nvec = 0;
};

static void plan_problem(Plan& p, const smps_mpo* U, const smps_mps* v, const smps_strategy& st, Layout& lay) {
    const int L = v->L;
    p.L = L;
    p.prec = st.precision;
    p.et = st.precision == SMPS_PREC_FP64 ? T_F64 : T_F32;
    p.es = p.et == T_F64 ? 8 : 4;
    p.e.resize(L);
    p.dv.resize(L);
    p.Dm.resize(L + 1);
    p.chiv = v->bonds;
    for (int k = 0; k < L; ++k) {
        p.e[k] = U->pout[k];
        p.dv[k] = v->phys[k];
        p.Dm[k] = U->bonds[k];
    }
    p.Dm[L] = U->bonds[L];
    // bond caps: max(min(max_bond, physical limit), bond of the guess)
    std::vector<long long> left(L + 1, 1), right(L + 1, 1);
    for (int k = 1; k <= L; ++k) left[k] = sat_mul(left[k - 1], p.e[k - 1]);
    for (int k = L - 1; k >= 0; --k) right[k] = sat_mul(right[k + 1], p.e[k]);
    p.capb.resize(L + 1);
    for (int k = 0; k <= L; ++k) {
        long long phys = std::min(left[k], right[k]);
        long long c = std::min<long long>(st.max_bond, phys);
        c = std::max<long long>(c, p.chiv[k]);
        p.capb[k] = (int)std::max<long long>(1, c);
    }
    p.capb[0] = p.capb[L] = 1;
    const auto& e = p.e;
    const auto& c = p.capb;
    const auto& Dm = p.Dm;
    const auto& cv = p.chiv;
    p.o_dims = lay.add(sizeof(int) * (L + 2));
    p.o_status = lay.add(sizeof(int));
    p.o_flag = lay.add(sizeof(int));
    p.o_norm2 = lay.add(sizeof(double));
    p.o_fro2 = lay.add(sizeof(double));
    p.o_psi.resize(L);
    p.o_L.resize(L + 1);
    p.o_R.resize(L + 1);
    p.o_XL.resize(L);
    p.o_XR.resize(L);
    size_t max_psi = 0;
    for (int k = 0; k < L; ++k) {
        size_t n = (size_t)c[k] * e[k] * c[k + 1];
        max_psi = std::max(max_psi, n);
        p.o_psi[k] = lay.add(8 * n);
    }
    for (int k = 0; k <= L; ++k) {
        size_t n = (size_t)c[k] * Dm[k] * cv[k];
        p.max_env = std::max(p.max_env, n);
        p.o_L[k] = lay.add(p.es * n);
        p.o_R[k] = lay.add(p.es * n);
    }
    for (int k = 0; k < L; ++k) {
        size_t nxl = (size_t)c[k] * e[k] * Dm[k + 1] * cv[k + 1];
        size_t nxr = (size_t)Dm[k] * cv[k] * e[k] * c[k + 1];
        p.o_XL[k] = lay.add(p.es * nxl);
        p.o_XR[k] = lay.add(p.es * nxr);
        p.max_xr = std::max(p.max_xr, nxr);
        p.max_tmp = std::max(p.max_tmp, (size_t)c[k] * Dm[k] * p.dv[k] * cv[k + 1]);
        p.max_tmp = std::max(p.max_tmp, (size_t)cv[k] * p.dv[k] * c[k + 1] * Dm[k + 1]);
    }
    p.max_theta = max_psi;
    p.max_nvec = 1;
    for (int k = 0; k + 1 < L; ++k) {
        size_t n = (size_t)c[k] * e[k] * e[k + 1] * c[k + 2];
        p.max_theta = std::max(p.max_theta, n);
        p.max_nvec = std::max(p.max_nvec, std::max(c[k] * e[k], e[k + 1] * c[k + 2]));
    }
    for (int k = 0; k < L; ++k) p.max_nvec = std::max(p.max_nvec, c[k]);
    p.o_tmp = lay.add(p.es * p.max_tmp);
    p.o_theta = lay.add(8 * p.max_theta);
    p.o_theta2 = lay.add(8 * p.max_theta);
    // per bond: the singular basis of the last factorization there (warm start)
    p.o_basis.assign(std::max(1, L - 1), 0);
    for (int k = 0; k + 1 < L; ++k) {
        const size_t nb = std::max((size_t)c[k] * e[k], (size_t)e[k + 1] * c[k + 2]);
        p.o_basis[k] = lay.add(8 * nb * nb);
    }
    p.o_Q = lay.add(8 * p.max_theta);
    p.o_carry = lay.add(8 * p.max_theta);
    p.o_tmpB = lay.add(8 * p.max_theta);
    p.o_sigma = lay.add(8 * (size_t)p.max_nvec);
    p.o_perm = lay.add(4 * (size_t)p.max_nvec);
    p.steps = st.max_sweeps * 2 * std::max(0, L - 1);
    p.o_ldelta = lay.add(8 * (size_t)std::max(1, p.steps));
    p.o_lrank = lay.add(4 * (size_t)std::max(1, p.steps));
    p.o_lspec = lay.add(8 * 32 * (size_t)std::max(1, p.steps));
    p.o_lnorm2 = lay.add(8 * (size_t)std::max(1, p.steps));
    p.o_lsweeps = lay.add(4 * (size_t)std::max(1, p.steps));
    if (p.et != T_F64) {
        p.o_R64a = lay.add(8 * p.max_env);
        p.o_R64b = lay.add(8 * p.max_env);
        p.o_XR64 = lay.add(8 * p.max_xr);
        size_t ymax = 0;
        for (int k = 0; k < L; ++k) ymax = std::max(ymax, (size_t)cv[k] * p.dv[k] * c[k + 1] * Dm[k + 1]);
        p.o_Y64 = lay.add(8 * ymax);
    }
}

// Kernels of one problem, enqueued on stream s with the workspace at base.
struct Enq {
    const Plan& p;
    const smps_mpo* U;
    const smps_mps* v;
    const smps_strategy& st;
    char* base;
    hipStream_t s;
    int* dims;
    mutable const char* where = "";
    smps_ctx* ctx = nullptr;

    // exact factorization, timed as category 0 when profiling is on
    hipError_t jac_launch(const JacobiDesc& d, int nvec_cap, int len_cap) const {
        const int tok = ctx ? prof_begin(ctx, s) : -1;
        hipError_t e = launch_jacobi(d, nvec_cap, len_cap, nullptr, at<int>(p.o_flag), s);
        if (ctx) prof_end(ctx, s, tok, 0);
        return e;
    }

    template <typename T = void>
    T* at(size_t off) const { return (T*)(base + off); }
    const double* vsite(int k) const { return v->data + v->off[k]; }
    const double* usite(int k) const { return U->data + U->off[k]; }

    hipError_t gemm(const void* A, int ta_type, const void* B, int tb_type, void* C, int tc_type, DimExpr M,
                    DimExpr N, DimExpr K, int ta, int tb, int tc, int Mcap, int Ncap, int prec) const {
        GemmDesc g{};
        g.A = A;
        g.B = B;
        g.C = C;
        g.dims = dims;
        g.M = M;
        g.N = N;
        g.K = K;
        g.ta = ta;
        g.tb = tb;
        g.tc = tc;
        g.a_type = ta_type;
        g.b_type = tb_type;
        g.c_type = tc_type;
        g.alpha = 1.0;
        return launch_gemm(g, Mcap, Ncap, 1, s, prec);
    }

    // XL[k] = (Lenv[k] A_k) B_k
    hipError_t build_XL(int k) const {
        const auto& c = p.capb;
        hipError_t e = gemm(at(p.o_L[k]), p.et, vsite(k), T_F64, at(p.o_tmp), p.et, ddyn(k, p.Dm[k]),
                            dconst(p.dv[k] * p.chiv[k + 1]), dconst(p.chiv[k]), 0, 0, 0, c[k] * p.Dm[k],
                            p.dv[k] * p.chiv[k + 1], p.prec);
        if (e != hipSuccess) return e;
        LeftMpoDesc d{};
        d.X = at(p.o_tmp);
        d.Y = at(p.o_XL[k]);
        d.B = usite(k);
        d.dims = dims;
        d.a = ddyn(k);
        d.Dl = p.Dm[k];
        d.e = p.e[k];
        d.d = p.dv[k];
        d.Dr = p.Dm[k + 1];
        d.ny = p.chiv[k + 1];
        d.x_type = p.et;
        d.y_type = p.et;
        return launch_left_mpo(d, c[k], s);
    }

    // XR[k] = B_k (A_k Renv[k+1]^T), with Renv given explicitly (type rt)
    hipError_t build_XR(int k, const void* Renv, void* tmp, void* XR, int rt, int prec) const {
        const auto& c = p.capb;
        hipError_t e = gemm(vsite(k), T_F64, Renv, rt, tmp, rt, dconst(p.chiv[k] * p.dv[k]),
                            ddyn(k + 1, p.Dm[k + 1]), dconst(p.chiv[k + 1]), 0, 1, 0, p.chiv[k] * p.dv[k],
                            c[k + 1] * p.Dm[k + 1], prec);
        if (e != hipSuccess) return e;
        RightMpoDesc d{};
        d.X = tmp;
        d.Y = XR;
        d.B = usite(k);
        d.dims = dims;
        d.c = ddyn(k + 1);
        d.Dl = p.Dm[k];
        d.e = p.e[k];
        d.d = p.dv[k];
        d.Dr = p.Dm[k + 1];
        d.nx = p.chiv[k];
        d.x_type = rt;
        d.y_type = rt;
        return launch_right_mpo(d, c[k + 1], s);
    }

    // Renv[k] = psi_k XR[k]^T
    hipError_t env_R(int k, const void* XR, void* R, int rt, int prec) const {
        const auto& c = p.capb;
        return gemm(at(p.o_psi[k]), T_F64, XR, rt, R, rt, ddyn(k), dconst(p.Dm[k] * p.chiv[k]),
                    ddyn(k + 1, p.e[k]), 0, 1, 0, c[k], p.Dm[k] * p.chiv[k], prec);
    }

    JacobiDesc jac(double* X, double* Q, DimExpr nvec, DimExpr len, int rank_idx, int max_rank, double tol,
                   int mode, int step) const {
        JacobiDesc d{};
        d.X = X;
        d.Q = Q;
        d.sigma = at<double>(p.o_sigma);
        d.perm = at<int>(p.o_perm);
        d.dims_in = dims;
        d.dims_out = dims;
        d.nvec = nvec;
        d.len = len;
        d.rank_idx = rank_idx;
        d.max_rank = max_rank;
        d.tol = tol;
        d.mode = mode;
        d.status = at<int>(p.o_status);
        d.fro2 = at<double>(p.o_fro2);
        if (step >= 0) {
            d.log_delta = at<double>(p.o_ldelta) + step;
            d.log_rank = at<int>(p.o_lrank) + step;
            d.log_spec = at<double>(p.o_lspec) + 32 * (size_t)step;
            d.log_norm2 = at<double>(p.o_lnorm2) + step;
            d.log_sweeps = at<int>(p.o_lsweeps) + step;
        }
        return d;
    }

    hipError_t run() const {
        const int L = p.L;
        const auto& c = p.capb;
        const auto& e = p.e;
        hipError_t er;
#define CK(x)                      \
    do {                           \
        er = (x);                  \
        if (er != hipSuccess) {    \
            where = #x;            \
            return er;             \
        }                          \
    } while (0)
        // ---- guess psi = v, bond dims, flags
        std::vector<int> hd(L + 2, 0);
        for (int k = 0; k <= L; ++k) hd[k] = p.chiv[k];
        CK(launch_set_dims(dims, hd.data(), L + 2, s));
        CK(launch_zero_ints(at<int>(p.o_status), 1, s));
        for (int k = 0; k < L; ++k)
            CK(hipMemcpyAsync(at(p.o_psi[k]), vsite(k), 8 * v->site_size(k), hipMemcpyDeviceToDevice, s));
        // ---- right-canonical form (Sec. 2.3): psi_k = V^T, carry psi_k V into site k-1
        const int RS = L + 1;  // scratch slot for a new rank
        for (int k = L - 1; k >= 1; --k) {
            double* theta = at<double>(p.o_theta);
            double* Q = at<double>(p.o_Q);
            const int lenc = e[k] * c[k + 1];
            CK(launch_copy(at<double>(p.o_psi[k]), theta, dims, ddyn(k), ddyn(k + 1, e[k]), c[k] * lenc, s));
            JacobiDesc d = jac(theta, Q, ddyn(k), ddyn(k + 1, e[k]), RS, c[k], 0.0, SMPS_TRUNC_REL_NORM2, -1);
            CK(jac_launch(d, c[k], lenc));
            // carry = psi_k Q^T  (chi_k x r)
            CK(gemm(at(p.o_psi[k]), T_F64, Q, T_F64, at(p.o_carry), T_F64, ddyn(k), ddyn(RS), ddyn(k + 1, e[k]),
                    0, 1, 0, c[k], c[k], P_F64));
            // tmpB = psi_{k-1} carry
            CK(gemm(at(p.o_psi[k - 1]), T_F64, at(p.o_carry), T_F64, at(p.o_tmpB), T_F64, ddyn(k - 1, e[k - 1]),
                    ddyn(RS), ddyn(k), 0, 0, 0, c[k - 1] * e[k - 1], c[k], P_F64));
            CK(launch_copy(Q, at<double>(p.o_psi[k]), dims, ddyn(RS), ddyn(k + 1, e[k]), c[k] * lenc, s));
            CK(launch_copy(at<double>(p.o_tmpB), at<double>(p.o_psi[k - 1]), dims, ddyn(k - 1, e[k - 1]), ddyn(RS),
                           c[k - 1] * e[k - 1] * c[k], s));
            CK(launch_copy_int(dims, RS, k, s));
        }
        // ---- boundary environments and the right environments of the guess
        CK(launch_fill_typed(at(p.o_L[0]), p.et, 1.0, 1, s));
        CK(launch_fill_typed(at(p.o_R[L]), p.et, 1.0, 1, s));
        for (int k = L - 1; k >= 1; --k) {
            CK(build_XR(k, at(p.o_R[k + 1]), at(p.o_tmp), at(p.o_XR[k]), p.et, p.prec));
            CK(env_R(k, at(p.o_XR[k]), at(p.o_R[k]), p.et, p.prec));
        }
        // ---- sweeps (Sec. 2.5)
        int step = 0;
        for (int sw = 0; sw < st.max_sweeps; ++sw) {
            for (int k = 0; k + 1 < L; ++k) {  // left to right
                CK(build_XL(k));
                double* theta = at<double>(p.o_theta);
                CK(gemm(at(p.o_XL[k]), p.et, at(p.o_XR[k + 1]), p.et, theta, T_F64, ddyn(k, e[k]),
                        ddyn(k + 2, e[k + 1]), dconst(p.Dm[k + 1] * p.chiv[k + 1]), 0, 0, 1, c[k] * e[k],
                        e[k + 1] * c[k + 2], p.prec));
                const int mr = std::min(st.max_bond, c[k + 1]);
                // warm start: rotate the columns by the right singular basis this bond
                // produced in the previous right-to-left pass (identity when it was not full)
                double* X = theta;
                if (sw > 0) {
                    X = at<double>(p.o_theta2);
                    CK(gemm(at(p.o_basis[k]), T_F64, theta, T_F64, X, T_F64, ddyn(k + 2, e[k + 1]), ddyn(k, e[k]),
                            ddyn(k + 2, e[k + 1]), 0, 0, 0, e[k + 1] * c[k + 2], c[k] * e[k], P_F64));
                }
                JacobiDesc d = jac(X, at<double>(p.o_Q), ddyn(k + 2, e[k + 1]), ddyn(k, e[k]), k + 1, mr, st.tol,
                                   st.trunc_mode, step);
                d.basis = at<double>(p.o_basis[k]);
                CK(jac_launch(d, e[k + 1] * c[k + 2], c[k] * e[k]));
                // Lenv[k+1] = Q XL[k]
                CK(gemm(at(p.o_Q), T_F64, at(p.o_XL[k]), p.et, at(p.o_L[k + 1]), p.et, ddyn(k + 1), dconst(p.Dm[k + 1] * p.chiv[k + 1]),
                        ddyn(k, e[k]), 0, 0, 0, c[k + 1], p.Dm[k + 1] * p.chiv[k + 1], p.prec));
                ++step;
            }
            for (int k = L - 2; k >= 0; --k) {  // right to left
                CK(build_XR(k + 1, at(p.o_R[k + 2]), at(p.o_tmp), at(p.o_XR[k + 1]), p.et, p.prec));
                double* theta = at<double>(p.o_theta);
                CK(gemm(at(p.o_XL[k]), p.et, at(p.o_XR[k + 1]), p.et, theta, T_F64, ddyn(k, e[k]),
                        ddyn(k + 2, e[k + 1]), dconst(p.Dm[k + 1] * p.chiv[k + 1]), 0, 0, 0, c[k] * e[k],
                        e[k + 1] * c[k + 2], p.prec));
                const int mr = std::min(st.max_bond, c[k + 1]);
                // warm start from the left singular basis of this pass's left-to-right visit
                double* X = at<double>(p.o_theta2);
                CK(gemm(at(p.o_basis[k]), T_F64, theta, T_F64, X, T_F64, ddyn(k, e[k]), ddyn(k + 2, e[k + 1]),
                        ddyn(k, e[k]), 0, 0, 0, c[k] * e[k], e[k + 1] * c[k + 2], P_F64));
                JacobiDesc d = jac(X, at<double>(p.o_psi[k + 1]), ddyn(k, e[k]), ddyn(k + 2, e[k + 1]), k + 1, mr,
                                   st.tol, st.trunc_mode, step);
                d.basis = at<double>(p.o_basis[k]);
                CK(jac_launch(d, c[k] * e[k], e[k + 1] * c[k + 2]));
                CK(env_R(k + 1, at(p.o_XR[k + 1]), at(p.o_R[k + 1]), p.et, p.prec));
                ++step;
            }
        }
        // ---- centre tensor psi_0 = B_0 A_0 Renv[1]: an exact projection on the
        // final right isometries; in the mixed precisions the right
        // environments are rebuilt in FP64 first.
        if (p.et == T_F64) {
            CK(build_XR(0, at(p.o_R[1]), at(p.o_tmp), at(p.o_XR[0]), T_F64, P_F64));
        } else {
            double* Ra = at<double>(p.o_R64a);
            double* Rb = at<double>(p.o_R64b);
            CK(launch_fill(Ra, 1.0, 1, s));
            for (int k = L - 1; k >= 1; --k) {
                CK(build_XR(k, Ra, at(p.o_Y64), at(p.o_XR64), T_F64, P_F64));
                CK(env_R(k, at(p.o_XR64), Rb, T_F64, P_F64));
                std::swap(Ra, Rb);
            }
            CK(build_XR(0, Ra, at(p.o_Y64), at(p.o_XR64), T_F64, P_F64));
        }
        CK(launch_sumsq(centre(), dims, ddyn(1, e[0]), e[0] * c[1], at<double>(p.o_norm2), s));
        CK(launch_check_finite(centre(), dims, ddyn(1, e[0]), e[0] * c[1], at<int>(p.o_status), s));
#undef CK
        return hipSuccess;
    }

    double* centre() const { return p.et == T_F64 ? at<double>(p.o_XR[0]) : at<double>(p.o_XR64); }
};

// Read back the bonds and logs, and build the output handle.
static int finish(smps_ctx* c, const Plan& p, const Enq& q, const smps_strategy& st, smps_mps** out,
                  double* trunc_err) {
    const int L = p.L;
    const int steps = p.steps;
    std::vector<int> hd(L + 2);
    int status = 0;
    double norm2 = 0.0;
    c->log_delta.assign(steps, 0.0);
    c->log_rank.assign(steps, 0);
    c->log_spec.assign((size_t)steps * 32, 0.0);
    c->log_norm2.assign(steps, 0.0);
    c->log_sweeps.assign(steps, 0);
    SMPS_HIP(c, hipMemcpyAsync(hd.data(), q.dims, sizeof(int) * (L + 2), hipMemcpyDeviceToHost, q.s));
    SMPS_HIP(c, hipMemcpyAsync(&status, q.at(p.o_status), sizeof(int), hipMemcpyDeviceToHost, q.s));
    SMPS_HIP(c, hipMemcpyAsync(&norm2, q.at(p.o_norm2), sizeof(double), hipMemcpyDeviceToHost, q.s));
    if (steps > 0) {
        SMPS_HIP(c, hipMemcpyAsync(c->log_delta.data(), q.at(p.o_ldelta), 8 * steps, hipMemcpyDeviceToHost, q.s));
        SMPS_HIP(c, hipMemcpyAsync(c->log_rank.data(), q.at(p.o_lrank), 4 * steps, hipMemcpyDeviceToHost, q.s));
        SMPS_HIP(c, hipMemcpyAsync(c->log_spec.data(), q.at(p.o_lspec), 8 * 32 * (size_t)steps,
                                   hipMemcpyDeviceToHost, q.s));
        SMPS_HIP(c, hipMemcpyAsync(c->log_norm2.data(), q.at(p.o_lnorm2), 8 * steps, hipMemcpyDeviceToHost, q.s));
        SMPS_HIP(c, hipMemcpyAsync(c->log_sweeps.data(), q.at(p.o_lsweeps), 4 * steps, hipMemcpyDeviceToHost, q.s));
    }
    SMPS_HIP(c, hipStreamSynchronize(q.s));
    prof_collect(c);
    if (status) return fail(c, SMPS_ENUMERIC, "non-finite values in a two-site tensor or the result");
    std::vector<int> bonds(hd.begin(), hd.begin() + L + 1);
    bonds[0] = bonds[L] = 1;
    smps_mps* m = new_mps(c, L, p.e, bonds);
    if (!m) return fail(c, SMPS_ENOMEM, "output allocation failed");
    for (int k = 0; k < L; ++k) {
        const double* src = k == 0 ? q.centre() : q.at<double>(p.o_psi[k]);
        SMPS_HIP(c, hipMemcpyAsync(m->data + m->off[k], src, 8 * m->site_size(k), hipMemcpyDeviceToDevice, q.s));
    }
    m->center = 0;
    double eb = 0.0, disc = 0.0;
    for (int i = 0; i < steps; ++i) {
        eb += std::sqrt(std::max(0.0, c->log_delta[i]));
        disc += c->log_delta[i];
    }
    c->info = smps_apply_info{};
    c->info.error_bound = eb;
    c->info.discarded = disc;
    c->info.norm = std::sqrt(norm2);
    c->info.sweeps_done = st.max_sweeps;
    c->info.steps = steps;
    for (int i = 0; i < steps; ++i) c->info.jacobi_sweeps += c->log_sweeps[i];
    if (trunc_err) *trunc_err = eb;
    *out = m;
    return SMPS_OK;
}

int run_apply(smps_ctx* c, const smps_mpo* U, const smps_mps* v, const smps_strategy& st, smps_mps** out,
              double* trunc_err) {
    Plan p;
    Layout lay;
    plan_problem(p, U, v, st, lay);
    int rc = ensure_arena(c, lay.total);
    if (rc != SMPS_OK) return rc;
    Enq q{p, U, v, st, c->arena, c->stream, (int*)(c->arena + p.o_dims)};
    q.ctx = c;
    hipError_t e = q.run();
    if (e != hipSuccess)
        return fail(c, SMPS_EHIP, std::string("enqueue failed at ") + q.where + ": " + hipGetErrorString(e));
    return finish(c, p, q, st, out, trunc_err);
}

int run_apply_batched(smps_ctx* c, int n, const smps_mpo* const* U, const smps_mps* const* v,
                      const smps_strategy& st, smps_mps** out, double* trunc_err) {
    for (int i = 0; i < n; ++i) {
        double te = 0.0;
        int rc = run_apply(c, U[i], v[i], st, &out[i], &te);
        if (rc != SMPS_OK) {
            for (int j = 0; j < i; ++j) {
                smps_mps_destroy(out[j]);
                out[j] = nullptr;
            }
            return rc;
        }
        if (trunc_err) trunc_err[i] = te;
    }
    return SMPS_OK;
}

}  // namespace smps
