// The apply + compression sweep (Sec. 2.3 Eq. simplification, Sec. 2.4.2,
// Sec. 2.5): host-side planning, the operation sequence of one problem, and
// its execution -- launched directly for one problem, or merged across many
// independent problems into batched launches captured in one HIP graph.
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
#include <set>
#include <tuple>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

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
    size_t o_dims, o_status, o_flag, o_done, o_norm2, o_fro2;
    std::vector<size_t> o_psi, o_L, o_R, o_XL, o_XR, o_basis;
    std::vector<size_t> o_accJ;  // per bond: J of the last accumulated factorization there
    size_t o_acctag = 0;         // per bond: validity tag of o_accJ (2 nvec + direction + 1)
    size_t o_tmp, o_theta, o_theta2, o_Q, o_carry, o_tmpB, o_sigma, o_perm;
    size_t o_gtd = 0;  // workspace of the Gram / tridiagonal split (single path only)
    size_t o_ldelta, o_lrank, o_lspec, o_lnorm2, o_lsweeps;
    size_t o_R64a, o_R64b, o_XR64, o_Y64;
    // randomized factorization scratch (allocated only when it is requested)
    int fact = SMPS_FACT_SVD;
    size_t o_rs_G = 0, o_rs_Y = 0, o_rs_P = 0, o_rs_T = 0, o_rs_C = 0, o_rs_W = 0, o_rs_Q = 0;
    size_t o_rs_tot = 0, o_rs_flag = 0, o_rs_feat = 0, o_rs_pred = 0;
    int steps = 0;
    size_t max_theta = 0, max_tmp = 0, max_env = 0, max_xr = 0;
    int max_nvec = 0;
    // linear combinations: the first term lives in the fields above (its state
    // is the guess); every further term has its own operator, state, weight and
    // environment buffers
    double w0 = 1.0;
    struct Term {
        const smps_mpo* U;
        const smps_mps* v;
        double w;
        std::vector<int> dv, Dm, chiv;
        std::vector<size_t> o_L, o_R, o_XL, o_XR;
        size_t o_tmp = 0;
    };
    std::vector<Term> more;
    size_t o_cacc = 0;  // centre accumulation scratch (mixed precision, several terms)
};

void plan_problem(Plan& p, const smps_mpo* U, const smps_mps* v, const smps_strategy& st, Layout& lay) {
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
    // bonds 0..L, a scratch rank slot (L + 1) and two for the randomized path
    p.o_dims = lay.add(sizeof(int) * (L + 4));
    p.o_status = lay.add(sizeof(int));
    p.o_flag = lay.add(sizeof(int));
    p.o_norm2 = lay.add(sizeof(double));
    p.o_fro2 = lay.add(sizeof(double));
    p.o_done = lay.add(sizeof(int));
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
    // accumulated factorizations run on the shorter side and in LDS only
    p.o_accJ.assign(std::max(1, L - 1), 0);
    for (int k = 0; k + 1 < L; ++k) {
        const int lo = std::min(c[k] * e[k], e[k + 1] * c[k + 2]), hi = std::max(c[k] * e[k], e[k + 1] * c[k + 2]);
        if (lo < hi && jacobi_fits_lds(lo, hi, true)) p.o_accJ[k] = lay.add(8 * (size_t)lo * lo);
    }
    p.o_acctag = lay.add(sizeof(int) * std::max(1, L - 1));
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
    p.fact = st.factorization;
    if (p.fact != SMPS_FACT_SVD) {
        // a sketch k < min(nvec, len) keeps every buffer below the two-site size
        for (size_t* o : {&p.o_rs_G, &p.o_rs_Y, &p.o_rs_P, &p.o_rs_T, &p.o_rs_C, &p.o_rs_W, &p.o_rs_Q})
            *o = lay.add(8 * p.max_theta);
        p.o_rs_tot = lay.add(sizeof(double));
        p.o_rs_flag = lay.add(sizeof(int));
        p.o_rs_feat = lay.add(sizeof(float) * 32 * (size_t)std::max(1, L));
        p.o_rs_pred = lay.add(sizeof(float) * (size_t)std::max(1, L));
    }
}


// Buffers of the further terms of a linear combination; the mixed-precision
// FP64 scratch of the first term is grown to the largest term.
void plan_terms(Plan& p, const std::vector<const smps_mpo*>& U, const std::vector<const smps_mps*>& v,
                const std::vector<double>& w, Layout& lay) {
    const int L = p.L;
    const auto& c = p.capb;
    p.w0 = w[0];
    size_t max_env = p.max_env, max_xr = p.max_xr, ymax = 0;
    for (size_t t = 1; t < U.size(); ++t) {
        Plan::Term T;
        T.U = U[t];
        T.v = v[t];
        T.w = w[t];
        T.dv = v[t]->phys;
        T.chiv = v[t]->bonds;
        T.Dm = U[t]->bonds;
        T.o_L.resize(L + 1);
        T.o_R.resize(L + 1);
        T.o_XL.resize(L);
        T.o_XR.resize(L);
        size_t max_tmp = 0;
        for (int k = 0; k <= L; ++k) {
            const size_t n = (size_t)c[k] * T.Dm[k] * T.chiv[k];
            max_env = std::max(max_env, n);
            T.o_L[k] = lay.add(p.es * n);
            T.o_R[k] = lay.add(p.es * n);
        }
        for (int k = 0; k < L; ++k) {
            const size_t nxl = (size_t)c[k] * p.e[k] * T.Dm[k + 1] * T.chiv[k + 1];
            const size_t nxr = (size_t)T.Dm[k] * T.chiv[k] * p.e[k] * c[k + 1];
            T.o_XL[k] = lay.add(p.es * nxl);
            T.o_XR[k] = lay.add(p.es * nxr);
            max_xr = std::max(max_xr, nxr);
            max_tmp = std::max(max_tmp, (size_t)c[k] * T.Dm[k] * T.dv[k] * T.chiv[k + 1]);
            max_tmp = std::max(max_tmp, (size_t)T.chiv[k] * T.dv[k] * c[k + 1] * T.Dm[k + 1]);
            ymax = std::max(ymax, (size_t)T.chiv[k] * T.dv[k] * c[k + 1] * T.Dm[k + 1]);
        }
        T.o_tmp = lay.add(p.es * max_tmp);
        p.more.push_back(std::move(T));
    }
    if (p.et != T_F64 && !p.more.empty()) {
        // FP64 rebuild scratch large enough for every term, and a centre accumulator
        for (int k = 0; k < L; ++k)
            ymax = std::max(ymax, (size_t)p.chiv[k] * p.dv[k] * c[k + 1] * p.Dm[k + 1]);
        p.o_R64a = lay.add(8 * max_env);
        p.o_R64b = lay.add(8 * max_env);
        p.o_XR64 = lay.add(8 * max_xr);
        p.o_Y64 = lay.add(8 * ymax);
        p.o_cacc = lay.add(8 * max_xr);
    }
}

// ---------------------------------------------------------------------------
// Operations.  The sequence of one problem is produced by Enq::run(); every
// operation carries an alignment tag (major phase, step j inside the phase,
// slot inside the step).  Problems of different lengths produce the same slot
// pattern for the same (major, j), so equal tags across problems can share a
// launch.
// ---------------------------------------------------------------------------

enum OpKind { OP_GEMM, OP_LEFT, OP_RIGHT, OP_JAC, OP_COPY, OP_INTCOPY, OP_SETINTS, OP_FILL, OP_NORM };

struct Op {
    OpKind kind;
    int major = 0, j = 0, slot = 0;
    GemmDesc g{};
    LeftMpoDesc l{};
    RightMpoDesc r{};
    JacobiDesc jd{};
    CopyDesc cp{};
    IntCopyDesc ic{};
    NormDesc nd{};
    int cap0 = 0, cap1 = 0, prec = 0;
    int* set_base = nullptr;
    std::vector<int> set_vals;
    void* fill_dst = nullptr;
    int fill_type = 0;
    double fill_val = 0.0;
};

struct Enq {
    const Plan& p;
    const smps_mpo* U;
    const smps_mps* v;
    const smps_strategy& st;
    char* base;
    hipStream_t s;
    int* dims;
    smps_ctx* ctx = nullptr;
    std::vector<Op>* rec = nullptr;  // record instead of launching
    mutable const char* where = "";
    mutable int cur_major = 0, cur_j = 0, cur_slot = 0;
    // phase of the contractions being emitted (kernel timing categories 3-5, -1: none of them)
    mutable int cur_phase = -1;
    // single path only: sweeps and steps actually run (early stop on sweep_tol),
    // the factorization log and the predicted log ranks of the current half-sweep
    mutable int sweeps_done = 0, steps_done = 0;
    mutable std::vector<int> fact_log;
    mutable std::vector<float> preds;
    mutable std::vector<int> prev_rank;
    mutable std::vector<int> hdims;

    template <typename T = void>
    T* at(size_t off) const { return (T*)(base + off); }
    // term t of a linear combination (t = 0: the fields of the plan itself)
    int nterms() const { return 1 + (int)p.more.size(); }
    const smps_mpo* Ut(int t) const { return t ? p.more[t - 1].U : U; }
    const smps_mps* vt(int t) const { return t ? p.more[t - 1].v : v; }
    double wt(int t) const { return t ? p.more[t - 1].w : p.w0; }
    const std::vector<int>& Dm_(int t) const { return t ? p.more[t - 1].Dm : p.Dm; }
    const std::vector<int>& chiv_(int t) const { return t ? p.more[t - 1].chiv : p.chiv; }
    const std::vector<int>& dv_(int t) const { return t ? p.more[t - 1].dv : p.dv; }
    size_t oL(int t, int k) const { return t ? p.more[t - 1].o_L[k] : p.o_L[k]; }
    size_t oR(int t, int k) const { return t ? p.more[t - 1].o_R[k] : p.o_R[k]; }
    size_t oXL(int t, int k) const { return t ? p.more[t - 1].o_XL[k] : p.o_XL[k]; }
    size_t oXR(int t, int k) const { return t ? p.more[t - 1].o_XR[k] : p.o_XR[k]; }
    size_t otmp(int t) const { return t ? p.more[t - 1].o_tmp : p.o_tmp; }
    const double* vsite(int k, int t = 0) const { return vt(t)->data + vt(t)->off[k]; }
    const double* usite(int k, int t = 0) const { return Ut(t)->data + Ut(t)->off[k]; }
    double* centre() const { return p.et == T_F64 ? at<double>(p.o_XR[0]) : at<double>(p.o_XR64); }

    void tag(int major, int j) const {
        cur_major = major;
        cur_j = j;
        cur_slot = 0;
    }

    hipError_t emit(Op&& op) const {
        op.major = cur_major;
        op.j = cur_j;
        op.slot = cur_slot++;
        if (rec) {
            rec->push_back(std::move(op));
            return hipSuccess;
        }
        if (op.kind != OP_JAC && ctx && ctx->profiling) {
            // per-phase timing: contractions (category 1, and 3-5 by phase), the rest (6)
            const bool contraction = op.kind == OP_GEMM || op.kind == OP_LEFT || op.kind == OP_RIGHT;
            const int tok = prof_begin(ctx, s);
            hipError_t e = launch_op(op);
            prof_end(ctx, s, tok, contraction ? 1 : 6, contraction ? cur_phase : -1);
            return e;
        }
        return launch_op(op);
    }

    hipError_t launch_op(const Op& op) const {
        switch (op.kind) {
            case OP_GEMM: return launch_gemm(op.g, op.cap0, op.cap1, 1, s, op.prec);
            case OP_LEFT: return launch_left_mpo(op.l, op.cap0, s);
            case OP_RIGHT: return launch_right_mpo(op.r, op.cap0, s);
            case OP_JAC: {
                const int tok = ctx ? prof_begin(ctx, s) : -1;
                // the blocked path stays host-driven here: measured at 512 and 1024
                // element rows, one launch per round beats a persistent team whose
                // members sit on different XCDs (team barriers cost more than launches)
                hipError_t e = launch_jacobi(op.jd, op.cap0, op.cap1,
                                             gtd_on(op.cap0, op.cap1) ? at<double>(p.o_gtd) : nullptr,
                                             at<int>(p.o_flag), s);
                // category 2 also counts the splits of the largest (bulk) two-site tensor
                if (ctx) prof_end(ctx, s, tok, 0, op.cap0 == p.max_nvec && op.cap1 == p.max_nvec ? 2 : -1);
                return e;
            }
            case OP_COPY: return launch_copy(op.cp.src, op.cp.dst, op.cp.dims, op.cp.a, op.cp.b, op.cap0, s);
            case OP_INTCOPY: return launch_copy_int(op.ic.dims, op.ic.from, op.ic.to, s);
            case OP_SETINTS: return launch_set_dims(op.set_base, op.set_vals.data(), (int)op.set_vals.size(), s);
            case OP_FILL: return launch_fill_typed(op.fill_dst, op.fill_type, op.fill_val, 1, s);
            case OP_NORM: {
                hipError_t e = launch_sumsq(op.nd.x, op.nd.dims, op.nd.n, op.cap0, op.nd.out, s);
                if (e != hipSuccess) return e;
                return launch_check_finite(op.nd.x, op.nd.dims, op.nd.n, op.cap0, op.nd.status, s);
            }
        }
        return hipErrorInvalidValue;
    }

    hipError_t gemm(const void* A, int ta_type, const void* B, int tb_type, void* C, int tc_type, DimExpr M,
                    DimExpr N, DimExpr K, int ta, int tb, int tc, int Mcap, int Ncap, int prec, double alpha = 1.0,
                    double beta = 0.0) const {
        Op op;
        op.kind = OP_GEMM;
        GemmDesc& g = op.g;
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
        g.alpha = alpha;
        g.beta = beta;
        op.cap0 = Mcap;
        op.cap1 = Ncap;
        op.prec = prec;
        return emit(std::move(op));
    }

    // y = a x + b y over m * n doubles: only linear combinations use it, and
    // they run on the single-problem path (no recording)
    hipError_t axpby(double* y, const double* x, double a, double b, DimExpr m, DimExpr n, int cap) const {
        if (rec) return hipErrorNotSupported;
        return launch_axpby(y, x, a, b, dims, m, n, cap, s);
    }

    hipError_t copy(const double* src, double* dst, DimExpr a, DimExpr b, int cap) const {
        Op op;
        op.kind = OP_COPY;
        op.cp = CopyDesc{src, dst, dims, a, b};
        op.cap0 = cap;
        return emit(std::move(op));
    }

    // XL[k] = (Lenv[k] A_k) B_k of term t
    hipError_t build_XL(int k, int t = 0) const {
        const auto& c = p.capb;
        const auto& Dm = Dm_(t);
        const auto& cv = chiv_(t);
        const auto& dv = dv_(t);
        hipError_t e = gemm(at(oL(t, k)), p.et, vsite(k, t), T_F64, at(otmp(t)), p.et, ddyn(k, Dm[k]),
                            dconst(dv[k] * cv[k + 1]), dconst(cv[k]), 0, 0, 0, c[k] * Dm[k], dv[k] * cv[k + 1],
                            p.prec);
        if (e != hipSuccess) return e;
        Op op;
        op.kind = OP_LEFT;
        LeftMpoDesc& d = op.l;
        d.X = at(otmp(t));
        d.Y = at(oXL(t, k));
        d.B = usite(k, t);
        d.dims = dims;
        d.a = ddyn(k);
        d.Dl = Dm[k];
        d.e = p.e[k];
        d.d = dv[k];
        d.Dr = Dm[k + 1];
        d.ny = cv[k + 1];
        d.x_type = p.et;
        d.y_type = p.et;
        op.cap0 = c[k];
        return emit(std::move(op));
    }

    // XR[k] = B_k (A_k Renv[k+1]^T) of term t, with Renv given explicitly (type rt)
    hipError_t build_XR(int k, const void* Renv, void* tmp, void* XR, int rt, int prec, int t = 0) const {
        const auto& c = p.capb;
        const auto& Dm = Dm_(t);
        const auto& cv = chiv_(t);
        const auto& dv = dv_(t);
        hipError_t e = gemm(vsite(k, t), T_F64, Renv, rt, tmp, rt, dconst(cv[k] * dv[k]), ddyn(k + 1, Dm[k + 1]),
                            dconst(cv[k + 1]), 0, 1, 0, cv[k] * dv[k], c[k + 1] * Dm[k + 1], prec);
        if (e != hipSuccess) return e;
        Op op;
        op.kind = OP_RIGHT;
        RightMpoDesc& d = op.r;
        d.X = tmp;
        d.Y = XR;
        d.B = usite(k, t);
        d.dims = dims;
        d.c = ddyn(k + 1);
        d.Dl = Dm[k];
        d.e = p.e[k];
        d.d = dv[k];
        d.Dr = Dm[k + 1];
        d.nx = cv[k];
        d.x_type = rt;
        d.y_type = rt;
        op.cap0 = c[k + 1];
        return emit(std::move(op));
    }

    // Renv[k] = psi_k XR[k]^T of term t
    hipError_t env_R(int k, const void* XR, void* R, int rt, int prec, int t = 0) const {
        const auto& c = p.capb;
        const auto& Dm = Dm_(t);
        const auto& cv = chiv_(t);
        return gemm(at(p.o_psi[k]), T_F64, XR, rt, R, rt, ddyn(k), dconst(Dm[k] * cv[k]), ddyn(k + 1, p.e[k]), 0,
                    1, 0, c[k], Dm[k] * cv[k], prec);
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
        d.conv = at<int>(p.o_flag);
        d.done = at<int>(p.o_done);
        d.floor_eps = 2.220446049250313e-16;
        if (step >= 0) {
            d.log_delta = at<double>(p.o_ldelta) + step;
            d.log_rank = at<int>(p.o_lrank) + step;
            d.log_spec = at<double>(p.o_lspec) + 32 * (size_t)step;
            d.log_norm2 = at<double>(p.o_lnorm2) + step;
            d.log_sweeps = at<int>(p.o_lsweeps) + step;
        }
        return d;
    }

    hipError_t jacobi(const JacobiDesc& d, int nvec_cap, int len_cap) const {
        Op op;
        op.kind = OP_JAC;
        op.jd = d;
        op.cap0 = nvec_cap;
        op.cap1 = len_cap;
        return emit(std::move(op));
    }

    hipError_t read_dims() const {
        hdims.assign(p.L + 4, 0);
        hipError_t e = hipMemcpyAsync(hdims.data(), dims, sizeof(int) * (p.L + 4), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);
    }

    // Predicted rank of every bond for the coming half-sweep (as log r), from
    // the step first + stride * k that last factorized bond k: the rank
    // predictor applied to that step's spectrum, or that step's kept rank.
    hipError_t predict_ranks(int first, int stride) const {
        const int nb = p.L - 1;
        preds.assign(nb, 0.f);
        if (p.fact == SMPS_FACT_RSVD_PREV) {
            std::vector<int> r(nb);
            const int lo = std::min(first, first + stride * (nb - 1));
            hipError_t e = hipMemcpyAsync(r.data(), at<int>(p.o_lrank) + lo, sizeof(int) * nb,
                                          hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) return e;
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) return e;
            prev_rank.assign(nb, 1);
            for (int k = 0; k < nb; ++k) prev_rank[k] = r[first + stride * k - lo];
            return hipSuccess;
        }
        float* feats = at<float>(p.o_rs_feat);
        float* pr = at<float>(p.o_rs_pred);
        hipError_t e = launch_rank_features(at<double>(p.o_lspec), first, stride, nb, feats, s);
        if (e != hipSuccess) return e;
        e = mlp_predict_device(ctx, feats, nb, pr, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(preds.data(), pr, sizeof(float) * nb, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);
    }

    // Sketch size for bond k at a step whose matrix is nv x ln; 0 means the
    // exact SVD (predicted rank at the cap, where the randomized step could
    // not meet the tolerance, or a sketch as large as the matrix).
    int sketch_size(int k, int nv, int ln) const {
        const int lim = std::min(std::min(nv, ln), st.max_bond);
        if (p.fact == SMPS_FACT_RSVD_FIXED) {  // sized by the cap: randomized whenever the cap is below the size
            const int ks = lim + RSVD_OVERSAMPLE;
            return ks < std::min(nv, ln) ? ks : 0;
        }
        int rhat;
        if (p.fact == SMPS_FACT_RSVD_PREV) {
            rhat = std::min(lim, prev_rank[k]);
        } else {
            // a sketch below the rank is refused and redone exactly, one above it
            // only costs its extra columns: the predicted rank is raised by
            // RSVD_PREDICT_MARGIN (measured on tolerance-bound spectra: no
            // fallback left at 1.25, against a quarter of the steps at 1)
            const double lr = std::min(30.0, std::max(0.0, (double)preds[k]));
            rhat = (int)std::min<double>(lim, std::ceil(RSVD_PREDICT_MARGIN * std::exp(lr)));
        }
        rhat = std::max(1, rhat);
        if (rhat >= lim) return 0;
        const int ks = rhat + RSVD_OVERSAMPLE;
        return ks < std::min(nv, ln) ? ks : 0;
    }

    // Randomized factorization of the rows of X (nv x ln, live sizes known on
    // the host) with sketch ks; on acceptance the kept rows go to dest, the
    // rank to dims[bond + 1], the log entries of `step` are written and the
    // warm-start basis of the bond becomes the identity.  *ok reports acceptance.
    hipError_t rsvd(const double* X, int nv, int ln, int ks, int step, int bond, int mr, double* dest,
                    double* basis, bool* ok) const {
        const int KS1 = p.L + 2, KS2 = p.L + 3;
        double* G = at<double>(p.o_rs_G);
        double* Y = at<double>(p.o_rs_Y);
        double* P = at<double>(p.o_rs_P);
        double* T = at<double>(p.o_rs_T);
        double* C = at<double>(p.o_rs_C);
        double* W = at<double>(p.o_rs_W);
        double* Qr = at<double>(p.o_rs_Q);
        double* tot = at<double>(p.o_rs_tot);
        int* flag = at<int>(p.o_rs_flag);
        hipError_t e;
#define RK(x)                   \
    do {                        \
        e = (x);                \
        if (e != hipSuccess) {  \
            where = #x;         \
            return e;           \
        }                       \
    } while (0)
        RK(launch_sumsq(X, dims, dconst(nv * ln), nv * ln, tot, s));
        RK(launch_sketch(G, ks, nv, (unsigned long long)step, s));
        // range finder Y = G X, orthonormalised by two Gram passes: C = Y Y^T = V L V^T
        // (Jacobi in Gram mode), P = L^(-1/2) V^T Y; the second pass on P restores
        // orthonormality lost to the squared condition number of the first
        double* sig = at<double>(p.o_sigma);
        RK(gemm(G, T_F64, X, T_F64, Y, T_F64, dconst(ks), dconst(ln), dconst(nv), 0, 0, 0, ks, ln, P_F64));
        RK(gemm(Y, T_F64, Y, T_F64, C, T_F64, dconst(ks), dconst(ks), dconst(ln), 0, 1, 0, ks, ks, P_F64));
        {
            JacobiDesc g1 = jac(C, W, dconst(ks), dconst(ks), KS1, ks, 0.0, SMPS_TRUNC_REL_NORM2, -1);
            g1.gram = 1;
            RK(jacobi(g1, ks, ks));
        }
        RK(launch_scale_rows(W, sig, dims, ddyn(KS1), dconst(ks), ks * ks, s));
        RK(gemm(W, T_F64, Y, T_F64, P, T_F64, ddyn(KS1), dconst(ln), dconst(ks), 0, 0, 0, ks, ln, P_F64));
        RK(gemm(P, T_F64, P, T_F64, C, T_F64, ddyn(KS1), ddyn(KS1), dconst(ln), 0, 1, 0, ks, ks, P_F64));
        {
            JacobiDesc g2 = jac(C, W, ddyn(KS1), ddyn(KS1), KS2, ks, 0.0, SMPS_TRUNC_REL_NORM2, -1);
            g2.gram = 1;
            RK(jacobi(g2, ks, ks));
        }
        RK(launch_scale_rows(W, sig, dims, ddyn(KS2), ddyn(KS1), ks * ks, s));
        RK(gemm(W, T_F64, P, T_F64, Y, T_F64, ddyn(KS2), dconst(ln), ddyn(KS1), 0, 0, 0, ks, ln, P_F64));
        // Rayleigh-Ritz: B = P X^T (P now in Y); SVD of B through B B^T with the
        // truncation rule and the exact total ||X||_F^2
        RK(gemm(Y, T_F64, X, T_F64, T, T_F64, ddyn(KS2), dconst(nv), dconst(ln), 0, 1, 0, ks, nv, P_F64));
        RK(gemm(T, T_F64, T, T_F64, C, T_F64, ddyn(KS2), ddyn(KS2), dconst(nv), 0, 1, 0, ks, ks, P_F64));
        JacobiDesc d = jac(C, W, ddyn(KS2), ddyn(KS2), bond + 1, mr, st.tol, st.trunc_mode, step);
        d.gram = 1;
        d.total_ext = tot;
        RK(jacobi(d, ks, ks));
        RK(gemm(W, T_F64, Y, T_F64, Qr, T_F64, ddyn(bond + 1), dconst(ln), ddyn(KS2), 0, 0, 0, ks, ln, P_F64));
        RK(launch_rsvd_accept(dims, bond + 1, at<double>(p.o_ldelta) + step, tot, sig, ks, RSVD_OVERSAMPLE, st.tol,
                              st.trunc_mode, at<int>(p.o_status), flag, s));
        int h = 0;
        RK(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        RK(hipStreamSynchronize(s));
        *ok = h != 0;
        if (*ok) {
            RK(copy(Qr, dest, ddyn(bond + 1), dconst(ln), ks * ln));
            RK(launch_identity(basis, dims, dconst(ln), ln, s));
        }
#undef RK
        return hipSuccess;
    }

    // Factorization of one sweep step.  theta holds the rows to orthogonalise
    // (nvec x len); rotate: pre-rotate by the bond's stored basis (warm start);
    // randomized: this bond was factorized before in this call and a
    // randomized method is requested.
    hipError_t factor(int k, int step, bool rotate, bool randomized, double* theta, DimExpr nvec, DimExpr len,
                      int nvec_cap, int len_cap, double* dest, int mr, bool acc = false, int dir = 0) const {
        if (randomized && !rec) {
            hipError_t e = read_dims();
            if (e != hipSuccess) return e;
            const int nv = eval_host(nvec), ln = eval_host(len);
            const int ks = sketch_size(k, nv, ln);
            if (ks > 0) {
                bool ok = false;
                e = rsvd(theta, nv, ln, ks, step, k, mr, dest, at<double>(p.o_basis[k]), &ok);
                if (e != hipSuccess) return e;
                fact_log[step] = ok ? ks : -ks;
                if (ok) return hipSuccess;
            }
        }
        double* X = theta;
        // an accumulated step pre-rotates by the J its last visit in the same
        // direction left (the kernel falls back to theta when that J's tag does
        // not match); any other step by the bond's basis
        const bool acc_warm = acc && p.o_accJ[k] != 0;
        if (rotate && gtd_on(nvec_cap, len_cap)) rotate = false;  // H = X^T X does not depend on it
        if (rotate) {
            X = at<double>(p.o_theta2);
            hipError_t e = gemm(at(acc_warm ? p.o_accJ[k] : p.o_basis[k]), T_F64, theta, T_F64, X, T_F64, nvec, len,
                                nvec, 0, 0, 0, nvec_cap, len_cap, P_F64);
            if (e != hipSuccess) return e;
        } else {
            ++cur_slot;  // the same slot numbering whether or not this step pre-rotates
        }
        JacobiDesc d = jac(X, dest, nvec, len, k + 1, mr, st.tol, st.trunc_mode, step);
        d.basis = at<double>(p.o_basis[k]);
        d.accumulate = acc;
        if (acc_warm) {
            d.X_raw = theta;
            d.acc_basis = at<double>(p.o_accJ[k]);
            d.acc_tag = at<int>(p.o_acctag) + k;
            d.acc_dir = dir;
        }
        return jacobi(d, nvec_cap, len_cap);
    }

    // One-sided Jacobi converges slowly on more vectors than their length (the
    // surplus must be rotated to zero) and such a step leaves no full basis to
    // warm-start from.  When the side a step needs is the longer one, the
    // vectors are taken along the shorter side instead and the rotations are
    // accumulated (the needed singular vectors are rows of the accumulated
    // matrix); exact factorizations in the LDS kernel only.
    bool use_acc(int need_side, int other_side) const {
        return st.factorization == SMPS_FACT_SVD && need_side < other_side &&
               jacobi_fits_lds(need_side, other_side, true) && !gtd_on(other_side, need_side);
    }

    int eval_host(DimExpr x) const { return x.idx < 0 ? x.mul : x.mul * hdims[x.idx]; }

    // The exact split of nvec_cap vectors of len_cap elements goes through the
    // Gram matrix and a tridiagonal eigensolver (single path, short vectors);
    // it needs neither a warm start nor the accumulated orientation.
    bool gtd_on(int nvec_cap, int len_cap) const {
        // the automatic choice keeps the one-sided Jacobi split: measured on one
        // CU the Gram split is no faster at 128 x 128 and slower below
        return !rec && ctx && ctx->split_method == SMPS_SPLIT_GRAM && p.o_gtd && gtd_supported(nvec_cap, len_cap);
    }

    hipError_t run() const {
        const int L = p.L;
        const auto& c = p.capb;
        const auto& e = p.e;
        const int S = st.max_sweeps;
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
        tag(0, 0);
        {
            Op op;
            op.kind = OP_SETINTS;
            op.set_base = dims;
            op.set_vals.assign(L + 4, 0);
            for (int k = 0; k <= L; ++k) op.set_vals[k] = p.chiv[k];
            CK(emit(std::move(op)));
        }
        {
            Op op;
            op.kind = OP_SETINTS;
            op.set_base = at<int>(p.o_status);
            op.set_vals.assign(1, 0);
            CK(emit(std::move(op)));
        }
        {  // no accumulated factorization has left a J yet
            Op op;
            op.kind = OP_SETINTS;
            op.set_base = at<int>(p.o_acctag);
            op.set_vals.assign(std::max(1, L - 1), 0);
            CK(emit(std::move(op)));
        }
        const int NT = nterms();
        for (int t = 0; t < NT; ++t) {
            Op a;
            a.kind = OP_FILL;
            a.fill_dst = at(oL(t, 0));
            a.fill_type = p.et;
            a.fill_val = 1.0;
            CK(emit(std::move(a)));
            Op b;
            b.kind = OP_FILL;
            b.fill_dst = at(oR(t, L));
            b.fill_type = p.et;
            b.fill_val = 1.0;
            CK(emit(std::move(b)));
        }
        for (int k = 0; k < L; ++k) {
            tag(0, 1 + k);
            const int n = (int)v->site_size(k);
            CK(copy(vsite(k), at<double>(p.o_psi[k]), dconst(n), dconst(1), n));
        }
        // ---- right-canonical form (Sec. 2.3): psi_k = V^T, carry psi_k V into site k-1
        const int RS = L + 1;  // scratch slot for a new rank
        for (int k = L - 1; k >= 1; --k) {
            tag(1, L - 1 - k);
            double* theta = at<double>(p.o_theta);
            double* Q = at<double>(p.o_Q);
            const int lenc = e[k] * c[k + 1];
            CK(copy(at<double>(p.o_psi[k]), theta, ddyn(k), ddyn(k + 1, e[k]), c[k] * lenc));
            JacobiDesc d = jac(theta, Q, ddyn(k), ddyn(k + 1, e[k]), RS, c[k], 0.0, SMPS_TRUNC_REL_NORM2, -1);
            CK(jacobi(d, c[k], lenc));
            // carry = psi_k Q^T  (chi_k x r)
            CK(gemm(at(p.o_psi[k]), T_F64, Q, T_F64, at(p.o_carry), T_F64, ddyn(k), ddyn(RS), ddyn(k + 1, e[k]),
                    0, 1, 0, c[k], c[k], P_F64));
            // tmpB = psi_{k-1} carry
            CK(gemm(at(p.o_psi[k - 1]), T_F64, at(p.o_carry), T_F64, at(p.o_tmpB), T_F64, ddyn(k - 1, e[k - 1]),
                    ddyn(RS), ddyn(k), 0, 0, 0, c[k - 1] * e[k - 1], c[k], P_F64));
            CK(copy(Q, at<double>(p.o_psi[k]), ddyn(RS), ddyn(k + 1, e[k]), c[k] * lenc));
            CK(copy(at<double>(p.o_tmpB), at<double>(p.o_psi[k - 1]), ddyn(k - 1, e[k - 1]), ddyn(RS),
                    c[k - 1] * e[k - 1] * c[k]));
            Op ic;
            ic.kind = OP_INTCOPY;
            ic.ic = IntCopyDesc{dims, RS, k};
            CK(emit(std::move(ic)));
        }
        // ---- right environments of the guess
        for (int k = L - 1; k >= 1; --k) {
            tag(2, L - 1 - k);
            for (int t = 0; t < NT; ++t) {
                CK(build_XR(k, at(oR(t, k + 1)), at(otmp(t)), at(oXR(t, k)), p.et, p.prec, t));
                CK(env_R(k, at(oXR(t, k)), at(oR(t, k)), p.et, p.prec, t));
            }
        }
        // ---- sweeps (Sec. 2.5)
        int step = 0;
        const bool rs = p.fact != SMPS_FACT_SVD;
        const bool predicts = rs && p.fact != SMPS_FACT_RSVD_FIXED;  // sizing needs a rank estimate
        if (!rec) fact_log.assign(std::max(1, p.steps), 0);
        sweeps_done = 0;
        for (int sw = 0; sw < S; ++sw) {
            // bond k was last factorized in the previous half-sweep, at step
            // (2 sw - 1)(L - 1) + (L - 2 - k)
            const bool rs_lr = rs && sw > 0;
            if (rs_lr && predicts && !rec) CK(predict_ranks((2 * sw - 1) * (L - 1) + (L - 2), -1));
            for (int k = 0; k + 1 < L; ++k) {  // left to right
                tag(3 + 2 * sw, k);
                double* theta = at<double>(p.o_theta);
                // the left singular vectors are needed: rows of theta^T, or (acc) the
                // accumulated rotations of theta's rows when those are the shorter side
                const bool acc = use_acc(c[k] * e[k], e[k + 1] * c[k + 2]);
                // theta = sum_t w_t XL_t[k] XR_t[k+1] (one term: the plain product)
                for (int t = 0; t < NT; ++t) {
                    cur_phase = 3;
                    CK(build_XL(k, t));
                    const int K = Dm_(t)[k + 1] * chiv_(t)[k + 1];
                    cur_phase = 4;
                    CK(gemm(at(oXL(t, k)), p.et, at(oXR(t, k + 1)), p.et, theta, T_F64, ddyn(k, e[k]),
                            ddyn(k + 2, e[k + 1]), dconst(K), 0, 0, acc ? 0 : 1, c[k] * e[k], e[k + 1] * c[k + 2],
                            p.prec, wt(t), t ? 1.0 : 0.0));
                }
                const int mr = std::min(st.max_bond, c[k + 1]);
                cur_phase = -1;  // the split and its warm-start rotation
                // warm start (sw > 0): rotate by the right singular basis this bond
                // produced in the previous right-to-left pass (identity when it was not full)
                if (acc)
                    CK(factor(k, step, sw > 0, rs_lr, theta, ddyn(k, e[k]), ddyn(k + 2, e[k + 1]), c[k] * e[k],
                              e[k + 1] * c[k + 2], at<double>(p.o_Q), mr, true, 0));
                else
                    CK(factor(k, step, sw > 0, rs_lr, theta, ddyn(k + 2, e[k + 1]), ddyn(k, e[k]),
                              e[k + 1] * c[k + 2], c[k] * e[k], at<double>(p.o_Q), mr));
                // Lenv_t[k+1] = Q XL_t[k]
                cur_phase = 5;
                for (int t = 0; t < NT; ++t) {
                    const int K = Dm_(t)[k + 1] * chiv_(t)[k + 1];
                    CK(gemm(at(p.o_Q), T_F64, at(oXL(t, k)), p.et, at(oL(t, k + 1)), p.et, ddyn(k + 1), dconst(K),
                            ddyn(k, e[k]), 0, 0, 0, c[k + 1], K, p.prec));
                }
                cur_phase = -1;
                ++step;
            }
            // bond k was last factorized in this sweep's left-to-right pass, at step 2 sw (L - 1) + k
            if (predicts && !rec) CK(predict_ranks(2 * sw * (L - 1), 1));
            for (int k = L - 2; k >= 0; --k) {  // right to left
                tag(4 + 2 * sw, L - 2 - k);
                double* theta = at<double>(p.o_theta);
                // the right singular vectors are needed: rows of theta, or (acc) the
                // accumulated rotations of theta^T's rows when those are the shorter side
                const bool acc = use_acc(e[k + 1] * c[k + 2], c[k] * e[k]);
                for (int t = 0; t < NT; ++t) {
                    cur_phase = 3;
                    CK(build_XR(k + 1, at(oR(t, k + 2)), at(otmp(t)), at(oXR(t, k + 1)), p.et, p.prec, t));
                    const int K = Dm_(t)[k + 1] * chiv_(t)[k + 1];
                    cur_phase = 4;
                    CK(gemm(at(oXL(t, k)), p.et, at(oXR(t, k + 1)), p.et, theta, T_F64, ddyn(k, e[k]),
                            ddyn(k + 2, e[k + 1]), dconst(K), 0, 0, acc ? 1 : 0, c[k] * e[k], e[k + 1] * c[k + 2],
                            p.prec, wt(t), t ? 1.0 : 0.0));
                }
                const int mr = std::min(st.max_bond, c[k + 1]);
                cur_phase = -1;
                // warm start from the left singular basis of this pass's left-to-right visit
                if (acc)
                    CK(factor(k, step, sw > 0, rs, theta, ddyn(k + 2, e[k + 1]), ddyn(k, e[k]), e[k + 1] * c[k + 2],
                              c[k] * e[k], at<double>(p.o_psi[k + 1]), mr, true, 1));
                else
                    CK(factor(k, step, true, rs, theta, ddyn(k, e[k]), ddyn(k + 2, e[k + 1]), c[k] * e[k],
                              e[k + 1] * c[k + 2], at<double>(p.o_psi[k + 1]), mr));
                cur_phase = 5;
                for (int t = 0; t < NT; ++t)
                    CK(env_R(k + 1, at(oXR(t, k + 1)), at(oR(t, k + 1)), p.et, p.prec, t));
                cur_phase = -1;
                ++step;
            }
            sweeps_done = sw + 1;
            steps_done = step;
            // early stop (single path): relative change of ||psi||^2 over the sweep
            if (!rec && st.sweep_tol > 0.0 && sw > 0 && L > 1) {
                double nn[2] = {0.0, 0.0};
                const int last = step - 1, prev = step - 1 - 2 * (L - 1);
                CK(hipMemcpyAsync(&nn[0], at<double>(p.o_lnorm2) + last, sizeof(double), hipMemcpyDeviceToHost, s));
                CK(hipMemcpyAsync(&nn[1], at<double>(p.o_lnorm2) + prev, sizeof(double), hipMemcpyDeviceToHost, s));
                CK(hipStreamSynchronize(s));
                if (std::fabs(nn[0] - nn[1]) <= st.sweep_tol * std::fabs(nn[0])) break;
            }
        }
        // ---- centre tensor psi_0 = B_0 A_0 Renv[1]: an exact projection on the
        // final right isometries; in the mixed precisions the right
        // environments are rebuilt in FP64 first.
        // A linear combination sums the terms' projections: psi_0 = sum_t w_t B_0 A_0 Renv_t[1].
        const bool weighted = NT > 1 || p.w0 != 1.0;
        const DimExpr cm = dconst(e[0]), cn = ddyn(1);
        if (p.et == T_F64) {
            tag(4 + 2 * S, 0);
            for (int t = 0; t < NT; ++t) {
                CK(build_XR(0, at(oR(t, 1)), at(otmp(t)), at(oXR(t, 0)), T_F64, P_F64, t));
                if (t == 0 && weighted) CK(axpby(centre(), centre(), 0.0, p.w0, cm, cn, e[0] * c[1]));
                if (t > 0) CK(axpby(centre(), at<double>(oXR(t, 0)), wt(t), 1.0, cm, cn, e[0] * c[1]));
            }
        } else {
            for (int t = 0; t < NT; ++t) {
                double* Ra = at<double>(p.o_R64a);
                double* Rb = at<double>(p.o_R64b);
                tag(3 + 2 * S, 0);
                Op f;
                f.kind = OP_FILL;
                f.fill_dst = Ra;
                f.fill_type = T_F64;
                f.fill_val = 1.0;
                CK(emit(std::move(f)));
                // term 0 leaves its projection in XR64 (the centre); later terms work in cacc
                void* xr = at(t == 0 ? p.o_XR64 : p.o_cacc);
                for (int k = L - 1; k >= 1; --k) {
                    tag(3 + 2 * S, 1 + (L - 1 - k));
                    CK(build_XR(k, Ra, at(p.o_Y64), xr, T_F64, P_F64, t));
                    CK(env_R(k, xr, Rb, T_F64, P_F64, t));
                    std::swap(Ra, Rb);
                }
                tag(4 + 2 * S, 0);
                if (t == 0) {
                    CK(build_XR(0, Ra, at(p.o_Y64), at(p.o_XR64), T_F64, P_F64, t));
                    if (weighted) CK(axpby(centre(), centre(), 0.0, p.w0, cm, cn, e[0] * c[1]));
                } else {
                    CK(build_XR(0, Ra, at(p.o_Y64), at(p.o_cacc), T_F64, P_F64, t));
                    CK(axpby(centre(), at<double>(p.o_cacc), wt(t), 1.0, cm, cn, e[0] * c[1]));
                }
            }
        }
        tag(5 + 2 * S, 0);
        {
            Op op;
            op.kind = OP_NORM;
            op.nd = NormDesc{centre(), dims, ddyn(1, e[0]), at<double>(p.o_norm2), at<int>(p.o_status)};
            op.cap0 = e[0] * c[1];
            CK(emit(std::move(op)));
        }
#undef CK
        return hipSuccess;
    }
};

static const char* status_message(int status) {
    if (status & 1) return "non-finite values in a two-site tensor or the result";
    if (status & 4) return "a persistent blocked factorization gave up waiting for its team (barrier time-out)";
    return "a blocked factorization did not converge within its sweep budget";
}

// Read back the bonds and logs, and build the output handle.
static int finish(smps_ctx* c, const Plan& p, const Enq& q, const smps_strategy& st, smps_mps** out,
                  double* trunc_err) {
    const int L = p.L;
    const int steps = q.steps_done;
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
    if (status) return fail(c, SMPS_ENUMERIC, status_message(status));
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
    c->info.sweeps_done = q.sweeps_done;
    c->info.steps = steps;
    c->log_fact.assign(q.fact_log.begin(), q.fact_log.begin() + std::min<size_t>(steps, q.fact_log.size()));
    c->log_L = L;
    for (int f : c->log_fact) {
        c->info.rsvd_accepted += f > 0;
        c->info.rsvd_fallbacks += f < 0;
    }
    for (int i = 0; i < steps; ++i) c->info.jacobi_sweeps += c->log_sweeps[i];
    if (trunc_err) *trunc_err = eb;
    *out = m;
    return SMPS_OK;
}

// One chain, one or several (weight, operator, state) terms; the first term's
// state is the guess.
// Plan of one chain (every term) with the workspace of the context's split.
static int plan_single(smps_ctx* c, int n, const double* w, const smps_mpo* const* U, const smps_mps* const* v,
                       const smps_strategy& st, Plan& p, Layout& lay) {
    plan_problem(p, U[0], v[0], st, lay);
    if (p.max_nvec > 2048)
        return fail(c, SMPS_EUNSUPPORTED, "two-site tensors with more than 2048 rows or columns are not supported");
    if (n > 1 || w[0] != 1.0)
        plan_terms(p, std::vector<const smps_mpo*>(U, U + n), std::vector<const smps_mps*>(v, v + n),
                   std::vector<double>(w, w + n), lay);
    if (c->split_method == SMPS_SPLIT_GRAM) {
        const int nc = std::min(p.max_nvec, 1024), lc = std::min(p.max_nvec, 128);
        if (gtd_supported(nc, lc)) p.o_gtd = lay.add(8 * gtd_work_doubles(nc, lc));
    }
    return SMPS_OK;
}

static int run_terms(smps_ctx* c, int n, const double* w, const smps_mpo* const* U, const smps_mps* const* v,
                     const smps_strategy& st, smps_mps** out, double* trunc_err) {
    Plan p;
    Layout lay;
    int rc = plan_single(c, n, w, U, v, st, p, lay);
    if (rc != SMPS_OK) return rc;
    rc = ensure_arena(c, lay.total);
    if (rc != SMPS_OK) return rc;
    if (st.factorization == SMPS_FACT_RSVD_MLP && !mlp_ready(c))
        return fail(c, SMPS_EINVAL, "the randomized factorization sized by the rank predictor needs "
                                    "smps_rank_mlp_init, _set or _train first");
    Enq q{p, U[0], v[0], st, c->arena, c->stream, (int*)(c->arena + p.o_dims)};
    q.ctx = c;
    hipError_t e = q.run();
    if (e != hipSuccess)
        return fail(c, SMPS_EHIP, std::string("enqueue failed at ") + q.where + ": " + hipGetErrorString(e));
    return finish(c, p, q, st, out, trunc_err);
}

int run_apply(smps_ctx* c, const smps_mpo* U, const smps_mps* v, const smps_strategy& st, smps_mps** out,
              double* trunc_err) {
    const double one = 1.0;
    return run_terms(c, 1, &one, &U, &v, st, out, trunc_err);
}

int run_combine(smps_ctx* c, int n, const double* w, const smps_mpo* const* U, const smps_mps* const* v,
                const smps_strategy& st, smps_mps** out, double* trunc_err) {
    return run_terms(c, n, w, U, v, st, out, trunc_err);
}

// Autotune every product shape one apply + compression would launch: the
// sequence is recorded (nothing runs), each GEMM's extents are evaluated at
// the allocation caps, and each distinct table key is timed once.
int run_autotune(smps_ctx* c, const smps_mpo* U, const smps_mps* v, const smps_strategy& st, int reps,
                 int* tuned) {
    Plan p;
    Layout lay;
    plan_problem(p, U, v, st, lay);
    std::vector<Op> ops;
    Enq q{p, U, v, st, nullptr, c->stream, nullptr};
    q.rec = &ops;
    hipError_t e = q.run();
    if (e != hipSuccess) return fail(c, SMPS_EHIP, std::string("autotune: recording failed at ") + q.where);
    const int L = p.L;
    const int cap_max = *std::max_element(p.capb.begin(), p.capb.end());
    auto cap_of = [&](DimExpr x) { return x.idx < 0 ? x.mul : x.mul * (x.idx <= L ? p.capb[x.idx] : cap_max); };
    std::set<std::tuple<int, int, int, int, int, int, int, int, int>> seen;
    int n = 0;
    for (const Op& op : ops) {
        if (op.kind != OP_GEMM) continue;
        const GemmDesc& g = op.g;
        const int M = op.cap0, N = op.cap1, K = cap_of(g.K);
        if (M < 1 || N < 1 || K < 1) continue;
        int bm = 1, bn = 1;
        while (bm < M) bm <<= 1;
        while (bn < N) bn <<= 1;
        if (!seen.insert({op.prec, g.a_type, g.b_type, g.c_type, g.ta, g.tb, g.tc, bm, bn}).second) continue;
        int best = 0;
        const int rc = tune_gemm_shape(c, op.prec, g.a_type, g.b_type, g.c_type, g.ta, g.tb, g.tc, M, N, K, reps, &best);
        if (rc != SMPS_OK) return rc;
        ++n;
    }
    if (tuned) *tuned = n;
    return SMPS_OK;
}

// ---------------------------------------------------------------------------
// Batched execution
// ---------------------------------------------------------------------------

// Kernel nodes one batched graph may hold.  Every operation of a step is a
// bounded number of kernels (the blocked factorization runs all its sweeps in
// one persistent launch), so a graph grows with the steps of its longest
// chain: a batch holding an L = 100 chain with 4 sweeps needs about 2e4.  The
// bound keeps host memory and instantiation time of one capture in check.
constexpr long long MAX_GRAPH_KERNELS = 100000;

struct IntSetDesc {
    int* dst;
    int val;
};
struct FillDesc {
    void* dst;
    int type;
    double val;
};
struct GatherDesc {
    const int* dims;
    int L;
    const int* status;
    const double* norm2;
    const double* ldelta;
    int steps;
    double* out;  // [error bound, discarded, norm2, status, dims[0..L]]
};

__global__ void set_ints_batched_kernel(const IntSetDesc* arr, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        *arr[i].dst = arr[i].val;
}

__global__ void fill_batched_kernel(const FillDesc* arr, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        if (arr[i].type == T_F64)
            *(double*)arr[i].dst = arr[i].val;
        else
            *(float*)arr[i].dst = (float)arr[i].val;
    }
}

// Per problem: the accumulated bound sum_i sqrt(delta_i), sum_i delta_i, the
// centre norm, the status word and the bond dimensions, gathered in one place.
__global__ void gather_batched_kernel(const GatherDesc* arr, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const GatherDesc g = arr[i];
        double eb = 0.0, disc = 0.0;
        for (int s = 0; s < g.steps; ++s) {
            const double dl = g.ldelta[s] > 0.0 ? g.ldelta[s] : 0.0;
            eb += sqrt(dl);
            disc += dl;
        }
        g.out[0] = eb;
        g.out[1] = disc;
        g.out[2] = *g.norm2;
        g.out[3] = (double)*g.status;
        for (int k = 0; k <= g.L; ++k) g.out[4 + k] = (double)g.dims[k];
    }
}

// Host staging of descriptor arrays: every batched launch reads its
// descriptors from one device buffer uploaded before the launches.
struct DescArena {
    std::vector<char> host;
    size_t add(const void* p, size_t bytes) {
        size_t o = (host.size() + 63) / 64 * 64;
        host.resize(o + bytes);
        std::memcpy(host.data() + o, p, bytes);
        return o;
    }
};

struct Launch {
    OpKind kind;
    size_t off = 0;  // descriptor array offset in the device arena
    int count = 0;
    int cap0 = 0, cap1 = 0, cap2 = 0, prec = 0, E = 0;
    size_t shm = 0;
    GemmDesc gtypes{};
    LeftMpoDesc ltypes{};
    RightMpoDesc rtypes{};
    bool panel = false;
    bool acc = false;  // LDS Jacobi launch: rotations accumulated
    int max_pairs = 0, max_nblk = 0, max_rows = 0;
    size_t queue_off = 0;  // persistent blocked launch: its queue state in the arena
};

struct BatchCache {
    std::vector<const void*> key;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    char* desc_dev = nullptr;
    size_t desc_bytes = 0;
    size_t results_off = 0;
    std::vector<Plan> plans;
};

// What must agree for ops to share one launch: the kind, and the template
// arguments their launch is compiled for (types, transposes, precision).
static std::vector<int> launch_signature(const Op& op) {
    switch (op.kind) {
        case OP_GEMM:
            return {op.kind, op.g.ta, op.g.tb, op.g.tc, op.g.a_type, op.g.b_type, op.g.c_type, op.prec};
        case OP_LEFT: return {op.kind, op.l.x_type, op.l.y_type};
        case OP_RIGHT: return {op.kind, op.r.x_type, op.r.y_type};
        default: return {op.kind};
    }
}

static void build_launches(const std::vector<std::vector<Op>>& ops, DescArena& da, std::vector<Launch>& out) {
    // the persistent blocked launches run one after another: they share one queue state
    size_t queue_off = SIZE_MAX;
    // group equal tags (phase, step, slot) across problems, in sequence order;
    // within a tag, problems whose ops differ in kind or template arguments (a
    // step can be shaped differently in chains of different lengths) get
    // launches of their own -- problems are independent, so their order does
    // not matter
    std::map<std::tuple<int, int, int>, std::map<std::vector<int>, std::vector<const Op*>>> tags;
    for (const auto& seq : ops)
        for (const Op& op : seq) tags[std::make_tuple(op.major, op.j, op.slot)][launch_signature(op)].push_back(&op);
    std::vector<const std::vector<const Op*>*> groups;
    for (auto& t : tags)
        for (auto& sg : t.second) groups.push_back(&sg.second);
    for (const auto* gp : groups) {
        const auto& g = *gp;
        const OpKind kind = g[0]->kind;
        Launch ln;
        ln.kind = kind;
        ln.count = (int)g.size();
        switch (kind) {
            case OP_GEMM: {
                std::vector<GemmDesc> d;
                for (const Op* o : g) {
                    d.push_back(o->g);
                    ln.cap0 = std::max(ln.cap0, o->cap0);
                    ln.cap1 = std::max(ln.cap1, o->cap1);
                }
                ln.gtypes = g[0]->g;
                ln.prec = g[0]->prec;
                ln.off = da.add(d.data(), sizeof(GemmDesc) * d.size());
                out.push_back(ln);
                break;
            }
            case OP_LEFT: {
                std::vector<LeftMpoDesc> d;
                for (const Op* o : g) {
                    d.push_back(o->l);
                    ln.cap0 = std::max(ln.cap0, o->cap0);
                    ln.cap1 = std::max(ln.cap1, o->l.ny);
                    ln.cap2 = std::max(ln.cap2, o->l.Dl * o->l.e * o->l.d * o->l.Dr);
                }
                ln.ltypes = g[0]->l;
                ln.off = da.add(d.data(), sizeof(LeftMpoDesc) * d.size());
                out.push_back(ln);
                break;
            }
            case OP_RIGHT: {
                std::vector<RightMpoDesc> d;
                for (const Op* o : g) {
                    d.push_back(o->r);
                    ln.cap0 = std::max(ln.cap0, o->cap0);
                    ln.cap1 = std::max(ln.cap1, o->r.nx);
                    ln.cap2 = std::max(ln.cap2, o->r.Dl * o->r.e * o->r.d * o->r.Dr);
                }
                ln.rtypes = g[0]->r;
                ln.off = da.add(d.data(), sizeof(RightMpoDesc) * d.size());
                out.push_back(ln);
                break;
            }
            case OP_JAC: {
                // LDS-resident factorizations grouped by register class; the rest blocked
                std::map<int, std::vector<JacobiDesc>> lds;
                std::map<int, size_t> lds_shm;
                std::vector<const Op*> blocked;
                Launch pl;
                pl.kind = OP_JAC;
                pl.panel = true;
                for (const Op* o : g) {
                    const bool acc = o->jd.accumulate != 0;
                    if (jacobi_fits_lds(o->cap0, o->cap1, acc)) {
                        // class key: register class E and whether rotations are accumulated
                        const int key = 2 * jacobi_lds_class(o->cap1) + (acc ? 1 : 0);
                        lds[key].push_back(o->jd);
                        lds_shm[key] = std::max(lds_shm[key], jacobi_lds_bytes(o->cap0, o->cap1, acc));
                    } else {
                        blocked.push_back(o);
                        pl.cap1 = std::max(pl.cap1, o->cap1);
                    }
                }
                // the blocked launch's row layout follows its longest rows: every
                // factorization in it takes that shape's block size.  The array is
                // the persistent launch's queue: largest (nvec^2 len) first
                std::stable_sort(blocked.begin(), blocked.end(), [](const Op* a, const Op* b) {
                    return (double)a->cap0 * a->cap0 * a->cap1 > (double)b->cap0 * b->cap0 * b->cap1;
                });
                std::vector<JacobiDesc> panel;
                for (const Op* o : blocked) {
                    JacobiDesc d = o->jd;
                    jacobi_panel_params(o->cap0, pl.cap1, &d.bs, &d.nblk);
                    panel.push_back(d);
                    pl.max_pairs = std::max(pl.max_pairs, d.nblk / 2);
                    pl.max_nblk = std::max(pl.max_nblk, d.nblk);
                    pl.max_rows = std::max(pl.max_rows, d.basis ? std::max(o->cap0, o->cap1) : o->cap0);
                    pl.shm = std::max(pl.shm, jacobi_panel_bytes(pl.cap1, d.bs));
                }
                for (auto& cls : lds) {
                    Launch l2;
                    l2.kind = OP_JAC;
                    l2.E = cls.first / 2;
                    l2.acc = (cls.first & 1) != 0;
                    l2.shm = lds_shm[cls.first];
                    l2.count = (int)cls.second.size();
                    l2.off = da.add(cls.second.data(), sizeof(JacobiDesc) * cls.second.size());
                    out.push_back(l2);
                }
                if (!panel.empty()) {
                    pl.count = (int)panel.size();
                    pl.off = da.add(panel.data(), sizeof(JacobiDesc) * panel.size());
                    if (queue_off == SIZE_MAX) {
                        const std::vector<char> zero(PANEL_QUEUE_BYTES, 0);
                        queue_off = da.add(zero.data(), zero.size());
                    }
                    pl.queue_off = queue_off;
                    out.push_back(pl);
                }
                break;
            }
            case OP_COPY: {
                std::vector<CopyDesc> d;
                for (const Op* o : g) {
                    d.push_back(o->cp);
                    ln.cap0 = std::max(ln.cap0, o->cap0);
                }
                ln.off = da.add(d.data(), sizeof(CopyDesc) * d.size());
                out.push_back(ln);
                break;
            }
            case OP_INTCOPY: {
                std::vector<IntCopyDesc> d;
                for (const Op* o : g) d.push_back(o->ic);
                ln.off = da.add(d.data(), sizeof(IntCopyDesc) * d.size());
                out.push_back(ln);
                break;
            }
            case OP_SETINTS: {
                std::vector<IntSetDesc> d;
                for (const Op* o : g)
                    for (size_t i = 0; i < o->set_vals.size(); ++i) d.push_back(IntSetDesc{o->set_base + i, o->set_vals[i]});
                ln.count = (int)d.size();
                ln.off = da.add(d.data(), sizeof(IntSetDesc) * d.size());
                out.push_back(ln);
                break;
            }
            case OP_FILL: {
                std::vector<FillDesc> d;
                for (const Op* o : g) d.push_back(FillDesc{o->fill_dst, o->fill_type, o->fill_val});
                ln.off = da.add(d.data(), sizeof(FillDesc) * d.size());
                out.push_back(ln);
                break;
            }
            case OP_NORM: {
                std::vector<NormDesc> d;
                for (const Op* o : g) d.push_back(o->nd);
                ln.off = da.add(d.data(), sizeof(NormDesc) * d.size());
                out.push_back(ln);
                break;
            }
        }
    }
}

// Kernels enqueue_launches issues for ls (an upper bound).
static long long graph_kernels(const std::vector<Launch>& ls) {
    long long n = 1;  // the gather
    for (const Launch& l : ls) {
        if (l.kind == OP_JAC && l.panel)
            n += 6;  // queue reset, norms, persistent sweeps, selection, write-back, basis completion
        else
            n += 2;
    }
    return n;
}

static hipError_t enqueue_launches(const std::vector<Launch>& ls, char* dev, hipStream_t s) {
    for (const Launch& l : ls) {
        const void* arr = dev + l.off;
        hipError_t e = hipSuccess;
        switch (l.kind) {
            case OP_GEMM:
                e = launch_gemm_batched((const GemmDesc*)arr, l.count, l.gtypes, l.cap0, l.cap1, s, l.prec);
                break;
            case OP_LEFT:
                e = launch_left_mpo_batched((const LeftMpoDesc*)arr, l.count, l.ltypes, l.cap0, l.cap1, l.cap2, s);
                break;
            case OP_RIGHT:
                e = launch_right_mpo_batched((const RightMpoDesc*)arr, l.count, l.rtypes, l.cap0, l.cap1, l.cap2, s);
                break;
            case OP_JAC:
                if (l.panel)
                    e = launch_jacobi_panel_batched((const JacobiDesc*)arr, l.count, l.max_pairs, l.max_rows, l.cap1,
                                                    l.shm, (PanelQueueState*)(dev + l.queue_off), s);
                else
                    e = launch_jacobi_lds_batched((const JacobiDesc*)arr, l.count, l.E, l.shm, s, l.acc);
                break;
            case OP_COPY: e = launch_copy_batched((const CopyDesc*)arr, l.count, l.cap0, s); break;
            case OP_INTCOPY: e = launch_copy_int_batched((const IntCopyDesc*)arr, l.count, s); break;
            case OP_SETINTS:
                hipLaunchKernelGGL(set_ints_batched_kernel, dim3((l.count + 255) / 256), dim3(256), 0, s,
                                   (const IntSetDesc*)arr, l.count);
                e = hipGetLastError();
                break;
            case OP_FILL:
                hipLaunchKernelGGL(fill_batched_kernel, dim3((l.count + 255) / 256), dim3(256), 0, s,
                                   (const FillDesc*)arr, l.count);
                e = hipGetLastError();
                break;
            case OP_NORM: e = launch_norm_check_batched((const NormDesc*)arr, l.count, s); break;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void batch_cache_free(smps_ctx* c) {
    BatchCache* bc = (BatchCache*)c->batch;
    if (!bc) return;
    if (bc->exec) hipGraphExecDestroy(bc->exec);
    if (bc->graph) hipGraphDestroy(bc->graph);
    if (bc->desc_dev) hipFree(bc->desc_dev);
    delete bc;
    c->batch = nullptr;
}

// The strategy of every problem of a batch: the shared one, with the
// problem's own bond cap when max_bonds is given.
static std::vector<smps_strategy> batch_strategies(int n, const smps_strategy& st, const int* max_bonds) {
    std::vector<smps_strategy> sts(n, st);
    if (max_bonds)
        for (int i = 0; i < n; ++i) sts[i].max_bond = max_bonds[i];
    return sts;
}

// Plans of all problems of a batch in one workspace.
static int plan_batch(smps_ctx* c, int n, const smps_mpo* const* U, const smps_mps* const* v,
                      const std::vector<smps_strategy>& sts, std::vector<Plan>& plans, Layout& lay) {
    if (n > 0 && sts[0].factorization != SMPS_FACT_SVD)
        return fail(c, SMPS_EUNSUPPORTED, "the batched path uses the exact factorization only");
    plans.resize(n);
    for (int i = 0; i < n; ++i) {
        plan_problem(plans[i], U[i], v[i], sts[i], lay);
        if (plans[i].max_nvec > 2048)
            return fail(c, SMPS_EUNSUPPORTED, "two-site tensors with more than 2048 rows or columns are not supported");
    }
    return SMPS_OK;
}

// Every problem's operation sequence recorded against the workspace at
// `base`, merged into batched launches (descriptors staged in da); *nodes is
// the kernel count of the graph that would hold them.  Host only.
static int record_batch(smps_ctx* c, const std::vector<Plan>& plans, const smps_mpo* const* U,
                        const smps_mps* const* v, const std::vector<smps_strategy>& sts, char* base, DescArena& da,
                        std::vector<Launch>& launches, long long* nodes, long long* nops) {
    const int n = (int)plans.size();
    std::vector<std::vector<Op>> ops(n);
    long long total = 0;
    for (int i = 0; i < n; ++i) {
        Enq q{plans[i], U[i], v[i], sts[i], base, c->stream, (int*)(base + plans[i].o_dims)};
        q.rec = &ops[i];
        hipError_t e = q.run();
        if (e != hipSuccess) return fail(c, SMPS_EHIP, std::string("recording failed at ") + q.where);
        total += (long long)ops[i].size();
    }
    build_launches(ops, da, launches);
    *nodes = graph_kernels(launches);
    if (nops) *nops = total;
    return SMPS_OK;
}

static int refuse_graph(smps_ctx* c, long long nodes) {
    return fail(c, SMPS_EUNSUPPORTED,
                "the batch would capture " + std::to_string(nodes) + " kernels (limit " +
                    std::to_string(MAX_GRAPH_KERNELS) +
                    "); chains whose two-site tensors exceed the LDS by far take the single-problem path");
}

// Gather descriptors of the per-problem results (addresses in the workspace at
// `base`) appended to da, followed by the results area of `stride` doubles
// per problem.
struct GatherLayout {
    size_t gd_off = 0, res_off = 0, stride = 0;
};
static GatherLayout append_gather(const std::vector<Plan>& plans, char* base, DescArena& da) {
    const int n = (int)plans.size();
    GatherLayout g;
    for (int i = 0; i < n; ++i) g.stride = std::max(g.stride, (size_t)(4 + plans[i].L + 1));
    std::vector<GatherDesc> gd(n);
    for (int i = 0; i < n; ++i) {
        const Plan& p = plans[i];
        gd[i] = GatherDesc{(const int*)(base + p.o_dims), p.L, (const int*)(base + p.o_status),
                           (const double*)(base + p.o_norm2), (const double*)(base + p.o_ldelta), p.steps, nullptr};
    }
    g.gd_off = da.add(gd.data(), sizeof(GatherDesc) * n);
    g.res_off = (da.host.size() + 63) / 64 * 64;
    da.host.resize(g.res_off + sizeof(double) * g.stride * n);
    return g;
}

int plan_apply(smps_ctx* c, int n, const smps_mpo* const* U, const smps_mps* const* v, const smps_strategy& st,
               const int* max_bonds, bool batched, smps_plan_info* info) {
    char* const base = (char*)PLAN_ADDRESS_BASE;  // notional workspace: recorded, never dereferenced
    if (!batched) {
        Plan p;
        Layout lay;
        const double one = 1.0;
        int rc = plan_single(c, 1, &one, U, v, st, p, lay);
        if (rc != SMPS_OK) return rc;
        info->workspace_bytes = lay.total;
        info->steps = p.steps;
        std::vector<Op> ops;
        Enq q{p, U[0], v[0], st, base, c->stream, (int*)(base + p.o_dims)};
        q.rec = &ops;
        if (q.run() != hipSuccess) return fail(c, SMPS_EHIP, std::string("planning: recording failed at ") + q.where);
        info->operations = info->launches = (long long)ops.size();
        return check_workspace_limit(c, lay.total);
    }
    if (n == 0) return SMPS_OK;
    const std::vector<smps_strategy> sts = batch_strategies(n, st, max_bonds);
    std::vector<Plan> plans;
    Layout lay;
    int rc = plan_batch(c, n, U, v, sts, plans, lay);
    if (rc != SMPS_OK) return rc;
    info->workspace_bytes = lay.total;
    for (const Plan& p : plans) info->steps += p.steps;
    DescArena da;
    std::vector<Launch> launches;
    long long nodes = 0, nops = 0;
    rc = record_batch(c, plans, U, v, sts, base, da, launches, &nodes, &nops);
    if (rc != SMPS_OK) return rc;
    append_gather(plans, base, da);
    info->operations = nops;
    info->launches = (long long)launches.size();
    info->graph_kernels = nodes;
    info->descriptor_bytes = da.host.size();
    rc = check_workspace_limit(c, lay.total);
    if (rc != SMPS_OK) return rc;
    return nodes > MAX_GRAPH_KERNELS ? refuse_graph(c, nodes) : SMPS_OK;
}

int run_apply_batched(smps_ctx* c, int n, const smps_mpo* const* U, const smps_mps* const* v,
                      const smps_strategy& st, const int* max_bonds, smps_mps** out, double* trunc_err) {
    if (n == 0) return st.factorization == SMPS_FACT_SVD
                           ? SMPS_OK
                           : fail(c, SMPS_EUNSUPPORTED, "the batched path uses the exact factorization only");
    // ---- plans of all problems in one workspace
    const std::vector<smps_strategy> sts = batch_strategies(n, st, max_bonds);
    std::vector<Plan> plans;
    Layout lay;
    int rc = plan_batch(c, n, U, v, sts, plans, lay);
    if (rc != SMPS_OK) return rc;
    rc = ensure_arena(c, lay.total);
    if (rc != SMPS_OK) return rc;
    // cache key: the handles, their data, the workspace and the strategy
    std::vector<const void*> key;
    key.push_back(c->arena);
    key.push_back((const void*)(uintptr_t)lay.total);
    for (int i = 0; i < n; ++i) {
        key.push_back(U[i]);
        key.push_back(U[i]->data);
        key.push_back(v[i]);
        key.push_back(v[i]->data);
    }
    const int* sp = (const int*)&st;
    for (size_t i = 0; i < sizeof(st) / sizeof(int); ++i) key.push_back((const void*)(uintptr_t)(unsigned)sp[i]);
    for (int i = 0; i < n; ++i) key.push_back((const void*)(uintptr_t)(unsigned)sts[i].max_bond);
    BatchCache* bc = (BatchCache*)c->batch;
    if (!bc || bc->key != key) {
        batch_cache_free(c);
        bc = new BatchCache();
        c->batch = bc;
        // ---- record every problem's operation sequence
        DescArena da;
        std::vector<Launch> launches;
        long long nodes = 0;
        rc = record_batch(c, plans, U, v, sts, c->arena, da, launches, &nodes, nullptr);
        if (rc == SMPS_OK && nodes > MAX_GRAPH_KERNELS) rc = refuse_graph(c, nodes);
        if (rc != SMPS_OK) {
            batch_cache_free(c);
            return rc;
        }
        // gather of the per-problem results into one buffer
        const GatherLayout gl = append_gather(plans, c->arena, da);
        const size_t gd_off = gl.gd_off, res_off = gl.res_off, stride = gl.stride;
        // device copy of the descriptors (results area follows them)
        SMPS_HIP(c, hipMalloc((void**)&bc->desc_dev, da.host.size()));
        bc->desc_bytes = da.host.size();
        for (int i = 0; i < n; ++i)
            ((GatherDesc*)(da.host.data() + gd_off))[i].out = (double*)(bc->desc_dev + res_off) + stride * i;
        SMPS_HIP(c, hipMemcpy(bc->desc_dev, da.host.data(), da.host.size(), hipMemcpyHostToDevice));
        bc->results_off = res_off;
        // ---- capture the whole sequence once
        hipStream_t cs;
        SMPS_HIP(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            e = enqueue_launches(launches, bc->desc_dev, cs);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(gather_batched_kernel, dim3((n + 255) / 256), dim3(256), 0, cs,
                                   (const GatherDesc*)(bc->desc_dev + gd_off), n);
                e = hipGetLastError();
            }
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(cs, &g);
            if (e == hipSuccess) e = e2;
            bc->graph = g;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&bc->exec, bc->graph, nullptr, nullptr, 0);
        hipStreamDestroy(cs);
        if (e != hipSuccess) {
            batch_cache_free(c);
            return fail(c, SMPS_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e));
        }
        bc->key = key;
        bc->plans = plans;
    }
    // ---- replay
    SMPS_HIP(c, hipGraphLaunch(bc->exec, c->stream));
    size_t stride = 0;
    for (int i = 0; i < n; ++i) stride = std::max(stride, (size_t)(4 + plans[i].L + 1));
    std::vector<double> res(stride * n);
    SMPS_HIP(c, hipMemcpyAsync(res.data(), bc->desc_dev + bc->results_off, sizeof(double) * res.size(),
                               hipMemcpyDeviceToHost, c->stream));
    SMPS_HIP(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < n; ++i) {
        const int status = (int)res[stride * i + 3];
        if (status) return fail(c, SMPS_ENUMERIC, std::string("problem ") + std::to_string(i) + ": " +
                                                      status_message(status));
    }
    // ---- outputs: exact-size handles and one batched copy of every site
    std::vector<CopyDesc> cps;
    int cap = 0;
    long long steps_total = 0;
    for (int i = 0; i < n; ++i) {
        const Plan& p = plans[i];
        std::vector<int> bonds(p.L + 1);
        for (int k = 0; k <= p.L; ++k) bonds[k] = (int)res[stride * i + 4 + k];
        bonds[0] = bonds[p.L] = 1;
        smps_mps* m = new_mps(c, p.L, p.e, bonds);
        if (!m) {
            for (int j = 0; j < i; ++j) {
                smps_mps_destroy(out[j]);
                out[j] = nullptr;
            }
            return fail(c, SMPS_ENOMEM, "output allocation failed");
        }
        m->center = 0;
        for (int k = 0; k < p.L; ++k) {
            const double* src = k == 0 ? (p.et == T_F64 ? (const double*)(c->arena + p.o_XR[0])
                                                        : (const double*)(c->arena + p.o_XR64))
                                       : (const double*)(c->arena + p.o_psi[k]);
            const int cnt = (int)m->site_size(k);
            cps.push_back(CopyDesc{src, m->data + m->off[k], nullptr, dconst(cnt), dconst(1)});
            cap = std::max(cap, cnt);
        }
        out[i] = m;
        if (trunc_err) trunc_err[i] = res[stride * i + 0];
        steps_total += p.steps;
    }
    if (!cps.empty()) {
        // descriptors of the output copies (exact sizes are only known now)
        const size_t bytes = sizeof(CopyDesc) * cps.size();
        int rc2 = ensure_pinned(c, bytes);
        if (rc2 != SMPS_OK) return rc2;
        if (c->out_desc_bytes < bytes) {
            if (c->out_desc) hipFree(c->out_desc);
            c->out_desc = nullptr;
            c->out_desc_bytes = 0;
            SMPS_HIP(c, hipMalloc((void**)&c->out_desc, bytes));
            c->out_desc_bytes = bytes;
        }
        std::memcpy(c->pinned, cps.data(), bytes);
        SMPS_HIP(c, hipMemcpyAsync(c->out_desc, c->pinned, bytes, hipMemcpyHostToDevice, c->stream));
        SMPS_HIP(c, launch_copy_batched((const CopyDesc*)c->out_desc, (int)cps.size(), cap, c->stream));
        SMPS_HIP(c, hipStreamSynchronize(c->stream));
    }
    c->info = smps_apply_info{};
    c->info.steps = (int)steps_total;
    c->info.sweeps_done = st.max_sweeps;
    c->log_fact.clear();
    c->log_L = 0;
    c->log_delta.clear();
    c->log_rank.clear();
    c->log_spec.clear();
    c->log_norm2.clear();
    c->log_sweeps.clear();
    return SMPS_OK;
}

}  // namespace smps
