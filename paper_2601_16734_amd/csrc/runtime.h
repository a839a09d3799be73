// Host runtime objects behind the C ABI handles.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "common.h"

struct smps_ctx {
    int device = 0;
    // a planning context (smps_ctx_create_planning) has no device: handles
    // hold shapes and notional addresses, validation and the planning entry
    // points work, nothing is allocated, copied or launched
    bool planning = false;
    size_t plan_next = 0;  // next notional address offset of a planning context
    // largest workspace arena the context may hold, in bytes (0: no limit)
    size_t workspace_limit = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // grow-only workspace arena for apply/simplify/scprod
    char* arena = nullptr;
    size_t arena_bytes = 0;
    // this device's copy of the fixed scratch array of smps_scprod_noalloc
    double* scratch = nullptr;
    // exact split of the single-problem sweep: SMPS_SPLIT_AUTO, _JACOBI or _GRAM
    int split_method = 0;
    // exact-size cache of device blocks released by destroyed handles
    std::multimap<size_t, void*> pool;
    // pinned staging for small read-backs
    char* pinned = nullptr;
    size_t pinned_bytes = 0;
    // diagnostics of the last apply
    smps_apply_info info{};
    std::vector<double> log_delta, log_spec, log_norm2;
    std::vector<int> log_rank, log_sweeps;
    // per step: 0 exact factorization, +k randomized with sketch k accepted,
    // -k randomized with sketch k replaced by the exact one
    std::vector<int> log_fact;
    int log_L = 0;  // chain length of the logged apply (0 for the batched path)
    // rank predictor state (device buffers, see mlp.hip)
    void* mlp = nullptr;
    // batched execution: captured graph of the last batch shape, and the
    // device buffer of the output-copy descriptors
    void* batch = nullptr;
    char* out_desc = nullptr;
    size_t out_desc_bytes = 0;
    // optional per-category kernel timing (events recorded on the stream)
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    static constexpr int PROF_CATEGORIES = 7;  // see smps_ctx_kernel_time
    std::vector<std::pair<int, int>> ev_pending[PROF_CATEGORIES];  // (start, stop) indices per category
    int ev_used = 0;
    double prof_ms[PROF_CATEGORIES] = {};
    long long prof_n[PROF_CATEGORIES] = {};
};

struct smps_mps {
    smps_ctx* ctx = nullptr;
    int L = 0;
    std::vector<int> phys, bonds;
    int center = -1;
    double* data = nullptr;
    size_t bytes = 0;
    std::vector<size_t> off;  // element offsets
    size_t site_size(int k) const { return (size_t)bonds[k] * phys[k] * bonds[k + 1]; }
};

struct smps_mpo {
    smps_ctx* ctx = nullptr;
    int L = 0;
    std::vector<int> pout, pin, bonds;
    double* data = nullptr;
    size_t bytes = 0;
    std::vector<size_t> off;
    size_t site_size(int k) const { return (size_t)bonds[k] * pout[k] * pin[k] * bonds[k + 1]; }
};

namespace smps {
int fail(smps_ctx* c, int code, const std::string& msg);
// SMPS_ENODEV when c is a planning context (call before any device work)
int need_device(smps_ctx* c);
// SMPS_ENOMEM when a workspace of `bytes` exceeds the context's limit
int check_workspace_limit(smps_ctx* c, size_t bytes);
// Notional device addresses of a planning context and of planned workspaces:
// distinct, aligned values above this base, so that recorded operations look
// like real ones; nothing ever dereferences them.
constexpr uintptr_t PLAN_ADDRESS_BASE = uintptr_t(1) << 44;
// Live-handle registry: every handle the library hands out is registered
// with its context and its destroy function until it is destroyed, so a
// destroyed or foreign pointer is refused instead of dereferenced, and a
// context destroys the handles it still owns.
void handle_track(const void* h, smps_ctx* c, int (*destroy)(void*));
bool handle_untrack(const void* h);  // false when h was not live
bool handle_live(const void* h);
int check_mps(smps_ctx* c, const smps_mps* m);  // non-NULL, live, owned by c
int check_mpo(smps_ctx* c, const smps_mpo* u);
int check_live(smps_ctx* c, const void* h, const smps_ctx* owner, const char* what);
void* dev_alloc(smps_ctx* c, size_t bytes);
void dev_release(smps_ctx* c, void* p, size_t bytes);
int ensure_arena(smps_ctx* c, size_t bytes);
int ensure_pinned(smps_ctx* c, size_t bytes);
// Kernel timing helpers: prof_begin returns a token (or -1 when profiling is
// off) that prof_end closes; prof_collect folds finished pairs into the totals
// (call after the stream has been synchronised).
int prof_begin(smps_ctx* c, hipStream_t s);
void prof_end(smps_ctx* c, hipStream_t s, int token, int category, int also = -1);
void prof_collect(smps_ctx* c);
smps_mps* new_mps(smps_ctx* c, int L, const std::vector<int>& phys, const std::vector<int>& bonds);
// operator handle with offsets; device storage allocated when alloc is set
smps_mpo* new_mpo(smps_ctx* c, int L, const std::vector<int>& pout, const std::vector<int>& pin,
                  const std::vector<int>& bonds, bool alloc = true);

// Enqueue one apply + compression and collect its results (used by the single
// and the batched entry points).
struct ApplyProblem {
    const smps_mpo* U;
    const smps_mps* v;
};
int run_apply(smps_ctx* c, const smps_mpo* U, const smps_mps* v, const smps_strategy& st, smps_mps** out,
              double* trunc_err);
// linear combination sum_l w[l] U[l] v[l] (every U[l] non-NULL here)
int run_combine(smps_ctx* c, int n, const double* w, const smps_mpo* const* U, const smps_mps* const* v,
                const smps_strategy& st, smps_mps** out, double* trunc_err);
void mlp_free(smps_ctx* c);
// two-site DMRG ground-state search (dmrg.hip)
int run_dmrg(smps_ctx* c, const smps_mpo* H, const smps_mps* guess, const smps_strategy& st, int krylov,
             smps_mps** out, double* energy);
// GEMM tile autotuning (autotune.hip / sweep.hip)
int tune_gemm_shape(smps_ctx* c, int prec, int a_type, int b_type, int c_type, int ta, int tb, int tc, int M, int N,
                    int K, int reps, int* best_out);
int run_autotune(smps_ctx* c, const smps_mpo* U, const smps_mps* v, const smps_strategy& st, int reps, int* tuned);
// rank predictor: log-rank predictions for n device feature rows (32 floats each)
hipError_t mlp_predict_device(smps_ctx* c, const float* feats_dev, int n, float* out_dev, hipStream_t s);
bool mlp_ready(const smps_ctx* c);
void batch_cache_free(smps_ctx* c);
// max_bonds (nullable): per-problem bond caps replacing st.max_bond
int run_apply_batched(smps_ctx* c, int n, const smps_mpo* const* U, const smps_mps* const* v,
                      const smps_strategy& st, const int* max_bonds, smps_mps** out, double* trunc_err);
// What an apply (n = 1) or a batched apply would allocate and enqueue; runs
// on the host only (any context kind).
int plan_apply(smps_ctx* c, int n, const smps_mpo* const* U, const smps_mps* const* v, const smps_strategy& st,
               const int* max_bonds, bool batched, smps_plan_info* info);
}  // namespace smps

#define SMPS_HIP(c, expr)                                                                         \
    do {                                                                                          \
        hipError_t e__ = (expr);                                                                  \
        if (e__ != hipSuccess)                                                                    \
            return smps::fail((c), SMPS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e__)); \
    } while (0)
