// C ABI entry points: context, handles, validation, scalar product and norm.

#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_map>

#include "runtime.h"

namespace smps {

int fail(smps_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int need_device(smps_ctx* c) {
    if (c->planning) return fail(c, SMPS_ENODEV, "a planning context has no device; this call needs one");
    return SMPS_OK;
}

// ---- live handles
namespace {
struct LiveEntry {
    smps_ctx* ctx;
    int (*destroy)(void*);
};
std::mutex live_mu;
std::unordered_map<const void*, LiveEntry>& live_handles() {
    static std::unordered_map<const void*, LiveEntry> m;
    return m;
}
}  // namespace

void handle_track(const void* h, smps_ctx* c, int (*destroy)(void*)) {
    std::lock_guard<std::mutex> g(live_mu);
    live_handles()[h] = LiveEntry{c, destroy};
}

bool handle_untrack(const void* h) {
    std::lock_guard<std::mutex> g(live_mu);
    return live_handles().erase(h) == 1;
}

bool handle_live(const void* h) {
    std::lock_guard<std::mutex> g(live_mu);
    return live_handles().count(h) != 0;
}

int check_live(smps_ctx* c, const void* h, const smps_ctx* owner, const char* what) {
    if (!h) return fail(c, SMPS_EINVAL, std::string("NULL ") + what + " handle");
    if (!handle_live(h))
        return fail(c, SMPS_EINVAL, std::string(what) + " handle is not live (destroyed, or not made by this library)");
    if (c && owner != c) return fail(c, SMPS_EINVAL, std::string(what) + " handle belongs to another context");
    return SMPS_OK;
}

int check_mps(smps_ctx* c, const smps_mps* m) {
    if (!m || !handle_live(m)) return check_live(c, m, nullptr, "MPS");
    return check_live(c, m, m->ctx, "MPS");
}

int check_mpo(smps_ctx* c, const smps_mpo* u) {
    if (!u || !handle_live(u)) return check_live(c, u, nullptr, "MPO");
    return check_live(c, u, u->ctx, "MPO");
}

void* dev_alloc(smps_ctx* c, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (c->planning) {
        const uintptr_t a = PLAN_ADDRESS_BASE + c->plan_next;
        c->plan_next += (bytes + 255) / 256 * 256;
        return (void*)a;
    }
    auto it = c->pool.find(bytes);
    if (it != c->pool.end()) {
        void* p = it->second;
        c->pool.erase(it);
        return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void dev_release(smps_ctx* c, void* p, size_t bytes) {
    if (!p || c->planning) return;
    if (bytes == 0) bytes = 8;
    c->pool.emplace(bytes, p);
}

int check_workspace_limit(smps_ctx* c, size_t bytes) {
    if (c->workspace_limit && bytes > c->workspace_limit)
        return fail(c, SMPS_ENOMEM, "the call needs " + std::to_string(bytes) +
                                        " bytes of workspace, above the context's limit of " +
                                        std::to_string(c->workspace_limit) + " bytes");
    return SMPS_OK;
}

int ensure_arena(smps_ctx* c, size_t bytes) {
    int rc = check_workspace_limit(c, bytes);
    if (rc) return rc;
    if (bytes <= c->arena_bytes) return SMPS_OK;
    rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipStreamSynchronize(c->stream));
    if (c->arena) hipFree(c->arena);
    c->arena = nullptr;
    c->arena_bytes = 0;
    size_t want = bytes + bytes / 8;
    if (c->workspace_limit) want = std::min(want, c->workspace_limit);
    if (hipMalloc((void**)&c->arena, want) != hipSuccess) {
        c->arena = nullptr;
        return fail(c, SMPS_ENOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    c->arena_bytes = want;
    return SMPS_OK;
}

int ensure_pinned(smps_ctx* c, size_t bytes) {
    if (bytes <= c->pinned_bytes) return SMPS_OK;
    SMPS_HIP(c, hipStreamSynchronize(c->stream));
    if (c->pinned) hipHostFree(c->pinned);
    c->pinned = nullptr;
    c->pinned_bytes = 0;
    SMPS_HIP(c, hipHostMalloc((void**)&c->pinned, bytes, hipHostMallocDefault));
    c->pinned_bytes = bytes;
    return SMPS_OK;
}

int prof_begin(smps_ctx* c, hipStream_t s) {
    if (!c->profiling) return -1;
    while ((int)c->ev_pool.size() < c->ev_used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        c->ev_pool.push_back(e);
    }
    const int tok = c->ev_used;
    c->ev_used += 2;
    if (hipEventRecord(c->ev_pool[tok], s) != hipSuccess) return -1;
    return tok;
}

void prof_end(smps_ctx* c, hipStream_t s, int token, int category, int also) {
    if (token < 0) return;
    if (hipEventRecord(c->ev_pool[token + 1], s) != hipSuccess) return;
    const int n = smps_ctx::PROF_CATEGORIES;
    if (category >= 0 && category < n) c->ev_pending[category].emplace_back(token, token + 1);
    if (also >= 0 && also < n && also != category) c->ev_pending[also].emplace_back(token, token + 1);
}

void prof_collect(smps_ctx* c) {
    for (int cat = 0; cat < smps_ctx::PROF_CATEGORIES; ++cat) {
        for (auto& pr : c->ev_pending[cat]) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, c->ev_pool[pr.first], c->ev_pool[pr.second]) == hipSuccess) {
                c->prof_ms[cat] += ms;
                c->prof_n[cat] += 1;
            }
        }
        c->ev_pending[cat].clear();
    }
    c->ev_used = 0;
}

static int destroy_mps_entry(void* h) { return smps_mps_destroy((smps_mps*)h); }
static int destroy_mpo_entry(void* h) { return smps_mpo_destroy((smps_mpo*)h); }

smps_mps* new_mps(smps_ctx* c, int L, const std::vector<int>& phys, const std::vector<int>& bonds) {
    smps_mps* m = new smps_mps();
    m->ctx = c;
    m->L = L;
    m->phys = phys;
    m->bonds = bonds;
    m->off.resize(L);
    size_t tot = 0;
    for (int k = 0; k < L; ++k) {
        m->off[k] = tot;
        tot += m->site_size(k);
    }
    m->bytes = 8 * tot;
    m->data = (double*)dev_alloc(c, m->bytes);
    if (!m->data) {
        delete m;
        return nullptr;
    }
    handle_track(m, c, destroy_mps_entry);
    return m;
}

smps_mpo* new_mpo(smps_ctx* c, int L, const std::vector<int>& pout, const std::vector<int>& pin,
                  const std::vector<int>& bonds, bool alloc) {
    smps_mpo* u = new smps_mpo();
    u->ctx = c;
    u->L = L;
    u->pout = pout;
    u->pin = pin;
    u->bonds = bonds;
    u->off.resize(L);
    size_t tot = 0;
    for (int k = 0; k < L; ++k) {
        u->off[k] = tot;
        tot += u->site_size(k);
    }
    u->bytes = 8 * tot;
    if (alloc) {
        u->data = (double*)dev_alloc(c, u->bytes);
        if (!u->data) {
            delete u;
            return nullptr;
        }
    }
    handle_track(u, c, destroy_mpo_entry);
    return u;
}

static int check_strategy(smps_ctx* c, const smps_strategy* st) {
    if (!st) return fail(c, SMPS_EINVAL, "strategy is NULL");
    if (st->max_bond < 1) return fail(c, SMPS_EINVAL, "max_bond must be >= 1");
    if (!(st->tol >= 0.0) || !std::isfinite(st->tol)) return fail(c, SMPS_EINVAL, "tol must be finite and >= 0");
    if (st->max_sweeps < 1) return fail(c, SMPS_EINVAL, "max_sweeps must be >= 1");
    if (st->trunc_mode != SMPS_TRUNC_REL_NORM2 && st->trunc_mode != SMPS_TRUNC_REL_SV)
        return fail(c, SMPS_EINVAL, "unknown truncation mode");
    if (st->precision < SMPS_PREC_FP64 || st->precision > SMPS_PREC_BF16)
        return fail(c, SMPS_EINVAL, "unknown precision");
    if (st->factorization != SMPS_FACT_SVD && st->factorization != SMPS_FACT_RSVD_MLP &&
        st->factorization != SMPS_FACT_RSVD_PREV && st->factorization != SMPS_FACT_RSVD_FIXED)
        return fail(c, SMPS_EINVAL, "unknown factorization");
    return SMPS_OK;
}

static int check_chain(smps_ctx* c, int L, const int* phys, const int* bonds) {
    if (L < 1) return fail(c, SMPS_EINVAL, "L must be >= 1");
    if (!phys || !bonds) return fail(c, SMPS_EINVAL, "phys/bonds is NULL");
    if (bonds[0] != 1 || bonds[L] != 1) return fail(c, SMPS_EINVAL, "open boundary bonds must be 1");
    for (int k = 0; k < L; ++k)
        if (phys[k] < 1) return fail(c, SMPS_EINVAL, "physical dimensions must be >= 1");
    for (int k = 0; k <= L; ++k)
        if (bonds[k] < 1) return fail(c, SMPS_EINVAL, "bond dimensions must be >= 1");
    return SMPS_OK;
}

// Scratch of smps_scprod_noalloc: the two transfer matrices of the sweep
// and one partial product, 4 MiB per device for the life of the process.
// Host code never uses the array's name as an address: each device's copy
// lives at its own address, looked up once per device when a context is
// created on it (scratch_for_device) and passed to the kernels from there.
constexpr size_t SCPROD_SCRATCH_BYTES = size_t(4) << 20;
__device__ __align__(256) double scratch[SCPROD_SCRATCH_BYTES / sizeof(double)];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_m;
double* g_scratch_ptr[MAX_DEVICES] = {};

// Address of this device's copy of `scratch`; the device must be current.
hipError_t scratch_for_device(int device, double** out) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_m);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = (double*)p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

}  // namespace smps

using namespace smps;

extern "C" {

int smps_ctx_create(int device, void* hip_stream, smps_ctx** out) {
    if (!out) return SMPS_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SMPS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return SMPS_EHIP;
    if (jacobi_init(device) != hipSuccess) return SMPS_EHIP;
    if (gtd_init() != hipSuccess) return SMPS_EHIP;
    double* scr = nullptr;
    if (scratch_for_device(device, &scr) != hipSuccess) return SMPS_EHIP;
    smps_ctx* c = new smps_ctx();
    c->device = device;
    c->scratch = scr;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return SMPS_OK;
}

int smps_ctx_create_planning(smps_ctx** out) {
    if (!out) return SMPS_EINVAL;
    smps_ctx* c = new smps_ctx();
    c->device = -1;
    c->planning = true;
    *out = c;
    return SMPS_OK;
}

int smps_ctx_destroy(smps_ctx* c) {
    if (!c) return SMPS_EINVAL;
    // the handles this context still owns go first (their storage returns to the pool)
    std::vector<std::pair<void*, int (*)(void*)>> owned;
    {
        std::lock_guard<std::mutex> g(live_mu);
        for (auto& kv : live_handles())
            if (kv.second.ctx == c) owned.emplace_back(const_cast<void*>(kv.first), kv.second.destroy);
    }
    for (auto& h : owned) h.second(h.first);
    if (c->planning) {
        delete c;
        return SMPS_OK;
    }
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    if (c->arena) hipFree(c->arena);
    if (c->pinned) hipHostFree(c->pinned);
    for (auto& kv : c->pool) hipFree(kv.second);
    for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
    batch_cache_free(c);
    if (c->out_desc) hipFree(c->out_desc);
    mlp_free(c);
    delete c;
    return SMPS_OK;
}

const char* smps_last_error(const smps_ctx* c) { return c ? c->err.c_str() : "context is NULL"; }

int smps_ctx_set_profiling(smps_ctx* c, int on) {
    if (!c) return SMPS_EINVAL;
    int rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipStreamSynchronize(c->stream));
    prof_collect(c);
    c->profiling = on != 0;
    for (int cat = 0; cat < smps_ctx::PROF_CATEGORIES; ++cat) {
        c->prof_ms[cat] = 0.0;
        c->prof_n[cat] = 0;
    }
    return SMPS_OK;
}

int smps_ctx_kernel_time(smps_ctx* c, int category, double* total_ms, long long* launches) {
    if (!c || category < 0 || category >= smps_ctx::PROF_CATEGORIES) return SMPS_EINVAL;
    int rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipStreamSynchronize(c->stream));
    prof_collect(c);
    if (total_ms) *total_ms = c->prof_ms[category];
    if (launches) *launches = c->prof_n[category];
    return SMPS_OK;
}

int smps_ctx_set_split(smps_ctx* c, int method) {
    if (!c) return SMPS_EINVAL;
    if (method != SMPS_SPLIT_AUTO && method != SMPS_SPLIT_JACOBI && method != SMPS_SPLIT_GRAM)
        return fail(c, SMPS_EINVAL, "unknown split method");
    c->split_method = method;
    return SMPS_OK;
}

int smps_ctx_workspace_bytes(const smps_ctx* c, size_t* bytes) {
    if (!c || !bytes) return SMPS_EINVAL;
    *bytes = c->arena_bytes;
    return SMPS_OK;
}

int smps_ctx_set_workspace_limit(smps_ctx* c, size_t bytes) {
    if (!c) return SMPS_EINVAL;
    c->workspace_limit = bytes;
    if (bytes && c->arena_bytes > bytes) {
        SMPS_HIP(c, hipStreamSynchronize(c->stream));
        SMPS_HIP(c, hipFree(c->arena));
        c->arena = nullptr;
        c->arena_bytes = 0;
        // a cached batch graph addresses the old arena
        batch_cache_free(c);
    }
    return SMPS_OK;
}

static int mps_create_impl(smps_ctx* c, int L, const int* phys, const int* bonds, int dtype,
                           const void* const* tensors, smps_mps** out, bool device) {
    if (!out) return fail(c, SMPS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c) return SMPS_EINVAL;
    int rc = check_chain(c, L, phys, bonds);
    if (rc) return rc;
    if (dtype != SMPS_F64 && dtype != SMPS_F32) return fail(c, SMPS_EINVAL, "unknown dtype");
    if (device || !c->planning) {
        rc = need_device(c);
        if (rc) return rc;
        SMPS_HIP(c, hipSetDevice(c->device));
    }
    smps_mps* m = new_mps(c, L, std::vector<int>(phys, phys + L), std::vector<int>(bonds, bonds + L + 1));
    if (!m) return fail(c, SMPS_ENOMEM, "MPS allocation failed");
    if (c->planning) {  // shapes only
        *out = m;
        return SMPS_OK;
    }
    std::vector<double> tmp;
    for (int k = 0; k < L; ++k) {
        const size_t n = m->site_size(k);
        double* dst = m->data + m->off[k];
        const void* src = tensors ? tensors[k] : nullptr;
        hipError_t e = hipSuccess;
        if (!src) {
            e = launch_fill(dst, 0.0, n, c->stream);
        } else if (device) {
            if (dtype == SMPS_F64)
                e = hipMemcpyAsync(dst, src, 8 * n, hipMemcpyDeviceToDevice, c->stream);
            else
                e = launch_convert_f32_f64((const float*)src, dst, n, c->stream);
        } else {
            if (dtype == SMPS_F64) {
                e = hipMemcpyAsync(dst, src, 8 * n, hipMemcpyHostToDevice, c->stream);
            } else {
                tmp.resize(n);
                const float* f = (const float*)src;
                for (size_t i = 0; i < n; ++i) tmp[i] = (double)f[i];
                e = hipMemcpyAsync(dst, tmp.data(), 8 * n, hipMemcpyHostToDevice, c->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            }
        }
        if (e != hipSuccess) {
            smps_mps_destroy(m);
            return fail(c, SMPS_EHIP, std::string("MPS upload failed: ") + hipGetErrorString(e));
        }
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        smps_mps_destroy(m);
        return fail(c, SMPS_EHIP, std::string("MPS upload failed: ") + hipGetErrorString(e));
    }
    *out = m;
    return SMPS_OK;
}

int smps_mps_create(smps_ctx* c, int L, const int* phys, const int* bonds, int dtype, const void* const* tensors,
                    smps_mps** out) {
    return mps_create_impl(c, L, phys, bonds, dtype, tensors, out, false);
}

int smps_mps_create_device(smps_ctx* c, int L, const int* phys, const int* bonds, int dtype,
                           const void* const* tensors, smps_mps** out) {
    return mps_create_impl(c, L, phys, bonds, dtype, tensors, out, true);
}

int smps_mps_destroy(smps_mps* m) {
    if (!m || !handle_untrack(m)) return SMPS_EINVAL;
    if (m->ctx) dev_release(m->ctx, m->data, m->bytes);
    m->data = nullptr;
    delete m;
    return SMPS_OK;
}

int smps_mps_shape(const smps_mps* m, int* L, int* phys, int* bonds, int* center) {
    if (!m || !handle_live(m)) return SMPS_EINVAL;
    if (L) *L = m->L;
    if (phys) std::memcpy(phys, m->phys.data(), sizeof(int) * m->L);
    if (bonds) std::memcpy(bonds, m->bonds.data(), sizeof(int) * (m->L + 1));
    if (center) *center = m->center;
    return SMPS_OK;
}

int smps_mps_read(smps_ctx* c, const smps_mps* m, int site, double* host_out, size_t count) {
    if (!c) return SMPS_EINVAL;
    int rc = check_mps(c, m);
    if (rc) return rc;
    if (!host_out) return fail(c, SMPS_EINVAL, "NULL argument");
    if (site < 0 || site >= m->L) return fail(c, SMPS_EINVAL, "site out of range");
    if (count != m->site_size(site)) return fail(c, SMPS_EINVAL, "count does not match the site size");
    rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipSetDevice(c->device));
    SMPS_HIP(c, hipMemcpyAsync(host_out, m->data + m->off[site], 8 * count, hipMemcpyDeviceToHost, c->stream));
    SMPS_HIP(c, hipStreamSynchronize(c->stream));
    return SMPS_OK;
}

int smps_mpo_shape(const smps_mpo* u, int* L, int* pout, int* pin, int* bonds) {
    if (!u || !handle_live(u)) return SMPS_EINVAL;
    if (L) *L = u->L;
    if (pout) std::memcpy(pout, u->pout.data(), sizeof(int) * u->L);
    if (pin) std::memcpy(pin, u->pin.data(), sizeof(int) * u->L);
    if (bonds) std::memcpy(bonds, u->bonds.data(), sizeof(int) * (u->L + 1));
    return SMPS_OK;
}

int smps_mpo_read(smps_ctx* c, const smps_mpo* u, int site, double* host_out, size_t count) {
    if (!c) return SMPS_EINVAL;
    int rc = check_mpo(c, u);
    if (rc) return rc;
    if (!host_out) return fail(c, SMPS_EINVAL, "NULL argument");
    if (site < 0 || site >= u->L) return fail(c, SMPS_EINVAL, "site out of range");
    if (count != u->site_size(site)) return fail(c, SMPS_EINVAL, "count does not match the site size");
    rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipSetDevice(c->device));
    SMPS_HIP(c, hipMemcpyAsync(host_out, u->data + u->off[site], 8 * count, hipMemcpyDeviceToHost, c->stream));
    SMPS_HIP(c, hipStreamSynchronize(c->stream));
    return SMPS_OK;
}

int smps_mps_device_ptr(const smps_mps* m, int site, const double** ptr) {
    if (!m || !handle_live(m) || !ptr || site < 0 || site >= m->L) return SMPS_EINVAL;
    if (m->ctx->planning) return SMPS_ENODEV;
    *ptr = m->data + m->off[site];
    return SMPS_OK;
}

int smps_mpo_create(smps_ctx* c, int L, const int* pout, const int* pin, const int* bonds, int dtype,
                    const void* const* tensors, smps_mpo** out) {
    if (!out) return fail(c, SMPS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c) return SMPS_EINVAL;
    int rc = check_chain(c, L, pout, bonds);
    if (rc) return rc;
    rc = check_chain(c, L, pin, bonds);
    if (rc) return rc;
    if (dtype != SMPS_F64 && dtype != SMPS_F32) return fail(c, SMPS_EINVAL, "unknown dtype");
    if (!c->planning) SMPS_HIP(c, hipSetDevice(c->device));
    smps_mpo* u = new_mpo(c, L, std::vector<int>(pout, pout + L), std::vector<int>(pin, pin + L),
                          std::vector<int>(bonds, bonds + L + 1));
    if (!u) return fail(c, SMPS_ENOMEM, "MPO allocation failed");
    if (c->planning) {  // shapes only
        *out = u;
        return SMPS_OK;
    }
    const size_t tot = u->bytes / 8;
    std::vector<double> h(tot, 0.0);
    for (int k = 0; k < L; ++k) {
        const void* src = tensors ? tensors[k] : nullptr;
        if (!src) continue;
        const size_t n = u->site_size(k);
        if (dtype == SMPS_F64)
            std::memcpy(h.data() + u->off[k], src, 8 * n);
        else
            for (size_t i = 0; i < n; ++i) h[u->off[k] + i] = ((const float*)src)[i];
    }
    hipError_t e = hipMemcpyAsync(u->data, h.data(), 8 * tot, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        smps_mpo_destroy(u);
        return fail(c, SMPS_EHIP, std::string("MPO upload failed: ") + hipGetErrorString(e));
    }
    *out = u;
    return SMPS_OK;
}

int smps_mpo_destroy(smps_mpo* u) {
    if (!u || !handle_untrack(u)) return SMPS_EINVAL;
    if (u->ctx) dev_release(u->ctx, u->data, u->bytes);
    delete u;
    return SMPS_OK;
}

static int check_pair(smps_ctx* c, const smps_mpo* U, const smps_mps* v) {
    int rc = check_mpo(c, U);
    if (rc) return rc;
    rc = check_mps(c, v);
    if (rc) return rc;
    if (U->L != v->L) return fail(c, SMPS_EINVAL, "MPO and MPS lengths differ");
    for (int k = 0; k < v->L; ++k)
        if (U->pin[k] != v->phys[k]) return fail(c, SMPS_EINVAL, "MPO input dimension differs from MPS physical dimension");
    for (int k = 0; k < v->L; ++k)
        if (U->pout[k] != U->pin[k])
            return fail(c, SMPS_EUNSUPPORTED, "the guess is the input state, so the operator must map each site "
                                              "space to itself (phys_out == phys_in)");
    return SMPS_OK;
}

int smps_mpo_apply(smps_ctx* c, const smps_mpo* U, const smps_mps* v, const smps_strategy* st, smps_mps** out,
                   double* trunc_err) {
    if (!c) return SMPS_EINVAL;
    if (!out) return fail(c, SMPS_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_pair(c, U, v);
    if (rc) return rc;
    rc = check_strategy(c, st);
    if (rc) return rc;
    // a planning context gets as far as the workspace: SMPS_ENOMEM above its
    // limit, else SMPS_ENODEV
    if (!c->planning) SMPS_HIP(c, hipSetDevice(c->device));
    return run_apply(c, U, v, *st, out, trunc_err);
}

int smps_simplify(smps_ctx* c, const smps_mps* v, const smps_strategy* st, smps_mps** out, double* trunc_err) {
    if (!c) return SMPS_EINVAL;
    if (!out) return fail(c, SMPS_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_mps(c, v);
    if (rc) return rc;
    rc = check_strategy(c, st);
    if (rc) return rc;
    rc = need_device(c);
    if (rc) return rc;
    // identity operator with bond 1 (Eq. simplification with phi = v)
    std::vector<int> bonds(v->L + 1, 1);
    std::vector<std::vector<double>> eye(v->L);
    std::vector<const void*> ptrs(v->L);
    for (int k = 0; k < v->L; ++k) {
        const int d = v->phys[k];
        eye[k].assign((size_t)d * d, 0.0);
        for (int i = 0; i < d; ++i) eye[k][(size_t)i * d + i] = 1.0;
        ptrs[k] = eye[k].data();
    }
    smps_mpo* I = nullptr;
    rc = smps_mpo_create(c, v->L, v->phys.data(), v->phys.data(), bonds.data(), SMPS_F64, ptrs.data(), &I);
    if (rc) return rc;
    rc = run_apply(c, I, v, *st, out, trunc_err);
    smps_mpo_destroy(I);
    return rc;
}

// identity operator with bond 1 on the site spaces of v
static int identity_mpo(smps_ctx* c, const smps_mps* v, smps_mpo** I) {
    std::vector<int> bonds(v->L + 1, 1);
    std::vector<std::vector<double>> eye(v->L);
    std::vector<const void*> ptrs(v->L);
    for (int k = 0; k < v->L; ++k) {
        const int d = v->phys[k];
        eye[k].assign((size_t)d * d, 0.0);
        for (int i = 0; i < d; ++i) eye[k][(size_t)i * d + i] = 1.0;
        ptrs[k] = eye[k].data();
    }
    return smps_mpo_create(c, v->L, v->phys.data(), v->phys.data(), bonds.data(), SMPS_F64, ptrs.data(), I);
}

// Compression of a linear combination (Sec. 2.4.1, Eq. mps-sum-opt).
int smps_combine(smps_ctx* c, int n, const double* w, const smps_mpo* const* U, const smps_mps* const* v,
                 const smps_strategy* st, smps_mps** out, double* trunc_err) {
    if (!c) return SMPS_EINVAL;
    if (!out) return fail(c, SMPS_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !w || !v) return fail(c, SMPS_EINVAL, "a combination needs n >= 1 weights and states");
    int rc = check_strategy(c, st);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) {
        rc = check_mps(c, v[i]);
        if (rc) return rc;
        if (!std::isfinite(w[i])) return fail(c, SMPS_EINVAL, "weights must be finite");
        if (v[i]->L != v[0]->L || v[i]->phys != v[0]->phys)
            return fail(c, SMPS_EINVAL, "the states of a combination must share length and physical dimensions");
        if (U && U[i]) {
            rc = check_pair(c, U[i], v[i]);
            if (rc) return rc;
        }
    }
    rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipSetDevice(c->device));
    std::vector<const smps_mpo*> ops(n);
    std::vector<smps_mpo*> owned;
    for (int i = 0; i < n; ++i) {
        if (U && U[i]) {
            ops[i] = U[i];
            continue;
        }
        smps_mpo* I = nullptr;
        rc = identity_mpo(c, v[i], &I);
        if (rc) break;
        owned.push_back(I);
        ops[i] = I;
    }
    if (rc == SMPS_OK) rc = run_combine(c, n, w, ops.data(), v, *st, out, trunc_err);
    for (smps_mpo* I : owned) smps_mpo_destroy(I);
    return rc;
}

// Transposed operator (real arithmetic: the adjoint), for products from the right.
int smps_mpo_transpose(smps_ctx* c, const smps_mpo* U, smps_mpo** out) {
    if (!c) return SMPS_EINVAL;
    if (!out) return fail(c, SMPS_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_mpo(c, U);
    if (rc) return rc;
    rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipSetDevice(c->device));
    smps_mpo* T = new_mpo(c, U->L, U->pin, U->pout, U->bonds);  // same site sizes as U
    if (!T) return fail(c, SMPS_ENOMEM, "MPO allocation failed");
    for (int k = 0; k < U->L; ++k) {
        const hipError_t e = launch_mpo_site_transpose(U->data + U->off[k], T->data + T->off[k], U->bonds[k],
                                                       U->pout[k], U->pin[k], U->bonds[k + 1], c->stream);
        if (e != hipSuccess) {
            smps_mpo_destroy(T);
            return fail(c, SMPS_EHIP, std::string("transpose: ") + hipGetErrorString(e));
        }
    }
    *out = T;
    return SMPS_OK;
}

// v @ U (Sec. 2.4.2): the operator applied from the right, U^T v in real arithmetic.
int smps_mpo_apply_right(smps_ctx* c, const smps_mps* v, const smps_mpo* U, const smps_strategy* st,
                         smps_mps** out, double* trunc_err) {
    if (!c) return SMPS_EINVAL;
    if (!out) return fail(c, SMPS_EINVAL, "out is NULL");
    *out = nullptr;
    smps_mpo* T = nullptr;
    int rc = smps_mpo_transpose(c, U, &T);
    if (rc) return rc;
    rc = smps_mpo_apply(c, T, v, st, out, trunc_err);
    smps_mpo_destroy(T);
    return rc;
}

// Sequential application of a list of operators, compressing after each
// product (Sec. 2.4.3): U[n-1] ... U[1] U[0] v.
int smps_mpo_list_apply(smps_ctx* c, int n, const smps_mpo* const* U, const smps_mps* v, const smps_strategy* st,
                        smps_mps** out, double* trunc_err) {
    if (!c) return SMPS_EINVAL;
    if (!out) return fail(c, SMPS_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !U || !v) return fail(c, SMPS_EINVAL, "an operator list needs n >= 1 operators and a state");
    const smps_mps* cur = v;
    smps_mps* owned = nullptr;
    double total = 0.0;
    for (int i = 0; i < n; ++i) {
        smps_mps* next = nullptr;
        double err = 0.0;
        const int rc = smps_mpo_apply(c, U[i], cur, st, &next, &err);
        if (owned) smps_mps_destroy(owned);
        if (rc) return rc;
        owned = next;
        cur = next;
        total += err;
    }
    if (trunc_err) *trunc_err = total;
    *out = owned;
    return SMPS_OK;
}

// Compression of an operator (the paper's simplify_mpo, Sec. 2.4.1): the MPO
// read as an MPS whose site space is (out, in) is compressed by simplify.
int smps_mpo_simplify(smps_ctx* c, const smps_mpo* U, const smps_strategy* st, smps_mpo** out, double* trunc_err) {
    if (!c) return SMPS_EINVAL;
    if (!out) return fail(c, SMPS_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_mpo(c, U);
    if (rc) return rc;
    rc = check_strategy(c, st);
    if (rc) return rc;
    rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipSetDevice(c->device));
    std::vector<int> phys(U->L);
    for (int k = 0; k < U->L; ++k) phys[k] = U->pout[k] * U->pin[k];
    smps_mps* m = new_mps(c, U->L, phys, U->bonds);
    if (!m) return fail(c, SMPS_ENOMEM, "allocation failed");
    SMPS_HIP(c, hipMemcpyAsync(m->data, U->data, U->bytes, hipMemcpyDeviceToDevice, c->stream));
    smps_mps* r = nullptr;
    rc = smps_simplify(c, m, st, &r, trunc_err);
    smps_mps_destroy(m);
    if (rc) return rc;
    smps_mpo* T = new_mpo(c, U->L, U->pout, U->pin, r->bonds, false);
    T->data = r->data;  // the MPS storage becomes the operator's (same sizes and offsets)
    r->data = nullptr;
    r->bytes = 0;
    smps_mps_destroy(r);
    *out = T;
    return SMPS_OK;
}

int smps_dmrg(smps_ctx* c, const smps_mpo* H, const smps_mps* guess, const smps_strategy* st, int krylov_dim,
              smps_mps** out, double* energy) {
    if (!c) return SMPS_EINVAL;
    if (!out) return fail(c, SMPS_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_mpo(c, H);
    if (rc) return rc;
    rc = check_mps(c, guess);
    if (rc) return rc;
    rc = check_strategy(c, st);
    if (rc) return rc;
    if (st->precision != SMPS_PREC_FP64 || st->factorization != SMPS_FACT_SVD)
        return fail(c, SMPS_EUNSUPPORTED, "DMRG runs in FP64 with the exact factorization");
    if (krylov_dim < 2 || krylov_dim > 128) return fail(c, SMPS_EINVAL, "krylov_dim must be in 2..128");
    if (H->L != guess->L) return fail(c, SMPS_EINVAL, "operator and guess lengths differ");
    if (guess->L < 2) return fail(c, SMPS_EUNSUPPORTED, "DMRG needs at least two sites");
    for (int k = 0; k < H->L; ++k)
        if (H->pout[k] != guess->phys[k] || H->pin[k] != guess->phys[k])
            return fail(c, SMPS_EINVAL, "operator site dimensions must equal the guess's");
    rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipSetDevice(c->device));
    return run_dmrg(c, H, guess, *st, krylov_dim, out, energy);
}

static int check_batch(smps_ctx* c, int n, const smps_mpo* const* U, const smps_mps* const* v,
                       const int* max_bonds, const smps_strategy* st) {
    if (n < 0 || (n > 0 && (!U || !v))) return fail(c, SMPS_EINVAL, "bad batch arguments");
    int rc = check_strategy(c, st);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) {
        rc = check_pair(c, U[i], v[i]);
        if (rc) return rc;
        if (max_bonds && max_bonds[i] < 1) return fail(c, SMPS_EINVAL, "max_bonds entries must be >= 1");
    }
    return SMPS_OK;
}

int smps_mpo_apply_batched_caps(smps_ctx* c, int n, const smps_mpo* const* U, const smps_mps* const* v,
                                const int* max_bonds, const smps_strategy* st, smps_mps** out, double* trunc_err) {
    if (!c) return SMPS_EINVAL;
    if (n > 0 && !out) return fail(c, SMPS_EINVAL, "bad batch arguments");
    for (int i = 0; i < n; ++i) out[i] = nullptr;
    int rc = check_batch(c, n, U, v, max_bonds, st);
    if (rc) return rc;
    if (!c->planning) SMPS_HIP(c, hipSetDevice(c->device));
    return run_apply_batched(c, n, U, v, *st, max_bonds, out, trunc_err);
}

int smps_mpo_apply_batched(smps_ctx* c, int n, const smps_mpo* const* U, const smps_mps* const* v,
                           const smps_strategy* st, smps_mps** out, double* trunc_err) {
    return smps_mpo_apply_batched_caps(c, n, U, v, nullptr, st, out, trunc_err);
}

int smps_plan_apply(smps_ctx* c, const smps_mpo* U, const smps_mps* v, const smps_strategy* st,
                    smps_plan_info* info) {
    if (!c) return SMPS_EINVAL;
    if (!info) return fail(c, SMPS_EINVAL, "info is NULL");
    *info = smps_plan_info{};
    int rc = check_pair(c, U, v);
    if (rc) return rc;
    rc = check_strategy(c, st);
    if (rc) return rc;
    return plan_apply(c, 1, &U, &v, *st, nullptr, false, info);
}

int smps_plan_apply_batched(smps_ctx* c, int n, const smps_mpo* const* U, const smps_mps* const* v,
                            const int* max_bonds, const smps_strategy* st, smps_plan_info* info) {
    if (!c) return SMPS_EINVAL;
    if (!info) return fail(c, SMPS_EINVAL, "info is NULL");
    *info = smps_plan_info{};
    int rc = check_batch(c, n, U, v, max_bonds, st);
    if (rc) return rc;
    return plan_apply(c, n, U, v, *st, max_bonds, true, info);
}

int smps_last_info(const smps_ctx* c, smps_apply_info* info) {
    if (!c || !info) return SMPS_EINVAL;
    *info = c->info;
    return SMPS_OK;
}

int smps_last_log(const smps_ctx* c, int max_steps, double* deltas, int* ranks, double* spectra, int* steps) {
    if (!c) return SMPS_EINVAL;
    const int n = (int)c->log_delta.size();
    if (steps) *steps = n;
    const int m = std::min(n, std::max(0, max_steps));
    if (deltas) std::memcpy(deltas, c->log_delta.data(), sizeof(double) * m);
    if (ranks) std::memcpy(ranks, c->log_rank.data(), sizeof(int) * m);
    if (spectra) std::memcpy(spectra, c->log_spec.data(), sizeof(double) * 32 * (size_t)m);
    return SMPS_OK;
}

int smps_autotune_apply(smps_ctx* c, const smps_mpo* U, const smps_mps* v, const smps_strategy* st, int reps,
                        int* tuned) {
    if (!c) return SMPS_EINVAL;
    int rc = check_pair(c, U, v);
    if (rc) return rc;
    rc = check_strategy(c, st);
    if (rc != SMPS_OK) return rc;
    if (reps < 1) return fail(c, SMPS_EINVAL, "reps must be >= 1");
    rc = need_device(c);
    if (rc) return rc;
    SMPS_HIP(c, hipSetDevice(c->device));
    return run_autotune(c, U, v, *st, reps, tuned);
}

int smps_last_jacobi_log(const smps_ctx* c, int max_steps, int* sweeps, int* steps) {
    if (!c) return SMPS_EINVAL;
    const int n = (int)c->log_sweeps.size();
    if (steps) *steps = n;
    const int m = std::min(n, std::max(0, max_steps));
    if (sweeps) std::memcpy(sweeps, c->log_sweeps.data(), sizeof(int) * m);
    return SMPS_OK;
}

int smps_last_factor_log(const smps_ctx* c, int max_steps, int* kinds, int* steps) {
    if (!c) return SMPS_EINVAL;
    const int n = (int)c->log_fact.size();
    if (steps) *steps = n;
    const int m = std::min(n, std::max(0, max_steps));
    if (kinds && m > 0) std::memcpy(kinds, c->log_fact.data(), sizeof(int) * m);
    return SMPS_OK;
}

// <a, b> by the transfer matrix E_{k+1} = a_k^T (E_k b_k)  (Sec. 2.4.4)
}  // extern "C"

namespace {

int check_scprod_args(smps_ctx* c, const smps_mps* a, const smps_mps* b, const double* out) {
    int rc = check_mps(c, a);
    if (rc) return rc;
    rc = check_mps(c, b);
    if (rc) return rc;
    if (!out) return fail(c, SMPS_EINVAL, "NULL argument");
    if (a->L != b->L) return fail(c, SMPS_EINVAL, "lengths differ");
    for (int k = 0; k < a->L; ++k)
        if (a->phys[k] != b->phys[k]) return fail(c, SMPS_EINVAL, "physical dimensions differ");
    return need_device(c);
}

// Workspace of the transfer-matrix sweep: offsets of E0, E1 (largest
// chi_a x chi_b) and F (largest chi_a d chi_b) and the total, in bytes.
struct ScprodLayout {
    size_t oE0, oE1, oF, total;
};
ScprodLayout scprod_layout(const smps_mps* a, const smps_mps* b) {
    size_t maxE = 1, maxF = 1;
    for (int k = 0; k < a->L; ++k) {
        maxE = std::max(maxE, (size_t)a->bonds[k + 1] * b->bonds[k + 1]);
        maxF = std::max(maxF, (size_t)a->bonds[k] * a->phys[k] * b->bonds[k + 1]);
    }
    ScprodLayout l{};
    l.oE0 = 0;
    l.oE1 = (8 * maxE + 255) / 256 * 256;
    l.oF = 2 * l.oE1;
    l.total = l.oF + (8 * maxF + 255) / 256 * 256;
    return l;
}

// <a|b> by the transfer-matrix sweep (Sec. 2.4.4) in the workspace `ws`;
// the 1 x 1 result is left at *result_dev (a device address inside ws).
int scprod_sweep(smps_ctx* c, const smps_mps* a, const smps_mps* b, char* ws, const ScprodLayout& lay,
                 const double** result_dev) {
    double* E0 = (double*)(ws + lay.oE0);
    double* E1 = (double*)(ws + lay.oE1);
    double* F = (double*)(ws + lay.oF);
    SMPS_HIP(c, launch_fill(E0, 1.0, 1, c->stream));
    for (int k = 0; k < a->L; ++k) {
        const int ca = a->bonds[k], cb = b->bonds[k], d = a->phys[k], ca2 = a->bonds[k + 1], cb2 = b->bonds[k + 1];
        GemmDesc g{};
        g.dims = nullptr;
        g.alpha = 1.0;
        // F = E b_k : (ca x cb)(cb x d cb2)
        g.A = E0;
        g.B = b->data + b->off[k];
        g.C = F;
        g.M = dconst(ca);
        g.N = dconst(d * cb2);
        g.K = dconst(cb);
        SMPS_HIP(c, launch_gemm(g, ca, d * cb2, 1, c->stream, P_F64));
        // E' = a_k^T F : a_k stored (ca d) x ca2
        GemmDesc h{};
        h.alpha = 1.0;
        h.A = a->data + a->off[k];
        h.B = F;
        h.C = E1;
        h.M = dconst(ca2);
        h.N = dconst(cb2);
        h.K = dconst(ca * d);
        h.ta = 1;
        SMPS_HIP(c, launch_gemm(h, ca2, cb2, 1, c->stream, P_F64));
        std::swap(E0, E1);
    }
    *result_dev = E0;
    return SMPS_OK;
}

}  // namespace

extern "C" {

int smps_scprod(smps_ctx* c, const smps_mps* a, const smps_mps* b, double* out) {
    if (!c) return SMPS_EINVAL;
    int rc = check_scprod_args(c, a, b, out);
    if (rc) return rc;
    SMPS_HIP(c, hipSetDevice(c->device));
    const ScprodLayout lay = scprod_layout(a, b);
    rc = ensure_arena(c, lay.total + 256);
    if (rc) return rc;
    const double* res = nullptr;
    rc = scprod_sweep(c, a, b, c->arena, lay, &res);
    if (rc) return rc;
    double r = 0.0;
    SMPS_HIP(c, hipMemcpyAsync(&r, res, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    SMPS_HIP(c, hipStreamSynchronize(c->stream));
    *out = r;
    return SMPS_OK;
}

int smps_scprod_noalloc(smps_ctx* c, const smps_mps* a, const smps_mps* b, double* out_dev) {
    if (!c) return SMPS_EINVAL;
    int rc = check_scprod_args(c, a, b, out_dev);
    if (rc) return rc;
    const ScprodLayout lay = scprod_layout(a, b);
    if (lay.total > SCPROD_SCRATCH_BYTES)
        return fail(c, SMPS_ENOMEM, "scprod_noalloc: needs " + std::to_string(lay.total) +
                                        " bytes of scratch, above its fixed " +
                                        std::to_string(SCPROD_SCRATCH_BYTES) + " bytes");
    if (!c->scratch) return fail(c, SMPS_EHIP, "scprod_noalloc: scratch address not resolved");
    SMPS_HIP(c, hipSetDevice(c->device));
    const double* res = nullptr;
    rc = scprod_sweep(c, a, b, (char*)c->scratch, lay, &res);
    if (rc) return rc;
    SMPS_HIP(c, hipMemcpyAsync(out_dev, res, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return SMPS_OK;
}

int smps_norm(smps_ctx* c, const smps_mps* a, double* out) {
    if (!c) return SMPS_EINVAL;
    int rc0 = check_mps(c, a);
    if (rc0) return rc0;
    if (!out) return fail(c, SMPS_EINVAL, "NULL argument");
    rc0 = need_device(c);
    if (rc0) return rc0;
    if (a->center < 0) {
        double s = 0.0;
        int rc = smps_scprod(c, a, a, &s);
        if (rc) return rc;
        *out = std::sqrt(std::max(0.0, s));
        return SMPS_OK;
    }
    SMPS_HIP(c, hipSetDevice(c->device));
    int rc = ensure_arena(c, 256);
    if (rc) return rc;
    double* acc = (double*)c->arena;
    const int n = (int)a->site_size(a->center);
    SMPS_HIP(c, launch_sumsq(a->data + a->off[a->center], nullptr, dconst(n), n, acc, c->stream));
    double r = 0.0;
    SMPS_HIP(c, hipMemcpyAsync(&r, acc, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    SMPS_HIP(c, hipStreamSynchronize(c->stream));
    *out = std::sqrt(r);
    return SMPS_OK;
}

}  // extern "C"
