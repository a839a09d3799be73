// GEMM tile autotuner.
//
// Every product of the sweep is launched with one of four output tiles
// (64 x 64, 64 x 32, 32 x 64, 32 x 32).  Small products have few 64 x 64
// tiles and leave most compute units idle; large ones prefer the bigger tile.
// The autotuner times each candidate on the real operand shapes and keeps the
// fastest per key (precision, operand/result types, transposes, and the
// power-of-two buckets of the M and N allocation caps).  The table is process
// wide, consulted by every GEMM launch, and can be saved to / loaded from a
// small JSON file.  Every tile computes each output with the same k order, so
// the choice changes timing only, never the result bits.

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "runtime.h"

namespace smps {

namespace {
struct TileKey {
    int prec, types, ta, tb, tc, mb, nb;
    bool operator<(const TileKey& o) const {
        return std::tie(prec, types, ta, tb, tc, mb, nb) < std::tie(o.prec, o.types, o.ta, o.tb, o.tc, o.mb, o.nb);
    }
};
struct TileEntry {
    int tile;
    float us[GEMM_TILES];
};
struct TileTable {
    std::mutex m;
    std::map<TileKey, TileEntry> t;
};
TileTable& table() {
    static TileTable tt;
    return tt;
}
int bucket(int x) {
    int b = 1;
    while (b < x) b <<= 1;
    return b;
}
TileKey make_key(int prec, int a_type, int b_type, int c_type, int ta, int tb, int tc, int M, int N) {
    return TileKey{prec, (a_type << 2) | (b_type << 1) | c_type, ta, tb, tc, bucket(M), bucket(N)};
}

__global__ void fill_pattern_kernel(void* p, int type, size_t n, unsigned seed) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        unsigned h = (unsigned)i * 2654435761u ^ seed;
        h ^= h >> 13;
        h *= 0x5bd1e995u;
        const double v = (double)(h & 0xFFFFFF) / 16777216.0 - 0.5;
        if (type == T_F64)
            ((double*)p)[i] = v;
        else
            ((float*)p)[i] = (float)v;
    }
}
}  // namespace

int gemm_tile_for(const GemmDesc& g, int M_cap, int N_cap, int prec) {
    TileTable& tt = table();
    std::lock_guard<std::mutex> lock(tt.m);
    if (tt.t.empty()) return 0;
    auto it = tt.t.find(make_key(prec, g.a_type, g.b_type, g.c_type, g.ta, g.tb, g.tc, M_cap, N_cap));
    return it == tt.t.end() ? 0 : it->second.tile;
}

// Time the four tiles on an M x N x K product with the given types and
// transposes (synthetic operands on the context's stream) and record the best.
int tune_gemm_shape(smps_ctx* c, int prec, int a_type, int b_type, int c_type, int ta, int tb, int tc, int M, int N,
                    int K, int reps, int* best_out) {
    if (M < 1 || N < 1 || K < 1 || reps < 1) return fail(c, SMPS_EINVAL, "autotune: bad shape");
    const TileKey key = make_key(prec, a_type, b_type, c_type, ta, tb, tc, M, N);
    auto bytes = [](int type) { return type == T_F64 ? 8 : 4; };
    const size_t na = (size_t)M * K, nb = (size_t)K * N, nc = (size_t)M * N;
    void *A = nullptr, *B = nullptr, *C = nullptr;
    SMPS_HIP(c, hipMalloc(&A, na * bytes(a_type)));
    SMPS_HIP(c, hipMalloc(&B, nb * bytes(b_type)));
    SMPS_HIP(c, hipMalloc(&C, nc * bytes(c_type)));
    hipLaunchKernelGGL(fill_pattern_kernel, dim3(256), dim3(256), 0, c->stream, A, a_type, na, 17u);
    hipLaunchKernelGGL(fill_pattern_kernel, dim3(256), dim3(256), 0, c->stream, B, b_type, nb, 91u);
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
    g.tc = tc;
    g.a_type = a_type;
    g.b_type = b_type;
    g.c_type = c_type;
    g.alpha = 1.0;
    hipEvent_t e0, e1;
    TileEntry ent{};
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    for (int t = 0; t < GEMM_TILES && err == hipSuccess; ++t) {
        err = launch_gemm_tile(g, nullptr, M, N, 1, c->stream, prec, t);  // warm-up
        if (err == hipSuccess) err = hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps && err == hipSuccess; ++r) err = launch_gemm_tile(g, nullptr, M, N, 1, c->stream, prec, t);
        if (err == hipSuccess) err = hipEventRecord(e1, c->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        ent.us[t] = 1000.f * ms / reps;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(A);
    hipFree(B);
    hipFree(C);
    if (err != hipSuccess) return fail(c, SMPS_EHIP, std::string("autotune: ") + hipGetErrorString(err));
    ent.tile = 0;
    for (int t = 1; t < GEMM_TILES; ++t)
        if (ent.us[t] < ent.us[ent.tile]) ent.tile = t;
    {
        TileTable& tt = table();
        std::lock_guard<std::mutex> lock(tt.m);
        tt.t[key] = ent;
    }
    if (best_out) *best_out = ent.tile;
    return SMPS_OK;
}

}  // namespace smps

using namespace smps;

extern "C" {

int smps_autotune_gemm(smps_ctx* c, int precision, int M, int N, int K, int ta, int tb, int tc, int a_type,
                       int b_type, int c_type, int reps, int* best_tile) {
    if (!c) return SMPS_EINVAL;
    if (precision < SMPS_PREC_FP64 || precision > SMPS_PREC_BF16) return fail(c, SMPS_EINVAL, "unknown precision");
    for (int t : {a_type, b_type, c_type})
        if (t != SMPS_F64 && t != SMPS_F32) return fail(c, SMPS_EINVAL, "unknown operand type");
    if (int rc_dev = need_device(c)) return rc_dev;
    SMPS_HIP(c, hipSetDevice(c->device));
    return tune_gemm_shape(c, precision, a_type, b_type, c_type, ta != 0, tb != 0, tc != 0, M, N, K, reps, best_tile);
}

int smps_autotune_clear(smps_ctx* c) {
    if (!c) return SMPS_EINVAL;
    TileTable& tt = table();
    std::lock_guard<std::mutex> lock(tt.m);
    tt.t.clear();
    return SMPS_OK;
}

int smps_autotune_entries(const smps_ctx* c, int* count) {
    if (!c || !count) return SMPS_EINVAL;
    TileTable& tt = table();
    std::lock_guard<std::mutex> lock(tt.m);
    *count = (int)tt.t.size();
    return SMPS_OK;
}

int smps_autotune_save(smps_ctx* c, const char* path) {
    if (!c) return SMPS_EINVAL;
    if (!path) return fail(c, SMPS_EINVAL, "path is NULL");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(c, SMPS_EINVAL, std::string("cannot write ") + path);
    TileTable& tt = table();
    std::lock_guard<std::mutex> lock(tt.m);
    std::fprintf(f, "[\n");
    size_t i = 0;
    for (const auto& kv : tt.t) {
        const TileKey& k = kv.first;
        const TileEntry& e = kv.second;
        std::fprintf(f,
                     "  {\"precision\": %d, \"types\": %d, \"ta\": %d, \"tb\": %d, \"tc\": %d, \"m_bucket\": %d, "
                     "\"n_bucket\": %d, \"tile\": %d, \"us\": [%.3f, %.3f, %.3f, %.3f]}%s\n",
                     k.prec, k.types, k.ta, k.tb, k.tc, k.mb, k.nb, e.tile, e.us[0], e.us[1], e.us[2], e.us[3],
                     ++i < tt.t.size() ? "," : "");
    }
    std::fprintf(f, "]\n");
    std::fclose(f);
    return SMPS_OK;
}

// Reads the format written by smps_autotune_save (one entry per line).
int smps_autotune_load(smps_ctx* c, const char* path) {
    if (!c) return SMPS_EINVAL;
    if (!path) return fail(c, SMPS_EINVAL, "path is NULL");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(c, SMPS_EINVAL, std::string("cannot read ") + path);
    std::vector<std::pair<TileKey, TileEntry>> got;
    char line[1024];
    bool bad = false;
    while (std::fgets(line, sizeof line, f)) {
        if (!std::strchr(line, '{')) continue;
        TileKey k{};
        TileEntry e{};
        const int n = std::sscanf(line,
                                  " {\"precision\": %d, \"types\": %d, \"ta\": %d, \"tb\": %d, \"tc\": %d, "
                                  "\"m_bucket\": %d, \"n_bucket\": %d, \"tile\": %d, \"us\": [%f, %f, %f, %f]",
                                  &k.prec, &k.types, &k.ta, &k.tb, &k.tc, &k.mb, &k.nb, &e.tile, &e.us[0], &e.us[1],
                                  &e.us[2], &e.us[3]);
        if (n != 12 || e.tile < 0 || e.tile >= GEMM_TILES) {
            bad = true;
            break;
        }
        got.emplace_back(k, e);
    }
    std::fclose(f);
    if (bad) return fail(c, SMPS_EINVAL, std::string("malformed autotune file ") + path);
    TileTable& tt = table();
    std::lock_guard<std::mutex> lock(tt.m);
    for (const auto& kv : got) tt.t[kv.first] = kv.second;
    return SMPS_OK;
}

}  // extern "C"
