// Host-side driver of the C ABI in a planning context (no device), built
// with the host parts of the library under the address and
// undefined-behaviour sanitizers.  It reads commands from stdin, one per
// line, and prints one result line per command:
//
//   ctx                                   -> "ctx <id>"   (planning context)
//   mps <ctx> L phys[L] bonds[L+1]        -> "rc <rc> <handle id>"
//   mpo <ctx> L pout[L] pin[L] bonds[L+1] -> "rc <rc> <handle id>"
//   destroy_mps <id> | destroy_mpo <id>   -> "rc <rc>"  (the id stays known,
//                                            so later commands pass a destroyed handle)
//   shape_mps <id>                        -> "rc <rc>"
//   limit <ctx> <bytes>                   -> "rc <rc>"
//   apply <ctx> <mpo> <mps> S             -> "rc <rc> <message>"
//   scprod <ctx> <mps> <mps>              -> "rc <rc> <message>"
//   plan <ctx> <mpo> <mps> S              -> "rc <rc> <info fields>"
//   planb <ctx> <n> (<mpo> <mps>){n} S    -> "rc <rc> <info fields>"
//   destroy_ctx <ctx>                     -> "rc <rc>"
// with S = max_bond tol trunc_mode sweeps precision factorization.  An id of
// -1 passes NULL.  Handles left alive are destroyed with their contexts at
// the end, so the leak checker sees every allocation returned.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "seemps_hip.h"

namespace {

std::vector<smps_ctx*> ctxs;
std::vector<smps_mps*> states;
std::vector<smps_mpo*> ops;

bool read_ints(int n, std::vector<int>& v) {
    v.resize(n);
    for (int i = 0; i < n; ++i)
        if (std::scanf("%d", &v[i]) != 1) return false;
    return true;
}

bool read_strategy(smps_strategy& st) {
    std::memset(&st, 0, sizeof st);
    return std::scanf("%d %lf %d %d %d %d", &st.max_bond, &st.tol, &st.trunc_mode, &st.max_sweeps, &st.precision,
                      &st.factorization) == 6;
}

smps_ctx* C(int i) { return i < 0 ? nullptr : ctxs.at(i); }
smps_mps* V(int i) { return i < 0 ? nullptr : states.at(i); }
smps_mpo* U(int i) { return i < 0 ? nullptr : ops.at(i); }

void print_info(int rc, const smps_plan_info& in) {
    std::printf("rc %d %zu %lld %lld %lld %lld %zu\n", rc, in.workspace_bytes, in.steps, in.operations, in.launches,
                in.graph_kernels, in.descriptor_bytes);
}

}  // namespace

int main() {
    char cmd[32];
    while (std::scanf("%31s", cmd) == 1) {
        const std::string c = cmd;
        int a = 0, b = 0, d = 0, L = 0;
        std::vector<int> x, y, z;
        smps_strategy st;
        if (c == "ctx") {
            smps_ctx* h = nullptr;
            const int rc = smps_ctx_create_planning(&h);
            if (rc) return 3;
            ctxs.push_back(h);
            std::printf("ctx %zu\n", ctxs.size() - 1);
        } else if (c == "mps") {
            if (std::scanf("%d %d", &a, &L) != 2 || !read_ints(L, x) || !read_ints(L + 1, y)) return 2;
            smps_mps* h = nullptr;
            const int rc = smps_mps_create(C(a), L, x.data(), y.data(), SMPS_F64, nullptr, &h);
            states.push_back(h);
            std::printf("rc %d %zu\n", rc, states.size() - 1);
        } else if (c == "mpo") {
            if (std::scanf("%d %d", &a, &L) != 2 || !read_ints(L, x) || !read_ints(L, y) || !read_ints(L + 1, z))
                return 2;
            smps_mpo* h = nullptr;
            const int rc = smps_mpo_create(C(a), L, x.data(), y.data(), z.data(), SMPS_F64, nullptr, &h);
            ops.push_back(h);
            std::printf("rc %d %zu\n", rc, ops.size() - 1);
        } else if (c == "destroy_mps") {
            if (std::scanf("%d", &a) != 1) return 2;
            std::printf("rc %d\n", smps_mps_destroy(V(a)));
        } else if (c == "destroy_mpo") {
            if (std::scanf("%d", &a) != 1) return 2;
            std::printf("rc %d\n", smps_mpo_destroy(U(a)));
        } else if (c == "shape_mps") {
            if (std::scanf("%d", &a) != 1) return 2;
            int n = 0;
            std::printf("rc %d\n", smps_mps_shape(V(a), &n, nullptr, nullptr, nullptr));
        } else if (c == "limit") {
            unsigned long long bytes = 0;
            if (std::scanf("%d %llu", &a, &bytes) != 2) return 2;
            std::printf("rc %d\n", smps_ctx_set_workspace_limit(C(a), (size_t)bytes));
        } else if (c == "apply") {
            if (std::scanf("%d %d %d", &a, &b, &d) != 3 || !read_strategy(st)) return 2;
            smps_mps* out = nullptr;
            double err = 0.0;
            const int rc = smps_mpo_apply(C(a), U(b), V(d), &st, &out, &err);
            if (out) return 4;  // nothing can be produced without a device
            std::printf("rc %d %s\n", rc, smps_last_error(C(a)));
        } else if (c == "scprod") {
            if (std::scanf("%d %d %d", &a, &b, &d) != 3) return 2;
            double r = 0.0;
            const int rc = smps_scprod(C(a), V(b), V(d), &r);
            std::printf("rc %d %s\n", rc, smps_last_error(C(a)));
        } else if (c == "plan") {
            if (std::scanf("%d %d %d", &a, &b, &d) != 3 || !read_strategy(st)) return 2;
            smps_plan_info in{};
            print_info(smps_plan_apply(C(a), U(b), V(d), &st, &in), in);
        } else if (c == "planb") {
            int n = 0;
            if (std::scanf("%d %d", &a, &n) != 2 || n < 0) return 2;
            std::vector<const smps_mpo*> us(n);
            std::vector<const smps_mps*> vs(n);
            for (int i = 0; i < n; ++i) {
                if (std::scanf("%d %d", &b, &d) != 2) return 2;
                us[i] = U(b);
                vs[i] = V(d);
            }
            if (!read_strategy(st)) return 2;
            smps_plan_info in{};
            print_info(smps_plan_apply_batched(C(a), n, us.data(), vs.data(), nullptr, &st, &in), in);
        } else if (c == "destroy_ctx") {
            if (std::scanf("%d", &a) != 1) return 2;
            std::printf("rc %d\n", smps_ctx_destroy(C(a)));
            if (a >= 0) ctxs.at(a) = nullptr;
        } else {
            return 2;
        }
        std::fflush(stdout);
    }
    for (smps_ctx* h : ctxs)
        if (h) smps_ctx_destroy(h);
    return 0;
}
