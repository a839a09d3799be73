// Rank predictor: a 32-64-64-1 ReLU network trained and evaluated on the
// device with hand-written kernels.
//
// The paper has no learned component; this network sizes the sketch of the
// randomized factorization (rsvd.hip).  Input: the 32 leading log(s_j / s_0)
// of a bond's spectrum in the previous sweep (padded with log 1e-30); output:
// the log of the kept rank.  Weights are used in bfloat16 (rounded to nearest
// even from an FP32 master copy), activations and every accumulation are
// FP32.  Loss: asymmetric Huber (threshold 1, weight 4 on under-prediction),
// mean over the batch; Adam on the FP32 master, straight-through rounding.
//
// One 256-thread workgroup handles a batch in chunks of 32 samples with all
// activations in LDS; each thread owns fixed gradient entries and sums them
// over the samples in order, so gradients are deterministic.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime.h"

namespace smps {

constexpr int NIN = 32, NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH, NPAR = OFF_B3 + 1;
constexpr int CH = 32;   // samples per chunk
constexpr int MT = 256;  // threads per workgroup
constexpr float UNDER_W = 4.0f, HUBER = 1.0f;

__device__ __forceinline__ float bf16r(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

// Forward (and, when grad != nullptr, backward) over B samples of (X,
// labels): sample s is row idx[s] (row s when idx is null).  pred (nullable)
// receives the outputs, loss (nullable) the batch-mean loss, grad (nullable)
// the gradient w.r.t. the master parameters.  The ReLU masks are read from
// the activations (z > 0 exactly when relu(z) > 0).
__global__ __launch_bounds__(MT) void mlp_kernel(const float* params, const float* X, const float* labels,
                                                 const int* idx, int B, float* pred, float* loss, float* grad) {
    __shared__ float W1[NH * NIN], W2[NH * NH], W3[NH], b1[NH], b2[NH];
    __shared__ float xs[CH * NIN], h1[CH * NH], h2[CH * NH], d2[CH * NH], d1[CH * NH];
    __shared__ float g[CH], lpart[CH], gw3[NH];
    __shared__ float b3;
    const int t = threadIdx.x;
    for (int i = t; i < NH * NIN; i += MT) W1[i] = bf16r(params[OFF_W1 + i]);
    for (int i = t; i < NH * NH; i += MT) W2[i] = bf16r(params[OFF_W2 + i]);
    for (int i = t; i < NH; i += MT) {
        W3[i] = bf16r(params[OFF_W3 + i]);
        b1[i] = params[OFF_B1 + i];
        b2[i] = params[OFF_B2 + i];
    }
    if (t == 0) b3 = params[OFF_B3];
    // gradient entries owned by this thread: 8 of W1, 16 of W2, one of
    // b2 / b1 / W3 (threads 0-63 / 64-127 / 128-191) and b3 (thread 0)
    float gW1[8], gW2[16], gB = 0.f, gB3 = 0.f, lsum = 0.f;
    for (int i = 0; i < 8; ++i) gW1[i] = 0.f;
    for (int i = 0; i < 16; ++i) gW2[i] = 0.f;
    __syncthreads();
    for (int c0 = 0; c0 < B; c0 += CH) {
        const int nc = min(CH, B - c0);
        for (int i = t; i < CH * NIN; i += MT) {
            const int s = i / NIN, f = i % NIN;
            const int row = idx ? idx[min(c0 + s, B - 1)] : min(c0 + s, B - 1);
            xs[i] = s < nc ? X[(size_t)row * NIN + f] : 0.f;
        }
        __syncthreads();
        for (int i = t; i < CH * NH; i += MT) {  // layer 1
            const int s = i / NH, u = i % NH;
            float a = b1[u];
            for (int f = 0; f < NIN; ++f) a = fmaf(W1[u * NIN + f], xs[s * NIN + f], a);
            h1[i] = fmaxf(a, 0.f);
        }
        __syncthreads();
        for (int i = t; i < CH * NH; i += MT) {  // layer 2
            const int s = i / NH, u = i % NH;
            float a = b2[u];
            for (int f = 0; f < NH; ++f) a = fmaf(W2[u * NH + f], h1[s * NH + f], a);
            h2[i] = fmaxf(a, 0.f);
        }
        __syncthreads();
        if (t < CH) {  // layer 3 and the loss
            float y = b3;
            for (int f = 0; f < NH; ++f) y = fmaf(W3[f], h2[t * NH + f], y);
            float gi = 0.f, li = 0.f;
            if (t < nc) {
                if (pred) pred[c0 + t] = y;
                if (labels) {
                    const int row = idx ? idx[c0 + t] : c0 + t;
                    const float e = y - labels[row];
                    const float w = e < 0.f ? UNDER_W : 1.f;
                    const float a = fabsf(e);
                    li = w * (a <= HUBER ? 0.5f * e * e : HUBER * (a - 0.5f * HUBER));
                    gi = w * fminf(fmaxf(e, -HUBER), HUBER) / (float)B;
                }
            }
            g[t] = gi;
            lpart[t] = li;
        }
        __syncthreads();
        if (t == 0)
            for (int s = 0; s < CH; ++s) lsum += lpart[s];
        if (grad) {
            for (int i = t; i < CH * NH; i += MT) {  // d2 = dL/dz2
                const int s = i / NH, u = i % NH;
                d2[i] = h2[i] > 0.f ? g[s] * W3[u] : 0.f;
            }
            __syncthreads();
            for (int q = 0; q < 16; ++q) {  // dW2[u][f] += sum_s d2[s][u] h1[s][f]
                const int e = t * 16 + q, u = e / NH, f = e % NH;
                float a = 0.f;
                for (int s = 0; s < CH; ++s) a = fmaf(d2[s * NH + u], h1[s * NH + f], a);
                gW2[q] += a;
            }
            if (t < NH) {  // db2 and dW3
                float a = 0.f, w3 = 0.f;
                for (int s = 0; s < CH; ++s) {
                    a += d2[s * NH + t];
                    w3 = fmaf(g[s], h2[s * NH + t], w3);
                }
                gB += a;
                gw3[t] = w3;
            }
            if (t == 0)
                for (int s = 0; s < CH; ++s) gB3 += g[s];
            for (int i = t; i < CH * NH; i += MT) {  // d1 = dL/dz1
                const int s = i / NH, f = i % NH;
                float a = 0.f;
                if (h1[i] > 0.f)
                    for (int u = 0; u < NH; ++u) a = fmaf(d2[s * NH + u], W2[u * NH + f], a);
                d1[i] = a;
            }
            __syncthreads();
            if (t >= 128 && t < 192) gB += gw3[t - 128];
            for (int q = 0; q < 8; ++q) {  // dW1[u][f] += sum_s d1[s][u] x[s][f]
                const int e = t * 8 + q, u = e / NIN, f = e % NIN;
                float a = 0.f;
                for (int s = 0; s < CH; ++s) a = fmaf(d1[s * NH + u], xs[s * NIN + f], a);
                gW1[q] += a;
            }
            if (t >= 64 && t < 128) {  // db1
                float a = 0.f;
                for (int s = 0; s < CH; ++s) a += d1[s * NH + (t - 64)];
                gB += a;
            }
        }
        __syncthreads();
    }
    if (loss && t == 0) *loss = lsum / (float)B;
    if (grad) {
        for (int q = 0; q < 8; ++q) grad[OFF_W1 + t * 8 + q] = gW1[q];
        for (int q = 0; q < 16; ++q) grad[OFF_W2 + t * 16 + q] = gW2[q];
        if (t < 64) grad[OFF_B2 + t] = gB;
        else if (t < 128) grad[OFF_B1 + (t - 64)] = gB;
        else if (t < 192) grad[OFF_W3 + (t - 128)] = gB;
        if (t == 0) grad[OFF_B3] = gB3;
    }
}

// Adam (Kingma & Ba 2015) on the FP32 master parameters.
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

struct MlpState {
    float* params = nullptr;  // NPAR
    float* m = nullptr;
    float* v = nullptr;
    float* grad = nullptr;
    float* loss = nullptr;  // scalars
    float* X = nullptr;
    float* y = nullptr;
    int* idx = nullptr;
    float* pred = nullptr;
    int cap = 0;
    long long steps = 0;
    bool init = false;
};

static MlpState* state(smps_ctx* c) {
    if (!c->mlp) c->mlp = new MlpState();
    return (MlpState*)c->mlp;
}

void mlp_free(smps_ctx* c) {
    MlpState* s = (MlpState*)c->mlp;
    if (!s) return;
    for (void* p : {(void*)s->params, (void*)s->m, (void*)s->v, (void*)s->grad, (void*)s->loss, (void*)s->X,
                    (void*)s->y, (void*)s->idx, (void*)s->pred})
        if (p) hipFree(p);
    delete s;
    c->mlp = nullptr;
}

static int ensure_data(smps_ctx* c, MlpState* s, int n) {
    if (!s->params) {
        SMPS_HIP(c, hipMalloc((void**)&s->params, sizeof(float) * NPAR));
        SMPS_HIP(c, hipMalloc((void**)&s->m, sizeof(float) * NPAR));
        SMPS_HIP(c, hipMalloc((void**)&s->v, sizeof(float) * NPAR));
        SMPS_HIP(c, hipMalloc((void**)&s->grad, sizeof(float) * NPAR));
        SMPS_HIP(c, hipMalloc((void**)&s->loss, sizeof(float) * 4096));
    }
    if (n > s->cap) {
        for (void* p : {(void*)s->X, (void*)s->y, (void*)s->idx, (void*)s->pred})
            if (p) hipFree(p);
        SMPS_HIP(c, hipMalloc((void**)&s->X, sizeof(float) * NIN * (size_t)n));
        SMPS_HIP(c, hipMalloc((void**)&s->y, sizeof(float) * (size_t)n));
        SMPS_HIP(c, hipMalloc((void**)&s->idx, sizeof(int) * (size_t)n));
        SMPS_HIP(c, hipMalloc((void**)&s->pred, sizeof(float) * (size_t)n));
        s->cap = n;
    }
    return SMPS_OK;
}

// splitmix64 (Steele, Lea, Flood 2014) for the deterministic initialisation
static unsigned long long splitmix(unsigned long long& x) {
    unsigned long long z = (x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Predicted log ranks for n feature rows already on the device (stream-ordered).
hipError_t mlp_predict_device(smps_ctx* c, const float* feats_dev, int n, float* out_dev, hipStream_t s) {
    MlpState* st = (MlpState*)c->mlp;
    if (!st || !st->init) return hipErrorNotInitialized;
    hipLaunchKernelGGL(mlp_kernel, dim3(1), dim3(MT), 0, s, st->params, feats_dev, nullptr, nullptr, n, out_dev,
                       nullptr, nullptr);
    return hipGetLastError();
}

bool mlp_ready(const smps_ctx* c) { return c->mlp && ((MlpState*)c->mlp)->init; }

}  // namespace smps

using namespace smps;

extern "C" {

int smps_rank_mlp_init(smps_ctx* c, unsigned long long seed) {
    if (!c) return SMPS_EINVAL;
    if (int rc_dev = need_device(c)) return rc_dev;
    SMPS_HIP(c, hipSetDevice(c->device));
    MlpState* s = state(c);
    int rc = ensure_data(c, s, 256);
    if (rc) return rc;
    // He-uniform weights, zero biases; the output bias starts at log(16)
    std::vector<float> p(NPAR, 0.f);
    unsigned long long x = seed * 0x2545F4914F6CDD1DULL + 1;
    auto uni = [&]() { return (float)((splitmix(x) >> 11) * (1.0 / 9007199254740992.0)) * 2.f - 1.f; };
    for (int i = 0; i < NH * NIN; ++i) p[OFF_W1 + i] = uni() * std::sqrt(6.f / NIN);
    for (int i = 0; i < NH * NH; ++i) p[OFF_W2 + i] = uni() * std::sqrt(6.f / NH);
    for (int i = 0; i < NH; ++i) p[OFF_W3 + i] = uni() * std::sqrt(6.f / NH) * 0.1f;
    p[OFF_B3] = std::log(16.f);
    std::vector<float> z(NPAR, 0.f);
    SMPS_HIP(c, hipMemcpy(s->params, p.data(), sizeof(float) * NPAR, hipMemcpyHostToDevice));
    SMPS_HIP(c, hipMemcpy(s->m, z.data(), sizeof(float) * NPAR, hipMemcpyHostToDevice));
    SMPS_HIP(c, hipMemcpy(s->v, z.data(), sizeof(float) * NPAR, hipMemcpyHostToDevice));
    s->steps = 0;
    s->init = true;
    return SMPS_OK;
}

int smps_rank_mlp_get(const smps_ctx* c, float* params, int count) {
    if (!c || !params || count != NPAR || !c->mlp || !((MlpState*)c->mlp)->init) return SMPS_EINVAL;
    if (c->planning) return SMPS_ENODEV;
    MlpState* s = (MlpState*)c->mlp;
    if (hipMemcpy(params, s->params, sizeof(float) * NPAR, hipMemcpyDeviceToHost) != hipSuccess) return SMPS_EHIP;
    return SMPS_OK;
}

int smps_rank_mlp_set(smps_ctx* c, const float* params, int count) {
    if (!c) return SMPS_EINVAL;
    if (!params || count != NPAR) return fail(c, SMPS_EINVAL, "expected 6337 parameters");
    if (int rc_dev = need_device(c)) return rc_dev;
    SMPS_HIP(c, hipSetDevice(c->device));
    MlpState* s = state(c);
    int rc = ensure_data(c, s, 256);
    if (rc) return rc;
    std::vector<float> z(NPAR, 0.f);
    SMPS_HIP(c, hipMemcpy(s->params, params, sizeof(float) * NPAR, hipMemcpyHostToDevice));
    SMPS_HIP(c, hipMemcpy(s->m, z.data(), sizeof(float) * NPAR, hipMemcpyHostToDevice));
    SMPS_HIP(c, hipMemcpy(s->v, z.data(), sizeof(float) * NPAR, hipMemcpyHostToDevice));
    s->steps = 0;
    s->init = true;
    return SMPS_OK;
}

static int upload_set(smps_ctx* c, MlpState* s, int n, const float* feats, const float* labels) {
    int rc = ensure_data(c, s, n);
    if (rc) return rc;
    SMPS_HIP(c, hipMemcpy(s->X, feats, sizeof(float) * NIN * (size_t)n, hipMemcpyHostToDevice));
    if (labels) SMPS_HIP(c, hipMemcpy(s->y, labels, sizeof(float) * (size_t)n, hipMemcpyHostToDevice));
    return SMPS_OK;
}

int smps_rank_mlp_grad(smps_ctx* c, int n, const float* feats, const float* labels, float* loss, float* grad,
                       int count) {
    if (!c) return SMPS_EINVAL;
    if (n < 1 || !feats || !labels || !loss || !grad || count != NPAR)
        return fail(c, SMPS_EINVAL, "bad arguments to smps_rank_mlp_grad");
    MlpState* s = (MlpState*)c->mlp;
    if (!s || !s->init) return fail(c, SMPS_EINVAL, "rank predictor not initialised");
    if (int rc_dev = need_device(c)) return rc_dev;
    SMPS_HIP(c, hipSetDevice(c->device));
    int rc = upload_set(c, s, n, feats, labels);
    if (rc) return rc;
    hipLaunchKernelGGL(mlp_kernel, dim3(1), dim3(MT), 0, c->stream, s->params, s->X, s->y, nullptr, n, nullptr,
                       s->loss, s->grad);
    SMPS_HIP(c, hipGetLastError());
    SMPS_HIP(c, hipMemcpyAsync(loss, s->loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    SMPS_HIP(c, hipMemcpyAsync(grad, s->grad, sizeof(float) * NPAR, hipMemcpyDeviceToHost, c->stream));
    SMPS_HIP(c, hipStreamSynchronize(c->stream));
    return SMPS_OK;
}

int smps_rank_mlp_train(smps_ctx* c, int n, const float* feats, const float* labels, int epochs, int batch,
                        float lr, float* final_loss) {
    if (!c) return SMPS_EINVAL;
    if (n < 1 || !feats || !labels || epochs < 1 || batch < 1 || !(lr > 0.f))
        return fail(c, SMPS_EINVAL, "bad arguments to smps_rank_mlp_train");
    MlpState* s = (MlpState*)c->mlp;
    if (!s || !s->init) return fail(c, SMPS_EINVAL, "rank predictor not initialised");
    if (int rc_dev = need_device(c)) return rc_dev;
    SMPS_HIP(c, hipSetDevice(c->device));
    int rc = upload_set(c, s, n, feats, labels);
    if (rc) return rc;
    const int nb = (n + batch - 1) / batch;
    if (nb > 4096) return fail(c, SMPS_EINVAL, "too many batches per epoch (at most 4096)");
    std::vector<int> perm(n);
    unsigned long long x = 0x5eed0001ULL + (unsigned long long)s->steps;
    float last = 0.f;
    for (int ep = 0; ep < epochs; ++ep) {
        // Fisher-Yates shuffle (deterministic in the number of steps taken so far)
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int i = n - 1; i > 0; --i) {
            const int j = (int)(splitmix(x) % (unsigned long long)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        SMPS_HIP(c, hipMemcpy(s->idx, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice));
        for (int b = 0; b < nb; ++b) {
            const int off = b * batch, cnt = std::min(batch, n - off);
            hipLaunchKernelGGL(mlp_kernel, dim3(1), dim3(MT), 0, c->stream, s->params, s->X, s->y, s->idx + off,
                               cnt, nullptr, s->loss + b, s->grad);
            s->steps += 1;
            const float b1 = 0.9f, b2 = 0.999f;
            const float c1 = 1.f - std::pow(b1, (float)s->steps), c2 = 1.f - std::pow(b2, (float)s->steps);
            hipLaunchKernelGGL(adam_kernel, dim3((NPAR + 255) / 256), dim3(256), 0, c->stream, s->params, s->grad,
                               s->m, s->v, NPAR, lr, b1, b2, 1e-8f, c1, c2);
        }
        SMPS_HIP(c, hipGetLastError());
        if (ep == epochs - 1) {
            std::vector<float> ls(nb);
            SMPS_HIP(c, hipMemcpyAsync(ls.data(), s->loss, sizeof(float) * nb, hipMemcpyDeviceToHost, c->stream));
            SMPS_HIP(c, hipStreamSynchronize(c->stream));
            double t = 0.0;
            for (int b = 0; b < nb; ++b) t += ls[b] * std::min(batch, n - b * batch);
            last = (float)(t / n);
        }
    }
    if (final_loss) *final_loss = last;
    return SMPS_OK;
}

int smps_rank_training_pairs(const smps_ctx* c, int max_pairs, float* feats, float* labels, int* count) {
    if (!c || !count) return SMPS_EINVAL;
    const int steps = (int)c->log_rank.size();
    const int L = c->log_L;
    const int nb = L - 1;
    if (nb < 1 || steps <= nb || (int)c->log_spec.size() < 32 * steps) {
        *count = 0;
        return SMPS_OK;
    }
    // step s = 2 nb sw + j: left-to-right bond j (j < nb), else right-to-left bond 2 nb - 1 - j
    auto prev_step = [&](int s) {
        const int sw = s / (2 * nb), j = s % (2 * nb);
        if (j < nb) return (2 * sw - 1) * nb + (nb - 1 - j);  // previous right-to-left visit
        const int k = 2 * nb - 1 - j;
        return 2 * sw * nb + k;  // this sweep's left-to-right visit
    };
    const int n = steps - nb;
    *count = n;
    const int m = std::min(n, std::max(0, max_pairs));
    for (int i = 0; i < m; ++i) {
        const int s = nb + i, ps = prev_step(s);
        const double* sp = c->log_spec.data() + 32 * (size_t)ps;
        if (feats) {
            const double s0 = sp[0];
            for (int j = 0; j < 32; ++j) {
                double v = std::log(1e-30);
                if (s0 > 0.0) {
                    const double r = sp[j] / s0;
                    if (r > 1e-30) v = std::log(r);
                }
                feats[32 * (size_t)i + j] = (float)v;
            }
        }
        if (labels) labels[i] = (float)std::log((double)std::max(1, c->log_rank[s]));
    }
    return SMPS_OK;
}

int smps_rank_mlp_predict(smps_ctx* c, int n, const float* feats, float* out) {
    if (!c) return SMPS_EINVAL;
    if (n < 1 || !feats || !out) return fail(c, SMPS_EINVAL, "bad arguments to smps_rank_mlp_predict");
    MlpState* s = (MlpState*)c->mlp;
    if (!s || !s->init) return fail(c, SMPS_EINVAL, "rank predictor not initialised");
    if (int rc_dev = need_device(c)) return rc_dev;
    SMPS_HIP(c, hipSetDevice(c->device));
    int rc = upload_set(c, s, n, feats, nullptr);
    if (rc) return rc;
    hipLaunchKernelGGL(mlp_kernel, dim3(1), dim3(MT), 0, c->stream, s->params, s->X, nullptr, nullptr, n, s->pred,
                       nullptr, nullptr);
    SMPS_HIP(c, hipGetLastError());
    SMPS_HIP(c, hipMemcpyAsync(out, s->pred, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream));
    SMPS_HIP(c, hipStreamSynchronize(c->stream));
    return SMPS_OK;
}

}  // extern "C"
