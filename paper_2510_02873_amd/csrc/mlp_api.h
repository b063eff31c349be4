// Host side of include/pino_mlp.h: the trainable network handle, the weight
// blob, its BF16 fragment layout for the collapse kernel, and the surrogate
// launches of a collapse context.  Included once, by pino_collapse.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pino_mlp.h"
#include "ctx.h"
#include "kernels_surrogate.h"

struct pino_mlp {
    int device = 0;
    float* d_params = nullptr;
    float* d_m1 = nullptr;
    float* d_m2 = nullptr;
    float* d_grad = nullptr;
    float* d_partial = nullptr;
    float* d_partial2 = nullptr;  // per-group sums of the partials
    float* d_pq = nullptr;        // BF16-rounded parameters (BF16 forward)
    int bf16_fwd = 0;
    int64_t step = 0;
    bool broken = false;
    std::string err = "no error";
};

namespace {

constexpr int64_t kMlpMaxBatch = 65536;  // samples per pino_mlp_grad call
constexpr char kMlpMagic[8] = {'P', 'I', 'N', 'O', 'M', 'L', 'P', '1'};

struct MlpBlobHeader {
    char magic[8];
    int32_t version;
    int32_t n_params;
};

constexpr int64_t kMlpBlobBytes = (int64_t)sizeof(MlpBlobHeader) + (int64_t)pino::kNParam * sizeof(float);

thread_local std::string g_mlp_error = "no error";

bool mlp_blob_valid(const void* blob, int64_t bytes, std::string& why)
{
    if (!blob || bytes != kMlpBlobBytes) {
        why = "expected a blob of " + std::to_string(kMlpBlobBytes) + " bytes from pino_mlp_export";
        return false;
    }
    MlpBlobHeader h;
    std::memcpy(&h, blob, sizeof(h));
    if (std::memcmp(h.magic, kMlpMagic, 8) != 0 || h.version != 1 || h.n_params != pino::kNParam) {
        why = "bad blob header";
        return false;
    }
    std::vector<float> p(pino::kNParam);
    std::memcpy(p.data(), static_cast<const char*>(blob) + sizeof(h), p.size() * sizeof(float));
    for (float v : p)
        if (!std::isfinite(v)) {
            why = "non-finite parameter";
            return false;
        }
    return true;
}

// BF16 fragments of the weights in the lane order of the MFMA operands
// (see NetFrags); biases and the output layer stay FP32.
pino::NetFrags build_frags(const float* P)
{
    using namespace pino;
    NetFrags f;
    std::memset(&f, 0, sizeof(f));
    for (int mt = 0; mt < 4; ++mt)
        for (int l = 0; l < 64; ++l) {
            const int o = 16 * mt + l % 16;
            const int g = l / 16;
            for (int j = 0; j < 8; ++j) {
                // layer 1: group 0 (W_hi, W_hi), group 1 (W_lo, 0) (see NetFrags)
                const float wv = P[kOffW1 + o * kIn + (j & 3)];
                const short whi = bf16_bits(wv);
                const short wlo = bf16_bits(wv - bf16_value(whi));
                f.w1[mt][l][j] = g == 0 ? whi : (g == 1 && j < 4 ? wlo : (short)0);
                for (int kt = 0; kt < 2; ++kt) {
                    const int kk = k32_neuron(kt, g, j);
                    f.w2[mt][kt][l][j] = bf16_bits(P[kOffW2 + o * kH + kk]);
                    f.w3[mt][kt][l][j] = bf16_bits(P[kOffW3 + o * kH + kk]);
                    // output weights in the same neuron order, every row alike
                    const float w4 = P[kOffW4 + kk];
                    f.w4h[kt][l][j] = bf16_bits(w4);
                    f.w4l[kt][l][j] = bf16_bits(w4 - bf16_value(bf16_bits(w4)));
                }
            }
        }
    for (int o = 0; o < kH; ++o) {
        f.b1[o] = P[kOffB1 + o];
        f.b2[o] = P[kOffB2 + o];
        f.b3[o] = P[kOffB3 + o];
    }
    f.b4 = P[kOffB4];
    return f;
}

// Deferred-particle queue of the surrogate path: items are processed in
// chunks of at most kQueueChunk particles, by at most kQueueBlocks blocks of
// kSurrogateBlock threads, each block owning a queue segment as long as the
// particles it visits; the segments then total less than
// kQueueChunk + kSurrogateBlock kQueueBlocks.
constexpr int64_t kQueueChunk = int64_t(1) << 24;
constexpr int64_t kQueueBlocks = 4096;
constexpr int kSurrogateBlock = 256;
constexpr int64_t kQueueCap = kQueueChunk + kSurrogateBlock * kQueueBlocks;

// Dynamic LDS of k_surrogate for the largest growth table of a context: the
// knots, their index and the 25 KB of weight fragments pass the default
// 64 KiB limit for tables of about 1000 knots or more, so the kernel's limit
// is raised on the context's device (CDNA4 gives a workgroup up to 160 KiB).
pino_status surrogate_lds_limit(pino_ctx* c, size_t need)
{
    if (need <= 65536)
        return PINO_OK;
    const void* fn = c->method == PINO_CLASSIC_LCDM ? (const void*)pino::k_surrogate<true>
                                                     : (const void*)pino::k_surrogate<false>;
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
    if (e != hipSuccess) {
        c->broken = true;
        c->err = std::string("surrogate LDS limit: ") + hipGetErrorString(e);
        return PINO_ERR_HIP;
    }
    return PINO_OK;
}

pino_status mlp_upload(pino_ctx* c, const void* blob, int64_t)
{
    std::vector<float> P(pino::kNParam);
    std::memcpy(P.data(), static_cast<const char*>(blob) + sizeof(MlpBlobHeader), P.size() * sizeof(float));
    const pino::NetFrags f = build_frags(P.data());
    hipError_t e = hipMalloc(&c->d_mlp, sizeof(f));
    if (e == hipSuccess)
        e = hipMemcpy(c->d_mlp, &f, sizeof(f), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMalloc((void**)&c->d_counters, 4 * kQueueBlocks * sizeof(int64_t));
    if (e == hipSuccess)
        e = hipMemset(c->d_counters, 0, 4 * kQueueBlocks * sizeof(int64_t));
    if (e == hipSuccess) {
        c->queue_cap = kQueueCap;
        e = hipMalloc((void**)&c->d_queue, (size_t)c->queue_cap * sizeof(int32_t));
    }
    if (e != hipSuccess) {
        c->broken = true;
        c->err = std::string("surrogate upload: ") + hipGetErrorString(e);
        return PINO_ERR_HIP;
    }
    return PINO_OK;
}

inline pino_status launch_fail(pino_ctx* c, const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->broken = true;
        c->err = std::string(what) + ": " + hipGetErrorString(e);
        return PINO_ERR_HIP;
    }
    return PINO_OK;
}

// One item in chunks of at most kQueueChunk particles (queue indices are
// chunk-relative int32): per chunk one k_surrogate launch, whose blocks each
// finish the particles they deferred to the full solve.
pino_status launch_surrogate(pino_ctx* c, const pino_item& it, const pino::ItemArgs& a0, uint32_t, hipStream_t st,
                             int, int)
{
    const int block = kSurrogateBlock;
    const bool lcdm = c->method == PINO_CLASSIC_LCDM;
    const size_t lds = pino::surrogate_lds_bytes(a0.nk, a0.gi.nb, lcdm);
    const double* kap = lcdm ? c->d_kap + (size_t)it.cosmo * 6 * c->nk_max : nullptr;
    pino::KappaSlope ks{};
    if (lcdm)
        ks = pino::KappaSlope{c->kslope[3 * it.cosmo], c->kslope[3 * it.cosmo + 1], c->kslope[3 * it.cosmo + 2]};
    auto* cnt = reinterpret_cast<unsigned long long*>(c->d_counters);
    const auto* net = static_cast<const pino::NetFrags*>(c->d_mlp);
    const int64_t cap_blocks = std::min<int64_t>((int64_t)c->cu_count * c->blocks_per_cu, kQueueBlocks);
    for (int64_t start = 0; start < a0.n; start += kQueueChunk) {
        pino::ItemArgs a = a0;
        a.n = std::min<int64_t>(kQueueChunk, a0.n - start);
        for (int k = 0; k < 6; ++k)
            a.h[k] = a0.h[k] + start;
        a.Fmax = a0.Fmax + start;
        a.Rmax = a0.Rmax + start;
        a.acoll = a0.acoll ? a0.acoll + start : nullptr;
        const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((a.n + block - 1) / block, cap_blocks));
        // a block visits at most ceil(n / stride) groups of `block` particles
        const int64_t stride = grid * block;
        const int64_t seg = (a.n + stride - 1) / stride * block;
        if (lcdm)
            hipLaunchKernelGGL(pino::k_surrogate<true>, dim3((unsigned)grid), dim3(block), lds, st, a, net,
                               it.sigma_R, c->omega[it.cosmo], c->certify_rtol, cnt, c->d_queue, seg, kap, ks);
        else
            hipLaunchKernelGGL(pino::k_surrogate<false>, dim3((unsigned)grid), dim3(block), lds, st, a, net,
                               it.sigma_R, c->omega[it.cosmo], c->certify_rtol, cnt, c->d_queue, seg, kap, ks);
        const pino_status ps = launch_fail(c, "surrogate launch");
        if (ps != PINO_OK)
            return ps;
    }
    return PINO_OK;
}

pino_status mlp_fail(pino_mlp* m, hipError_t e, const char* what)
{
    m->broken = true;
    m->err = std::string(what) + ": " + hipGetErrorString(e);
    g_mlp_error = m->err;
    return PINO_ERR_HIP;
}

#define MLP_HIP(m, call)                         \
    do {                                         \
        hipError_t e_ = (call);                  \
        if (e_ != hipSuccess)                    \
            return mlp_fail((m), e_, #call);     \
    } while (0)

// splitmix64 (Steele, Lea, Flood 2014) for the initial weights
uint64_t splitmix64(uint64_t& s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

extern "C" {

pino_status pino_mlp_create(int32_t device, uint64_t seed, pino_mlp** out)
{
    if (!out || device < 0) {
        g_mlp_error = "bad arguments";
        return PINO_ERR_ARG;
    }
    *out = nullptr;
    pino_mlp* m = new (std::nothrow) pino_mlp();
    if (!m)
        return PINO_ERR_ALLOC;
    m->device = device;
    using namespace pino;
    // He-uniform weights, zero hidden biases, output bias 1 (w ~ 1 typically)
    std::vector<float> P(kNParam, 0.0f);
    uint64_t s = seed;
    auto fill = [&](int off, int rows, int cols) {
        const double lim = std::sqrt(6.0 / cols);
        for (int r = 0; r < rows * cols; ++r) {
            const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
            P[off + r] = (float)((2.0 * u - 1.0) * lim);
        }
    };
    fill(kOffW1, kH, kIn);
    fill(kOffW2, kH, kH);
    fill(kOffW3, kH, kH);
    fill(kOffW4, 1, kH);
    P[kOffB4] = 1.0f;
    const int64_t nblk = (kMlpMaxBatch + kTB - 1) / kTB;
    pino_status st = PINO_OK;
    auto fail = [&](hipError_t e, const char* what) {
        st = mlp_fail(m, e, what);
    };
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) fail(e, "hipSetDevice");
    // the gradient kernel's LDS (about 99 KiB) exceeds the default dynamic limit
    if (st == PINO_OK &&
        (e = hipFuncSetAttribute((const void*)k_mlp_grad_block, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)mlp_grad_lds_bytes())) != hipSuccess)
        fail(e, "hipFuncSetAttribute");
    if (st == PINO_OK && (e = hipMalloc(&m->d_params, kNParam * sizeof(float))) != hipSuccess) fail(e, "hipMalloc");
    if (st == PINO_OK && (e = hipMalloc(&m->d_m1, kNParam * sizeof(float))) != hipSuccess) fail(e, "hipMalloc");
    if (st == PINO_OK && (e = hipMalloc(&m->d_m2, kNParam * sizeof(float))) != hipSuccess) fail(e, "hipMalloc");
    if (st == PINO_OK && (e = hipMalloc(&m->d_grad, kNParam * sizeof(float))) != hipSuccess) fail(e, "hipMalloc");
    if (st == PINO_OK && (e = hipMalloc(&m->d_partial, nblk * (kNParam + 1) * sizeof(float))) != hipSuccess)
        fail(e, "hipMalloc");
    if (st == PINO_OK &&
        (e = hipMalloc(&m->d_partial2, (size_t)kReduceGroups * (kNParam + 1) * sizeof(float))) != hipSuccess)
        fail(e, "hipMalloc");
    if (st == PINO_OK && (e = hipMalloc(&m->d_pq, kNParam * sizeof(float))) != hipSuccess) fail(e, "hipMalloc");
    if (st == PINO_OK && (e = hipMemcpy(m->d_params, P.data(), kNParam * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
        fail(e, "hipMemcpy");
    if (st == PINO_OK && (e = hipMemset(m->d_m1, 0, kNParam * sizeof(float))) != hipSuccess) fail(e, "hipMemset");
    if (st == PINO_OK && (e = hipMemset(m->d_m2, 0, kNParam * sizeof(float))) != hipSuccess) fail(e, "hipMemset");
    if (st != PINO_OK) {
        pino_mlp_free(m);
        return st;
    }
    *out = m;
    return PINO_OK;
}

pino_status pino_mlp_set_params(pino_mlp* m, const float* host_params)
{
    if (!m || !host_params)
        return PINO_ERR_ARG;
    if (m->broken)
        return PINO_ERR_STATE;
    MLP_HIP(m, hipSetDevice(m->device));
    MLP_HIP(m, hipMemcpy(m->d_params, host_params, pino::kNParam * sizeof(float), hipMemcpyHostToDevice));
    MLP_HIP(m, hipMemset(m->d_m1, 0, pino::kNParam * sizeof(float)));
    MLP_HIP(m, hipMemset(m->d_m2, 0, pino::kNParam * sizeof(float)));
    m->step = 0;
    return PINO_OK;
}

pino_status pino_mlp_get_params(pino_mlp* m, float* host_params)
{
    if (!m || !host_params)
        return PINO_ERR_ARG;
    if (m->broken)
        return PINO_ERR_STATE;
    MLP_HIP(m, hipSetDevice(m->device));
    MLP_HIP(m, hipDeviceSynchronize());
    MLP_HIP(m, hipMemcpy(host_params, m->d_params, pino::kNParam * sizeof(float), hipMemcpyDeviceToHost));
    return PINO_OK;
}

pino_status pino_mlp_forward(pino_mlp* m, const float* x, float* y, int64_t n, void* hip_stream)
{
    if (!m || n < 0 || (n > 0 && (!x || !y)))
        return PINO_ERR_ARG;
    if (m->broken)
        return PINO_ERR_STATE;
    if (n == 0)
        return PINO_OK;
    MLP_HIP(m, hipSetDevice(m->device));
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(pino::k_mlp_forward, dim3((unsigned)((n + 255) / 256)), dim3(256),
                       pino::kNParam * sizeof(float), st, m->d_params, x, y, n);
    MLP_HIP(m, hipGetLastError());
    return PINO_OK;
}

pino_status pino_mlp_grad(pino_mlp* m, const float* x, const float* w, int64_t n, float* grad, float* loss,
                          void* hip_stream)
{
    if (!m || n <= 0 || n > kMlpMaxBatch || !x || !w || !grad) {
        g_mlp_error = "need 0 < n <= 65536 and non-NULL x, w, grad";
        if (m)
            m->err = g_mlp_error;
        return PINO_ERR_ARG;
    }
    if (m->broken)
        return PINO_ERR_STATE;
    MLP_HIP(m, hipSetDevice(m->device));
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int nblk = (int)((n + pino::kTB - 1) / pino::kTB);
    if (m->bf16_fwd) {
        hipLaunchKernelGGL(pino::k_mlp_round_bf16, dim3((pino::kNParam + 255) / 256), dim3(256), 0, st, m->d_params,
                           m->d_pq);
        MLP_HIP(m, hipGetLastError());
    }
    hipLaunchKernelGGL(pino::k_mlp_grad_block, dim3(nblk), dim3(pino::kGradThreads), pino::mlp_grad_lds_bytes(), st,
                       m->d_params, m->bf16_fwd ? m->d_pq : m->d_params, m->bf16_fwd, x, w, n, m->d_partial);
    MLP_HIP(m, hipGetLastError());
    const unsigned cols = (unsigned)((pino::kNParam + 1 + 255) / 256);
    hipLaunchKernelGGL(pino::k_mlp_reduce_groups, dim3(cols, pino::kReduceGroups), dim3(256), 0, st, m->d_partial,
                       nblk, m->d_partial2);
    MLP_HIP(m, hipGetLastError());
    hipLaunchKernelGGL(pino::k_mlp_reduce, dim3(cols), dim3(256), 0, st, m->d_partial2, n, grad, loss);
    MLP_HIP(m, hipGetLastError());
    return PINO_OK;
}

pino_status pino_mlp_set_bf16_forward(pino_mlp* m, int32_t on)
{
    if (!m || (on != 0 && on != 1))
        return PINO_ERR_ARG;
    m->bf16_fwd = on;
    return PINO_OK;
}

pino_status pino_mlp_adam(pino_mlp* m, const float* grad, float lr, float beta1, float beta2, float eps,
                          void* hip_stream)
{
    if (!m || !grad || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return PINO_ERR_ARG;
    if (m->broken)
        return PINO_ERR_STATE;
    MLP_HIP(m, hipSetDevice(m->device));
    m->step += 1;
    const float c1 = 1.0f - (float)std::pow((double)beta1, (double)m->step);
    const float c2 = 1.0f - (float)std::pow((double)beta2, (double)m->step);
    hipLaunchKernelGGL(pino::k_mlp_adam, dim3((pino::kNParam + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), m->d_params, m->d_m1, m->d_m2, grad, lr, beta1, beta2,
                       eps, c1, c2);
    MLP_HIP(m, hipGetLastError());
    return PINO_OK;
}

pino_status pino_mlp_train_step(pino_mlp* m, const float* x, const float* w, int64_t n, float lr, float* loss,
                                void* hip_stream)
{
    pino_status s = pino_mlp_grad(m, x, w, n, m ? m->d_grad : nullptr, loss, hip_stream);
    if (s != PINO_OK)
        return s;
    return pino_mlp_adam(m, m->d_grad, lr, 0.9f, 0.999f, 1e-8f, hip_stream);
}

pino_status pino_mlp_export(pino_mlp* m, void* blob, int64_t bytes, int64_t* needed)
{
    if (!m)
        return PINO_ERR_ARG;
    if (needed)
        *needed = kMlpBlobBytes;
    if (!blob)
        return PINO_OK;
    if (bytes < kMlpBlobBytes)
        return PINO_ERR_ARG;
    std::vector<float> P(pino::kNParam);
    const pino_status s = pino_mlp_get_params(m, P.data());
    if (s != PINO_OK)
        return s;
    MlpBlobHeader h;
    std::memcpy(h.magic, kMlpMagic, 8);
    h.version = 1;
    h.n_params = pino::kNParam;
    std::memcpy(blob, &h, sizeof(h));
    std::memcpy(static_cast<char*>(blob) + sizeof(h), P.data(), P.size() * sizeof(float));
    return PINO_OK;
}

pino_status pino_mlp_free(pino_mlp* m)
{
    if (!m)
        return PINO_OK;
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    float* ptrs[] = {m->d_params, m->d_m1, m->d_m2, m->d_grad, m->d_partial, m->d_partial2, m->d_pq};
    for (float* p : ptrs)
        if (p)
            (void)hipFree(p);
    delete m;
    return PINO_OK;
}

}  // extern "C"
