// Learned surrogate of the Classic collapse: network inputs, FP32 training
// kernels (forward, backward, Adam), the BF16 MFMA inference used by the
// collapse kernel, and the FP64 Newton certificate.
#pragma once

#include "device_collapse.h"

namespace pino {

// ---------------------------------------------------------------------------
// Parameter layout (FP32): W1[64][4], b1[64], W2[64][64], b2[64],
// W3[64][64], b3[64], W4[64], b4.
// ---------------------------------------------------------------------------
constexpr int kH = 64;
constexpr int kIn = 4;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH * kIn;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kH * kH;
constexpr int kOffW4 = kOffB3 + kH;
constexpr int kOffB4 = kOffW4 + kH;
constexpr int kNParam = kOffB4 + 1;  // 8705

// FP32 -> BF16 bits, round to nearest even (finite inputs)
__host__ __device__ __forceinline__ short bf16_bits(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__host__ __device__ __forceinline__ float bf16_value(short b)
{
    return __builtin_bit_cast(float, (uint32_t)(uint16_t)b << 16);
}

// the network is consulted only where l1 >= kGate * max|l| (and l1 > 0)
constexpr double kGate = 0.1;

// Network inputs from l1, s = l2 + l3, pp = l2 l3: sorted eigenvalues over
// sigma and the centred matter density.  Returns whether the network is
// consulted (l1 > 0 and l1 >= kGate * |l3|, l3 the smallest eigenvalue).
__host__ __device__ __forceinline__ bool net_inputs(double l1, double s, double pp, double sigma, double omega_m,
                                                    float x[4])
{
    const double disc = fmax(0.25 * s * s - pp, 0.0);
    const double rt = sqrt(disc);
    const double l2 = 0.5 * s + rt;
    const double l3 = 0.5 * s - rt;
    const double is = 1.0 / sigma;
    x[0] = (float)(l1 * is);
    x[1] = (float)(l2 * is);
    x[2] = (float)(l3 * is);
    x[3] = (float)((omega_m - 0.3) * 20.0);
    return l1 > 0.0 && l1 >= kGate * fabs(l3);
}

// ---------------------------------------------------------------------------
// FP32 training kernels.  A block takes kTB samples (one per lane) and
// kWaves waves; wave q owns hidden units [q kUw, (q + 1) kUw) of every layer,
// so the weight rows it reads are wave-uniform (scalar loads) while the
// activations and back-propagated errors of the block's samples sit in LDS
// as [unit][sample].  The weight gradients, sums over the block's samples,
// are spread over all threads and written as a per-block partial that
// k_mlp_reduce_groups and k_mlp_reduce sum in a fixed order
// (deterministic).
// ---------------------------------------------------------------------------
constexpr int kTB = 64;                 // samples per block
constexpr int kWaves = 8;               // waves per block
constexpr int kGradThreads = kTB * kWaves;
constexpr int kUw = kH / kWaves;        // hidden units per wave
constexpr int kLd = kTB + 1;            // padded row stride of [unit][sample] arrays

__host__ __device__ inline size_t mlp_grad_lds_bytes()
{
    return sizeof(float) * ((size_t)6 * kH * kLd + kIn * kLd + 2 * kTB);
}

// out[u] = b[u0 + u] + sum_k W[(u0 + u) * K + k] in[k][s], u < kUw
template <int K>
__device__ __forceinline__ void dense_rows(const float* __restrict__ W, const float* __restrict__ b, int u0,
                                           const float* in, int s, float out[kUw])
{
#pragma unroll
    for (int u = 0; u < kUw; ++u)
        out[u] = b[u0 + u];
#pragma unroll 8
    for (int k = 0; k < K; ++k) {
        const float v = in[k * kLd + s];
#pragma unroll
        for (int u = 0; u < kUw; ++u)
            out[u] = fmaf(W[(u0 + u) * K + k], v, out[u]);
    }
}

// out[u] = sum_o W[o * kH + u0 + u] d[o][s]: the transposed product of the
// backward pass
__device__ __forceinline__ void dense_cols(const float* __restrict__ W, int u0, const float* d, int s,
                                           float out[kUw])
{
#pragma unroll
    for (int u = 0; u < kUw; ++u)
        out[u] = 0.0f;
#pragma unroll 8
    for (int o = 0; o < kH; ++o) {
        const float v = d[o * kLd + s];
#pragma unroll
        for (int u = 0; u < kUw; ++u)
            out[u] = fmaf(W[o * kH + u0 + u], v, out[u]);
    }
}

// pq: the parameters whose W2 and W3 the hidden layers use (the BF16-rounded
// copy when bf16, else p itself).  bf16 applies the surrogate's BF16
// rounding rule, which the inference network below follows too: the weights
// of the two 64 x 64 layers and the inputs of those layers and of the output
// layer (the ReLU outputs of layers 1, 2 and 3) rounded to BF16 (nearest,
// ties to even); layer 1, the output layer's weights and the biases in FP32.
// The backward pass uses the same weights and stored activations and treats
// the rounding as the identity (straight-through).
__global__ void __launch_bounds__(kGradThreads) k_mlp_grad_block(const float* __restrict__ p,
                                                                const float* __restrict__ pq, int bf16,
                                                                const float* __restrict__ X,
                                                                const float* __restrict__ Wt, int64_t n,
                                                                float* __restrict__ partial)
{
    extern __shared__ float sm[];
    float* h1 = sm;
    float* h2 = h1 + kH * kLd;
    float* h3 = h2 + kH * kLd;
    float* d1 = h3 + kH * kLd;
    float* d2 = d1 + kH * kLd;
    float* d3 = d2 + kH * kLd;
    float* xs = d3 + kH * kLd;
    float* dys = xs + kIn * kLd;
    float* ls = dys + kTB;
    const int tid = threadIdx.x;
    const int s = tid % kTB;
    const int u0 = __builtin_amdgcn_readfirstlane(tid / kTB) * kUw;
    const int64_t smp = (int64_t)blockIdx.x * kTB + s;
    const bool valid = smp < n;
    if (tid < kTB)
        for (int k = 0; k < kIn; ++k)
            xs[k * kLd + s] = valid ? X[smp * kIn + k] : 0.0f;
    __syncthreads();
    float z[kUw];
    // forward
    dense_rows<kIn>(p + kOffW1, p + kOffB1, u0, xs, s, z);
#pragma unroll
    for (int u = 0; u < kUw; ++u) {
        const float hv = fmaxf(z[u], 0.0f);
        h1[(u0 + u) * kLd + s] = bf16 ? bf16_value(bf16_bits(hv)) : hv;
    }
    __syncthreads();
    dense_rows<kH>(pq + kOffW2, p + kOffB2, u0, h1, s, z);
#pragma unroll
    for (int u = 0; u < kUw; ++u) {
        const float hv = fmaxf(z[u], 0.0f);
        h2[(u0 + u) * kLd + s] = bf16 ? bf16_value(bf16_bits(hv)) : hv;
    }
    __syncthreads();
    dense_rows<kH>(pq + kOffW3, p + kOffB3, u0, h2, s, z);
    float yp = 0.0f;  // this wave's share of the output
#pragma unroll
    for (int u = 0; u < kUw; ++u) {
        const float hr = fmaxf(z[u], 0.0f);
        const float hv = bf16 ? bf16_value(bf16_bits(hr)) : hr;
        h3[(u0 + u) * kLd + s] = hv;
        yp = fmaf(p[kOffW4 + u0 + u], hv, yp);
    }
    d1[(u0 / kUw) * kLd + s] = yp;  // d1 is free until the last layer of the backward pass
    __syncthreads();
    if (tid < kTB) {
        float y = p[kOffB4];
        for (int q = 0; q < kWaves; ++q)
            y += d1[q * kLd + s];
        // loss ((y - w)/w)^2 averaged over all n samples; dL/dy
        const float w = valid ? Wt[smp] : 0.0f;
        const bool use = valid && w > 0.0f;
        const float r = use ? (y - w) / w : 0.0f;
        dys[s] = use ? 2.0f * r / (w * (float)n) : 0.0f;
        ls[s] = r * r;
    }
    __syncthreads();
    // backward through the hidden layers, per sample
    const float dy = dys[s];
#pragma unroll
    for (int u = 0; u < kUw; ++u)
        d3[(u0 + u) * kLd + s] = h3[(u0 + u) * kLd + s] > 0.0f ? dy * p[kOffW4 + u0 + u] : 0.0f;
    __syncthreads();
    dense_cols(pq + kOffW3, u0, d3, s, z);
#pragma unroll
    for (int u = 0; u < kUw; ++u)
        d2[(u0 + u) * kLd + s] = h2[(u0 + u) * kLd + s] > 0.0f ? z[u] : 0.0f;
    __syncthreads();
    dense_cols(pq + kOffW2, u0, d2, s, z);
#pragma unroll
    for (int u = 0; u < kUw; ++u)
        d1[(u0 + u) * kLd + s] = h1[(u0 + u) * kLd + s] > 0.0f ? z[u] : 0.0f;
    __syncthreads();
    // weight gradients of W2 and W3: thread -> rows 2i, 2i + 1 and columns
    // c, c + 16, c + 32, c + 48 (conflict-free LDS rows across a half-wave)
    float* out = partial + (int64_t)blockIdx.x * (kNParam + 1);
    {
        const int r0 = 2 * (tid / 16);
        const int c0 = tid % 16;
        float g2[2][4] = {}, g3[2][4] = {};
#pragma unroll 4
        for (int t = 0; t < kTB; ++t) {
            const float a2[2] = {d2[r0 * kLd + t], d2[(r0 + 1) * kLd + t]};
            const float a3[2] = {d3[r0 * kLd + t], d3[(r0 + 1) * kLd + t]};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float v1 = h1[(c0 + 16 * j) * kLd + t];
                const float v2 = h2[(c0 + 16 * j) * kLd + t];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    g2[i][j] = fmaf(a2[i], v1, g2[i][j]);
                    g3[i][j] = fmaf(a3[i], v2, g3[i][j]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                out[kOffW2 + (r0 + i) * kH + c0 + 16 * j] = g2[i][j];
                out[kOffW3 + (r0 + i) * kH + c0 + 16 * j] = g3[i][j];
            }
    }
    // W1 (threads 0..255) and b1, b2, b3, W4 (threads 256..511)
    if (tid < kH * kIn) {
        const int o = tid / kIn, k = tid % kIn;
        float g = 0.0f;
        for (int t = 0; t < kTB; ++t)
            g = fmaf(d1[o * kLd + t], xs[k * kLd + t], g);
        out[kOffW1 + o * kIn + k] = g;
    } else {
        const int which = (tid - kH * kIn) / kH, o = (tid - kH * kIn) % kH;
        float g = 0.0f;
        if (which == 3) {
            for (int t = 0; t < kTB; ++t)
                g = fmaf(dys[t], h3[o * kLd + t], g);
            out[kOffW4 + o] = g;
        } else {
            const float* d = which == 0 ? d1 : which == 1 ? d2 : d3;
            for (int t = 0; t < kTB; ++t)
                g += d[o * kLd + t];
            out[(which == 0 ? kOffB1 : which == 1 ? kOffB2 : kOffB3) + o] = g;
        }
    }
    if (tid == 0) {
        float gb4 = 0.0f, lsum = 0.0f;
        for (int t = 0; t < kTB; ++t) {
            gb4 += dys[t];
            lsum += ls[t];
        }
        out[kOffB4] = gb4;
        out[kNParam] = lsum;
    }
}

// Deterministic two-level sum of the per-block partials: group g (blockIdx.y)
// adds blocks g, g + groups, g + 2 groups, ... in that order into
// partial2[g][j]; k_mlp_reduce then adds the groups in order.  The summation
// tree depends only on the number of blocks.
constexpr int kReduceGroups = 32;

__global__ void __launch_bounds__(256) k_mlp_reduce_groups(const float* __restrict__ partial, int nblk,
                                                          float* __restrict__ partial2)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    if (j > kNParam)
        return;
    float s = 0.0f;
    for (int b = g; b < nblk; b += kReduceGroups)
        s += partial[(int64_t)b * (kNParam + 1) + j];
    partial2[(int64_t)g * (kNParam + 1) + j] = s;
}

// grad[j] = sum over groups of partial2[g][j] (fixed order); loss likewise / n
__global__ void __launch_bounds__(256) k_mlp_reduce(const float* __restrict__ partial2, int64_t n,
                                                   float* __restrict__ grad, float* __restrict__ loss)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > kNParam)
        return;
    float s = 0.0f;
    for (int g = 0; g < kReduceGroups; ++g)
        s += partial2[(int64_t)g * (kNParam + 1) + j];
    if (j < kNParam)
        grad[j] = s;
    else if (loss)
        *loss = s / (float)n;
}

// q[j] = P[j] rounded to BF16 (nearest even), as FP32
__global__ void __launch_bounds__(256) k_mlp_round_bf16(const float* __restrict__ P, float* __restrict__ q)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < kNParam)
        q[j] = bf16_value(bf16_bits(P[j]));
}

__global__ void __launch_bounds__(256) k_mlp_adam(float* __restrict__ P, float* __restrict__ m1,
                                                 float* __restrict__ m2, const float* __restrict__ g, float lr,
                                                 float b1, float b2, float eps, float c1, float c2)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kNParam)
        return;
    const float gj = g[j];
    const float a = b1 * m1[j] + (1.0f - b1) * gj;
    const float v = b2 * m2[j] + (1.0f - b2) * gj * gj;
    m1[j] = a;
    m2[j] = v;
    P[j] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// FP32 inference, one sample per lane, parameters in LDS
__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ P, const float* __restrict__ X,
                                                    float* __restrict__ Y, int64_t n)
{
    extern __shared__ float p[];
    for (int k = threadIdx.x; k < kNParam; k += blockDim.x)
        p[k] = P[k];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    // activations in registers: every array index is a compile-time constant
    float a[kH], b[kH];
    float x[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k)
        x[k] = X[i * kIn + k];
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        float z = p[kOffB1 + o];
#pragma unroll
        for (int k = 0; k < kIn; ++k)
            z += p[kOffW1 + o * kIn + k] * x[k];
        a[o] = fmaxf(z, 0.0f);
    }
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        float z = p[kOffB2 + o];
#pragma unroll
        for (int k = 0; k < kH; ++k)
            z += p[kOffW2 + o * kH + k] * a[k];
        b[o] = fmaxf(z, 0.0f);
    }
    float y = p[kOffB4];
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        float z = p[kOffB3 + o];
#pragma unroll
        for (int k = 0; k < kH; ++k)
            z += p[kOffW3 + o * kH + k] * b[k];
        y += p[kOffW4 + o] * fmaxf(z, 0.0f);
    }
    Y[i] = y;
}

// ---------------------------------------------------------------------------
// BF16 MFMA inference with v_mfma_f32_16x16x32_bf16: lane l (g = l/16,
// q = l%16) holds A[i = q][k = 8g + j] and B[k = 8g + j][n = q], j = 0..7, and
// receives D[i = 4g + j][n = q], j = 0..3.  Weights are A (rows = 16 output
// neurons of tile mt), activations B (columns = the 16 particles of group nt).
// A layer's output tiles mt = 2kt and 2kt + 1 hold, in lane (g, q), neurons
// 32kt + 4g + j and 32kt + 16 + 4g + j of particle q: together, the 8 values
// the lane supplies as B of the next layer's K tile kt, once the next layer's
// weight columns are permuted to match (done when the fragments are built).
// So the network stays in registers; the FP32 -> BF16 step is the hardware
// packed convert (round to nearest even).  Rounding rule: the weights of the
// two 64 x 64 layers and the inputs of those layers and of the output layer
// are BF16; layer 1 and the output layer's weights carry FP32 accuracy as
// BF16 high + low pairs; biases and accumulation are FP32.
// ---------------------------------------------------------------------------
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Layer 1 has K = 4 inputs in a K = 32 tile: lanes of group 0 carry
// (x_hi, x_lo) against (W_hi, W_hi), group 1 carries (x_hi, 0) against
// (W_lo, 0), groups 2 and 3 are zero, so the first layer is accurate to
// ~2^-16 although its operands are BF16.
struct NetFrags {
    s16x8 w1[4][64];     // [mt][lane], BF16 bits
    s16x8 w2[4][2][64];  // [mt][kt][lane]
    s16x8 w3[4][2][64];
    s16x8 w4h[2][64];    // [kt][lane]: W4 (BF16 high part) as an MFMA A operand, every row the same
    s16x8 w4l[2][64];    // the low part (W4 - high), so the output weights are ~FP32-accurate
    float b1[kH], b2[kH], b3[kH];
    float b4;
    float pad[3];
};

static_assert(sizeof(NetFrags) % 16 == 0, "NetFrags is staged into LDS in 16-byte pieces");

// Input neuron of K tile kt carried at slot j of lane group g (see above).
__host__ __device__ __forceinline__ int k32_neuron(int kt, int g, int j)
{
    return 32 * kt + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
}


typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16, round to nearest even, two values per packed convert (a
// four-wide conversion is split into one convert per value plus a permute)
__device__ __forceinline__ bf16x4 to_bf16(f32x4 v)
{
    const bf16x2 a = __builtin_convertvector(f32x2{v[0], v[1]}, bf16x2);
    const bf16x2 b = __builtin_convertvector(f32x2{v[2], v[3]}, bf16x2);
    return __builtin_shufflevector(a, b, 0, 1, 2, 3);
}

__device__ __forceinline__ f32x4 relu4(f32x4 v)
{
    return f32x4{fmaxf(v[0], 0.0f), fmaxf(v[1], 0.0f), fmaxf(v[2], 0.0f), fmaxf(v[3], 0.0f)};
}

__device__ __forceinline__ bf16x8 join(bf16x4 a, bf16x4 b)
{
    return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
}

__device__ __forceinline__ f32x4 bias4(const float* b, int mt, int g)
{
    return *reinterpret_cast<const f32x4*>(b + 16 * mt + 4 * g);
}

__device__ __forceinline__ bf16x8 frag(const s16x8& w)
{
    return __builtin_bit_cast(bf16x8, w);
}

// ReLU and BF16 packing of two output tiles.  The ReLU is applied to the
// rounded values as a packed signed 16-bit max with 0: a negative BF16 (or
// -0) has its sign bit set, so exactly those become +0, which is what
// rounding after the FP32 ReLU gives.
__device__ __forceinline__ s16x2 relu_bf16x2(float a, float b)
{
    const s16x2 v = __builtin_bit_cast(s16x2, __builtin_convertvector(f32x2{a, b}, bf16x2));
    return __builtin_elementwise_max(v, s16x2{0, 0});
}

__device__ __forceinline__ bf16x8 pack_pair(f32x4 a, f32x4 b)
{
    const s16x2 p0 = relu_bf16x2(a[0], a[1]), p1 = relu_bf16x2(a[2], a[3]);
    const s16x2 p2 = relu_bf16x2(b[0], b[1]), p3 = relu_bf16x2(b[2], b[3]);
    const s16x8 v = __builtin_shufflevector(__builtin_shufflevector(p0, p1, 0, 1, 2, 3),
                                            __builtin_shufflevector(p2, p3, 0, 1, 2, 3), 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_bit_cast(bf16x8, v);
}

#ifndef PINO_NET_GROUPS
#define PINO_NET_GROUPS 2
#endif

// Network output for this lane's particle (all 64 lanes of the wave must
// call it together; x of inactive lanes may be anything finite).  The four
// 16-particle groups of the wave go through the layers two at a time: each
// weight fragment read from LDS feeds two independent MFMA chains, which
// hides the MFMA latency without the register cost of four.
__device__ __forceinline__ float net_bf16(const NetFrags& N, const float x[4])
{
    constexpr int G = PINO_NET_GROUPS;  // groups per pass
    const int l = threadIdx.x & 63;
    const int q = l & 15;
    const int g = l >> 4;
    const bf16x4 zero4 = to_bf16(f32x4{0.0f, 0.0f, 0.0f, 0.0f});
    float out = 0.0f;
    for (int p = 0; p < 4; p += G) {
        bf16x8 hb[G][2];
        f32x4 acc[G][4];
        {
            bf16x8 bx[G];
            for (int e = 0; e < G; ++e) {
                const int src = 16 * (p + e) + q;
                const f32x4 f{__shfl(x[0], src, 64), __shfl(x[1], src, 64), __shfl(x[2], src, 64),
                              __shfl(x[3], src, 64)};
                const bf16x4 hi = to_bf16(f);
                const bf16x4 lo = to_bf16(f - __builtin_convertvector(hi, f32x4));
                bx[e] = join(g <= 1 ? hi : zero4, g == 0 ? lo : zero4);
            }
            for (int mt = 0; mt < 4; ++mt) {
                const bf16x8 w = frag(N.w1[mt][l]);
                const f32x4 b = bias4(N.b1, mt, g);
                for (int e = 0; e < G; ++e)
                    acc[e][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, bx[e], b, 0, 0, 0);
            }
        }
        for (int e = 0; e < G; ++e)
            for (int kt = 0; kt < 2; ++kt)
                hb[e][kt] = pack_pair(acc[e][2 * kt], acc[e][2 * kt + 1]);
        for (int mt = 0; mt < 4; ++mt) {
            const f32x4 b = bias4(N.b2, mt, g);
            const bf16x8 w0 = frag(N.w2[mt][0][l]);
            const bf16x8 w1 = frag(N.w2[mt][1][l]);
            for (int e = 0; e < G; ++e) {
                const f32x4 t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0, hb[e][0], b, 0, 0, 0);
                acc[e][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, hb[e][1], t, 0, 0, 0);
            }
        }
        for (int e = 0; e < G; ++e)
            for (int kt = 0; kt < 2; ++kt)
                hb[e][kt] = pack_pair(acc[e][2 * kt], acc[e][2 * kt + 1]);
        for (int mt = 0; mt < 4; ++mt) {
            const f32x4 b = bias4(N.b3, mt, g);
            const bf16x8 w0 = frag(N.w3[mt][0][l]);
            const bf16x8 w1 = frag(N.w3[mt][1][l]);
            for (int e = 0; e < G; ++e) {
                const f32x4 t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0, hb[e][0], b, 0, 0, 0);
                acc[e][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, hb[e][1], t, 0, 0, 0);
            }
        }
        // output layer on the matrix cores: layer 3's ReLU outputs packed to
        // BF16 as the B operand, and an A operand holding W4 (BF16 high and
        // low parts) in every row, so every row of D is the particle's
        // output and the lanes of group p + e take it from their own column
        for (int e = 0; e < G; ++e)
            for (int kt = 0; kt < 2; ++kt)
                hb[e][kt] = pack_pair(acc[e][2 * kt], acc[e][2 * kt + 1]);
        for (int e = 0; e < G; ++e) {
            f32x4 o{N.b4, N.b4, N.b4, N.b4};
            for (int kt = 0; kt < 2; ++kt) {
                o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag(N.w4h[kt][l]), hb[e][kt], o, 0, 0, 0);
                o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag(N.w4l[kt][l]), hb[e][kt], o, 0, 0, 0);
            }
            if (g == p + e)
                out = o[0];
        }
    }
    return out;
}

// ---------------------------------------------------------------------------
// Certificate.  From the prediction u0 = 1/y (u = l1 D), one FP64 Newton
// step u1 = u0 - g(u0)/g'(u0).  u1 is accepted as the collapse when the
// smallest positive root of g provably lies in [lo, hi] = u1 (1 -/+ rtol):
//   (i)   g(lo) > e and g(hi) < -e, with e a bound on the rounding error of
//         the evaluation of g (so g changes sign downward inside [lo, hi]);
//   (ii)  g has no local minimum with g <= 0 below lo.  g(0) = 1 and
//         g'(0) = -1, so the first positive critical point of g,
//         u_m = 1/(b + sqrt(b^2 + 3c)), is a local minimum; if g(u_m) > 0 or
//         u_m >= lo, g stays positive on (0, lo] (after u_m, g rises to its
//         local maximum and then falls monotonically to g(lo) > 0).
// Together (i) and (ii) put the first crossing within rtol of u1, whatever
// the prediction was; a prediction near another root is rejected by (ii).
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ double g_bound(const CubicU& k, double u)
{
    // 8 ulp of the sum of the magnitudes of the Horner terms
    return 8.0 * 1.1102230246251565e-16 * (1.0 + u * (1.0 + u * (fabs(k.b) + fabs(k.c) * u)));
}

__host__ __device__ __forceinline__ bool certify(const CubicU& k, double y, double rtol, double& u1)
{
    if (!(y > 0.0) || !isfinite(y))
        return false;
    const double u0 = rcp2(y);
    const double g0 = g_u(k, u0);
    const double d0 = -1.0 + u0 * (2.0 * k.b + 3.0 * k.c * u0);
    u1 = u0 - g0 * rcp2(d0);
    const double lo = u1 * (1.0 - rtol);
    const double hi = u1 * (1.0 + rtol);
    const bool bracket = g_u(k, lo) > g_bound(k, lo) && g_u(k, hi) < -g_bound(k, hi);
    const double disc = k.b * k.b + 3.0 * k.c;
    const double den = k.b + sqrt(fmax(disc, 0.0));
    bool earlier = false;
    if (disc >= 0.0 && den > 0.0) {
        const double um = rcp2(den);
        earlier = um < lo && g_u(k, um) <= 0.0;
    }
    return lo > 0.0 && bracket && !earlier && isfinite(u1);
}

}  // namespace pino
