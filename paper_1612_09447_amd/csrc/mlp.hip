// Start-vector network for the learned form: a multilayer perceptron
// 32 -> 64 -> 64 -> 16 (SiLU hidden activations, linear output) trained online
// with mean-squared error and Adam. Sec. IV of the paper builds CG start
// vectors from a POD basis of earlier solutions; here the small reduced solve
// is replaced by this learned map, and CG stays the judge of the result.
//
// One workgroup of 256 threads runs a whole minibatch (B <= 64): forward,
// loss, backward and the Adam update, all in one launch with the matmul
// weights and the activations in LDS.
// Matmul operands are rounded to bfloat16 (round to nearest even) in BF16
// mode, products accumulate in FP32; master weights, gradients and Adam
// moments are FP32. Every sum runs in a fixed order, so results are
// deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "eqs_internal.h"

namespace eqs {

constexpr int kIn = 32, kH = 64, kOut = 16, kMaxB = 64;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kOut * kH, kNParam = oB3 + kOut;
static_assert(kNParam == 7312, "parameter layout");

__device__ __forceinline__ float bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return x;  // inf / nan unchanged
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    return __uint_as_float(u);
}

template <bool BF16>
__device__ __forceinline__ float q(float x) {
    return BF16 ? bf16_round(x) : x;
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

struct MlpState {
    float lr, beta1, beta2, eps;
    int32_t step;  // Adam steps taken
    float loss;    // loss of the last training batch
};

// wq: matmul copies of the weights (bf16-rounded in BF16 mode); master: FP32.
// The matmul weights and every activation of the minibatch live in LDS (about
// 104 KiB of gfx950's 160 KiB): the SiLU of each pre-activation is evaluated
// once (its bfloat16 rounding where it is read as a matmul operand), and every
// sum runs in the same fixed order over k or over the batch.
template <bool TRAIN, bool BF16>
__global__ __launch_bounds__(256) void k_mlp(const float* __restrict__ x, const float* __restrict__ tgt, float* __restrict__ y,
                                             int32_t B, float* __restrict__ master, float* __restrict__ wq,
                                             float* __restrict__ grad, float* __restrict__ m1, float* __restrict__ m2,
                                             MlpState* __restrict__ st) {
    __shared__ float sw1[kH * kIn], sw2[kH * kH], sw3[kOut * kH];  // matmul weights
    __shared__ float sb[kH + kH + kOut];                              // biases (master)
    __shared__ float sx[kMaxB * kIn];
    __shared__ float sh1[kMaxB * kH], sa1[kMaxB * kH];  // pre-activation, activation
    __shared__ float sh2[kMaxB * kH], sa2[kMaxB * kH];
    __shared__ float sy[kMaxB * kOut];
    __shared__ float sred[256];
    const int tid = threadIdx.x;

    for (int i = tid; i < kH * kIn; i += 256) sw1[i] = wq[oW1 + i];
    for (int i = tid; i < kH * kH; i += 256) sw2[i] = wq[oW2 + i];
    for (int i = tid; i < kOut * kH; i += 256) sw3[i] = wq[oW3 + i];
    for (int i = tid; i < kH; i += 256) {
        sb[i] = master[oB1 + i];
        sb[kH + i] = master[oB2 + i];
    }
    for (int i = tid; i < kOut; i += 256) sb[2 * kH + i] = master[oB3 + i];
    for (int i = tid; i < B * kIn; i += 256) sx[i] = x[i];
    __syncthreads();
    // h1 = W1 x + b1, a1 = silu(h1)
    for (int i = tid; i < B * kH; i += 256) {
        const int b = i / kH, o = i % kH;
        float acc = 0.0f;
        for (int k = 0; k < kIn; ++k) acc += sw1[o * kIn + k] * q<BF16>(sx[b * kIn + k]);
        const float h = acc + sb[o];
        sh1[i] = h;
        sa1[i] = silu(h);
    }
    __syncthreads();
    // h2 = W2 a1 + b2, a2 = silu(h2)
    for (int i = tid; i < B * kH; i += 256) {
        const int b = i / kH, o = i % kH;
        float acc = 0.0f;
        for (int k = 0; k < kH; ++k) acc += sw2[o * kH + k] * q<BF16>(sa1[b * kH + k]);
        const float h = acc + sb[kH + o];
        sh2[i] = h;
        sa2[i] = silu(h);
    }
    __syncthreads();
    // y = W3 a2 + b3
    for (int i = tid; i < B * kOut; i += 256) {
        const int b = i / kOut, o = i % kOut;
        float acc = 0.0f;
        for (int k = 0; k < kH; ++k) acc += sw3[o * kH + k] * q<BF16>(sa2[b * kH + k]);
        sy[i] = acc + sb[2 * kH + o];
    }
    __syncthreads();
    if (!TRAIN) {
        for (int i = tid; i < B * kOut; i += 256) y[i] = sy[i];
        return;
    }

    // loss and dy = 2 (y - t) / (B * 16), in place of y
    float part = 0.0f;
    const float inv = 1.0f / (float)(B * kOut);
    for (int i = tid; i < B * kOut; i += 256) {
        const float d = sy[i] - tgt[i];
        part += d * d;
    }
    sred[tid] = part;
    __syncthreads();
    for (int i = tid; i < B * kOut; i += 256) sy[i] = 2.0f * (sy[i] - tgt[i]) * inv;
    if (tid == 0) {
        float s = 0.0f;
        for (int k = 0; k < 256; ++k) s += sred[k];
        st->loss = s * inv;
    }
    __syncthreads();

    // layer 3: gW3 = dy^T a2, gb3 = sum_b dy
    for (int i = tid; i < kOut * kH; i += 256) {
        const int o = i / kH, k = i % kH;
        float acc = 0.0f;
        for (int b = 0; b < B; ++b) acc += q<BF16>(sy[b * kOut + o]) * q<BF16>(sa2[b * kH + k]);
        grad[oW3 + i] = acc;
    }
    for (int o = tid; o < kOut; o += 256) {
        float acc = 0.0f;
        for (int b = 0; b < B; ++b) acc += sy[b * kOut + o];
        grad[oB3 + o] = acc;
    }
    __syncthreads();
    // dh2 = (dy W3) * silu'(h2), written over h2 (each thread reads its own h2 first)
    for (int i = tid; i < B * kH; i += 256) {
        const int b = i / kH, k = i % kH;
        float acc = 0.0f;
        for (int o = 0; o < kOut; ++o) acc += q<BF16>(sy[b * kOut + o]) * sw3[o * kH + k];
        sh2[i] = acc * silu_grad(sh2[i]);
    }
    __syncthreads();
    // layer 2: gW2 = dh2^T a1, gb2 = sum_b dh2
    for (int i = tid; i < kH * kH; i += 256) {
        const int o = i / kH, k = i % kH;
        float acc = 0.0f;
        for (int b = 0; b < B; ++b) acc += q<BF16>(sh2[b * kH + o]) * q<BF16>(sa1[b * kH + k]);
        grad[oW2 + i] = acc;
    }
    for (int o = tid; o < kH; o += 256) {
        float acc = 0.0f;
        for (int b = 0; b < B; ++b) acc += sh2[b * kH + o];
        grad[oB2 + o] = acc;
    }
    __syncthreads();
    // dh1 = (dh2 W2) * silu'(h1), over h1
    for (int i = tid; i < B * kH; i += 256) {
        const int b = i / kH, k = i % kH;
        float acc = 0.0f;
        for (int o = 0; o < kH; ++o) acc += q<BF16>(sh2[b * kH + o]) * sw2[o * kH + k];
        sh1[i] = acc * silu_grad(sh1[i]);
    }
    __syncthreads();
    // layer 1: gW1 = dh1^T x, gb1 = sum_b dh1
    for (int i = tid; i < kH * kIn; i += 256) {
        const int o = i / kIn, k = i % kIn;
        float acc = 0.0f;
        for (int b = 0; b < B; ++b) acc += q<BF16>(sh1[b * kH + o]) * q<BF16>(sx[b * kIn + k]);
        grad[oW1 + i] = acc;
    }
    for (int o = tid; o < kH; o += 256) {
        float acc = 0.0f;
        for (int b = 0; b < B; ++b) acc += sh1[b * kH + o];
        grad[oB1 + o] = acc;
    }
    __syncthreads();

    // Adam (Kingma & Ba): bias-corrected first and second moments
    const int t = st->step + 1;
    const float bc1 = 1.0f - powf(st->beta1, (float)t);
    const float bc2 = 1.0f - powf(st->beta2, (float)t);
    for (int i = tid; i < kNParam; i += 256) {
        const float g = grad[i];
        const float a = st->beta1 * m1[i] + (1.0f - st->beta1) * g;
        const float v = st->beta2 * m2[i] + (1.0f - st->beta2) * g * g;
        m1[i] = a;
        m2[i] = v;
        const float w = master[i] - st->lr * (a / bc1) / (sqrtf(v / bc2) + st->eps);
        master[i] = w;
        wq[i] = q<BF16>(w);
    }
    __syncthreads();
    if (tid == 0) st->step = t;
}

// Inference for one feature vector, followed by the map from the network's
// 16 outputs to the 16 snapshot coefficients of the start vector:
// alpha = bias + P y (P carries the POD basis change and the output scale).
// With a guard block g (K = V^T M V [16 x 16], d = V^T (r_j - r_{j-1}) [16],
// scale s) the correction c = s y is kept only if it lowers the M-norm of the
// error of the start vector: |x* - x0 - V c|_M^2 = |x* - x0|_M^2 - (2 c.d -
// c.K c) when M x0 = r_{j-1}, so the test needs no product with M; otherwise
// alpha = bias. stat[0] / stat[1] count kept / dropped corrections.
struct MlpIn {
    float x[kIn];
    double P[kOut * kOut];
    double bias[kOut];
};

template <bool BF16>
__global__ __launch_bounds__(64) void k_mlp_alpha(MlpIn in, const float* __restrict__ master,
                                                   const float* __restrict__ wq, double* __restrict__ alpha,
                                                   const double* __restrict__ guard, int32_t* __restrict__ stat) {
    __shared__ float a1[kH], a2[kH], yv[kOut];
    const int tid = threadIdx.x;
    {
        float acc = 0.0f;
        for (int k = 0; k < kIn; ++k) acc += wq[oW1 + tid * kIn + k] * q<BF16>(in.x[k]);
        a1[tid] = silu(acc + master[oB1 + tid]);
    }
    __syncthreads();
    {
        float acc = 0.0f;
        for (int k = 0; k < kH; ++k) acc += wq[oW2 + tid * kH + k] * q<BF16>(a1[k]);
        a2[tid] = silu(acc + master[oB2 + tid]);
    }
    __syncthreads();
    if (tid < kOut) {
        float acc = 0.0f;
        for (int k = 0; k < kH; ++k) acc += wq[oW3 + tid * kH + k] * q<BF16>(a2[k]);
        yv[tid] = acc + master[oB3 + tid];
    }
    __syncthreads();
    __shared__ int take;
    if (tid == 0) {
        take = 1;
        if (guard) {
            const double sc = guard[kOut * kOut + kOut];
            double yd = 0.0, yky = 0.0;
            for (int p = 0; p < kOut; ++p) {
                yd += (double)yv[p] * guard[kOut * kOut + p];
                double ky = 0.0;
                for (int q = 0; q < kOut; ++q) ky += guard[p * kOut + q] * (double)yv[q];
                yky += (double)yv[p] * ky;
            }
            const double gain = 2.0 * sc * yd - sc * sc * yky;
            take = gain > 0.0 ? 1 : 0;
            stat[take ? 0 : 1] += 1;
        }
    }
    __syncthreads();
    if (tid < kOut) {
        double acc = in.bias[tid];
        if (take)
            for (int k = 0; k < kOut; ++k) acc += in.P[tid * kOut + k] * (double)yv[k];
        alpha[tid] = acc;
    }
}

}  // namespace eqs

struct eqs_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    eqs_ctx* owner = nullptr;  // context whose device memory holds the buffers, or NULL
    int bf16 = 1;
    float *master = nullptr, *wq = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
    eqs::MlpState* st = nullptr;
};

namespace eqs {

static void mlp_launch(eqs_mlp* n, bool train, const float* x, const float* t, float* y, int32_t B) {
    dim3 g(1), b(256);
    if (train) {
        if (n->bf16)
            hipLaunchKernelGGL((k_mlp<true, true>), g, b, 0, n->stream, x, t, y, B, n->master, n->wq, n->grad, n->m1,
                               n->m2, n->st);
        else
            hipLaunchKernelGGL((k_mlp<true, false>), g, b, 0, n->stream, x, t, y, B, n->master, n->wq, n->grad, n->m1,
                               n->m2, n->st);
    } else {
        if (n->bf16)
            hipLaunchKernelGGL((k_mlp<false, true>), g, b, 0, n->stream, x, t, y, B, n->master, n->wq, n->grad,
                               n->m1, n->m2, n->st);
        else
            hipLaunchKernelGGL((k_mlp<false, false>), g, b, 0, n->stream, x, t, y, B, n->master, n->wq, n->grad,
                               n->m1, n->m2, n->st);
    }
}

static float host_bf16(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return x;
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    float r;
    std::memcpy(&r, &u, 4);
    return r;
}

eqs_mlp* mlp_create(int device, hipStream_t stream, const float* params, int bf16, double lr, eqs_ctx* owner) {
    eqs_mlp* n = new eqs_mlp();
    n->device = device;
    n->stream = stream;
    n->owner = owner;
    n->bf16 = bf16 ? 1 : 0;
    const size_t bytes = sizeof(float) * kNParam;
    auto alloc = [&](void** p, size_t nb) {
        if (owner) *p = dev_alloc(owner, nb);
        else EQS_HIP(hipMalloc(p, nb));
    };
    try {
        alloc((void**)&n->master, bytes);
        alloc((void**)&n->wq, bytes);
        alloc((void**)&n->grad, bytes);
        alloc((void**)&n->m1, bytes);
        alloc((void**)&n->m2, bytes);
        alloc((void**)&n->st, sizeof(MlpState));
        std::vector<float> w(params, params + kNParam), wq(kNParam);
        for (int i = 0; i < kNParam; ++i) wq[i] = n->bf16 ? host_bf16(w[i]) : w[i];
        std::vector<float> zero(kNParam, 0.0f);
        EQS_HIP(hipMemcpy(n->master, w.data(), bytes, hipMemcpyHostToDevice));
        EQS_HIP(hipMemcpy(n->wq, wq.data(), bytes, hipMemcpyHostToDevice));
        EQS_HIP(hipMemcpy(n->grad, zero.data(), bytes, hipMemcpyHostToDevice));
        EQS_HIP(hipMemcpy(n->m1, zero.data(), bytes, hipMemcpyHostToDevice));
        EQS_HIP(hipMemcpy(n->m2, zero.data(), bytes, hipMemcpyHostToDevice));
        MlpState s{(float)lr, 0.9f, 0.999f, 1e-8f, 0, 0.0f};
        EQS_HIP(hipMemcpy(n->st, &s, sizeof s, hipMemcpyHostToDevice));
    } catch (...) {
        mlp_destroy(n);
        throw;
    }
    return n;
}

void mlp_destroy(eqs_mlp* n) {
    if (!n) return;
    for (void* p : {(void*)n->master, (void*)n->wq, (void*)n->grad, (void*)n->m1, (void*)n->m2, (void*)n->st}) {
        if (!p) continue;
        if (n->owner) dev_free(n->owner, p);
        else (void)hipFree(p);
    }
    delete n;
}

int64_t mlp_device_bytes() {
    auto r = [](int64_t b) { return (b + 255) / 256 * 256; };
    return 5 * r((int64_t)sizeof(float) * kNParam) + r((int64_t)sizeof(MlpState));
}

void mlp_visit(eqs_mlp* n, const std::function<void(void**)>& f) {
    if (!n) return;
    f((void**)&n->master);
    f((void**)&n->wq);
    f((void**)&n->grad);
    f((void**)&n->m1);
    f((void**)&n->m2);
    f((void**)&n->st);
}

void mlp_forward(eqs_mlp* n, const float* x, float* y, int32_t B) {
    for (int32_t b0 = 0; b0 < B; b0 += kMaxB) {
        const int32_t nb = std::min<int32_t>(kMaxB, B - b0);
        mlp_launch(n, false, x + (int64_t)b0 * kIn, nullptr, y + (int64_t)b0 * kOut, nb);
    }
}

void mlp_train(eqs_mlp* n, const float* x, const float* t, int32_t B) { mlp_launch(n, true, x, t, nullptr, B); }

void mlp_forward_coeffs(eqs_mlp* n, hipStream_t s, const float* x, const double* P, const double* bias,
                        double* alpha, const double* guard, int32_t* stat) {
    MlpIn in;
    std::memcpy(in.x, x, sizeof in.x);
    std::memcpy(in.P, P, sizeof in.P);
    std::memcpy(in.bias, bias, sizeof in.bias);
    if (n->bf16)
        hipLaunchKernelGGL(k_mlp_alpha<true>, dim3(1), dim3(64), 0, s, in, n->master, n->wq, alpha, guard, stat);
    else
        hipLaunchKernelGGL(k_mlp_alpha<false>, dim3(1), dim3(64), 0, s, in, n->master, n->wq, alpha, guard, stat);
}

void mlp_get(eqs_mlp* n, float* params, float* grad) {
    if (params) EQS_HIP(hipMemcpyAsync(params, n->master, sizeof(float) * kNParam, hipMemcpyDeviceToHost, n->stream));
    if (grad) EQS_HIP(hipMemcpyAsync(grad, n->grad, sizeof(float) * kNParam, hipMemcpyDeviceToHost, n->stream));
    EQS_HIP(hipStreamSynchronize(n->stream));
}

// Checkpoint of the network: master and matmul weights, Adam moments and
// state (the gradient is rewritten by every step). Synchronises its stream.
int64_t mlp_state_bytes() { return (int64_t)(sizeof(float) * 4 * kNParam + sizeof(MlpState)); }
void mlp_save_state(eqs_mlp* n, void* host) {
    char* p = static_cast<char*>(host);
    const size_t b = sizeof(float) * kNParam;
    for (float* src : {n->master, n->wq, n->m1, n->m2}) {
        EQS_HIP(hipMemcpyAsync(p, src, b, hipMemcpyDeviceToHost, n->stream));
        p += b;
    }
    EQS_HIP(hipMemcpyAsync(p, n->st, sizeof(MlpState), hipMemcpyDeviceToHost, n->stream));
    EQS_HIP(hipStreamSynchronize(n->stream));
}
void mlp_load_state(eqs_mlp* n, const void* host) {
    const char* p = static_cast<const char*>(host);
    const size_t b = sizeof(float) * kNParam;
    for (float* dst : {n->master, n->wq, n->m1, n->m2}) {
        EQS_HIP(hipMemcpyAsync(dst, p, b, hipMemcpyHostToDevice, n->stream));
        p += b;
    }
    EQS_HIP(hipMemcpyAsync(n->st, p, sizeof(MlpState), hipMemcpyHostToDevice, n->stream));
    EQS_HIP(hipStreamSynchronize(n->stream));
}

float mlp_last_loss(eqs_mlp* n) {
    MlpState s;
    EQS_HIP(hipMemcpyAsync(&s, n->st, sizeof s, hipMemcpyDeviceToHost, n->stream));
    EQS_HIP(hipStreamSynchronize(n->stream));
    return s.loss;
}

}  // namespace eqs
