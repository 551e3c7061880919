// Order / leaf-capacity predictor: forward, loss gradient and Adam (HIP, FP32).
//
// Network: z = (x - mean)/std;  h1 = relu(z W1 + b1);  h2 = relu(h1 W2 + b2);
// logits = h2 W3 + b3 with two 4-way softmax heads (order class, capacity
// class); loss = mean over rows of (CE_order + CE_capacity)/2.  Adam with
// bias correction; mean/std are input scaling, not trained.
// Every reduction is a per-thread loop in a fixed order: no atomics.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "../../include/stkfmm.h"

namespace {

constexpr int F = 12, H = 64, C = 8;
constexpr int OFF_MEAN = 0, OFF_STD = F, OFF_W1 = 2 * F, OFF_B1 = OFF_W1 + F * H, OFF_W2 = OFF_B1 + H,
              OFF_B2 = OFF_W2 + H * H, OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H * C, NPARAM = OFF_B3 + C;
// workspace per row: Z, A1, H1, A2, H2, logits, dlogits, dH2, dH1, row loss
constexpr int WS_Z = 0, WS_A1 = F, WS_H1 = WS_A1 + H, WS_A2 = WS_H1 + H, WS_H2 = WS_A2 + H, WS_L = WS_H2 + H,
              WS_DL = WS_L + C, WS_DH2 = WS_DL + C, WS_DH1 = WS_DH2 + H, WS_LOSS = WS_DH1 + H,
              WS_ROW = WS_LOSS + 1;

__global__ void standardize(int64_t B, const float *__restrict__ p, const float *__restrict__ x, float *ws) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= B * F) return;
    int64_t b = i / F;
    int k = int(i % F);
    ws[b * WS_ROW + WS_Z + k] = (x[b * F + k] - p[OFF_MEAN + k]) / p[OFF_STD + k];
}

// out[b][n] = sum_k in[b][k] W[k][n] + bias[n]; relu copy into act if given
__global__ void dense(int64_t B, int K, int N, const float *__restrict__ W, const float *__restrict__ bias,
                      const float *in, int in_off, float *out, int out_off, int act_off, int ldo) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= B * N) return;
    int64_t b = i / N;
    int n = int(i % N);
    const float *r = in + b * WS_ROW + in_off;
    float s = bias[n];
    for (int k = 0; k < K; ++k) s = fmaf(r[k], W[k * N + n], s);
    if (ldo == 0) {
        out[b * WS_ROW + out_off + n] = s;
        if (act_off >= 0) out[b * WS_ROW + act_off + n] = s > 0.0f ? s : 0.0f;
    } else {
        out[b * ldo + n] = s;
    }
}

// dlogits and row loss of the two softmax cross-entropy heads
__global__ void softmax_ce(int64_t B, const int32_t *__restrict__ labels, float *ws) {
    int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float *r = ws + b * WS_ROW;
    float loss = 0.0f;
    for (int h = 0; h < 2; ++h) {
        const float *l = r + WS_L + 4 * h;
        float m = fmaxf(fmaxf(l[0], l[1]), fmaxf(l[2], l[3]));
        float e[4], s = 0.0f;
        for (int k = 0; k < 4; ++k) {
            e[k] = expf(l[k] - m);
            s += e[k];
        }
        int y = labels[2 * b + h];
        for (int k = 0; k < 4; ++k) r[WS_DL + 4 * h + k] = 0.5f * (e[k] / s - (k == y ? 1.0f : 0.0f)) / float(B);
        loss += -(l[y] - m - logf(s));
    }
    r[WS_LOSS] = 0.5f * loss;
}

__global__ void loss_sum(int64_t B, const float *ws, float *loss) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double s = 0.0;
    for (int64_t b = 0; b < B; ++b) s += ws[b * WS_ROW + WS_LOSS];
    *loss = float(s / double(B));
}

// dW[k][n] = sum_b in[b][k] d[b][n];  db[n] = sum_b d[b][n]
__global__ void weight_grad(int64_t B, int K, int N, const float *ws, int in_off, int d_off, float *dW, float *db) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (K + 1) * N) return;
    int k = i / N, n = i % N;
    float s = 0.0f;
    if (k < K) {
        for (int64_t b = 0; b < B; ++b) s = fmaf(ws[b * WS_ROW + in_off + k], ws[b * WS_ROW + d_off + n], s);
        dW[k * N + n] = s;
    } else {
        for (int64_t b = 0; b < B; ++b) s += ws[b * WS_ROW + d_off + n];
        db[n] = s;
    }
}

// d_in[b][k] = (sum_n d[b][n] W[k][n]) * [pre[b][k] > 0]
__global__ void input_grad(int64_t B, int K, int N, const float *__restrict__ W, float *ws, int d_off, int pre_off,
                           int out_off) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= B * K) return;
    int64_t b = i / K;
    int k = int(i % K);
    float *r = ws + b * WS_ROW;
    float s = 0.0f;
    for (int n = 0; n < N; ++n) s = fmaf(r[d_off + n], W[k * N + n], s);
    r[out_off + k] = r[pre_off + k] > 0.0f ? s : 0.0f;
}

__global__ void zero(float *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

__global__ void adam(float *p, const float *__restrict__ g, float *m, float *v, float b1t, float b2t, float lr) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM || i < OFF_W1) return;   // input scaling is not trained
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    float mi = beta1 * m[i] + (1.0f - beta1) * g[i];
    float vi = beta2 * v[i] + (1.0f - beta2) * g[i] * g[i];
    m[i] = mi;
    v[i] = vi;
    float mh = mi / (1.0f - b1t), vh = vi / (1.0f - b2t);
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}

inline int nb(int64_t n) { return int((n + 255) / 256); }

hipError_t run_forward(const float *p, int64_t B, const float *x, float *ws, float *logits, hipStream_t s) {
    hipLaunchKernelGGL(standardize, dim3(nb(B * F)), dim3(256), 0, s, B, p, x, ws);
    hipLaunchKernelGGL(dense, dim3(nb(B * H)), dim3(256), 0, s, B, F, H, p + OFF_W1, p + OFF_B1, ws, WS_Z, ws,
                       WS_A1, WS_H1, 0);
    hipLaunchKernelGGL(dense, dim3(nb(B * H)), dim3(256), 0, s, B, H, H, p + OFF_W2, p + OFF_B2, ws, WS_H1, ws,
                       WS_A2, WS_H2, 0);
    if (logits)
        hipLaunchKernelGGL(dense, dim3(nb(B * C)), dim3(256), 0, s, B, H, C, p + OFF_W3, p + OFF_B3, ws, WS_H2,
                           logits, 0, -1, C);
    else
        hipLaunchKernelGGL(dense, dim3(nb(B * C)), dim3(256), 0, s, B, H, C, p + OFF_W3, p + OFF_B3, ws, WS_H2,
                           ws, WS_L, -1, 0);
    return hipGetLastError();
}

}  // namespace

extern "C" {

int stkfmm_mlp_nparam(void) { return NPARAM; }

int64_t stkfmm_mlp_workspace(int64_t batch) { return batch < 0 ? -1 : batch * int64_t(WS_ROW); }

stkfmm_status stkfmm_mlp_forward(const float *params, int64_t batch, const float *x, float *logits, float *work,
                                 void *stream) {
    if (!params || batch < 0 || (batch > 0 && (!x || !logits || !work))) return STKFMM_E_ARG;
    if (batch == 0) return STKFMM_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (run_forward(params, batch, x, work, logits, s) != hipSuccess) return STKFMM_E_DEVICE;
    return hipStreamSynchronize(s) == hipSuccess ? STKFMM_OK : STKFMM_E_DEVICE;
}

stkfmm_status stkfmm_mlp_loss_grad(const float *params, int64_t batch, const float *x, const int32_t *labels,
                                   float *grad, float *loss, float *work, void *stream) {
    if (!params || batch <= 0 || !x || !labels || !grad || !loss || !work) return STKFMM_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t B = batch;
    {   // softmax_ce indexes the logits by label: every label must name one of the 4 classes
        std::vector<int32_t> h(size_t(2 * B));
        if (hipMemcpyAsync(h.data(), labels, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return STKFMM_E_DEVICE;
        for (int32_t y : h)
            if (y < 0 || y > 3) return STKFMM_E_ARG;
    }
    if (run_forward(params, B, x, work, nullptr, s) != hipSuccess) return STKFMM_E_DEVICE;
    hipLaunchKernelGGL(softmax_ce, dim3(nb(B)), dim3(256), 0, s, B, labels, work);
    hipLaunchKernelGGL(loss_sum, dim3(1), dim3(1), 0, s, B, work, loss);
    hipLaunchKernelGGL(zero, dim3(1), dim3(64), 0, s, grad, 2 * F);
    hipLaunchKernelGGL(weight_grad, dim3(nb((H + 1) * C)), dim3(256), 0, s, B, H, C, work, WS_H2, WS_DL,
                       grad + OFF_W3, grad + OFF_B3);
    hipLaunchKernelGGL(input_grad, dim3(nb(B * H)), dim3(256), 0, s, B, H, C, params + OFF_W3, work, WS_DL, WS_A2,
                       WS_DH2);
    hipLaunchKernelGGL(weight_grad, dim3(nb((H + 1) * H)), dim3(256), 0, s, B, H, H, work, WS_H1, WS_DH2,
                       grad + OFF_W2, grad + OFF_B2);
    hipLaunchKernelGGL(input_grad, dim3(nb(B * H)), dim3(256), 0, s, B, H, H, params + OFF_W2, work, WS_DH2,
                       WS_A1, WS_DH1);
    hipLaunchKernelGGL(weight_grad, dim3(nb((F + 1) * H)), dim3(256), 0, s, B, F, H, work, WS_Z, WS_DH1,
                       grad + OFF_W1, grad + OFF_B1);
    if (hipGetLastError() != hipSuccess) return STKFMM_E_DEVICE;
    return hipStreamSynchronize(s) == hipSuccess ? STKFMM_OK : STKFMM_E_DEVICE;
}

stkfmm_status stkfmm_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step, float lr,
                              void *stream) {
    if (!params || !grad || !m || !v || step < 1 || !(lr > 0)) return STKFMM_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    float b1t = float(std::pow(0.9, double(step))), b2t = float(std::pow(0.999, double(step)));
    hipLaunchKernelGGL(adam, dim3(nb(NPARAM)), dim3(256), 0, s, params, grad, m, v, b1t, b2t, lr);
    if (hipGetLastError() != hipSuccess) return STKFMM_E_DEVICE;
    return hipStreamSynchronize(s) == hipSuccess ? STKFMM_OK : STKFMM_E_DEVICE;
}

}  // extern "C"
