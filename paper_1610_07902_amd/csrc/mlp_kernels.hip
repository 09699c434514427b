// Schedule-selector MLP: 6 features -> 64 ReLU -> 64 ReLU -> 10 logits
// (classes: push with 2^(c+4) buckets for c = 0..8, pull for c = 9), fp32
// with plain FMA arithmetic: about 10.6K multiply-adds per sample, far too
// small for matrix cores to matter.
//
// Parameter layout (flat, 5258 floats): W1[64][6], b1[64], W2[64][64],
// b2[64], W3[10][64], b3[10].
//
// k_mlp_train_step runs one optimisation step on a batch of <= 128 samples
// in a single workgroup: forward into LDS, softmax cross-entropy, backward
// layer by layer (every gradient is a fixed-order sum over the batch, so the
// result is deterministic), then Adam.  k_mlp_forward evaluates a batch, one
// thread per sample.  k_select computes the six features of the frontier in
// the control block and writes the predicted class.

#include "decide.h"

namespace spv {

namespace {

constexpr int MI = kMI, MH1 = kMH1, MH2 = kMH2, MO = kMO;
constexpr int OW1 = kOW1, OB1 = kOB1, OW2 = kOW2, OB2 = kOB2, OW3 = kOW3, OB3 = kOB3;

constexpr int TB = 1024;   // threads of the training workgroup

__device__ __forceinline__ void forward_one(const float* __restrict__ p, const float* x, float* logits) {
    float h1[MH1], h2[MH2];
#pragma unroll 4
    for (int i = 0; i < MH1; ++i) {
        float z = p[OB1 + i];
#pragma unroll
        for (int c = 0; c < MI; ++c) z = fmaf(p[OW1 + i * MI + c], x[c], z);
        h1[i] = z > 0.f ? z : 0.f;
    }
    for (int j = 0; j < MH2; ++j) {
        float z = p[OB2 + j];
#pragma unroll 8
        for (int i = 0; i < MH1; ++i) z = fmaf(p[OW2 + j * MH1 + i], h1[i], z);
        h2[j] = z > 0.f ? z : 0.f;
    }
    for (int k = 0; k < MO; ++k) {
        float z = p[OB3 + k];
#pragma unroll 8
        for (int j = 0; j < MH2; ++j) z = fmaf(p[OW3 + k * MH2 + j], h2[j], z);
        logits[k] = z;
    }
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* p, const float* X, int B, float* logits) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= B) return;
    float x[MI];
#pragma unroll
    for (int c = 0; c < MI; ++c) x[c] = X[s * MI + c];
    float z[MO];
    forward_one(p, x, z);
#pragma unroll
    for (int k = 0; k < MO; ++k) logits[s * MO + k] = z[k];
}

__global__ __launch_bounds__(TB) void k_mlp_train_step(float* p, float* am, float* av, int step, float lr,
                                                       const float* X, const int32_t* labels, int B,
                                                       float* grad_out, float* loss_out) {
    __shared__ float xs[kMlpBatchMax * MI];
    __shared__ float a1[kMlpBatchMax * MH1];   // h1, later dz1
    __shared__ float a2[kMlpBatchMax * MH2];   // h2, later dz2
    __shared__ float d3[kMlpBatchMax * MO];    // logits, later dL/dlogits
    __shared__ float g[kMlpParams];
    __shared__ float ls[kMlpBatchMax];
    const int tid = threadIdx.x;
    for (int e = tid; e < B * MI; e += TB) xs[e] = X[e];
    __syncthreads();
    for (int e = tid; e < B * MH1; e += TB) {
        const int s = e / MH1, i = e % MH1;
        float z = p[OB1 + i];
        for (int c = 0; c < MI; ++c) z = fmaf(p[OW1 + i * MI + c], xs[s * MI + c], z);
        a1[e] = z > 0.f ? z : 0.f;
    }
    __syncthreads();
    for (int e = tid; e < B * MH2; e += TB) {
        const int s = e / MH2, j = e % MH2;
        float z = p[OB2 + j];
        for (int i = 0; i < MH1; ++i) z = fmaf(p[OW2 + j * MH1 + i], a1[s * MH1 + i], z);
        a2[e] = z > 0.f ? z : 0.f;
    }
    __syncthreads();
    for (int e = tid; e < B * MO; e += TB) {
        const int s = e / MO, k = e % MO;
        float z = p[OB3 + k];
        for (int j = 0; j < MH2; ++j) z = fmaf(p[OW3 + k * MH2 + j], a2[s * MH2 + j], z);
        d3[e] = z;
    }
    __syncthreads();
    if (tid < B) {   // softmax cross-entropy of sample tid; dL/dlogit = (softmax - onehot) / B
        float* z = d3 + tid * MO;
        float mx = z[0];
        for (int k = 1; k < MO; ++k) mx = fmaxf(mx, z[k]);
        float se = 0.f;
        for (int k = 0; k < MO; ++k) se += expf(z[k] - mx);
        int y = labels[tid];
        y = y < 0 ? 0 : (y >= MO ? MO - 1 : y);   // out-of-range labels are clamped (memory safety)
        ls[tid] = -(z[y] - mx - logf(se));
        for (int k = 0; k < MO; ++k) z[k] = (expf(z[k] - mx) / se - (k == y ? 1.f : 0.f)) / (float)B;
    }
    __syncthreads();
    if (tid == 0) {
        float L = 0.f;
        for (int s = 0; s < B; ++s) L += ls[s];
        if (loss_out) *loss_out = L / (float)B;
    }
    for (int q = tid; q < MO * MH2 + MO; q += TB) {   // layer 3
        float acc = 0.f;
        if (q < MO * MH2) {
            const int k = q / MH2, j = q % MH2;
            for (int s = 0; s < B; ++s) acc = fmaf(d3[s * MO + k], a2[s * MH2 + j], acc);
            g[OW3 + q] = acc;
        } else {
            const int k = q - MO * MH2;
            for (int s = 0; s < B; ++s) acc += d3[s * MO + k];
            g[OB3 + k] = acc;
        }
    }
    __syncthreads();
    for (int e = tid; e < B * MH2; e += TB) {   // dz2 = W3^T d3, masked by ReLU (in place over h2)
        const int s = e / MH2, j = e % MH2;
        float t = 0.f;
        for (int k = 0; k < MO; ++k) t = fmaf(p[OW3 + k * MH2 + j], d3[s * MO + k], t);
        a2[e] = a2[e] > 0.f ? t : 0.f;
    }
    __syncthreads();
    for (int q = tid; q < MH2 * MH1 + MH2; q += TB) {   // layer 2
        float acc = 0.f;
        if (q < MH2 * MH1) {
            const int j = q / MH1, i = q % MH1;
            for (int s = 0; s < B; ++s) acc = fmaf(a2[s * MH2 + j], a1[s * MH1 + i], acc);
            g[OW2 + q] = acc;
        } else {
            const int j = q - MH2 * MH1;
            for (int s = 0; s < B; ++s) acc += a2[s * MH2 + j];
            g[OB2 + j] = acc;
        }
    }
    __syncthreads();
    for (int e = tid; e < B * MH1; e += TB) {   // dz1 = W2^T dz2, masked by ReLU (in place over h1)
        const int s = e / MH1, i = e % MH1;
        float t = 0.f;
        for (int j = 0; j < MH2; ++j) t = fmaf(p[OW2 + j * MH1 + i], a2[s * MH2 + j], t);
        a1[e] = a1[e] > 0.f ? t : 0.f;
    }
    __syncthreads();
    for (int q = tid; q < MH1 * MI + MH1; q += TB) {   // layer 1
        float acc = 0.f;
        if (q < MH1 * MI) {
            const int i = q / MI, c = q % MI;
            for (int s = 0; s < B; ++s) acc = fmaf(a1[s * MH1 + i], xs[s * MI + c], acc);
            g[OW1 + q] = acc;
        } else {
            const int i = q - MH1 * MI;
            for (int s = 0; s < B; ++s) acc += a1[s * MH1 + i];
            g[OB1 + i] = acc;
        }
    }
    __syncthreads();
    // Adam (Kingma and Ba): beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias corrected.
    const float b1t = 1.f - powf(0.9f, (float)step), b2t = 1.f - powf(0.999f, (float)step);
    for (int q = tid; q < kMlpParams; q += TB) {
        const float gq = g[q];
        if (grad_out) grad_out[q] = gq;
        if (lr > 0.f) {
            const float mq = 0.9f * am[q] + 0.1f * gq;
            const float vq = 0.999f * av[q] + 0.001f * gq * gq;
            am[q] = mq;
            av[q] = vq;
            p[q] -= lr * (mq / b1t) / (sqrtf(vq / b2t) + 1e-8f);
        }
    }
}

// Features of the frontier in the control block (log2(1 + v) each, then
// standardised with the training mean / std):
//   nnz(x), sum of selected column lengths, max selected column length, n,
//   mean column length nnz / n, vertices not yet reached.
// The maximum column length is handed to maxlen_last here only when the
// pull direction will run (the scatter does it on the push path).
// forced >= 0 replaces the network's decision (a given class sequence).
__global__ void k_select(Ctrl* ctrl, const float* sel, int32_t n, int64_t nnz, int has_pull, int set_dir,
                         int forced) {
    __shared__ int s_done;
    if (threadIdx.x == 0) s_done = set_dir && ctrl->bfs_mode && consume_chain(ctrl);
    __syncthreads();
    if (s_done) return;   // the scan of this BFS level already decided
    const int32_t f = dc_ld(&ctrl->f), W = dc_ld(&ctrl->W), mx = dc_ld(&ctrl->maxlen), fnz = dc_ld(&ctrl->fnz);
    select_step(ctrl, sel, n, nnz, has_pull, set_dir, forced, f, W, mx, fnz);
}

}  // namespace

hipError_t launch_mlp_forward(const float* p, const float* X, int B, float* logits, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3((B + 255) / 256), dim3(256), 0, s, p, X, B, logits);
    return hipGetLastError();
}

hipError_t launch_mlp_train_step(float* p, float* am, float* av, int step, float lr, const float* X,
                                 const int32_t* labels, int B, float* grad_out, float* loss_out, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_train_step, dim3(1), dim3(TB), 0, s, p, am, av, step, lr, X, labels, B, grad_out,
                       loss_out);
    return hipGetLastError();
}

hipError_t launch_select(Ctrl* ctrl, const float* sel, int32_t n, int64_t nnz, int has_pull, int set_dir,
                         int forced, hipStream_t s) {
    hipLaunchKernelGGL(k_select, dim3(1), dim3(64), 0, s, ctrl, sel, n, nnz, has_pull, set_dir, forced);
    return hipGetLastError();
}

}  // namespace spv
