// qtm_mlp.hip -- training and gradient kernels of the learned step proposal:
// an MLP 16 -> 64 -> 64 -> 3 with GELU (exact, erf form), BF16-valued weights
// and FP32 accumulation.  Loss per sample: (o0 - log h*)^2 plus, when the
// segment ended in a jump, the pinball losses at quantiles 0.05 and 0.95 of
// log tau (tau = jump time - segment start).
//
// mlp_grad_kernel: 32 samples per block, 4 threads per sample (16 hidden
// units each); forward and backward activations live in LDS, then the block's
// weight gradients are summed over its samples and written to a per-block
// partial row.  mlp_reduce_kernel sums the partial rows in block order (the
// result does not depend on scheduling) and scales by 1/batch.
#include <hip/hip_runtime.h>
#include "qtm_internal.h"

namespace qtm {

constexpr int kSPB = 32;            // samples per block
constexpr int kTPS = 4;             // threads per sample
constexpr int kMlpThreads = kSPB * kTPS;

// parameter offsets (same packing as the public layout)
constexpr int oW1 = 0, ob1 = oW1 + kNH * kNF, oW2 = ob1 + kNH, ob2 = oW2 + kNH * kNH, oW3 = ob2 + kNH,
              ob3 = oW3 + kNO * kNH, omu = ob3 + kNO, osd = omu + kNF;

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// P: [kNTotal] weights as used by the forward (BF16-valued W, FP32 b, mu, sd)
__global__ void __launch_bounds__(kMlpThreads) mlp_grad_kernel(const float* __restrict__ P, const float* __restrict__ feat,
                                                               const float* __restrict__ tgt, const int* __restrict__ perm,
                                                               long long base, int n, float* __restrict__ partial,
                                                               float* __restrict__ loss_part) {
    __shared__ float xs[kSPB][kNF];
    __shared__ float a1[kSPB][kNH], g1[kSPB][kNH], a2[kSPB][kNH], g2[kSPB][kNH];
    __shared__ float dz1[kSPB][kNH], dz2[kSPB][kNH];
    __shared__ float dO[kSPB][kNO];
    __shared__ float lsum[kSPB];
    const int tid = threadIdx.x, s = tid / kTPS, part = tid % kTPS;
    const int gs = blockIdx.x * kSPB + s;          // sample index within the batch
    const bool valid = gs < n;
    long long row = 0;
    if (valid) row = perm ? (long long)perm[base + gs] : base + gs;
    // standardised inputs
    if (part == 0) {
        for (int i = 0; i < kNF; ++i)
            xs[s][i] = valid ? (feat[row * kNF + i] - P[omu + i]) / P[osd + i] : 0.f;
    }
    __syncthreads();
    // layer 1 (16 hidden units per thread)
    for (int hh = 0; hh < 16; ++hh) {
        int h = part * 16 + hh;
        float z = P[ob1 + h];
        for (int i = 0; i < kNF; ++i) z = fmaf(P[oW1 + h * kNF + i], xs[s][i], z);
        a1[s][h] = gelu(z);
        g1[s][h] = gelu_d(z);
    }
    __syncthreads();
    for (int hh = 0; hh < 16; ++hh) {
        int h = part * 16 + hh;
        float z = P[ob2 + h];
        for (int i = 0; i < kNH; ++i) z = fmaf(P[oW2 + h * kNH + i], a1[s][i], z);
        a2[s][h] = gelu(z);
        g2[s][h] = gelu_d(z);
    }
    __syncthreads();
    if (part == 0) {
        float o[kNO];
        for (int k = 0; k < kNO; ++k) {
            float z = P[ob3 + k];
            for (int i = 0; i < kNH; ++i) z = fmaf(P[oW3 + k * kNH + i], a2[s][i], z);
            o[k] = z;
        }
        float L = 0.f, d0 = 0.f, d1 = 0.f, d2 = 0.f;
        if (valid) {
            float lh = tgt[row * 3 + 0], lt = tgt[row * 3 + 1];
            bool cens = tgt[row * 3 + 2] != 0.f;
            float r0 = o[0] - lh;
            L = r0 * r0;
            d0 = 2.f * r0;
            if (!cens) {
                float z1 = lt - o[1], z2 = lt - o[2];
                float i1 = z1 < 0.f ? 1.f : 0.f, i2 = z2 < 0.f ? 1.f : 0.f;
                L += z1 * (0.05f - i1) + z2 * (0.95f - i2);
                d1 = -(0.05f - i1);
                d2 = -(0.95f - i2);
            }
        }
        dO[s][0] = d0; dO[s][1] = d1; dO[s][2] = d2;
        lsum[s] = L;
    }
    __syncthreads();
    for (int hh = 0; hh < 16; ++hh) {
        int h = part * 16 + hh;
        float g = 0.f;
        for (int k = 0; k < kNO; ++k) g = fmaf(P[oW3 + k * kNH + h], dO[s][k], g);
        dz2[s][h] = g * g2[s][h];
    }
    __syncthreads();
    for (int ii = 0; ii < 16; ++ii) {
        int i = part * 16 + ii;
        float g = 0.f;
        for (int h = 0; h < kNH; ++h) g = fmaf(P[oW2 + h * kNH + i], dz2[s][h], g);
        dz1[s][i] = g * g1[s][i];
    }
    __syncthreads();
    // block partial gradients: sum over the block's samples in sample order
    float* out = partial + (size_t)blockIdx.x * kNParam;
    for (int p = tid; p < kNParam; p += kMlpThreads) {
        float g = 0.f;
        if (p < ob1) {                      // W1[h][i]
            int h = p / kNF, i = p % kNF;
            for (int q = 0; q < kSPB; ++q) g = fmaf(dz1[q][h], xs[q][i], g);
        } else if (p < oW2) {               // b1[h]
            int h = p - ob1;
            for (int q = 0; q < kSPB; ++q) g += dz1[q][h];
        } else if (p < ob2) {               // W2[h][i]
            int h = (p - oW2) / kNH, i = (p - oW2) % kNH;
            for (int q = 0; q < kSPB; ++q) g = fmaf(dz2[q][h], a1[q][i], g);
        } else if (p < oW3) {               // b2[h]
            int h = p - ob2;
            for (int q = 0; q < kSPB; ++q) g += dz2[q][h];
        } else if (p < ob3) {               // W3[k][h]
            int k = (p - oW3) / kNH, h = (p - oW3) % kNH;
            for (int q = 0; q < kSPB; ++q) g = fmaf(dO[q][k], a2[q][h], g);
        } else {                            // b3[k]
            int k = p - ob3;
            for (int q = 0; q < kSPB; ++q) g += dO[q][k];
        }
        out[p] = g;
    }
    if (tid == 0) {
        float L = 0.f;
        for (int q = 0; q < kSPB; ++q) L += lsum[q];
        loss_part[blockIdx.x] = L;
    }
}

__global__ void mlp_reduce_kernel(const float* __restrict__ partial, const float* __restrict__ loss_part, int nblk,
                                  float inv_n, float* __restrict__ grad, float* __restrict__ loss) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNParam) {
        float g = 0.f;
        for (int b = 0; b < nblk; ++b) g += partial[(size_t)b * kNParam + p];
        grad[p] = g * inv_n;
    }
    if (p == 0) {
        float L = 0.f;
        for (int b = 0; b < nblk; ++b) L += loss_part[b];
        *loss = L * inv_n;
    }
}

__device__ __forceinline__ float bf16r(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

// Adam on the FP32 masters, then the BF16-valued working copy of the weights.
__global__ void mlp_adam_kernel(float* __restrict__ master, float* __restrict__ work, const float* __restrict__ grad,
                                float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2, float eps,
                                float c1, float c2) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNParam) return;
    float g = grad[p];
    float mm = b1 * m[p] + (1.f - b1) * g;
    float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    float w = master[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    master[p] = w;
    bool is_w = p < ob1 || (p >= oW2 && p < ob2) || (p >= oW3 && p < ob3);
    work[p] = is_w ? bf16r(w) : w;
}

int launch_mlp_grad(const float* P, const float* feat, const float* tgt, const int* perm, long long base, int n,
                    float* partial, float* loss_part, float* grad, float* loss, hipStream_t st) {
    int nblk = (n + kSPB - 1) / kSPB;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblk), dim3(kMlpThreads), 0, st, P, feat, tgt, perm, base, n, partial, loss_part);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kNParam + 255) / 256), dim3(256), 0, st, partial, loss_part, nblk,
                       1.0f / (float)n, grad, loss);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_mlp_adam(float* master, float* work, const float* grad, float* m, float* v, float lr, int step, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kNParam + 255) / 256), dim3(256), 0, st, master, work, grad, m, v, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int mlp_partial_rows(int n) { return (n + kSPB - 1) / kSPB; }

}  // namespace qtm
