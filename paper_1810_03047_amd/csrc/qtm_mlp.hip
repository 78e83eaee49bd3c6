// qtm_mlp.hip -- training and gradient kernels of the learned step proposal:
// an MLP 16 -> 64 -> 64 -> 3 with GELU (exact, erf form), BF16-valued weights
// and FP32 accumulation.  Loss per sample: (o0 - log h*)^2 plus, when the
// segment ended in a jump, the pinball losses at quantiles 0.05 and 0.95 of
// log tau (tau = jump time - segment start).
//
// mlp_grad_kernel: one wavefront per block, 16 samples at a time as the 16
// columns of FP32 16x16x4 matrix-core products (the BF16-valued weights are exact
// FP32 operands; activations stay FP32).  Forward and backward run in registers in
// the accumulator layout (hidden unit 16 s + 4 lg + i in slot i of tile s, sample =
// column), as in the kernels' inference; the weight gradients, contractions over
// samples, are products of activation tiles staged in LDS with the sample index as
// the contraction index.  A block takes 16-sample tiles blk, blk + nblk, ... and
// writes its summed gradients to a partial row.  mlp_reduce_kernel (a gradient alone)
// and mlp_reduce_adam_kernel (a training step: the gradient, then Adam) sum the
// partial rows in a fixed order (the result does not depend on scheduling) and scale
// by 1/batch.
#include <hip/hip_runtime.h>
#include "qtm_internal.h"
#include <algorithm>

namespace qtm {

typedef float mf4 __attribute__((ext_vector_type(4)));

constexpr int kGradMaxBlocks = 1024;   // partial rows at most (blocks loop over tiles)

// parameter offsets (same packing as the public layout)
constexpr int oW1 = 0, ob1 = oW1 + kNH * kNF, oW2 = ob1 + kNH, ob2 = oW2 + kNH * kNH, oW3 = ob2 + kNH,
              ob3 = oW3 + kNO * kNH, omu = ob3 + kNO, osd = omu + kNF;

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}
__device__ __forceinline__ mf4 mma(float a, float b, mf4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// P: [kNTotal] weights as used by the forward (BF16-valued W, FP32 b, mu, sd)
__global__ void __launch_bounds__(64) mlp_grad_kernel(const float* __restrict__ P, const float* __restrict__ feat,
                                                      const float* __restrict__ tgt, const int* __restrict__ perm,
                                                      long long base, int n, float* __restrict__ partial,
                                                      float* __restrict__ loss_part) {
    // LDS tiles [unit][sample] of one 16-sample tile
    __shared__ float Xl[kNF * 16], H1l[kNH * 16], H2l[kNH * 16], D1l[kNH * 16], D2l[kNH * 16], DOl[4 * 16];
    const int lane = threadIdx.x, c16 = lane & 15, lg = lane >> 4, r16 = lane & 15, k4 = lane >> 4;
    const float* W1 = P + oW1;
    const float* W2 = P + oW2;
    const float* W3 = P + oW3;
    mf4 gW1[4], gW2[4][4], gW3[4];
    float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f, lsum = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = 0; gW3[a] = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) gW2[a][b] = 0;
    }
    const int ntile = (n + 15) / 16;
    for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int gs = tile * 16 + c16;                // this lane's sample (column)
        const bool valid = gs < n;
        const long long row = valid ? (perm ? (long long)perm[base + gs] : base + gs) : 0;
        // layer 1: x = standardised features 4 lg + j of the lane's sample
        float x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int f = 4 * lg + j;
            x[j] = valid ? (feat[row * kNF + f] - P[omu + f]) / P[osd + f] : 0.f;
        }
        mf4 z1[4], z2[4], o = 0;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            z1[rt] = 0;
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) z1[rt] = mma(W1[(16 * rt + r16) * kNF + 4 * k4 + kb], x[kb], z1[rt]);
        }
        float h1[4][4], h2[4][4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                z1[rt][i] += P[ob1 + 16 * rt + 4 * lg + i];
                h1[rt][i] = gelu(z1[rt][i]);
            }
        // layer 2: K-step (s, i) takes unit 16 s + 4 k + i from lane group k
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            z2[rt] = 0;
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    z2[rt] = mma(W2[(16 * rt + r16) * kNH + 16 * s2 + 4 * k4 + i], h1[s2][i], z2[rt]);
        }
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                z2[rt][i] += P[ob2 + 16 * rt + 4 * lg + i];
                h2[rt][i] = gelu(z2[rt][i]);
            }
        // layer 3: output rows 0..2 of one tile (rows 3..15 are zero)
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                o = mma(r16 < kNO ? W3[r16 * kNH + 16 * s2 + 4 * k4 + i] : 0.f, h2[s2][i], o);
        // loss and its gradient for the lane's sample (outputs in slots 0..2 of lane group 0)
        const float o0 = __shfl(o[0], c16) + P[ob3 + 0], o1 = __shfl(o[1], c16) + P[ob3 + 1],
                    o2 = __shfl(o[2], c16) + P[ob3 + 2];
        float L = 0.f, d0 = 0.f, d1 = 0.f, d2 = 0.f;
        if (valid) {
            const float lh = tgt[row * 3 + 0], lt = tgt[row * 3 + 1];
            const bool cens = tgt[row * 3 + 2] != 0.f;
            const float r0 = o0 - lh;
            L = r0 * r0;
            d0 = 2.f * r0;
            if (!cens) {
                const float e1 = lt - o1, e2 = lt - o2;
                const float i1 = e1 < 0.f ? 1.f : 0.f, i2 = e2 < 0.f ? 1.f : 0.f;
                L += e1 * (0.05f - i1) + e2 * (0.95f - i2);
                d1 = -(0.05f - i1);
                d2 = -(0.95f - i2);
            }
        }
        if (lg == 0) lsum += L;
        // dH2 = W3^T dO: K index k = output k, taken from lane group k
        const float dk = lg == 0 ? d0 : lg == 1 ? d1 : lg == 2 ? d2 : 0.f;
        mf4 dz2[4], dz1[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            dz2[s] = mma(k4 < kNO ? W3[k4 * kNH + 16 * s + r16] : 0.f, dk, (mf4)0);
#pragma unroll
            for (int i = 0; i < 4; ++i) dz2[s][i] *= gelu_d(z2[s][i]);
        }
        // dH1 = W2^T dZ2
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            dz1[s] = 0;
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    dz1[s] = mma(W2[(16 * s2 + 4 * k4 + i) * kNH + 16 * s + r16], dz2[s2][i], dz1[s]);
#pragma unroll
            for (int i = 0; i < 4; ++i) dz1[s][i] *= gelu_d(z1[s][i]);
        }
        // stage [unit][sample] tiles for the contractions over samples
        __syncthreads();                               // the previous tile's readers are done
#pragma unroll
        for (int j = 0; j < 4; ++j) Xl[(4 * lg + j) * 16 + c16] = x[j];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int u = (16 * s + 4 * lg + i) * 16 + c16;
                H1l[u] = h1[s][i]; H2l[u] = h2[s][i]; D1l[u] = dz1[s][i]; D2l[u] = dz2[s][i];
            }
        DOl[lg * 16 + c16] = dk;
        __syncthreads();
        // weight gradients: K index = sample 4 ks + k
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int q = 4 * ks + k4;
            const float xb = Xl[r16 * 16 + q];
            const float ob = r16 < kNO ? DOl[r16 * 16 + q] : 0.f;
#pragma unroll
            for (int jt = 0; jt < 4; ++jt) {
                const float h1b = H1l[(16 * jt + r16) * 16 + q], h2b = H2l[(16 * jt + r16) * 16 + q];
                gW3[jt] = mma(ob, h2b, gW3[jt]);
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) gW2[rt][jt] = mma(D2l[(16 * rt + r16) * 16 + q], h1b, gW2[rt][jt]);
            }
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) gW1[rt] = mma(D1l[(16 * rt + r16) * 16 + q], xb, gW1[rt]);
        }
        // bias gradients: lane u sums unit u over the tile's samples
        {
            float a = 0.f, b = 0.f, c = 0.f;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                a += D1l[lane * 16 + q];
                b += D2l[lane * 16 + q];
                if (lane < kNO) c += DOl[lane * 16 + q];
            }
            gb1 += a; gb2 += b; gb3 += c;
        }
    }
    // the block's partial row: accumulator slot i of lane (c16, lg) is row 4 lg + i, column c16
    float* out = partial + (size_t)blockIdx.x * kNParam;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * rt + 4 * lg + i;
            out[oW1 + r * kNF + c16] = gW1[rt][i];
#pragma unroll
            for (int jt = 0; jt < 4; ++jt) out[oW2 + r * kNH + 16 * jt + c16] = gW2[rt][jt][i];
        }
#pragma unroll
    for (int jt = 0; jt < 4; ++jt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (lg == 0 && i < kNO) out[oW3 + i * kNH + 16 * jt + c16] = gW3[jt][i];
    out[ob1 + lane] = gb1;
    out[ob2 + lane] = gb2;
    if (lane < kNO) out[ob3 + lane] = gb3;
    // the block's loss: lane group 0 holds one sample per lane
    float l = lsum;
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1) l += __shfl_xor(l, m);
    if (lane == 0) loss_part[blockIdx.x] = l;
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

// One training step's update: the batch gradient (partial rows summed in block order,
// scaled by 1/batch), then Adam on the FP32 masters and the BF16-valued working copy of
// the weights.  Four threads per parameter each sum a quarter of the rows (rows r with
// r % 4 == their part), combined in part order: the result does not depend on scheduling.
constexpr int kRedParts = 4, kRedThreads = 256, kRedParams = kRedThreads / kRedParts;
__global__ void __launch_bounds__(kRedThreads) mlp_reduce_adam_kernel(
        const float* __restrict__ partial, const float* __restrict__ loss_part, int nblk, float inv_n,
        float* __restrict__ loss, float* __restrict__ master, float* __restrict__ work, float* __restrict__ m,
        float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    __shared__ float part[kRedParts][kRedParams];
    const int lp = threadIdx.x % kRedParams, k = threadIdx.x / kRedParams;
    const int p = blockIdx.x * kRedParams + lp;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float L = 0.f;
        for (int b = 0; b < nblk; ++b) L += loss_part[b];
        *loss = L * inv_n;
    }
    float g = 0.f;
    if (p < kNParam)
        for (int b = k; b < nblk; b += kRedParts) g += partial[(size_t)b * kNParam + p];
    part[k][lp] = g;
    __syncthreads();
    if (k != 0 || p >= kNParam) return;
    g = ((part[0][lp] + part[1][lp]) + (part[2][lp] + part[3][lp])) * inv_n;
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
    const int nblk = mlp_partial_rows(n);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblk), dim3(64), 0, st, P, feat, tgt, perm, base, n, partial, loss_part);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kNParam + 255) / 256), dim3(256), 0, st, partial, loss_part, nblk,
                       1.0f / (float)n, grad, loss);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_mlp_train_step(float* master, float* work, float* m, float* v, const float* feat, const float* tgt,
                          const int* perm, long long base, int n, float* partial, float* loss_part, float* loss, float lr,
                          int step, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    const int nblk = mlp_partial_rows(n);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblk), dim3(64), 0, st, work, feat, tgt, perm, base, n, partial, loss_part);
    hipLaunchKernelGGL(mlp_reduce_adam_kernel, dim3((kNParam + kRedParams - 1) / kRedParams), dim3(kRedThreads), 0, st,
                       partial, loss_part, nblk, 1.0f / (float)n, loss, master, work, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int mlp_partial_rows(int n) { return std::min((n + 15) / 16, kGradMaxBlocks); }

}  // namespace qtm
