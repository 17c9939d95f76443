// Load predictor on the GPU: per-fault features, a 6-64-64-1 ReLU network in
// FP32 (inference, minibatch gradient, Adam), all hand-written kernels.
// Parameter vector: W1[64][6] b1[64] W2[64][64] b2[64] W3[64] b3, then the
// input normalisation mean[6] std[6].
#include "device_common.hpp"
#include "mlp.hpp"

namespace riros {

constexpr int kIn = 6, kH = 64;
constexpr int oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH, ob3 = oW3 + kH;
constexpr int oMean = kMlpParams, oStd = kMlpParams + kIn;
static_assert(ob3 + 1 == kMlpParams, "parameter layout");

// ---------------------------------------------------------------------------
// Features: the site's graph features plus two statistics of the site bit over
// the golden trace, read from its bit-plane (64 cycles per word).
// ---------------------------------------------------------------------------
__global__ void k_features(DevDesign d, GoldenView gw, const float4* __restrict__ nodefeat,
                           const riros_fault* __restrict__ faults, uint32_t F, float* __restrict__ out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F) return;
    const riros_fault f = faults[i];
    const uint32_t site = d.u2i[f.site];
    const float4 nf = nodefeat[site];
    const uint64_t* row = gw.Bp + (size_t)(d.bp_off[site] + f.bit) * gw.TW;
    const uint32_t T = gw.T;
    uint64_t ones = 0, toggles = 0;
    uint64_t prev_top = 0;
    for (uint32_t w = 0; w < gw.TW; ++w) {
        const uint32_t valid = min(64u, T - w * 64);
        const uint64_t vm = valid == 64 ? ~0ull : ((1ull << valid) - 1ull);
        const uint64_t x = row[w] & vm;
        ones += __popcll(x);
        // bit t differs from bit t-1; cycle 0 has no predecessor
        uint64_t ch = (x ^ ((x << 1) | prev_top)) & vm;
        if (w == 0) ch &= ~1ull;
        toggles += __popcll(ch);
        prev_top = x >> 63;
    }
    const uint64_t excited = f.stuck == RIROS_FAULT_FLIP ? (uint64_t)(f.t0 < T) : (f.stuck ? (uint64_t)T - ones : ones);
    float* o = out + (size_t)i * kMlpFeatures;
    o[0] = nf.x;
    o[1] = nf.y;
    o[2] = nf.z;
    o[3] = nf.w;
    o[4] = (float)toggles / (float)max(1u, T - 1);
    o[5] = (float)excited / (float)T;
}

hipError_t launch_features(const DevDesign& d, const GoldenView& gw, const float4* nodefeat,
                           const riros_fault* faults, uint32_t F, float* out, hipStream_t s)
{
    if (F == 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3((F + 255) / 256), dim3(256), 0, s, d, gw, nodefeat, faults, F, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Normalisation statistics: mean and standard deviation of each feature
// (population), accumulated in double by one workgroup.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_norm_stats(const float* __restrict__ x, uint32_t S, float* __restrict__ w)
{
    __shared__ double red[256];
    const uint32_t tid = threadIdx.x;
    for (int k = 0; k < kIn; ++k) {
        double sum = 0;
        for (uint32_t s = tid; s < S; s += 256) sum += x[(size_t)s * kIn + k];
        red[tid] = sum;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (tid < (uint32_t)h) red[tid] += red[tid + h];
            __syncthreads();
        }
        const double mean = red[0] / (double)max(1u, S);
        __syncthreads();
        double sq = 0;
        for (uint32_t s = tid; s < S; s += 256) {
            const double dv = x[(size_t)s * kIn + k] - mean;
            sq += dv * dv;
        }
        red[tid] = sq;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (tid < (uint32_t)h) red[tid] += red[tid + h];
            __syncthreads();
        }
        if (tid == 0) {
            double sd = sqrt(red[0] / (double)max(1u, S));
            w[oMean + k] = (float)mean;
            w[oStd + k] = (float)(sd > 1e-6 ? sd : 1.0);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Inference: one sample per thread, weights staged in LDS (broadcast reads).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ wts, const float* __restrict__ x,
                                                     uint32_t S, float* __restrict__ out)
{
    __shared__ float W[kMlpWeights];
    for (uint32_t i = threadIdx.x; i < (uint32_t)kMlpWeights; i += blockDim.x) W[i] = wts[i];
    __syncthreads();
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    float xin[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) xin[k] = (x[(size_t)s * kIn + k] - W[oMean + k]) / W[oStd + k];
    float h1[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float z = W[ob1 + j];
#pragma unroll
        for (int k = 0; k < kIn; ++k) z = fmaf(W[oW1 + j * kIn + k], xin[k], z);
        h1[j] = fmaxf(z, 0.f);
    }
    float o = W[ob3];
    for (int j = 0; j < kH; ++j) {
        float z = W[ob2 + j];
#pragma unroll
        for (int i = 0; i < kH; ++i) z = fmaf(W[oW2 + j * kH + i], h1[i], z);
        o = fmaf(W[oW3 + j], fmaxf(z, 0.f), o);
    }
    out[s] = o;
}

// ---------------------------------------------------------------------------
// Gradient of the mean squared error over a minibatch.  A workgroup of 64
// threads takes kGB samples: thread q < kGB runs sample q forward and backward
// to the per-sample vectors (h1, h2, dz2, dz1), which are staged in LDS; the
// workgroup then reduces them to a partial gradient (thread j owns row j of
// W2, W1 and entry j of W3, b1, b2) written to partial[block][param].
// ---------------------------------------------------------------------------
constexpr int kGB = 32;   // samples per gradient workgroup

__global__ __launch_bounds__(64) void k_mlp_grad(const float* __restrict__ wts, const float* __restrict__ x,
                                                  const float* __restrict__ y, uint32_t B, float inv_b,
                                                  float* __restrict__ partial, float* __restrict__ loss_part)
{
    __shared__ float W[kMlpWeights];
    __shared__ float sx[kGB][kIn + 1];
    __shared__ float sh1[kGB][kH + 1];
    __shared__ float sh2[kGB][kH + 1];
    __shared__ float sdz2[kGB][kH + 1];
    __shared__ float sdz1[kGB][kH + 1];
    __shared__ float sdo[kGB];
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < (uint32_t)kMlpWeights; i += 64) W[i] = wts[i];
    __syncthreads();
    if (t < (uint32_t)kGB) {
    const uint32_t s = blockIdx.x * kGB + t;
    const bool live = s < B;
    float xin[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) {
        xin[k] = live ? (x[(size_t)s * kIn + k] - W[oMean + k]) / W[oStd + k] : 0.f;
        sx[t][k] = xin[k];
    }
    float h1[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float z = W[ob1 + j];
#pragma unroll
        for (int k = 0; k < kIn; ++k) z = fmaf(W[oW1 + j * kIn + k], xin[k], z);
        h1[j] = fmaxf(z, 0.f);
        sh1[t][j] = h1[j];
    }
    float o = W[ob3];
    for (int j = 0; j < kH; ++j) {
        float z = W[ob2 + j];
#pragma unroll
        for (int i = 0; i < kH; ++i) z = fmaf(W[oW2 + j * kH + i], h1[i], z);
        const float h2 = fmaxf(z, 0.f);
        sh2[t][j] = h2;
        sdz2[t][j] = z > 0.f ? 1.f : 0.f;   // ReLU mask for now, scaled below
        o = fmaf(W[oW3 + j], h2, o);
    }
    const float r = live ? o - y[s] : 0.f;
    const float dout = 2.f * r * inv_b;
    sdo[t] = dout;
    // dz2 = dout * W3 * mask; dh1 = dz2 . W2; dz1 = dh1 * mask1
    float dh1[kH];
#pragma unroll
    for (int i = 0; i < kH; ++i) dh1[i] = 0.f;
    for (int j = 0; j < kH; ++j) {
        const float dz2 = dout * W[oW3 + j] * sdz2[t][j];
        sdz2[t][j] = dz2;
#pragma unroll
        for (int i = 0; i < kH; ++i) dh1[i] = fmaf(dz2, W[oW2 + j * kH + i], dh1[i]);
    }
#pragma unroll
    for (int i = 0; i < kH; ++i) sdz1[t][i] = h1[i] > 0.f ? dh1[i] : 0.f;
    }
    __syncthreads();
    // Reduce over the workgroup's samples; thread j owns unit j.
    const uint32_t j = t;
    float* P = partial + (size_t)blockIdx.x * kMlpParams;
    float gW3 = 0.f, gb2 = 0.f, gb1 = 0.f;
    for (int q = 0; q < kGB; ++q) {
        gW3 = fmaf(sdo[q], sh2[q][j], gW3);
        gb2 += sdz2[q][j];
        gb1 += sdz1[q][j];
    }
    P[oW3 + j] = gW3;
    P[ob2 + j] = gb2;
    P[ob1 + j] = gb1;
    for (int i = 0; i < kH; ++i) {
        float g = 0.f;
        for (int q = 0; q < kGB; ++q) g = fmaf(sdz2[q][j], sh1[q][i], g);
        P[oW2 + j * kH + i] = g;
    }
#pragma unroll
    for (int k = 0; k < kIn; ++k) {
        float g = 0.f;
        for (int q = 0; q < kGB; ++q) g = fmaf(sdz1[q][j], sx[q][k], g);
        P[oW1 + j * kIn + k] = g;
    }
    if (t == 0) {
        float gb3 = 0.f, l = 0.f;
        for (int q = 0; q < kGB; ++q) gb3 += sdo[q];
        P[ob3] = gb3;
        // loss partial: sum of squared residuals of this workgroup
        for (int q = 0; q < kGB; ++q) {
            const float rr = sdo[q] / (2.f * inv_b);
            l = fmaf(rr, rr, l);
        }
        loss_part[blockIdx.x] = l;
    }
}

// Sum the partial gradients (in workgroup order, so the result is
// deterministic), then either store the gradient or apply one Adam step.
__global__ void k_mlp_apply(float* __restrict__ wts, const float* __restrict__ partial, uint32_t nparts,
                            const float* __restrict__ loss_part, float inv_b, float* __restrict__ m,
                            float* __restrict__ v, float* __restrict__ grad_out, float* __restrict__ loss_out,
                            uint32_t step, float lr, float beta1, float beta2, float eps)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && loss_out) {
        float l = 0.f;
        for (uint32_t b = 0; b < nparts; ++b) l += loss_part[b];
        *loss_out = l * inv_b;
    }
    if (p >= (uint32_t)kMlpParams) return;
    float g = 0.f;
    for (uint32_t b = 0; b < nparts; ++b) g += partial[(size_t)b * kMlpParams + p];
    if (grad_out) {
        grad_out[p] = g;
        return;
    }
    const float mm = beta1 * m[p] + (1.f - beta1) * g;
    const float vv = beta2 * v[p] + (1.f - beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mhat = mm / (1.f - powf(beta1, (float)step));
    const float vhat = vv / (1.f - powf(beta2, (float)step));
    wts[p] -= lr * mhat / (sqrtf(vhat) + eps);
}

hipError_t mlp_norm_stats(const float* x, uint32_t S, float* wts, hipStream_t s)
{
    hipLaunchKernelGGL(k_norm_stats, dim3(1), dim3(256), 0, s, x, S, wts);
    return hipGetLastError();
}

hipError_t mlp_forward(const float* wts, const float* x, uint32_t S, float* out, hipStream_t s)
{
    if (S == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3((S + 255) / 256), dim3(256), 0, s, wts, x, S, out);
    return hipGetLastError();
}

size_t mlp_partial_floats(uint32_t B) { return (size_t)((B + kGB - 1) / kGB) * kMlpParams; }

hipError_t mlp_step(float* wts, const float* x, const float* y, uint32_t B, float* partial, float* loss_part,
                    float* m, float* v, float* grad_out, float* loss_out, uint32_t step, const MlpHyper& h,
                    hipStream_t s)
{
    const uint32_t nb = (B + kGB - 1) / kGB;
    const float inv_b = 1.f / (float)B;
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(64), 0, s, wts, x, y, B, inv_b, partial, loss_part);
    hipLaunchKernelGGL(k_mlp_apply, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, wts, partial, nb, loss_part,
                       inv_b, m, v, grad_out, loss_out, step, h.lr, h.beta1, h.beta2, h.eps);
    return hipGetLastError();
}

}  // namespace riros
