// su2_learned.hip -- gfx950 kernels that train the learned a0 proposal.
//
// The network maps f(alpha) (log-scaled alpha in [0.5, 30]) through an MLP
// 1 -> 32 -> 32 -> 47 (tanh, tanh, linear) to the 47 parameters of a 16-bin
// monotone rational-quadratic spline g on [-1, 1] (Durkan et al. 2019; widths
// and heights 2 (m + (1 - 16 m) softmax), m = 1e-3; interior derivatives
// 1e-3 + softplus, boundary derivatives 1).  The proposal density of a0 is
// q(a0 | alpha) = g'(a0) / 2.  Training minimises the negative
// log-likelihood of exact heat-bath draws (Sec. 2 density of a0) with Adam:
//   data       one thread per sample: alpha log-uniform, a0 exact sampler
//   fwd_bwd    one thread per sample: forward, analytic backward to the
//              pre-activations; per-sample rows stored for the weight gradient
//   wgrad      one workgroup per parameter: fixed-order sum over the batch
//   adam       one thread per parameter
// Every sum has a fixed order, so training is bit-reproducible.
#include "su2_internal.h"

using namespace su2dev;

namespace su2rt {

namespace {

constexpr int OFF_W1 = 0, OFF_B1 = 32, OFF_W2 = 64, OFF_B2 = 1088, OFF_W3 = 1120,
              OFF_B3 = 2624;
constexpr int NBINS = 16;
constexpr float MIN_BIN = 1e-3f, MIN_DERIV = 1e-3f;
// rows of the per-sample record (structure of arrays over the batch)
constexpr int ACT_F = 0, ACT_H1 = 1, ACT_H2 = 33, ACT_DZ1 = 65, ACT_DZ2 = 97, ACT_DO = 129;

__device__ __forceinline__ float nn_feature(float alpha)
{
    return 2.0f * __log2f(alpha / kNNAlphaLo) / kNNLog2Range - 1.0f;
}

__device__ __forceinline__ float softplusf(float t) { return t > 20.0f ? t : log1pf(expf(t)); }
__device__ __forceinline__ float sigmoidf(float t) { return 1.0f / (1.0f + expf(-t)); }

__device__ __forceinline__ double block_sum_d(double v)
{
    __shared__ double wsum[16];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) wsum[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) r += wsum[i];
    }
    __syncthreads();
    return r;
}

// MLP forward from parameters P (global or LDS).
__device__ __forceinline__ void mlp_forward(const float *P, float f, float h1[32], float h2[32],
                                            float o[47])
{
#pragma unroll
    for (int j = 0; j < 32; ++j) h1[j] = tanhf(P[OFF_W1 + j] * f + P[OFF_B1 + j]);
    for (int j = 0; j < 32; ++j) {
        float a = P[OFF_B2 + j];
#pragma unroll
        for (int m = 0; m < 32; ++m) a += P[OFF_W2 + j * 32 + m] * h1[m];
        h2[j] = tanhf(a);
    }
    for (int i = 0; i < 47; ++i) {
        float a = P[OFF_B3 + i];
#pragma unroll
        for (int m = 0; m < 32; ++m) a += P[OFF_W3 + i * 32 + m] * h2[m];
        o[i] = a;
    }
}

// Softmax of 16 logits into bin sizes 2 (m + (1 - 16 m) p); p returned too.
__device__ __forceinline__ void bin_sizes(const float *logit, float p[16], float sz[16])
{
    float mx = logit[0];
#pragma unroll
    for (int i = 1; i < 16; ++i) mx = fmaxf(mx, logit[i]);
    float sum = 0.0f;
#pragma unroll
    for (int i = 0; i < 16; ++i) sum += (p[i] = expf(logit[i] - mx));
    const float inv = 1.0f / sum;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        p[i] *= inv;
        sz[i] = 2.0f * (MIN_BIN + (1.0f - NBINS * MIN_BIN) * p[i]);
    }
}

// ------------------------------------------------------------------- data
__global__ void nn_data_kernel(float *__restrict__ alpha, float *__restrict__ a0, int64_t n,
                               float lo, float log2ratio, uint32_t k0, uint32_t k1)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t site = (uint32_t)i;
    const U4 wa = philox(site, 0u, word2(0u, TAG_TRAIN, 0u), 0u, k0, k1);
    const float al = lo * exp2f(u01(wa.a) * log2ratio);
    const uint32_t w2 = word2(1u, TAG_TRAIN, 0u);
    const U4 w0 = philox(site, 0u, w2, 0u, k0, k1);
    alpha[i] = al;
    a0[i] = 1.0f - sample_delta(al, w0, site, 0u, w2, k0, k1);
}

// ---------------------------------------------------------- forward/backward
// loss_b = -(ln 1/2 + ln g'(a0)); the record stores f, h1, h2 and the
// gradients of the mean loss w.r.t. the pre-activations of each layer.
__global__ __launch_bounds__(256) void nn_fwd_bwd_kernel(const float *__restrict__ params,
                                                         const float *__restrict__ alpha,
                                                         const float *__restrict__ a0,
                                                         int64_t offset, int batch, int64_t n,
                                                         float *__restrict__ act,
                                                         float *__restrict__ loss, float inv_batch)
{
    __shared__ float P[kNNParams];
    for (int i = threadIdx.x; i < kNNParams; i += blockDim.x) P[i] = params[i];
    __syncthreads();
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const int64_t idx = (offset + b) % n;
    const float f = nn_feature(alpha[idx]);
    const float xv = a0[idx];
    float h1[32], h2[32], o[47];
    mlp_forward(P, f, h1, h2, o);

    // spline parameters
    float pw[16], W[16], ph[16], H[16];
    bin_sizes(o, pw, W);
    bin_sizes(o + 16, ph, H);
    // bin k of xv and its left knot x_k (cumulative widths)
    int k = 0;
    float xk = -1.0f, acc = -1.0f;
#pragma unroll
    for (int j = 0; j < 15; ++j) {
        acc += W[j];
        if (xv >= acc) {
            k = j + 1;
            xk = acc;
        }
    }
    float Wk = 0.0f, Hk = 0.0f, dl = 1.0f, dh = 1.0f, thl = 0.0f, thh = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if (j == k) {
            Wk = W[j];
            Hk = H[j];
        }
    // interior derivative d_j = 1e-3 + softplus(o[32 + j - 1]), j = 1..15
#pragma unroll
    for (int j = 1; j < 16; ++j) {
        if (j == k) {
            thl = o[32 + j - 1];
            dl = MIN_DERIV + softplusf(thl);
        }
        if (j == k + 1) {
            thh = o[32 + j - 1];
            dh = MIN_DERIV + softplusf(thh);
        }
    }
    if (k == NBINS - 1) Wk = 1.0f - xk;  // last knot is exactly 1
    const float s = Hk / Wk;
    const float xi = (xv - xk) / Wk;
    const float om = xi * (1.0f - xi);
    const float tt = dh + dl - 2.0f * s;
    const float den = s + tt * om;
    const float num = dh * xi * xi + 2.0f * s * om + dl * (1.0f - xi) * (1.0f - xi);
    const float ell = 2.0f * logf(s) + logf(num) - 2.0f * logf(den);
    loss[b] = -(-0.69314718055994531f + ell);

    // d ell / d(s, xi, d_k, d_k+1)
    const float dN_ds = 2.0f * om, dD_ds = 1.0f - 2.0f * om;
    const float dN_dxi = 2.0f * dh * xi + 2.0f * s * (1.0f - 2.0f * xi) - 2.0f * dl * (1.0f - xi);
    const float dD_dxi = tt * (1.0f - 2.0f * xi);
    const float inum = 1.0f / num, iden = 1.0f / den;
    const float l_s = 2.0f / s + dN_ds * inum - 2.0f * dD_ds * iden;
    const float l_xi = dN_dxi * inum - 2.0f * dD_dxi * iden;
    const float l_dl = (1.0f - xi) * (1.0f - xi) * inum - 2.0f * om * iden;
    const float l_dh = xi * xi * inum - 2.0f * om * iden;
    // chain to the bin width, height and left knot
    const float l_H = l_s / Wk;
    const float l_W = -(l_s * s + l_xi * xi) / Wk;
    const float l_x = -l_xi / Wk;
    // widths: gW_j = [j == k] l_W + [j < k] l_x; heights: gH_j = [j == k] l_H
    // softmax backward: d/dtheta_m = 2 (1 - 16 m) p_m (g_m - sum_j p_j g_j)
    float sw = 0.0f, sh = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const float gw = (j == k ? l_W : 0.0f) + (j < k ? l_x : 0.0f);
        const float gh = j == k ? l_H : 0.0f;
        sw += pw[j] * gw;
        sh += ph[j] * gh;
    }
    const float cs = 2.0f * (1.0f - NBINS * MIN_BIN);
    // the mean loss is -ell / batch per sample: scale = -inv_batch
    const float sc = -inv_batch;
    float dout[47];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const float gw = (j == k ? l_W : 0.0f) + (j < k ? l_x : 0.0f);
        const float gh = j == k ? l_H : 0.0f;
        dout[j] = sc * cs * pw[j] * (gw - sw);
        dout[16 + j] = sc * cs * ph[j] * (gh - sh);
    }
#pragma unroll
    for (int j = 1; j < 16; ++j) {
        float g = 0.0f;
        if (j == k) g += l_dl * sigmoidf(thl);
        if (j == k + 1) g += l_dh * sigmoidf(thh);
        dout[32 + j - 1] = sc * g;
    }
    // backward through the MLP
    float dz2[32];
    for (int m = 0; m < 32; ++m) {
        float a = 0.0f;
#pragma unroll
        for (int i = 0; i < 47; ++i) a += P[OFF_W3 + i * 32 + m] * dout[i];
        dz2[m] = a * (1.0f - h2[m] * h2[m]);
    }
    float dz1[32];
    for (int m = 0; m < 32; ++m) {
        float a = 0.0f;
#pragma unroll
        for (int j = 0; j < 32; ++j) a += P[OFF_W2 + j * 32 + m] * dz2[j];
        dz1[m] = a * (1.0f - h1[m] * h1[m]);
    }
    float *r = act + b;
    r[(size_t)ACT_F * batch] = f;
#pragma unroll
    for (int m = 0; m < 32; ++m) {
        r[(size_t)(ACT_H1 + m) * batch] = h1[m];
        r[(size_t)(ACT_H2 + m) * batch] = h2[m];
        r[(size_t)(ACT_DZ1 + m) * batch] = dz1[m];
        r[(size_t)(ACT_DZ2 + m) * batch] = dz2[m];
    }
#pragma unroll
    for (int i = 0; i < 47; ++i) r[(size_t)(ACT_DO + i) * batch] = dout[i];
}

// One workgroup per parameter: the gradient is a fixed-order dot product over
// the batch of two record rows (or the sum of one row for a bias).
__global__ __launch_bounds__(256) void nn_wgrad_kernel(const float *__restrict__ act, int batch,
                                                       float *__restrict__ grad)
{
    const int p = blockIdx.x;
    int ra, rb = -1;
    if (p < OFF_B1) {
        ra = ACT_DZ1 + p;
        rb = ACT_F;
    } else if (p < OFF_W2) {
        ra = ACT_DZ1 + (p - OFF_B1);
    } else if (p < OFF_B2) {
        ra = ACT_DZ2 + (p - OFF_W2) / 32;
        rb = ACT_H1 + (p - OFF_W2) % 32;
    } else if (p < OFF_W3) {
        ra = ACT_DZ2 + (p - OFF_B2);
    } else if (p < OFF_B3) {
        ra = ACT_DO + (p - OFF_W3) / 32;
        rb = ACT_H2 + (p - OFF_W3) % 32;
    } else {
        ra = ACT_DO + (p - OFF_B3);
    }
    const float *A = act + (size_t)ra * batch;
    const float *B = rb >= 0 ? act + (size_t)rb * batch : nullptr;
    double s = 0.0;
    for (int b = threadIdx.x; b < batch; b += blockDim.x) s += (double)(B ? A[b] * B[b] : A[b]);
    const double t = block_sum_d(s);
    if (threadIdx.x == 0) grad[p] = (float)t;
}

__global__ __launch_bounds__(256) void nn_loss_kernel(const float *__restrict__ loss, int batch,
                                                      double *__restrict__ out)
{
    double s = 0.0;
    for (int b = threadIdx.x; b < batch; b += blockDim.x) s += (double)loss[b];
    const double t = block_sum_d(s);
    if (threadIdx.x == 0) *out = t / batch;
}

// Adam (Kingma & Ba 2015) with bias corrections bc1 = 1 - b1^t, bc2 = 1 - b2^t.
__global__ void nn_adam_kernel(float *__restrict__ params, const float *__restrict__ grad,
                               float *__restrict__ m, float *__restrict__ v, int n, float lr,
                               float b1, float b2, float eps, float bc1, float bc2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    params[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// One thread per table row: rows at f = -1 + 2 j / 255.
__global__ void nn_table_kernel(const float *__restrict__ params, float *__restrict__ table)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kNNRows) return;
    const float f = -1.0f + 2.0f * (float)j / (float)(kNNRows - 1);
    float h1[32], h2[32], o[47];
    mlp_forward(params, f, h1, h2, o);
    float p[16], sz[16];
    float *row = table + (size_t)j * kNNRow;
    for (int part = 0; part < 2; ++part) {
        bin_sizes(o + 16 * part, p, sz);
        float c = -1.0f;
        for (int i = 0; i < 15; ++i) {
            c += sz[i];
            row[16 * part + i] = c;
        }
        row[16 * part + 15] = 1.0f;
    }
    for (int i = 0; i < 15; ++i) row[32 + i] = MIN_DERIV + softplusf(o[32 + i]);
    row[47] = 1.0f;
}

__global__ void test_learned_kernel(const float *__restrict__ table, const float4 *__restrict__ V,
                                    const float4 *__restrict__ Uold, int64_t n, float beta,
                                    uint32_t k0, uint32_t k1, uint32_t sweep, uint32_t mu,
                                    uint32_t replica, float orw, float4 *__restrict__ out,
                                    int32_t *__restrict__ accepted)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 v = V[i], u = Uold[i];
    int acc = 0;
    const Q r = learned_link(Q{v.x, v.y, v.z, v.w}, Q{u.x, u.y, u.z, u.w}, table, beta,
                             (uint32_t)i, sweep, mu, replica, k0, k1, acc, orw);
    out[i] = make_float4(r.w, r.x, r.y, r.z);
    if (accepted) accepted[i] = acc;
}

inline unsigned nblk(uint64_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_nn_data(float *alpha, float *a0, int64_t n, float lo, float hi, uint64_t seed,
                          hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(nn_data_kernel, dim3(nblk((uint64_t)n, 256)), dim3(256), 0, stream, alpha,
                       a0, n, lo, log2f(hi / lo), (uint32_t)seed, (uint32_t)(seed >> 32));
    return hipGetLastError();
}

hipError_t launch_nn_step(const NNBuffers &nb, int64_t offset, int batch, int64_t n,
                          double *loss_out, hipStream_t stream)
{
    hipLaunchKernelGGL(nn_fwd_bwd_kernel, dim3(nblk((uint64_t)batch, 256)), dim3(256), 0, stream,
                       nb.params, nb.alpha, nb.a0, offset, batch, n, nb.act, nb.loss,
                       1.0f / (float)batch);
    hipLaunchKernelGGL(nn_wgrad_kernel, dim3(kNNParams), dim3(256), 0, stream, nb.act, batch,
                       nb.grad);
    if (loss_out)
        hipLaunchKernelGGL(nn_loss_kernel, dim3(1), dim3(256), 0, stream, nb.loss, batch,
                           loss_out);
    return hipGetLastError();
}

hipError_t launch_nn_adam(const NNBuffers &nb, float lr, int step, hipStream_t stream)
{
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = 1.0f - powf(b1, (float)step), bc2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(nn_adam_kernel, dim3(nblk(kNNParams, 256)), dim3(256), 0, stream,
                       nb.params, nb.grad, nb.m, nb.v, kNNParams, lr, b1, b2, 1e-8f, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_nn_table(const float *params, float *table, hipStream_t stream)
{
    hipLaunchKernelGGL(nn_table_kernel, dim3(1), dim3(kNNRows), 0, stream, params, table);
    return hipGetLastError();
}

hipError_t launch_test_learned(const float *table, const float *V, const float *Uold, int64_t n,
                               float beta, uint64_t seed, uint32_t sweep, uint32_t mu,
                               uint32_t replica, float orw, float *out, int32_t *accepted,
                               hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(test_learned_kernel, dim3(nblk((uint64_t)n, 256)), dim3(256), 0, stream,
                       table, (const float4 *)V, (const float4 *)Uold, n, beta, (uint32_t)seed,
                       (uint32_t)(seed >> 32), sweep, mu, replica, orw, (float4 *)out, accepted);
    return hipGetLastError();
}

}  // namespace su2rt
