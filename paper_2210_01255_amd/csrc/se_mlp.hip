// se_mlp.hip -- FP32 kernels of the learned parameter selector: a fully
// connected network 10 -> 64 (tanh) -> 64 (tanh) -> 4 (linear), its mean
// squared error, the gradient by backpropagation, and the Adam update
// (Kingma and Ba, 2015).
//
// Parameter vector theta (SE_MLP_NPARAM floats): W1[64][10], b1[64],
// W2[64][64], b2[64], W3[4][64], b3[4]; row-major, output index first.
//
// Training kernel: one 256-thread block per 32 samples holds the whole
// network in LDS (plus W2 transposed, so that both the forward product and
// the backward product read consecutive addresses across a wavefront), the
// activations of its samples and their back-propagated errors, and writes
// one partial gradient; a second kernel sums the partials in a fixed order,
// so that a step's result does not depend on scheduling.
#include "se_internal.h"

#include <cmath>
#include <cstring>
#include <mutex>

namespace {

constexpr int kIn = SE_MLP_IN, kHid = SE_MLP_HID, kOut = SE_MLP_OUT;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kOut * kHid, kNP = oB3 + kOut;
static_assert(kNP == SE_MLP_NPARAM, "parameter layout");
constexpr int kS = 32;  // samples per block

struct se_mlp_norm {
    float xm[kIn], xs[kIn], ym[kOut], ys[kOut];
};

// Sample at position pos of an epoch: (a pos + c) mod n, a bijection when
// gcd(a, n) = 1 (a = 1, c = 0: the identity order).
__device__ inline int64_t sample_at(int64_t pos, uint64_t a, uint64_t c, int64_t n)
{
    return (int64_t)((a * (uint64_t)pos + c) % (uint64_t)n);
}

__global__ void __launch_bounds__(256) k_mlp_grad(const float* __restrict__ th, const float* __restrict__ X,
                                                  const float* __restrict__ Y, int64_t n, uint64_t a, uint64_t c,
                                                  int64_t start, int cnt, float inv, float* __restrict__ part)
{
    __shared__ float w[kNP];
    __shared__ float w2t[kHid * kHid];
    __shared__ float xs[kS][kIn];
    __shared__ float h1[kS][kHid];
    __shared__ float h2[kS][kHid];  // later: back-propagated error of layer 1
    __shared__ float d2[kS][kHid];
    __shared__ float d3[kS][kOut];
    __shared__ float red[kS * kOut];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int i = t; i < kNP; i += 256) w[i] = th[i];
    for (int i = t; i < kHid * kHid; i += 256) {
        const int j = i >> 6, k = i & 63;  // w2t[k][j] = W2[j][k]
        w2t[k * kHid + j] = th[oW2 + i];
    }
    const int base = blockIdx.x * kS;
    for (int i = t; i < kS * kIn; i += 256) {
        const int s = i / kIn, f = i % kIn;
        float v = 0.f;
        if (base + s < cnt) v = X[sample_at(start + base + s, a, c, n) * kIn + f];
        xs[s][f] = v;
    }
    __syncthreads();
    // layer 1: lane = hidden unit, 8 samples per thread
    for (int s = wv; s < kS; s += 4) {
        float acc = w[oB1 + lane];
#pragma unroll
        for (int i = 0; i < kIn; i++) acc += w[oW1 + lane * kIn + i] * xs[s][i];
        h1[s][lane] = tanhf(acc);
    }
    __syncthreads();
    for (int s = wv; s < kS; s += 4) {
        float acc = w[oB2 + lane];
#pragma unroll 8
        for (int k = 0; k < kHid; k++) acc += w2t[k * kHid + lane] * h1[s][k];
        h2[s][lane] = tanhf(acc);
    }
    __syncthreads();
    // output, residual and its error signal
    if (t < kS * kOut) {
        const int s = t >> 2, o = t & 3;
        float acc = w[oB3 + o];
        for (int j = 0; j < kHid; j++) acc += w[oW3 + o * kHid + j] * h2[s][j];
        float r = 0.f;
        if (base + s < cnt) r = acc - Y[sample_at(start + base + s, a, c, n) * kOut + o];
        d3[s][o] = 2.f * r * inv;
        red[t] = r * r * inv;
    }
    __syncthreads();
    float* g = part + (size_t)blockIdx.x * (kNP + 1);
    if (t == 0) {
        float l = 0.f;
        for (int i = 0; i < kS * kOut; i++) l += red[i];
        g[kNP] = l;
    }
    // layer 3 gradients
    {
        const int o = t >> 6, j = lane;
        float acc = 0.f;
        for (int s = 0; s < kS; s++) acc += d3[s][o] * h2[s][j];
        g[oW3 + o * kHid + j] = acc;
        if (t < kOut) {
            float b = 0.f;
            for (int s = 0; s < kS; s++) b += d3[s][t];
            g[oB3 + t] = b;
        }
    }
    for (int s = wv; s < kS; s += 4) {
        float acc = 0.f;
#pragma unroll
        for (int o = 0; o < kOut; o++) acc += w[oW3 + o * kHid + lane] * d3[s][o];
        const float hv = h2[s][lane];
        d2[s][lane] = (1.f - hv * hv) * acc;
    }
    __syncthreads();
    // layer 2 gradients
    for (int j = wv; j < kHid; j += 4) {
        float acc = 0.f;
        for (int s = 0; s < kS; s++) acc += d2[s][j] * h1[s][lane];
        g[oW2 + j * kHid + lane] = acc;
    }
    if (t < kHid) {
        float b = 0.f;
        for (int s = 0; s < kS; s++) b += d2[s][t];
        g[oB2 + t] = b;
    }
    // error of layer 1 (into h2's storage: h2 is no longer needed)
    for (int s = wv; s < kS; s += 4) {
        float acc = 0.f;
#pragma unroll 8
        for (int j = 0; j < kHid; j++) acc += w[oW2 + j * kHid + lane] * d2[s][j];
        const float hv = h1[s][lane];
        h2[s][lane] = (1.f - hv * hv) * acc;
    }
    __syncthreads();
    for (int q = t; q < kHid * kIn; q += 256) {
        const int k = q / kIn, i = q % kIn;
        float acc = 0.f;
        for (int s = 0; s < kS; s++) acc += h2[s][k] * xs[s][i];
        g[oW1 + q] = acc;
    }
    if (t < kHid) {
        float b = 0.f;
        for (int s = 0; s < kS; s++) b += h2[s][t];
        g[oB1 + t] = b;
    }
}

// Sums nb partial gradients (and losses) in block order.
__global__ void k_mlp_reduce(const float* __restrict__ part, int nb, float* __restrict__ grad, float* __restrict__ loss)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > kNP) return;
    float acc = 0.f;
    for (int b = 0; b < nb; b++) acc += part[(size_t)b * (kNP + 1) + j];
    if (j < kNP)
        grad[j] = acc;
    else if (loss)
        *loss = acc;
}

__global__ void k_mlp_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps, float c1,
                           float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// One sample per thread; raw features in, raw outputs out (the stored
// normalisation applied on both sides; norm = nullptr: normalised data).
__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ th, const float* __restrict__ X,
                                                     int64_t n, float* __restrict__ Y, se_mlp_norm nm, int use_norm)
{
    __shared__ float w[kNP];
    for (int i = threadIdx.x; i < kNP; i += 256) w[i] = th[i];
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    float x[kIn];
#pragma unroll
    for (int i = 0; i < kIn; i++) {
        x[i] = X[s * kIn + i];
        if (use_norm) x[i] = (x[i] - nm.xm[i]) / nm.xs[i];
    }
    float h[kHid];
#pragma unroll
    for (int j = 0; j < kHid; j++) {
        float acc = w[oB1 + j];
#pragma unroll
        for (int i = 0; i < kIn; i++) acc += w[oW1 + j * kIn + i] * x[i];
        h[j] = tanhf(acc);
    }
    float y[kOut];
#pragma unroll
    for (int o = 0; o < kOut; o++) y[o] = w[oB3 + o];
    for (int j = 0; j < kHid; j++) {
        float acc = w[oB2 + j];
#pragma unroll
        for (int k = 0; k < kHid; k++) acc += w[oW2 + j * kHid + k] * h[k];
        const float hj = tanhf(acc);
#pragma unroll
        for (int o = 0; o < kOut; o++) y[o] += w[oW3 + o * kHid + j] * hj;
    }
#pragma unroll
    for (int o = 0; o < kOut; o++) Y[s * kOut + o] = use_norm ? y[o] * nm.ys[o] + nm.ym[o] : y[o];
}

__global__ void k_mlp_fill(float* p, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

size_t se_mlp_part_floats(int cnt) { return (size_t)((cnt + kS - 1) / kS) * (kNP + 1); }

void se_mlp_launch_grad(const float* th, const float* X, const float* Y, int64_t n, uint64_t a, uint64_t c,
                        int64_t start, int cnt, float* part, float* grad, float* loss, hipStream_t s)
{
    const int nb = (cnt + kS - 1) / kS;
    const float inv = 1.f / ((float)cnt * kOut);
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, s, th, X, Y, n, a, c, start, cnt, inv, part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kNP + 1 + 255) / 256), dim3(256), 0, s, part, nb, grad, loss);
}

void se_mlp_launch_adam(float* th, float* m, float* v, const float* g, int64_t n, int t, float lr, float b1,
                        float b2, float eps, hipStream_t s)
{
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)t));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)t));
    hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, th, m, v, g, n, lr, b1, b2,
                       eps, c1, c2);
}

void se_mlp_launch_forward(const float* th, const float* X, int64_t n, float* Y, const float* norm, hipStream_t s)
{
    se_mlp_norm nm;
    std::memset(&nm, 0, sizeof(nm));
    if (norm) {
        for (int i = 0; i < kIn; i++) {
            nm.xm[i] = norm[i];
            nm.xs[i] = norm[kIn + i];
        }
        for (int o = 0; o < kOut; o++) {
            nm.ym[o] = norm[2 * kIn + o];
            nm.ys[o] = norm[2 * kIn + kOut + o];
        }
    }
    if (n > 0)
        hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, th, X, n, Y, nm,
                           norm ? 1 : 0);
}

void se_mlp_launch_fill(float* p, int64_t n, float v, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_mlp_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
}

// ---------------------------------------------------------------------------
// Allocation-free loss and gradient.  The per-block partial sums of
// k_mlp_grad go to this file-scope array instead of a buffer allocated per
// call.  Every block writes all SE_MLP_NPARAM + 1 entries of its slot and
// k_mlp_reduce reads only the slots of the blocks just launched, so the array
// needs no clearing between calls.  In host code `scratch` names a host-side
// stand-in: its device address, one per GPU, comes from hipGetSymbolAddress.
static __device__ __align__(256) float scratch[(SE_MLP_NOALLOC_MAX_N / kS) * (SE_MLP_NPARAM + 1)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
se_status scratch_on_current_device(float** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SE_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return SE_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SE_ERR_HIP;
        g_scratch_ptr[dev] = (float*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return SE_OK;
}

}  // namespace

se_status se_mlp_loss_grad_noalloc(const float* theta, const float* X, const float* Y, int64_t n, float* grad,
                                   float* loss, void* stream)
{
    if (!theta || !X || !Y || !grad || !loss || n < 1) return SE_ERR_ARG;
    if (n > SE_MLP_NOALLOC_MAX_N) return SE_ERR_SCRATCH;
    float* part = nullptr;
    const se_status st = scratch_on_current_device(&part);
    if (st != SE_OK) return st;
    se_mlp_launch_grad(theta, X, Y, n, 1, 0, 0, (int)n, part, grad, loss, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? SE_OK : SE_ERR_HIP;
}
