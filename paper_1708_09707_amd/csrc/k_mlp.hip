// Rank predictor for the admissible blocks: an MLP 8 -> 64 -> 64 -> 64 -> 1
// (ReLU) on geometric block features, trained on the ranks the adaptive ACA
// produces, used to size each block's ACA up front.
//
// Parameters are one float array packed as W1 (64x8, row-major), b1, W2
// (64x64), b2, W3 (64x64), b3, W4 (1x64), b4.  Inputs are standardised with a
// fixed per-feature mean / scale.  Training minimises the pinball (quantile)
// loss with Adam.  Every kernel maps one thread to one output element and
// sums in a fixed order, so forward, backward and updates are deterministic.
#include "hmx_internal.h"

namespace hmx {

namespace {

constexpr int kIn = 8;
constexpr int kH = 64;
constexpr int64_t kOffW1 = 0, kOffB1 = kOffW1 + kH * kIn, kOffW2 = kOffB1 + kH,
                  kOffB2 = kOffW2 + kH * kH, kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH * kH,
                  kOffW4 = kOffB3 + kH, kOffB4 = kOffW4 + kH, kNParam = kOffB4 + 1;

// Y[b, i] = act(sum_k W[i, k] X[b, k] + bias[i]) (X rows of length in, Y of out)
__global__ void layer_fwd_kernel(const float* __restrict__ X, int64_t B, int in, int out,
                                 const float* __restrict__ W, const float* __restrict__ bias,
                                 int relu, const float* __restrict__ mean,
                                 const float* __restrict__ scale, float* __restrict__ Y) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= B * out) return;
    const int64_t b = e / out;
    const int i = (int)(e - b * out);
    float s = bias[i];
    const float* x = X + b * in;
    for (int k = 0; k < in; ++k) {
        const float xv = mean ? (x[k] - mean[k]) * scale[k] : x[k];
        s += W[(int64_t)i * in + k] * xv;
    }
    Y[e] = relu ? (s > 0.f ? s : 0.f) : s;
}

// pinball loss: dout[b] = -(q - [y - o < 0]) / B, lpart[b] = rho_q(y - o)
__global__ void loss_kernel(const float* __restrict__ o, const float* __restrict__ y, int64_t B,
                            float q, float* __restrict__ dout, float* __restrict__ lpart) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float u = y[b] - o[b];
    const float ind = u < 0.f ? 1.f : 0.f;
    dout[b] = -(q - ind) / (float)B;
    lpart[b] = u * (q - ind);
}

// dZ[b, k] = [A[b, k] > 0] * sum_j W[j, k] dN[b, j]  (W: next layer, nout x nin)
__global__ void delta_kernel(const float* __restrict__ dN, const float* __restrict__ W,
                             const float* __restrict__ A, int64_t B, int nin, int nout,
                             float* __restrict__ dZ) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= B * nin) return;
    const int64_t b = e / nin;
    const int k = (int)(e - b * nin);
    float s = 0.f;
    for (int j = 0; j < nout; ++j) s += W[(int64_t)j * nin + k] * dN[b * nout + j];
    dZ[e] = A[e] > 0.f ? s : 0.f;
}

// Weight gradients in two passes with a fixed summation order: pass 1 gives
// every chunk of kGradChunk samples its partial sums
//   part[c, i * (in + 1) + k] = sum_{b in chunk c} dZ[b, i] X[b, k]   (k < in)
//   part[c, i * (in + 1) + in] = sum_{b in chunk c} dZ[b, i]
// and pass 2 adds the chunks in order into gW (out x in) and gbias (out).
constexpr int kGradChunk = 256;

__global__ void wgrad_partial_kernel(const float* __restrict__ dZ, const float* __restrict__ X,
                                     int64_t B, int in, int out, const float* __restrict__ mean,
                                     const float* __restrict__ scale, float* __restrict__ part) {
    const int P = out * (in + 1);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (e >= P) return;
    const int i = e / (in + 1), k = e - i * (in + 1);
    const int64_t b0 = c * kGradChunk;
    const int64_t b1 = b0 + kGradChunk < B ? b0 + kGradChunk : B;
    float s = 0.f;
    if (k < in) {
        const float mu = mean ? mean[k] : 0.f, sc = mean ? scale[k] : 1.f;
        for (int64_t b = b0; b < b1; ++b) {
            const float xv = mean ? (X[b * in + k] - mu) * sc : X[b * in + k];
            s += dZ[b * out + i] * xv;
        }
    } else {
        for (int64_t b = b0; b < b1; ++b) s += dZ[b * out + i];
    }
    part[c * P + e] = s;
}

__global__ void wgrad_reduce_kernel(const float* __restrict__ part, int64_t nchunks, int in,
                                    int out, float* __restrict__ gW, float* __restrict__ gb) {
    const int P = out * (in + 1);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P) return;
    float s = 0.f;
    for (int64_t c = 0; c < nchunks; ++c) s += part[c * P + e];
    const int i = e / (in + 1), k = e - i * (in + 1);
    if (k < in)
        gW[(int64_t)i * in + k] = s;
    else
        gb[i] = s;
}

// Adam step t >= 1 on n parameters (bias-corrected), FP32
__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// *out = mean of a[0..n), accumulated in FP64 (one workgroup, fixed tree)
__global__ void sum_kernel(const float* __restrict__ a, int64_t n, double* __restrict__ out) {
    if (blockIdx.x != 0) return;
    __shared__ double sh[4];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += a[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *out = (sh[0] + sh[1] + sh[2] + sh[3]) / (double)n;
}

// per-feature mean and 1 / std over n samples (FP64 sums, one workgroup per feature)
__global__ void norm_kernel(const float* __restrict__ X, int64_t n, float* __restrict__ mean,
                            float* __restrict__ scale) {
    __shared__ double sh[2][4];
    const int k = blockIdx.x;
    double s = 0.0, s2 = 0.0;
    for (int64_t b = threadIdx.x; b < n; b += blockDim.x) {
        const double v = X[b * kIn + k];
        s += v;
        s2 += v * v;
    }
    s = wave_sum(s);
    s2 = wave_sum(s2);
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = s;
        sh[1][threadIdx.x >> 6] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double S = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
        const double S2 = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
        const double mu = S / (double)n;
        const double var = S2 / (double)n - mu * mu;
        mean[k] = (float)mu;
        scale[k] = (float)(var > 1e-12 ? 1.0 / sqrt(var) : 1.0);
    }
}

// gather a batch of samples by index (indices outside [0, n) are clamped)
__global__ void gather_batch_kernel(const float* __restrict__ X, const float* __restrict__ y,
                                    int64_t n, const int64_t* __restrict__ idx, int64_t B,
                                    float* __restrict__ Xb, float* __restrict__ yb) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= B) return;
    int64_t s = idx[b];
    s = s < 0 ? 0 : (s >= n ? n - 1 : s);
    for (int k = 0; k < kIn; ++k) Xb[b * kIn + k] = X[s * kIn + k];
    yb[b] = y[s];
}

// Block features (FP64, cast to float): [log2 m, log2 n, diam_t / l,
// diam_s / l, dist / l, min(diam) / max(dist, 1e-12), d, log10 l^2], from the
// boxes of the block's two clusters (node ids t, s; boxes d-major per node)
// (d: box stride, dfeat: the problem's dimension, feature 6; boxes of a
// batched build are padded to 3 dimensions with zeros, which add exact zeros)
__device__ void block_features(int4 bl, int64_t t, int64_t s, const double* __restrict__ bmin,
                               const double* __restrict__ bmax, int d, int dfeat, double ell,
                               float* f) {
    double dt = 0.0, ds = 0.0, dist2 = 0.0;
    for (int k = 0; k < d; ++k) {
        const double ta = bmin[t * d + k], tb = bmax[t * d + k];
        const double sa = bmin[s * d + k], sb = bmax[s * d + k];
        dt += (tb - ta) * (tb - ta);
        ds += (sb - sa) * (sb - sa);
        double g1 = ta - sb, g2 = sa - tb;
        g1 = g1 < 0.0 ? 0.0 : g1;
        g2 = g2 < 0.0 ? 0.0 : g2;
        dist2 += g1 * g1 + g2 * g2;
    }
    const double Dt = sqrt(dt), Ds = sqrt(ds), dist = sqrt(dist2);
    f[0] = (float)log2((double)(bl.y - bl.x));
    f[1] = (float)log2((double)(bl.w - bl.z));
    f[2] = (float)(Dt / ell);
    f[3] = (float)(Ds / ell);
    f[4] = (float)(dist / ell);
    f[5] = (float)((Dt < Ds ? Dt : Ds) / (dist > 1e-12 ? dist : 1e-12));
    f[6] = (float)dfeat;
    f[7] = (float)log10(ell * ell);
}

// training pairs: features of every block and (optionally) its ACA rank as float
__global__ void features_kernel(const int4* __restrict__ blocks, const int2* __restrict__ ids,
                                int64_t nb, const double* __restrict__ bmin,
                                const double* __restrict__ bmax, int d, double ell,
                                const int32_t* __restrict__ rank, float* __restrict__ F,
                                float* __restrict__ y) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nb) return;
    float f[kIn];
    block_features(blocks[b], ids[b].x, ids[b].y, bmin, bmax, d, d, ell, f);
    for (int k = 0; k < kIn; ++k) F[b * kIn + k] = f[k];
    if (y) y[b] = (float)rank[b];
}

// Fused rank prediction, one thread per admissible block: features, input
// standardisation, the four layers with the weights staged in LDS (every lane
// reads the same weight at the same time, so LDS broadcasts), and the ACA
// target clamp(ceil(pred) + 1, 1, min(kmax, m, n)).  The sums run in the same
// order as in the layer kernels.
constexpr int kInferThreads = 256;

__global__ __launch_bounds__(kInferThreads) void rank_predict_kernel(
    const int4* __restrict__ blocks, const int2* __restrict__ ids, int64_t nb,
    const double* __restrict__ bmin, const double* __restrict__ bmax, int d, double ell,
    const float* __restrict__ w, const float* __restrict__ mean, const float* __restrict__ scale,
    int kmax, float* __restrict__ pred_out, int32_t* __restrict__ target,
    const int64_t* __restrict__ pbase, int np, const double* __restrict__ ell_p,
    const int32_t* __restrict__ dim_p) {
    __shared__ float sw[kNParam];
    for (int i = threadIdx.x; i < kNParam; i += kInferThreads) sw[i] = w[i];
    __syncthreads();
    const int64_t b = blockIdx.x * (int64_t)kInferThreads + threadIdx.x;
    if (b >= nb) return;
    const int4 bl = blocks[b];
    float x[kIn];
    if (pbase) {  // many problems: the block's problem gives l and d
        const int p = problem_of(pbase, np, bl.x);
        block_features(bl, ids[b].x, ids[b].y, bmin, bmax, 3, dim_p[p], ell_p[p], x);
    } else {
        block_features(bl, ids[b].x, ids[b].y, bmin, bmax, d, d, ell, x);
    }
    for (int k = 0; k < kIn; ++k) x[k] = (x[k] - mean[k]) * scale[k];
    float h1[kH], h2[kH];
#pragma unroll
    for (int i = 0; i < kH; ++i) {
        float s = sw[kOffB1 + i];
        for (int k = 0; k < kIn; ++k) s += sw[kOffW1 + i * kIn + k] * x[k];
        h1[i] = s > 0.f ? s : 0.f;
    }
#pragma unroll
    for (int i = 0; i < kH; ++i) {
        float s = sw[kOffB2 + i];
#pragma unroll
        for (int k = 0; k < kH; ++k) s += sw[kOffW2 + i * kH + k] * h1[k];
        h2[i] = s > 0.f ? s : 0.f;
    }
    float o = sw[kOffB4];
#pragma unroll
    for (int i = 0; i < kH; ++i) {
        float s = sw[kOffB3 + i];
#pragma unroll
        for (int k = 0; k < kH; ++k) s += sw[kOffW3 + i * kH + k] * h2[k];
        h1[i] = s > 0.f ? s : 0.f;  // third hidden layer reuses h1
    }
    for (int k = 0; k < kH; ++k) o += sw[kOffW4 + k] * h1[k];
    if (pred_out) pred_out[b] = o;
    if (target) {
        int R = kmax;
        R = (bl.y - bl.x) < R ? (bl.y - bl.x) : R;
        R = (bl.w - bl.z) < R ? (bl.w - bl.z) : R;
        int r;
        if (!(o == o)) {
            r = R;  // NaN prediction: full capacity
        } else {
            const float c = ceilf(o) + 1.f;
            r = c < 1.f ? 1 : (c > (float)R ? R : (int)c);
        }
        target[b] = r;
    }
}

// ---- fallback lists of the one-shot ACA ----
__global__ void fail_flags_kernel(const int32_t* __restrict__ rank, int64_t nb,
                                  int64_t* __restrict__ flag) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b < nb) flag[b] = rank[b] < 0 ? 1 : 0;
}

__global__ void over_flags_kernel(const int32_t* __restrict__ rank, const int32_t* __restrict__ rt,
                                  int64_t nb, int64_t* __restrict__ flag) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b < nb) flag[b] = rt[b] > 0 && rank[b] > rt[b] ? 1 : 0;
}

__global__ void gather_failed_kernel(const int32_t* __restrict__ rank,
                                     const int64_t* __restrict__ pos, int64_t nb,
                                     const int4* __restrict__ blocks,
                                     const int32_t* __restrict__ level,
                                     const int32_t* __restrict__ rt, int32_t* __restrict__ list,
                                     int4* __restrict__ blocks_out,
                                     int32_t* __restrict__ level_out,
                                     int32_t* __restrict__ rt_out) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nb || rank[b] >= 0) return;
    const int64_t i = pos[b];
    list[i] = (int32_t)b;
    blocks_out[i] = blocks[b];
    level_out[i] = level[b];
    rt_out[i] = rt[b];
}

__global__ void scatter_i32_kernel(const int32_t* __restrict__ list, int64_t nl,
                                   const int32_t* __restrict__ src, int32_t* __restrict__ dst,
                                   int add) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nl) return;
    const int32_t b = list[i];
    dst[b] = add ? dst[b] + src[i] : src[i];
}

__global__ void scatter_i64_kernel(const int32_t* __restrict__ list, int64_t nl,
                                   const int64_t* __restrict__ src, int64_t* __restrict__ dst) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < nl) dst[list[i]] = src[i];
}

unsigned g1d(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int64_t mlp_nparams() { return kNParam; }

// activations: buffer of B * (3 * 64 + 1) floats
hipError_t mlp_forward(const float* w, const float* mean, const float* scale, const float* X,
                       int64_t B, float* act, hipStream_t st) {
    if (B == 0) return hipSuccess;
    float* A1 = act;
    float* A2 = A1 + B * kH;
    float* A3 = A2 + B * kH;
    float* O = A3 + B * kH;
    hipLaunchKernelGGL(layer_fwd_kernel, dim3(g1d(B * kH)), dim3(256), 0, st, X, B, kIn, kH,
                       w + kOffW1, w + kOffB1, 1, mean, scale, A1);
    hipLaunchKernelGGL(layer_fwd_kernel, dim3(g1d(B * kH)), dim3(256), 0, st, A1, B, kH, kH,
                       w + kOffW2, w + kOffB2, 1, nullptr, nullptr, A2);
    hipLaunchKernelGGL(layer_fwd_kernel, dim3(g1d(B * kH)), dim3(256), 0, st, A2, B, kH, kH,
                       w + kOffW3, w + kOffB3, 1, nullptr, nullptr, A3);
    hipLaunchKernelGGL(layer_fwd_kernel, dim3(g1d(B)), dim3(256), 0, st, A3, B, kH, 1, w + kOffW4,
                       w + kOffB4, 0, nullptr, nullptr, O);
    return hipGetLastError();
}

size_t mlp_grad_scratch_floats(int64_t B) {
    const int64_t nch = (B + kGradChunk - 1) / kGradChunk;
    return (size_t)(B * (3 * kH + 2) + nch * kH * (kH + 1));
}

namespace {
void wgrad(const float* dZ, const float* X, int64_t B, int in, int out, const float* mean,
           const float* scale, float* part, float* gW, float* gb, hipStream_t st) {
    const int P = out * (in + 1);
    const int64_t nch = (B + kGradChunk - 1) / kGradChunk;
    hipLaunchKernelGGL(wgrad_partial_kernel, dim3(g1d(P), (unsigned)nch), dim3(256), 0, st, dZ, X,
                       B, in, out, mean, scale, part);
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(g1d(P)), dim3(256), 0, st, part, nch, in, out, gW,
                       gb);
}
}  // namespace

// gradient of the mean pinball loss over the batch (act from mlp_forward on
// the same batch); scratch: mlp_grad_scratch_floats(B) floats; loss (device
// double) optional
hipError_t mlp_backward(const float* w, const float* mean, const float* scale, const float* X,
                        const float* y, int64_t B, float q, const float* act, float* grad,
                        float* scratch, double* loss, hipStream_t st) {
    if (B == 0) return hipSuccess;
    const float* A1 = act;
    const float* A2 = A1 + B * kH;
    const float* A3 = A2 + B * kH;
    const float* O = A3 + B * kH;
    float* dO = scratch;
    float* lp = dO + B;
    float* D3 = lp + B;
    float* D2 = D3 + B * kH;
    float* D1 = D2 + B * kH;
    float* part = D1 + B * kH;
    hipLaunchKernelGGL(loss_kernel, dim3(g1d(B)), dim3(256), 0, st, O, y, B, q, dO, lp);
    if (loss) hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, lp, B, loss);
    // output layer (linear): gW4 = sum_b dO[b] A3[b, :], gb4 = sum_b dO[b]
    wgrad(dO, A3, B, kH, 1, nullptr, nullptr, part, grad + kOffW4, grad + kOffB4, st);
    hipLaunchKernelGGL(delta_kernel, dim3(g1d(B * kH)), dim3(256), 0, st, dO, w + kOffW4, A3, B,
                       kH, 1, D3);
    wgrad(D3, A2, B, kH, kH, nullptr, nullptr, part, grad + kOffW3, grad + kOffB3, st);
    hipLaunchKernelGGL(delta_kernel, dim3(g1d(B * kH)), dim3(256), 0, st, D3, w + kOffW3, A2, B,
                       kH, kH, D2);
    wgrad(D2, A1, B, kH, kH, nullptr, nullptr, part, grad + kOffW2, grad + kOffB2, st);
    hipLaunchKernelGGL(delta_kernel, dim3(g1d(B * kH)), dim3(256), 0, st, D2, w + kOffW2, A1, B,
                       kH, kH, D1);
    wgrad(D1, X, B, kIn, kH, mean, scale, part, grad + kOffW1, grad + kOffB1, st);
    return hipGetLastError();
}

hipError_t mlp_adam(float* w, float* m, float* v, const float* g, int64_t t, float lr, float b1,
                    float b2, float eps, hipStream_t st) {
    const float c1 = (float)(1.0 - pow((double)b1, (double)t));
    const float c2 = (float)(1.0 - pow((double)b2, (double)t));
    hipLaunchKernelGGL(adam_kernel, dim3(g1d(kNParam)), dim3(256), 0, st, w, m, v, g, kNParam, lr,
                       b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_norm(const float* X, int64_t n, float* mean, float* scale, hipStream_t st) {
    hipLaunchKernelGGL(norm_kernel, dim3(kIn), dim3(256), 0, st, X, n, mean, scale);
    return hipGetLastError();
}

hipError_t mlp_gather_batch(const float* X, const float* y, int64_t n, const int64_t* idx,
                            int64_t B, float* Xb, float* yb, hipStream_t st) {
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_batch_kernel, dim3(g1d(B)), dim3(256), 0, st, X, y, n, idx, B, Xb,
                       yb);
    return hipGetLastError();
}

hipError_t launch_features(const int4* blocks, const int2* ids, int64_t nb, const double* bmin,
                           const double* bmax, int d, double ell, const int32_t* rank, float* F,
                           float* y, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(features_kernel, dim3(g1d(nb)), dim3(256), 0, st, blocks, ids, nb, bmin,
                       bmax, d, ell, rank, F, y);
    return hipGetLastError();
}

hipError_t launch_rank_predict(const int4* blocks, const int2* ids, int64_t nb, const double* bmin,
                               const double* bmax, int d, double ell, const float* w,
                               const float* mean, const float* scale, int kmax, float* pred,
                               int32_t* target, hipStream_t st, const int64_t* pbase, int np,
                               const double* ell_p, const int32_t* dim_p) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(rank_predict_kernel, dim3(g1d(nb, kInferThreads)), dim3(kInferThreads), 0,
                       st, blocks, ids, nb, bmin, bmax, d, ell, w, mean, scale, kmax, pred, target,
                       pbase, np, ell_p, dim_p);
    return hipGetLastError();
}

hipError_t launch_fail_flags(const int32_t* rank, int64_t nb, int64_t* flag, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(fail_flags_kernel, dim3(g1d(nb)), dim3(256), 0, st, rank, nb, flag);
    return hipGetLastError();
}

hipError_t launch_over_flags(const int32_t* rank, const int32_t* rt, int64_t nb, int64_t* flag,
                             hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(over_flags_kernel, dim3(g1d(nb)), dim3(256), 0, st, rank, rt, nb, flag);
    return hipGetLastError();
}

hipError_t launch_gather_failed(const int32_t* rank, const int64_t* pos, int64_t nb,
                                const int4* blocks, const int32_t* level, const int32_t* rt,
                                int32_t* list, int4* blocks_out, int32_t* level_out,
                                int32_t* rt_out, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_failed_kernel, dim3(g1d(nb)), dim3(256), 0, st, rank, pos, nb,
                       blocks, level, rt, list, blocks_out, level_out, rt_out);
    return hipGetLastError();
}

hipError_t launch_scatter_i32(const int32_t* list, int64_t nl, const int32_t* src, int32_t* dst,
                              int add, hipStream_t st) {
    if (nl == 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_i32_kernel, dim3(g1d(nl)), dim3(256), 0, st, list, nl, src, dst,
                       add);
    return hipGetLastError();
}

hipError_t launch_scatter_i64(const int32_t* list, int64_t nl, const int64_t* src, int64_t* dst,
                              hipStream_t st) {
    if (nl == 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_i64_kernel, dim3(g1d(nl)), dim3(256), 0, st, list, nl, src, dst);
    return hipGetLastError();
}

}  // namespace hmx
