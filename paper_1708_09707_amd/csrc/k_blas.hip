// BLAS-1 kernels of the conjugate-gradient solve of (H + sigma2 I) c = y
// (the kernel ridge regression / Gaussian process system of Section 1).
// Vectors are in the compute type; every inner product is accumulated in
// FP64 with a fixed reduction tree (grid-stride partial sums per thread,
// wave and block reduction, then one workgroup sums the block partials in
// order), so the solve is bit-reproducible.
#include "hmx_internal.h"

namespace hmx {

namespace {

constexpr int kDotThreads = 256;
constexpr int kDotBlocks = 1024;

__device__ __forceinline__ double block_sum_f64(double v, double* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kDotThreads / 64; ++q) r += sh[q];
    return r;
}

// partial[block] = sum over the block's grid-stride elements of a[i] * b[i]
template <typename T>
__global__ __launch_bounds__(kDotThreads) void dot_partial_kernel(const T* __restrict__ a,
                                                                  const T* __restrict__ b,
                                                                  int64_t n,
                                                                  double* __restrict__ partial) {
    __shared__ double sh[kDotThreads / 64];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kDotThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kDotThreads)
        acc += (double)a[i] * (double)b[i];
    const double s = block_sum_f64(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out[slot] = sum of nparts partials, in order
__global__ void dot_final_kernel(const double* __restrict__ partial, int nparts,
                                 double* __restrict__ out) {
    __shared__ double sh[kDotThreads / 64];
    double acc = 0.0;
    for (int q = threadIdx.x; q < nparts; q += kDotThreads) acc += partial[q];
    const double s = block_sum_f64(acc, sh);
    if (threadIdx.x == 0) *out = s;
}

// x += alpha p ; r -= alpha q ; partial sums of r.r
template <typename T>
__global__ __launch_bounds__(kDotThreads) void cg_update_kernel(T* __restrict__ x,
                                                                T* __restrict__ r,
                                                                const T* __restrict__ p,
                                                                const T* __restrict__ q,
                                                                const double* __restrict__ scal,
                                                                int64_t n,
                                                                double* __restrict__ partial) {
    __shared__ double sh[kDotThreads / 64];
    // (r.r) / (p.q); a step with p.q <= 0 (the operator is not positive
    // definite on p: CG breaks down) is not taken, so x and r keep the last
    // iterate's values
    const double pq = scal[1];
    const T alpha = pq > 0.0 ? (T)(scal[0] / pq) : (T)0;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kDotThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kDotThreads) {
        x[i] += alpha * p[i];
        const T ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += (double)ri * (double)ri;
    }
    const double s = block_sum_f64(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// p = r + beta p with beta = (r'.r') / (r.r)
template <typename T>
__global__ void cg_direction_kernel(T* __restrict__ p, const T* __restrict__ r,
                                    const double* __restrict__ scal, int64_t n) {
    const T beta = (T)(scal[2] / scal[0]);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = r[i] + beta * p[i];
}

template <typename T>
__global__ void copy_kernel(T* __restrict__ dst, const T* __restrict__ src, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

template <typename T>
__global__ void sub_kernel(T* __restrict__ out, const T* __restrict__ a, const T* __restrict__ b,
                           int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] - b[i];
}

template <typename T>
__global__ void fill_zero_kernel(T* __restrict__ dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (T)0;
}

unsigned blocks_for(int64_t n) {
    const int64_t b = (n + kDotThreads - 1) / kDotThreads;
    return (unsigned)(b < kDotBlocks ? (b < 1 ? 1 : b) : kDotBlocks);
}

}  // namespace

size_t cg_scratch_bytes() { return (size_t)(kDotBlocks + 8) * sizeof(double); }

// scal: device doubles; the dot product goes to scal[slot]
hipError_t launch_dot(const void* a, const void* b, int64_t n, int f64, double* partial,
                      double* out, hipStream_t st) {
    const unsigned g = blocks_for(n);
    if (f64)
        hipLaunchKernelGGL(dot_partial_kernel<double>, dim3(g), dim3(kDotThreads), 0, st,
                           (const double*)a, (const double*)b, n, partial);
    else
        hipLaunchKernelGGL(dot_partial_kernel<float>, dim3(g), dim3(kDotThreads), 0, st,
                           (const float*)a, (const float*)b, n, partial);
    hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kDotThreads), 0, st, partial, (int)g, out);
    return hipGetLastError();
}

hipError_t launch_cg_update(void* x, void* r, const void* p, const void* q, const double* scal,
                            int64_t n, int f64, double* partial, double* out, hipStream_t st) {
    const unsigned g = blocks_for(n);
    if (f64)
        hipLaunchKernelGGL(cg_update_kernel<double>, dim3(g), dim3(kDotThreads), 0, st,
                           (double*)x, (double*)r, (const double*)p, (const double*)q, scal, n,
                           partial);
    else
        hipLaunchKernelGGL(cg_update_kernel<float>, dim3(g), dim3(kDotThreads), 0, st, (float*)x,
                           (float*)r, (const float*)p, (const float*)q, scal, n, partial);
    hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kDotThreads), 0, st, partial, (int)g, out);
    return hipGetLastError();
}

hipError_t launch_cg_direction(void* p, const void* r, const double* scal, int64_t n, int f64,
                               hipStream_t st) {
    const unsigned g = blocks_for(n);
    if (f64)
        hipLaunchKernelGGL(cg_direction_kernel<double>, dim3(g), dim3(kDotThreads), 0, st,
                           (double*)p, (const double*)r, scal, n);
    else
        hipLaunchKernelGGL(cg_direction_kernel<float>, dim3(g), dim3(kDotThreads), 0, st,
                           (float*)p, (const float*)r, scal, n);
    return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, int64_t n, int f64, hipStream_t st) {
    const unsigned g = blocks_for(n);
    if (f64)
        hipLaunchKernelGGL(copy_kernel<double>, dim3(g), dim3(kDotThreads), 0, st, (double*)dst,
                           (const double*)src, n);
    else
        hipLaunchKernelGGL(copy_kernel<float>, dim3(g), dim3(kDotThreads), 0, st, (float*)dst,
                           (const float*)src, n);
    return hipGetLastError();
}

hipError_t launch_sub(void* out, const void* a, const void* b, int64_t n, int f64,
                      hipStream_t st) {
    const unsigned g = blocks_for(n);
    if (f64)
        hipLaunchKernelGGL(sub_kernel<double>, dim3(g), dim3(kDotThreads), 0, st, (double*)out,
                           (const double*)a, (const double*)b, n);
    else
        hipLaunchKernelGGL(sub_kernel<float>, dim3(g), dim3(kDotThreads), 0, st, (float*)out,
                           (const float*)a, (const float*)b, n);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* dst, int64_t n, int f64, hipStream_t st) {
    const unsigned g = blocks_for(n);
    if (f64)
        hipLaunchKernelGGL(fill_zero_kernel<double>, dim3(g), dim3(kDotThreads), 0, st,
                           (double*)dst, n);
    else
        hipLaunchKernelGGL(fill_zero_kernel<float>, dim3(g), dim3(kDotThreads), 0, st, (float*)dst,
                           n);
    return hipGetLastError();
}

}  // namespace hmx
