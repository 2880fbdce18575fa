// Assembly of many independent problems into one block-diagonal H-matrix
// (batched build): index shifts of the per-problem orderings, leaf lists and
// row tiles, and the coordinates of every problem scaled by its kernel's
// length so that one kernel parameter serves all problems, padded to three
// dimensions with zeros (distances unchanged).
#include "hmx_internal.h"

namespace hmx {

namespace {

unsigned g1d(int64_t n) { return (unsigned)((n + 255) / 256); }

__global__ void add_i32_kernel(int32_t* __restrict__ dst, const int32_t* __restrict__ src,
                               int64_t cnt, int32_t c) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < cnt) dst[i] = src[i] + c;
}

__global__ void shift_blocks_kernel(int4* __restrict__ dst, const int4* __restrict__ src,
                                    int64_t cnt, int32_t base) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    const int4 b = src[i];
    dst[i] = make_int4(b.x + base, b.y + base, b.z + base, b.w + base);
}

__global__ void fill_i32_kernel(int32_t* __restrict__ dst, int64_t cnt, int32_t v) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < cnt) dst[i] = v;
}

// dst (3 x ntot, FP64 and optionally FP32) rows [base, base + n) from src
// (d x n FP64) times scale; dimensions d..2 are zero
__global__ void scale_coords_kernel(const double* __restrict__ src, int64_t n, int d,
                                    double scale, double* __restrict__ dst64,
                                    float* __restrict__ dst32, int64_t ntot, int64_t base) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < 3; ++k) {
        const double v = k < d ? src[(int64_t)k * n + i] * scale : 0.0;
        dst64[(int64_t)k * ntot + base + i] = v;
        if (dst32) dst32[(int64_t)k * ntot + base + i] = (float)v;
    }
}

}  // namespace

hipError_t launch_add_i32(int32_t* dst, const int32_t* src, int64_t cnt, int32_t c,
                          hipStream_t st) {
    if (cnt == 0) return hipSuccess;
    hipLaunchKernelGGL(add_i32_kernel, dim3(g1d(cnt)), dim3(256), 0, st, dst, src, cnt, c);
    return hipGetLastError();
}

hipError_t launch_shift_blocks(int4* dst, const int4* src, int64_t cnt, int32_t base,
                               hipStream_t st) {
    if (cnt == 0) return hipSuccess;
    hipLaunchKernelGGL(shift_blocks_kernel, dim3(g1d(cnt)), dim3(256), 0, st, dst, src, cnt, base);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* dst, int64_t cnt, int32_t v, hipStream_t st) {
    if (cnt == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(g1d(cnt)), dim3(256), 0, st, dst, cnt, v);
    return hipGetLastError();
}

hipError_t launch_scale_coords(const double* src, int64_t n, int d, double scale, double* dst64,
                               float* dst32, int64_t ntot, int64_t base, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(scale_coords_kernel, dim3(g1d(n)), dim3(256), 0, st, src, n, d, scale,
                       dst64, dst32, ntot, base);
    return hipGetLastError();
}

}  // namespace hmx
