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

// the union coordinates (3 x N FP64, Morton order) scaled by each point's
// problem factor 1 / l_p, in FP64 and optionally FP32
__global__ void forest_scale_kernel(const double* __restrict__ src, int64_t N, int np,
                                    const int64_t* __restrict__ pbase,
                                    const double* __restrict__ inv_ell, double* __restrict__ dst64,
                                    float* __restrict__ dst32) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double s = inv_ell[problem_of(pbase, np, i)];
    for (int k = 0; k < 3; ++k) {
        const double v = src[(int64_t)k * N + i] * s;
        dst64[(int64_t)k * N + i] = v;
        if (dst32) dst32[(int64_t)k * N + i] = (float)v;
    }
}

// size class of every admissible leaf from its problem's level thresholds
// (cuts[p] = the first levels of the 512-thread, 256-thread and single-wave
// classes), as the sort key of a stable pass that groups the classes
__global__ void forest_class_kernel(const int4* __restrict__ adm, const int32_t* __restrict__ level,
                                    int64_t nadm, int np, const int64_t* __restrict__ pbase,
                                    const int4* __restrict__ cuts, uint64_t* __restrict__ keys,
                                    uint32_t* __restrict__ vals) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nadm) return;
    const int4 c = cuts[problem_of(pbase, np, adm[b].x)];
    const int l = level[b];
    keys[b] = l < c.x ? 0 : (l < c.y ? 1 : (l < c.z ? 2 : 3));
    vals[b] = (uint32_t)b;
}

__global__ void narrow_u64_kernel(const uint64_t* __restrict__ src, int64_t n,
                                  int32_t* __restrict__ dst) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (int32_t)src[i];
}

// largest cluster side among the admissible leaves (integer maximum)
__global__ void max_side_kernel(const int4* __restrict__ adm, int64_t nadm,
                                int* __restrict__ out) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int v = 0;
    if (b < nadm) {
        const int4 q = adm[b];
        v = q.y - q.x > q.w - q.z ? q.y - q.x : q.w - q.z;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const int w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(out, v);
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

// lstart[l] / lend[l]: first / one past the last index of level l in a
// level-sorted list (levels absent from the list keep the preset zeros)
__global__ void level_bounds_kernel(const int32_t* __restrict__ level, int64_t nb,
                                    int64_t* __restrict__ lstart, int64_t* __restrict__ lend) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int32_t l = level[i];
    if (i == 0 || level[i - 1] != l) lstart[l] = i;
    if (i == nb - 1 || level[i + 1] != l) lend[l] = i + 1;
}

// key (slice << 8 | level): block i at position pos of its level's c blocks
// belongs to slice floor(pos nch / c), so every slice holds a contiguous
// share of every level; a stable sort by the key keeps each slice level-sorted
__global__ void interleave_keys_kernel(const int32_t* __restrict__ level, int64_t nb,
                                       const int64_t* __restrict__ lstart,
                                       const int64_t* __restrict__ lend, int nch,
                                       uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int32_t l = level[i];
    const int64_t s = lstart[l], c = lend[l] - s;
    const uint64_t slice = (uint64_t)((i - s) * (int64_t)nch / c);
    keys[i] = (slice << 8) | (uint64_t)l;
    vals[i] = (uint32_t)i;
}

// the blocks, levels and (optional) two per-block int32 arrays in the order perm
__global__ void gather_blocks_kernel(const uint32_t* __restrict__ perm, int64_t n,
                                     const int4* __restrict__ blocks,
                                     const int32_t* __restrict__ level,
                                     const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                                     int4* __restrict__ blocks_out, int32_t* __restrict__ level_out,
                                     int32_t* __restrict__ a_out, int32_t* __restrict__ b_out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = perm[i];
    blocks_out[i] = blocks[j];
    level_out[i] = level[j];
    if (a) a_out[i] = a[j];
    if (b) b_out[i] = b[j];
}

}  // namespace

hipError_t launch_level_bounds(const int32_t* level, int64_t nb, int64_t* lstart, int64_t* lend,
                               hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(level_bounds_kernel, dim3(g1d(nb)), dim3(256), 0, st, level, nb, lstart,
                       lend);
    return hipGetLastError();
}

hipError_t launch_interleave_keys(const int32_t* level, int64_t nb, const int64_t* lstart,
                                  const int64_t* lend, int nch, uint64_t* keys, uint32_t* vals,
                                  hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(interleave_keys_kernel, dim3(g1d(nb)), dim3(256), 0, st, level, nb, lstart,
                       lend, nch, keys, vals);
    return hipGetLastError();
}

hipError_t launch_gather_blocks(const uint32_t* perm, int64_t n, const int4* blocks,
                                const int32_t* level, const int32_t* a, const int32_t* b,
                                int4* blocks_out, int32_t* level_out, int32_t* a_out,
                                int32_t* b_out, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_blocks_kernel, dim3(g1d(n)), dim3(256), 0, st, perm, n, blocks,
                       level, a, b, blocks_out, level_out, a_out, b_out);
    return hipGetLastError();
}

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

hipError_t launch_forest_scale(const double* src, int64_t N, int np, const int64_t* pbase,
                               const double* inv_ell, double* dst64, float* dst32,
                               hipStream_t st) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(forest_scale_kernel, dim3(g1d(N)), dim3(256), 0, st, src, N, np, pbase,
                       inv_ell, dst64, dst32);
    return hipGetLastError();
}

hipError_t launch_forest_class(const int4* adm, const int32_t* level, int64_t nadm, int np,
                               const int64_t* pbase, const int4* cuts, uint64_t* keys,
                               uint32_t* vals, hipStream_t st) {
    if (nadm == 0) return hipSuccess;
    hipLaunchKernelGGL(forest_class_kernel, dim3(g1d(nadm)), dim3(256), 0, st, adm, level, nadm,
                       np, pbase, cuts, keys, vals);
    return hipGetLastError();
}

hipError_t launch_narrow_u64(const uint64_t* src, int64_t n, int32_t* dst, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(narrow_u64_kernel, dim3(g1d(n)), dim3(256), 0, st, src, n, dst);
    return hipGetLastError();
}

hipError_t launch_max_side(const int4* adm, int64_t nadm, int* out, hipStream_t st) {
    if (nadm == 0) return hipSuccess;
    hipLaunchKernelGGL(max_side_kernel, dim3(g1d(nadm)), dim3(256), 0, st, adm, nadm, out);
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
