// Z-order ordering of the point set (Section 4.4, Algorithm 6):
//   global bounding box -> Morton codes -> stable LSD radix sort of
//   (code, index) -> Morton-ordered SoA coordinates (Section 5.1 point_set).
//
// Compiled with -ffp-contract=off: the fixed-point conversion must be the
// exact IEEE sequence (y - lo) / (hi - lo) * 2^B, floor, clamp.
#include "hmx_internal.h"

namespace hmx {

namespace {

constexpr int kBoxThreads = 256;

__device__ __forceinline__ double load_coord(const void* pts, int f64, int64_t i) {
    return f64 ? ((const double*)pts)[i] : (double)((const float*)pts)[i];
}

// partial min/max over a grid-strided range of points
__global__ __launch_bounds__(kBoxThreads) void box_partial_kernel(const void* __restrict__ pts,
                                                                  int f64, int64_t n, int d,
                                                                  double* __restrict__ partial) {
    __shared__ double smin[3][kBoxThreads / kWave], smax[3][kBoxThreads / kWave];
    double mn[3], mx[3];
    for (int k = 0; k < 3; ++k) {
        mn[k] = INFINITY;
        mx[k] = -INFINITY;
    }
    bool nan_seen = false;
    for (int64_t i = blockIdx.x * (int64_t)kBoxThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBoxThreads) {
        for (int k = 0; k < d; ++k) {
            double v = load_coord(pts, f64, i * d + k);
            nan_seen |= (v != v);
            mn[k] = v < mn[k] ? v : mn[k];
            mx[k] = v > mx[k] ? v : mx[k];
        }
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int k = 0; k < d; ++k) {
        double a = mn[k], b = mx[k];
        for (int o = 32; o > 0; o >>= 1) {
            double a2 = __shfl_xor(a, o, 64), b2 = __shfl_xor(b, o, 64);
            a = a2 < a ? a2 : a;
            b = b2 > b ? b2 : b;
        }
        if (lane == 0) {
            smin[k][w] = a;
            smax[k][w] = b;
        }
    }
    // a NaN coordinate poisons the box so the host rejects the input
    unsigned long long anynan = __ballot(nan_seen);
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < d; ++k) {
            double a = smin[k][0], b = smax[k][0];
            for (int q = 1; q < kBoxThreads / kWave; ++q) {
                a = smin[k][q] < a ? smin[k][q] : a;
                b = smax[k][q] > b ? smax[k][q] : b;
            }
            partial[(int64_t)blockIdx.x * 6 + k] = a;
            partial[(int64_t)blockIdx.x * 6 + 3 + k] = b;
        }
    }
    if (anynan && lane == 0) partial[(int64_t)blockIdx.x * 6] = NAN;
}

__global__ void box_final_kernel(const double* __restrict__ partial, int nparts, int d,
                                 double* __restrict__ box) {
    if (threadIdx.x != 0) return;
    for (int k = 0; k < d; ++k) {
        double a = partial[k], b = partial[3 + k];
        bool nan = (a != a);
        for (int p = 1; p < nparts; ++p) {
            double a2 = partial[(int64_t)p * 6 + k], b2 = partial[(int64_t)p * 6 + 3 + k];
            nan |= (a2 != a2);
            a = a2 < a ? a2 : a;
            b = b2 > b ? b2 : b;
        }
        box[k] = nan ? NAN : a;
        box[d + k] = b;
    }
}

// spread the low bits of v so that consecutive bits land `step` apart
__device__ __forceinline__ uint64_t spread2(uint64_t x) {
    x &= 0xffffffffull;
    x = (x | (x << 16)) & 0x0000ffff0000ffffull;
    x = (x | (x << 8)) & 0x00ff00ff00ff00ffull;
    x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}
__device__ __forceinline__ uint64_t spread3(uint64_t x) {
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// Algorithm 6: per point, fixed-point representation of each coordinate
// relative to the global box, then bit interleaving (dimension 0 in the
// most significant position of every group of d bits).
// the code of one point y (d coordinates) in the box [lo, hi]
__device__ __forceinline__ uint64_t morton_code(const double* y, int d, const double* lo,
                                                const double* hi) {
    const int B = d == 1 ? 32 : (d == 2 ? 32 : 21);
    const double scale = d == 3 ? 2097152.0 : 4294967296.0;  // 2^B
    const uint64_t qmax = (1ull << B) - 1ull;
    uint64_t q[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) {
        if (hi[k] == lo[k]) continue;
        double t = (y[k] - lo[k]) / (hi[k] - lo[k]);
        double f = floor(t * scale);
        q[k] = (f >= (double)qmax) ? qmax : (uint64_t)f;
    }
    if (d == 1) return q[0];
    if (d == 2) return (spread2(q[0]) << 1) | spread2(q[1]);
    return (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
}

__global__ __launch_bounds__(256) void morton_kernel(const void* __restrict__ pts, int f64,
                                                     int64_t n, int d,
                                                     const double* __restrict__ box,
                                                     uint64_t* __restrict__ codes,
                                                     uint32_t* __restrict__ idx) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double y[3];
    for (int k = 0; k < d; ++k) y[k] = load_coord(pts, f64, i * d + k);
    codes[i] = morton_code(y, d, box, box + d);
    idx[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// many independent problems at once (the forest of a batched build): the
// problems' points one after another in a union index space, problem p
// owning [pbase[p], pbase[p + 1]); every problem is ordered in its own box,
// exactly as a build of it alone would order it
// ---------------------------------------------------------------------------

// the union points as N x 3 FP64 (coordinates beyond a problem's d are 0)
__global__ void forest_points_kernel(const ForestInput* __restrict__ in, int np,
                                     const int64_t* __restrict__ pbase, int64_t N, int f64,
                                     double* __restrict__ P) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int p = problem_of(pbase, np, i);
    const ForestInput q = in[p];
    const int64_t j = i - pbase[p];
    for (int k = 0; k < 3; ++k) P[i * 3 + k] = k < q.d ? load_coord(q.pts, f64, j * q.d + k) : 0.0;
}

// per-problem partial boxes: workgroup (x, p) reduces a grid-strided share
// of problem p's points over its d dimensions (a NaN poisons the box)
__global__ __launch_bounds__(kBoxThreads) void forest_box_partial_kernel(
    const double* __restrict__ P, const int64_t* __restrict__ pbase,
    const int32_t* __restrict__ dims, double* __restrict__ partial) {
    __shared__ double smin[3][kBoxThreads / kWave], smax[3][kBoxThreads / kWave];
    const int p = blockIdx.y;
    const int d = dims[p];
    const int64_t a = pbase[p], b = pbase[p + 1];
    double mn[3], mx[3];
    for (int k = 0; k < 3; ++k) {
        mn[k] = INFINITY;
        mx[k] = -INFINITY;
    }
    bool nan_seen = false;
    for (int64_t i = a + blockIdx.x * (int64_t)kBoxThreads + threadIdx.x; i < b;
         i += (int64_t)gridDim.x * kBoxThreads) {
        for (int k = 0; k < d; ++k) {
            double v = P[i * 3 + k];
            nan_seen |= (v != v);
            mn[k] = v < mn[k] ? v : mn[k];
            mx[k] = v > mx[k] ? v : mx[k];
        }
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int k = 0; k < d; ++k) {
        double u = mn[k], v = mx[k];
        for (int o = 32; o > 0; o >>= 1) {
            double u2 = __shfl_xor(u, o, 64), v2 = __shfl_xor(v, o, 64);
            u = u2 < u ? u2 : u;
            v = v2 > v ? v2 : v;
        }
        if (lane == 0) {
            smin[k][w] = u;
            smax[k][w] = v;
        }
    }
    unsigned long long anynan = __ballot(nan_seen);
    __syncthreads();
    double* out = partial + ((int64_t)p * gridDim.x + blockIdx.x) * 6;
    if (threadIdx.x == 0) {
        for (int k = 0; k < d; ++k) {
            double u = smin[k][0], v = smax[k][0];
            for (int q = 1; q < kBoxThreads / kWave; ++q) {
                u = smin[k][q] < u ? smin[k][q] : u;
                v = smax[k][q] > v ? smax[k][q] : v;
            }
            out[k] = u;
            out[3 + k] = v;
        }
    }
    if (anynan && lane == 0) out[0] = NAN;
}

// box of problem p: lo in box[6 p + k], hi in box[6 p + 3 + k]
__global__ void forest_box_final_kernel(const double* __restrict__ partial, int nparts, int np,
                                        const int32_t* __restrict__ dims,
                                        double* __restrict__ box) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int d = dims[p];
    const double* pp = partial + (int64_t)p * nparts * 6;
    for (int k = 0; k < 3; ++k) {
        double a = k < d ? pp[k] : 0.0, b = k < d ? pp[3 + k] : 0.0;
        bool nan = (a != a);
        for (int q = 1; q < nparts && k < d; ++q) {
            double a2 = pp[(int64_t)q * 6 + k], b2 = pp[(int64_t)q * 6 + 3 + k];
            nan |= (a2 != a2);
            a = a2 < a ? a2 : a;
            b = b2 > b ? b2 : b;
        }
        box[6 * p + k] = nan ? NAN : a;
        box[6 * p + 3 + k] = b;
    }
}

__global__ __launch_bounds__(256) void forest_morton_kernel(const double* __restrict__ P,
                                                            int64_t N, int np,
                                                            const int64_t* __restrict__ pbase,
                                                            const int32_t* __restrict__ dims,
                                                            const double* __restrict__ box,
                                                            uint64_t* __restrict__ codes,
                                                            uint32_t* __restrict__ idx) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int p = problem_of(pbase, np, i);
    codes[i] = morton_code(P + i * 3, dims[p], box + 6 * p, box + 6 * p + 3);
    idx[i] = (uint32_t)i;
}

// sort key of the second, stable pass: the problem of each sorted point
__global__ void forest_problem_keys_kernel(const uint32_t* __restrict__ idx, int64_t N, int np,
                                           const int64_t* __restrict__ pbase,
                                           uint64_t* __restrict__ keys) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < N) keys[i] = (uint64_t)problem_of(pbase, np, (int64_t)idx[i]);
}

__global__ void gather_u64_kernel(const uint64_t* __restrict__ src, const uint32_t* __restrict__ idx,
                                  int64_t n, uint64_t* __restrict__ dst) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits, digit-major tile histograms
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 keys per workgroup
constexpr int kSortWaves = kSortThreads / kWave;

__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const uint64_t* __restrict__ keys,
                                                                  int64_t n, int shift,
                                                                  int64_t ntiles,
                                                                  int64_t* __restrict__ counts) {
    __shared__ int hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = blockIdx.x * (int64_t)kSortTile;
    for (int k = 0; k < kSortItems; ++k) {
        int64_t i = base + k * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&hist[(keys[i] >> shift) & 255], 1);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = hist[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, int64_t n, int shift,
    int64_t ntiles, const int64_t* __restrict__ offsets, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout) {
    __shared__ int64_t gbase[256];
    __shared__ int running[256];
    __shared__ int wcnt[kSortWaves][256];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    gbase[tid] = offsets[(int64_t)tid * ntiles + blockIdx.x];
    running[tid] = 0;
    const int64_t base = blockIdx.x * (int64_t)kSortTile;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int k = 0; k < kSortItems; ++k) {
        for (int q = 0; q < kSortWaves; ++q) wcnt[q][tid] = 0;
        __syncthreads();
        const int64_t i = base + k * kSortThreads + tid;
        const bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0;
        uint32_t val = valid ? vin[i] : 0;
        const int dig = (int)((key >> shift) & 255);
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dig >> b) & 1;
            const uint64_t bal = __ballot(valid && bit);
            peers &= bit ? bal : ~bal;
        }
        const int rank_in_wave = __popcll(peers & lt_mask);
        if (valid && rank_in_wave == 0) wcnt[w][dig] = __popcll(peers);
        __syncthreads();
        int before = 0;
        for (int q = 0; q < w; ++q) before += wcnt[q][dig];
        if (valid) {
            const int64_t pos = gbase[dig] + running[dig] + before + rank_in_wave;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        int tot = 0;
        for (int q = 0; q < kSortWaves; ++q) tot += wcnt[q][tid];
        running[tid] += tot;
    }
}

__global__ void gather_coords_kernel(const void* __restrict__ pts, int f64, int64_t n, int d,
                                     const uint32_t* __restrict__ perm, double* __restrict__ soa64,
                                     float* __restrict__ soa32) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t p = perm[i];
    for (int k = 0; k < d; ++k) {
        double v = load_coord(pts, f64, p * d + k);
        soa64[(int64_t)k * n + i] = v;
        if (soa32) soa32[(int64_t)k * n + i] = (float)v;
    }
}

}  // namespace

int global_box_parts(int64_t n) {
    int64_t p = (n + 16 * kBoxThreads - 1) / (16 * kBoxThreads);
    return (int)(p < 1 ? 1 : (p > 1024 ? 1024 : p));
}

hipError_t launch_global_box(const void* pts, int pts_f64, int64_t n, int d, double* partial,
                             int nparts, double* box, hipStream_t st) {
    hipLaunchKernelGGL(box_partial_kernel, dim3(nparts), dim3(kBoxThreads), 0, st, pts, pts_f64,
                       n, d, partial);
    hipLaunchKernelGGL(box_final_kernel, dim3(1), dim3(64), 0, st, partial, nparts, d, box);
    return hipGetLastError();
}

hipError_t launch_morton(const void* pts, int pts_f64, int64_t n, int d, const double* box,
                         uint64_t* codes, uint32_t* idx, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(morton_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pts,
                       pts_f64, n, d, box, codes, idx);
    return hipGetLastError();
}

static int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

size_t radix_sort_scratch_bytes(int64_t n) {
    const int64_t nt = sort_tiles(n);
    return (size_t)n * (sizeof(uint64_t) + sizeof(uint32_t)) + 256 + (size_t)(256 * nt) * 8 +
           scan_scratch_bytes(256 * nt) + 64;
}

hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, int64_t n, int bits, void* scratch,
                            hipStream_t st) {
    if (n <= 1 || bits <= 0) return hipSuccess;
    const int64_t nt = sort_tiles(n);
    char* p = (char*)scratch;
    uint64_t* k2 = (uint64_t*)p;
    p += n * sizeof(uint64_t);
    uint32_t* v2 = (uint32_t*)p;
    p += n * sizeof(uint32_t);
    p = (char*)(((uintptr_t)p + 255) & ~(uintptr_t)255);
    int64_t* counts = (int64_t*)p;
    p += 256 * nt * 8;
    void* sscr = p;
    uint64_t *ka = keys, *kb = k2;
    uint32_t *va = vals, *vb = v2;
    const int passes = (bits + 7) / 8;
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = 8 * ps;
        hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)nt), dim3(kSortThreads), 0, st, ka,
                           n, shift, nt, counts);
        hipError_t e = exclusive_scan_i64(counts, 256 * nt, nullptr, sscr, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)nt), dim3(kSortThreads), 0, st, ka,
                           va, n, shift, nt, counts, kb, vb);
        uint64_t* tk = ka;
        ka = kb;
        kb = tk;
        uint32_t* tv = va;
        va = vb;
        vb = tv;
    }
    if (ka != keys) {
        hipError_t e = hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t launch_forest_points(const ForestInput* in, int np, const int64_t* pbase, int64_t N,
                                int f64, double* P, hipStream_t st) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(forest_points_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
                       in, np, pbase, N, f64, P);
    return hipGetLastError();
}

int forest_box_parts() { return 64; }

hipError_t launch_forest_box(const double* P, int np, const int64_t* pbase, const int32_t* dims,
                             double* partial, double* box, hipStream_t st) {
    hipLaunchKernelGGL(forest_box_partial_kernel, dim3(forest_box_parts(), np), dim3(kBoxThreads),
                       0, st, P, pbase, dims, partial);
    hipLaunchKernelGGL(forest_box_final_kernel, dim3((np + 63) / 64), dim3(64), 0, st, partial,
                       forest_box_parts(), np, dims, box);
    return hipGetLastError();
}

hipError_t launch_forest_morton(const double* P, int64_t N, int np, const int64_t* pbase,
                                const int32_t* dims, const double* box, uint64_t* codes,
                                uint32_t* idx, hipStream_t st) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(forest_morton_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
                       P, N, np, pbase, dims, box, codes, idx);
    return hipGetLastError();
}

hipError_t launch_forest_problem_keys(const uint32_t* idx, int64_t N, int np,
                                      const int64_t* pbase, uint64_t* keys, hipStream_t st) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(forest_problem_keys_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0,
                       st, idx, N, np, pbase, keys);
    return hipGetLastError();
}

hipError_t launch_gather_u64(const uint64_t* src, const uint32_t* idx, int64_t n, uint64_t* dst,
                             hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       src, idx, n, dst);
    return hipGetLastError();
}

hipError_t launch_gather_coords(const void* pts, int pts_f64, int64_t n, int d,
                                const uint32_t* perm, double* soa64, float* soa32,
                                hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_coords_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       pts, pts_f64, n, d, perm, soa64, soa32);
    return hipGetLastError();
}

}  // namespace hmx
