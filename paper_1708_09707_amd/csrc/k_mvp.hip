// Near-field assembly and the batched H-matrix-vector product (Algorithm 3
// in flat form, Section 5.4).
//
// Storage (all column-major, one contiguous region per block):
//   near pool : A|tau x sigma for every dense leaf (m x n)
//   U pool    : U (m x r) for every admissible leaf, V pool: V (n x r)
//   vector pool: [ x in Morton order (n) | t_b = V_b^T x|sigma (sum r) ]
// Matvec = gather x -> phase 1 (t_b for every admissible leaf) -> phase 2
// (one workgroup per leaf cluster of rows: z|tile = sum of its pieces, where
// a piece is the tile's rows of a dense block times x|sigma or of U_b times
// t_b) -> scatter to the original order with alpha, beta, sigma2.
// Every z row is written by exactly one workgroup and every sum has a fixed
// order, so the product is deterministic.
#include "hmx_internal.h"

namespace hmx {

namespace {

// ---------------------------------------------------------------------------
// near field: A[q m + i] = phi(y_{tlo+i}, y_{slo+q})
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void near_kernel(const T* __restrict__ soa, int64_t n, int d,
                                                   KernelEval<T> K,
                                                   const int4* __restrict__ blocks,
                                                   int64_t nblocks,
                                                   const int64_t* __restrict__ off,
                                                   T* __restrict__ A) {
    for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
        const int4 bl = blocks[b];
        const int m = bl.y - bl.x, nc = bl.w - bl.z;
        T* __restrict__ out = A + off[b];
        const int64_t tot = (int64_t)m * nc;
        int i = threadIdx.x, q = 0;
        while (i >= m) {
            i -= m;
            ++q;
        }
        for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
            T x[3], y[3];
            load_pt(soa, n, d, (int64_t)bl.x + i, x);
            load_pt(soa, n, d, (int64_t)bl.z + q, y);
            out[e] = phi(K, x, y, d);
            i += blockDim.x;
            while (i >= m) {
                i -= m;
                ++q;
            }
        }
    }
}

// per-block sizes: mode 0: m * mult, 1: n * mult, 2: m * n, 3: r * m, 4: r * n,
// 5: r, 6: number of row tiles covered (0 if rank == 0 for an admissible list)
__global__ void extent_kernel(const int4* __restrict__ blocks, int64_t nb, int mode, int64_t mult,
                              const int32_t* __restrict__ rank,
                              const int32_t* __restrict__ tile_of_point,
                              int64_t* __restrict__ out) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int4 bl = blocks[b];
    const int64_t m = bl.y - bl.x, nc = bl.w - bl.z;
    int64_t v = 0;
    switch (mode) {
        case 0: v = m * mult; break;
        case 1: v = nc * mult; break;
        case 2: v = m * nc; break;
        case 3: v = (int64_t)rank[b] * m; break;
        case 4: v = (int64_t)rank[b] * nc; break;
        case 5: v = rank[b]; break;
        default:
            v = (rank && rank[b] == 0) ? 0
                                       : (int64_t)(tile_of_point[bl.y - 1] - tile_of_point[bl.x] + 1);
    }
    out[b] = v;
}

__global__ void piece_fill_kernel(const int4* __restrict__ blocks, int64_t nb,
                                  const int32_t* __restrict__ rank,
                                  const int32_t* __restrict__ tile_of_point,
                                  const int32_t* __restrict__ tile_lo,
                                  const int64_t* __restrict__ piece_off,
                                  const int64_t* __restrict__ data_off,
                                  const int64_t* __restrict__ vec_off_blk, int64_t vec_base,
                                  int pool, int64_t piece_base, Piece* __restrict__ pieces,
                                  uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int4 bl = blocks[b];
    const int r = rank ? rank[b] : 0;
    if (rank && r == 0) return;
    const int m = bl.y - bl.x;
    const int t0 = tile_of_point[bl.x], t1 = tile_of_point[bl.y - 1];
    int64_t p = piece_base + piece_off[b];
    for (int t = t0; t <= t1; ++t, ++p) {
        Piece pc;
        pc.a_off = data_off[b] + (tile_lo[t] - bl.x);
        pc.v_off = rank ? vec_base + vec_off_blk[b] : (int64_t)bl.z;
        pc.ld = m;
        pc.ncols = rank ? r : (bl.w - bl.z);
        pc.pool = pool;
        pc.pad = 0;
        pieces[p] = pc;
        keys[p] = (uint64_t)t;
        vals[p] = (uint32_t)p;
    }
}

__global__ void piece_gather_kernel(const Piece* __restrict__ src, const uint32_t* __restrict__ order,
                                    int64_t np, Piece* __restrict__ dst) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < np) dst[i] = src[order[i]];
}

// tile_ptr[t] = number of pieces with tile < t (lower bound in the sorted keys)
__global__ void tile_ptr_kernel(const uint64_t* __restrict__ keys, int64_t np, int64_t ntiles,
                                int64_t* __restrict__ ptr) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    int64_t lo = 0, hi = np;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < (uint64_t)t)
            lo = mid + 1;
        else
            hi = mid;
    }
    ptr[t] = lo;
}

template <typename T>
__global__ void gather_x_kernel(const T* __restrict__ x, const int32_t* __restrict__ perm,
                                int64_t n, T* __restrict__ xm) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) xm[i] = x[perm[i]];
}

// phase 1: t_b[l] = sum_j V_b[j, l] x[slo + j], one wave per column l
template <typename T>
__global__ __launch_bounds__(256) void far_phase1_kernel(const int4* __restrict__ adm,
                                                         int64_t nadm,
                                                         const int32_t* __restrict__ rank,
                                                         const int64_t* __restrict__ voff,
                                                         const int64_t* __restrict__ toff,
                                                         const T* __restrict__ V,
                                                         T* __restrict__ vec, int64_t n) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t b = blockIdx.x; b < nadm; b += gridDim.x) {
        const int4 bl = adm[b];
        const int nc = bl.w - bl.z, r = rank[b];
        const T* __restrict__ Vb = V + voff[b];
        const T* __restrict__ xs = vec + bl.z;
        for (int l = w; l < r; l += 4) {
            const T* __restrict__ col = Vb + (int64_t)l * nc;
            T acc = 0;
            for (int j = lane; j < nc; j += 64) acc += col[j] * xs[j];
            acc = wave_sum(acc);
            if (lane == 0) vec[n + toff[b] + l] = acc;
        }
    }
}

// phase 2: one workgroup per row tile; G column groups of GS threads, each
// thread owns up to kMaxRpt rows of the tile
constexpr int kTileThreads = 256;
constexpr int kMaxRpt = 8;

template <typename T>
__global__ __launch_bounds__(kTileThreads) void rowtile_kernel(
    int64_t ntiles, const int32_t* __restrict__ tile_lo, const int64_t* __restrict__ tile_ptr,
    const Piece* __restrict__ pieces, const T* __restrict__ near, const T* __restrict__ U,
    const T* __restrict__ vec, const int32_t* __restrict__ perm, int64_t n, T alpha, T beta,
    T sigma2, T* __restrict__ z, int G, int GS) {
    __shared__ T red[kTileThreads * kMaxRpt];
    const int tid = threadIdx.x;
    const int g = tid / GS, rr = tid - g * GS;
    const int chunk = GS * kMaxRpt;  // rows handled per pass over the pieces
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int32_t t0 = tile_lo[t];
        const int mt_all = tile_lo[t + 1] - t0;
        const int64_t p0 = tile_ptr[t], p1 = tile_ptr[t + 1];
        for (int rb = 0; rb < mt_all; rb += chunk) {
            const int mt = (mt_all - rb) < chunk ? (mt_all - rb) : chunk;
            T acc[kMaxRpt];
#pragma unroll
            for (int k = 0; k < kMaxRpt; ++k) acc[k] = 0;
            for (int64_t p = p0; p < p1; ++p) {
                const Piece pc = pieces[p];
                const T* __restrict__ base = (pc.pool ? U : near) + pc.a_off + rb;
                const T* __restrict__ v = vec + pc.v_off;
                for (int c = g; c < pc.ncols; c += G) {
                    const T wv = v[c];
                    const T* __restrict__ col = base + (int64_t)c * pc.ld;
#pragma unroll
                    for (int k = 0; k < kMaxRpt; ++k) {
                        const int row = rr + GS * k;
                        if (row < mt) acc[k] += col[row] * wv;
                    }
                }
            }
            if (G > 1) {
#pragma unroll
                for (int k = 0; k < kMaxRpt; ++k) red[(g * kMaxRpt + k) * GS + rr] = acc[k];
                __syncthreads();
                if (g == 0) {
                    for (int q = 1; q < G; ++q)
#pragma unroll
                        for (int k = 0; k < kMaxRpt; ++k)
                            acc[k] += red[(q * kMaxRpt + k) * GS + rr];
                }
                __syncthreads();
            }
            if (g == 0) {
#pragma unroll
                for (int k = 0; k < kMaxRpt; ++k) {
                    const int row = rr + GS * k;
                    if (row < mt) {
                        const int64_t i = (int64_t)t0 + rb + row;
                        const int32_t pi = perm[i];
                        T out = alpha * (sigma2 != (T)0 ? acc[k] + sigma2 * vec[i] : acc[k]);
                        if (beta != (T)0) out += beta * z[pi];
                        z[pi] = out;
                    }
                }
            }
        }
    }
}

unsigned grid_cap(int64_t nb, int64_t cap) { return (unsigned)(nb < cap ? nb : cap); }

}  // namespace

hipError_t launch_near_assemble(const void* soa, int64_t n, int d, KernelFn kern,
                                const int4* blocks, int64_t nblocks, const int64_t* off, void* A,
                                int f64, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    const unsigned grid = grid_cap(nblocks, 1 << 20);
    if (f64)
        hipLaunchKernelGGL(near_kernel<double>, dim3(grid), dim3(256), 0, st, (const double*)soa,
                           n, d, KernelEval<double>(kern), blocks, nblocks, off, (double*)A);
    else
        hipLaunchKernelGGL(near_kernel<float>, dim3(grid), dim3(256), 0, st, (const float*)soa, n,
                           d, KernelEval<float>(kern), blocks, nblocks, off, (float*)A);
    return hipGetLastError();
}

hipError_t launch_extent(const int4* blocks, int64_t nb, int mode, int64_t mult,
                         const int32_t* rank, const int32_t* tile_of_point, int64_t* out,
                         hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(extent_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st,
                       blocks, nb, mode, mult, rank, tile_of_point, out);
    return hipGetLastError();
}

hipError_t launch_piece_fill(const int4* blocks, int64_t nblocks, const int32_t* rank,
                             const int32_t* tile_of_point, const int32_t* tile_lo,
                             const int64_t* piece_off, const int64_t* data_off,
                             const int64_t* vec_off_blk, int64_t vec_base, int pool,
                             int64_t piece_base, Piece* pieces, uint64_t* keys, uint32_t* vals,
                             hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(piece_fill_kernel, dim3((unsigned)((nblocks + 255) / 256)), dim3(256), 0,
                       st, blocks, nblocks, rank, tile_of_point, tile_lo, piece_off, data_off,
                       vec_off_blk, vec_base, pool, piece_base, pieces, keys, vals);
    return hipGetLastError();
}

hipError_t launch_piece_gather(const Piece* src, const uint32_t* order, int64_t npieces,
                               Piece* dst, hipStream_t st) {
    if (npieces == 0) return hipSuccess;
    hipLaunchKernelGGL(piece_gather_kernel, dim3((unsigned)((npieces + 255) / 256)), dim3(256), 0,
                       st, src, order, npieces, dst);
    return hipGetLastError();
}

hipError_t launch_tile_offsets(const uint64_t* sorted_tile, int64_t npieces, int64_t ntiles,
                               int64_t* tile_ptr, hipStream_t st) {
    hipLaunchKernelGGL(tile_ptr_kernel, dim3((unsigned)((ntiles + 1 + 255) / 256)), dim3(256), 0,
                       st, sorted_tile, npieces, ntiles, tile_ptr);
    return hipGetLastError();
}

hipError_t launch_gather_x(const void* x, const int32_t* perm, int64_t n, void* xm, int f64,
                           hipStream_t st) {
    if (f64)
        hipLaunchKernelGGL(gather_x_kernel<double>, dim3((unsigned)((n + 255) / 256)), dim3(256),
                           0, st, (const double*)x, perm, n, (double*)xm);
    else
        hipLaunchKernelGGL(gather_x_kernel<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           st, (const float*)x, perm, n, (float*)xm);
    return hipGetLastError();
}

hipError_t launch_far_phase1(const int4* adm, int64_t nadm, const int32_t* rank,
                             const int64_t* voff, const int64_t* toff, const void* V,
                             void* vecpool, int64_t n, int f64, hipStream_t st) {
    if (nadm == 0) return hipSuccess;
    const unsigned grid = grid_cap(nadm, 1 << 20);
    if (f64)
        hipLaunchKernelGGL(far_phase1_kernel<double>, dim3(grid), dim3(256), 0, st, adm, nadm,
                           rank, voff, toff, (const double*)V, (double*)vecpool, n);
    else
        hipLaunchKernelGGL(far_phase1_kernel<float>, dim3(grid), dim3(256), 0, st, adm, nadm,
                           rank, voff, toff, (const float*)V, (float*)vecpool, n);
    return hipGetLastError();
}

hipError_t launch_rowtile(int64_t ntiles, const int32_t* tile_lo, const int64_t* tile_ptr,
                          const Piece* pieces, const void* near, const void* U,
                          const void* vecpool, const int32_t* perm, int64_t n, double alpha,
                          double beta, double sigma2, void* z, int max_tile, int f64,
                          hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    // rows per group: the smallest power of two >= max_tile / kMaxRpt, at least 64
    // group size: the smallest power of two >= the largest tile (64..256);
    // tiles above GS * kMaxRpt rows are processed in several row passes
    int GS = 64;
    while (GS < max_tile && GS < kTileThreads) GS *= 2;
    const int G = kTileThreads / GS;
    const unsigned grid = grid_cap(ntiles, 1 << 20);
    if (f64)
        hipLaunchKernelGGL(rowtile_kernel<double>, dim3(grid), dim3(kTileThreads), 0, st, ntiles,
                           tile_lo, tile_ptr, pieces, (const double*)near, (const double*)U,
                           (const double*)vecpool, perm, n, alpha, beta, sigma2, (double*)z, G,
                           GS);
    else
        hipLaunchKernelGGL(rowtile_kernel<float>, dim3(grid), dim3(kTileThreads), 0, st, ntiles,
                           tile_lo, tile_ptr, pieces, (const float*)near, (const float*)U,
                           (const float*)vecpool, perm, n, (float)alpha, (float)beta,
                           (float)sigma2, (float*)z, G, GS);
    return hipGetLastError();
}

}  // namespace hmx
