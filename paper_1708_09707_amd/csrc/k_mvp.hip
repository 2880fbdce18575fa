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

// 16-byte vector of T: 4 floats or 2 doubles
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = float4;
    static constexpr int n = 4;
};
template <>
struct Vec16<double> {
    using type = double2;
    static constexpr int n = 2;
};

template <typename V, typename T>
__device__ __forceinline__ T vget(const V& v, int e);
template <>
__device__ __forceinline__ float vget<float4, float>(const float4& v, int e) {
    return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}
template <>
__device__ __forceinline__ double vget<double2, double>(const double2& v, int e) {
    return e == 0 ? v.x : v.y;
}

// phase 1: t_b[l] = sum_j V_b[j, l] x[slo + j]; one wave per column of the
// flattened list of all factor columns (col_block maps a column to its leaf)
template <typename T>
__global__ __launch_bounds__(256) void far_phase1_kernel(
    const int4* __restrict__ adm, const int32_t* __restrict__ col_block,
    const int64_t* __restrict__ voff, const int64_t* __restrict__ toff, const T* __restrict__ V,
    T* __restrict__ vec, int64_t n, int64_t ncols_total) {
    using V16 = typename Vec16<T>::type;
    constexpr int VEC = Vec16<T>::n;
    const int lane = threadIdx.x & 63;
    const int64_t k = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    if (k >= ncols_total) return;
    const int b = col_block[k];
    const int4 bl = adm[b];
    const int nc = bl.w - bl.z;
    const int l = (int)(k - toff[b]);
    const int64_t cofs = voff[b] + (int64_t)l * nc;
    const T* __restrict__ col = V + cofs;
    const T* __restrict__ xs = vec + bl.z;
    T acc = 0;
    if (((cofs | (int64_t)bl.z | (int64_t)nc) % VEC) == 0) {
        const V16* __restrict__ c16 = (const V16*)col;
        const V16* __restrict__ x16 = (const V16*)xs;
        const int nv = nc / VEC;
        int j = lane;
        for (; j + 64 < nv; j += 128) {
            const V16 a0 = c16[j], a1 = c16[j + 64];
            const V16 x0 = x16[j], x1 = x16[j + 64];
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                acc += vget<V16, T>(a0, e) * vget<V16, T>(x0, e) +
                       vget<V16, T>(a1, e) * vget<V16, T>(x1, e);
        }
        for (; j < nv; j += 64) {
            const V16 a0 = c16[j], x0 = x16[j];
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc += vget<V16, T>(a0, e) * vget<V16, T>(x0, e);
        }
    } else {
        for (int j = lane; j < nc; j += 64) acc += col[j] * xs[j];
    }
    acc = wave_sum(acc);
    if (lane == 0) vec[n + k] = acc;
}

// out[0] = max, out[1] = sum of n int32 values (integer atomics: order-free)
__global__ void int_stats_kernel(const int32_t* __restrict__ a, int64_t n,
                                 unsigned long long* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int32_t v = i < n ? a[i] : 0;
    int32_t mx = v;
    int64_t sm = v;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t u = __shfl_xor(mx, o, 64);
        mx = u > mx ? u : mx;
        sm += __shfl_xor(sm, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&out[0], (unsigned long long)mx);
        atomicAdd(&out[1], (unsigned long long)sm);
    }
}

// column -> admissible leaf map for the flattened factor columns
__global__ void col_block_kernel(const int32_t* __restrict__ rank, const int64_t* __restrict__ toff,
                                 int64_t nadm, int32_t* __restrict__ col_block) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nadm) return;
    const int64_t o = toff[b];
    for (int l = 0; l < rank[b]; ++l) col_block[o + l] = (int32_t)b;
}

// phase 2: one workgroup per row tile.  The 4 waves split into G = 4 * (64/L)
// column groups of L lanes; lane q of a group owns RV vectors of VEC rows
// (vector v*L + q), so a group covers L*RV*VEC rows with 16-byte loads when
// the piece is aligned (scalar loads otherwise).  Groups take interleaved
// columns of every piece; their partial rows are summed in LDS in a fixed
// order and the tile is scattered to the original order.
constexpr int kTileThreads = 256;

template <typename T, int RV>
__global__ __launch_bounds__(kTileThreads) void rowtile_kernel(
    int64_t ntiles, const int32_t* __restrict__ tile_lo, const int64_t* __restrict__ tile_ptr,
    const Piece* __restrict__ pieces, const T* __restrict__ near, const T* __restrict__ U,
    const T* __restrict__ vec, const int32_t* __restrict__ perm, T alpha, T beta, T sigma2,
    T* __restrict__ z, int L) {
    using V16 = typename Vec16<T>::type;
    constexpr int VEC = Vec16<T>::n;
    extern __shared__ unsigned char red_raw[];
    T* red = (T*)red_raw;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int S = 64 / L;
    const int G = 4 * S;
    const int g = w * S + lane / L;
    const int q = lane % L;
    const int rpg = L * RV * VEC;  // rows per group pass
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int32_t t0 = tile_lo[t];
        const int mt = tile_lo[t + 1] - t0;
        const int64_t p0 = tile_ptr[t], p1 = tile_ptr[t + 1];
        for (int rb = 0; rb < mt; rb += rpg) {
            const int mc = (mt - rb) < rpg ? (mt - rb) : rpg;
            T acc[RV][VEC];
#pragma unroll
            for (int v = 0; v < RV; ++v)
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[v][e] = 0;
            for (int64_t p = p0; p < p1; ++p) {
                const Piece pc = pieces[p];
                const int64_t aoff = pc.a_off + rb;
                const T* __restrict__ base = (pc.pool ? U : near) + aoff;
                const T* __restrict__ wv = vec + pc.v_off;
                const int ld = pc.ld, ncols = pc.ncols;
                if (((aoff | (int64_t)ld | (int64_t)mt) % VEC) == 0) {
                    int c = g;
                    for (; c + 3 * G < ncols; c += 4 * G) {
                        const T w0 = wv[c], w1 = wv[c + G], w2 = wv[c + 2 * G], w3 = wv[c + 3 * G];
                        const V16* c0 = (const V16*)(base + (int64_t)c * ld);
                        const V16* c1 = (const V16*)(base + (int64_t)(c + G) * ld);
                        const V16* c2 = (const V16*)(base + (int64_t)(c + 2 * G) * ld);
                        const V16* c3 = (const V16*)(base + (int64_t)(c + 3 * G) * ld);
#pragma unroll
                        for (int v = 0; v < RV; ++v) {
                            const int vi = v * L + q;
                            if (vi * VEC < mc) {
                                const V16 a0 = c0[vi], a1 = c1[vi], a2 = c2[vi], a3 = c3[vi];
#pragma unroll
                                for (int e = 0; e < VEC; ++e)
                                    acc[v][e] += vget<V16, T>(a0, e) * w0 + vget<V16, T>(a1, e) * w1 +
                                                 vget<V16, T>(a2, e) * w2 + vget<V16, T>(a3, e) * w3;
                            }
                        }
                    }
                    for (; c < ncols; c += G) {
                        const T w0 = wv[c];
                        const V16* c0 = (const V16*)(base + (int64_t)c * ld);
#pragma unroll
                        for (int v = 0; v < RV; ++v) {
                            const int vi = v * L + q;
                            if (vi * VEC < mc) {
                                const V16 a0 = c0[vi];
#pragma unroll
                                for (int e = 0; e < VEC; ++e) acc[v][e] += vget<V16, T>(a0, e) * w0;
                            }
                        }
                    }
                } else {
                    for (int c = g; c < ncols; c += G) {
                        const T w0 = wv[c];
                        const T* __restrict__ col = base + (int64_t)c * ld;
#pragma unroll
                        for (int v = 0; v < RV; ++v)
#pragma unroll
                            for (int e = 0; e < VEC; ++e) {
                                const int row = (v * L + q) * VEC + e;
                                if (row < mc) acc[v][e] += col[row] * w0;
                            }
                    }
                }
            }
            // sum the G partial row sets in a fixed order
#pragma unroll
            for (int v = 0; v < RV; ++v)
#pragma unroll
                for (int e = 0; e < VEC; ++e) red[g * rpg + (v * L + q) * VEC + e] = acc[v][e];
            __syncthreads();
            for (int row = tid; row < mc; row += kTileThreads) {
                T sum = red[row];
                for (int gg = 1; gg < G; ++gg) sum += red[gg * rpg + row];
                const int64_t i = (int64_t)t0 + rb + row;
                const int32_t pi = perm[i];
                T out = alpha * (sigma2 != (T)0 ? sum + sigma2 * vec[i] : sum);
                if (beta != (T)0) out += beta * z[pi];
                z[pi] = out;
            }
            __syncthreads();
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

hipError_t launch_int_stats(const int32_t* a, int64_t n, unsigned long long* out,
                            hipStream_t st) {
    hipError_t e = hipMemsetAsync(out, 0, 2 * sizeof(unsigned long long), st);
    if (e != hipSuccess || n == 0) return e;
    hipLaunchKernelGGL(int_stats_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a,
                       n, out);
    return hipGetLastError();
}

hipError_t launch_col_block(const int32_t* rank, const int64_t* toff, int64_t nadm,
                            int32_t* col_block, hipStream_t st) {
    if (nadm == 0) return hipSuccess;
    hipLaunchKernelGGL(col_block_kernel, dim3((unsigned)((nadm + 255) / 256)), dim3(256), 0, st,
                       rank, toff, nadm, col_block);
    return hipGetLastError();
}

hipError_t launch_far_phase1(const int4* adm, const int32_t* col_block, const int64_t* voff,
                             const int64_t* toff, int64_t ncols_total, const void* V,
                             void* vecpool, int64_t n, int f64, hipStream_t st) {
    if (ncols_total == 0) return hipSuccess;
    const int64_t nblk = (ncols_total + 3) / 4;  // 4 waves (columns) per workgroup
    if (nblk > 0x7fffffffll) return hipErrorInvalidValue;
    if (f64)
        hipLaunchKernelGGL(far_phase1_kernel<double>, dim3((unsigned)nblk), dim3(256), 0, st, adm,
                           col_block, voff, toff, (const double*)V, (double*)vecpool, n,
                           ncols_total);
    else
        hipLaunchKernelGGL(far_phase1_kernel<float>, dim3((unsigned)nblk), dim3(256), 0, st, adm,
                           col_block, voff, toff, (const float*)V, (float*)vecpool, n,
                           ncols_total);
    return hipGetLastError();
}

template <typename T>
static hipError_t rowtile_dispatch(int64_t ntiles, const int32_t* tile_lo, const int64_t* tile_ptr,
                                   const Piece* pieces, const void* near, const void* U,
                                   const void* vecpool, const int32_t* perm, double alpha,
                                   double beta, double sigma2, void* z, int max_tile,
                                   hipStream_t st) {
    constexpr int VEC = Vec16<T>::n;
    const int need = (max_tile + VEC - 1) / VEC;  // vectors per tile column
    int L = 8, RV = 1;
    while (L < need && L < 64) L *= 2;
    while (L * RV < need && RV < 8) RV *= 2;
    const size_t lds = (size_t)(4 * (64 / L)) * L * RV * VEC * sizeof(T);
    const unsigned grid = grid_cap(ntiles, 1 << 20);
#define HMX_ROWTILE(RVV)                                                                          \
    hipLaunchKernelGGL((rowtile_kernel<T, RVV>), dim3(grid), dim3(kTileThreads), lds, st, ntiles, \
                       tile_lo, tile_ptr, pieces, (const T*)near, (const T*)U, (const T*)vecpool, \
                       perm, (T)alpha, (T)beta, (T)sigma2, (T*)z, L)
    switch (RV) {
        case 1: HMX_ROWTILE(1); break;
        case 2: HMX_ROWTILE(2); break;
        case 4: HMX_ROWTILE(4); break;
        default: HMX_ROWTILE(8); break;
    }
#undef HMX_ROWTILE
    return hipGetLastError();
}

hipError_t launch_rowtile(int64_t ntiles, const int32_t* tile_lo, const int64_t* tile_ptr,
                          const Piece* pieces, const void* near, const void* U,
                          const void* vecpool, const int32_t* perm, int64_t n, double alpha,
                          double beta, double sigma2, void* z, int max_tile, int f64,
                          hipStream_t st) {
    (void)n;
    if (ntiles == 0) return hipSuccess;
    if (f64)
        return rowtile_dispatch<double>(ntiles, tile_lo, tile_ptr, pieces, near, U, vecpool, perm,
                                        alpha, beta, sigma2, z, max_tile, st);
    return rowtile_dispatch<float>(ntiles, tile_lo, tile_ptr, pieces, near, U, vecpool, perm,
                                   alpha, beta, sigma2, z, max_tile, st);
}

}  // namespace hmx
