// The far field without precomputation (Section 5.4: the ACA factors are not
// kept; every H-matrix-vector product approximates the admissible blocks
// again, batch by batch, and applies each batch's factors at once).
//
// The admissible blocks to approximate (every admissible leaf, or with the
// symmetric far field the primary ones) form a list cut into chunks whose ACA
// column scratch fits a budget (the paper's bs_ACA).  After a chunk's ACA,
// U_b and V_b of its blocks sit in the scratch (column-major, leading
// dimensions |tau_b| and |sigma_b|), and two kernels apply them:
//   * np_t:     t_b = V_b^T x|sigma_b (and, for a primary whose mirror
//               (sigma, tau) is another leaf, t'_b = U_b^T x|tau_b, since
//               A|sigma x tau ~ V_b U_b^T), one workgroup per block;
//   * np_apply: z|tau += alpha U_b t_b (and z|sigma += alpha V_b t'_b), one
//               workgroup per row tile (leaf cluster) that the chunk's blocks
//               touch, summing that tile's pieces in a fixed order, so the
//               product is deterministic and needs no atomics: within one
//               launch every tile is owned by one workgroup, and the chunks
//               run one after the other.
// The pieces (block, side) of each (chunk, tile) are sorted once at build
// time: key = chunk * 2^tbits + tile, stable, so a tile's pieces keep the
// list order, U side before the mirror side of the same block.
#include "hmx_internal.h"

namespace hmx {

namespace {

inline unsigned grid1(int64_t n, int b = 256) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + b - 1) / b, 1 << 20));
}

__device__ __forceinline__ bool has_mirror(int sym, int4 b) {
    return sym && (b.x != b.z || b.y != b.w);
}

__device__ __forceinline__ int64_t tiles_of(const int32_t* __restrict__ tile_of_point, int lo,
                                            int hi) {
    return (int64_t)tile_of_point[hi - 1] - tile_of_point[lo] + 1;
}

// the chunk holding list position q: bounds[c] <= q < bounds[c + 1]
__device__ __forceinline__ int chunk_of(const int64_t* __restrict__ bounds, int nch, int64_t q) {
    int lo = 0, hi = nch;  // bounds[lo] <= q < bounds[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bounds[mid] <= q)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__global__ void np_iota_kernel(int32_t* __restrict__ a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = (int32_t)i;
}

__global__ void np_piece_count_kernel(const int4* __restrict__ blk, int64_t nl, int sym,
                                      const int32_t* __restrict__ tile_of_point,
                                      int64_t* __restrict__ cnt) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nl;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int4 b = blk[q];
        int64_t c = tiles_of(tile_of_point, b.x, b.y);
        if (has_mirror(sym, b)) c += tiles_of(tile_of_point, b.z, b.w);
        cnt[q] = c;
    }
}

// piece p = off[q] + i of list entry q: its tiles of tau (side 0), then of
// sigma (side 1, mirrors only)
__global__ void np_piece_fill_kernel(const int4* __restrict__ blk, int64_t nl, int sym,
                                     const int32_t* __restrict__ tile_of_point,
                                     const int64_t* __restrict__ off,
                                     const int64_t* __restrict__ bounds, int nch, int tbits,
                                     uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                     int2* __restrict__ pcs) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nl;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int4 b = blk[q];
        const uint64_t c = (uint64_t)chunk_of(bounds, nch, q) << tbits;
        int64_t p = off[q];
        for (int side = 0; side < (has_mirror(sym, b) ? 2 : 1); ++side) {
            const int lo = side ? b.z : b.x, hi = side ? b.w : b.y;
            const int t0 = tile_of_point[lo], t1 = tile_of_point[hi - 1];
            for (int t = t0; t <= t1; ++t, ++p) {
                keys[p] = c | (uint64_t)t;
                vals[p] = (uint32_t)p;
                pcs[p] = make_int2((int)q, side);
            }
        }
    }
}

__global__ void np_seg_flags_kernel(const uint64_t* __restrict__ keys, int64_t np,
                                    int64_t* __restrict__ flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np;
         i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// sidx: exclusive scan of the flags (segment of each sorted position)
__global__ void np_seg_fill_kernel(const uint64_t* __restrict__ keys,
                                   const uint32_t* __restrict__ vals,
                                   const int2* __restrict__ pcs, const int64_t* __restrict__ sidx,
                                   int64_t np, int64_t nseg, int tbits,
                                   int64_t* __restrict__ seg_start, int32_t* __restrict__ seg_tile,
                                   int2* __restrict__ spcs) {
    const uint64_t tmask = ((uint64_t)1 << tbits) - 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np;
         i += (int64_t)gridDim.x * blockDim.x) {
        spcs[i] = pcs[vals[i]];
        if (i == 0 || keys[i] != keys[i - 1]) {
            const int64_t s = sidx[i];
            seg_start[s] = i;
            seg_tile[s] = (int32_t)(keys[i] & tmask);
        }
        if (i == 0) seg_start[nseg] = np;
    }
}

// cseg[c]: the first segment of chunk c (cseg[nch] = nseg)
__global__ void np_chunk_segs_kernel(const uint64_t* __restrict__ keys,
                                     const int64_t* __restrict__ seg_start, int64_t nseg,
                                     int tbits, int nch, int64_t* __restrict__ cseg) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nseg;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(keys[seg_start[s]] >> tbits);
        const int cp = s == 0 ? -1 : (int)(keys[seg_start[s - 1]] >> tbits);
        for (int k = cp + 1; k <= c; ++k) cseg[k] = s;
        if (s == nseg - 1)
            for (int k = c + 1; k <= nch; ++k) cseg[k] = nseg;
    }
}

// t_b = V_b^T x|sigma (and t'_b = U_b^T x|tau for a mirrored primary): one
// workgroup of four waves per block, a wave per column, lane-strided partial
// sums combined by a butterfly (a fixed order)
template <typename T>
__global__ __launch_bounds__(256) void np_t_kernel(const int4* __restrict__ blk, int64_t nbk,
                                                   const int32_t* __restrict__ rank,
                                                   const int64_t* __restrict__ cu,
                                                   const int64_t* __restrict__ cv, int64_t ubase,
                                                   int64_t vbase, const T* __restrict__ U,
                                                   const T* __restrict__ V,
                                                   const T* __restrict__ xm, int kmax, int sym,
                                                   T* __restrict__ t, T* __restrict__ t2) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t q = blockIdx.x; q < nbk; q += gridDim.x) {
        const int4 b = blk[q];
        const int r = max(rank[q], 0);
        const int m = b.y - b.x, nn = b.w - b.z;
        const T* Vb = V + (cv[q] - vbase);
        for (int k = w; k < r; k += 4) {
            const T* col = Vb + (int64_t)k * nn;
            T s = 0;
            for (int j = lane; j < nn; j += 64) s += col[j] * xm[b.z + j];
            s = wave_sum(s);
            if (lane == 0) t[q * kmax + k] = s;
        }
        if (has_mirror(sym, b)) {
            const T* Ub = U + (cu[q] - ubase);
            for (int k = w; k < r; k += 4) {
                const T* col = Ub + (int64_t)k * m;
                T s = 0;
                for (int i = lane; i < m; i += 64) s += col[i] * xm[b.x + i];
                s = wave_sum(s);
                if (lane == 0) t2[q * kmax + k] = s;
            }
        }
    }
}

// z|tile += alpha sum over the tile's pieces of F_b(tile rows) t_b, one
// workgroup per (chunk, tile) segment; q indexes the whole list, the
// chunk's blocks start at b0 (t and t2 are chunk-local)
template <typename T>
__global__ __launch_bounds__(256) void np_apply_kernel(
    const int64_t* __restrict__ seg_start, const int32_t* __restrict__ seg_tile, int64_t s0,
    int64_t ns, const int2* __restrict__ spcs, const int4* __restrict__ blk,
    const int32_t* __restrict__ rank, const int64_t* __restrict__ cu,
    const int64_t* __restrict__ cv, int64_t ubase, int64_t vbase, int64_t b0,
    const T* __restrict__ U, const T* __restrict__ V, const T* __restrict__ t,
    const T* __restrict__ t2, int kmax, const int32_t* __restrict__ tile_lo,
    const int32_t* __restrict__ perm, T alpha, T* __restrict__ z) {
    for (int64_t s = s0 + blockIdx.x; s < s0 + ns; s += gridDim.x) {
        const int tile = seg_tile[s];
        const int r0 = tile_lo[tile], r1 = tile_lo[tile + 1];
        const int64_t p0 = seg_start[s], p1 = seg_start[s + 1];
        for (int row = r0 + (int)threadIdx.x; row < r1; row += blockDim.x) {
            T acc = 0;
            for (int64_t p = p0; p < p1; ++p) {
                const int2 pc = spcs[p];
                const int4 b = blk[pc.x];
                const int r = max(rank[pc.x], 0);
                const T* F;
                const T* tv;
                int64_t ld;
                if (pc.y == 0) {
                    ld = b.y - b.x;
                    F = U + (cu[pc.x] - ubase) + (row - b.x);
                    tv = t + (pc.x - b0) * kmax;
                } else {
                    ld = b.w - b.z;
                    F = V + (cv[pc.x] - vbase) + (row - b.z);
                    tv = t2 + (pc.x - b0) * kmax;
                }
                for (int k = 0; k < r; ++k) acc += F[k * ld] * tv[k];
            }
            const int64_t o = perm[row];
            z[o] = z[o] + alpha * acc;
        }
    }
}

}  // namespace

hipError_t launch_np_iota(int32_t* a, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(np_iota_kernel, dim3(grid1(n)), dim3(256), 0, st, a, n);
    return hipGetLastError();
}

hipError_t launch_np_piece_count(const int4* blk, int64_t nl, int sym,
                                 const int32_t* tile_of_point, int64_t* cnt, hipStream_t st) {
    if (nl <= 0) return hipSuccess;
    hipLaunchKernelGGL(np_piece_count_kernel, dim3(grid1(nl)), dim3(256), 0, st, blk, nl, sym,
                       tile_of_point, cnt);
    return hipGetLastError();
}

hipError_t launch_np_piece_fill(const int4* blk, int64_t nl, int sym,
                                const int32_t* tile_of_point, const int64_t* off,
                                const int64_t* bounds, int nch, int tbits, uint64_t* keys,
                                uint32_t* vals, int2* pcs, hipStream_t st) {
    if (nl <= 0) return hipSuccess;
    hipLaunchKernelGGL(np_piece_fill_kernel, dim3(grid1(nl)), dim3(256), 0, st, blk, nl, sym,
                       tile_of_point, off, bounds, nch, tbits, keys, vals, pcs);
    return hipGetLastError();
}

hipError_t launch_np_seg_flags(const uint64_t* keys, int64_t np, int64_t* flag, hipStream_t st) {
    if (np <= 0) return hipSuccess;
    hipLaunchKernelGGL(np_seg_flags_kernel, dim3(grid1(np)), dim3(256), 0, st, keys, np, flag);
    return hipGetLastError();
}

hipError_t launch_np_seg_fill(const uint64_t* keys, const uint32_t* vals, const int2* pcs,
                              const int64_t* sidx, int64_t np, int64_t nseg, int tbits,
                              int64_t* seg_start, int32_t* seg_tile, int2* spcs, hipStream_t st) {
    if (np <= 0) return hipSuccess;
    hipLaunchKernelGGL(np_seg_fill_kernel, dim3(grid1(np)), dim3(256), 0, st, keys, vals, pcs,
                       sidx, np, nseg, tbits, seg_start, seg_tile, spcs);
    return hipGetLastError();
}

hipError_t launch_np_chunk_segs(const uint64_t* keys, const int64_t* seg_start, int64_t nseg,
                                int tbits, int nch, int64_t* cseg, hipStream_t st) {
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(np_chunk_segs_kernel, dim3(grid1(nseg)), dim3(256), 0, st, keys,
                       seg_start, nseg, tbits, nch, cseg);
    return hipGetLastError();
}

hipError_t launch_np_t(const int4* blk, int64_t nbk, const int32_t* rank, const int64_t* cu,
                       const int64_t* cv, int64_t ubase, int64_t vbase, const void* U,
                       const void* V, const void* xm, int kmax, int sym, void* t, void* t2,
                       int f64, hipStream_t st) {
    if (nbk <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>(nbk, 1 << 20);
    if (f64)
        hipLaunchKernelGGL(np_t_kernel<double>, dim3(g), dim3(256), 0, st, blk, nbk, rank, cu, cv,
                           ubase, vbase, (const double*)U, (const double*)V, (const double*)xm,
                           kmax, sym, (double*)t, (double*)t2);
    else
        hipLaunchKernelGGL(np_t_kernel<float>, dim3(g), dim3(256), 0, st, blk, nbk, rank, cu, cv,
                           ubase, vbase, (const float*)U, (const float*)V, (const float*)xm, kmax,
                           sym, (float*)t, (float*)t2);
    return hipGetLastError();
}

hipError_t launch_np_apply(const int64_t* seg_start, const int32_t* seg_tile, int64_t s0,
                           int64_t ns, const int2* spcs, const int4* blk, const int32_t* rank,
                           const int64_t* cu, const int64_t* cv, int64_t ubase, int64_t vbase,
                           int64_t b0, const void* U, const void* V, const void* t,
                           const void* t2, int kmax, const int32_t* tile_lo,
                           const int32_t* perm, double alpha, void* z, int max_tile, int f64,
                           hipStream_t st) {
    if (ns <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>(ns, 1 << 20);
    const int nt = (int)std::min<int64_t>(256, std::max<int64_t>(64, (max_tile + 63) / 64 * 64));
    if (f64)
        hipLaunchKernelGGL(np_apply_kernel<double>, dim3(g), dim3(nt), 0, st, seg_start, seg_tile,
                           s0, ns, spcs, blk, rank, cu, cv, ubase, vbase, b0, (const double*)U,
                           (const double*)V, (const double*)t, (const double*)t2, kmax, tile_lo,
                           perm, alpha, (double*)z);
    else
        hipLaunchKernelGGL(np_apply_kernel<float>, dim3(g), dim3(nt), 0, st, seg_start, seg_tile,
                           s0, ns, spcs, blk, rank, cu, cv, ubase, vbase, b0, (const float*)U,
                           (const float*)V, (const float*)t, (const float*)t2, kmax, tile_lo,
                           perm, (float)alpha, (float*)z);
    return hipGetLastError();
}

}  // namespace hmx
