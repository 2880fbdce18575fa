// Far-field phase 1 of the H-matrix-vector product, t_b = V_b^T x|sigma_b for
// every admissible leaf b (Algorithm 3, the first product of a low-rank
// block; batched over all blocks as in Section 5.4.1), and the symmetric
// storage of the far field.
//
// The factor V_b is read row tile by row tile, like the near field and U in
// phase 2: its rows are the points of sigma_b, so the part of V_b inside one
// row tile (leaf cluster) T is a "source piece", stored with the tile's
// other source pieces as one contiguous column-major ld_T x C matrix.  One
// workgroup per tile streams that matrix once and forms, for every column,
// the partial inner product with x|T; a second pass sums each column's
// partials over the tiles of sigma_b in tile order (a fixed order, so the
// product is deterministic).
//
// Where the source pieces come from:
//   * plain storage: V_b of every block, in a pool of its own;
//   * symmetric far field: the kernel matrix is symmetric, so the block
//     (sigma, tau) mirroring an admissible (tau, sigma) satisfies
//     A|sigma x tau ~ V U^T.  Only the block with tau before sigma (the
//     "primary") is approximated; its U and V rows are the row-tile factor
//     pieces of (tau, sigma) and of (sigma, tau) respectively, so the
//     factor pool that phase 2 streams also holds every V: the source
//     pieces of a block are its mirror's factor pieces.  Blocks that are
//     their own mirror (tau = sigma, only possible for clusters of
//     coincident points) keep their V in the separate pool.
#include "hmx_internal.h"

namespace hmx {

namespace {

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int p1_ld(int rows, int R) { return (rows + R - 1) / R * R; }

// 16-byte vector -> values of T (storage S: double, float or bfloat16 bits)
template <typename S, typename T>
struct P1Dec;
template <>
struct P1Dec<double, double> {
    static constexpr int n = 2;
    static __device__ __forceinline__ void get(const u32x4& r, double* o) {
        o[0] = __hiloint2double((int)r[1], (int)r[0]);
        o[1] = __hiloint2double((int)r[3], (int)r[2]);
    }
};
template <>
struct P1Dec<float, float> {
    static constexpr int n = 4;
    static __device__ __forceinline__ void get(const u32x4& r, float* o) {
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = __uint_as_float(r[k]);
    }
};
template <>
struct P1Dec<uint16_t, float> {
    static constexpr int n = 8;
    static __device__ __forceinline__ void get(const u32x4& r, float* o) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            o[2 * k] = __uint_as_float(r[k] << 16);
            o[2 * k + 1] = __uint_as_float(r[k] & 0xffff0000u);
        }
    }
};

constexpr int kP1Threads = 256;
constexpr int kP1Cols = 16;     // columns per lane group in flight
constexpr int kP1Stage = 2048;  // rows of x a tile stages in LDS (taller tiles read x directly)

// Tile pass.  meta[ms * t + 1] = first source column of tile t (tile t + 1's
// entry ends it), meta[ms * t + 2] = data offset of the tile's matrix in
// pool.  The tile's x rows are staged in LDS.  The workgroup's 256 threads
// form groups of L lanes; a group takes kP1Cols consecutive columns at a
// time, lane q covering 16-byte row vectors q, q + L, ... of each, and sums
// each lane's products in registers; the kP1Cols sums are then reduced over
// the group's lanes by a butterfly that halves the values per lane at each
// of the first four exchanges (one shuffle per column instead of log2 L),
// after which every lane holds the total of one column.  Narrow groups (16
// lanes) give each lane several row vectors per column before the
// reduction, so the exchanges are a small share of the work on tall tiles.
template <typename S, typename T, int L>
__global__ __launch_bounds__(kP1Threads) void p1_tile_kernel(
    int64_t ntiles, const int32_t* __restrict__ tile_lo, const int64_t* __restrict__ meta, int ms,
    int R, const S* __restrict__ pool, const T* __restrict__ vec, T* __restrict__ partial,
    int64_t pbase) {
    constexpr int VS = P1Dec<S, T>::n;
    constexpr int G = kP1Threads / L;
    static_assert(L >= 8 && L <= 64, "groups of 8, 16, 32 or 64 lanes");
    // halving exchanges (at most four: 16 values per lane down to one);
    // with 8 lanes three, and each lane keeps two column totals
    constexpr int HS = L >= 16 ? 4 : 3;
    constexpr int KEEP = kP1Cols >> HS;
    __shared__ T sx[kP1Stage];
    const int g = threadIdx.x / L;
    const int q = threadIdx.x % L;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t c0 = meta[ms * t + 1];
        const int nc = (int)(meta[ms * (t + 1) + 1] - c0);
        if (nc <= 0) continue;
        const int32_t r0 = tile_lo[t];
        const int mt = tile_lo[t + 1] - r0;
        const int ld = p1_ld(mt, R);
        const int nvec = ld / VS;
        const S* __restrict__ base = pool + meta[ms * t + 2];
        // x of the tile (rows past it read as zero)
        const bool staged = ld <= kP1Stage;
        if (staged) {
            for (int i = threadIdx.x; i < ld; i += kP1Threads) sx[i] = i < mt ? vec[r0 + i] : (T)0;
            __syncthreads();
        }
        for (int cb = g * kP1Cols; cb < nc; cb += G * kP1Cols) {
            T acc[kP1Cols];
#pragma unroll
            for (int u = 0; u < kP1Cols; ++u) acc[u] = 0;
            for (int vi = q; vi < nvec; vi += L) {
                u32x4 raw[kP1Cols];
#pragma unroll
                for (int u = 0; u < kP1Cols; ++u) {
                    const int c = cb + u < nc ? cb + u : nc - 1;  // past the end: never stored
                    raw[u] = __builtin_nontemporal_load((const u32x4*)(base + (int64_t)c * ld) + vi);
                }
                T xv[VS];
#pragma unroll
                for (int e = 0; e < VS; ++e) {
                    const int row = vi * VS + e;
                    xv[e] = staged ? sx[row] : (row < mt ? vec[r0 + row] : (T)0);
                }
#pragma unroll
                for (int u = 0; u < kP1Cols; ++u) {
                    T a[VS];
                    P1Dec<S, T>::get(raw[u], a);
#pragma unroll
                    for (int e = 0; e < VS; ++e) acc[u] += a[e] * xv[e];
                }
            }
            // butterfly over the group's lanes: the first HS exchanges (L/2,
            // L/4, ...) halve the values held per lane, the rest add the one
            // left; each lane ends with the totals of KEEP consecutive columns
            int off = 0;
#pragma unroll
            for (int s = 0, m = L / 2; m >= 1; ++s, m >>= 1) {
                const bool hi = (q & m) != 0;
                if (s < HS) {
                    const int h = kP1Cols >> (s + 1);
#pragma unroll
                    for (int i = 0; i < kP1Cols / 2; ++i) {
                        if (i < h) {
                            const T send = hi ? acc[i] : acc[i + h];
                            const T keep = hi ? acc[i + h] : acc[i];
                            acc[i] = keep + __shfl_xor(send, m, 64);
                        }
                    }
                    if (hi) off += h;
                } else {
                    acc[0] += __shfl_xor(acc[0], m, 64);
                }
            }
            if ((q & (L >= 16 ? L / 16 - 1 : 0)) == 0) {
#pragma unroll
                for (int i = 0; i < KEEP; ++i)
                    if (cb + off + i < nc) partial[pbase + c0 + cb + off + i] = acc[i];
            }
        }
        if (staged) __syncthreads();  // sx is refilled by the next tile
    }
}

// Column sums: target column k (t entry k of the vector pool) adds the
// partials of its nt source pieces, rec[k] = {base (low, high), nt, l}:
// partial[pfc[base + j] + l] for j = 0 .. nt - 1 in tile order.
template <typename T>
__global__ void p1_reduce_kernel(const int4* __restrict__ rec, int64_t ncols,
                                 const int64_t* __restrict__ pfc, const T* __restrict__ partial,
                                 T* __restrict__ vec, int64_t n) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= ncols) return;
    const int4 r = rec[k];
    const int64_t b = (int64_t)(((uint64_t)(uint32_t)r.y << 32) | (uint32_t)r.x);
    T s = 0;
    for (int j = 0; j < r.z; ++j) s += partial[pfc[b + j] + r.w];
    vec[n + k] = s;
}

// records of the target columns of every admissible leaf c: its source
// pieces start at pbase[c] (nt of them)
__global__ void p1_rec_kernel(const int32_t* __restrict__ rank, const int64_t* __restrict__ toff,
                              const int64_t* __restrict__ sbase, const int32_t* __restrict__ snt,
                              int64_t nadm, int4* __restrict__ rec) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nadm) return;
    const int r = rank[c];
    const int64_t o = toff[c];
    const int64_t b = sbase[c];
    const int nt = snt[c];
    for (int l = 0; l < r; ++l) rec[o + l] = int4{(int)(uint32_t)b, (int)(uint32_t)(b >> 32), nt, l};
}

// where the phase-1 sources of leaf c start in pfc: its own V pieces (kept
// leaves: vbase + cntv[c], sigma_c's row tiles) or its mirror's factor
// pieces (cnt[partner], the same row tiles)
__global__ void p1_source_kernel(int64_t nadm, const int32_t* __restrict__ partner,
                                 const int64_t* __restrict__ cnt, const int64_t* __restrict__ cntv,
                                 int64_t vbase, int64_t* __restrict__ sbase,
                                 int32_t* __restrict__ snt) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nadm) return;
    const int32_t p = partner ? partner[c] : (int32_t)c;
    if (p == (int32_t)c) {
        sbase[c] = vbase + cntv[c];
        snt[c] = (int32_t)(cntv[c + 1] - cntv[c]);
    } else {
        sbase[c] = cnt[p];
        snt[c] = (int32_t)(cnt[p + 1] - cnt[p]);
    }
}

// first source column of every piece, indexed by its position before the
// sort by tile (order[i] = that position of sorted piece i); colscan: the
// sorted pieces' first factor columns; only factor pieces (blk >= 0) with
// order[i] < limit are written
__global__ void pfc_kernel(const Piece* __restrict__ sorted, const uint32_t* __restrict__ order,
                           const int64_t* __restrict__ colscan, int64_t np, int64_t limit,
                           int64_t cbase, int64_t* __restrict__ pfc) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= np) return;
    const uint32_t o = order[i];
    if (sorted[i].blk >= 0 && (int64_t)o < limit) pfc[o] = cbase + colscan[i];
}

// symmetric far field: key (tlo, slo) of every admissible leaf (the leaves
// partition I x I, so the pair names one leaf)
__global__ void mirror_keys_kernel(const int4* __restrict__ adm, int64_t nadm,
                                   uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nadm) return;
    const int4 bl = adm[b];
    keys[b] = ((uint64_t)(uint32_t)bl.x << 32) | (uint32_t)bl.z;
    vals[b] = (uint32_t)b;
}

// partner[b] = the leaf (slo, tlo) of leaf (tlo, slo); -1 when the partition
// has no mirror (*bad set)
__global__ void mirror_find_kernel(const int4* __restrict__ adm, int64_t nadm,
                                   const uint64_t* __restrict__ keys,
                                   const uint32_t* __restrict__ vals,
                                   int32_t* __restrict__ partner, int* __restrict__ bad) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nadm) return;
    const int4 bl = adm[b];
    const uint64_t want = ((uint64_t)(uint32_t)bl.z << 32) | (uint32_t)bl.x;
    int64_t lo = 0, hi = nadm;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < want)
            lo = mid + 1;
        else
            hi = mid;
    }
    int32_t p = -1;
    if (lo < nadm && keys[lo] == want) {
        const int4 o = adm[vals[lo]];
        if (o.x == bl.z && o.y == bl.w && o.z == bl.x && o.w == bl.y) p = (int32_t)vals[lo];
    }
    partner[b] = p;
    if (p < 0) atomicOr(bad, 1);
}

// flag[b] = 1 for the leaves the ACA approximates: every leaf (sym = 0) or
// the primary ones, tlo <= slo (sym = 1)
__global__ void primary_flags_kernel(const int4* __restrict__ adm, int64_t nadm, int sym,
                                     int64_t* __restrict__ flag) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nadm) return;
    const int4 bl = adm[b];
    flag[b] = (!sym || bl.x <= bl.z) ? 1 : 0;
}

// the flagged leaves in order (pos: exclusive scan of the 0/1 flags, nadm + 1
// entries, so leaf b is flagged when pos[b + 1] > pos[b])
__global__ void gather_list_kernel(const int64_t* __restrict__ pos,
                                   int64_t nadm, const int4* __restrict__ adm,
                                   const int32_t* __restrict__ level,
                                   const int32_t* __restrict__ rt, int32_t* __restrict__ list,
                                   int4* __restrict__ blocks, int32_t* __restrict__ lev,
                                   int32_t* __restrict__ rt_out) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nadm || pos[b + 1] == pos[b]) return;
    const int64_t i = pos[b];
    list[i] = (int32_t)b;
    blocks[i] = adm[b];
    lev[i] = level[b];
    if (rt) rt_out[i] = rt[b];
}

// results of the ACA list back to the leaves: rank and steps of list entry
// i go to its leaf (steps of a mirror are 0: it is not approximated); the
// row factor of a leaf is its U (primary) or its mirror's V, its phase-1
// source V is its own (kept only for leaves stored with a V pool)
__global__ void scatter_list_kernel(const int32_t* __restrict__ list, int64_t nl,
                                    const int32_t* __restrict__ partner,
                                    const int32_t* __restrict__ rank_l,
                                    const int32_t* __restrict__ steps_l,
                                    const int64_t* __restrict__ ue, const int64_t* __restrict__ ve,
                                    int32_t* __restrict__ rank, int32_t* __restrict__ steps,
                                    int64_t* __restrict__ rfo, int64_t* __restrict__ vfo) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nl) return;
    const int32_t b = list ? list[i] : (int32_t)i;
    rank[b] = rank_l[i];
    steps[b] = steps_l[i];
    if (rfo) rfo[b] = ue[i];
    if (vfo) vfo[b] = ve[i];
    if (partner) {
        const int32_t p = partner[b];
        if (p != b) {
            rank[p] = rank_l[i];
            steps[p] = 0;
            if (rfo) rfo[p] = ve[i];
        }
    }
}

// pieces of the V pool: cnt[b] = row tiles covered by sigma_b for the leaves
// kept with a V (every leaf, or with a mirror table only the leaves that are
// their own mirror) of nonzero rank, else 0
__global__ void vpiece_count_kernel(const int4* __restrict__ adm, int64_t nadm,
                                    const int32_t* __restrict__ rank,
                                    const int32_t* __restrict__ partner,
                                    const int32_t* __restrict__ tile_of_point,
                                    int64_t* __restrict__ cnt) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nadm) return;
    const int4 bl = adm[b];
    const bool kept = !partner || partner[b] == (int32_t)b;
    cnt[b] = (kept && rank[b] > 0)
                 ? (int64_t)(tile_of_point[bl.w - 1] - tile_of_point[bl.z] + 1)
                 : 0;
}

// one V piece per (kept leaf, row tile of sigma_b); key = tile
__global__ void vpiece_fill_kernel(const int4* __restrict__ adm, int64_t nadm,
                                   const int32_t* __restrict__ rank,
                                   const int64_t* __restrict__ cnt,
                                   const int32_t* __restrict__ tile_of_point,
                                   const int32_t* __restrict__ tile_lo, Piece* __restrict__ pieces,
                                   uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nadm || cnt[b + 1] == cnt[b]) return;
    const int4 bl = adm[b];
    const int t0 = tile_of_point[bl.z];
    int64_t p = cnt[b];
    for (int t = t0; p < cnt[b + 1]; ++t, ++p) {
        Piece pc;
        pc.d_off = 0;
        pc.v_off = 0;
        pc.blk = (int32_t)b;
        pc.tile = t;
        pc.ncols = rank[b];
        pc.row0 = tile_lo[t] - bl.z;
        pieces[p] = pc;
        keys[p] = (uint64_t)t;
        vals[p] = (uint32_t)p;
    }
}

// sorted V pieces: data size and column count; then data offsets
__global__ void vpiece_sizes_kernel(const Piece* __restrict__ src, const uint32_t* __restrict__ order,
                                    int64_t np, Piece* __restrict__ dst,
                                    const int32_t* __restrict__ tile_lo, int R,
                                    int64_t* __restrict__ size, int64_t* __restrict__ cols) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= np) return;
    const Piece pc = src[order[i]];
    dst[i] = pc;
    const int mt = tile_lo[pc.tile + 1] - tile_lo[pc.tile];
    size[i] = (int64_t)p1_ld(mt, R) * pc.ncols;
    cols[i] = pc.ncols;
}

__global__ void vpiece_layout_kernel(Piece* __restrict__ pieces, int64_t np,
                                     const int64_t* __restrict__ doff) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < np) pieces[i].d_off = doff[i];
}

// copy the V rows of the V pieces (source: column-major V_b at vfo[b] in the
// exact pool, |sigma_b| rows), zero padding rows; one workgroup per piece
template <typename S>
__global__ __launch_bounds__(256) void vpiece_data_kernel(const Piece* __restrict__ pieces,
                                                          int64_t np,
                                                          const int32_t* __restrict__ tile_lo,
                                                          const int4* __restrict__ adm,
                                                          const int64_t* __restrict__ vfo,
                                                          const S* __restrict__ src, int R,
                                                          S* __restrict__ pool) {
    for (int64_t p = blockIdx.x; p < np; p += gridDim.x) {
        const Piece pc = pieces[p];
        const int mt = tile_lo[pc.tile + 1] - tile_lo[pc.tile];
        const int ld = p1_ld(mt, R);
        const int4 bl = adm[pc.blk];
        const int64_t len = bl.w - bl.z;
        const S* __restrict__ s = src + vfo[pc.blk] + pc.row0;
        S* __restrict__ d = pool + pc.d_off;
        const int tot = ld * pc.ncols;  // one piece: at most ld x 128 entries
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int c = e / ld;
            const int i = e - c * ld;
            d[e] = i < mt ? s[(int64_t)c * len + i] : (S)0;
        }
    }
}

unsigned g1(int64_t n, int bs = 256) {
    const int64_t b = (n + bs - 1) / bs;
    return (unsigned)(b < (1 << 30) ? b : (1 << 30));
}

// lanes: 8, 16, 32 or 64 lanes per column group; 0 picks the narrowest
// group that leaves each lane at most 8 row vectors of the tallest tile and
// no lane idle
template <typename S, typename T>
hipError_t p1_tile_dispatch(int64_t ntiles, const int32_t* tile_lo, const int64_t* meta, int ms,
                            int R, int max_ld, const void* pool, const void* vec, void* partial,
                            int64_t pbase, int lanes, hipStream_t st) {
    constexpr int VS = P1Dec<S, T>::n;
    const int need = (max_ld + VS - 1) / VS;  // row vectors of the tallest tile
    if (lanes == 0) lanes = need <= 8 ? 8 : (need <= 8 * 16 ? 16 : (need <= 8 * 32 ? 32 : 64));
    const unsigned grid = (unsigned)(ntiles < (1 << 30) ? ntiles : (1 << 30));
#define HMX_P1(LL)                                                                             \
    hipLaunchKernelGGL((p1_tile_kernel<S, T, LL>), dim3(grid), dim3(kP1Threads), 0, st, ntiles, \
                       tile_lo, meta, ms, R, (const S*)pool, (const T*)vec, (T*)partial, pbase)
    if (lanes == 8)
        HMX_P1(8);
    else if (lanes == 16)
        HMX_P1(16);
    else if (lanes == 32)
        HMX_P1(32);
    else
        HMX_P1(64);
#undef HMX_P1
    return hipGetLastError();
}

}  // namespace

hipError_t launch_p1_tile(int64_t ntiles, const int32_t* tile_lo, const int64_t* meta, int ms,
                          int R, int max_tile, const void* pool, const void* vec, void* partial,
                          int64_t pbase, int smode, int lanes, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    const int max_ld = (max_tile + R - 1) / R * R;
    if (smode == 0)
        return p1_tile_dispatch<double, double>(ntiles, tile_lo, meta, ms, R, max_ld, pool, vec,
                                                partial, pbase, lanes, st);
    if (smode == 1)
        return p1_tile_dispatch<float, float>(ntiles, tile_lo, meta, ms, R, max_ld, pool, vec,
                                              partial, pbase, lanes, st);
    return p1_tile_dispatch<uint16_t, float>(ntiles, tile_lo, meta, ms, R, max_ld, pool, vec,
                                             partial, pbase, lanes, st);
}

hipError_t launch_p1_reduce(const int4* rec, int64_t ncols, const int64_t* pfc,
                            const void* partial, void* vec, int64_t n, int f64, hipStream_t st) {
    if (ncols == 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(p1_reduce_kernel<double>, dim3(g1(ncols)), dim3(256), 0, st, rec, ncols,
                           pfc, (const double*)partial, (double*)vec, n);
    else
        hipLaunchKernelGGL(p1_reduce_kernel<float>, dim3(g1(ncols)), dim3(256), 0, st, rec, ncols,
                           pfc, (const float*)partial, (float*)vec, n);
    return hipGetLastError();
}

hipError_t launch_p1_rec(const int32_t* rank, const int64_t* toff, const int64_t* sbase,
                         const int32_t* snt, int64_t nadm, int4* rec, hipStream_t st) {
    if (nadm == 0) return hipSuccess;
    hipLaunchKernelGGL(p1_rec_kernel, dim3(g1(nadm)), dim3(256), 0, st, rank, toff, sbase, snt,
                       nadm, rec);
    return hipGetLastError();
}

hipError_t launch_p1_source(int64_t nadm, const int32_t* partner, const int64_t* cnt,
                            const int64_t* cntv, int64_t vbase, int64_t* sbase, int32_t* snt,
                            hipStream_t st) {
    if (nadm == 0) return hipSuccess;
    hipLaunchKernelGGL(p1_source_kernel, dim3(g1(nadm)), dim3(256), 0, st, nadm, partner, cnt,
                       cntv, vbase, sbase, snt);
    return hipGetLastError();
}

hipError_t launch_pfc(const Piece* sorted, const uint32_t* order, const int64_t* colscan,
                      int64_t np, int64_t limit, int64_t cbase, int64_t* pfc, hipStream_t st) {
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(pfc_kernel, dim3(g1(np)), dim3(256), 0, st, sorted, order, colscan, np,
                       limit, cbase, pfc);
    return hipGetLastError();
}

hipError_t launch_mirror_keys(const int4* adm, int64_t nadm, uint64_t* keys, uint32_t* vals,
                              hipStream_t st) {
    if (nadm == 0) return hipSuccess;
    hipLaunchKernelGGL(mirror_keys_kernel, dim3(g1(nadm)), dim3(256), 0, st, adm, nadm, keys,
                       vals);
    return hipGetLastError();
}

hipError_t launch_mirror_find(const int4* adm, int64_t nadm, const uint64_t* keys,
                              const uint32_t* vals, int32_t* partner, int* bad, hipStream_t st) {
    if (nadm == 0) return hipSuccess;
    hipLaunchKernelGGL(mirror_find_kernel, dim3(g1(nadm)), dim3(256), 0, st, adm, nadm, keys,
                       vals, partner, bad);
    return hipGetLastError();
}

hipError_t launch_primary_flags(const int4* adm, int64_t nadm, int sym, int64_t* flag,
                                hipStream_t st) {
    if (nadm == 0) return hipSuccess;
    hipLaunchKernelGGL(primary_flags_kernel, dim3(g1(nadm)), dim3(256), 0, st, adm, nadm, sym,
                       flag);
    return hipGetLastError();
}

hipError_t launch_gather_list(const int64_t* pos, int64_t nadm, const int4* adm,
                              const int32_t* level, const int32_t* rt, int32_t* list,
                              int4* blocks, int32_t* lev, int32_t* rt_out, hipStream_t st) {
    if (nadm == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_list_kernel, dim3(g1(nadm)), dim3(256), 0, st, pos, nadm, adm,
                       level, rt, list, blocks, lev, rt_out);
    return hipGetLastError();
}

hipError_t launch_scatter_list(const int32_t* list, int64_t nl, const int32_t* partner,
                               const int32_t* rank_l, const int32_t* steps_l, const int64_t* ue,
                               const int64_t* ve, int32_t* rank, int32_t* steps, int64_t* rfo,
                               int64_t* vfo, hipStream_t st) {
    if (nl == 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_list_kernel, dim3(g1(nl)), dim3(256), 0, st, list, nl, partner,
                       rank_l, steps_l, ue, ve, rank, steps, rfo, vfo);
    return hipGetLastError();
}

hipError_t launch_vpiece_count(const int4* adm, int64_t nadm, const int32_t* rank,
                               const int32_t* partner, const int32_t* tile_of_point, int64_t* cnt,
                               hipStream_t st) {
    if (nadm == 0) return hipSuccess;
    hipLaunchKernelGGL(vpiece_count_kernel, dim3(g1(nadm)), dim3(256), 0, st, adm, nadm, rank,
                       partner, tile_of_point, cnt);
    return hipGetLastError();
}

hipError_t launch_vpiece_fill(const int4* adm, int64_t nadm, const int32_t* rank,
                              const int64_t* cnt, const int32_t* tile_of_point,
                              const int32_t* tile_lo, Piece* pieces, uint64_t* keys,
                              uint32_t* vals, hipStream_t st) {
    if (nadm == 0) return hipSuccess;
    hipLaunchKernelGGL(vpiece_fill_kernel, dim3(g1(nadm)), dim3(256), 0, st, adm, nadm, rank, cnt,
                       tile_of_point, tile_lo, pieces, keys, vals);
    return hipGetLastError();
}

hipError_t launch_vpiece_sizes(const Piece* src, const uint32_t* order, int64_t np, Piece* dst,
                               const int32_t* tile_lo, int R, int64_t* size, int64_t* cols,
                               hipStream_t st) {
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(vpiece_sizes_kernel, dim3(g1(np)), dim3(256), 0, st, src, order, np, dst,
                       tile_lo, R, size, cols);
    return hipGetLastError();
}

hipError_t launch_vpiece_layout(Piece* pieces, int64_t np, const int64_t* doff, hipStream_t st) {
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(vpiece_layout_kernel, dim3(g1(np)), dim3(256), 0, st, pieces, np, doff);
    return hipGetLastError();
}

hipError_t launch_vpiece_data(const Piece* pieces, int64_t np, const int32_t* tile_lo,
                              const int4* adm, const int64_t* vfo, const void* src, int R,
                              void* pool, int smode, hipStream_t st) {
    if (np == 0) return hipSuccess;
    const unsigned grid = (unsigned)(np < (1 << 20) ? np : (1 << 20));
    if (smode == 0)
        hipLaunchKernelGGL(vpiece_data_kernel<double>, dim3(grid), dim3(256), 0, st, pieces, np,
                           tile_lo, adm, vfo, (const double*)src, R, (double*)pool);
    else if (smode == 1)
        hipLaunchKernelGGL(vpiece_data_kernel<float>, dim3(grid), dim3(256), 0, st, pieces, np,
                           tile_lo, adm, vfo, (const float*)src, R, (float*)pool);
    else
        hipLaunchKernelGGL(vpiece_data_kernel<uint16_t>, dim3(grid), dim3(256), 0, st, pieces, np,
                           tile_lo, adm, vfo, (const uint16_t*)src, R, (uint16_t*)pool);
    return hipGetLastError();
}

}  // namespace hmx
