// Near-field assembly and the batched H-matrix-vector product (Algorithm 3
// in flat form, Section 5.4).
//
// Storage.  The rows of the matrix are cut into row tiles, the leaf clusters
// of the cluster tree.  A piece is the part of one leaf block that falls in
// one tile: the tile's rows of the factor U of an admissible block (ncols =
// rank, weights t_b = V_b^T x|sigma) or of a dense block A|tau x sigma
// (ncols = |sigma|, weights x|sigma).  Factor pieces live in the factor pool,
// dense pieces in the near-field pool (each with its own storage type); in
// both, the pieces of a tile are stored one after another, column-major with
// the tile's leading dimension ld_t (tile rows rounded up to R, the rows of
// one 16-byte vector of the narrower type), so each tile is one contiguous
// ld_t x C matrix per pool and column k of the tile is multiplied by
// vec[widx[k]] (factor columns first, then dense columns).  Padding rows hold
// zeros.
//   vector pool: [ x in Morton order (n) | t_b for every admissible leaf ]
//   V pool     : V_b (n_b x r_b) column-major per admissible leaf.
// Matvec = gather x -> phase 1 (all t_b) -> phase 2 (one workgroup per tile,
// streaming its two contiguous regions) -> scatter to the original order with
// alpha, beta, sigma2.  Each z row is written by one workgroup and every sum
// has a fixed order, so the product is deterministic.
#include "hmx_internal.h"

namespace hmx {

namespace {

unsigned grid_cap(int64_t nb, int64_t cap) { return (unsigned)(nb < cap ? nb : cap); }

// padded tile height: rows rounded up to R (R = 16 / narrowest entry size)
__device__ __host__ __forceinline__ int tile_ld(int rows, int R) { return (rows + R - 1) / R * R; }

// ---------------------------------------------------------------------------
// storage types: the pools hold S (double, float or bfloat16 bits), the
// arithmetic runs in T (double or float).  bfloat16 = the upper 16 bits of an
// IEEE float; conversion rounds to nearest, ties to even.
// ---------------------------------------------------------------------------
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// the hardware conversion (round to nearest even, NaN stays NaN)
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

// two values in one packed conversion: a in the low half, b in the high half
__device__ __forceinline__ uint32_t f32x2_to_bf16x2(float a, float b) {
    const f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

template <typename S, typename T>
struct Store;
template <>
struct Store<double, double> {
    static __device__ __forceinline__ double put(double v) { return v; }
};
template <>
struct Store<float, float> {
    static __device__ __forceinline__ float put(float v) { return v; }
};
template <>
struct Store<uint16_t, float> {
    static __device__ __forceinline__ uint16_t put(float v) { return f32_to_bf16(v); }
};

// decode one 16-byte vector of S into 16 / sizeof(S) values of T
template <typename S, typename T>
struct Dec;
template <>
struct Dec<float, float> {
    static constexpr int n = 4;
    static __device__ __forceinline__ void get(const u32x4& r, float* o) {
        o[0] = __uint_as_float(r[0]);
        o[1] = __uint_as_float(r[1]);
        o[2] = __uint_as_float(r[2]);
        o[3] = __uint_as_float(r[3]);
    }
};
template <>
struct Dec<double, double> {
    static constexpr int n = 2;
    // one bit cast of the whole vector: assembling each double from two
    // 32-bit halves let the compiler re-load the low halves with separate
    // 8-byte loads, doubling the loads of the FP64 row tile
    static __device__ __forceinline__ void get(const u32x4& r, double* o) {
        const f64x2 v = __builtin_bit_cast(f64x2, r);
        o[0] = v[0];
        o[1] = v[1];
    }
};
template <>
struct Dec<uint16_t, float> {
    static constexpr int n = 8;
    static __device__ __forceinline__ void get(const u32x4& r, float* o) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            o[2 * k] = __uint_as_float(r[k] << 16);
            o[2 * k + 1] = __uint_as_float(r[k] & 0xffff0000u);
        }
    }
};

// near-field "storage" type of the recompute mode: entries are evaluated
// from the coordinates in the matvec, with the compute type's row grouping
template <typename T>
struct Recompute {};
template <typename S>
struct is_recompute {
    static constexpr bool value = false;
};
template <typename T>
struct is_recompute<Recompute<T>> {
    static constexpr bool value = true;
};
template <>
struct Dec<Recompute<float>, float> {
    static constexpr int n = 4;
};
template <>
struct Dec<Recompute<double>, double> {
    static constexpr int n = 2;
};

__device__ __forceinline__ u32x4 nt_load(const u32x4* p) { return __builtin_nontemporal_load(p); }

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
        // ranks < 0 (blocks waiting for a fallback approximation) count as 0
        case 3: v = rank[b] > 0 ? (int64_t)rank[b] * m : 0; break;
        case 4: v = rank[b] > 0 ? (int64_t)rank[b] * nc : 0; break;
        case 5: v = rank[b] > 0 ? rank[b] : 0; break;
        case 7: v = (m + nc) * mult; break;
        case 8: v = (m + nc) * (int64_t)rank[b]; break;
        default:
            v = (rank && rank[b] == 0)
                    ? 0
                    : (int64_t)(tile_of_point[bl.y - 1] - tile_of_point[bl.x] + 1);
    }
    out[b] = v;
}

// one piece per (leaf block, tile of its rows); key = tile for the stable sort
__global__ void piece_fill_kernel(const int4* __restrict__ blocks, int64_t nb,
                                  const int32_t* __restrict__ rank,
                                  const int32_t* __restrict__ tile_of_point,
                                  const int32_t* __restrict__ tile_lo,
                                  const int64_t* __restrict__ piece_off,
                                  const int64_t* __restrict__ toff, int64_t vec_base,
                                  int64_t piece_base, Piece* __restrict__ pieces,
                                  uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int4 bl = blocks[b];
    const int r = rank ? rank[b] : 0;
    if (rank && r == 0) return;
    const int t0 = tile_of_point[bl.x], t1 = tile_of_point[bl.y - 1];
    int64_t p = piece_base + piece_off[b];
    for (int t = t0; t <= t1; ++t, ++p) {
        Piece pc;
        pc.d_off = 0;
        pc.v_off = rank ? vec_base + toff[b] : (int64_t)bl.z;
        pc.blk = rank ? (int32_t)b : -(int32_t)b - 1;
        pc.tile = t;
        pc.ncols = rank ? r : (bl.w - bl.z);
        pc.row0 = tile_lo[t] - bl.x;
        pieces[p] = pc;
        keys[p] = (uint64_t)t;
        vals[p] = (uint32_t)p;
    }
}

// sorted order -> pieces; each piece's data size in its pool and columns
__global__ void piece_gather_kernel(const Piece* __restrict__ src,
                                    const uint32_t* __restrict__ order, int64_t np,
                                    Piece* __restrict__ dst, int64_t* __restrict__ size_u,
                                    int64_t* __restrict__ size_n, int64_t* __restrict__ cols,
                                    int64_t* __restrict__ cols_u,
                                    const int32_t* __restrict__ tile_lo, int R,
                                    int near_stored) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= np) return;
    const Piece pc = src[order[i]];
    dst[i] = pc;
    const int mt = tile_lo[pc.tile + 1] - tile_lo[pc.tile];
    const int64_t sz = (int64_t)tile_ld(mt, R) * pc.ncols;
    const bool f = pc.blk >= 0;
    size_u[i] = f ? sz : 0;
    size_n[i] = f || !near_stored ? 0 : sz;
    cols[i] = pc.ncols;
    cols_u[i] = f ? pc.ncols : 0;
}

// after the scans: piece data offsets, and the weight index of every column
__global__ void piece_layout_kernel(Piece* __restrict__ pieces, int64_t np,
                                    const int64_t* __restrict__ doff_u,
                                    const int64_t* __restrict__ doff_n,
                                    const int64_t* __restrict__ coff,
                                    int64_t* __restrict__ widx) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= np) return;
    Piece pc = pieces[i];
    pc.d_off = pc.blk >= 0 ? doff_u[i] : doff_n[i];
    pieces[i] = pc;
    const int64_t c0 = coff[i];
    for (int c = 0; c < pc.ncols; ++c) widx[c0 + c] = pc.v_off + c;
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

// per tile (from its first piece): first column, first factor column, and
// data offsets in the two pools; entry ntiles holds the totals
__global__ void tile_meta_kernel(const int64_t* __restrict__ tile_ptr, int64_t ntiles,
                                 int64_t np, const int64_t* __restrict__ coff,
                                 const int64_t* __restrict__ coff_u,
                                 const int64_t* __restrict__ doff_u,
                                 const int64_t* __restrict__ doff_n, int64_t* __restrict__ meta) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    const int64_t p = tile_ptr[t];  // <= np; the scans hold the totals at index np
    meta[4 * t + 0] = coff[p];
    meta[4 * t + 1] = coff_u[p];
    meta[4 * t + 2] = doff_u[p];
    meta[4 * t + 3] = doff_n[p];
}

// Fill the matrix pool piece by piece: dense pieces evaluate phi (the near
// field, Section 5.4.2), factor pieces copy the tile's rows of U_b from the
// ACA capacity pool.  Padding rows are zero.
// R values of S at an R-aligned element offset, as 16-byte stores
template <typename S, int R>
__device__ __forceinline__ void store_unit(S* __restrict__ dst, const S (&v)[R]) {
    static_assert((R * sizeof(S)) % 16 == 0, "a unit is whole 16-byte vectors");
    constexpr int kVec = (int)(R * sizeof(S) / 16);
    u32x4 w[kVec];
    __builtin_memcpy(w, v, sizeof(w));
    u32x4* out = reinterpret_cast<u32x4*>(dst);
#pragma unroll
    for (int q = 0; q < kVec; ++q) out[q] = w[q];
}

// R values of T, converted to S, stored as one unit
template <typename S, typename T, int R>
struct UnitStore {
    static __device__ __forceinline__ void put(S* __restrict__ dst, const T (&v)[R]) {
        S o[R];
#pragma unroll
        for (int e = 0; e < R; ++e) o[e] = Store<S, T>::put(v[e]);
        store_unit<S, R>(dst, o);
    }
};
template <int R>
struct UnitStore<uint16_t, float, R> {
    static __device__ __forceinline__ void put(uint16_t* __restrict__ dst, const float (&v)[R]) {
        static_assert(R % 8 == 0, "BF16 units are whole 16-byte vectors");
        uint32_t w[R / 2];
#pragma unroll
        for (int e = 0; e < R / 2; ++e) w[e] = f32x2_to_bf16x2(v[2 * e], v[2 * e + 1]);
        u32x4* out = reinterpret_cast<u32x4*>(dst);
#pragma unroll
        for (int q = 0; q < R / 8; ++q) out[q] = u32x4{w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]};
    }
};

// the near-field columns c = cstart, cstart + per, ... < ncols of rows
// i0 .. i0 + R - 1 (coordinates x, zero past the tile's mt rows) for one
// kernel kind; four columns' coordinates are loaded before they are used
template <int KIND, typename SN, typename T, int R>
__device__ __forceinline__ void fill_near(const KernelEval<T>& K, const T* __restrict__ soa, int64_t n,
                                          int d, int64_t ybase, const T (&x)[R][3], int i0, int mt,
                                          int cstart, int per, int ncols, int ld,
                                          SN* __restrict__ dst) {
    int c = cstart;
    for (; c + 3 * per < ncols; c += 4 * per) {
        T y[4][3];
#pragma unroll
        for (int q = 0; q < 4; ++q) load_pt(soa, n, d, ybase + c + q * per, y[q]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            T v[R];
#pragma unroll
            for (int e = 0; e < R; ++e) v[e] = i0 + e < mt ? phi_kind<KIND>(K, x[e], y[q]) : (T)0;
            UnitStore<SN, T, R>::put(dst + (int64_t)(c + q * per) * ld + i0, v);
        }
    }
    for (; c < ncols; c += per) {
        T y[3];
        load_pt(soa, n, d, ybase + c, y);
        T v[R];
#pragma unroll
        for (int e = 0; e < R; ++e) v[e] = i0 + e < mt ? phi_kind<KIND>(K, x[e], y) : (T)0;
        UnitStore<SN, T, R>::put(dst + (int64_t)c * ld + i0, v);
    }
}

// the near-field fill specialised on the kernel kind
template <typename SN, typename T, int R>
__device__ __forceinline__ void near_dispatch(const KernelEval<T>& K, const T* __restrict__ soa,
                                              int64_t n, int d, int64_t ybase, const T (&x)[R][3],
                                              int i0, int mt, int cstart, int per, int ncols,
                                              int ld, SN* __restrict__ dst) {
    switch (K.kind) {
        case HMX_GAUSSIAN:
            fill_near<HMX_GAUSSIAN, SN, T, R>(K, soa, n, d, ybase, x, i0, mt, cstart, per,
                                              ncols, ld, dst);
            break;
        case HMX_MATERN32:
            fill_near<HMX_MATERN32, SN, T, R>(K, soa, n, d, ybase, x, i0, mt, cstart, per,
                                              ncols, ld, dst);
            break;
        case HMX_MATERN_NU1:
            fill_near<HMX_MATERN_NU1, SN, T, R>(K, soa, n, d, ybase, x, i0, mt, cstart, per,
                                                ncols, ld, dst);
            break;
        case HMX_TEST_CONST:
            fill_near<HMX_TEST_CONST, SN, T, R>(K, soa, n, d, ybase, x, i0, mt, cstart, per,
                                                ncols, ld, dst);
            break;
        default:
            fill_near<HMX_TEST_LOWRANK, SN, T, R>(K, soa, n, d, ybase, x, i0, mt, cstart, per,
                                                  ncols, ld, dst);
            break;
    }
}

// One workgroup per piece.  Each thread owns a group of R consecutive rows
// of the tile (their coordinates stay in registers) and sweeps a set of the
// piece's columns, writing R entries per column with 16-byte stores; rows
// past the tile's end are zero.  A factor piece copies rows row0 .. of its U
// columns, a near-field piece evaluates phi.
template <typename SU, typename SN, typename T, int R>
__global__ __launch_bounds__(256) void piece_data_kernel(
    const Piece* __restrict__ pieces, int64_t np, const int32_t* __restrict__ tile_lo,
    const int4* __restrict__ adm, const int4* __restrict__ dense,
    const int64_t* __restrict__ uoff, const SU* __restrict__ Usrc, const T* __restrict__ soa,
    int64_t n, int d, KernelEval<T> K, SU* __restrict__ upool, SN* __restrict__ npool,
    int which) {
    const int tid = threadIdx.x;
    for (int64_t p = blockIdx.x; p < np; p += gridDim.x) {
        const Piece pc = pieces[p];
        if (is_recompute<SN>::value && pc.blk < 0) continue;  // near field evaluated per product
        if ((which == 1 && pc.blk < 0) || (which == 2 && pc.blk >= 0)) continue;
        const int32_t r0 = tile_lo[pc.tile];
        const int mt = tile_lo[pc.tile + 1] - r0;
        const int ld = tile_ld(mt, R);
        const int upc = ld / R;  // row groups per column
        const bool is_factor = pc.blk >= 0;
        const int4 bl = is_factor ? adm[pc.blk] : dense[-pc.blk - 1];
        const int m = bl.y - bl.x;
        // thread -> row group g and columns cstart, cstart + per, ...
        const int per = upc <= 256 ? 256 / upc : 1;
        for (int gs = 0; gs < upc; gs += 256) {
            const int g = upc <= 256 ? tid % upc : gs + tid;
            const int cstart = upc <= 256 ? tid / upc : 0;
            if (upc <= 256 ? tid >= per * upc : g >= upc) continue;
            const int i0 = g * R;
            if (is_factor) {
                const SU* __restrict__ src = Usrc + uoff[pc.blk] + pc.row0 + i0;
                for (int c = cstart; c < pc.ncols; c += per) {
                    SU v[R];
#pragma unroll
                    for (int e = 0; e < R; ++e) v[e] = i0 + e < mt ? src[(int64_t)c * m + e] : (SU)0;
                    store_unit<SU, R>(upool + pc.d_off + (int64_t)c * ld + i0, v);
                }
            } else if constexpr (!is_recompute<SN>::value) {
                T x[R][3];
#pragma unroll
                for (int e = 0; e < R; ++e) {
                    const int i = i0 + e < mt ? i0 + e : mt - 1;
                    load_pt(soa, n, d, (int64_t)r0 + i, x[e]);
                }
                SN* __restrict__ dst = npool + pc.d_off;
                near_dispatch<SN, T, R>(K, soa, n, d, bl.z, x, i0, mt, cstart, per, pc.ncols, ld,
                                        dst);
            }
        }
    }
}

template <typename T>
__global__ void gather_x_kernel(const T* __restrict__ x, const int32_t* __restrict__ perm,
                                int64_t n, T* __restrict__ xm, int64_t base) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) xm[i] = x[perm[i] - base];
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

// compaction of the first r_b columns of each U_b (rows = 1: m rows) or V_b
// (rows = 0: n rows) from the capacity pool into the exact-rank pool,
// converted to the storage type
template <typename S, typename T>
__global__ __launch_bounds__(256) void compact_kernel(const int4* __restrict__ blocks,
                                                      int64_t nblocks,
                                                      const int32_t* __restrict__ rank,
                                                      const int64_t* __restrict__ coff,
                                                      int64_t cbase,
                                                      const int64_t* __restrict__ eoff,
                                                      const T* __restrict__ src,
                                                      S* __restrict__ dst, int rows) {
    constexpr int kU = 8;  // elements per thread per pass, loaded before any is stored
    for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
        const int4 bl = blocks[b];
        const int64_t len = rows ? bl.y - bl.x : bl.w - bl.z, r = rank[b];
        const int64_t tot = r * len;
        const T* sv = src + (coff[b] - cbase);
        S* dv = dst + eoff[b];
        for (int64_t e0 = 0; e0 < tot; e0 += (int64_t)kU * blockDim.x) {
            T v[kU];
#pragma unroll
            for (int k = 0; k < kU; ++k) {
                const int64_t e = e0 + threadIdx.x + (int64_t)k * blockDim.x;
                v[k] = sv[e < tot ? e : tot - 1];
            }
#pragma unroll
            for (int k = 0; k < kU; ++k) {
                const int64_t e = e0 + threadIdx.x + (int64_t)k * blockDim.x;
                if (e < tot) dv[e] = Store<S, T>::put(v[k]);
            }
        }
    }
}

__global__ void add_const_kernel(int64_t* __restrict__ a, int64_t n, int64_t c) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) a[i] += c;
}

// bnd[k] = lower bound of k * step in the non-decreasing cap_off[0..nb]
__global__ void chunk_bounds_kernel(const int64_t* __restrict__ cap_off, int64_t nb, int64_t step,
                                    int nchunks, int64_t* __restrict__ bnd) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nchunks) return;
    if (k == nchunks) {
        bnd[k] = nb;
        return;
    }
    const int64_t target = (int64_t)k * step;
    int64_t lo = 0, hi = nb;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cap_off[mid] < target)
            lo = mid + 1;
        else
            hi = mid;
    }
    bnd[k] = lo;
}

// phase 2: one workgroup per row tile (or per row pass of a tile, the split
// grid of the autotuner's third group).  The tile is a contiguous ld x C
// column-major matrix; column k is weighted by vec[widx[k]].  Weights are
// gathered into LDS a chunk of kChunk columns at a time, so the streaming
// loads never wait on an index lookup.  The 4 waves split into
// G = 4 * (64 / L) column groups of L lanes; lane q of a group owns RV
// 16-byte vectors of rows (vector v * L + q).  Groups take interleaved
// columns, kUnroll in flight per lane (raw 16-byte vectors, decoded one
// column at a time: two waves per SIMD with 16 columns in flight each move
// more bytes than three with 8; a chunk's last batch is masked), with
// non-temporal loads (every matrix byte is read once per product); the G
// partial row sets are summed in LDS in a fixed order and the tile is
// scattered to the original order.
constexpr int kTileThreads = 256;
constexpr int kChunk = 2048;
constexpr int kUnroll = 16;
constexpr int kEvalUnroll = 4;  // near-field columns evaluated per iteration (recompute mode)


// sw[j] = vec[wi[j]] for j < cnt: eight indices, then eight weights, in
// flight per thread at a time (the gather's latency is paid once per eight)
template <typename T>
__device__ __forceinline__ void stage_weights(const int64_t* __restrict__ wi, int cnt,
                                              const T* __restrict__ vec, T* __restrict__ sw) {
    constexpr int kG = 8;
    for (int j0 = threadIdx.x; j0 < cnt; j0 += kG * kTileThreads) {
        int64_t idx[kG];
#pragma unroll
        for (int u = 0; u < kG; ++u) {
            const int j = j0 + u * kTileThreads;
            idx[u] = wi[j < cnt ? j : cnt - 1];
        }
        T val[kG];
#pragma unroll
        for (int u = 0; u < kG; ++u) val[u] = vec[idx[u]];
#pragma unroll
        for (int u = 0; u < kG; ++u) {
            const int j = j0 + u * kTileThreads;
            if (j < cnt) sw[j] = val[u];
        }
    }
}

// raw 16-byte vectors of kUnroll columns c, c + G, ... of a chunk (b: its
// first column) for lane unit vi; MASKED: columns at or past cnt read column
// cnt - 1 (their weight is zero)
template <typename S, typename T, int R, int G, bool MASKED>
__device__ __forceinline__ void batch_load(const S* __restrict__ b, int ld, int c, int cnt,
                                           int vi, u32x4 (&raw)[kUnroll][R / Dec<S, T>::n]) {
    constexpr int VS = Dec<S, T>::n;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        int cu = c + u * G;
        if (MASKED) cu = cu < cnt ? cu : cnt - 1;
        const u32x4* p = (const u32x4*)(b + (int64_t)cu * ld + (int64_t)vi * R);
#pragma unroll
        for (int k = 0; k < R / VS; ++k) raw[u][k] = nt_load(p + k);
    }
}

// acc += the batch's columns times their weights, decoded one column at a time
template <typename S, typename T, int R, int G, bool MASKED>
__device__ __forceinline__ void batch_fma(const u32x4 (&raw)[kUnroll][R / Dec<S, T>::n], int c,
                                          int cnt, const T* __restrict__ sw, T (&acc)[R]) {
    constexpr int VS = Dec<S, T>::n;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int cu = c + u * G;
        const T w = (!MASKED || cu < cnt) ? sw[MASKED && cu >= cnt ? cnt - 1 : cu] : (T)0;
        T a[R];
#pragma unroll
        for (int k = 0; k < R / VS; ++k) Dec<S, T>::get(raw[u][k], a + k * VS);
#pragma unroll
        for (int e = 0; e < R; ++e) acc[e] += a[e] * w;
    }
}

// accumulate nk columns of one pool segment (base: row pass start of the
// tile's first column in this segment) into acc
template <typename S, typename T, int L, int RV, int R, int G>
__device__ __forceinline__ void rowtile_segment(const S* __restrict__ base, int ld, int64_t nk,
                                                const int64_t* __restrict__ wi,
                                                const T* __restrict__ vec, T* __restrict__ sw,
                                                int g, int q, int nvec, T (&acc)[RV][R]) {
    for (int64_t kc = 0; kc < nk; kc += kChunk) {
        const int cnt = (nk - kc) < kChunk ? (int)(nk - kc) : kChunk;
        stage_weights(wi + kc, cnt, vec, sw);
        __syncthreads();
        const S* __restrict__ b = base + kc * ld;
        // kUnroll columns per group in flight; full batches are pipelined (the
        // next batch's loads are issued before the current one is used, two
        // register sets in turn); the last batch of the chunk is masked (its
        // missing columns weigh zero and read a valid column: pool entries are
        // finite, so they add exact zeros)
        constexpr int VS = Dec<S, T>::n;
#pragma unroll
        for (int v = 0; v < RV; ++v) {
            const int vi = v * L + q;
            if (vi >= nvec) continue;
            for (int c = g; c < cnt; c += kUnroll * G) {
                u32x4 ra[kUnroll][R / VS];
                if (c + (kUnroll - 1) * G < cnt) {
                    batch_load<S, T, R, G, false>(b, ld, c, cnt, vi, ra);
                    batch_fma<S, T, R, G, false>(ra, c, cnt, sw, acc[v]);
                } else {
                    batch_load<S, T, R, G, true>(b, ld, c, cnt, vi, ra);
                    batch_fma<S, T, R, G, true>(ra, c, cnt, sw, acc[v]);
                }
            }
        }
        __syncthreads();
    }
}

// near-field columns of a tile evaluated on the fly (recompute mode): the
// column's point coordinates are staged in LDS with its weight, each lane
// keeps the coordinates of its rows; phi as in the stored mode's assembly.
// Rows past the tile (padding) read the tile's last point and are never
// written out.
template <typename T, int L, int RV, int R, int G>
__device__ __forceinline__ void rowtile_near_eval(const T* __restrict__ soa, int64_t n, int d,
                                                  const KernelEval<T>& K, int64_t row0,
                                                  int rows, int64_t nk,
                                                  const int64_t* __restrict__ wi,
                                                  const T* __restrict__ vec, T* __restrict__ sw,
                                                  T* __restrict__ sy, int g, int q, int nvec,
                                                  T (&acc)[RV][R]) {
    T xr[RV][R][3];
#pragma unroll
    for (int v = 0; v < RV; ++v)
#pragma unroll
        for (int e = 0; e < R; ++e) {
            int i = (v * L + q) * R + e;
            i = i < rows ? i : rows - 1;
            load_pt(soa, n, d, row0 + i, xr[v][e]);
        }
    for (int64_t kc = 0; kc < nk; kc += kChunk) {
        const int cnt = (nk - kc) < kChunk ? (int)(nk - kc) : kChunk;
        for (int j = threadIdx.x; j < cnt; j += kTileThreads) {
            const int64_t w = wi[kc + j];
            sw[j] = vec[w];
#pragma unroll
            for (int k = 0; k < 3; ++k) sy[k * kChunk + j] = k < d ? soa[(int64_t)k * n + w] : (T)0;
        }
        __syncthreads();
        // kEvalUnroll columns per iteration: their LDS reads are issued
        // together and the entries' exponentials overlap
        int c = g;
        for (; c + (kEvalUnroll - 1) * G < cnt; c += kEvalUnroll * G) {
            T w[kEvalUnroll], y[kEvalUnroll][3];
#pragma unroll
            for (int u = 0; u < kEvalUnroll; ++u) {
                const int cc = c + u * G;
                w[u] = sw[cc];
                y[u][0] = sy[cc];
                y[u][1] = sy[kChunk + cc];
                y[u][2] = sy[2 * kChunk + cc];
            }
#pragma unroll
            for (int v = 0; v < RV; ++v) {
                if (v * L + q < nvec) {
#pragma unroll
                    for (int u = 0; u < kEvalUnroll; ++u)
#pragma unroll
                        for (int e = 0; e < R; ++e) acc[v][e] += phi(K, xr[v][e], y[u], d) * w[u];
                }
            }
        }
        for (; c < cnt; c += G) {
            const T w0 = sw[c];
            const T y[3] = {sy[c], sy[kChunk + c], sy[2 * kChunk + c]};
#pragma unroll
            for (int v = 0; v < RV; ++v) {
                if (v * L + q < nvec) {
#pragma unroll
                    for (int e = 0; e < R; ++e) acc[v][e] += phi(K, xr[v][e], y, d) * w0;
                }
            }
        }
        __syncthreads();
    }
}

template <typename SU, typename SN, typename T, int L, int RV>
__global__ __launch_bounds__(kTileThreads) void rowtile_kernel(
    int64_t ntiles, const int32_t* __restrict__ tile_lo, const int64_t* __restrict__ meta,
    const int64_t* __restrict__ widx, const SU* __restrict__ upool, const SN* __restrict__ npool,
    const T* __restrict__ vec, const int32_t* __restrict__ perm, T alpha, T beta, T sigma2,
    T* __restrict__ z, const T* __restrict__ soa, int64_t n, int d, KernelEval<T> K,
    int split) {
    constexpr int VU = Dec<SU, T>::n, VN = Dec<SN, T>::n;
    constexpr int R = VU > VN ? VU : VN;  // rows per lane unit
    constexpr int SUB = 64 / L;
    constexpr int G = 4 * SUB;
    constexpr int RPG = L * RV * R;  // rows per pass
    constexpr bool NR = is_recompute<SN>::value;
    __shared__ T red[G * RPG];
    __shared__ T sw[kChunk];
    __shared__ T sy[NR ? 3 * kChunk : 1];
    const int tid = threadIdx.x, lane = tid & 63;
    // the group index is wave-uniform when a group is a whole wave
    const int g = (SUB == 1) ? __builtin_amdgcn_readfirstlane(tid >> 6) : (tid >> 6) * SUB + lane / L;
    const int q = lane % L;
    // split > 0: one workgroup per (tile, row pass), the passes of a tile
    // consecutive in the grid, so the workgroups running together read whole
    // columns of a few tiles rather than one pass of every tile
    const int64_t nwork = split ? ntiles * split : ntiles;
    for (int64_t w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int64_t t = split ? w / split : w;
        const int pass = split ? (int)(w - t * split) : 0;
        const int32_t r0 = tile_lo[t];
        const int mt = tile_lo[t + 1] - r0;
        const int ld = tile_ld(mt, R);
        const int64_t k0 = meta[4 * t], k1 = meta[4 * t + 4];
        const int64_t ku = meta[4 * t + 5] - meta[4 * t + 1];  // factor columns of the tile
        const SU* __restrict__ ubase = upool + meta[4 * t + 2];
        const SN* __restrict__ nbase = NR ? npool : npool + meta[4 * t + 3];
        // split: this workgroup's row pass only, else all of them
        for (int rb = split ? pass * RPG : 0; rb < ld; rb += split ? ld : RPG) {
            const int nvec = ((ld - rb) < RPG ? (ld - rb) : RPG) / R;  // lane units in this pass
            T acc[RV][R];
#pragma unroll
            for (int v = 0; v < RV; ++v)
#pragma unroll
                for (int e = 0; e < R; ++e) acc[v][e] = 0;
            rowtile_segment<SU, T, L, RV, R, G>(ubase + rb, ld, ku, widx + k0, vec, sw, g, q,
                                                 nvec, acc);
            if constexpr (NR)
                rowtile_near_eval<T, L, RV, R, G>(soa, n, d, K, (int64_t)r0 + rb, mt - rb,
                                                  k1 - k0 - ku, widx + k0 + ku, vec, sw, sy, g, q,
                                                  nvec, acc);
            else
                rowtile_segment<SN, T, L, RV, R, G>(nbase + rb, ld, k1 - k0 - ku, widx + k0 + ku,
                                                     vec, sw, g, q, nvec, acc);
            // sum the G partial row sets in a fixed order
#pragma unroll
            for (int v = 0; v < RV; ++v)
#pragma unroll
                for (int e = 0; e < R; ++e) red[g * RPG + (v * L + q) * R + e] = acc[v][e];
            __syncthreads();
            const int mc = (mt - rb) < RPG ? (mt - rb) : RPG;  // real rows of this pass
            for (int row = tid; row < mc; row += kTileThreads) {
                T sum = red[row];
#pragma unroll
                for (int gg = 1; gg < G; ++gg) sum += red[gg * RPG + row];
                const int64_t i = (int64_t)r0 + rb + row;
                const int32_t pi = perm[i];
                T out = alpha * (sigma2 != (T)0 ? sum + sigma2 * vec[i] : sum);
                if (beta != (T)0) out += beta * z[pi];
                z[pi] = out;
            }
            __syncthreads();
        }
    }
}

// tile shapes of the row-tile kernel, (lanes per row group L, row vectors per
// lane RV) = (16, 1), (32, 1), (64, 1), (64, 2), (64, 4), (8, 1) (the last for
// tiles of at most 8 row vectors, whose columns would leave lanes of wider
// groups without rows); the grid is one workgroup per tile, a fixed
// persistent grid looping over the tiles, or one workgroup per row pass

template <typename SU, typename SN, typename T>
hipError_t rowtile_dispatch(int64_t ntiles, const int32_t* tile_lo, const int64_t* meta,
                            const int64_t* widx, const void* upool, const void* npool,
                            const void* vecpool, const int32_t* perm, double alpha, double beta,
                            double sigma2, void* z, int max_tile, int config, const void* soa,
                            int64_t n, int d, KernelFn kern, hipStream_t st) {
    constexpr int VU = Dec<SU, T>::n, VN = Dec<SN, T>::n;
    constexpr int R = VU > VN ? VU : VN;
    int shape, mode = 0;
    if (config < 0) {
        // default: one workgroup per row pass of 128 rows (L = 128 / R lanes
        // per row group, one row vector per lane: 64 lanes in FP64, 32 in
        // FP32, 16 in BF16), narrower when the largest tile is shorter.
        // Timed on the N = 2^20 workload (256-point tiles) this is the
        // fastest of the 15 configurations in FP32 and BF16 (configurations
        // 11 and 10) and within 1% of the fastest in FP64 (configuration 12
        // against 32-lane 64-row passes); the shapes with two or four row
        // vectors per lane take 4-10% longer in FP64 and FP32, 40% in BF16
        const int need = (max_tile + R - 1) / R;  // lane units per tile column
        int L = 16;
        while (L < need && L * R < 128 && L < 64) L *= 2;
        shape = L == 16 ? 0 : (L == 32 ? 1 : 2);
        mode = 2;
    } else if (config < 15) {
        shape = config % 5;
        mode = config / 5;
    } else {  // the 8-lane shape, for tiles of at most 8 row vectors
        shape = 5;
        mode = config - 15;
    }
    static constexpr int kL[kRowtileShapes] = {16, 32, 64, 64, 64, 8};
    static constexpr int kRV[kRowtileShapes] = {1, 1, 1, 2, 4, 1};
    const int rpg = kL[shape] * kRV[shape] * R;  // rows per pass
    const unsigned passes =
        mode == 2 ? (unsigned)((tile_ld(max_tile, R) + rpg - 1) / rpg) : 1u;
    const dim3 grid(mode == 1 ? (unsigned)(ntiles < kPersistentGrid ? ntiles : kPersistentGrid)
                              : grid_cap(mode == 2 ? ntiles * passes : ntiles, 1 << 20));
    const int split = mode == 2 ? (int)passes : 0;
#define HMX_RT(LL, RR)                                                                       \
    hipLaunchKernelGGL((rowtile_kernel<SU, SN, T, LL, RR>), grid, dim3(kTileThreads), 0, st,  \
                       ntiles, tile_lo, meta, widx, (const SU*)upool, (const SN*)npool,      \
                       (const T*)vecpool, perm, (T)alpha, (T)beta, (T)sigma2, (T*)z,         \
                       (const T*)soa, n, d, KernelEval<T>(kern), split)
    switch (shape) {
        case 0: HMX_RT(16, 1); break;
        case 1: HMX_RT(32, 1); break;
        case 2: HMX_RT(64, 1); break;
        case 3: HMX_RT(64, 2); break;
        case 4: HMX_RT(64, 4); break;
        default: HMX_RT(8, 1); break;
    }
#undef HMX_RT
    return hipGetLastError();
}

}  // namespace

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
                             const int64_t* piece_off, const int64_t* toff, int64_t vec_base,
                             int64_t piece_base, Piece* pieces, uint64_t* keys, uint32_t* vals,
                             hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(piece_fill_kernel, dim3((unsigned)((nblocks + 255) / 256)), dim3(256), 0,
                       st, blocks, nblocks, rank, tile_of_point, tile_lo, piece_off, toff,
                       vec_base, piece_base, pieces, keys, vals);
    return hipGetLastError();
}

hipError_t launch_piece_gather(const Piece* src, const uint32_t* order, int64_t npieces,
                               Piece* dst, int64_t* size_u, int64_t* size_n, int64_t* cols,
                               int64_t* cols_u, const int32_t* tile_lo, int R, int near_stored,
                               hipStream_t st) {
    if (npieces == 0) return hipSuccess;
    hipLaunchKernelGGL(piece_gather_kernel, dim3((unsigned)((npieces + 255) / 256)), dim3(256), 0,
                       st, src, order, npieces, dst, size_u, size_n, cols, cols_u, tile_lo, R,
                       near_stored);
    return hipGetLastError();
}

hipError_t launch_piece_layout(Piece* pieces, int64_t np, const int64_t* doff_u,
                               const int64_t* doff_n, const int64_t* coff, int64_t* widx,
                               hipStream_t st) {
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(piece_layout_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st,
                       pieces, np, doff_u, doff_n, coff, widx);
    return hipGetLastError();
}

hipError_t launch_tile_offsets(const uint64_t* sorted_tile, int64_t npieces, int64_t ntiles,
                               int64_t* tile_ptr, hipStream_t st) {
    hipLaunchKernelGGL(tile_ptr_kernel, dim3((unsigned)((ntiles + 1 + 255) / 256)), dim3(256), 0,
                       st, sorted_tile, npieces, ntiles, tile_ptr);
    return hipGetLastError();
}

hipError_t launch_tile_meta(const int64_t* tile_ptr, int64_t ntiles, int64_t np,
                            const int64_t* coff, const int64_t* coff_u, const int64_t* doff_u,
                            const int64_t* doff_n, int64_t* meta, hipStream_t st) {
    hipLaunchKernelGGL(tile_meta_kernel, dim3((unsigned)((ntiles + 1 + 255) / 256)), dim3(256), 0,
                       st, tile_ptr, ntiles, np, coff, coff_u, doff_u, doff_n, meta);
    return hipGetLastError();
}

// storage modes: 0 = F64 (F64 arithmetic), 1 = F32, 2 = BF16 (F32 arithmetic)
int rows_per_unit(int fmode, int nmode) {
    auto v = [](int m) { return m == 0 ? 2 : (m == 1 ? 4 : 8); };
    // recompute mode (3): the compute type's grouping (F64 with F64 factors)
    const int vn = nmode == 3 ? (fmode == 0 ? 2 : 4) : v(nmode);
    return v(fmode) > vn ? v(fmode) : vn;
}

hipError_t launch_piece_data(const Piece* pieces, int64_t np, const int32_t* tile_lo,
                             const int4* adm, const int4* dense, const int64_t* uoff,
                             const void* Usrc, const void* soa, int64_t n, int d, KernelFn kern,
                             void* upool, void* npool, int fmode, int nmode, int which,
                             hipStream_t st) {
    if (np == 0) return hipSuccess;
    const unsigned grid = grid_cap(np, 1 << 20);
// each combination's unit (rows_per_unit) is a template argument
#define HMX_PD(SU, SN, T, R)                                                                  \
    if (R != rows_per_unit(fmode, nmode)) return hipErrorInvalidValue;                        \
    else hipLaunchKernelGGL((piece_data_kernel<SU, SN, T, R>), dim3(grid), dim3(256), 0, st,     \
                       pieces, np, tile_lo, adm, dense, uoff, (const SU*)Usrc, (const T*)soa, \
                       n, d, KernelEval<T>(kern), (SU*)upool, (SN*)npool, which)
    if (fmode == 0 && nmode == 0) {
        HMX_PD(double, double, double, 2);
    } else if (fmode == 1 && nmode == 1) {
        HMX_PD(float, float, float, 4);
    } else if (fmode == 2 && nmode == 2) {
        HMX_PD(uint16_t, uint16_t, float, 8);
    } else if (fmode == 2 && nmode == 1) {
        HMX_PD(uint16_t, float, float, 8);
    } else if (nmode == 3 && fmode == 0) {
        HMX_PD(double, Recompute<double>, double, 2);
    } else if (nmode == 3 && fmode == 1) {
        HMX_PD(float, Recompute<float>, float, 4);
    } else if (nmode == 3 && fmode == 2) {
        HMX_PD(uint16_t, Recompute<float>, float, 8);
    } else {
        return hipErrorInvalidValue;
    }
#undef HMX_PD
    return hipGetLastError();
}

namespace {
hipError_t compact(const int4* blocks, int64_t nblocks, const int32_t* rank, const int64_t* coff,
                   int64_t cbase, const int64_t* eoff, const void* src, void* dst, int smode,
                   int rows, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    const unsigned grid = grid_cap(nblocks, 1 << 20);
    if (smode == 0)
        hipLaunchKernelGGL((compact_kernel<double, double>), dim3(grid), dim3(256), 0, st, blocks,
                           nblocks, rank, coff, cbase, eoff, (const double*)src, (double*)dst,
                           rows);
    else if (smode == 1)
        hipLaunchKernelGGL((compact_kernel<float, float>), dim3(grid), dim3(256), 0, st, blocks,
                           nblocks, rank, coff, cbase, eoff, (const float*)src, (float*)dst, rows);
    else
        hipLaunchKernelGGL((compact_kernel<uint16_t, float>), dim3(grid), dim3(256), 0, st,
                           blocks, nblocks, rank, coff, cbase, eoff, (const float*)src,
                           (uint16_t*)dst, rows);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_compact_v(const int4* blocks, int64_t nblocks, const int32_t* rank,
                            const int64_t* cap_voff, int64_t cap_base, const int64_t* voff,
                            const void* Vcap, void* V, int smode, hipStream_t st) {
    return compact(blocks, nblocks, rank, cap_voff, cap_base, voff, Vcap, V, smode, 0, st);
}

hipError_t launch_compact_u(const int4* blocks, int64_t nblocks, const int32_t* rank,
                            const int64_t* cap_uoff, int64_t cap_base, const int64_t* uoff,
                            const void* Ucap, void* U, int smode, hipStream_t st) {
    return compact(blocks, nblocks, rank, cap_uoff, cap_base, uoff, Ucap, U, smode, 1, st);
}

hipError_t launch_add_const(int64_t* data, int64_t n, int64_t c, hipStream_t st) {
    if (n <= 0 || c == 0) return hipSuccess;
    hipLaunchKernelGGL(add_const_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, data,
                       n, c);
    return hipGetLastError();
}

hipError_t launch_chunk_bounds(const int64_t* cap_off, int64_t nb, int64_t step, int nchunks,
                               int64_t* bnd, hipStream_t st) {
    hipLaunchKernelGGL(chunk_bounds_kernel, dim3((unsigned)((nchunks + 1 + 255) / 256)), dim3(256),
                       0, st, cap_off, nb, step, nchunks, bnd);
    return hipGetLastError();
}

hipError_t launch_gather_x(const void* x, const int32_t* perm, int64_t n, void* xm, int f64,
                           hipStream_t st, int64_t base) {
    if (n <= 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(gather_x_kernel<double>, dim3((unsigned)((n + 255) / 256)), dim3(256),
                           0, st, (const double*)x, perm, n, (double*)xm, base);
    else
        hipLaunchKernelGGL(gather_x_kernel<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           st, (const float*)x, perm, n, (float*)xm, base);
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

hipError_t launch_rowtile(int64_t ntiles, const int32_t* tile_lo, const int64_t* meta,
                          const int64_t* widx, const void* upool, const void* npool,
                          const void* vecpool, const int32_t* perm, double alpha, double beta,
                          double sigma2, void* z, int max_tile, int fmode, int nmode,
                          int config, const void* soa, int64_t n, int d, KernelFn kern,
                          hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
#define HMX_RTD(SU, SN, T)                                                                     \
    return rowtile_dispatch<SU, SN, T>(ntiles, tile_lo, meta, widx, upool, npool, vecpool, perm, \
                                       alpha, beta, sigma2, z, max_tile, config, soa, n, d, kern, \
                                       st)
    if (fmode == 0 && nmode == 0) HMX_RTD(double, double, double);
    if (fmode == 1 && nmode == 1) HMX_RTD(float, float, float);
    if (fmode == 2 && nmode == 2) HMX_RTD(uint16_t, uint16_t, float);
    if (fmode == 2 && nmode == 1) HMX_RTD(uint16_t, float, float);
    if (fmode == 0 && nmode == 3) HMX_RTD(double, Recompute<double>, double);
    if (fmode == 1 && nmode == 3) HMX_RTD(float, Recompute<float>, float);
    if (fmode == 2 && nmode == 3) HMX_RTD(uint16_t, Recompute<float>, float);
#undef HMX_RTD
    return hipErrorInvalidValue;
}

}  // namespace hmx
