// Near-field assembly and the batched H-matrix-vector product (Algorithm 3
// in flat form, Section 5.4).
//
// Storage.  The rows of the matrix are cut into row tiles, the leaf clusters
// of the cluster tree.  A piece is the part of one leaf block that falls in
// one tile: the tile's rows of a dense block A|tau x sigma (ncols = |sigma|,
// weights x|sigma), or the tile's rows of the factor U of an admissible block
// (ncols = rank, weights t_b = V_b^T x|sigma).  All pieces of a tile are
// stored one after another, column-major with the tile's leading dimension
// ld_t = (tile rows rounded up to 16 bytes), so a tile is one contiguous
// ld_t x C_t matrix in the matrix pool and column k of it is multiplied by
// vec[widx[k]].  Padding rows hold zeros.
//   vector pool: [ x in Morton order (n) | t_b for every admissible leaf ]
//   V pool     : V_b (n_b x r_b) column-major per admissible leaf.
// Matvec = gather x -> phase 1 (all t_b) -> phase 2 (one workgroup per tile,
// streaming its contiguous region) -> scatter to the original order with
// alpha, beta, sigma2.  Each z row is written by one workgroup and every sum
// has a fixed order, so the product is deterministic.
#include "hmx_internal.h"

namespace hmx {

namespace {

unsigned grid_cap(int64_t nb, int64_t cap) { return (unsigned)(nb < cap ? nb : cap); }

// elements per 16-byte vector for an entry size, and the padded tile height
__device__ __host__ __forceinline__ int vec_elems(int esz) { return 16 / esz; }
__device__ __host__ __forceinline__ int tile_ld(int rows, int esz) {
    const int v = vec_elems(esz);
    return (rows + v - 1) / v * v;
}

// ---------------------------------------------------------------------------
// storage types: the pools hold S (double, float or bfloat16 bits), the
// arithmetic runs in T (double or float).  bfloat16 = the upper 16 bits of an
// IEEE float; conversion rounds to nearest, ties to even.
// ---------------------------------------------------------------------------
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
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
    static __device__ __forceinline__ void get(const u32x4& r, double* o) {
        o[0] = __hiloint2double((int)r[1], (int)r[0]);
        o[1] = __hiloint2double((int)r[3], (int)r[2]);
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
        case 3: v = (int64_t)rank[b] * m; break;
        case 4: v = (int64_t)rank[b] * nc; break;
        case 5: v = rank[b]; break;
        case 7: v = (m + nc) * mult; break;
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

// sorted order -> pieces; also each piece's data size and column count
__global__ void piece_gather_kernel(const Piece* __restrict__ src,
                                    const uint32_t* __restrict__ order, int64_t np,
                                    Piece* __restrict__ dst, int64_t* __restrict__ size,
                                    int64_t* __restrict__ cols, const int32_t* __restrict__ tile_lo,
                                    int esz) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= np) return;
    const Piece pc = src[order[i]];
    dst[i] = pc;
    const int mt = tile_lo[pc.tile + 1] - tile_lo[pc.tile];
    size[i] = (int64_t)tile_ld(mt, esz) * pc.ncols;
    cols[i] = pc.ncols;
}

// after the scans: piece data offsets, and the weight index of every column
__global__ void piece_layout_kernel(Piece* __restrict__ pieces, int64_t np,
                                    const int64_t* __restrict__ doff,
                                    const int64_t* __restrict__ coff,
                                    int64_t* __restrict__ widx) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= np) return;
    Piece pc = pieces[i];
    pc.d_off = doff[i];
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

// per tile: first column and data offset (from its first piece)
__global__ void tile_meta_kernel(const int64_t* __restrict__ tile_ptr, int64_t ntiles,
                                 int64_t np, const int64_t* __restrict__ doff,
                                 const int64_t* __restrict__ coff, int64_t total_cols,
                                 int64_t total_data, int64_t* __restrict__ tile_col,
                                 int64_t* __restrict__ tile_doff) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    const int64_t p = tile_ptr[t];
    tile_col[t] = p < np ? coff[p] : total_cols;
    tile_doff[t] = p < np ? doff[p] : total_data;
}

// Fill the matrix pool piece by piece: dense pieces evaluate phi (the near
// field, Section 5.4.2), factor pieces copy the tile's rows of U_b from the
// ACA capacity pool.  Padding rows are zero.
template <typename S, typename T>
__global__ __launch_bounds__(256) void piece_data_kernel(
    const Piece* __restrict__ pieces, int64_t np, const int32_t* __restrict__ tile_lo,
    const int4* __restrict__ adm, const int4* __restrict__ dense,
    const int64_t* __restrict__ ucap_off, const T* __restrict__ Ucap, const T* __restrict__ soa,
    int64_t n, int d, KernelEval<T> K, S* __restrict__ pool) {
    constexpr int ssz = sizeof(S);
    for (int64_t p = blockIdx.x; p < np; p += gridDim.x) {
        const Piece pc = pieces[p];
        const int32_t r0 = tile_lo[pc.tile];
        const int mt = tile_lo[pc.tile + 1] - r0;
        const int ld = tile_ld(mt, ssz);
        S* __restrict__ out = pool + pc.d_off;
        const int64_t tot = (int64_t)ld * pc.ncols;
        const bool is_factor = pc.blk >= 0;
        const int4 bl = is_factor ? adm[pc.blk] : dense[-pc.blk - 1];
        const int m = bl.y - bl.x;
        const T* __restrict__ src = is_factor ? Ucap + ucap_off[pc.blk] + pc.row0 : nullptr;
        int i = threadIdx.x, c = 0;
        while (i >= ld) {
            i -= ld;
            ++c;
        }
        for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
            T v = (T)0;
            if (i < mt) {
                if (is_factor) {
                    v = src[(int64_t)c * m + i];
                } else {
                    T x[3], y[3];
                    load_pt(soa, n, d, (int64_t)r0 + i, x);
                    load_pt(soa, n, d, (int64_t)bl.z + c, y);
                    v = phi(K, x, y, d);
                }
            }
            out[e] = Store<S, T>::put(v);
            i += blockDim.x;
            while (i >= ld) {
                i -= ld;
                ++c;
            }
        }
    }
}

template <typename T>
__global__ void gather_x_kernel(const T* __restrict__ x, const int32_t* __restrict__ perm,
                                int64_t n, T* __restrict__ xm) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) xm[i] = x[perm[i]];
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

// V compaction: the first r_b columns of each V_b from the capacity pool
template <typename S, typename T>
__global__ __launch_bounds__(256) void compact_v_kernel(const int4* __restrict__ blocks,
                                                        int64_t nblocks,
                                                        const int32_t* __restrict__ rank,
                                                        const int64_t* __restrict__ cv,
                                                        int64_t cbase,
                                                        const int64_t* __restrict__ ev,
                                                        const T* __restrict__ Vcap,
                                                        S* __restrict__ V) {
    for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
        const int4 bl = blocks[b];
        const int64_t nc = bl.w - bl.z, r = rank[b];
        const T* sv = Vcap + (cv[b] - cbase);
        S* dv = V + ev[b];
        for (int64_t e = threadIdx.x; e < r * nc; e += blockDim.x) dv[e] = Store<S, T>::put(sv[e]);
    }
}

// U compaction into the exact per-block pool (compute type, source of the
// tile-major matrix pool)
template <typename T>
__global__ __launch_bounds__(256) void compact_u_kernel(const int4* __restrict__ blocks,
                                                        int64_t nblocks,
                                                        const int32_t* __restrict__ rank,
                                                        const int64_t* __restrict__ cu,
                                                        int64_t cbase,
                                                        const int64_t* __restrict__ eu,
                                                        const T* __restrict__ Ucap,
                                                        T* __restrict__ U) {
    for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
        const int4 bl = blocks[b];
        const int64_t m = bl.y - bl.x, r = rank[b];
        const T* su = Ucap + (cu[b] - cbase);
        T* du = U + eu[b];
        for (int64_t e = threadIdx.x; e < r * m; e += blockDim.x) du[e] = su[e];
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

// column -> admissible leaf map for the flattened factor columns
__global__ void col_block_kernel(const int32_t* __restrict__ rank,
                                 const int64_t* __restrict__ toff, int64_t nadm,
                                 int32_t* __restrict__ col_block) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nadm) return;
    const int64_t o = toff[b];
    for (int l = 0; l < rank[b]; ++l) col_block[o + l] = (int32_t)b;
}

// phase 1: t_b[l] = sum_j V_b[j, l] x[slo + j]; one wave per column of the
// flattened list of all factor columns
template <typename T>
__device__ __forceinline__ void load_x16(const T* p, T* o);
template <>
__device__ __forceinline__ void load_x16<float>(const float* p, float* o) {
    const f32x4 v = *(const f32x4*)p;
    o[0] = v[0];
    o[1] = v[1];
    o[2] = v[2];
    o[3] = v[3];
}
template <>
__device__ __forceinline__ void load_x16<double>(const double* p, double* o) {
    const f64x2 v = *(const f64x2*)p;
    o[0] = v[0];
    o[1] = v[1];
}

template <typename S, typename T>
__global__ __launch_bounds__(256) void far_phase1_kernel(
    const int4* __restrict__ adm, const int32_t* __restrict__ col_block,
    const int64_t* __restrict__ voff, const int64_t* __restrict__ toff, const S* __restrict__ V,
    T* __restrict__ vec, int64_t n, int64_t ncols_total) {
    constexpr int VS = Dec<S, T>::n;  // values per 16-byte load of V
    constexpr int VT = 16 / sizeof(T);
    const int lane = threadIdx.x & 63;
    const int64_t k = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    if (k >= ncols_total) return;
    const int b = col_block[k];
    const int4 bl = adm[b];
    const int nc = bl.w - bl.z;
    const int l = (int)(k - toff[b]);
    const int64_t cofs = voff[b] + (int64_t)l * nc;
    const S* __restrict__ col = V + cofs;
    const T* __restrict__ xs = vec + bl.z;
    T acc = 0;
    if ((cofs % VS) == 0 && (nc % VS) == 0 && ((int64_t)bl.z % VT) == 0) {
        const u32x4* __restrict__ c16 = (const u32x4*)col;
        const int nv = nc / VS;
        for (int j = lane; j < nv; j += 64) {
            T a[VS], xv[VS];
            Dec<S, T>::get(nt_load(c16 + j), a);
#pragma unroll
            for (int u = 0; u < VS / VT; ++u) load_x16<T>(xs + (int64_t)j * VS + u * VT, xv + u * VT);
#pragma unroll
            for (int e = 0; e < VS; ++e) acc += a[e] * xv[e];
        }
    } else {
        for (int j = lane; j < nc; j += 64) {
            T a;
            if constexpr (sizeof(S) == 2)
                a = __uint_as_float((uint32_t)(*(const uint16_t*)(col + j)) << 16);
            else
                a = (T)col[j];
            acc += a * xs[j];
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) vec[n + k] = acc;
}

// phase 2: one workgroup per row tile.  The tile is a contiguous ld x C
// column-major matrix; column k is weighted by vec[widx[k]].  Weights are
// gathered into LDS a chunk of kChunk columns at a time, so the streaming
// loads never wait on an index lookup.  The 4 waves split into
// G = 4 * (64 / L) column groups of L lanes; lane q of a group owns RV
// 16-byte vectors of rows (vector v * L + q).  Groups take interleaved
// columns, kUnroll in flight per lane, with non-temporal loads (every matrix
// byte is read once per product); the G partial row sets are summed in LDS
// in a fixed order and the tile is scattered to the original order.
constexpr int kTileThreads = 256;
constexpr int kChunk = 1024;
constexpr int kUnroll = 8;

template <typename S, typename T, int L, int RV>
__global__ __launch_bounds__(kTileThreads) void rowtile_kernel(
    int64_t ntiles, const int32_t* __restrict__ tile_lo, const int64_t* __restrict__ tile_col,
    const int64_t* __restrict__ tile_doff, const int64_t* __restrict__ widx,
    const S* __restrict__ pool, const T* __restrict__ vec, const int32_t* __restrict__ perm,
    T alpha, T beta, T sigma2, T* __restrict__ z) {
    constexpr int VEC = Dec<S, T>::n;  // rows per 16-byte vector
    constexpr int SUB = 64 / L;
    constexpr int G = 4 * SUB;
    constexpr int RPG = L * RV * VEC;  // rows per pass
    __shared__ T red[G * RPG];
    __shared__ T sw[kChunk];
    const int tid = threadIdx.x, lane = tid & 63;
    // the group index is wave-uniform when a group is a whole wave
    const int g = (SUB == 1) ? __builtin_amdgcn_readfirstlane(tid >> 6) : (tid >> 6) * SUB + lane / L;
    const int q = lane % L;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int32_t r0 = tile_lo[t];
        const int mt = tile_lo[t + 1] - r0;
        const int ld = (mt + VEC - 1) / VEC * VEC;
        const int64_t k0 = tile_col[t], nk = tile_col[t + 1] - k0;
        const S* __restrict__ base0 = pool + tile_doff[t];
        const int64_t* __restrict__ wi = widx + k0;
        for (int rb = 0; rb < ld; rb += RPG) {
            const int nvec = ((ld - rb) < RPG ? (ld - rb) : RPG) / VEC;  // vectors in this pass
            T acc[RV][VEC];
#pragma unroll
            for (int v = 0; v < RV; ++v)
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[v][e] = 0;
            for (int64_t kc = 0; kc < nk; kc += kChunk) {
                const int cnt = (nk - kc) < kChunk ? (int)(nk - kc) : kChunk;
                for (int j = tid; j < cnt; j += kTileThreads) sw[j] = vec[wi[kc + j]];
                __syncthreads();
                const S* __restrict__ base = base0 + rb + kc * ld;
                int c = g;
                for (; c + (kUnroll - 1) * G < cnt; c += kUnroll * G) {
                    T w[kUnroll];
                    const u32x4* cp[kUnroll];
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u) {
                        w[u] = sw[c + u * G];
                        cp[u] = (const u32x4*)(base + (int64_t)(c + u * G) * ld);
                    }
#pragma unroll
                    for (int v = 0; v < RV; ++v) {
                        const int vi = v * L + q;
                        if (vi < nvec) {
                            u32x4 raw[kUnroll];
#pragma unroll
                            for (int u = 0; u < kUnroll; ++u) raw[u] = nt_load(cp[u] + vi);
#pragma unroll
                            for (int u = 0; u < kUnroll; ++u) {
                                T a[VEC];
                                Dec<S, T>::get(raw[u], a);
#pragma unroll
                                for (int e = 0; e < VEC; ++e) acc[v][e] += a[e] * w[u];
                            }
                        }
                    }
                }
                for (; c < cnt; c += G) {
                    const T w0 = sw[c];
                    const u32x4* c0 = (const u32x4*)(base + (int64_t)c * ld);
#pragma unroll
                    for (int v = 0; v < RV; ++v) {
                        const int vi = v * L + q;
                        if (vi < nvec) {
                            T a[VEC];
                            Dec<S, T>::get(nt_load(c0 + vi), a);
#pragma unroll
                            for (int e = 0; e < VEC; ++e) acc[v][e] += a[e] * w0;
                        }
                    }
                }
                __syncthreads();
            }
            // sum the G partial row sets in a fixed order
#pragma unroll
            for (int v = 0; v < RV; ++v)
#pragma unroll
                for (int e = 0; e < VEC; ++e) red[g * RPG + (v * L + q) * VEC + e] = acc[v][e];
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

template <typename S, typename T>
hipError_t rowtile_dispatch(int64_t ntiles, const int32_t* tile_lo, const int64_t* tile_col,
                            const int64_t* tile_doff, const int64_t* widx, const void* pool,
                            const void* vecpool, const int32_t* perm, double alpha, double beta,
                            double sigma2, void* z, int max_tile, hipStream_t st) {
    constexpr int VEC = Dec<S, T>::n;
    const int need = (max_tile + VEC - 1) / VEC;  // vectors per tile column
    int L = 16, RV = 1;
    while (L < need && L < 64) L *= 2;
    while (L * RV < need && RV < 4) RV *= 2;
    const unsigned grid = grid_cap(ntiles, 1 << 20);
#define HMX_RT(LL, RR)                                                                          \
    hipLaunchKernelGGL((rowtile_kernel<S, T, LL, RR>), dim3(grid), dim3(kTileThreads), 0, st, \
                       ntiles, tile_lo, tile_col, tile_doff, widx, (const S*)pool,             \
                       (const T*)vecpool, perm, (T)alpha, (T)beta, (T)sigma2, (T*)z)
    if (L == 16)
        HMX_RT(16, 1);
    else if (L == 32)
        HMX_RT(32, 1);
    else if (RV == 1)
        HMX_RT(64, 1);
    else if (RV == 2)
        HMX_RT(64, 2);
    else
        HMX_RT(64, 4);
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
                               Piece* dst, int64_t* size, int64_t* cols, const int32_t* tile_lo,
                               int esz, hipStream_t st) {
    if (npieces == 0) return hipSuccess;
    hipLaunchKernelGGL(piece_gather_kernel, dim3((unsigned)((npieces + 255) / 256)), dim3(256), 0,
                       st, src, order, npieces, dst, size, cols, tile_lo, esz);
    return hipGetLastError();
}

hipError_t launch_piece_layout(Piece* pieces, int64_t np, const int64_t* doff,
                               const int64_t* coff, int64_t* widx, hipStream_t st) {
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(piece_layout_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st,
                       pieces, np, doff, coff, widx);
    return hipGetLastError();
}

hipError_t launch_tile_offsets(const uint64_t* sorted_tile, int64_t npieces, int64_t ntiles,
                               int64_t* tile_ptr, hipStream_t st) {
    hipLaunchKernelGGL(tile_ptr_kernel, dim3((unsigned)((ntiles + 1 + 255) / 256)), dim3(256), 0,
                       st, sorted_tile, npieces, ntiles, tile_ptr);
    return hipGetLastError();
}

hipError_t launch_tile_meta(const int64_t* tile_ptr, int64_t ntiles, int64_t np,
                            const int64_t* doff, const int64_t* coff, int64_t total_cols,
                            int64_t total_data, int64_t* tile_col, int64_t* tile_doff,
                            hipStream_t st) {
    hipLaunchKernelGGL(tile_meta_kernel, dim3((unsigned)((ntiles + 1 + 255) / 256)), dim3(256), 0,
                       st, tile_ptr, ntiles, np, doff, coff, total_cols, total_data, tile_col,
                       tile_doff);
    return hipGetLastError();
}

// storage modes: 0 = F64/F64, 1 = F32/F32, 2 = BF16 storage with F32 arithmetic
hipError_t launch_piece_data(const Piece* pieces, int64_t np, const int32_t* tile_lo,
                             const int4* adm, const int4* dense, const int64_t* ucap_off,
                             const void* Ucap, const void* soa, int64_t n, int d, KernelFn kern,
                             void* pool, int smode, hipStream_t st) {
    if (np == 0) return hipSuccess;
    const unsigned grid = grid_cap(np, 1 << 20);
    if (smode == 0)
        hipLaunchKernelGGL((piece_data_kernel<double, double>), dim3(grid), dim3(256), 0, st,
                           pieces, np, tile_lo, adm, dense, ucap_off, (const double*)Ucap,
                           (const double*)soa, n, d, KernelEval<double>(kern), (double*)pool);
    else if (smode == 1)
        hipLaunchKernelGGL((piece_data_kernel<float, float>), dim3(grid), dim3(256), 0, st,
                           pieces, np, tile_lo, adm, dense, ucap_off, (const float*)Ucap,
                           (const float*)soa, n, d, KernelEval<float>(kern), (float*)pool);
    else
        hipLaunchKernelGGL((piece_data_kernel<uint16_t, float>), dim3(grid), dim3(256), 0, st,
                           pieces, np, tile_lo, adm, dense, ucap_off, (const float*)Ucap,
                           (const float*)soa, n, d, KernelEval<float>(kern), (uint16_t*)pool);
    return hipGetLastError();
}

hipError_t launch_compact_v(const int4* blocks, int64_t nblocks, const int32_t* rank,
                            const int64_t* cap_voff, int64_t cap_base, const int64_t* voff,
                            const void* Vcap, void* V, int smode, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    const unsigned grid = grid_cap(nblocks, 1 << 20);
    if (smode == 0)
        hipLaunchKernelGGL((compact_v_kernel<double, double>), dim3(grid), dim3(256), 0, st,
                           blocks, nblocks, rank, cap_voff, cap_base, voff, (const double*)Vcap,
                           (double*)V);
    else if (smode == 1)
        hipLaunchKernelGGL((compact_v_kernel<float, float>), dim3(grid), dim3(256), 0, st,
                           blocks, nblocks, rank, cap_voff, cap_base, voff, (const float*)Vcap,
                           (float*)V);
    else
        hipLaunchKernelGGL((compact_v_kernel<uint16_t, float>), dim3(grid), dim3(256), 0, st,
                           blocks, nblocks, rank, cap_voff, cap_base, voff, (const float*)Vcap,
                           (uint16_t*)V);
    return hipGetLastError();
}

hipError_t launch_compact_u(const int4* blocks, int64_t nblocks, const int32_t* rank,
                            const int64_t* cap_uoff, int64_t cap_base, const int64_t* uoff,
                            const void* Ucap, void* U, int f64, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    const unsigned grid = grid_cap(nblocks, 1 << 20);
    if (f64)
        hipLaunchKernelGGL(compact_u_kernel<double>, dim3(grid), dim3(256), 0, st, blocks, nblocks,
                           rank, cap_uoff, cap_base, uoff, (const double*)Ucap, (double*)U);
    else
        hipLaunchKernelGGL(compact_u_kernel<float>, dim3(grid), dim3(256), 0, st, blocks, nblocks,
                           rank, cap_uoff, cap_base, uoff, (const float*)Ucap, (float*)U);
    return hipGetLastError();
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
                             void* vecpool, int64_t n, int smode, hipStream_t st) {
    if (ncols_total == 0) return hipSuccess;
    const int64_t nblk = (ncols_total + 3) / 4;  // 4 waves (columns) per workgroup
    if (nblk > 0x7fffffffll) return hipErrorInvalidValue;
    if (smode == 0)
        hipLaunchKernelGGL((far_phase1_kernel<double, double>), dim3((unsigned)nblk), dim3(256),
                           0, st, adm, col_block, voff, toff, (const double*)V, (double*)vecpool,
                           n, ncols_total);
    else if (smode == 1)
        hipLaunchKernelGGL((far_phase1_kernel<float, float>), dim3((unsigned)nblk), dim3(256), 0,
                           st, adm, col_block, voff, toff, (const float*)V, (float*)vecpool, n,
                           ncols_total);
    else
        hipLaunchKernelGGL((far_phase1_kernel<uint16_t, float>), dim3((unsigned)nblk), dim3(256),
                           0, st, adm, col_block, voff, toff, (const uint16_t*)V,
                           (float*)vecpool, n, ncols_total);
    return hipGetLastError();
}

hipError_t launch_rowtile(int64_t ntiles, const int32_t* tile_lo, const int64_t* tile_col,
                          const int64_t* tile_doff, const int64_t* widx, const void* pool,
                          const void* vecpool, const int32_t* perm, double alpha, double beta,
                          double sigma2, void* z, int max_tile, int smode, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    if (smode == 0)
        return rowtile_dispatch<double, double>(ntiles, tile_lo, tile_col, tile_doff, widx, pool,
                                                vecpool, perm, alpha, beta, sigma2, z, max_tile,
                                                st);
    if (smode == 1)
        return rowtile_dispatch<float, float>(ntiles, tile_lo, tile_col, tile_doff, widx, pool,
                                              vecpool, perm, alpha, beta, sigma2, z, max_tile, st);
    return rowtile_dispatch<uint16_t, float>(ntiles, tile_lo, tile_col, tile_doff, widx, pool,
                                             vecpool, perm, alpha, beta, sigma2, z, max_tile, st);
}

}  // namespace hmx
