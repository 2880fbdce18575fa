// The H-matrix product with several right-hand sides, Z = alpha H X + beta Z
// (X with m columns): the same two phases as the single-vector product
// (Algorithm 3 batched as in Section 5.4), with every stored entry read
// once for up to M = 16 right-hand sides instead of once per vector.
//
// Vectors are held point-major, M values per point: vec[i * M + c] is
// right-hand side c at Morton position i (the first n entries), or at
// far-field column n + k (the t entries), so a column's M weights are one
// contiguous run.
//
//   * gather:    vec[(col0 + i) M + c] = X[perm[col0 + i] - col0 + c ldx];
//   * phase 1:   T_b = V_b^T X|sigma_b by row tiles, partial sums per
//                (column, tile);
//   * reduce:    the partials of each t entry summed over its tiles in tile
//                order (as for one vector);
//   * row tiles: Z rows = sum over the tile's columns of column x weights
//                (factor columns with the t entries, near-field columns with
//                x), near-field columns read from the pool or evaluated from
//                the coordinates.
// With 8 or 16 sides (stored near field) both contractions run on the
// matrix cores (the mfma kernels below): a stored entry then carries 32
// flops, more than the vector units sustain at HBM speed.  With 1, 2 or 4
// sides, or a near field evaluated in the product, they run on the vector
// units: phase 1 with groups of 8 lanes taking two source columns at a time
// and a butterfly over the group; row tiles with one wave per pass of 64 VR
// rows, each lane owning VR consecutive rows, weights staged in LDS.
// All sums run in a fixed order, so the product is deterministic; column c
// of the result sums the same terms as the single-vector product of X's
// column c, in another order.
#include "hmx_internal.h"

namespace hmx {

namespace {

// rows a lane owns per load: 4 for FP32 and BF16 (16- and 8-byte loads),
// 2 for FP64 (16 bytes)
template <typename S>
struct MmUnit;
template <>
struct MmUnit<double> {
    static constexpr int VR = 2;
    typedef double2 Raw;
    static __device__ __forceinline__ void get(const Raw& v, double* o) {
        o[0] = v.x;
        o[1] = v.y;
    }
};
template <>
struct MmUnit<float> {
    static constexpr int VR = 4;
    typedef float4 Raw;
    static __device__ __forceinline__ void get(const Raw& v, float* o) {
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
};
template <>
struct MmUnit<uint16_t> {
    static constexpr int VR = 4;
    typedef uint2 Raw;
    static __device__ __forceinline__ void get(const Raw& v, float* o) {
        o[0] = __uint_as_float(v.x << 16);
        o[1] = __uint_as_float(v.x & 0xffff0000u);
        o[2] = __uint_as_float(v.y << 16);
        o[3] = __uint_as_float(v.y & 0xffff0000u);
    }
};

template <typename S>
__device__ __forceinline__ typename MmUnit<S>::Raw mm_raw(const S* p) {
    return *(const typename MmUnit<S>::Raw*)p;
}

// M weights of one column, 16 bytes at a time when M allows
template <typename T, int M>
__device__ __forceinline__ void mm_copy_weights(T* __restrict__ dst, const T* __restrict__ src) {
    constexpr int W = 16 / (int)sizeof(T);  // values per 16-byte move
    if constexpr (M % W == 0) {
        typedef T V __attribute__((ext_vector_type(W)));
#pragma unroll
        for (int c = 0; c < M; c += W) *(V*)(dst + c) = *(const V*)(src + c);
    } else {
#pragma unroll
        for (int c = 0; c < M; ++c) dst[c] = src[c];
    }
}

__device__ __host__ __forceinline__ int mm_ld(int rows, int R) { return (rows + R - 1) / R * R; }

inline unsigned mm_grid(int64_t n, int b = 256) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + b - 1) / b, 1 << 20));
}

// sides c >= mr (a group padded to the matrix cores' width) are zero
template <typename T, int M>
__global__ void mm_gather_kernel(const T* __restrict__ X, int64_t ldx,
                                 const int32_t* __restrict__ perm, int64_t ncols, int64_t col0,
                                 int mr, T* __restrict__ vec) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ncols * M;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / M;
        const int c = (int)(e % M);
        vec[(col0 + i) * M + c] = c < mr ? X[(perm[col0 + i] - col0) + c * ldx] : (T)0;
    }
}

// one lane's share of U source columns (col, col + ld, ...; nu of them
// real, the others repeat the first and count zero) against M right-hand
// sides: row vectors q, q + L, ... of each column, B row vectors of every
// column loaded before any is used, each X row read once (from LDS with row
// stride XS, or from the point-major vector xt) for all U columns
template <typename S, typename T, int M, int B, int L, int U, bool STAGED>
__device__ __forceinline__ void mm_p1_rows(const S* __restrict__ col, int ld, int nu, int mt,
                                           int q, const T* __restrict__ xs, int xstride,
                                           T (&acc)[U][M]) {
    constexpr int VR = MmUnit<S>::VR;
    for (int u0 = q * VR; u0 < ld; u0 += B * L * VR) {
        typename MmUnit<S>::Raw raw[U][B];
#pragma unroll
        for (int k = 0; k < U; ++k)
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int u = u0 + b * L * VR;
                raw[k][b] = mm_raw(col + (int64_t)(k < nu ? k : 0) * ld + (u < ld ? u : u0));
            }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int u = u0 + b * L * VR;
            const bool in = u < ld;
            const int uu = in ? u : u0;
            T a[U][VR];
#pragma unroll
            for (int k = 0; k < U; ++k) MmUnit<S>::get(raw[k][b], a[k]);
#pragma unroll
            for (int e = 0; e < VR; ++e) {
                const int row = uu + e;
                // rows past the tile (or past a column group's end) count zero
                const bool live = in && (STAGED || row < mt);
                const T* __restrict__ xr = xs + (int64_t)(STAGED || row < mt ? row : 0) * xstride;
                T xv[M];
#pragma unroll
                for (int c = 0; c < M; ++c) xv[c] = xr[c];
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const T ae = (live && k < nu) ? a[k][e] : (T)0;
#pragma unroll
                    for (int c = 0; c < M; ++c) acc[k][c] += ae * xv[c];
                }
            }
        }
    }
}

template <typename S, typename T, int M>
__global__ __launch_bounds__(256) void mm_p1_kernel(int64_t ntiles,
                                                    const int32_t* __restrict__ tile_lo,
                                                    const int64_t* __restrict__ meta, int ms,
                                                    int R, const S* __restrict__ pool,
                                                    const T* __restrict__ vec,
                                                    T* __restrict__ partial, int64_t pbase) {
    constexpr int L = 8;         // lanes per column group
    constexpr int G = 256 / L;   // column groups per workgroup
    constexpr int U = 2;         // columns a group takes at a time
    constexpr int B = 8 / U;     // row vectors of each column loaded ahead
    constexpr int XS = M + 1;    // padded LDS row stride: a group's 8 lanes read 8 banks
    constexpr int SROWS = 16384 / (XS * (int)sizeof(T));  // rows of X staged in LDS
    __shared__ __align__(16) T sx[SROWS * XS];
    const int g = threadIdx.x / L, q = threadIdx.x % L;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t c0 = meta[ms * t + 1];
        const int nc = (int)(meta[ms * (t + 1) + 1] - c0);
        if (nc <= 0) continue;
        const int32_t r0 = tile_lo[t];
        const int mt = tile_lo[t + 1] - r0;
        const int ld = mm_ld(mt, R);
        const S* __restrict__ base = pool + meta[ms * t + 2];
        const bool staged = ld <= SROWS;
        if (staged) {
            for (int i = threadIdx.x; i < ld * M; i += 256)
                sx[(i / M) * XS + i % M] =
                    i / M < mt ? vec[(int64_t)(r0 + i / M) * M + i % M] : (T)0;
            __syncthreads();
        }
        for (int cb = g * U; cb < nc; cb += G * U) {
            const int nu = nc - cb < U ? nc - cb : U;
            T acc[U][M];
#pragma unroll
            for (int k = 0; k < U; ++k)
#pragma unroll
                for (int c = 0; c < M; ++c) acc[k][c] = 0;
            const S* __restrict__ col = base + (int64_t)cb * ld;
            // X rows from LDS (staged tiles) or from the vector itself: the
            // choice is made once per tile, not per value
            if (staged)
                mm_p1_rows<S, T, M, B, L, U, true>(col, ld, nu, mt, q, sx, XS, acc);
            else
                mm_p1_rows<S, T, M, B, L, U, false>(col, ld, nu, mt, q, vec + (int64_t)r0 * M,
                                                    M, acc);
#pragma unroll
            for (int m = L / 2; m >= 1; m >>= 1)
#pragma unroll
                for (int k = 0; k < U; ++k)
#pragma unroll
                    for (int c = 0; c < M; ++c) acc[k][c] += __shfl_xor(acc[k][c], m, 64);
            // every lane of the group holds the totals; lane q writes sides q, q + 8
#pragma unroll
            for (int k = 0; k < U; ++k)
#pragma unroll
                for (int c = 0; c < M; ++c)
                    if (c % L == q && k < nu) partial[(pbase + c0 + cb + k) * M + c] = acc[k][c];
        }
        if (staged) __syncthreads();  // sx is refilled by the next tile
    }
}

template <typename T, int M>
__global__ void mm_p1_reduce_kernel(const int4* __restrict__ rec, int64_t ncols,
                                    const int64_t* __restrict__ pfc,
                                    const T* __restrict__ partial, T* __restrict__ vec,
                                    int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ncols;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int4 r = rec[k];
        const int64_t b = (int64_t)(((uint64_t)(uint32_t)r.y << 32) | (uint32_t)r.x);
        T s[M];
#pragma unroll
        for (int c = 0; c < M; ++c) s[c] = 0;
        for (int j = 0; j < r.z; ++j) {
            const T* p = partial + (pfc[b + j] + r.w) * M;
#pragma unroll
            for (int c = 0; c < M; ++c) s[c] += p[c];
        }
#pragma unroll
        for (int c = 0; c < M; ++c) vec[(n + k) * M + c] = s[c];
    }
}

template <typename SU, typename SN, typename T, int M, bool NR>
__global__ __launch_bounds__(64) void mm_rowtile_kernel(
    int64_t ntiles, const int32_t* __restrict__ tile_lo, const int64_t* __restrict__ meta,
    const int64_t* __restrict__ widx, const SU* __restrict__ upool, const SN* __restrict__ npool,
    const T* __restrict__ vec, const int32_t* __restrict__ perm, T alpha, T beta, T sigma2,
    T* __restrict__ Z, int64_t ldz, int R, const T* __restrict__ soa, int64_t n, int d,
    KernelEval<T> K) {
    constexpr int VR = MmUnit<SU>::VR;
    static_assert(NR || MmUnit<SN>::VR == VR, "one row unit for both pools");
    constexpr int KC = 256;  // columns whose weights are staged at a time
    constexpr int B = 8;     // columns each lane loads before using them
    __shared__ __align__(16) T sw[KC * M];
    const int lane = threadIdx.x;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int32_t r0 = tile_lo[t];
        const int mt = tile_lo[t + 1] - r0;
        const int ld = mm_ld(mt, R);
        const int rb = (int)blockIdx.y * 64 * VR;
        if (rb >= ld) continue;  // the same for the whole wave
        const int64_t k0 = meta[4 * t], k1 = meta[4 * t + 4];
        const int64_t ku = meta[4 * t + 5] - meta[4 * t + 1];
        const SU* __restrict__ ubase = upool + meta[4 * t + 2];
        const SN* __restrict__ nbase = NR ? npool : npool + meta[4 * t + 3];
        const int row = rb + lane * VR;
        const int lrow = row + VR <= ld ? row : ld - VR;  // loads stay inside the tile
        T acc[VR][M];
#pragma unroll
        for (int e = 0; e < VR; ++e)
#pragma unroll
            for (int c = 0; c < M; ++c) acc[e][c] = 0;
        T py[VR][3];
        if constexpr (NR) {
#pragma unroll
            for (int e = 0; e < VR; ++e) {
                const int64_t i = r0 + min(lrow + e, mt - 1);
#pragma unroll
                for (int k = 0; k < 3; ++k) py[e][k] = k < d ? soa[(int64_t)k * n + i] : (T)0;
            }
        }
        for (int64_t kc = k0; kc < k1; kc += KC) {
            const int nk = (int)min((int64_t)KC, k1 - kc);
            __syncthreads();  // the previous chunk's weights are used up
            {
                // each lane moves the M weights of columns lane, lane + 64, ...
                // (all their index loads first, then the weights)
                int64_t w[KC / 64];
#pragma unroll
                for (int u = 0; u < KC / 64; ++u) {
                    const int col = lane + 64 * u;
                    w[u] = col < nk ? widx[kc + col] : 0;
                }
#pragma unroll
                for (int u = 0; u < KC / 64; ++u) {
                    const int col = lane + 64 * u;
                    if (col < nk) mm_copy_weights<T, M>(sw + col * M, vec + w[u] * M);
                }
            }
            __syncthreads();
            const int ju = (int)max((int64_t)0, min((int64_t)nk, k0 + ku - kc));
            for (int j0 = 0; j0 < ju; j0 += B) {
                typename MmUnit<SU>::Raw raw[B];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int j = j0 + b < ju ? j0 + b : ju - 1;
                    raw[b] = mm_raw(ubase + (kc + j - k0) * ld + lrow);
                }
                // straight-line use of all B loads (columns past the part
                // repeat its last one and count zero), so they stay in flight
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int j = j0 + b < ju ? j0 + b : ju - 1;
                    const T msk = j0 + b < ju ? (T)1 : (T)0;
                    T a[VR];
                    MmUnit<SU>::get(raw[b], a);
                    const T* __restrict__ wj = sw + j * M;
#pragma unroll
                    for (int e = 0; e < VR; ++e) {
                        const T ae = a[e] * msk;
#pragma unroll
                        for (int c = 0; c < M; ++c) acc[e][c] += ae * wj[c];
                    }
                }
            }
            if constexpr (NR) {
                for (int j = ju; j < nk; ++j) {
                    const int64_t pj = widx[kc + j];
                    T y[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) y[k] = k < d ? soa[(int64_t)k * n + pj] : (T)0;
                    T a[VR];
#pragma unroll
                    for (int e = 0; e < VR; ++e) a[e] = phi(K, py[e], y, d);
#pragma unroll
                    for (int e = 0; e < VR; ++e)
#pragma unroll
                        for (int c = 0; c < M; ++c) acc[e][c] += a[e] * sw[j * M + c];
                }
            } else {
                for (int j0 = ju; j0 < nk; j0 += B) {
                    typename MmUnit<SN>::Raw raw[B];
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        const int j = j0 + b < nk ? j0 + b : nk - 1;
                        raw[b] = mm_raw(nbase + (kc + j - k0 - ku) * ld + lrow);
                    }
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        const int j = j0 + b < nk ? j0 + b : nk - 1;
                        const T msk = j0 + b < nk ? (T)1 : (T)0;
                        T a[VR];
                        MmUnit<SN>::get(raw[b], a);
                        const T* __restrict__ wj = sw + j * M;
#pragma unroll
                        for (int e = 0; e < VR; ++e) {
                            const T ae = a[e] * msk;
#pragma unroll
                            for (int c = 0; c < M; ++c) acc[e][c] += ae * wj[c];
                        }
                    }
                }
            }
        }
        if (row == lrow) {
#pragma unroll
            for (int e = 0; e < VR; ++e) {
                if (row + e >= mt) continue;
                const int64_t gi = r0 + row + e;
                const int64_t pi = perm[gi];
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    T s = acc[e][c];
                    if (sigma2 != (T)0) s += sigma2 * vec[gi * M + c];
                    T out = alpha * s;
                    if (beta != (T)0) out += beta * Z[pi + c * ldz];
                    Z[pi + c * ldz] = out;
                }
            }
        }
    }
}

// ---- matrix-core forms (8 or 16 right-hand sides) ----
//
// Both phases are contractions with 16 right-hand sides on one side, so they
// run on the 16 x 16 x 4 matrix instructions (FP32 for FP32 and BF16
// storage, BF16 decoded exactly to FP32; FP64 for FP64).  With 16 sides a
// stored entry carries 32 flops, which the vector units (FP32 fused
// multiply-add without packing: half the matrix rate) cannot keep up with at
// HBM speed.  Lane l = i + 16 k supplies A[i][k] and B[k][j = i]; its four
// results are D[drow(k, v)][i], v = 0..3, with drow(k, v) = 4 k + v for the
// FP32 instruction and k + 4 v for the FP64 one.  A lane's 16-byte load holds VR
// consecutive rows of one column, and element e of it feeds the e-th of VR
// instructions, so instruction e sums the rows congruent to e mod VR.

typedef float mm_f4 __attribute__((ext_vector_type(4)));
typedef double mm_d4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MfmaOp;
template <>
struct MfmaOp<float> {
    typedef mm_f4 Acc;
    static __device__ __forceinline__ Acc mac(float a, float b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int k, int v) { return 4 * k + v; }
};
template <>
struct MfmaOp<double> {
    typedef mm_d4 Acc;
    static __device__ __forceinline__ Acc mac(double a, double b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int k, int v) { return k + 4 * v; }
};

// VR consecutive rows of one column in one load (raw 32-bit words, so the
// load can be marked non-temporal: every entry is read once per product),
// decoded to the arithmetic type
typedef uint32_t mm_u4 __attribute__((ext_vector_type(4)));
typedef uint32_t mm_u2 __attribute__((ext_vector_type(2)));
template <typename S, int VR>
struct MfUnit;
template <>
struct MfUnit<double, 2> {
    typedef mm_u4 Raw;
    static __device__ __forceinline__ void get(const Raw& v, double* o) {
        o[0] = __builtin_bit_cast(double, ((uint64_t)v.y << 32) | v.x);
        o[1] = __builtin_bit_cast(double, ((uint64_t)v.w << 32) | v.z);
    }
};
template <>
struct MfUnit<float, 4> {
    typedef mm_u4 Raw;
    static __device__ __forceinline__ void get(const Raw& v, float* o) {
        o[0] = __uint_as_float(v.x);
        o[1] = __uint_as_float(v.y);
        o[2] = __uint_as_float(v.z);
        o[3] = __uint_as_float(v.w);
    }
};
template <>
struct MfUnit<uint16_t, 4> {
    typedef mm_u2 Raw;
    static __device__ __forceinline__ void get(const Raw& v, float* o) {
        o[0] = __uint_as_float(v.x << 16);
        o[1] = __uint_as_float(v.x & 0xffff0000u);
        o[2] = __uint_as_float(v.y << 16);
        o[3] = __uint_as_float(v.y & 0xffff0000u);
    }
};
template <>
struct MfUnit<uint16_t, 8> {
    typedef mm_u4 Raw;
    static __device__ __forceinline__ void get(const Raw& v, float* o) {
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o[2 * i] = __uint_as_float(w[i] << 16);
            o[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
        }
    }
};

// columns [ja, jb) of a staged chunk against their weights: column j's rows
// for this lane start at base + j ld, its weights at sw[j M].  PB K-steps of
// four columns are loaded (non-temporal: every entry is read once per
// product) and only then used; past jb a load repeats column jb - 1 and its
// weight is zero
template <typename S, typename T, int M, int VR, int PB>
__device__ __forceinline__ void mf_rows_part(const S* __restrict__ base, int ld, int ja, int jb,
                                             const T* __restrict__ sw, int li, int lk,
                                             typename MfmaOp<T>::Acc (&acc)[VR]) {
    typedef MfUnit<S, VR> Un;
    for (int j0 = ja; j0 < jb; j0 += 4 * PB) {
        typename Un::Raw raw[PB];
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const int j = j0 + 4 * b + lk;
            raw[b] = __builtin_nontemporal_load(
                (const typename Un::Raw*)(base + (int64_t)(j < jb ? j : jb - 1) * ld));
        }
        // all PB loads issued before the first use: keeps the scheduler from
        // sinking them next to their instructions (two in flight otherwise)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const int j = j0 + 4 * b + lk;
            const bool live = j < jb && li < M;
            const T wv = sw[(live ? j : ja) * M + (li < M ? li : 0)];
            const T w = live ? wv : (T)0;
            T a[VR];
            Un::get(raw[b], a);
#pragma unroll
            for (int e = 0; e < VR; ++e) acc[e] = MfmaOp<T>::mac(a[e], w, acc[e]);
        }
    }
}

// row tiles on the matrix cores: a workgroup of nw waves (blockDim.x / 64)
// per (tile, group of nw slabs); wave w owns the 16 VR rows of its slab and
// all M <= 16 right-hand sides.  The column weights pass through LDS, one
// column per staging thread per chunk (KC columns, 16 KB of weights),
// double-buffered: while a chunk is multiplied, the weights of the next one
// are loaded into registers and the column indices of the one after are
// read, so one barrier per chunk remains and no load waits on another.
// Factor columns first, then the stored near field
template <typename SU, typename SN, typename T, int M, int VR, int PB>
__global__ __launch_bounds__(256) void mm_rowtile_mfma_kernel(
    int64_t ntiles, const int32_t* __restrict__ tile_lo, const int64_t* __restrict__ meta,
    const int64_t* __restrict__ widx, const SU* __restrict__ upool, const SN* __restrict__ npool,
    const T* __restrict__ vec, const int32_t* __restrict__ perm, T alpha, T beta, T sigma2,
    T* __restrict__ Z, int64_t ldz, int R, int mr, int npass) {
    typedef MfmaOp<T> Op;
    constexpr int RS = 16 * VR;              // rows of a wave's slab
    constexpr int WV = 16 / (int)sizeof(T);  // weights per 16-byte move
    static_assert(M % WV == 0, "whole 16-byte moves of weights");
    typedef T WVec __attribute__((ext_vector_type(WV)));
    constexpr int KCM = 16384 / (M * (int)sizeof(T));  // 16 KB of weights per buffer
    __shared__ __align__(16) T sw[2][KCM * M];
    const int nw = (int)(blockDim.x >> 6);
    const int KC = min((int)blockDim.x, KCM);  // columns per chunk: one per staging thread
    const int wv = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int li = lane & 15, lk = lane >> 4;
    const int me = (int)threadIdx.x;
    const bool stager = me < KC;
    // one workgroup per (tile, group of nw slabs), the groups of a tile
    // consecutive in the grid (workgroups running together read whole columns)
    for (int64_t w = blockIdx.x; w < ntiles * npass; w += gridDim.x) {
        const int64_t t = w / npass;
        const int32_t r0 = tile_lo[t];
        const int mt = tile_lo[t + 1] - r0;
        const int ld = mm_ld(mt, R);
        const int slab0 = (int)(w - t * npass) * nw * RS;
        if (slab0 >= ld) continue;  // the same for the whole workgroup
        const int slab = slab0 + wv * RS;
        const bool active = slab < ld;
        // loads stay inside the column (a clamped lane's rows are past ld and discarded)
        const int lrow = min(slab + li * VR, ld - VR);
        const int64_t k0 = meta[4 * t], k1 = meta[4 * t + 4];
        const int64_t ku = meta[4 * t + 5] - meta[4 * t + 1];
        const SU* __restrict__ ubase = upool + meta[4 * t + 2] + lrow;
        const SN* __restrict__ nbase = npool + meta[4 * t + 3] + lrow;
        typename Op::Acc acc[VR];
#pragma unroll
        for (int e = 0; e < VR; ++e)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[e][v] = 0;
        // this thread's column of chunk c is k0 + c KC + me
        const int nch = (int)((k1 - k0 + KC - 1) / KC);
        int64_t idx_next = stager && k0 + KC + me < k1 ? widx[k0 + KC + me] : 0;  // chunk 1
        {
            const bool own = stager && k0 + me < k1;
            const int64_t i0 = own ? widx[k0 + me] : 0;
            if (own)
#pragma unroll
                for (int c = 0; c < M; c += WV)
                    *(WVec*)(&sw[0][me * M + c]) = *(const WVec*)(vec + i0 * M + c);
        }
        __syncthreads();
        for (int ch = 0; ch < nch; ++ch) {
            const int64_t kc = k0 + (int64_t)ch * KC;
            const int nk = (int)min((int64_t)KC, k1 - kc);
            // the next chunk's weights into registers, the indices of the one after
            WVec wr[M / WV];
            const bool has_next = stager && kc + KC + me < k1;
            if (has_next)
#pragma unroll
                for (int c = 0; c < M / WV; ++c) wr[c] = *(const WVec*)(vec + idx_next * M + c * WV);
            idx_next = stager && kc + 2 * KC + me < k1 ? widx[kc + 2 * KC + me] : 0;
            if (active) {
                const T* __restrict__ swc = sw[ch & 1];
                const int ju = (int)max((int64_t)0, min((int64_t)nk, k0 + ku - kc));
                if (ju > 0)
                    mf_rows_part<SU, T, M, VR, PB>(ubase + (kc - k0) * ld, ld, 0, ju, swc, li, lk,
                                                   acc);
                if (ju < nk)
                    mf_rows_part<SN, T, M, VR, PB>(nbase + (kc - k0 - ku) * ld, ld, ju, nk, swc,
                                                   li, lk, acc);
            }
            if (has_next)
#pragma unroll
                for (int c = 0; c < M / WV; ++c) *(WVec*)(&sw[(ch + 1) & 1][me * M + c * WV]) = wr[c];
            __syncthreads();
        }
        if (active && li < mr) {  // the group's real sides (mr <= M)
#pragma unroll
            for (int e = 0; e < VR; ++e)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = slab + VR * Op::drow(lk, v) + e;
                    if (row >= mt) continue;
                    const int64_t gi = r0 + row;
                    const int64_t zi = perm[gi] + li * ldz;
                    T s = acc[e][v];
                    if (sigma2 != (T)0) s += sigma2 * vec[gi * M + li];
                    T out = alpha * s;
                    if (beta != (T)0) out += beta * Z[zi];
                    Z[zi] = out;
                }
        }
    }
}

// phase 1 on the matrix cores: T = V^T X per row tile, the contraction over
// the tile's rows.  A wave takes 16 source columns (lane i's column cb + i)
// and runs down all rows, 4 VR per K-step; the tile's X rows are staged in
// LDS transposed (side-major, row stride XT), so a lane's VR rows of one side
// are one contiguous read; wider tiles read X from the vector itself
template <typename S, typename T, int M, int VR>
__global__ __launch_bounds__(256) void mm_p1_mfma_kernel(int64_t ntiles,
                                                         const int32_t* __restrict__ tile_lo,
                                                         const int64_t* __restrict__ meta,
                                                         int ms, int R,
                                                         const S* __restrict__ pool,
                                                         const T* __restrict__ vec,
                                                         T* __restrict__ partial, int64_t pbase) {
    typedef MfmaOp<T> Op;
    typedef MfUnit<S, VR> Un;
    constexpr int KS = 4 * VR;                       // rows per K-step
    constexpr int PB = 8;                            // K-steps in flight
    constexpr int SROWS = 256;                       // rows of X staged in LDS
    constexpr int XT = SROWS + 16 / (int)sizeof(T);  // padded: 8 lanes' reads on distinct banks
    __shared__ __align__(16) T sx[M * XT];
    const int nw = (int)(blockDim.x >> 6);
    const int wv = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int li = lane & 15, lk = lane >> 4;
    const int lj = li < M ? li : 0;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t c0 = meta[ms * t + 1];
        const int nc = (int)(meta[ms * (t + 1) + 1] - c0);
        if (nc <= 0) continue;
        const int32_t r0 = tile_lo[t];
        const int mt = tile_lo[t + 1] - r0;
        const int ld = mm_ld(mt, R);
        const int kr = (ld + KS - 1) / KS * KS;  // rows padded to whole K-steps
        const S* __restrict__ base = pool + meta[ms * t + 2];
        const bool staged = kr <= SROWS;
        if (staged) {
            for (int i = (int)threadIdx.x; i < kr * M; i += (int)blockDim.x) {
                const int row = i / M, j = i % M;
                sx[j * XT + row] = row < mt ? vec[(int64_t)(r0 + row) * M + j] : (T)0;
            }
            __syncthreads();
        }
        for (int cb = wv * 16; cb < nc; cb += nw * 16) {
            // columns past nc repeat the last one; their sums are not stored
            const S* __restrict__ cp = base + (int64_t)min(cb + li, nc - 1) * ld;
            typename Op::Acc acc;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] = 0;
            for (int k0 = 0; k0 < kr; k0 += KS * PB) {
                typename Un::Raw raw[PB];
#pragma unroll
                for (int b = 0; b < PB; ++b) {
                    const int r = k0 + KS * b + VR * lk;
                    raw[b] = __builtin_nontemporal_load(
                        (const typename Un::Raw*)(cp + (r < ld ? r : ld - VR)));
                }
                __builtin_amdgcn_sched_barrier(0);  // every load in flight before the first use
#pragma unroll
                for (int b = 0; b < PB; ++b) {
                    const int r = k0 + KS * b + VR * lk;
                    T a[VR], xb[VR];
                    Un::get(raw[b], a);
                    if (staged) {
                        const T* xp = sx + lj * XT + (r < kr ? r : 0);
#pragma unroll
                        for (int e = 0; e < VR; ++e) xb[e] = (r < kr && li < M) ? xp[e] : (T)0;
                    } else {
#pragma unroll
                        for (int e = 0; e < VR; ++e)
                            xb[e] = (r + e < mt && li < M)
                                        ? vec[(int64_t)(r0 + (r + e < mt ? r + e : 0)) * M + lj]
                                        : (T)0;
                    }
#pragma unroll
                    for (int e = 0; e < VR; ++e) acc = Op::mac(a[e], xb[e], acc);
                }
            }
            if (li < M) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = cb + Op::drow(lk, v);
                    if (c < nc) partial[(pbase + c0 + c) * M + li] = acc[v];
                }
            }
        }
        if (staged) __syncthreads();  // sx is refilled by the next tile
    }
}

#define HMX_MM_SWITCH(M, CALL) \
    switch (M) {               \
        case 1: CALL(1); break; \
        case 2: CALL(2); break; \
        case 4: CALL(4); break; \
        case 8: CALL(8); break; \
        case 16: CALL(16); break; \
        default: return hipErrorInvalidValue; \
    }

template <typename S, typename T>
hipError_t mm_p1_dispatch(int M, int64_t ntiles, const int32_t* tile_lo, const int64_t* meta,
                          int ms, int R, const void* pool, const void* vec, void* partial,
                          int64_t pbase, hipStream_t st) {
    const unsigned g = (unsigned)std::min<int64_t>(ntiles, 1 << 20);
#define HMX_P1(MM)                                                                             \
    hipLaunchKernelGGL((mm_p1_kernel<S, T, MM>), dim3(g), dim3(256), 0, st, ntiles, tile_lo, \
                       meta, ms, R, (const S*)pool, (const T*)vec, (T*)partial, pbase)
    HMX_MM_SWITCH(M, HMX_P1)
#undef HMX_P1
    return hipGetLastError();
}

}  // namespace

hipError_t launch_mm_gather(const void* X, int64_t ldx, const int32_t* perm, int64_t ncols,
                            int64_t col0, void* vec, int M, int mr, int f64, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    if (mr < 1 || mr > M) return hipErrorInvalidValue;
    const unsigned g = mm_grid(ncols * M);
#define HMX_G(MM)                                                                               \
    if (f64)                                                                                    \
        hipLaunchKernelGGL((mm_gather_kernel<double, MM>), dim3(g), dim3(256), 0, st,          \
                           (const double*)X, ldx, perm, ncols, col0, mr, (double*)vec);        \
    else                                                                                        \
        hipLaunchKernelGGL((mm_gather_kernel<float, MM>), dim3(g), dim3(256), 0, st,           \
                           (const float*)X, ldx, perm, ncols, col0, mr, (float*)vec)
    HMX_MM_SWITCH(M, HMX_G)
#undef HMX_G
    return hipGetLastError();
}

hipError_t launch_mm_p1(int M, int64_t ntiles, const int32_t* tile_lo, const int64_t* meta,
                        int ms, int R, const void* pool, const void* vec, void* partial,
                        int64_t pbase, int smode, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    if (M == 8 || M == 16) {
        // matrix cores; R (entries per 16 bytes) is a multiple of the load's rows
        const unsigned g = (unsigned)std::min<int64_t>(ntiles, 1 << 20);
#define HMX_P1M(S, T, VR)                                                                       \
    if (M == 8)                                                                                 \
        hipLaunchKernelGGL((mm_p1_mfma_kernel<S, T, 8, VR>), dim3(g), dim3(256), 0, st, ntiles,  \
                           tile_lo, meta, ms, R, (const S*)pool, (const T*)vec, (T*)partial,     \
                           pbase);                                                              \
    else                                                                                        \
        hipLaunchKernelGGL((mm_p1_mfma_kernel<S, T, 16, VR>), dim3(g), dim3(256), 0, st, ntiles, \
                           tile_lo, meta, ms, R, (const S*)pool, (const T*)vec, (T*)partial,     \
                           pbase)
        if (smode == 0) {
            if (R % 2) return hipErrorInvalidValue;
            HMX_P1M(double, double, 2);
        } else if (smode == 1) {
            if (R % 4) return hipErrorInvalidValue;
            HMX_P1M(float, float, 4);
        } else {
            if (R % 8) return hipErrorInvalidValue;
            HMX_P1M(uint16_t, float, 8);
        }
#undef HMX_P1M
        return hipGetLastError();
    }
    if (smode == 0)
        return mm_p1_dispatch<double, double>(M, ntiles, tile_lo, meta, ms, R, pool, vec, partial,
                                              pbase, st);
    if (smode == 1)
        return mm_p1_dispatch<float, float>(M, ntiles, tile_lo, meta, ms, R, pool, vec, partial,
                                            pbase, st);
    return mm_p1_dispatch<uint16_t, float>(M, ntiles, tile_lo, meta, ms, R, pool, vec, partial,
                                           pbase, st);
}

hipError_t launch_mm_p1_reduce(int M, const int4* rec, int64_t ncols, const int64_t* pfc,
                               const void* partial, void* vec, int64_t n, int f64,
                               hipStream_t st) {
    if (ncols == 0) return hipSuccess;
    const unsigned g = mm_grid(ncols);
#define HMX_R(MM)                                                                               \
    if (f64)                                                                                    \
        hipLaunchKernelGGL((mm_p1_reduce_kernel<double, MM>), dim3(g), dim3(256), 0, st, rec,  \
                           ncols, pfc, (const double*)partial, (double*)vec, n);               \
    else                                                                                        \
        hipLaunchKernelGGL((mm_p1_reduce_kernel<float, MM>), dim3(g), dim3(256), 0, st, rec,   \
                           ncols, pfc, (const float*)partial, (float*)vec, n)
    HMX_MM_SWITCH(M, HMX_R)
#undef HMX_R
    return hipGetLastError();
}

#ifndef HMX_MM_PB
#define HMX_MM_PB 16
#endif
#ifndef HMX_MM_BF16_VR
#define HMX_MM_BF16_VR 8
#endif

hipError_t launch_mm_rowtile(int M, int64_t ntiles, const int32_t* tile_lo, const int64_t* meta,
                             const int64_t* widx, const void* upool, const void* npool,
                             const void* vec, const int32_t* perm, double alpha, double beta,
                             double sigma2, void* Z, int64_t ldz, int R, int max_tile,
                             int fmode, int nmode, const void* soa, int64_t n, int d,
                             KernelFn kern, int mr, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    if (mr < 1 || mr > M) return hipErrorInvalidValue;
    if ((M == 8 || M == 16) && nmode != 3) {
        // matrix cores: a wave per slab of 16 VR rows, up to four slabs per workgroup
        const int vr = fmode == 0 ? 2 : (fmode == 2 && nmode == 2 ? HMX_MM_BF16_VR : 4);
        if (R % vr) return hipErrorInvalidValue;
        const int ldmax = mm_ld(max_tile, R), rs = 16 * vr;
        const int nw = std::max(1, std::min(4, (ldmax + rs - 1) / rs));
        const int passes = (ldmax + nw * rs - 1) / (nw * rs);
        const dim3 grid((unsigned)std::min<int64_t>(ntiles * passes, 1 << 20));
#define HMX_RTM(SU, SN, T, VR)                                                                   \
    if (M == 8)                                                                                  \
        hipLaunchKernelGGL((mm_rowtile_mfma_kernel<SU, SN, T, 8, VR, HMX_MM_PB>), grid, dim3(64 * nw), 0, st, \
                           ntiles, tile_lo, meta, widx, (const SU*)upool, (const SN*)npool,      \
                           (const T*)vec, perm, (T)alpha, (T)beta, (T)sigma2, (T*)Z, ldz, R, mr, \
                           passes);                                                              \
    else                                                                                         \
        hipLaunchKernelGGL((mm_rowtile_mfma_kernel<SU, SN, T, 16, VR, HMX_MM_PB>), grid, dim3(64 * nw), 0,   \
                           st, ntiles, tile_lo, meta, widx, (const SU*)upool, (const SN*)npool,  \
                           (const T*)vec, perm, (T)alpha, (T)beta, (T)sigma2, (T*)Z, ldz, R, mr, \
                           passes)
        if (fmode == 0 && nmode == 0) {
            HMX_RTM(double, double, double, 2);
        } else if (fmode == 1 && nmode == 1) {
            HMX_RTM(float, float, float, 4);
        } else if (fmode == 2 && nmode == 2) {
            HMX_RTM(uint16_t, uint16_t, float, HMX_MM_BF16_VR);
        } else if (fmode == 2 && nmode == 1) {
            HMX_RTM(uint16_t, float, float, 4);
        } else {
            return hipErrorInvalidValue;
        }
#undef HMX_RTM
        return hipGetLastError();
    }
    if (mr != M) return hipErrorInvalidValue;  // the vector-unit forms take whole groups
    const int vr = fmode == 0 ? 2 : 4;
    const unsigned passes = (unsigned)((mm_ld(max_tile, R) + 64 * vr - 1) / (64 * vr));
    const dim3 grid((unsigned)std::min<int64_t>(ntiles, 1 << 20), passes);
#define HMX_RT(SU, SN, T, NR, MM)                                                               \
    hipLaunchKernelGGL((mm_rowtile_kernel<SU, SN, T, MM, NR>), grid, dim3(64), 0, st, ntiles,  \
                       tile_lo, meta, widx, (const SU*)upool, (const SN*)npool, (const T*)vec,  \
                       perm, (T)alpha, (T)beta, (T)sigma2, (T*)Z, ldz, R, (const T*)soa, n, d,  \
                       KernelEval<T>(kern))
#define HMX_RT_D(MM) HMX_RT(double, double, double, false, MM)
#define HMX_RT_F(MM) HMX_RT(float, float, float, false, MM)
#define HMX_RT_B(MM) HMX_RT(uint16_t, uint16_t, float, false, MM)
#define HMX_RT_BF(MM) HMX_RT(uint16_t, float, float, false, MM)
#define HMX_RT_DR(MM) HMX_RT(double, double, double, true, MM)
#define HMX_RT_FR(MM) HMX_RT(float, float, float, true, MM)
#define HMX_RT_BR(MM) HMX_RT(uint16_t, float, float, true, MM)
    if (fmode == 0 && nmode == 0) {
        HMX_MM_SWITCH(M, HMX_RT_D)
    } else if (fmode == 1 && nmode == 1) {
        HMX_MM_SWITCH(M, HMX_RT_F)
    } else if (fmode == 2 && nmode == 2) {
        HMX_MM_SWITCH(M, HMX_RT_B)
    } else if (fmode == 2 && nmode == 1) {
        HMX_MM_SWITCH(M, HMX_RT_BF)
    } else if (fmode == 0 && nmode == 3) {
        HMX_MM_SWITCH(M, HMX_RT_DR)
    } else if (fmode == 1 && nmode == 3) {
        HMX_MM_SWITCH(M, HMX_RT_FR)
    } else if (fmode == 2 && nmode == 3) {
        HMX_MM_SWITCH(M, HMX_RT_BR)
    } else {
        return hipErrorInvalidValue;
    }
#undef HMX_RT_D
#undef HMX_RT_F
#undef HMX_RT_B
#undef HMX_RT_BF
#undef HMX_RT_DR
#undef HMX_RT_FR
#undef HMX_RT_BR
#undef HMX_RT
    return hipGetLastError();
}

}  // namespace hmx
