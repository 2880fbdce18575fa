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
//   * phase 1:   T_b = V_b^T X|sigma_b by row tiles: one workgroup of four
//                waves per tile, the tile's X rows staged in LDS, groups of 8
//                lanes taking two source columns at a time (eight row vectors
//                per lane in flight), each lane summing its rows for all M
//                sides, then a butterfly over the 8 lanes; partials per
//                (column, tile);
//   * reduce:    the partials of each t entry summed over its tiles in tile
//                order (as for one vector);
//   * row tiles: one wave per (tile, pass of 64 x VR rows): each lane owns VR
//                consecutive rows and accumulates VR x M sums; the column
//                weights (M per column) are staged in LDS 128 columns at a
//                time; near-field columns are read from the pool or
//                evaluated from the coordinates.
// All sums run in a fixed order, so the product is deterministic; column c
// of the result sums the same terms as the single-vector product of X's
// column c, in another order (per lane instead of per lane group).
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

template <typename T, int M>
__global__ void mm_gather_kernel(const T* __restrict__ X, int64_t ldx,
                                 const int32_t* __restrict__ perm, int64_t ncols, int64_t col0,
                                 T* __restrict__ vec) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ncols * M;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / M;
        const int c = (int)(e % M);
        vec[(col0 + i) * M + c] = X[(perm[col0 + i] - col0) + c * ldx];
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
                            int64_t col0, void* vec, int M, int f64, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    const unsigned g = mm_grid(ncols * M);
#define HMX_G(MM)                                                                               \
    if (f64)                                                                                    \
        hipLaunchKernelGGL((mm_gather_kernel<double, MM>), dim3(g), dim3(256), 0, st,          \
                           (const double*)X, ldx, perm, ncols, col0, (double*)vec);            \
    else                                                                                        \
        hipLaunchKernelGGL((mm_gather_kernel<float, MM>), dim3(g), dim3(256), 0, st,           \
                           (const float*)X, ldx, perm, ncols, col0, (float*)vec)
    HMX_MM_SWITCH(M, HMX_G)
#undef HMX_G
    return hipGetLastError();
}

hipError_t launch_mm_p1(int M, int64_t ntiles, const int32_t* tile_lo, const int64_t* meta,
                        int ms, int R, const void* pool, const void* vec, void* partial,
                        int64_t pbase, int smode, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
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

hipError_t launch_mm_rowtile(int M, int64_t ntiles, const int32_t* tile_lo, const int64_t* meta,
                             const int64_t* widx, const void* upool, const void* npool,
                             const void* vec, const int32_t* perm, double alpha, double beta,
                             double sigma2, void* Z, int64_t ldz, int R, int max_tile,
                             int fmode, int nmode, const void* soa, int64_t n, int d,
                             KernelFn kern, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
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
