// Batched adaptive cross approximation (Algorithm 2, Section 5.4.1).
//
// One workgroup per admissible block, each running its own rank loop, so
// blocks stop independently (no global "voting" bounded by the slowest
// block).  Blocks of the upper tree levels (many rows) get 512-thread
// workgroups, those of the lowest levels (at most 512 rows) one wave, the rest
// 256 threads (the very largest run on many workgroups each, k_aca_split.hip);
// every chunk of blocks handed to the ACA is level-sorted (the canonical leaf
// order is level order; a list cut into several chunks is first reordered so
// that each chunk holds a share of every level), so each class is a contiguous
// range of a chunk and the classes of a chunk run concurrently.  Per step r:
//   1. residual column  u^ = A[:, j] - sum_{l<r} u_l (v_l)_j   (rows over threads)
//   2. row pivot        i  = argmax over unused rows |u^_i| (lowest index on ties)
//      a column whose largest residual entry is <= eps0 times the column's own
//      largest |entry| adds no rank (zero or rounding-noise residual); the
//      lowest unused column is tried next, and kmax such columns end the block
//   3. u_r = u^ / u^_i,  v_r = A[i, :]^T - sum_{l<r} (u_l)_i v_l  (cols over threads)
//   4. |S_r|_F^2 += 2 sum_{l<r} (u_r.u_l)(v_r.v_l) + |u_r|^2 |v_r|^2   in FP64
//   5. stop if |u_r| |v_r| <= eps (1 - aca_eta) / (1 + eps) |S_r|_F
//   6. next column pivot j = argmax over unused columns |(v_r)_j|
// The inner products of step 4 are FP64.  With the test applied every step,
// term r's products with the earlier terms are gathered during the residual
// passes of step r + 1, which read those columns anyway (term r + 1 is then
// speculative and dropped if term r's test passes); otherwise the whole
// workgroup computes them after the row, eight previous columns per pass.
// Every pass issues the loads of several previous columns before using them.
// Learned rank sizing gives every block a predicted target: storage for that
// many columns with the test in 5 applied every step (sizing form), or
// exactly that many steps with the test applied to the last term only
// (one-shot form).  A block that reaches its target unfinished continues
// adaptively (the fallback), or, when its storage holds only the target,
// reports rank -1 to be approximated again with k_max columns.
// The first column is the sigma point nearest (FP64, no contraction) to the
// centre of tau's bounding box, so the first cross runs through the block's
// largest entries.
// Used rows/columns are bitmasks in LDS.  U (m x cap) and V (n x cap) are
// column-major in a capacity pool; column r of U doubles as the scratch for
// the residual column.  All reductions have a fixed tree, so the result is
// bit-reproducible from run to run.
#include <climits>

#include "hmx_internal.h"

namespace hmx {

namespace {

constexpr int kDotCols = 8;     // previous columns per inner-product pass
constexpr int kRows = 4;        // rows per thread per residual pass
constexpr int kLU = 8;          // previous columns whose loads are in flight together
constexpr int kBigThreads = 512;  // workgroup size of the upper-level class

template <int NT>
constexpr int dot_cols() {
    return kDotCols;
}

template <typename T>
struct Arg {
    T best;  // |value|; -1 = none
    int idx;
    T val;   // signed value
};

template <typename T>
__device__ __forceinline__ void arg_combine(Arg<T>& a, const Arg<T>& b) {
    if (b.best > a.best || (b.best == a.best && b.idx < a.idx)) a = b;
}

template <typename T>
__device__ __forceinline__ Arg<T> wave_argmax(Arg<T> a) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        Arg<T> b;
        b.best = __shfl_xor(a.best, o, 64);
        b.idx = __shfl_xor(a.idx, o, 64);
        b.val = __shfl_xor(a.val, o, 64);
        arg_combine(a, b);
    }
    return a;
}

// ---------------------------------------------------------------------------
// Wave reductions on the DPP crossbar: the quad swaps (lane i with i ^ 1, then
// i ^ 2), the half-row mirror (i with 7 - i) and the row mirror (i with
// 15 - i) leave every lane of a row of 16 holding the row's total; the four
// rows are then combined from scalar reads.  The result is the same on every
// lane and needs no permute indices or LDS traffic.
constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
    return dpp_i<CTRL>(v);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)dpp_i<CTRL>((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)dpp_i<CTRL>((int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int lane_read(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float lane_read(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_read(double v, int l) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// sum over the wave, (row 0 + row 1) + (row 2 + row 3)
__device__ __forceinline__ double wave_total(double v) {
    v += dpp<kDppXor1>(v);
    v += dpp<kDppXor2>(v);
    v += dpp<kDppHalfMirror>(v);
    v += dpp<kDppMirror>(v);
    return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}

__device__ __forceinline__ double wave_max(double v) {
    double u = dpp<kDppXor1>(v);
    v = u > v ? u : v;
    u = dpp<kDppXor2>(v);
    v = u > v ? u : v;
    u = dpp<kDppHalfMirror>(v);
    v = u > v ? u : v;
    u = dpp<kDppMirror>(v);
    v = u > v ? u : v;
    double r = lane_read(v, 0);
#pragma unroll
    for (int q = 16; q < 64; q += 16) {
        const double t = lane_read(v, q);
        r = t > r ? t : r;
    }
    return r;
}

template <typename T, int CTRL>
__device__ __forceinline__ Arg<T> dpp_arg(const Arg<T>& a) {
    return Arg<T>{dpp<CTRL>(a.best), dpp<CTRL>(a.idx), dpp<CTRL>(a.val)};
}

// the largest |value| of the wave, lowest index on ties (the same element
// whatever the order of combination)
template <typename T>
__device__ __forceinline__ Arg<T> wave_argmax_u(Arg<T> a) {
    arg_combine(a, dpp_arg<T, kDppXor1>(a));
    arg_combine(a, dpp_arg<T, kDppXor2>(a));
    arg_combine(a, dpp_arg<T, kDppHalfMirror>(a));
    arg_combine(a, dpp_arg<T, kDppMirror>(a));
    Arg<T> r{lane_read(a.best, 0), lane_read(a.idx, 0), lane_read(a.val, 0)};
#pragma unroll
    for (int q = 16; q < 64; q += 16)
        arg_combine(r, Arg<T>{lane_read(a.best, q), lane_read(a.idx, q), lane_read(a.val, q)});
    return r;
}

template <typename T, int NW>
struct AcaShared {
    T vec[kMaxRankCap];         // broadcast row of V (step 1) / row of U (step 3)
    double gu[kMaxRankCap];     // u_r . u_l
    double gv[kMaxRankCap];     // v_r . v_l
    double part[NW][kDotCols];  // per-wave partial inner products
    T abest[NW];
    T aval[NW];
    int aidx[NW];
    double dsum[2][NW];
    int imin[NW];
    double dkey[NW];
    int dkidx[NW];
    long long ovf;  // overflow offset granted to the block, or -1
    long long uo, vo;  // the block's current storage offsets (moved by an overflow)
};

// overflow storage of the learned sizing pass (see AcaArgs)
struct Overflow {
    unsigned long long* used;
    int64_t cap, u0, v0;
    int64_t* moved;  // per block of the launch: the offset granted, else left as is
};

template <typename T, int NW>
__device__ Arg<T> block_argmax(Arg<T> a, AcaShared<T, NW>& sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    a = wave_argmax(a);
    if (lane == 0) {
        sh.abest[w] = a.best;
        sh.aidx[w] = a.idx;
        sh.aval[w] = a.val;
    }
    __syncthreads();
    Arg<T> r{sh.abest[0], sh.aidx[0], sh.aval[0]};
    for (int q = 1; q < NW; ++q) {
        Arg<T> b{sh.abest[q], sh.aidx[q], sh.aval[q]};
        arg_combine(r, b);
    }
    __syncthreads();
    return r;
}

// sum of a double across the workgroup, same tree on every thread
template <typename T, int NW>
__device__ double block_sum(double a, AcaShared<T, NW>& sh, int slot) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    a = wave_sum(a);
    if (lane == 0) sh.dsum[slot][w] = a;
    __syncthreads();
    double s = sh.dsum[slot][0];
    for (int q = 1; q < NW; ++q) s += sh.dsum[slot][q];
    __syncthreads();
    return s;
}

template <typename T, int NW>
__device__ int block_min_int(int v, AcaShared<T, NW>& sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        int u = __shfl_xor(v, o, 64);
        v = u < v ? u : v;
    }
    if (lane == 0) sh.imin[w] = v;
    __syncthreads();
    int r = sh.imin[0];
    for (int q = 1; q < NW; ++q) r = sh.imin[q] < r ? sh.imin[q] : r;
    __syncthreads();
    return r;
}

// min (op = 0) or max (op = 1) of a double across the workgroup
template <typename T, int NW>
__device__ double block_minmax(double v, int op, AcaShared<T, NW>& sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double u = __shfl_xor(v, o, 64);
        v = op ? (u > v ? u : v) : (u < v ? u : v);
    }
    if (lane == 0) sh.dkey[w] = v;
    __syncthreads();
    double r = sh.dkey[0];
    for (int q = 1; q < NW; ++q) r = op ? (sh.dkey[q] > r ? sh.dkey[q] : r)
                                        : (sh.dkey[q] < r ? sh.dkey[q] : r);
    __syncthreads();
    return r;
}

// index of the smallest key (lowest index on ties)
template <typename T, int NW>
__device__ int block_argmin_f64(double key, int idx, AcaShared<T, NW>& sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double k2 = __shfl_xor(key, o, 64);
        const int i2 = __shfl_xor(idx, o, 64);
        if (k2 < key || (k2 == key && i2 < idx)) {
            key = k2;
            idx = i2;
        }
    }
    if (lane == 0) {
        sh.dkey[w] = key;
        sh.dkidx[w] = idx;
    }
    __syncthreads();
    double bk = sh.dkey[0];
    int bi = sh.dkidx[0];
    for (int q = 1; q < NW; ++q)
        if (sh.dkey[q] < bk || (sh.dkey[q] == bk && sh.dkidx[q] < bi)) {
            bk = sh.dkey[q];
            bi = sh.dkidx[q];
        }
    __syncthreads();
    return bi;
}

// reduce acc[0..DC) across the workgroup into out[0..nk) (fixed tree)
template <int DC, typename T, int NW>
__device__ void block_sum_cols(double* acc, int nk, double* out, AcaShared<T, NW>& sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < DC; ++k) acc[k] = wave_sum(acc[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < DC; ++k) sh.part[w][k] = acc[k];
    }
    __syncthreads();
    if ((int)threadIdx.x < nk) {
        double s = sh.part[0][threadIdx.x];
        for (int q = 1; q < NW; ++q) s += sh.part[q][threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// first column: the sigma point nearest to the centre 0.5 (a + b) of tau's
// bounding box, squared distance summed in dimension order, all in FP64
// without contraction
template <typename T, int NT>
__device__ int first_column(const double* __restrict__ soa64, int64_t n, int d, int4 bl,
                            AcaShared<T, NT / kWave>& sh) {
    const int m = bl.y - bl.x, nc = bl.w - bl.z;
    double c[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < d; ++k) {
        double mn = INFINITY, mx = -INFINITY;
        for (int i = threadIdx.x; i < m; i += NT) {
            const double v = soa64[(int64_t)k * n + bl.x + i];
            mn = v < mn ? v : mn;
            mx = v > mx ? v : mx;
        }
        mn = block_minmax(mn, 0, sh);
        mx = block_minmax(mx, 1, sh);
        c[k] = __dmul_rn(0.5, __dadd_rn(mn, mx));
    }
    double best = INFINITY;
    int bi = INT_MAX;
    for (int q = threadIdx.x; q < nc; q += NT) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) {
            const double t = __dsub_rn(soa64[(int64_t)k * n + bl.z + q], c[k]);
            s = __dadd_rn(s, __dmul_rn(t, t));
        }
        if (s < best) {
            best = s;
            bi = q;
        }
    }
    return block_argmin_f64(best, bi, sh);
}

__device__ __forceinline__ bool bit_get(const uint32_t* m, int i) {
    return (m[i >> 5] >> (i & 31)) & 1u;
}

// products of column p of a column-major matrix X (len rows) with its columns
// l < p into out[0..p), eight columns per pass, FP64, fixed reduction tree
template <typename T, int NT, int DC>
__device__ void column_products(const T* __restrict__ X, int len, int p, double* out,
                                AcaShared<T, NT / kWave>& sh) {
    const T* __restrict__ Xp = X + (int64_t)p * len;
    for (int c0 = 0; c0 < p; c0 += DC) {
        const int nk = p - c0 < DC ? p - c0 : DC;
        const T* __restrict__ Xc = X + (int64_t)c0 * len;
        double acc[DC];
#pragma unroll
        for (int k = 0; k < DC; ++k) acc[k] = 0.0;
        for (int ib = 0; ib < len; ib += kRows * NT) {
#pragma unroll
            for (int e = 0; e < kRows; ++e) {
                const int i = ib + threadIdx.x + e * NT;
                if (i < len) {
                    const double x = (double)Xp[i];
#pragma unroll
                    for (int k = 0; k < DC; ++k)
                        if (k < nk) acc[k] += x * (double)Xc[k * len + i];
                }
            }
        }
        block_sum_cols<DC>(acc, nk, out + c0, sh);
    }
}

// Rows i0 + k NT (k < kRows) of a pass: indices clamped into [0, len) so that
// every load is issued unconditionally (the loads of a batch then overlap
// instead of each waiting behind the branch of its own bounds test).
template <int NT>
__device__ __forceinline__ void clamp_rows(int i0, int len, int (&ic)[kRows], bool (&ok)[kRows]) {
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int i = i0 + k * NT;
        ok[k] = i < len;
        ic[k] = ok[k] ? i : len - 1;
    }
}

// element at a 32-bit byte offset from a wave-uniform base
template <typename T>
__device__ __forceinline__ T ld_at(const T* __restrict__ base, uint32_t byte_off) {
    return *(const T*)((const char*)base + byte_off);
}

// Loads through a raw buffer descriptor on a wave-uniform base: the per-lane
// part of the address is one 32-bit offset shared by all columns of a pass,
// the column offset a scalar.  Every index is clamped into its array before
// the load, so the descriptor's range check never applies (its size is the
// largest the field holds).
constexpr int kBufWord3 = 0x00020000;  // 32-bit data format, the raw-buffer form on CDNA

template <typename T>
struct BufView {
    __amdgpu_buffer_rsrc_t rs;
    __device__ __forceinline__ explicit BufView(const T* base)
        : rs(__builtin_amdgcn_make_buffer_rsrc((void*)base, 0, 0x7fffffff, kBufWord3)) {}
    __device__ __forceinline__ T at(uint32_t voff, uint32_t soff) const;
};

template <>
__device__ __forceinline__ float BufView<float>::at(uint32_t voff, uint32_t soff) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, (int)soff, 0));
}

template <>
__device__ __forceinline__ double BufView<double>::at(uint32_t voff, uint32_t soff) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0));
}

// coordinates of point first + row (row's byte offset boff) of a d x n SoA array
template <typename T>
__device__ __forceinline__ void load_pt_buf(const BufView<T>& pts, int64_t n, int d, uint32_t boff,
                                            T* p) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
        p[k] = (k < d) ? pts.at(boff, (uint32_t)((int64_t)k * n * (int64_t)sizeof(T))) : (T)0;
}

// a[k] -= X_l[row k] c_l for l = 0, 1, ..., r - 1 in that order (columns of
// the column-major X, leading dimension ld; coefficients c in LDS), kLU
// columns' loads in flight at once; padding columns beyond r weigh zero.
// With pend, also the products of column p's rows xp[k] (zero on rows outside
// the block) with every column l < p, per column a wave sum added to acc[l]
// (lane 0): the deferred inner products of the open term.
template <typename T>
__device__ __forceinline__ void subtract_columns(const T* __restrict__ X, int64_t ld, int r,
                                                 const T* coef, const int (&ic)[kRows],
                                                 T (&a)[kRows], bool pend, int p,
                                                 const T (&xp)[kRows], double* acc, int lane) {
    // r and p are the same on every lane; saying so keeps the column bases scalar
    r = __builtin_amdgcn_readfirstlane(r);
    p = __builtin_amdgcn_readfirstlane(p);
    uint32_t off[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) off[k] = (uint32_t)ic[k] * (uint32_t)sizeof(T);
    for (int l0 = 0; l0 < r; l0 += kLU) {
        const BufView<T> cols(X + (int64_t)l0 * ld);
        T c[kLU], val[kLU][kRows];
#pragma unroll
        for (int q = 0; q < kLU; ++q) {
            const bool in = l0 + q < r;
            const int l = in ? l0 + q : r - 1;
            c[q] = in ? coef[l] : (T)0;
            const uint32_t soff = (uint32_t)((int64_t)(l - l0) * ld * (int64_t)sizeof(T));
#pragma unroll
            for (int k = 0; k < kRows; ++k) val[q][k] = cols.at(off[k], soff);
        }
#pragma unroll
        for (int q = 0; q < kLU; ++q)
#pragma unroll
            for (int k = 0; k < kRows; ++k) a[k] -= val[q][k] * c[q];
        if (pend) {
#pragma unroll
            for (int q = 0; q < kLU; ++q) {
                if (l0 + q < p) {
                    double sum = 0.0;
#pragma unroll
                    for (int k = 0; k < kRows; ++k) sum += (double)xp[k] * (double)val[q][k];
                    sum = wave_total(sum);
                    if (lane == 0) acc[l0 + q] += sum;
                }
            }
        }
    }
}

// the same products in the order of the deferred accumulation of the step
// loop (per batch of kRows rows per thread and per column: a wave sum, added
// to the wave's row of acc; the waves' rows are summed in order by the caller),
// so that a test taken on them decides as the deferred one would
template <typename T, int NT>
__device__ void column_products_waved(const T* __restrict__ X, int len, int p,
                                      double (*acc)[kMaxRankCap]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    p = __builtin_amdgcn_readfirstlane(p);
    for (int l = lane; l < p; l += kWave) acc[w][l] = 0.0;
    __syncthreads();
    for (int ib = 0; ib < len; ib += kRows * NT) {
        int ic[kRows];
        bool ok[kRows];
        clamp_rows<NT>(ib + threadIdx.x, len, ic, ok);
        uint32_t off[kRows];
        T xp[kRows];
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            off[k] = (uint32_t)ic[k] * (uint32_t)sizeof(T);
            const T v = ld_at(X + (int64_t)p * len, off[k]);
            xp[k] = ok[k] ? v : (T)0;
        }
        for (int l0 = 0; l0 < p; l0 += kLU) {
            const BufView<T> cols(X + (int64_t)l0 * len);
            T val[kLU][kRows];
#pragma unroll
            for (int q = 0; q < kLU; ++q) {
                const int l = l0 + q < p ? l0 + q : p - 1;
                const uint32_t soff = (uint32_t)((int64_t)(l - l0) * len * (int64_t)sizeof(T));
#pragma unroll
                for (int k = 0; k < kRows; ++k) val[q][k] = cols.at(off[k], soff);
            }
#pragma unroll
            for (int q = 0; q < kLU; ++q) {
                if (l0 + q < p) {
                    double sum = 0.0;
#pragma unroll
                    for (int k = 0; k < kRows; ++k) sum += (double)xp[k] * (double)val[q][k];
                    sum = wave_total(sum);
                    if (lane == 0) acc[w][l0 + q] += sum;
                }
            }
        }
    }
    __syncthreads();
}

// a value known to be the same on every lane, in scalar registers
__device__ __forceinline__ long long uniform_i64(long long v) {
    const unsigned long long u = (unsigned long long)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// A block of the learned sizing pass that reached its target unfinished:
// request R columns of overflow storage (one atomic, by thread 0), copy the
// r columns computed so far and return the offset granted (the same on every
// thread), or -1 when the reserve is exhausted.  Kept out of line: the step
// loop's code stays compact.
template <typename T, int NT>
__device__ __noinline__ long long aca_overflow_move(const Overflow& ovf, int m, int nc, int R, int r,
                                                    const T* __restrict__ U,
                                                    const T* __restrict__ V,
                                                    T* __restrict__ Upool, T* __restrict__ Vpool,
                                                    int64_t ubase, int64_t vbase, long long* slot) {
    if (threadIdx.x == 0) {
        const unsigned long long need = (unsigned long long)(m > nc ? m : nc) * (unsigned long long)R;
        const unsigned long long old = atomicAdd(ovf.used, need);
        *slot = old + need <= (unsigned long long)ovf.cap ? (long long)old : -1;
    }
    __syncthreads();
    const long long off = *slot;
    if (off < 0) return -1;
    T* __restrict__ Un = Upool + (ovf.u0 + off - ubase);
    T* __restrict__ Vn = Vpool + (ovf.v0 + off - vbase);
    for (int e = threadIdx.x; e < r * m; e += NT) Un[e] = U[e];
    for (int e = threadIdx.x; e < r * nc; e += NT) Vn[e] = V[e];
    __syncthreads();
    return off;
}

// waves per SIMD the compiler must leave room for: four for the multi-wave
// classes in FP32 (their latency-bound steps gain from the occupancy more
// than the 112-128 spilled bytes per lane cost: at two waves, without
// spills, the N = 2^20 ACA took 46 ms instead of 38), two in FP64 (whose
// values take twice the registers: at four waves it spilled 480 bytes per
// lane, and the N = 2^20 FP64 ACA took 137 ms instead of 84), the
// register-limited default for the single-wave class (whose blocks are many
// and short)
template <typename T, int NT>
constexpr int aca_min_waves() {
    return NT > kWave ? (sizeof(T) == 8 ? 2 : 4) : 1;
}

template <typename T, int NT>
__global__ __launch_bounds__(NT, (aca_min_waves<T, NT>())) void aca_kernel(
    const T* __restrict__ soa, const double* __restrict__ soa64, int64_t n, int d, KernelEval<T> K,
    const int4* __restrict__ blocks, int64_t nblocks, const int64_t* __restrict__ uoff,
    const int64_t* __restrict__ voff, int64_t ubase, int64_t vbase, int kmax, double eps, double aca_eta, T eps0, int fixed,
    const int32_t* __restrict__ rtarget, int one_shot_mode, int cap_only, Overflow ovf,
    int lds_words, T* __restrict__ Upool, T* __restrict__ Vpool,
    int32_t* __restrict__ rank_out, int32_t* __restrict__ steps_out) {
    constexpr int NW = NT / kWave;
    constexpr int DC = dot_cols<NT>();
    extern __shared__ uint32_t smask[];
    __shared__ AcaShared<T, NW> sh;
    __shared__ double accu[NW][kMaxRankCap];  // deferred products, one row per wave
    __shared__ double accv[NW][kMaxRankCap];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const double tol = eps * (1.0 - aca_eta) / (1.0 + eps);

    for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
        const int4 bl = blocks[b];
        const int m = bl.y - bl.x, nc = bl.w - bl.z;
        int R = kmax;
        R = m < R ? m : R;
        R = nc < R ? nc : R;
        // the block's storage offsets live in LDS and are read at every step
        // (they move once if the block outgrows its target into overflow
        // storage; a loop-carried pointer would cost the loop its hoisting)
        if (tid == 0) {
            sh.uo = uoff[b] - ubase;
            sh.vo = voff[b] - vbase;
        }
        const BufView<T> rows_pts(soa + bl.x), cols_pts(soa + bl.z);
        const int mw = (m + 31) >> 5, nw = (nc + 31) >> 5;
        const bool single = m <= kRows * NT;  // one pass covers every row
        if (mw + nw > lds_words) {  // outside this launch's size class (never by construction)
            if (tid == 0) {
                rank_out[b] = 0;
                if (steps_out) steps_out[b] = 0;
            }
            continue;
        }
        uint32_t* rmask = smask;
        uint32_t* cmask = smask + mw;
        for (int q = tid; q < mw + nw; q += NT) smask[q] = 0u;
        __syncthreads();

        // rtarget[b] > 0 bounds the block's columns to a predicted target.
        // Sizing form (one_shot_mode = 0): the stopping test runs every step
        // as in the adaptive method.  One-shot form: the target is reached
        // without the test, which then judges the last term.  A block that
        // reaches its target unfinished either continues adaptively (storage
        // for k_max columns) or, with cap_only (storage for the target only),
        // ends with rank -1 to be approximated again with k_max columns.
        const bool sized = rtarget && rtarget[b] > 0;
        bool one_shot = sized && one_shot_mode;
        int target = sized ? (rtarget[b] < R ? rtarget[b] : R) : R;
        bool refused = false;
        double last_p = 0.0;  // |u_r|^2 |v_r|^2 of the last term
        // With the test applied every step, term p's products with the
        // earlier terms are gathered while the passes of term p + 1 read
        // those columns anyway; term p's test is taken once they are
        // complete, and term p + 1 is dropped if it passes (it was computed
        // speculatively).  The decisions are those of the step-by-step order.
        const bool fuse = !fixed && !one_shot;
        bool pending = false;     // term r - 1's test is still open
        double nu2p = 0.0, nv2p = 0.0;

        int r = 0, ncols_used = 0, nfailed = 0, steps = 0;
        int j = first_column<T, NT>(soa64, n, d, bl, sh);  // (its barriers publish sh.uo, sh.vo)
        double S2 = 0.0;
        for (;;) {
            if (r >= target) {
                if (r >= R) break;
                if (one_shot) {
                    one_shot = false;
                    if (sqrt(last_p) <= tol * sqrt(S2)) break;
                }
                if (pending) {
                    // no room for a speculative term: term r - 1's products now,
                    // summed in the order of the deferred accumulation
                    column_products_waved<T, NT>(Upool + uniform_i64(sh.uo), m, r - 1, accu);
                    column_products_waved<T, NT>(Vpool + uniform_i64(sh.vo), nc, r - 1, accv);
                    double cross = 0.0;
                    for (int l = 0; l < r - 1; ++l) {
                        double gu = accu[0][l], gv = accv[0][l];
                        for (int q = 1; q < NW; ++q) {
                            gu += accu[q][l];
                            gv += accv[q][l];
                        }
                        cross += gu * gv;
                    }
                    __syncthreads();  // every wave has read the rows before any clears them
                    S2 += 2.0 * cross + nu2p * nv2p;
                    last_p = nu2p * nv2p;
                    pending = false;
                    if (sqrt(last_p) <= tol * sqrt(S2)) break;
                }
                if (cap_only) {
                    // storage for the target only: continue in overflow
                    // storage for R columns if the reserve has room
                    const long long off = uniform_i64(
                        ovf.used ? aca_overflow_move<T, NT>(ovf, m, nc, R, r,
                                                            Upool + uniform_i64(sh.uo),
                                                            Vpool + uniform_i64(sh.vo), Upool,
                                                            Vpool, ubase, vbase, &sh.ovf)
                                 : -1);
                    if (off < 0) {
                        refused = true;
                        break;
                    }
                    if (tid == 0) {
                        sh.uo = ovf.u0 + off - ubase;
                        sh.vo = ovf.v0 + off - vbase;
                        ovf.moved[b] = off;
                    }
                    __syncthreads();
                }
                target = R;
            }
            // columns l < r are only read in a step, column r only written
            T* __restrict__ U = Upool + uniform_i64(sh.uo);
            T* __restrict__ V = Vpool + uniform_i64(sh.vo);
            const T* __restrict__ Uread = U;
            const T* __restrict__ Vread = V;
            const int p = r - 1;  // the open term, when pending
            // ---- step 1: residual column j into U[:, r] ----
            for (int l = tid; l < r; l += NT) sh.vec[l] = V[(int64_t)l * nc + j];
            if (tid == 0) cmask[j >> 5] |= 1u << (j & 31);
            if (pending)
                for (int l = lane; l < p; l += kWave) {
                    accu[w][l] = 0.0;
                    accv[w][l] = 0.0;
                }
            __syncthreads();
            ++ncols_used;
            ++steps;
            T yj[3];
            load_pt(soa, n, d, (int64_t)bl.z + j, yj);
            Arg<T> am{(T)-1, INT_MAX, (T)0};
            double colmax = 0.0;
            T keep[kRows];  // the residual column itself when the block has one pass of rows
            // kRows rows per thread per pass; the trip count is the same for
            // every thread of the workgroup
            for (int ib = 0; ib < m; ib += kRows * NT) {
                int ic[kRows];
                bool ok[kRows];
                clamp_rows<NT>(ib + tid, m, ic, ok);
                T xi[kRows][3], a[kRows], up[kRows];
#pragma unroll
                for (int k = 0; k < kRows; ++k) {
                    const uint32_t off = (uint32_t)ic[k] * (uint32_t)sizeof(T);
                    load_pt_buf(rows_pts, n, d, off, xi[k]);
                    up[k] = (T)0;
                    if (pending) {
                        const T v = ld_at(Uread + (int64_t)p * m, off);
                        up[k] = ok[k] ? v : (T)0;
                    }
                }
#pragma unroll
                for (int k = 0; k < kRows; ++k) {
                    a[k] = ok[k] ? phi(K, xi[k], yj, d) : (T)0;
                    const double aa0 = a[k] < (T)0 ? -(double)a[k] : (double)a[k];
                    colmax = aa0 > colmax ? aa0 : colmax;
                }
                subtract_columns(Uread, m, r, sh.vec, ic, a, pending, p, up, accu[w], lane);
#pragma unroll
                for (int k = 0; k < kRows; ++k) {
                    keep[k] = a[k];
                    if (ok[k]) {
                        const int i = ic[k];
                        if (!single) U[(int64_t)r * m + i] = a[k];
                        const T aa = a[k] < (T)0 ? -a[k] : a[k];
                        if (!bit_get(rmask, i) && aa > am.best) {
                            am.best = aa;
                            am.idx = i;
                            am.val = a[k];
                        }
                    }
                }
            }
            // row pivot and the column's largest |entry| in one reduction
            am = wave_argmax_u(am);
            colmax = wave_max(colmax);
            if constexpr (NW > 1) {
                if (lane == 0) {
                    sh.abest[w] = am.best;
                    sh.aidx[w] = am.idx;
                    sh.aval[w] = am.val;
                    sh.dkey[w] = colmax;
                }
                __syncthreads();
                am = Arg<T>{sh.abest[0], sh.aidx[0], sh.aval[0]};
                colmax = sh.dkey[0];
                for (int q = 1; q < NW; ++q) {
                    arg_combine(am, Arg<T>{sh.abest[q], sh.aidx[q], sh.aval[q]});
                    colmax = sh.dkey[q] > colmax ? sh.dkey[q] : colmax;
                }
                __syncthreads();
            }
            if (am.idx == INT_MAX || (double)am.best <= (double)eps0 * colmax) {
                // no usable pivot in this column: try the lowest unused column
                ++nfailed;
                if (ncols_used >= nc || nfailed >= kmax) break;
                int cand = INT_MAX;
                for (int q = tid; q < nw; q += NT) {
                    const uint32_t word = cmask[q];
                    if (word != 0xffffffffu) {
                        const int c = (q << 5) + __ffs(~word) - 1;
                        if (c < nc && c < cand) cand = c;
                    }
                }
                cand = block_min_int(cand, sh);
                if (cand == INT_MAX) break;
                j = cand;
                continue;
            }
            const int ip = am.idx;
            const T piv = am.val;
            // ---- step 3a: u_r = u^ / pivot; |u_r|^2 is reduced with the row's sums ----
            double nu2 = 0.0;
            T* __restrict__ Ur = U + (int64_t)r * m;
            if (single) {
                int ic[kRows];
                bool ok[kRows];
                clamp_rows<NT>(tid, m, ic, ok);
#pragma unroll
                for (int k = 0; k < kRows; ++k) {
                    if (ok[k]) {
                        const T u = keep[k] / piv;
                        Ur[ic[k]] = u;
                        nu2 += (double)u * (double)u;
                    }
                }
            } else {
                for (int ib = 0; ib < m; ib += kRows * NT) {
                    int ic[kRows];
                    bool ok[kRows];
                    clamp_rows<NT>(ib + tid, m, ic, ok);
                    T u[kRows];
#pragma unroll
                    for (int k = 0; k < kRows; ++k)
                        u[k] = ld_at(Ur, (uint32_t)ic[k] * (uint32_t)sizeof(T));
#pragma unroll
                    for (int k = 0; k < kRows; ++k) {
                        if (ok[k]) {
                            u[k] = u[k] / piv;
                            Ur[ic[k]] = u[k];
                            nu2 += (double)u[k] * (double)u[k];
                        }
                    }
                }
            }
            if (!fuse && !fixed) column_products<T, NT, DC>(Uread, m, r, sh.gu, sh);
            for (int l = tid; l < r; l += NT) sh.vec[l] = U[(int64_t)l * m + ip];
            if (tid == 0) rmask[ip >> 5] |= 1u << (ip & 31);
            __syncthreads();
            // ---- step 3b: residual row i_r into V[:, r] ----
            T xp[3];
            load_pt(soa, n, d, (int64_t)bl.x + ip, xp);
            double nv2 = 0.0;
            Arg<T> cm{(T)-1, INT_MAX, (T)0};
            for (int qb = 0; qb < nc; qb += kRows * NT) {
                int ic[kRows];
                bool ok[kRows];
                clamp_rows<NT>(qb + tid, nc, ic, ok);
                T yq[kRows][3], a[kRows], vp[kRows];
#pragma unroll
                for (int k = 0; k < kRows; ++k) {
                    const uint32_t off = (uint32_t)ic[k] * (uint32_t)sizeof(T);
                    load_pt_buf(cols_pts, n, d, off, yq[k]);
                    vp[k] = (T)0;
                    if (pending) {
                        const T v = ld_at(Vread + (int64_t)p * nc, off);
                        vp[k] = ok[k] ? v : (T)0;
                    }
                }
#pragma unroll
                for (int k = 0; k < kRows; ++k) a[k] = ok[k] ? phi(K, xp, yq[k], d) : (T)0;
                subtract_columns(Vread, nc, r, sh.vec, ic, a, pending, p, vp, accv[w], lane);
#pragma unroll
                for (int k = 0; k < kRows; ++k) {
                    if (ok[k]) {
                        const int q = ic[k];
                        V[(int64_t)r * nc + q] = a[k];
                        nv2 += (double)a[k] * (double)a[k];
                        const T aa = a[k] < (T)0 ? -a[k] : a[k];
                        if (!bit_get(cmask, q) && aa > cm.best) {
                            cm.best = aa;
                            cm.idx = q;
                            cm.val = a[k];
                        }
                    }
                }
            }
            // next column pivot, |u_r|^2, |v_r|^2 and (term p's products being
            // complete) the cross sum of term p, in one reduction; the rows of
            // the deferred products are read before its closing barrier so
            // that no wave clears them for the next step while another reads
            cm = wave_argmax_u(cm);
            nu2 = wave_total(nu2);
            nv2 = wave_total(nv2);
            if constexpr (NW > 1) {
                if (lane == 0) {
                    sh.abest[w] = cm.best;
                    sh.aidx[w] = cm.idx;
                    sh.aval[w] = cm.val;
                    sh.dsum[0][w] = nu2;
                    sh.dsum[1][w] = nv2;
                }
                __syncthreads();
                cm = Arg<T>{sh.abest[0], sh.aidx[0], sh.aval[0]};
                nu2 = sh.dsum[0][0];
                nv2 = sh.dsum[1][0];
                for (int q = 1; q < NW; ++q) {
                    arg_combine(cm, Arg<T>{sh.abest[q], sh.aidx[q], sh.aval[q]});
                    nu2 += sh.dsum[0][q];
                    nv2 += sh.dsum[1][q];
                }
            }
            double cross_p = 0.0;
            if (pending) {
                for (int l = 0; l < p; ++l) {
                    double gu = accu[0][l], gv = accv[0][l];
                    for (int q = 1; q < NW; ++q) {
                        gu += accu[q][l];
                        gv += accv[q][l];
                    }
                    cross_p += gu * gv;
                }
            }
            if constexpr (NW > 1) __syncthreads();
            // ---- step 4: the norm recursion and the stopping test ----
            ++r;
            if (!fuse) {
                double cross = 0.0;
                if (!fixed) {
                    column_products<T, NT, DC>(Vread, nc, r - 1, sh.gv, sh);
                    for (int l = 0; l < r - 1; ++l) cross += sh.gu[l] * sh.gv[l];
                }
                S2 += 2.0 * cross + nu2 * nv2;
                last_p = nu2 * nv2;
                if (!fixed && !one_shot && sqrt(last_p) <= tol * sqrt(S2)) break;
            } else {
                if (pending) {
                    // term r - 2 = p, its products summed over the waves in order
                    S2 += 2.0 * cross_p + nu2p * nv2p;
                    last_p = nu2p * nv2p;
                    if (sqrt(last_p) <= tol * sqrt(S2)) {
                        r -= 1;  // the speculative term is dropped
                        break;
                    }
                }
                if (r == 1) {  // the first term has no products
                    S2 = nu2 * nv2;
                    last_p = S2;
                    pending = false;
                    if (sqrt(last_p) <= tol * sqrt(S2)) break;
                } else {
                    pending = true;
                    nu2p = nu2;
                    nv2p = nv2;
                }
            }
            // ---- step 6: next column pivot ----
            if (cm.idx == INT_MAX) break;
            j = cm.idx;
        }
        if (tid == 0) {
            rank_out[b] = refused ? -1 : r;
            if (steps_out) steps_out[b] = steps;
        }
        __syncthreads();
    }
}

template <typename T, int NT>
void launch_class(const AcaArgs& a, int64_t b0, int64_t nb, int lds_words, hipStream_t st) {
    if (nb <= 0) return;
    const unsigned grid = (unsigned)(nb < 0x7fffffff ? nb : 0x7fffffff);
    KernelEval<T> K(a.kern);
    hipLaunchKernelGGL((aca_kernel<T, NT>), dim3(grid), dim3(NT),
                       (size_t)lds_words * sizeof(uint32_t), st, (const T*)a.soa, a.soa64, a.n,
                       a.d, K, a.blocks + b0, nb, a.uoff + b0, a.voff + b0, a.ubase, a.vbase,
                       a.kmax, a.eps, a.aca_eta, (T)a.eps0, a.fixed,
                       a.rtarget ? a.rtarget + b0 : nullptr, a.one_shot, a.cap_only,
                       Overflow{a.ovf_used, a.ovf_cap, a.ovf_u0, a.ovf_v0,
                                a.ovf_moved ? a.ovf_moved + b0 : nullptr},
                       lds_words, (T*)a.U, (T*)a.V, a.rank + b0,
                       a.steps ? a.steps + b0 : nullptr);
}

// blocks that continued in overflow storage: their storage offsets move there
__global__ void apply_moved_kernel(const int64_t* __restrict__ moved, int64_t nb, int64_t u0,
                                   int64_t v0, int64_t* __restrict__ uoff,
                                   int64_t* __restrict__ voff) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b < nb && moved[b] >= 0) {
        uoff[b] = u0 + moved[b];
        voff[b] = v0 + moved[b];
    }
}

// first index b with level[b] >= lvl in the non-decreasing level[0..nb)
__global__ void level_split_kernel(const int32_t* __restrict__ level, int64_t nb, int lvl,
                                   int64_t* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t lo = 0, hi = nb;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (level[mid] < lvl)
            lo = mid + 1;
        else
            hi = mid;
    }
    *out = lo;
}

}  // namespace

hipError_t launch_level_split(const int32_t* level, int64_t nb, int lvl, int64_t* out,
                              hipStream_t st) {
    hipLaunchKernelGGL(level_split_kernel, dim3(1), dim3(64), 0, st, level, nb, lvl, out);
    return hipGetLastError();
}

// Size classes of the level-ordered block list, each in its own launch:
// blocks [nsplit, nbig) in kBigThreads-thread workgroups, [nbig, nmed) in
// 256-thread ones, [nmed, nblocks) (the leaf levels) in single-wave
// workgroups; each class reserves the LDS mask words of its largest block.
// (Blocks [0, nsplit) take the multi-workgroup path of k_aca_split.hip.)
// aca_classes_begin queues the classes on the streams aux[0..2] (or on st
// where null) after the work already queued on st; aca_classes_join makes
// st wait for them.  Running the classes concurrently keeps the few large
// blocks of the upper levels from holding back the many small ones.
hipError_t launch_apply_moved(const int64_t* moved, int64_t nb, int64_t u0, int64_t v0,
                              int64_t* uoff, int64_t* voff, hipStream_t st) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(apply_moved_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st,
                       moved, nb, u0, v0, uoff, voff);
    return hipGetLastError();
}

hipError_t aca_classes_begin(const AcaArgs& a, int f64, hipStream_t st, const hipStream_t* aux) {
    const int64_t lo = a.nsplit < a.nblocks ? a.nsplit : a.nblocks;
    const int64_t nbig = a.nbig < lo ? lo : (a.nbig < a.nblocks ? a.nbig : a.nblocks);
    const int64_t nmed = a.nmed < nbig ? nbig : (a.nmed < a.nblocks ? a.nmed : a.nblocks);
    hipStream_t s0 = aux && aux[0] ? aux[0] : st;
    hipStream_t s1 = aux && aux[1] ? aux[1] : s0;
    hipStream_t s2 = aux && aux[2] ? aux[2] : s1;
    hipError_t e = hipSuccess;
    if (aux) {
        hipEvent_t go = nullptr;
        e = hipEventCreateWithFlags(&go, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(go, st);
        for (int k = 0; k < 3 && e == hipSuccess; ++k)
            if (aux[k]) e = hipStreamWaitEvent(aux[k], go, 0);
        if (go) (void)hipEventDestroy(go);
    }
    if (e != hipSuccess) return e;
    if (f64) {
        launch_class<double, kBigThreads>(a, lo, nbig - lo, a.big_words, s0);
        launch_class<double, 256>(a, nbig, nmed - nbig, a.med_words, s1);
        launch_class<double, 64>(a, nmed, a.nblocks - nmed, a.tiny_words, s2);
    } else {
        launch_class<float, kBigThreads>(a, lo, nbig - lo, a.big_words, s0);
        launch_class<float, 256>(a, nbig, nmed - nbig, a.med_words, s1);
        launch_class<float, 64>(a, nmed, a.nblocks - nmed, a.tiny_words, s2);
    }
    return hipGetLastError();
}

hipError_t aca_classes_join(hipStream_t st, const hipStream_t* aux) {
    if (!aux) return hipSuccess;
    hipError_t e = hipSuccess;
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
        if (!aux[k]) continue;
        hipEvent_t done = nullptr;
        e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(done, aux[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, done, 0);
        if (done) (void)hipEventDestroy(done);
    }
    return e;
}

namespace {
// out[0] += steps_b m_b + rank_b n_b (kernel evaluations: a column per step,
// a row per accepted step), out[1] += 2 rank_b (rank_b - 1) (m_b + n_b)
// (multiply-adds of the residual updates and of the norm recursion's inner
// products); integer atomics, order-free
__global__ void aca_work_kernel(const int4* __restrict__ blocks, const int32_t* __restrict__ rank,
                                const int32_t* __restrict__ steps, int64_t nb,
                                unsigned long long* __restrict__ out) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    unsigned long long ev = 0, fl = 0;
    if (b < nb) {
        const int4 bl = blocks[b];
        const unsigned long long m = bl.y - bl.x, nc = bl.w - bl.z;
        const unsigned long long r = rank[b] > 0 ? rank[b] : 0, s = steps[b] > 0 ? steps[b] : 0;
        ev = s * m + r * nc;
        fl = r > 0 ? 2ull * r * (r - 1) * (m + nc) : 0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        ev += __shfl_xor(ev, o, 64);
        fl += __shfl_xor(fl, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&out[0], ev);
        atomicAdd(&out[1], fl);
    }
}
}  // namespace

hipError_t launch_aca_work(const int4* blocks, const int32_t* rank, const int32_t* steps,
                           int64_t nb, unsigned long long* out, hipStream_t st) {
    hipError_t e = hipMemsetAsync(out, 0, 2 * sizeof(unsigned long long), st);
    if (e != hipSuccess || nb == 0) return e;
    hipLaunchKernelGGL(aca_work_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st,
                       blocks, rank, steps, nb, out);
    return hipGetLastError();
}


}  // namespace hmx
