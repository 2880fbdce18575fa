// Batched ACA (Algorithm 2) of the largest admissible blocks with many
// workgroups per block (by default those of clusters of 2^18 or more points,
// whose used-row bitmasks would not fit one workgroup's LDS).  One workgroup
// per block serialises such a block on one compute unit for every rank-one
// step; here every step of
// every such block is a short sequence of launches over row and column tiles
// of all the blocks at once, with the per-block decisions (pivots, the FP64
// norm recursion, the stopping test) in one workgroup per block:
//   col   : residual column of tile rows, partial argmax / column maximum
//   pivot : row pivot from the partials, or the next column when rejected
//   norm  : u_r = u^ / pivot on tile rows, partial u_r.u_l and |u_r|^2
//   row   : residual row on tile columns, partial argmax, |v_r|^2, v_r.v_l
//   update: |S_r|^2 += 2 sum (u_r.u_l)(v_r.v_l) + |u_r|^2 |v_r|^2, the
//           stopping test, the next column pivot
// The arithmetic per entry and the pivoting rules are those of the
// single-workgroup kernel; partial sums are combined in tile order, so the
// result is bit-reproducible.  No workgroup ever waits for another: the host
// issues the steps and polls how many blocks are still active.
#include <climits>

#include "hmx_internal.h"

namespace hmx {

namespace {

constexpr int kST = 256;           // threads per workgroup
constexpr int kSRows = 8;          // rows (columns) per thread per tile
constexpr int kTile = kST * kSRows;  // rows per row tile, columns per column tile
constexpr int kSDot = 8;           // previous columns per inner-product pass
constexpr int kSLU = 4;            // previous columns whose loads are in flight together
static_assert(kST > kMaxRankCap, "one thread per previous column and the pivot slot");

template <typename T>
struct Arg {
    T best;
    int idx;
    T val;
};

template <typename T>
__device__ __forceinline__ void arg_combine(Arg<T>& a, const Arg<T>& b) {
    if (b.best > a.best || (b.best == a.best && b.idx < a.idx)) a = b;
}

template <typename T>
__device__ Arg<T> wg_argmax(Arg<T> a, Arg<T>* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        Arg<T> b;
        b.best = __shfl_xor(a.best, o, 64);
        b.idx = __shfl_xor(a.idx, o, 64);
        b.val = __shfl_xor(a.val, o, 64);
        arg_combine(a, b);
    }
    if (lane == 0) sh[w] = a;
    __syncthreads();
    Arg<T> r = sh[0];
    for (int q = 1; q < kST / 64; ++q) arg_combine(r, sh[q]);
    __syncthreads();
    return r;
}

__device__ double wg_sum(double v, double* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = sh[0];
    for (int q = 1; q < kST / 64; ++q) s += sh[q];
    __syncthreads();
    return s;
}

__device__ double wg_max(double v, double* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = sh[0];
    for (int q = 1; q < kST / 64; ++q) s = sh[q] > s ? sh[q] : s;
    __syncthreads();
    return s;
}

__device__ __forceinline__ bool bit_get(const uint32_t* m, int i) {
    return (m[i >> 5] >> (i & 31)) & 1u;
}

// rows tile0 + threadIdx.x + k kST of a tile, clamped into [0, len) so that
// every load is issued unconditionally and a batch of loads overlaps
__device__ __forceinline__ void tile_rows(int first, int len, int (&ic)[kSRows], bool (&ok)[kSRows]) {
#pragma unroll
    for (int k = 0; k < kSRows; ++k) {
        const int i = first + k * kST;
        ok[k] = i < len;
        ic[k] = ok[k] ? i : len - 1;
    }
}

template <typename T>
__device__ __forceinline__ void load_pts(const T* __restrict__ soa, int64_t n, int d, int64_t base,
                                         const int (&ic)[kSRows], T (&p)[kSRows][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < kSRows; ++k)
            p[k][c] = c < d ? soa[(int64_t)c * n + base + ic[k]] : (T)0;
}

// x[k] -= X_l[row k] coef_l for l = 0 .. r - 1 in that order, kSLU columns'
// loads in flight at once (padding columns weigh zero)
template <typename T>
__device__ __forceinline__ void tile_subtract(const T* __restrict__ X, int64_t ld, int r,
                                              const T* coef, const int (&ic)[kSRows],
                                              T (&x)[kSRows]) {
    r = __builtin_amdgcn_readfirstlane(r);
    for (int l0 = 0; l0 < r; l0 += kSLU) {
        T c[kSLU], val[kSLU][kSRows];
#pragma unroll
        for (int q = 0; q < kSLU; ++q) {
            const bool in = l0 + q < r;
            const int l = in ? l0 + q : r - 1;
            c[q] = in ? coef[l] : (T)0;
            const T* __restrict__ Xl = X + (int64_t)l * ld;
#pragma unroll
            for (int k = 0; k < kSRows; ++k) val[q][k] = Xl[ic[k]];
        }
#pragma unroll
        for (int q = 0; q < kSLU; ++q)
#pragma unroll
            for (int k = 0; k < kSRows; ++k) x[k] -= val[q][k] * c[q];
    }
}

// dp[l] = sum over the tile of y[k] X_l[row k] (l < r; y zero outside the
// block), per column: rows in k order per thread, a wave sum, the waves in
// order; kSLU columns' loads in flight at once
template <typename T>
__device__ __forceinline__ void tile_products(const T* __restrict__ X, int64_t ld, int r,
                                              const int (&ic)[kSRows], const T (&y)[kSRows],
                                              double (*shp)[kSDot], double* dp) {
    r = __builtin_amdgcn_readfirstlane(r);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int c0 = 0; c0 < r; c0 += kSDot) {
        const int nk = r - c0 < kSDot ? r - c0 : kSDot;
        double acc[kSDot];
#pragma unroll
        for (int q = 0; q < kSDot; ++q) acc[q] = 0.0;
#pragma unroll
        for (int h = 0; h < kSDot; h += kSLU) {
            T val[kSLU][kSRows];
#pragma unroll
            for (int q = 0; q < kSLU; ++q) {
                const int l = c0 + h + q < r ? c0 + h + q : r - 1;
                const T* __restrict__ Xl = X + (int64_t)l * ld;
#pragma unroll
                for (int k = 0; k < kSRows; ++k) val[q][k] = Xl[ic[k]];
            }
#pragma unroll
            for (int q = 0; q < kSLU; ++q)
#pragma unroll
                for (int k = 0; k < kSRows; ++k) acc[h + q] += (double)y[k] * (double)val[q][k];
        }
#pragma unroll
        for (int q = 0; q < kSDot; ++q) acc[q] = wave_sum(acc[q]);
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < kSDot; ++q) shp[w][q] = acc[q];
        __syncthreads();
        if ((int)threadIdx.x < nk) {
            double t = shp[0][threadIdx.x];
            for (int q = 1; q < kST / 64; ++q) t += shp[q][threadIdx.x];
            dp[c0 + threadIdx.x] = t;
        }
        __syncthreads();
    }
}

// per-block state of the step loop
struct SplitState {
    int r, j, ip, nfailed, ncols, steps, target, R;
    int done, skip, refused, one_shot;
    double S2, last_p;
};

template <typename T>
struct ColPart {
    T best, val;
    int idx;
    double colmax;
};

template <typename T>
struct RowPart {
    T best, val;
    int idx;
    double nv2;
};

struct SplitArgs {
    const void* soa;
    const double* soa64;
    int64_t n;
    int d;
    KernelFn kern;
    const int4* blocks;
    const int64_t* uoff;
    const int64_t* voff;
    int64_t ubase, vbase;
    int kmax;
    double eps, aca_eta, eps0;
    int fixed;
    const int32_t* rtarget;
    int one_shot, cap_only;
    void* U;
    void* V;
};

// ---------------------------------------------------------------------------
// initial state, cleared masks, the first column (the sigma point nearest to
// the centre of tau's bounding box, FP64 without contraction)
template <typename T>
__global__ __launch_bounds__(kST) void split_init_kernel(SplitArgs a, int64_t nb,
                                                         const int64_t* __restrict__ moff,
                                                         uint32_t* __restrict__ masks,
                                                         SplitState* __restrict__ state) {
    __shared__ double shd[kST / 64];
    __shared__ int shi[kST / 64];
    const int64_t b = blockIdx.x;
    if (b >= nb) return;
    const int4 bl = a.blocks[b];
    const int m = bl.y - bl.x, nc = bl.w - bl.z;
    uint32_t* mk = masks + moff[b];
    const int words = (m + 31) / 32 + (nc + 31) / 32;
    for (int q = threadIdx.x; q < words; q += kST) mk[q] = 0u;
    double c[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < a.d; ++k) {
        double mn = INFINITY, mx = -INFINITY;
        for (int i = threadIdx.x; i < m; i += kST) {
            const double v = a.soa64[(int64_t)k * a.n + bl.x + i];
            mn = v < mn ? v : mn;
            mx = v > mx ? v : mx;
        }
        mn = -wg_max(-mn, shd);
        mx = wg_max(mx, shd);
        c[k] = __dmul_rn(0.5, __dadd_rn(mn, mx));
    }
    double best = INFINITY;
    int bi = INT_MAX;
    for (int q = threadIdx.x; q < nc; q += kST) {
        double s = 0.0;
        for (int k = 0; k < a.d; ++k) {
            const double t = __dsub_rn(a.soa64[(int64_t)k * a.n + bl.z + q], c[k]);
            s = __dadd_rn(s, __dmul_rn(t, t));
        }
        if (s < best) {
            best = s;
            bi = q;
        }
    }
    // argmin with the lowest index on ties
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double k2 = __shfl_xor(best, o, 64);
        const int i2 = __shfl_xor(bi, o, 64);
        if (k2 < best || (k2 == best && i2 < bi)) {
            best = k2;
            bi = i2;
        }
    }
    if (lane == 0) {
        shd[w] = best;
        shi[w] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double bk = shd[0];
        int j = shi[0];
        for (int q = 1; q < kST / 64; ++q)
            if (shd[q] < bk || (shd[q] == bk && shi[q] < j)) {
                bk = shd[q];
                j = shi[q];
            }
        int R = a.kmax;
        R = m < R ? m : R;
        R = nc < R ? nc : R;
        SplitState s{};
        s.R = R;
        s.j = j;
        const bool sized = a.rtarget && a.rtarget[b] > 0;
        s.one_shot = sized && a.one_shot;
        s.target = sized ? (a.rtarget[b] < R ? a.rtarget[b] : R) : R;
        state[b] = s;
    }
}

// residual column j of every active block on one row tile
template <typename T>
__global__ __launch_bounds__(kST) void split_col_kernel(SplitArgs a, KernelEval<T> K,
                                                        const int2* __restrict__ tiles,
                                                        const int64_t* __restrict__ moff,
                                                        const uint32_t* __restrict__ masks,
                                                        const SplitState* __restrict__ state,
                                                        ColPart<T>* __restrict__ part) {
    __shared__ T vec[kMaxRankCap];
    __shared__ Arg<T> sha[kST / 64];
    __shared__ double shd[kST / 64];
    const int2 tl = tiles[blockIdx.x];
    const SplitState s = state[tl.x];
    if (s.done) return;
    const int4 bl = a.blocks[tl.x];
    const int m = bl.y - bl.x, nc = bl.w - bl.z;
    const T* __restrict__ soa = (const T*)a.soa;
    T* __restrict__ U = (T*)a.U + (a.uoff[tl.x] - a.ubase);
    const T* __restrict__ V = (const T*)a.V + (a.voff[tl.x] - a.vbase);
    const T* __restrict__ Uread = U;
    const int r = s.r, j = s.j;
    if ((int)threadIdx.x < r) vec[threadIdx.x] = V[(int64_t)threadIdx.x * nc + j];
    __syncthreads();
    const uint32_t* rmask = masks + moff[tl.x];
    T yj[3];
    load_pt(soa, a.n, a.d, (int64_t)bl.z + j, yj);
    Arg<T> am{(T)-1, INT_MAX, (T)0};
    double colmax = 0.0;
    int ic[kSRows];
    bool ok[kSRows];
    tile_rows(tl.y * kTile + threadIdx.x, m, ic, ok);
    T xi[kSRows][3], v[kSRows];
    load_pts(soa, a.n, a.d, (int64_t)bl.x, ic, xi);
#pragma unroll
    for (int k = 0; k < kSRows; ++k) {
        v[k] = ok[k] ? phi(K, xi[k], yj, a.d) : (T)0;
        const double aa0 = v[k] < (T)0 ? -(double)v[k] : (double)v[k];
        colmax = aa0 > colmax ? aa0 : colmax;
    }
    tile_subtract(Uread, m, r, vec, ic, v);
#pragma unroll
    for (int k = 0; k < kSRows; ++k) {
        if (ok[k]) {
            const int i = ic[k];
            U[(int64_t)r * m + i] = v[k];
            const T aa = v[k] < (T)0 ? -v[k] : v[k];
            if (!bit_get(rmask, i) && aa > am.best) {
                am.best = aa;
                am.idx = i;
                am.val = v[k];
            }
        }
    }
    am = wg_argmax(am, sha);
    colmax = wg_max(colmax, shd);
    if (threadIdx.x == 0) part[blockIdx.x] = ColPart<T>{am.best, am.val, am.idx, colmax};
}

// row pivot of every active block from its tiles' partials, or the next
// column when the residual column is rejected
template <typename T>
__global__ __launch_bounds__(kST) void split_pivot_kernel(SplitArgs a, int64_t nb,
                                                          const int64_t* __restrict__ toff,
                                                          const int64_t* __restrict__ moff,
                                                          uint32_t* __restrict__ masks,
                                                          SplitState* __restrict__ state,
                                                          const ColPart<T>* __restrict__ part,
                                                          T* __restrict__ urow) {
    __shared__ Arg<T> sha[kST / 64];
    __shared__ double shd[kST / 64];
    __shared__ int shi[kST / 64];
    const int64_t b = blockIdx.x;
    if (b >= nb) return;
    SplitState s = state[b];
    if (s.done) return;
    const int4 bl = a.blocks[b];
    const int m = bl.y - bl.x, nc = bl.w - bl.z;
    uint32_t* rmask = masks + moff[b];
    uint32_t* cmask = rmask + (m + 31) / 32;
    // combine the tiles' partials in tile order within each thread, then the tree
    Arg<T> am{(T)-1, INT_MAX, (T)0};
    double colmax = 0.0;
    for (int64_t t = toff[b] + threadIdx.x; t < toff[b + 1]; t += kST) {
        const ColPart<T> p = part[t];
        arg_combine(am, Arg<T>{p.best, p.idx, p.val});
        colmax = p.colmax > colmax ? p.colmax : colmax;
    }
    am = wg_argmax(am, sha);
    colmax = wg_max(colmax, shd);
    __syncthreads();
    if (threadIdx.x == 0) cmask[s.j >> 5] |= 1u << (s.j & 31);
    s.ncols += 1;
    s.steps += 1;
    if (am.idx == INT_MAX || (double)am.best <= a.eps0 * colmax) {
        // no usable pivot: the lowest unused column, or the end of the block
        s.nfailed += 1;
        s.skip = 1;
        if (s.ncols >= nc || s.nfailed >= a.kmax) {
            s.done = 1;
        } else {
            __syncthreads();
            int cand = INT_MAX;
            for (int q = threadIdx.x; q < (nc + 31) / 32; q += kST) {
                const uint32_t word = cmask[q];
                if (word != 0xffffffffu) {
                    const int c = (q << 5) + __ffs(~word) - 1;
                    if (c < nc && c < cand) cand = c;
                }
            }
            const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const int u = __shfl_xor(cand, o, 64);
                cand = u < cand ? u : cand;
            }
            if (lane == 0) shi[w] = cand;
            __syncthreads();
            cand = shi[0];
            for (int q = 1; q < kST / 64; ++q) cand = shi[q] < cand ? shi[q] : cand;
            if (cand == INT_MAX)
                s.done = 1;
            else
                s.j = cand;
        }
    } else {
        s.skip = 0;
        s.ip = am.idx;
        const T* __restrict__ U = (const T*)a.U + (a.uoff[b] - a.ubase);
        // row ip of the previous columns, and the pivot value itself
        if ((int)threadIdx.x < s.r) urow[b * (kMaxRankCap + 1) + threadIdx.x] = U[(int64_t)threadIdx.x * m + s.ip];
        if (threadIdx.x == 0) {
            urow[b * (kMaxRankCap + 1) + kMaxRankCap] = am.val;
            rmask[s.ip >> 5] |= 1u << (s.ip & 31);
        }
    }
    if (threadIdx.x == 0) state[b] = s;
}

// u_r = u^ / pivot on one row tile; partial u_r.u_l (l < r) and |u_r|^2
template <typename T>
__global__ __launch_bounds__(kST) void split_norm_kernel(SplitArgs a, const int2* __restrict__ tiles,
                                                         const SplitState* __restrict__ state,
                                                         const T* __restrict__ urow,
                                                         double* __restrict__ dpart) {
    __shared__ double shp[kST / 64][kSDot];
    __shared__ double shd[kST / 64];
    const int2 tl = tiles[blockIdx.x];
    const SplitState s = state[tl.x];
    if (s.done || s.skip) return;
    const int4 bl = a.blocks[tl.x];
    const int m = bl.y - bl.x;
    T* __restrict__ U = (T*)a.U + (a.uoff[tl.x] - a.ubase);
    const int r = s.r;
    const T piv = urow[(int64_t)tl.x * (kMaxRankCap + 1) + kMaxRankCap];
    double* dp = dpart + (int64_t)blockIdx.x * (kMaxRankCap + 1);
    int ic[kSRows];
    bool ok[kSRows];
    tile_rows(tl.y * kTile + threadIdx.x, m, ic, ok);
    T u[kSRows];
#pragma unroll
    for (int k = 0; k < kSRows; ++k) u[k] = U[(int64_t)r * m + ic[k]];
    double nu2 = 0.0;
#pragma unroll
    for (int k = 0; k < kSRows; ++k) {
        if (ok[k]) {
            u[k] = u[k] / piv;
            U[(int64_t)r * m + ic[k]] = u[k];
            nu2 += (double)u[k] * (double)u[k];
        } else {
            u[k] = (T)0;
        }
    }
    nu2 = wg_sum(nu2, shd);
    if (threadIdx.x == 0) dp[kMaxRankCap] = nu2;
    tile_products(U, m, r, ic, u, shp, dp);
}

// residual row i_r on one column tile: V[:, r], partial argmax over unused
// columns, |v_r|^2, v_r.v_l (l < r)
template <typename T>
__global__ __launch_bounds__(kST) void split_row_kernel(SplitArgs a, KernelEval<T> K,
                                                        const int2* __restrict__ tiles,
                                                        const int64_t* __restrict__ moff,
                                                        const uint32_t* __restrict__ masks,
                                                        const SplitState* __restrict__ state,
                                                        const T* __restrict__ urow,
                                                        RowPart<T>* __restrict__ part,
                                                        double* __restrict__ dpart) {
    __shared__ T vec[kMaxRankCap];
    __shared__ Arg<T> sha[kST / 64];
    __shared__ double shd[kST / 64];
    __shared__ double shp[kST / 64][kSDot];
    const int2 tl = tiles[blockIdx.x];
    const SplitState s = state[tl.x];
    if (s.done || s.skip) return;
    const int4 bl = a.blocks[tl.x];
    const int m = bl.y - bl.x, nc = bl.w - bl.z;
    const T* __restrict__ soa = (const T*)a.soa;
    T* __restrict__ V = (T*)a.V + (a.voff[tl.x] - a.vbase);
    const T* __restrict__ Vread = V;
    const int r = s.r;
    if ((int)threadIdx.x < r) vec[threadIdx.x] = urow[(int64_t)tl.x * (kMaxRankCap + 1) + threadIdx.x];
    __syncthreads();
    const uint32_t* cmask = masks + moff[tl.x] + (m + 31) / 32;
    T xp[3];
    load_pt(soa, a.n, a.d, (int64_t)bl.x + s.ip, xp);
    int ic[kSRows];
    bool ok[kSRows];
    tile_rows(tl.y * kTile + threadIdx.x, nc, ic, ok);
    T yq[kSRows][3], v[kSRows];
    load_pts(soa, a.n, a.d, (int64_t)bl.z, ic, yq);
#pragma unroll
    for (int k = 0; k < kSRows; ++k) v[k] = ok[k] ? phi(K, xp, yq[k], a.d) : (T)0;
    tile_subtract(Vread, nc, r, vec, ic, v);
    Arg<T> cm{(T)-1, INT_MAX, (T)0};
    double nv2 = 0.0;
#pragma unroll
    for (int k = 0; k < kSRows; ++k) {
        if (ok[k]) {
            const int q = ic[k];
            V[(int64_t)r * nc + q] = v[k];
            nv2 += (double)v[k] * (double)v[k];
            const T aa = v[k] < (T)0 ? -v[k] : v[k];
            if (!bit_get(cmask, q) && aa > cm.best) {
                cm.best = aa;
                cm.idx = q;
                cm.val = v[k];
            }
        } else {
            v[k] = (T)0;
        }
    }
    cm = wg_argmax(cm, sha);
    nv2 = wg_sum(nv2, shd);
    if (threadIdx.x == 0) part[blockIdx.x] = RowPart<T>{cm.best, cm.val, cm.idx, nv2};
    double* dp = dpart + (int64_t)blockIdx.x * (kMaxRankCap + 1);
    tile_products(Vread, nc, r, ic, v, shp, dp);
}

// the norm recursion, the stopping test and the next column pivot
template <typename T>
__global__ __launch_bounds__(kST) void split_update_kernel(SplitArgs a, int64_t nb,
                                                           const int64_t* __restrict__ rtoff,
                                                           const int64_t* __restrict__ ctoff,
                                                           SplitState* __restrict__ state,
                                                           const double* __restrict__ udpart,
                                                           const RowPart<T>* __restrict__ rpart,
                                                           const double* __restrict__ vdpart) {
    __shared__ double gu[kMaxRankCap + 1];
    __shared__ double gv[kMaxRankCap + 1];
    __shared__ Arg<T> sha[kST / 64];
    __shared__ double shd[kST / 64];
    const int64_t b = blockIdx.x;
    if (b >= nb) return;
    SplitState s = state[b];
    if (s.done || s.skip) return;
    const int r = s.r;
    // u_r.u_l (l < r) and |u_r|^2 summed over the row tiles in order
    for (int l = threadIdx.x; l <= kMaxRankCap; l += kST) {
        if (l < r || l == kMaxRankCap) {
            double t = 0.0;
            for (int64_t k = rtoff[b]; k < rtoff[b + 1]; ++k) t += udpart[k * (kMaxRankCap + 1) + l];
            gu[l] = t;
        }
        if (l < r) {
            double t = 0.0;
            for (int64_t k = ctoff[b]; k < ctoff[b + 1]; ++k) t += vdpart[k * (kMaxRankCap + 1) + l];
            gv[l] = t;
        }
    }
    Arg<T> cm{(T)-1, INT_MAX, (T)0};
    double nv2 = 0.0;
    if (threadIdx.x == 0)
        for (int64_t k = ctoff[b]; k < ctoff[b + 1]; ++k) nv2 += rpart[k].nv2;
    for (int64_t k = ctoff[b] + threadIdx.x; k < ctoff[b + 1]; k += kST) {
        const RowPart<T> p = rpart[k];
        arg_combine(cm, Arg<T>{p.best, p.idx, p.val});
    }
    cm = wg_argmax(cm, sha);
    if (threadIdx.x == 0) {
        const double tol = a.eps * (1.0 - a.aca_eta) / (1.0 + a.eps);
        const double nu2 = gu[kMaxRankCap];
        double cross = 0.0;
        for (int l = 0; l < r; ++l) cross += gu[l] * gv[l];
        s.r = r + 1;
        s.S2 += 2.0 * cross + nu2 * nv2;
        s.last_p = nu2 * nv2;
        if (!a.fixed && !s.one_shot && sqrt(s.last_p) <= tol * sqrt(s.S2)) {
            s.done = 1;
        } else if (cm.idx == INT_MAX) {
            s.done = 1;
        } else {
            s.j = cm.idx;
            // the top of the next step: target reached?
            if (s.r >= s.target) {
                if (s.r >= s.R) {
                    s.done = 1;
                } else {
                    bool fin = false;
                    if (s.one_shot) {
                        s.one_shot = 0;
                        if (sqrt(s.last_p) <= tol * sqrt(s.S2)) fin = true;
                    }
                    if (fin) {
                        s.done = 1;
                    } else if (a.cap_only) {
                        s.refused = 1;
                        s.done = 1;
                    } else {
                        s.target = s.R;
                    }
                }
            }
        }
        state[b] = s;
    }
    (void)shd;
}

__global__ void split_count_kernel(const SplitState* __restrict__ state, int64_t nb,
                                   int* __restrict__ active) {
    __shared__ int sh[kST / 64];
    int c = 0;
    for (int64_t b = threadIdx.x; b < nb; b += kST) c += state[b].done ? 0 : 1;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) *active = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void split_finish_kernel(const SplitState* __restrict__ state, int64_t nb,
                                    int32_t* __restrict__ rank, int32_t* __restrict__ steps) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const SplitState s = state[b];
    rank[b] = s.refused ? -1 : s.r;
    if (steps) steps[b] = s.steps;
}

template <typename T>
hipError_t run_split(const AcaArgs& A, const SplitPlan& P, hipStream_t st) {
    SplitArgs a{A.soa, A.soa64, A.n, A.d, A.kern, A.blocks, A.uoff, A.voff, A.ubase, A.vbase,
                A.kmax, A.eps, A.aca_eta, A.eps0, A.fixed, A.rtarget, A.one_shot, A.cap_only,
                A.U, A.V};
    KernelEval<T> K(A.kern);
    const int64_t nb = P.nblocks;
    SplitState* state = (SplitState*)P.state;
    ColPart<T>* cpart = (ColPart<T>*)P.colpart;
    RowPart<T>* rpart = (RowPart<T>*)P.rowpart;
    T* urow = (T*)P.urow;
    hipLaunchKernelGGL(split_init_kernel<T>, dim3((unsigned)nb), dim3(kST), 0, st, a, nb, P.moff,
                       P.masks, state);
    hipError_t e = hipGetLastError();
    // at most k_max rank-one steps and k_max rejected columns per block
    const int max_iter = 2 * A.kmax;
    for (int it = 0; it < max_iter && e == hipSuccess; ++it) {
        hipLaunchKernelGGL(split_col_kernel<T>, dim3((unsigned)P.nrowtiles), dim3(kST), 0, st, a,
                           K, P.rowtiles, P.moff, P.masks, state, cpart);
        hipLaunchKernelGGL(split_pivot_kernel<T>, dim3((unsigned)nb), dim3(kST), 0, st, a, nb,
                           P.rtoff, P.moff, P.masks, state, cpart, urow);
        hipLaunchKernelGGL(split_norm_kernel<T>, dim3((unsigned)P.nrowtiles), dim3(kST), 0, st, a,
                           P.rowtiles, state, urow, P.udpart);
        hipLaunchKernelGGL(split_row_kernel<T>, dim3((unsigned)P.ncoltiles), dim3(kST), 0, st, a,
                           K, P.coltiles, P.moff, P.masks, state, urow, rpart, P.vdpart);
        hipLaunchKernelGGL(split_update_kernel<T>, dim3((unsigned)nb), dim3(kST), 0, st, a, nb,
                           P.rtoff, P.ctoff, state, P.udpart, rpart, P.vdpart);
        e = hipGetLastError();
        if (e == hipSuccess && (it & 7) == 7) {
            // poll: stop once every block has finished
            hipLaunchKernelGGL(split_count_kernel, dim3(1), dim3(kST), 0, st, state, nb,
                               P.active_dev);
            e = hipMemcpyAsync(P.active_host, P.active_dev, sizeof(int), hipMemcpyDeviceToHost,
                               st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e == hipSuccess && *P.active_host == 0) break;
        }
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(split_finish_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st,
                       state, nb, A.rank, A.steps);
    return hipGetLastError();
}

}  // namespace

size_t split_state_bytes() { return sizeof(SplitState); }
size_t split_colpart_bytes(int f64) { return f64 ? sizeof(ColPart<double>) : sizeof(ColPart<float>); }
size_t split_rowpart_bytes(int f64) { return f64 ? sizeof(RowPart<double>) : sizeof(RowPart<float>); }
int split_tile() { return kTile; }

// blocks A.blocks[0 .. P.nblocks) (the chunk's largest) with many workgroups
// each; A.rank / A.steps receive their ranks and evaluated columns
hipError_t launch_aca_split(const AcaArgs& A, const SplitPlan& P, int f64, hipStream_t st) {
    if (P.nblocks == 0) return hipSuccess;
    return f64 ? run_split<double>(A, P, st) : run_split<float>(A, P, st);
}

}  // namespace hmx
