// Batched adaptive cross approximation (Algorithm 2, Section 5.4.1).
//
// One workgroup per admissible block, each running its own rank loop, so
// blocks stop independently (no global "voting" bounded by the slowest
// block).  Blocks of the upper tree levels (many rows) get 512-thread
// workgroups, those of the leaf levels (at most 256 rows) one wave, the rest
// 256 threads (the very largest run on many workgroups each, k_aca_split.hip);
// the canonical leaf order is level order, so each class is a contiguous
// range of every block list.  Per step r:
//   1. residual column  u^ = A[:, j] - sum_{l<r} u_l (v_l)_j   (rows over threads)
//   2. row pivot        i  = argmax over unused rows |u^_i| (lowest index on ties)
//      a column whose largest residual entry is <= eps0 times the column's own
//      largest |entry| adds no rank (zero or rounding-noise residual); the
//      lowest unused column is tried next, and kmax such columns end the block
//   3. u_r = u^ / u^_i,  v_r = A[i, :]^T - sum_{l<r} (u_l)_i v_l  (cols over threads)
//   4. |S_r|_F^2 += 2 sum_{l<r} (u_r.u_l)(v_r.v_l) + |u_r|^2 |v_r|^2   in FP64
//   5. stop if |u_r| |v_r| <= eps (1 - aca_eta) / (1 + eps) |S_r|_F
//   6. next column pivot j = argmax over unused columns |(v_r)_j|
// The inner products of step 4 are computed by the whole workgroup, eight
// previous columns per pass, in FP64; the U products ride along with the
// normalisation of u_r.
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

// the same products in the order of the deferred accumulation of the step
// loop (per batch of kRows rows per thread and per column: a wave sum, added
// to the wave's row of acc; the waves' rows are summed in order by the caller),
// so that a test taken on them decides as the deferred one would
template <typename T, int NT>
__device__ void column_products_waved(const T* __restrict__ X, int len, int p,
                                      double (*acc)[kMaxRankCap]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int l = lane; l < p; l += kWave) acc[w][l] = 0.0;
    __syncthreads();
    for (int ib = 0; ib < len; ib += kRows * NT) {
        const int i0 = ib + threadIdx.x;
        T xp[kRows];
#pragma unroll
        for (int k = 0; k < kRows; ++k)
            xp[k] = i0 + k * NT < len ? X[(int64_t)p * len + i0 + k * NT] : (T)0;
        for (int l = 0; l < p; ++l) {
            const T* __restrict__ Xl = X + (int64_t)l * len;
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < kRows; ++k)
                s += (double)xp[k] * (double)(i0 + k * NT < len ? Xl[i0 + k * NT] : (T)0);
            s = wave_sum(s);
            if (lane == 0) acc[w][l] += s;
        }
    }
    __syncthreads();
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void aca_kernel(
    const T* __restrict__ soa, const double* __restrict__ soa64, int64_t n, int d, KernelEval<T> K,
    const int4* __restrict__ blocks, int64_t nblocks, const int64_t* __restrict__ uoff,
    const int64_t* __restrict__ voff, int64_t ubase, int64_t vbase, int kmax, double eps,
    double aca_eta, T eps0, int fixed, const int32_t* __restrict__ rtarget, int one_shot_mode,
    int cap_only, int lds_words, T* __restrict__ Upool, T* __restrict__ Vpool,
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
        T* __restrict__ U = Upool + (uoff[b] - ubase);
        T* __restrict__ V = Vpool + (voff[b] - vbase);
        // columns l < r are only read in a step, column r only written
        const T* __restrict__ Uread = U;
        const T* __restrict__ Vread = V;
        const int mw = (m + 31) >> 5, nw = (nc + 31) >> 5;
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
        int j = first_column<T, NT>(soa64, n, d, bl, sh);
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
                    column_products_waved<T, NT>(Uread, m, r - 1, accu);
                    column_products_waved<T, NT>(Vread, nc, r - 1, accv);
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
                    refused = true;
                    break;
                }
                target = R;
            }
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
            // kRows rows per thread per pass (kRows * r loads in flight); the
            // trip count is the same for every thread of the workgroup
            for (int ib = 0; ib < m; ib += kRows * NT) {
                const int i0 = ib + tid;
                T a[kRows], up[kRows];
#pragma unroll
                for (int k = 0; k < kRows; ++k) {
                    const int i = i0 + k * NT;
                    a[k] = 0;
                    up[k] = 0;
                    if (i < m) {
                        T xi[3];
                        load_pt(soa, n, d, (int64_t)bl.x + i, xi);
                        a[k] = phi(K, xi, yj, d);
                        const double aa0 = a[k] < (T)0 ? -(double)a[k] : (double)a[k];
                        colmax = aa0 > colmax ? aa0 : colmax;
                        if (pending) up[k] = Uread[(int64_t)p * m + i];
                    }
                }
                for (int l = 0; l < r; ++l) {
                    const T vl = sh.vec[l];
                    const T* __restrict__ Ul = Uread + (int64_t)l * m;
                    T val[kRows];
#pragma unroll
                    for (int k = 0; k < kRows; ++k) {
                        val[k] = i0 + k * NT < m ? Ul[i0 + k * NT] : (T)0;
                        a[k] -= val[k] * vl;
                    }
                    if (pending && l < p) {
                        double s = 0.0;
#pragma unroll
                        for (int k = 0; k < kRows; ++k) s += (double)up[k] * (double)val[k];
                        s = wave_sum(s);
                        if (lane == 0) accu[w][l] += s;
                    }
                }
#pragma unroll
                for (int k = 0; k < kRows; ++k) {
                    const int i = i0 + k * NT;
                    if (i < m) {
                        U[(int64_t)r * m + i] = a[k];
                        const T aa = a[k] < (T)0 ? -a[k] : a[k];
                        if (!bit_get(rmask, i) && aa > am.best) {
                            am.best = aa;
                            am.idx = i;
                            am.val = a[k];
                        }
                    }
                }
            }
            am = block_argmax(am, sh);
            colmax = block_minmax(colmax, 1, sh);
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
            // ---- step 3a: normalise u_r, |u_r|^2 ----
            double nu2 = 0.0;
            T* __restrict__ Ur = U + (int64_t)r * m;
            for (int ib = 0; ib < m; ib += kRows * NT) {
#pragma unroll
                for (int e = 0; e < kRows; ++e) {
                    const int i = ib + tid + e * NT;
                    if (i < m) {
                        const T u = Ur[i] / piv;
                        Ur[i] = u;
                        nu2 += (double)u * (double)u;
                    }
                }
            }
            nu2 = block_sum(nu2, sh, 0);
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
                const int q0 = qb + tid;
                T a[kRows], vp[kRows];
#pragma unroll
                for (int k = 0; k < kRows; ++k) {
                    const int q = q0 + k * NT;
                    a[k] = 0;
                    vp[k] = 0;
                    if (q < nc) {
                        T yq[3];
                        load_pt(soa, n, d, (int64_t)bl.z + q, yq);
                        a[k] = phi(K, xp, yq, d);
                        if (pending) vp[k] = Vread[(int64_t)p * nc + q];
                    }
                }
                for (int l = 0; l < r; ++l) {
                    const T ul = sh.vec[l];
                    const T* __restrict__ Vl = Vread + (int64_t)l * nc;
                    T val[kRows];
#pragma unroll
                    for (int k = 0; k < kRows; ++k) {
                        val[k] = q0 + k * NT < nc ? Vl[q0 + k * NT] : (T)0;
                        a[k] -= ul * val[k];
                    }
                    if (pending && l < p) {
                        double s = 0.0;
#pragma unroll
                        for (int k = 0; k < kRows; ++k) s += (double)vp[k] * (double)val[k];
                        s = wave_sum(s);
                        if (lane == 0) accv[w][l] += s;
                    }
                }
#pragma unroll
                for (int k = 0; k < kRows; ++k) {
                    const int q = q0 + k * NT;
                    if (q < nc) {
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
            nv2 = block_sum(nv2, sh, 1);
            // term p's products are complete once every wave has passed the
            // barrier of the sum above; they are read here, before the
            // barriers of the argmax, so that no wave clears its row for the
            // next step while another still reads it
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
            cm = block_argmax(cm, sh);
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
                       a.rtarget ? a.rtarget + b0 : nullptr, a.one_shot, a.cap_only, lds_words,
                       (T*)a.U, (T*)a.V, a.rank + b0, a.steps ? a.steps + b0 : nullptr);
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

}  // namespace hmx
