// Cluster tree, cluster bounding boxes and the level-by-level block cluster
// tree traversal (Section 2.1-2.3, Algorithm 1 in the breadth-first form of
// Algorithm 4, Section 5.2-5.3), plus the scan primitives they use.
//
// Compiled with -ffp-contract=off: the admissibility test (eq. (3), squared)
// must be the exact IEEE operation sequence so the partition is reproducible
// bit for bit.
//
// Cluster tree: implicit and heap-indexed.  Node (level l, k) has id
// 2^l - 1 + k; its children are 2 id + 1 (first, floor half of the Morton
// range) and 2 id + 2.  Slots whose parent did not split hold lo = hi = -1.
#include "hmx_internal.h"

namespace hmx {

namespace {

// ---------------------------------------------------------------------------
// reduce-then-scan exclusive scan (int64 and int32), deterministic
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* sh /*kScanThreads/64 + 1*/, T* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int q = 0; q < kScanThreads / 64; ++q) {
            T t = sh[q];
            sh[q] = run;
            run += t;
        }
        sh[kScanThreads / 64] = run;
    }
    __syncthreads();
    T res = sh[w] + x - v;
    *total = sh[kScanThreads / 64];
    __syncthreads();
    return res;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const T* __restrict__ in,
                                                                   int64_t n,
                                                                   int64_t* __restrict__ bsum) {
    __shared__ int64_t sh[kScanThreads / 64 + 1];
    const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * (int64_t)kScanItems;
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += (int64_t)in[base + k];
    int64_t tot;
    block_exclusive_scan<int64_t>(s, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// exclusive scan of nb block sums by one workgroup; total written to total_dev
__global__ __launch_bounds__(kScanThreads) void scan_blocks_kernel(int64_t* __restrict__ bsum,
                                                                   int64_t nb,
                                                                   int64_t* __restrict__ total_dev) {
    __shared__ int64_t sh[kScanThreads / 64 + 1];
    const int64_t chunk = (nb + kScanThreads - 1) / kScanThreads;
    const int64_t b0 = threadIdx.x * chunk;
    int64_t s = 0;
    for (int64_t q = 0; q < chunk; ++q)
        if (b0 + q < nb) s += bsum[b0 + q];
    int64_t tot;
    int64_t run = block_exclusive_scan<int64_t>(s, sh, &tot);
    for (int64_t q = 0; q < chunk; ++q)
        if (b0 + q < nb) {
            int64_t t = bsum[b0 + q];
            bsum[b0 + q] = run;
            run += t;
        }
    if (threadIdx.x == 0 && total_dev) *total_dev = tot;
}

// out[i] = exclusive (or inclusive) prefix of in, plus the block offset
template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const T* __restrict__ in,
                                                                  T* __restrict__ out, int64_t n,
                                                                  const int64_t* __restrict__ bsum,
                                                                  int inclusive) {
    __shared__ int64_t sh[kScanThreads / 64 + 1];
    const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * (int64_t)kScanItems;
    T v[kScanItems];
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : (T)0;
        s += (int64_t)v[k];
    }
    int64_t tot;
    int64_t run = block_exclusive_scan<int64_t>(s, sh, &tot) + bsum[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) {
            if (inclusive) {
                run += (int64_t)v[k];
                out[base + k] = (T)run;
            } else {
                out[base + k] = (T)run;
                run += (int64_t)v[k];
            }
        }
    }
}

template <typename T>
hipError_t scan_generic(const T* in, T* out, int64_t n, int inclusive, int64_t* total_dev,
                        void* scratch, hipStream_t st) {
    if (n <= 0) {
        if (total_dev) return hipMemsetAsync(total_dev, 0, sizeof(int64_t), st);
        return hipSuccess;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    int64_t* bsum = (int64_t*)scratch;
    hipLaunchKernelGGL(scan_reduce_kernel<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in,
                       n, bsum);
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(kScanThreads), 0, st, bsum, nb,
                       total_dev);
    hipLaunchKernelGGL(scan_apply_kernel<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in,
                       out, n, bsum, inclusive);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// cluster tree (Section 2.1; Z-order halving, Section 4.4)
// ---------------------------------------------------------------------------
// node k of `level` in the tree whose slots start at B: a leaf's parent slot
// that does not split leaves it empty (lo = hi = -1); the root holds [r0, r1)
__device__ __forceinline__ void tree_node(int64_t B, int level, int64_t k, int32_t r0, int32_t r1,
                                          int leaf, int32_t* __restrict__ lo,
                                          int32_t* __restrict__ hi) {
    const int64_t local = (1ll << level) - 1 + k;
    const int64_t id = B + local;
    if (level == 0) {
        lo[id] = r0;
        hi[id] = r1;
        return;
    }
    const int64_t p = B + (local - 1) / 2;
    const int32_t plo = lo[p], phi = hi[p];
    if (plo >= 0 && phi - plo > leaf) {
        const int32_t mid = plo + (phi - plo) / 2;
        if (local & 1) {
            lo[id] = plo;
            hi[id] = mid;
        } else {
            lo[id] = mid;
            hi[id] = phi;
        }
    } else {
        lo[id] = -1;
        hi[id] = -1;
    }
}

__global__ void tree_level_kernel(int level, int64_t n, int leaf, int32_t* __restrict__ lo,
                                  int32_t* __restrict__ hi) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= (1ll << level)) return;
    tree_node(0, level, k, 0, (int32_t)n, leaf, lo, hi);
}

// the same level of every problem's tree (grid y = problem; problem p's
// slots start at nbase[p], its tree has levels 0 .. depth[p])
__global__ void forest_tree_level_kernel(int level, const int64_t* __restrict__ pbase,
                                         const int64_t* __restrict__ nbase,
                                         const int32_t* __restrict__ depth, int leaf,
                                         int32_t* __restrict__ lo, int32_t* __restrict__ hi) {
    const int p = blockIdx.y;
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (level > depth[p] || k >= (1ll << level)) return;
    tree_node(nbase[p], level, k, (int32_t)pbase[p], (int32_t)pbase[p + 1], leaf, lo, hi);
}

// one wave per node: a leaf cluster reduces its points, an inner cluster
// takes the union of its two children (min/max are exact, so both give the
// brute-force box of Section 2.2 bit for bit)
__device__ __forceinline__ void box_node(int64_t id, int64_t c0, int lane, int d, int leaf,
                                         const int32_t* __restrict__ lo,
                                         const int32_t* __restrict__ hi,
                                         const double* __restrict__ soa, int64_t n,
                                         double* __restrict__ bmin, double* __restrict__ bmax) {
    const int32_t a = lo[id], b = hi[id];
    if (a < 0) return;
    if (b - a <= leaf) {
        for (int q = 0; q < d; ++q) {
            double mn = INFINITY, mx = -INFINITY;
            for (int64_t i = a + lane; i < b; i += 64) {
                double v = soa[(int64_t)q * n + i];
                mn = v < mn ? v : mn;
                mx = v > mx ? v : mx;
            }
            for (int o = 32; o > 0; o >>= 1) {
                double m2 = __shfl_xor(mn, o, 64), x2 = __shfl_xor(mx, o, 64);
                mn = m2 < mn ? m2 : mn;
                mx = x2 > mx ? x2 : mx;
            }
            if (lane == 0) {
                bmin[id * d + q] = mn;
                bmax[id * d + q] = mx;
            }
        }
    } else if (lane == 0) {
        const int64_t c1 = c0 + 1;
        for (int q = 0; q < d; ++q) {
            double m0 = bmin[c0 * d + q], m1 = bmin[c1 * d + q];
            double x0 = bmax[c0 * d + q], x1 = bmax[c1 * d + q];
            bmin[id * d + q] = m1 < m0 ? m1 : m0;
            bmax[id * d + q] = x1 > x0 ? x1 : x0;
        }
    }
}

__global__ __launch_bounds__(256) void box_level_kernel(int level, int d, int leaf,
                                                        const int32_t* __restrict__ lo,
                                                        const int32_t* __restrict__ hi,
                                                        const double* __restrict__ soa, int64_t n,
                                                        double* __restrict__ bmin,
                                                        double* __restrict__ bmax) {
    const int64_t k = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 64;
    const int64_t cnt = 1ll << level;
    if (k >= cnt) return;
    const int64_t id = cnt - 1 + k;
    box_node(id, 2 * id + 1, threadIdx.x & 63, d, leaf, lo, hi, soa, n, bmin, bmax);
}

// the same level of every problem's tree (grid y = problem); boxes of the
// union's 3 x N coordinates (a problem's missing dimensions are zero there,
// so its boxes are [0, 0] in them)
__global__ __launch_bounds__(256) void forest_box_level_kernel(
    int level, const int64_t* __restrict__ nbase, const int32_t* __restrict__ depth, int leaf,
    const int32_t* __restrict__ lo, const int32_t* __restrict__ hi,
    const double* __restrict__ soa, int64_t N, double* __restrict__ bmin,
    double* __restrict__ bmax) {
    const int p = blockIdx.y;
    const int64_t k = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 64;
    if (level > depth[p] || k >= (1ll << level)) return;
    const int64_t local = (1ll << level) - 1 + k;
    const int64_t B = nbase[p];
    box_node(B + local, B + 2 * local + 1, threadIdx.x & 63, 3, leaf, lo, hi, soa, N, bmin, bmax);
}

// slot -> first slot of its problem's tree
__global__ void forest_slot_base_kernel(const int64_t* __restrict__ nbase, int np, int64_t nslots,
                                        int32_t* __restrict__ base) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < nslots) base[i] = (int32_t)nbase[problem_of(nbase, np, i)];
}

// ---------------------------------------------------------------------------
// block cluster tree traversal (Algorithm 1 via Algorithm 4)
// ---------------------------------------------------------------------------
constexpr int kTravThreads = 256;
constexpr int kTravItems = 4;
constexpr int kTravTile = kTravThreads * kTravItems;

// eq. (3) squared: min(diam_t^2, diam_s^2) <= eta^2 dist^2, sums in dimension order
__device__ __forceinline__ bool admissible(const double* __restrict__ bmin,
                                           const double* __restrict__ bmax, int64_t t, int64_t s,
                                           int d, double eta) {
    double dt = 0.0, ds = 0.0, dist2 = 0.0;
    for (int k = 0; k < d; ++k) {
        double w = bmax[t * d + k] - bmin[t * d + k];
        dt += w * w;
    }
    for (int k = 0; k < d; ++k) {
        double w = bmax[s * d + k] - bmin[s * d + k];
        ds += w * w;
    }
    for (int k = 0; k < d; ++k) {
        double g1 = bmin[t * d + k] - bmax[s * d + k];
        double g2 = bmin[s * d + k] - bmax[t * d + k];
        g1 = g1 < 0.0 ? 0.0 : g1;
        g2 = g2 < 0.0 ? 0.0 : g2;
        double q = g1 * g1 + g2 * g2;
        dist2 += q;
    }
    double dmin = dt < ds ? dt : ds;
    return dmin <= (eta * eta) * dist2;
}

// 0 = admissible leaf, 1 = split into four children, 2 = dense leaf
__device__ __forceinline__ int classify(int2 ts, const int32_t* __restrict__ lo,
                                        const int32_t* __restrict__ hi,
                                        const double* __restrict__ bmin,
                                        const double* __restrict__ bmax, int d, int leaf,
                                        double eta) {
    if (admissible(bmin, bmax, ts.x, ts.y, d, eta)) return 0;
    const int32_t mt = hi[ts.x] - lo[ts.x], ms = hi[ts.y] - lo[ts.y];
    return (mt > leaf && ms > leaf) ? 1 : 2;
}

__global__ __launch_bounds__(kTravThreads) void traverse_count_kernel(
    const int2* __restrict__ cur, int64_t ncur, const int32_t* __restrict__ lo,
    const int32_t* __restrict__ hi, const double* __restrict__ bmin,
    const double* __restrict__ bmax, int d, int leaf, double eta,
    int64_t* __restrict__ block_counts) {
    __shared__ int cnt[3];
    if (threadIdx.x < 3) cnt[threadIdx.x] = 0;
    __syncthreads();
    int c[3] = {0, 0, 0};
    const int64_t base = blockIdx.x * (int64_t)kTravTile + threadIdx.x * (int64_t)kTravItems;
    for (int k = 0; k < kTravItems; ++k)
        if (base + k < ncur) c[classify(cur[base + k], lo, hi, bmin, bmax, d, leaf, eta)]++;
    for (int q = 0; q < 3; ++q) {
        int v = wave_sum(c[q]);
        if ((threadIdx.x & 63) == 0) atomicAdd(&cnt[q], v);  // integer: order-free
    }
    __syncthreads();
    if (threadIdx.x < 3) block_counts[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void traverse_totals_kernel(const int64_t* __restrict__ scanned, int64_t nblk,
                                       const int64_t* __restrict__ grand, int64_t* __restrict__ totals) {
    if (threadIdx.x != 0) return;
    const int64_t b1 = scanned[nblk], b2 = scanned[2 * nblk];
    totals[0] = b1;
    totals[1] = b2 - b1;
    totals[2] = *grand - b2;
}

__global__ __launch_bounds__(kTravThreads) void traverse_write_kernel(
    const int2* __restrict__ cur, int64_t ncur, const int32_t* __restrict__ lo,
    const int32_t* __restrict__ hi, const double* __restrict__ bmin,
    const double* __restrict__ bmax, int d, int leaf, double eta,
    const int64_t* __restrict__ block_off, int level, int2* __restrict__ next,
    int4* __restrict__ adm, int32_t* __restrict__ adm_level, int2* __restrict__ adm_ids,
    int64_t adm_base, int4* __restrict__ dense, int32_t* __restrict__ dense_level,
    int64_t dense_base, const int32_t* __restrict__ slot_base) {
    __shared__ int64_t sh[kScanThreads / 64 + 1];
    const int64_t nblk = gridDim.x;
    const int64_t base = blockIdx.x * (int64_t)kTravTile + threadIdx.x * (int64_t)kTravItems;
    int cls[kTravItems];
    int2 ts[kTravItems];
    int c[3] = {0, 0, 0};
    for (int k = 0; k < kTravItems; ++k) {
        cls[k] = -1;
        if (base + k < ncur) {
            ts[k] = cur[base + k];
            cls[k] = classify(ts[k], lo, hi, bmin, bmax, d, leaf, eta);
            c[cls[k]]++;
        }
    }
    int64_t off[3];
    for (int q = 0; q < 3; ++q) {
        int64_t tot;
        off[q] = block_exclusive_scan<int64_t>((int64_t)c[q], sh, &tot) +
                 block_off[q * nblk + blockIdx.x] - block_off[q * nblk];
    }
    for (int k = 0; k < kTravItems; ++k) {
        if (cls[k] < 0) continue;
        const int64_t t = ts[k].x, s = ts[k].y;
        if (cls[k] == 1) {
            // children 2 i + 1, 2 i + 2 in the node's own tree (whose slots
            // start at slot_base[i]; 0 for a single tree)
            const int64_t t1 = 2 * t + 1 - (slot_base ? slot_base[t] : 0);
            const int64_t s1 = 2 * s + 1 - (slot_base ? slot_base[s] : 0);
            int2* o = next + 4 * off[1];
            o[0] = make_int2((int)t1, (int)s1);
            o[1] = make_int2((int)t1, (int)(s1 + 1));
            o[2] = make_int2((int)(t1 + 1), (int)s1);
            o[3] = make_int2((int)(t1 + 1), (int)(s1 + 1));
            off[1]++;
        } else {
            const int4 r = make_int4(lo[t], hi[t], lo[s], hi[s]);
            if (cls[k] == 0) {
                adm[adm_base + off[0]] = r;
                adm_level[adm_base + off[0]] = level;
                adm_ids[adm_base + off[0]] = ts[k];
                off[0]++;
            } else {
                dense[dense_base + off[2]] = r;
                dense_level[dense_base + off[2]] = level;
                off[2]++;
            }
        }
    }
}

// leaf clusters mark their first point
__global__ void mark_leaves_kernel(int leaf, const int32_t* __restrict__ lo,
                                   const int32_t* __restrict__ hi, int64_t nslots,
                                   int32_t* __restrict__ flags) {
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= nslots) return;
    const int32_t a = lo[id], b = hi[id];
    if (a >= 0 && b - a <= leaf) flags[a] = 1;
}

// after an inclusive scan of the flags: tile of point i = scan[i] - 1;
// the first point of each tile records the tile's start
__global__ void tile_finish_kernel(int32_t* __restrict__ scan_to_tile, int64_t n,
                                   const int32_t* __restrict__ flags_copy,
                                   int32_t* __restrict__ tile_lo) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t t = scan_to_tile[i] - 1;
    scan_to_tile[i] = t;
    if (flags_copy[i]) tile_lo[t] = (int32_t)i;
    if (i == n - 1) tile_lo[t + 1] = (int32_t)n;
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
    return (size_t)(((n + kScanTile - 1) / kScanTile) + 1) * sizeof(int64_t);
}

hipError_t exclusive_scan_i64(int64_t* data, int64_t n, int64_t* total_dev, void* scratch,
                              hipStream_t st) {
    return scan_generic<int64_t>(data, data, n, 0, total_dev, scratch, st);
}

hipError_t launch_tree_level(int level, int64_t n, int leaf, int32_t* node_lo, int32_t* node_hi,
                             hipStream_t st) {
    const int64_t cnt = 1ll << level;
    hipLaunchKernelGGL(tree_level_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st,
                       level, n, leaf, node_lo, node_hi);
    return hipGetLastError();
}

hipError_t launch_box_level(int level, int d, int leaf, const int32_t* node_lo,
                            const int32_t* node_hi, const double* soa, int64_t n, double* bmin,
                            double* bmax, hipStream_t st) {
    const int64_t cnt = 1ll << level;
    const int64_t threads = cnt * 64;
    hipLaunchKernelGGL(box_level_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                       st, level, d, leaf, node_lo, node_hi, soa, n, bmin, bmax);
    return hipGetLastError();
}

int64_t traverse_blocks(int64_t nodes) { return (nodes + kTravTile - 1) / kTravTile; }

size_t traverse_scratch_bytes(int64_t max_nodes) {
    const int64_t nb = traverse_blocks(max_nodes);
    return (size_t)(3 * nb + 8) * sizeof(int64_t) + scan_scratch_bytes(3 * nb + 1) + 256;
}

hipError_t launch_traverse_count(const int2* cur, int64_t ncur, const int32_t* node_lo,
                                 const int32_t* node_hi, const double* bmin, const double* bmax,
                                 int d, int leaf, double eta, int64_t* block_counts,
                                 hipStream_t st) {
    const int64_t nb = traverse_blocks(ncur);
    hipLaunchKernelGGL(traverse_count_kernel, dim3((unsigned)nb), dim3(kTravThreads), 0, st, cur,
                       ncur, node_lo, node_hi, bmin, bmax, d, leaf, eta, block_counts);
    return hipGetLastError();
}

// block_counts holds 3*nblk counts followed by scratch: scan them and
// produce per-class totals
hipError_t launch_traverse_scan(int64_t* block_counts, int64_t nblk, int64_t* totals,
                                hipStream_t st) {
    int64_t* grand = totals + 3;
    void* sscr = (void*)(block_counts + 3 * nblk + 8);
    // one extra element so scanned[3 nblk] exists: write 0 there first
    hipError_t e = hipMemsetAsync(block_counts + 3 * nblk, 0, sizeof(int64_t), st);
    if (e != hipSuccess) return e;
    e = exclusive_scan_i64(block_counts, 3 * nblk + 1, grand, sscr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(traverse_totals_kernel, dim3(1), dim3(64), 0, st, block_counts, nblk,
                       grand, totals);
    return hipGetLastError();
}

hipError_t launch_traverse_write(const int2* cur, int64_t ncur, const int32_t* node_lo,
                                 const int32_t* node_hi, const double* bmin, const double* bmax,
                                 int d, int leaf, double eta, const int64_t* block_offsets,
                                 int level, int2* next, int4* adm, int32_t* adm_level,
                                 int2* adm_ids, int64_t adm_base, int4* dense,
                                 int32_t* dense_level, int64_t dense_base,
                                 const int32_t* slot_base, hipStream_t st) {
    const int64_t nb = traverse_blocks(ncur);
    hipLaunchKernelGGL(traverse_write_kernel, dim3((unsigned)nb), dim3(kTravThreads), 0, st, cur,
                       ncur, node_lo, node_hi, bmin, bmax, d, leaf, eta, block_offsets, level,
                       next, adm, adm_level, adm_ids, adm_base, dense, dense_level, dense_base,
                       slot_base);
    return hipGetLastError();
}

hipError_t launch_forest_tree_level(int level, int np, const int64_t* pbase, const int64_t* nbase,
                                    const int32_t* depth, int leaf, int32_t* node_lo,
                                    int32_t* node_hi, hipStream_t st) {
    const int64_t cnt = 1ll << level;
    hipLaunchKernelGGL(forest_tree_level_kernel, dim3((unsigned)((cnt + 255) / 256), np),
                       dim3(256), 0, st, level, pbase, nbase, depth, leaf, node_lo, node_hi);
    return hipGetLastError();
}

hipError_t launch_forest_box_level(int level, int np, const int64_t* nbase, const int32_t* depth,
                                   int leaf, const int32_t* node_lo, const int32_t* node_hi,
                                   const double* soa, int64_t N, double* bmin, double* bmax,
                                   hipStream_t st) {
    const int64_t threads = (1ll << level) * 64;
    hipLaunchKernelGGL(forest_box_level_kernel, dim3((unsigned)((threads + 255) / 256), np),
                       dim3(256), 0, st, level, nbase, depth, leaf, node_lo, node_hi, soa, N, bmin,
                       bmax);
    return hipGetLastError();
}

hipError_t launch_forest_slot_base(const int64_t* nbase, int np, int64_t nslots, int32_t* base,
                                   hipStream_t st) {
    if (nslots == 0) return hipSuccess;
    hipLaunchKernelGGL(forest_slot_base_kernel, dim3((unsigned)((nslots + 255) / 256)), dim3(256),
                       0, st, nbase, np, nslots, base);
    return hipGetLastError();
}

hipError_t launch_mark_leaves(int L, int leaf, const int32_t* node_lo, const int32_t* node_hi,
                              int64_t nslots, int32_t* flags, hipStream_t st) {
    (void)L;
    hipLaunchKernelGGL(mark_leaves_kernel, dim3((unsigned)((nslots + 255) / 256)), dim3(256), 0,
                       st, leaf, node_lo, node_hi, nslots, flags);
    return hipGetLastError();
}

size_t tile_scan_scratch_bytes(int64_t n) { return scan_scratch_bytes(n) + (size_t)n * 4 + 256; }

// flags_to_tile: in = leaf-start flags (0/1) over n points; out = tile id of
// every point.  tile_lo gets ntiles + 1 entries (tile starts and n).
hipError_t launch_iota_scan_tiles(int32_t* flags_to_tile, int64_t n, int32_t* tile_lo,
                                  int64_t* ntiles_dev, void* scratch, hipStream_t st) {
    int32_t* flags_copy = (int32_t*)scratch;
    void* sscr = (void*)((char*)scratch + (((size_t)n * 4 + 255) & ~(size_t)255));
    hipError_t e =
        hipMemcpyAsync(flags_copy, flags_to_tile, n * 4, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    e = scan_generic<int32_t>(flags_to_tile, flags_to_tile, n, 1, ntiles_dev, sscr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tile_finish_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       flags_to_tile, n, flags_copy, tile_lo);
    return hipGetLastError();
}

}  // namespace hmx
