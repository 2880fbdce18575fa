// Internal declarations shared by the HIP translation units of libhmx.
// Device helpers (kernel functions, reductions) and the host-side launchers
// each .hip file exports to the orchestration in hmx_api.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "../../include/hmx.h"

namespace hmx {

constexpr int kMaxRankCap = 128;  // largest supported k_max
constexpr int kWave = 64;         // CDNA wavefront width

struct KernelFn {
    int kind;
    double p0;
    double norm = 1.0;  // HMX_MATERN_NU1: 1 / (2^(beta-1) Gamma(beta)), beta = 1 + d/2
};

// ---------------------------------------------------------------------------
// kernel functions phi(x, y) (matrix entries of eq. (2)); T = float or double
// ---------------------------------------------------------------------------
template <typename T>
struct KernelEval {
    int kind;
    T inv_p0;   // 1 / p0
    T s3_inv;   // sqrt(3) / p0 (Matern-3/2)
    T norm;     // Matern nu = 1 normalisation
    __host__ __device__ KernelEval() {}
    __host__ KernelEval(const KernelFn& k)
        : kind(k.kind),
          inv_p0((T)(1.0 / k.p0)),
          s3_inv((T)(1.7320508075688772 / k.p0)),
          norm((T)k.norm) {}
};

__device__ __forceinline__ float kexp(float a) { return __expf(a); }
__device__ __forceinline__ double kexp(double a) { return exp(a); }
__device__ __forceinline__ float ksqrt(float a) { return __fsqrt_rn(a); }
__device__ __forceinline__ double ksqrt(double a) { return sqrt(a); }
__device__ __forceinline__ float klog(float a) { return __logf(a); }
__device__ __forceinline__ double klog(double a) { return log(a); }

// s K_1(s), K_1 the modified Bessel function of the second kind of order 1
// (the Matern kernel of the model problem, Section 6.2, with
// beta - d/2 = 1); the limit 1 at s = 0.
//  * s <= 2: the power series of K_1 (Abramowitz & Stegun 9.6.11) in
//    q = s^2/4:  s K_1(s) = 1 + 2 q ln(s/2) sum_k a_k - q sum_k c_k a_k with
//    a_k = q^k / (k! (k+1)!), c_k = psi(k+1) + psi(k+2), truncated where a_k
//    drops below the type's rounding at q = 1 (12 terms FP64, 7 FP32).
//  * s > 2: K_1(s) = int_0^inf exp(-s cosh t) cosh t dt (A&S 9.6.24) with
//    the substitution w = 2 sqrt(s) sinh(t/2), which turns the integrand
//    into a Gaussian times a smooth factor:
//      s K_1(s) = s e^-s int_0^inf e^(-w^2/2) (1 + w^2/(2s)) 2 / sqrt(4s + w^2) dw,
//    summed by the trapezoidal rule on w = k h (the factor is analytic for
//    |Im w| < 2 sqrt(s), so the rule converges geometrically): h = 0.45 and
//    20 nodes for FP64, h = 0.8 and 8 nodes for FP32.  The node weights
//    exp(-(k h)^2 / 2) are the literals below.
struct K1Nodes64 {
    static constexpr double h = 0.45;
    static constexpr int n = 20;
};
struct K1Nodes32 {
    static constexpr float h = 0.8f;
    static constexpr int n = 8;
};
__device__ __forceinline__ double k1_node(const K1Nodes64&, int k) {
    constexpr double w[20] = {
        0.90370707787319604,   0.66697681085847438,   0.40202138309465485,
        0.19789869908361465,   0.079559508718227687,  0.026121409853918223,
        0.0070041671493624221, 0.001533810679324463,  0.00027431046749340119,
        4.0065297392951069e-05, 4.7791397322046383e-06, 4.6557157157830781e-07,
        3.7040645507943341e-08, 2.406722436301052e-09, 1.2771115545128334e-10,
        5.5346100717010135e-12, 1.9588473410004431e-13, 5.6619955169489504e-15,
        1.3365764918318395e-16, 2.576757109154981e-18};
    return w[k];
}
__device__ __forceinline__ float k1_node(const K1Nodes32&, int k) {
    constexpr float w[8] = {0.72614902f, 0.27803731f, 0.056134764f, 0.0059760227f,
                            0.00033546262f, 9.9295039e-06f, 1.5497531e-07f, 1.2754077e-09f};
    return w[k];
}

template <typename T>
__device__ __forceinline__ T xk1(T s) {
    using Nodes = typename std::conditional<sizeof(T) == 8, K1Nodes64, K1Nodes32>::type;
    if (s <= (T)2) {
        constexpr int nt = sizeof(T) == 8 ? 12 : 7;
        const T q = (T)0.25 * s * s;
        T a = (T)1, s1 = (T)0, s2 = (T)0;
        T c = (T)(1.0 - 2.0 * 0.57721566490153286061);  // psi(1) + psi(2)
#pragma unroll
        for (int k = 0; k < nt; ++k) {
            s1 += a;
            s2 += c * a;
            a = a * q * (T)(1.0 / ((k + 1.0) * (k + 2.0)));
            c += (T)(1.0 / (k + 1.0) + 1.0 / (k + 2.0));
        }
        // q ln(s/2) is 0 * -inf at s = 0: the limit there is 1
        return s > (T)0 ? (T)1 + (T)2 * q * klog((T)0.5 * s) * s1 - q * s2 : (T)1;
    }
    const T four_s = (T)4 * s, inv_2s = (T)1 / ((T)2 * s);
    T acc = (T)1 / ksqrt(four_s);  // the w = 0 node, halved
#pragma unroll
    for (int k = 1; k <= Nodes::n; ++k) {
        const T w = (T)k * Nodes::h;
        const T w2 = w * w;
        acc += k1_node(Nodes{}, k - 1) * ((T)1 + w2 * inv_2s) * ((T)2 / ksqrt(four_s + w2));
    }
    return s * kexp(-s) * Nodes::h * acc;
}

// phi for points x (d coords) and y (d coords)
template <typename T>
__device__ __forceinline__ T phi(const KernelEval<T>& K, const T* x, const T* y, int d) {
    T r2 = 0, dot = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (k < d) {
            T t = x[k] - y[k];
            r2 += t * t;
            dot += x[k] * y[k];
        }
    switch (K.kind) {
        case HMX_GAUSSIAN:
            return kexp(-r2 * K.inv_p0);
        case HMX_MATERN32: {
            T s = ksqrt(r2) * K.s3_inv;
            return ((T)1 + s) * kexp(-s);
        }
        case HMX_MATERN_NU1:
            return K.norm * xk1(ksqrt(r2) * K.inv_p0);
        case HMX_TEST_CONST:
            return (T)1;
        default: {  // HMX_TEST_LOWRANK
            T u = (T)1 + dot;
            return u * u;
        }
    }
}

// phi for a fixed kernel kind, coordinates padded to three with zeros (the
// padding adds exact zeros, so the value equals phi's)
template <int KIND, typename T>
__device__ __forceinline__ T phi_kind(const KernelEval<T>& K, const T* x, const T* y) {
    T r2 = 0, dot = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T t = x[k] - y[k];
        r2 += t * t;
        if constexpr (KIND == HMX_TEST_LOWRANK) dot += x[k] * y[k];
    }
    if constexpr (KIND == HMX_GAUSSIAN) {
        return kexp(-r2 * K.inv_p0);
    } else if constexpr (KIND == HMX_MATERN32) {
        T s = ksqrt(r2) * K.s3_inv;
        return ((T)1 + s) * kexp(-s);
    } else if constexpr (KIND == HMX_MATERN_NU1) {
        return K.norm * xk1(ksqrt(r2) * K.inv_p0);
    } else if constexpr (KIND == HMX_TEST_CONST) {
        (void)r2;
        return (T)1;
    } else {
        T u = (T)1 + dot;
        return u * u;
    }
}

// many problems in one union index space (batched builds): problem p owns
// [pbase[p], pbase[p + 1]); the problem of index i (binary search, np small)
__device__ __forceinline__ int problem_of(const int64_t* __restrict__ pbase, int np, int64_t i) {
    int lo = 0, hi = np;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pbase[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// a problem's input points (device, n_p x d row-major, the build's dtype)
struct ForestInput {
    const void* pts;
    int32_t d;
};

// load point i of a d x n SoA array
template <typename T>
__device__ __forceinline__ void load_pt(const T* __restrict__ soa, int64_t n, int d, int64_t i,
                                        T* p) {
#pragma unroll
    for (int k = 0; k < 3; ++k) p[k] = (k < d) ? soa[(int64_t)k * n + i] : (T)0;
}

// ---------------------------------------------------------------------------
// wave / block reductions (wave64)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------
// launchers (host side); every launcher enqueues on `st` and returns
// hipSuccess or the launch error
// ---------------------------------------------------------------------------
// ordering (k_order.hip)
hipError_t launch_global_box(const void* pts, int pts_f64, int64_t n, int d, double* partial,
                             int nparts, double* box /*2d: lo then hi*/, hipStream_t st);
int global_box_parts(int64_t n);
hipError_t launch_morton(const void* pts, int pts_f64, int64_t n, int d, const double* box,
                         uint64_t* codes, uint32_t* idx, hipStream_t st);
// many problems at once (batched builds): the union points as N x 3 FP64,
// per-problem boxes (6 doubles each: lo[3], hi[3]), Morton codes of every
// point in its problem's box, the problem key of each sorted point, a gather
hipError_t launch_forest_points(const ForestInput* in, int np, const int64_t* pbase, int64_t N,
                                int f64, double* P, hipStream_t st);
int forest_box_parts();
hipError_t launch_forest_box(const double* P, int np, const int64_t* pbase, const int32_t* dims,
                             double* partial /*np x forest_box_parts() x 6*/, double* box,
                             hipStream_t st);
hipError_t launch_forest_morton(const double* P, int64_t N, int np, const int64_t* pbase,
                                const int32_t* dims, const double* box, uint64_t* codes,
                                uint32_t* idx, hipStream_t st);
hipError_t launch_forest_problem_keys(const uint32_t* idx, int64_t N, int np,
                                      const int64_t* pbase, uint64_t* keys, hipStream_t st);
hipError_t launch_gather_u64(const uint64_t* src, const uint32_t* idx, int64_t n, uint64_t* dst,
                             hipStream_t st);
// stable LSD radix sort of (key, value) pairs on the low `bits` key bits;
// scratch from radix_sort_scratch_bytes; results end in keys/vals
size_t radix_sort_scratch_bytes(int64_t n);
hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, int64_t n, int bits, void* scratch,
                            hipStream_t st);
hipError_t launch_gather_coords(const void* pts, int pts_f64, int64_t n, int d,
                                const uint32_t* perm, double* soa64, float* soa32,
                                hipStream_t st);

// scans (k_tree.hip): exclusive scan of n int64 values in place; total to *total_dev
size_t scan_scratch_bytes(int64_t n);
hipError_t exclusive_scan_i64(int64_t* data, int64_t n, int64_t* total_dev, void* scratch,
                              hipStream_t st);

// cluster tree and traversal (k_tree.hip)
hipError_t launch_tree_level(int level, int64_t n, int leaf, int32_t* node_lo, int32_t* node_hi,
                             hipStream_t st);
hipError_t launch_box_level(int level, int d, int leaf, const int32_t* node_lo,
                            const int32_t* node_hi, const double* soa, int64_t n, double* bmin,
                            double* bmax, hipStream_t st);
// traversal of one block-tree level: classify (t, s) pairs, write children of
// split nodes to next (4 per split node) and leaves to adm/dense (as
// int4 ranges + level) at the given bases; counts_dev[0..2] = (#adm, #split,
// #dense) of this level.  Two phases: count, then write.
size_t traverse_scratch_bytes(int64_t max_nodes);
int64_t traverse_blocks(int64_t nodes);
hipError_t launch_traverse_count(const int2* cur, int64_t ncur, const int32_t* node_lo,
                                 const int32_t* node_hi, const double* bmin, const double* bmax,
                                 int d, int leaf, double eta, int64_t* block_counts,
                                 hipStream_t st);
hipError_t launch_traverse_scan(int64_t* block_counts, int64_t nblk, int64_t* totals,
                                hipStream_t st);
hipError_t launch_traverse_write(const int2* cur, int64_t ncur, const int32_t* node_lo,
                                 const int32_t* node_hi, const double* bmin, const double* bmax,
                                 int d, int leaf, double eta, const int64_t* block_offsets,
                                 int level, int2* next, int4* adm, int32_t* adm_level,
                                 int2* adm_ids, int64_t adm_base, int4* dense,
                                 int32_t* dense_level, int64_t dense_base,
                                 const int32_t* slot_base /*null: one tree*/, hipStream_t st);
// the forest of a batched build: problem p's tree in slots [nbase[p],
// nbase[p + 1]) (heap-indexed from nbase[p]), depth[p] its deepest level
hipError_t launch_forest_tree_level(int level, int np, const int64_t* pbase, const int64_t* nbase,
                                    const int32_t* depth, int leaf, int32_t* node_lo,
                                    int32_t* node_hi, hipStream_t st);
hipError_t launch_forest_box_level(int level, int np, const int64_t* nbase, const int32_t* depth,
                                   int leaf, const int32_t* node_lo, const int32_t* node_hi,
                                   const double* soa, int64_t N, double* bmin, double* bmax,
                                   hipStream_t st);
hipError_t launch_forest_slot_base(const int64_t* nbase, int np, int64_t nslots, int32_t* base,
                                   hipStream_t st);

// leaf tiles (k_tree.hip): tile_of_point via leaf-start flags and a scan
hipError_t launch_mark_leaves(int L, int leaf, const int32_t* node_lo, const int32_t* node_hi,
                              int64_t nslots, int32_t* flags, hipStream_t st);
hipError_t launch_iota_scan_tiles(int32_t* flags_to_tile, int64_t n, int32_t* tile_lo,
                                  int64_t* ntiles_dev, void* scratch, hipStream_t st);
size_t tile_scan_scratch_bytes(int64_t n);

// ACA (k_aca.hip)
struct AcaArgs {
    const void* soa;      // d x n compute-type coords
    const double* soa64;  // d x n FP64 coords (first-column choice)
    int64_t n;
    int d;
    KernelFn kern;
    const int4* blocks;
    int64_t nblocks;
    const int64_t* uoff;  // per block, capacity offsets (entries)
    const int64_t* voff;
    int64_t ubase, vbase; // subtracted from uoff / voff (offset of the chunk's first block)
    int kmax;
    double eps, aca_eta, eps0;
    int fixed;
    const int32_t* rtarget;  // per-block target ranks, or null (adaptive)
    int one_shot;            // targets are run without the test, then judged by it
    int cap_only;            // storage holds only the target: unfinished blocks get rank -1
    // with cap_only, a block that reaches its target unfinished takes k_max
    // columns of overflow storage (one request on *ovf_used, in entries of
    // both U and V) and continues; ovf_moved[b] (preset to -1) receives the
    // offset granted, and launch_apply_moved moves the block's uoff / voff
    // there.  Overflow regions: uoff ovf_u0 / voff ovf_v0 onwards, ovf_cap
    // entries each.  ovf_used null: no overflow (rank -1 instead).
    unsigned long long* ovf_used;
    int64_t ovf_cap, ovf_u0, ovf_v0;
    int64_t* ovf_moved;
    void* U;
    void* V;
    int32_t* rank;
    int32_t* steps;
    // size classes of the level-ordered list: [0, nsplit) many workgroups per
    // block, [nsplit, nbig) 512-thread workgroups, [nbig, nmed) 256-thread
    // ones, the rest (leaf levels) single-wave ones; each single-workgroup
    // class reserves the used-row + used-col bitmask words of its largest block
    int64_t nsplit, nbig, nmed;
    int big_words, med_words, tiny_words;
};
// queue the single-workgroup classes on aux[0..2] (3 streams, or null: all on
// st) after the work queued on st; join makes st wait for them
// chunking the ACA's level-ordered block list into slices that each hold a
// share of every level (k_batch.hip): level bounds of a level-sorted list
// (lstart/lend preset to zero, 64 entries each), interleave keys for a stable
// sort, and the gather of blocks, levels and two optional int32 arrays
hipError_t launch_level_bounds(const int32_t* level, int64_t nb, int64_t* lstart, int64_t* lend,
                               hipStream_t st);
hipError_t launch_interleave_keys(const int32_t* level, int64_t nb, const int64_t* lstart,
                                  const int64_t* lend, int nch, uint64_t* keys, uint32_t* vals,
                                  hipStream_t st);
hipError_t launch_gather_blocks(const uint32_t* perm, int64_t n, const int4* blocks,
                                const int32_t* level, const int32_t* a, const int32_t* b,
                                int4* blocks_out, int32_t* level_out, int32_t* a_out,
                                int32_t* b_out, hipStream_t st);
hipError_t launch_apply_moved(const int64_t* moved, int64_t nb, int64_t u0, int64_t v0,
                              int64_t* uoff, int64_t* voff, hipStream_t st);
hipError_t aca_classes_begin(const AcaArgs& a, int f64, hipStream_t st, const hipStream_t* aux);
hipError_t aca_classes_join(hipStream_t st, const hipStream_t* aux);

// multi-workgroup ACA of blocks [0, nblocks) of an AcaArgs list (k_aca_split.hip)
struct SplitPlan {
    int64_t nblocks, nrowtiles, ncoltiles;
    const int2* rowtiles;  // (block, tile) per row tile of split_tile() rows
    const int2* coltiles;  // (block, tile) per column tile
    const int64_t* rtoff;  // first row tile of each block (nblocks + 1)
    const int64_t* ctoff;  // first column tile of each block (nblocks + 1)
    const int64_t* moff;   // first bitmask word of each block
    uint32_t* masks;       // used rows then used columns, per block
    void* state;           // nblocks x split_state_bytes()
    void* colpart;         // nrowtiles x split_colpart_bytes()
    void* rowpart;         // ncoltiles x split_rowpart_bytes()
    void* urow;            // nblocks x (kMaxRankCap + 1) compute-type values
    double* udpart;        // nrowtiles x (kMaxRankCap + 1)
    double* vdpart;        // ncoltiles x (kMaxRankCap + 1)
    int* active_dev;       // one int
    int* active_host;      // one int in pinned host memory (the poll's target)
};
size_t split_state_bytes();
size_t split_colpart_bytes(int f64);
size_t split_rowpart_bytes(int f64);
int split_tile();
hipError_t launch_aca_split(const AcaArgs& a, const SplitPlan& p, int f64, hipStream_t st);
// *out = first index with level[index] >= lvl in the non-decreasing level[0..nb)
hipError_t launch_level_split(const int32_t* level, int64_t nb, int lvl, int64_t* out,
                              hipStream_t st);

// near field and matvec (k_mvp.hip)
// A piece is the part of one leaf block inside one row tile (leaf cluster);
// the matrix pool stores the pieces of each tile contiguously (tile-major).
struct Piece {
    int64_t d_off;  // element offset of the piece in the matrix pool
    int64_t v_off;  // element offset of its weights in the vector pool
    int32_t blk;    // admissible leaf b >= 0 (factor piece), or -(dense leaf + 1)
    int32_t tile;
    int32_t ncols;
    int32_t row0;   // first row of the tile inside the block's tau
};
// per-block sizes: mode 0: m * mult, 1: n * mult, 2: m * n, 3: r * m, 4: r * n,
// 5: r, 6: row tiles covered by tau (0 for an admissible leaf of rank 0),
// 7: (m + n) * mult, 8: (m + n) * r; negative ranks count as 0 in 3, 4, 5
hipError_t launch_extent(const int4* blocks, int64_t nb, int mode, int64_t mult,
                         const int32_t* rank, const int32_t* tile_of_point, int64_t* out,
                         hipStream_t st);
hipError_t launch_piece_fill(const int4* blocks, int64_t nblocks, const int32_t* rank,
                             const int32_t* tile_of_point, const int32_t* tile_lo,
                             const int64_t* piece_off, const int64_t* toff, int64_t vec_base,
                             int64_t piece_base, Piece* pieces, uint64_t* keys, uint32_t* vals,
                             hipStream_t st);
hipError_t launch_piece_gather(const Piece* src, const uint32_t* order, int64_t npieces,
                               Piece* dst, int64_t* size_u, int64_t* size_n, int64_t* cols,
                               int64_t* cols_u, const int32_t* tile_lo, int R, int near_stored,
                               hipStream_t st);
hipError_t launch_piece_layout(Piece* pieces, int64_t np, const int64_t* doff_u,
                               const int64_t* doff_n, const int64_t* coff, int64_t* widx,
                               hipStream_t st);
hipError_t launch_tile_offsets(const uint64_t* sorted_tile, int64_t npieces, int64_t ntiles,
                               int64_t* tile_ptr, hipStream_t st);
// meta[4 t + 0..3] = first column, first factor column, factor-pool and
// near-pool data offsets of tile t (t = 0..ntiles; entry ntiles = totals)
hipError_t launch_tile_meta(const int64_t* tile_ptr, int64_t ntiles, int64_t np,
                            const int64_t* coff, const int64_t* coff_u, const int64_t* doff_u,
                            const int64_t* doff_n, int64_t* meta, hipStream_t st);
// rows per 16-byte lane unit for the factor / near storage modes (0 F64, 1 F32, 2 BF16)
int rows_per_unit(int fmode, int nmode);
hipError_t launch_piece_data(const Piece* pieces, int64_t np, const int32_t* tile_lo,
                             const int4* adm, const int4* dense, const int64_t* uoff,
                             const void* Usrc /* storage type */, const void* soa, int64_t n,
                             int d, KernelFn kern,
                             void* upool, void* npool, int fmode, int nmode,
                             int which /*0 all, 1 factor pieces, 2 near-field pieces*/,
                             hipStream_t st);
// smode: storage mode 0 = F64, 1 = F32, 2 = BF16 storage with F32 arithmetic
hipError_t launch_compact_v(const int4* blocks, int64_t nblocks, const int32_t* rank,
                            const int64_t* cap_voff, int64_t cap_base, const int64_t* voff,
                            const void* Vcap, void* V, int smode, hipStream_t st);
// xm[i] = x[perm[i] - base] for i < n (base: the first column's index in
// the union of a rectangular handle's two point sets, else 0)
hipError_t launch_gather_x(const void* x, const int32_t* perm, int64_t n, void* xm, int f64,
                           hipStream_t st, int64_t base = 0);
// data[i] += c for i < n
hipError_t launch_add_const(int64_t* data, int64_t n, int64_t c, hipStream_t st);
// U compaction into the exact per-block pool (compute type)
hipError_t launch_compact_u(const int4* blocks, int64_t nblocks, const int32_t* rank,
                            const int64_t* cap_uoff, int64_t cap_base, const int64_t* uoff,
                            const void* Ucap, void* U, int smode, hipStream_t st);
// chunk boundaries: bnd[k] = first block whose capacity offset is >= k * step
hipError_t launch_chunk_bounds(const int64_t* cap_off, int64_t nb, int64_t step, int nchunks,
                               int64_t* bnd, hipStream_t st);
// out[0] = max and out[1] = sum of n non-negative int32 values (device)
// out[0] = sum over blocks of steps m + rank n (ACA kernel evaluations),
// out[1] = sum of 2 rank (rank - 1) (m + n) (update and inner-product flops)
hipError_t launch_aca_work(const int4* blocks, const int32_t* rank, const int32_t* steps,
                           int64_t nb, unsigned long long* out, hipStream_t st);
hipError_t launch_int_stats(const int32_t* a, int64_t n, unsigned long long* out,
                            hipStream_t st);
// config < 0: default tile shape; config < 15: shape config % 5 of the first
// five, grid config / 5; config 15-17: shape 5 (8 lanes per row group), grid
// config - 15.  Grids: one workgroup per tile, a persistent grid of
// kPersistentGrid workgroups, or one workgroup per (tile, row pass)
constexpr int kRowtileShapes = 6;
constexpr int kRowtileConfigs = 3 * kRowtileShapes;
constexpr unsigned kPersistentGrid = 2048;
// nmode 3: near field recomputed from soa (compute type, d x n) with kern
hipError_t launch_rowtile(int64_t ntiles, const int32_t* tile_lo, const int64_t* meta,
                          const int64_t* widx, const void* upool, const void* npool,
                          const void* vecpool, const int32_t* perm, double alpha, double beta,
                          double sigma2, void* z, int max_tile, int fmode, int nmode, int config,
                          const void* soa, int64_t n, int d, KernelFn kern, hipStream_t st);

// conjugate gradients (k_blas.hip): FP64-accumulated inner products
size_t cg_scratch_bytes();
hipError_t launch_dot(const void* a, const void* b, int64_t n, int f64, double* partial,
                      double* out, hipStream_t st);
// x += alpha p, r -= alpha q with alpha = scal[0] / scal[1]; *out = r.r
hipError_t launch_cg_update(void* x, void* r, const void* p, const void* q, const double* scal,
                            int64_t n, int f64, double* partial, double* out, hipStream_t st);
// p = r + (scal[2] / scal[0]) p
hipError_t launch_cg_direction(void* p, const void* r, const double* scal, int64_t n, int f64,
                               hipStream_t st);
hipError_t launch_copy(void* dst, const void* src, int64_t n, int f64, hipStream_t st);
hipError_t launch_fill_zero(void* dst, int64_t n, int f64, hipStream_t st);
hipError_t launch_sub(void* out, const void* a, const void* b, int64_t n, int f64,
                      hipStream_t st);


// learned rank sizing (k_mlp.hip): MLP 8 -> 64 -> 64 -> 64 -> 1 (ReLU), FP32
int64_t mlp_nparams();
size_t mlp_grad_scratch_floats(int64_t B);
// act: B * (3 * 64 + 1) floats (hidden activations, then the outputs)
hipError_t mlp_forward(const float* w, const float* mean, const float* scale, const float* X,
                       int64_t B, float* act, hipStream_t st);
hipError_t mlp_backward(const float* w, const float* mean, const float* scale, const float* X,
                        const float* y, int64_t B, float q, const float* act, float* grad,
                        float* scratch, double* loss, hipStream_t st);
hipError_t mlp_adam(float* w, float* m, float* v, const float* g, int64_t t, float lr, float b1,
                    float b2, float eps, hipStream_t st);
hipError_t mlp_norm(const float* X, int64_t n, float* mean, float* scale, hipStream_t st);
hipError_t mlp_gather_batch(const float* X, const float* y, int64_t n, const int64_t* idx,
                            int64_t B, float* Xb, float* yb, hipStream_t st);
hipError_t launch_features(const int4* blocks, const int2* ids, int64_t nb, const double* bmin,
                           const double* bmax, int d, double ell, const int32_t* rank, float* F,
                           float* y, hipStream_t st);
hipError_t launch_rank_predict(const int4* blocks, const int2* ids, int64_t nb, const double* bmin,
                               const double* bmax, int d, double ell, const float* w,
                               const float* mean, const float* scale, int kmax, float* pred,
                               int32_t* target, hipStream_t st, const int64_t* pbase = nullptr,
                               int np = 0, const double* ell_p = nullptr,
                               const int32_t* dim_p = nullptr);
// fallback lists: flag[b] = rank[b] < 0 (int64, scanned by the caller into
// positions pos), then the flagged blocks gathered in order
hipError_t launch_fail_flags(const int32_t* rank, int64_t nb, int64_t* flag, hipStream_t st);
// flag[b] = 1 where rank[b] > rt[b] > 0 (the block outgrew its target)
hipError_t launch_over_flags(const int32_t* rank, const int32_t* rt, int64_t nb, int64_t* flag,
                             hipStream_t st);
hipError_t launch_gather_failed(const int32_t* rank, const int64_t* pos, int64_t nb,
                                const int4* blocks, const int32_t* level, const int32_t* rt,
                                int32_t* list, int4* blocks_out, int32_t* level_out,
                                int32_t* rt_out, hipStream_t st);
// dst[list[i]] = src[i] (i32 / i64), or += for add != 0 (i32)
hipError_t launch_scatter_i32(const int32_t* list, int64_t nl, const int32_t* src, int32_t* dst,
                              int add, hipStream_t st);
hipError_t launch_scatter_i64(const int32_t* list, int64_t nl, const int64_t* src, int64_t* dst,
                              hipStream_t st);

// far-field phase 1 by row tiles and the symmetric far field (k_phase1.hip)
// tile pass: partial[pbase + c] for every source column c of every tile
// (meta[ms t + 1]: first source column of tile t, meta[ms t + 2]: its data
// offset in pool; tiles padded to multiples of R rows)
hipError_t launch_p1_tile(int64_t ntiles, const int32_t* tile_lo, const int64_t* meta, int ms,
                          int R, int max_tile, const void* pool, const void* vec, void* partial,
                          int64_t pbase, int smode, int lanes /*8, 16, 32, 64; 0 = by tile height*/,
                          hipStream_t st);
// t entries: vec[n + k] = sum over j < rec[k].nt of partial[pfc[base + j] + l]
hipError_t launch_p1_reduce(const int4* rec, int64_t ncols, const int64_t* pfc,
                            const void* partial, void* vec, int64_t n, int f64, hipStream_t st);
hipError_t launch_p1_rec(const int32_t* rank, const int64_t* toff, const int64_t* sbase,
                         const int32_t* snt, int64_t nadm, int4* rec, hipStream_t st);
hipError_t launch_p1_source(int64_t nadm, const int32_t* partner, const int64_t* cnt,
                            const int64_t* cntv, int64_t vbase, int64_t* sbase, int32_t* snt,
                            hipStream_t st);
hipError_t launch_pfc(const Piece* sorted, const uint32_t* order, const int64_t* colscan,
                      int64_t np, int64_t limit, int64_t cbase, int64_t* pfc, hipStream_t st);
// mirror table of the admissible leaves (keys/vals: sort scratch of nadm)
hipError_t launch_mirror_keys(const int4* adm, int64_t nadm, uint64_t* keys, uint32_t* vals,
                              hipStream_t st);
hipError_t launch_mirror_find(const int4* adm, int64_t nadm, const uint64_t* keys,
                              const uint32_t* vals, int32_t* partner, int* bad, hipStream_t st);
hipError_t launch_primary_flags(const int4* adm, int64_t nadm, int sym, int64_t* flag,
                                hipStream_t st);
hipError_t launch_gather_list(const int64_t* pos, int64_t nadm, const int4* adm,
                              const int32_t* level, const int32_t* rt, int32_t* list,
                              int4* blocks, int32_t* lev, int32_t* rt_out, hipStream_t st);
// list null: entry i is leaf i; partner null: no mirrors
hipError_t launch_scatter_list(const int32_t* list, int64_t nl, const int32_t* partner,
                               const int32_t* rank_l, const int32_t* steps_l, const int64_t* ue,
                               const int64_t* ve, int32_t* rank, int32_t* steps, int64_t* rfo,
                               int64_t* vfo, hipStream_t st);
// the V pool: pieces of V_b rows per row tile of sigma_b (partner null: every
// leaf, else the leaves that are their own mirror)
hipError_t launch_vpiece_count(const int4* adm, int64_t nadm, const int32_t* rank,
                               const int32_t* partner, const int32_t* tile_of_point, int64_t* cnt,
                               hipStream_t st);
hipError_t launch_vpiece_fill(const int4* adm, int64_t nadm, const int32_t* rank,
                              const int64_t* cnt, const int32_t* tile_of_point,
                              const int32_t* tile_lo, Piece* pieces, uint64_t* keys,
                              uint32_t* vals, hipStream_t st);
hipError_t launch_vpiece_sizes(const Piece* src, const uint32_t* order, int64_t np, Piece* dst,
                               const int32_t* tile_lo, int R, int64_t* size, int64_t* cols,
                               hipStream_t st);
hipError_t launch_vpiece_layout(Piece* pieces, int64_t np, const int64_t* doff, hipStream_t st);
hipError_t launch_vpiece_data(const Piece* pieces, int64_t np, const int32_t* tile_lo,
                              const int4* adm, const int64_t* vfo, const void* src, int R,
                              void* pool, int smode, hipStream_t st);

// batched build assembly (k_batch.hip)
hipError_t launch_add_i32(int32_t* dst, const int32_t* src, int64_t cnt, int32_t c,
                          hipStream_t st);
hipError_t launch_shift_blocks(int4* dst, const int4* src, int64_t cnt, int32_t base,
                               hipStream_t st);
hipError_t launch_fill_i32(int32_t* dst, int64_t cnt, int32_t v, hipStream_t st);
hipError_t launch_forest_scale(const double* src, int64_t N, int np, const int64_t* pbase,
                               const double* inv_ell, double* dst64, float* dst32, hipStream_t st);
hipError_t launch_forest_class(const int4* adm, const int32_t* level, int64_t nadm, int np,
                               const int64_t* pbase, const int4* cuts, uint64_t* keys,
                               uint32_t* vals, hipStream_t st);
hipError_t launch_max_side(const int4* adm, int64_t nadm, int* out, hipStream_t st);
hipError_t launch_narrow_u64(const uint64_t* src, int64_t n, int32_t* dst, hipStream_t st);
hipError_t launch_scale_coords(const double* src, int64_t n, int d, double scale, double* dst64,
                               float* dst32, int64_t ntot, int64_t base, hipStream_t st);

// the far field without precomputation (k_np.hip): the ACA list's pieces
// (block, side) per (chunk, row tile), and per chunk of a matvec t_b = V_b^T x
// (t'_b = U_b^T x for mirrored primaries) and z|tile += alpha F_b t_b
hipError_t launch_np_iota(int32_t* a, int64_t n, hipStream_t st);
hipError_t launch_np_piece_count(const int4* blk, int64_t nl, int sym,
                                 const int32_t* tile_of_point, int64_t* cnt, hipStream_t st);
hipError_t launch_np_piece_fill(const int4* blk, int64_t nl, int sym,
                                const int32_t* tile_of_point, const int64_t* off,
                                const int64_t* bounds, int nch, int tbits, uint64_t* keys,
                                uint32_t* vals, int2* pcs, hipStream_t st);
hipError_t launch_np_seg_flags(const uint64_t* keys, int64_t np, int64_t* flag, hipStream_t st);
hipError_t launch_np_seg_fill(const uint64_t* keys, const uint32_t* vals, const int2* pcs,
                              const int64_t* sidx, int64_t np, int64_t nseg, int tbits,
                              int64_t* seg_start, int32_t* seg_tile, int2* spcs, hipStream_t st);
hipError_t launch_np_chunk_segs(const uint64_t* keys, const int64_t* seg_start, int64_t nseg,
                                int tbits, int nch, int64_t* cseg, hipStream_t st);
// blk, rank, cu, cv: the chunk's first entry; t, t2: kmax entries per block
hipError_t launch_np_t(const int4* blk, int64_t nbk, const int32_t* rank, const int64_t* cu,
                       const int64_t* cv, int64_t ubase, int64_t vbase, const void* U,
                       const void* V, const void* xm, int kmax, int sym, void* t, void* t2,
                       int f64, hipStream_t st);
// segments [s0, s0 + ns) of one chunk; blk, rank, cu, cv: the whole list
hipError_t launch_np_apply(const int64_t* seg_start, const int32_t* seg_tile, int64_t s0,
                           int64_t ns, const int2* spcs, const int4* blk, const int32_t* rank,
                           const int64_t* cu, const int64_t* cv, int64_t ubase, int64_t vbase,
                           int64_t b0, const void* U, const void* V, const void* t,
                           const void* t2, int kmax, const int32_t* tile_lo,
                           const int32_t* perm, double alpha, void* z, int max_tile, int f64,
                           hipStream_t st);

// several right-hand sides (k_mm.hip), M in {1, 2, 4, 8, 16} per launch:
// vectors point-major (vec[i * M + c]); mr <= M real sides (the matrix-core
// forms pad a group to M = 8 or 16 with zero sides, the others take mr = M)
hipError_t launch_mm_gather(const void* X, int64_t ldx, const int32_t* perm, int64_t ncols,
                            int64_t col0, void* vec, int M, int mr, int f64, hipStream_t st);
hipError_t launch_mm_p1(int M, int64_t ntiles, const int32_t* tile_lo, const int64_t* meta,
                        int ms, int R, const void* pool, const void* vec, void* partial,
                        int64_t pbase, int smode, hipStream_t st);
hipError_t launch_mm_p1_reduce(int M, const int4* rec, int64_t ncols, const int64_t* pfc,
                               const void* partial, void* vec, int64_t n, int f64,
                               hipStream_t st);
hipError_t launch_mm_rowtile(int M, int64_t ntiles, const int32_t* tile_lo, const int64_t* meta,
                             const int64_t* widx, const void* upool, const void* npool,
                             const void* vec, const int32_t* perm, double alpha, double beta,
                             double sigma2, void* Z, int64_t ldz, int R, int max_tile,
                             int fmode, int nmode, const void* soa, int64_t n, int d,
                             KernelFn kern, int mr, hipStream_t st);

}  // namespace hmx
