/*
 * hmx.h -- C ABI of the MI355X (gfx950) H-matrix library.
 *
 * The library builds an H-matrix approximation of the kernel matrix
 *     A_ij = phi(y_i, y_j),  i, j = 1..N                     (paper eq. (2))
 * for points y_i in R^d (d = 1, 2, 3) and applies it to vectors:
 *     z := alpha (A + sigma2 I) x + beta z                    (Section 2.5,
 *                                                              Algorithm 3;
 *                                                              shift from the
 *                                                              GPR / kernel
 *                                                              ridge setting
 *                                                              of Section 1)
 * following Zaspel, "Algorithmic patterns for H-matrices on many-core
 * processors" (arXiv:1708.09707):
 *   - Z-order (Morton) ordering of the points                 Section 4.4, Alg. 6
 *   - cardinality-based cluster tree on that order            Section 2.1
 *   - block cluster tree traversal, level by level, with the
 *     bounding-box admissibility condition                    Alg. 1, Alg. 4, eq. (3)
 *   - batched adaptive cross approximation (ACA) of the
 *     admissible blocks                                       Alg. 2, Section 5.4.1
 *   - batched H-matrix-vector product (dense near field plus
 *     U (V^T x) far field)                                    Alg. 3, Section 5.4
 *
 * Conventions (every function):
 *   - Pointers documented as "device" must be HIP device allocations on the
 *     current device; "host" pointers are ordinary host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All device work is enqueued on it.
 *   - Functions return an hmx_status and never abort; on error the message of
 *     hmx_last_error() (thread-local) says what failed.  A failed build
 *     produces no handle and leaks no device memory.
 *   - One handle must not be used from two threads at once; distinct handles
 *     may be.
 *   - Limits: 1 <= N < 2^31, d in {1,2,3}, 1 <= max_rank <= 128.
 */
#ifndef HMX_H
#define HMX_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hmx_hmatrix_s* hmx_hmatrix; /* opaque; owns all device memory it allocates */

typedef enum {
    HMX_OK = 0,
    HMX_ERR_INVALID_ARG = 1,
    HMX_ERR_OOM = 2,
    HMX_ERR_DEVICE = 3,
    HMX_ERR_NOT_CONVERGED = 4,
    HMX_ERR_UNSUPPORTED = 5
} hmx_status;

typedef enum { HMX_F64 = 0, HMX_F32 = 1, HMX_BF16 = 2 } hmx_dtype;

/* Kernel functions phi(x, y) with r = |x - y| (Euclidean).
 *  HMX_GAUSSIAN  : exp(-r^2 / p0)                    (Section 6.2 with a length
 *                                                     scale, p0 = l^2 > 0)
 *  HMX_MATERN32  : (1 + sqrt(3) r / p0) exp(-sqrt(3) r / p0), p0 = l > 0
 *  HMX_MATERN_NU1: the Matern kernel of Section 6.2 with beta - d/2 = 1,
 *                  K_1(s) s / (2^(beta-1) Gamma(beta)), s = r / p0, beta =
 *                  1 + d/2 (K_1: modified Bessel function of the second
 *                  kind; value 1/(2^(d/2) Gamma(1 + d/2)) at r = 0); p0 = l
 *                  > 0, the paper's unscaled kernel is p0 = 1.  Not for
 *                  hmx_build_batched (its normalisation depends on d)
 *  HMX_TEST_CONST: 1 (rank-one matrix; test kernel)
 *  HMX_TEST_LOWRANK: (1 + x.y)^2 (rank <= 1 + d + d(d+1)/2; test kernel) */
typedef enum {
    HMX_GAUSSIAN = 0,
    HMX_MATERN32 = 1,
    HMX_MATERN_NU1 = 2,
    HMX_TEST_CONST = 3,
    HMX_TEST_LOWRANK = 4
} hmx_kernel_kind;

typedef struct {
    hmx_kernel_kind kind;
    double p0;
    double p1; /* reserved, 0 */
} hmx_kernel;

/* ACA rank control.
 *  HMX_RANK_ADAPTIVE: Algorithm 2 with its stopping criterion, at most max_rank.
 *  HMX_RANK_LEARNED : a rank predictor (hmx_mlp, below) sizes every
 *                     admissible block before the ACA, so that one batched
 *                     pass replaces k_max-sized scratch: each block gets
 *                     storage for r^ = clamp(ceil(pred) + 1, 1,
 *                     min(max_rank, m, n)) columns.
 *                     Sizing form (learned_one_shot = 0): Algorithm 2 with
 *                     its stopping test every step; a block that fills its
 *                     r^ columns unfinished is approximated again with
 *                     max_rank storage.  The ranks and factors are those of
 *                     HMX_RANK_ADAPTIVE (bit for bit); the prediction only
 *                     sizes memory.
 *                     One-shot form (learned_one_shot = 1): exactly r^ steps
 *                     without the test, which then judges the last term; a
 *                     failing block is approximated again with max_rank
 *                     storage (the same r^ steps, then adaptive).  Either
 *                     way Algorithm 2's test judges every block.
 *  HMX_RANK_FIXED   : exactly min(max_rank, m, n) rank-one steps, no stopping
 *                     test (the fixed-k mode of the paper's experiments). */
typedef enum { HMX_RANK_ADAPTIVE = 0, HMX_RANK_LEARNED = 1, HMX_RANK_FIXED = 2 } hmx_rank_mode;

/* Rank predictor: an MLP 8 -> 64 -> 64 -> 64 -> 1 with ReLU on the hidden
 * layers, FP32, on the features of an admissible block tau x sigma
 *   [log2 |tau|, log2 |sigma|, diam(tau) / l, diam(sigma) / l, dist / l,
 *    min(diam(tau), diam(sigma)) / max(dist, 1e-12), d, log10 l^2]
 * (bounding-box diameters and distance of eq. (3); l the kernel's length
 * scale: sqrt(p0) for the Gaussian, p0 for the Matern kernels, 1 for the test
 * kernels), standardised per feature as (f - mean) * scale.  Parameters are
 * packed W1 (64 x 8, row-major), b1, W2 (64 x 64), b2, W3 (64 x 64), b3,
 * W4 (1 x 64), b4: HMX_MLP_NPARAMS floats.  Trained with the pinball
 * (quantile) loss rho_q(y - pred) = (y - pred)(q - [y < pred]) averaged over
 * the batch, and Adam. */
#define HMX_MLP_NPARAMS 8961
#define HMX_MLP_FEATURES 8
typedef struct hmx_mlp_s* hmx_mlp; /* opaque; owns its device parameters */

typedef struct {
    int32_t leaf_size;       /* C_leaf >= 1: clusters with more points split (Section 2.1) */
    double eta;              /* admissibility parameter eta >= 0 (eq. (3)) */
    double aca_eps;          /* ACA relative accuracy epsilon >= 0 (Algorithm 2) */
    double aca_eta;          /* the (1 - eta) factor of Algorithm 2's stopping test,
                                in [0, 1); default 0 (see the stopping test) */
    double aca_eps0;         /* a residual column whose largest entry is <= eps0
                                times the column's own largest |entry| adds no
                                rank (Section 2.4); < 0 selects the default
                                1e-14 (F64) or 1e-7 (F32) */
    int32_t max_rank;        /* k_max, 1..128 */
    double sigma2;           /* diagonal shift sigma^2 >= 0 of (A + sigma^2 I) */
    hmx_dtype compute_dtype; /* HMX_F64 or HMX_F32: kernel evaluation, ACA and
                                matvec accumulation (the ACA norm estimate is
                                always FP64) */
    hmx_dtype storage_dtype; /* stored factors U and V: HMX_F64 (requires F64
                                compute), HMX_F32 or HMX_BF16 (require F32
                                compute; BF16 rounds to nearest even) */
    hmx_dtype near_dtype;    /* stored near field: equal to storage_dtype, or
                                HMX_F32 with BF16 factors */
    hmx_rank_mode rank_mode;
    int32_t aca_chunk_mb;    /* ACA scratch budget per chunk of admissible blocks,
                                MiB; 0 selects 40% of the device memory free
                                when the ACA starts.  Blocks are approximated in
                                chunks whose column scratch (k_max, or the
                                predicted target) fits the budget, then
                                compacted to their exact ranks */
    int32_t aca_only;        /* 1: stop after the ACA (no matrix pool).  The
                                handle then serves partition, ranks, features
                                and stats; hmx_matvec returns UNSUPPORTED.
                                Used to collect predictor training data */
    hmx_mlp mlp;             /* predictor for HMX_RANK_LEARNED (borrowed; must
                                outlive hmx_build only), else NULL */
    int32_t learned_one_shot; /* HMX_RANK_LEARNED form: 0 sizing, 1 one-shot */
    int32_t near_recompute;  /* 1: the near field is not stored; every matvec
                                evaluates the dense leaves' entries from the
                                Morton-ordered coordinates in the compute type
                                (the paper's no-storage mode for dense blocks,
                                Section 5.4), same arithmetic as the stored
                                assembly.  near_dtype is then ignored */
    int32_t aca_split_rows;  /* admissible blocks whose clusters hold at least
                                this many points run their ACA on many
                                workgroups each (0: 262144, which also bounds
                                the single-workgroup classes' LDS bitmasks) */
    int32_t symmetric_far;   /* 1: symmetric far field.  The kernel matrix is
                                symmetric, and the partition is too: with every
                                admissible leaf (tau, sigma) its mirror
                                (sigma, tau) is a leaf.  Only the leaf with
                                tau before sigma is approximated by the ACA;
                                the mirror uses its factors transposed
                                (A|sigma x tau ~ V U^T), which halves the
                                ACA work and the stored factors and makes H
                                exactly symmetric (as CG on (H + sigma2 I)
                                assumes).  0: Algorithm 1's separate
                                approximations of both leaves.  The matvec
                                reads every stored factor twice (as a leaf's
                                U and as its mirror's V) */
    /* Optional device allocator (both NULL: the library's own, which keeps
     * released blocks in a process-wide cache for later builds; hmx_trim
     * empties it).  When dev_alloc is set, every device buffer of this build
     * and of the handle's later calls (hmx_autotune's scratch vectors,
     * hmx_cg_solve's work vectors) is obtained as dev_alloc(bytes, alloc_ctx)
     * (bytes a multiple of 256; the memory must be device memory of the
     * current device, aligned to 256 bytes) and returned exactly once as
     * dev_free(ptr, bytes, alloc_ctx): temporary buffers during the build,
     * the handle's buffers by hmx_destroy.  A NULL return fails the call
     * with HMX_ERR_OOM after every buffer obtained so far has been returned
     * (no handle is produced).  The library synchronises before it returns a
     * buffer that queued work may still use.  Both must be set, or neither. */
    void* (*dev_alloc)(size_t bytes, void* ctx);
    void (*dev_free)(void* ptr, size_t bytes, void* ctx);
    void* alloc_ctx;
    int32_t far_recompute;   /* 1: no precomputation of the far field (the
                                paper's default mode, Section 5.4).  The build
                                runs ordering, cluster tree, traversal and the
                                chunk plan of the ACA list only (no ACA, no
                                factors); every hmx_matvec approximates the
                                admissible leaves again, chunk by chunk within
                                the aca_chunk_mb budget (bs_ACA of Section
                                5.4.1), applying each chunk's U (V^T x) at
                                once, so the device holds one chunk's ACA
                                scratch instead of all factors.  The ACA is
                                Algorithm 2 with the same pivots and tests as
                                the stored mode, so the ranks and factors equal
                                a stored build's; the sums run in another
                                order (per chunk), so products agree to
                                rounding.  With near_recompute also the near
                                field is evaluated in every product.  Adaptive
                                or fixed rank modes only (LEARNED:
                                UNSUPPORTED); excludes aca_only.  hmx_matvec
                                then waits for its stream to finish;
                                hmx_matvec_graph, hmx_cg_solve_noalloc and
                                hmx_get_factors return UNSUPPORTED;
                                hmx_get_ranks reports the ranks of the last
                                matvec (0 before the first) */
} hmx_params;

/* Statistics of a built H-matrix (host struct). */
typedef struct {
    int64_t n;
    int32_t d;
    int32_t levels;           /* block-tree levels |V(l)| > 0 */
    int64_t n_adm, n_dense;   /* admissible / dense leaves */
    int64_t n_tiles;          /* leaf clusters (row tiles of the matvec) */
    int64_t sum_rank;         /* sum of ACA ranks */
    int32_t max_rank_used;
    int32_t entry_bytes;      /* bytes per stored factor entry (storage dtype) */
    int64_t factor_entries;   /* stored factor entries: sum over the approximated
                                 leaves of rank * (|tau| + |sigma|) (with
                                 symmetric_far only the primary leaves) */
    int64_t u_entries;        /* sum over all admissible leaves of rank * |tau|
                                 (the U rows phase 2 of a matvec reads) */
    int64_t v_entries;        /* sum over all admissible leaves of rank * |sigma|
                                 (the V rows phase 1 reads) */
    int64_t near_entries;     /* sum_dense |tau| * |sigma| */
    int64_t aca_columns;      /* ACA residual columns evaluated (incl. skipped) */
    int64_t aca_chunks;       /* chunks the admissible leaves were approximated in */
    int32_t near_entry_bytes; /* bytes per stored near-field entry */
    int32_t tile_config;      /* row-tile kernel configuration in use (-1:
                                 default shape; see hmx_autotune) */
    double matvec_bytes;      /* algorithmic HBM bytes of one matvec (beta = 0) */
    double phase_ms[8];       /* build phases: order, tree, traversal, aca,
                                 compaction, near field, matvec plan, total */
    int64_t device_bytes;     /* device memory held by the handle */
    int64_t level_sizes[64];  /* |V(l)| per level */
    int64_t aca_fallback;     /* HMX_RANK_LEARNED: blocks left unfinished by
                                 their target that did not fit the overflow
                                 reserve, approximated again in a second pass */
    int64_t aca_capacity;     /* entries of ACA storage reserved: sum over the
                                 blocks of (target or max_rank) * (m + n) */
    double predict_ms;        /* HMX_RANK_LEARNED: rank prediction time */
    int64_t aca_overflow;     /* HMX_RANK_LEARNED: blocks that outgrew their
                                 target and continued, in the same launch, in
                                 overflow storage for max_rank columns */
    int64_t aca_kernel_evals; /* ACA kernel evaluations: sum over admissible
                                 blocks of steps m + rank n */
    double aca_flops;         /* ACA multiply-add flops: sum of
                                 2 rank (rank - 1) (m + n) (residual updates
                                 and the norm recursion's inner products) */
    int64_t rows, cols;       /* the matrix's shape: n x n, or n1 x n2 for
                                 hmx_build_rect */
    int64_t alloc_fresh_bytes; /* device bytes the build obtained from the
                                  driver instead of the library's block cache
                                  (memory the process released before is
                                  cleared by the driver on allocation) */
    int64_t alloc_flushes;    /* cache flushes during the build (an allocation
                                 failed and every cached block was freed) */
} hmx_stats;

/* Fill *p with the defaults: leaf 256, eta 1.5, eps 1e-5, aca_eta 0,
 * eps0 default, max_rank 64, sigma2 0, F32 compute and storage, adaptive. */
hmx_status hmx_params_default(hmx_params* p);

/* Build the H-matrix of phi over the points.
 *   points : device, n x d row-major, pts_dtype F64 or F32 (F32 values are
 *            promoted exactly to F64 for ordering and boxes).  Read only; the
 *            handle keeps its own Morton-ordered copy, so points may be freed
 *            after the call.
 *   kernel, params : host structs (see above).
 *   out    : host; receives the handle on HMX_OK, NULL otherwise.
 * Host-blocking: synchronises `stream` once per block-tree level and at pool
 * sizing; every step runs in device kernels. */
hmx_status hmx_build(const void* points, hmx_dtype pts_dtype, int64_t n, int32_t d,
                     const hmx_kernel* kernel, const hmx_params* params, void* stream,
                     hmx_hmatrix* out);

/* Batched build of nprob independent problems (the same kind of kernel,
 * Gaussian or Matern-3/2, each with its own p0 and point set, one shared
 * params) as ONE handle: the block-diagonal H-matrix diag(H_1, ..., H_nprob)
 * over the concatenated index set, problem p owning indices
 * [off_p, off_p + n_p) with off_p = n_0 + ... + n_{p-1}.  Every problem's
 * ordering, cluster tree and block partition are those of its own build (bit
 * for bit), computed for all problems at once: one launch per step (boxes,
 * Morton codes, the sort, each tree and box level, each block-tree level of
 * the traversal, with one host readback per block-tree level for all
 * problems).  The ACA of all problems' admissible leaves, the near field and
 * every matvec then run as single batched launches over the union.  hmx_matvec and
 * hmx_cg_solve on the handle act on concatenated vectors of n_0 + ... +
 * n_{nprob-1} entries (each problem in its own original point order).
 * Internally problem p's coordinates are divided by its kernel length
 * (sqrt(p0) Gaussian, p0 Matern) and padded to d = 3 with zeros, so matrix
 * entries may differ from a single build's in the last bits.
 *   points : host array of nprob device pointers (n_p x d_p row-major, all
 *            in pts_dtype); n, d, kernels: host arrays of nprob entries.
 * hmx_get_partition lists the leaves of all problems in union indices, each
 * problem's leaves in its canonical order (the admissible leaves grouped by
 * the ACA's size classes, the dense ones level by level);
 * hmx_get_boxes, hmx_block_features and hmx_rank_predict return UNSUPPORTED.
 * Limits: sum of n_p < 2^31.  Host-blocking like hmx_build. */
hmx_status hmx_build_batched(int32_t nprob, const void* const* points, hmx_dtype pts_dtype,
                             const int64_t* n, const int32_t* d, const hmx_kernel* kernels,
                             const hmx_params* params, void* stream, hmx_hmatrix* out);

/* Rectangular H-matrix of A_{phi, Y1 x Y2} = [phi(y_i, y'_j)] for two point
 * sets (Section 6: the library's problem is the kernel matrix between sets
 * Y1 and Y2): rows Y1 (n1 points), columns Y2 (n2 points), both
 * d-dimensional (n x d row-major device arrays in pts_dtype).  Each set is
 * ordered by its own Morton codes (Algorithm 6 relative to its own bounding
 * box) and clustered in its own tree (Section 2.1); the block cluster tree
 * starts from the single block Y1 x Y2 and follows Algorithm 1 with eq. (3)
 * (a block splits into 4 when it is not admissible and both clusters hold
 * more than leaf_size points).  ACA, near field, matvec, NP mode and the
 * autotuner work as for hmx_build; the matvec maps x (n2 entries, Y2's
 * order) to z (n1 entries, Y1's order).  Internally the two sets are one
 * union of n1 + n2 points (Y2 after Y1), their coordinates divided by the
 * kernel length and padded to 3 dimensions, so entries may differ from a
 * direct evaluation in the last bits.  hmx_get_partition reports union
 * indices (columns offset by n1) and hmx_get_batch the two sets as two
 * problems.  Kernels: Gaussian, Matern-3/2, Matern nu = 1.  params.sigma2
 * must be 0 and symmetric_far 0 (INVALID_ARG); hmx_cg_solve and
 * hmx_cg_solve_noalloc return UNSUPPORTED; hmx_get_boxes, hmx_block_features
 * and hmx_rank_predict return UNSUPPORTED.  Limits: n1 + n2 < 2^31.
 * Host-blocking like hmx_build. */
hmx_status hmx_build_rect(const void* rows, int64_t n1, const void* cols, int64_t n2,
                          hmx_dtype pts_dtype, int32_t d, const hmx_kernel* kernel,
                          const hmx_params* params, void* stream, hmx_hmatrix* out);

/* Problems of a handle: *nprob (1 for hmx_build, 2 for hmx_build_rect) and,
 * if offsets != NULL (host, nprob + 1 entries), each problem's first index
 * and the total. */
hmx_status hmx_get_batch(hmx_hmatrix h, int32_t* nprob, int64_t* offsets);

/* z := alpha (H + sigma2 I) x + beta z in the ORIGINAL point order
 * (Algorithm 3; x is permuted to Morton order and z back, Section 5.1).
 *   x, z : device vectors in vec_dtype, which must equal the handle's
 *          compute dtype (F32 for BF16 storage): x of stats.cols and z of
 *          stats.rows entries (both n, except for hmx_build_rect).  x and z
 *          must not overlap.
 * Fully asynchronous on `stream`; allocates nothing. */
hmx_status hmx_matvec(hmx_hmatrix h, const void* x, void* z, hmx_dtype vec_dtype, double alpha,
                      double beta, void* stream);

/* Z := alpha (H + sigma2 I) X + beta Z for m right-hand sides (the product
 * of Algorithm 3 for a block of vectors; for many vectors V^T X and the row
 * tiles become products with m columns).  Every stored entry is read once
 * per group of up to 16 right-hand sides: groups of 16, the rest as one
 * group (on the matrix cores, padded to 8 or 16 with zero sides, when the
 * near field is stored; in power-of-two groups when it is evaluated in the
 * product), a last single side as hmx_matvec.
 *   X : device, column-major stats.cols x m, leading dimension ldx >= cols
 *       (right-hand side c at X + c ldx, original point order);
 *   Z : device, column-major stats.rows x m, leading dimension ldz >= rows;
 *       vec_dtype as for hmx_matvec; X and Z must not overlap.
 * Column c of Z sums the same terms as hmx_matvec of X's column c, in
 * another order (results agree to rounding).  The first call on a handle
 * allocates work vectors of 16 (n + sum_rank) compute-type values and the
 * partial sums, kept by the handle (hmx_destroy returns them); later calls
 * allocate nothing.  Asynchronous on `stream`.  far_recompute handles:
 * UNSUPPORTED. */
hmx_status hmx_matmat(hmx_hmatrix h, const void* X, int64_t ldx, void* Z, int64_t ldz,
                      int32_t m, hmx_dtype vec_dtype, double alpha, double beta, void* stream);

/* Matvecs of nprob separately built handles on one stream:
 * z[q] := alpha (H_q + sigma2_q I) x[q] + beta z[q] for q = 0..nprob-1 (host
 * arrays of nprob handles and device pointers; each pair of vectors as for
 * hmx_matvec on its handle).  Every argument is checked before the first
 * launch.  The fused form of many problems is one handle from
 * hmx_build_batched, whose every matvec is a single pass over all problems;
 * this call serves handles built one by one.  Asynchronous; allocates
 * nothing. */
hmx_status hmx_matvec_batched(int32_t nprob, const hmx_hmatrix* handles, const void* const* x,
                              void* const* z, hmx_dtype vec_dtype, double alpha, double beta,
                              void* stream);

/* ---- hipGraph-captured matvecs ---- */
typedef struct hmx_graph_s* hmx_graph; /* opaque; an instantiated HIP graph */

/* Capture reps consecutive hmx_matvec(h, x, z, vec_dtype, alpha, beta) into
 * one HIP graph (captured on a private stream; nothing runs yet).  x and z
 * (device) are baked into the graph: they and h must stay alive while the
 * graph is used, and the graph uses the tile configuration h had when it was
 * captured.  The matvec kernels record no memory-set nodes.  reps in
 * [1, 4096]. */
hmx_status hmx_matvec_graph(hmx_hmatrix h, const void* x, void* z, hmx_dtype vec_dtype,
                            double alpha, double beta, int32_t reps, hmx_graph* out);
/* Replay the captured matvecs on `stream` (asynchronous). */
hmx_status hmx_graph_launch(hmx_graph g, void* stream);
/* Release the graph (synchronises the device). */
hmx_status hmx_graph_destroy(hmx_graph g);

/* ---- autotuner of the matvec's row-tile kernel ---- */
/* Row-tile configurations: for c < 15 shape c % 5 of (lanes per row group,
 * row vectors per lane) = (16,1), (32,1), (64,1), (64,2), (64,4) and grid
 * c / 5; c = 15, 16, 17: the shape (8,1), for tiles of at most 8 row vectors
 * (16 rows in FP64, 32 in FP32, 64 in BF16), with grid c - 15.  Grids: 0 one
 * workgroup per tile, 1 a persistent grid of 2048 workgroups looping over the
 * tiles, 2 one workgroup per row pass of a tile (shapes whose pass covers
 * fewer rows than a tile split each tile's rows over several workgroups).
 * Configurations sum in different orders, so results may differ in the last
 * bits. */
#define HMX_TILE_CONFIGS 18

/* Time every configuration on this handle (reps row-tile launches each, HIP
 * events on `stream`, on scratch vectors it allocates) and keep the fastest
 * for later matvecs (lowest index on ties); likewise the lanes per column
 * group (8, 16, 32 or 64) of the far field's first product t = V^T x, whose
 * partial sums change order with it (results within rounding).  choice
 * (host, optional): the row-tile configuration chosen; times_ms (host,
 * optional, HMX_TILE_CONFIGS entries): mean milliseconds per row-tile
 * launch.  Host-blocking. */
hmx_status hmx_autotune(hmx_hmatrix h, int32_t reps, void* stream, int32_t* choice,
                        double* times_ms);
/* Select a row-tile configuration directly (-1: the default, one workgroup
 * per row pass of 128 rows (configuration 10, 11 or 12: 16, 32 or 64 lanes
 * per row group for 8, 4 or 2 rows per 16-byte vector), narrower when the
 * handle's largest tile is shorter; and the default phase-1 lanes too, so a
 * handle returns to its untuned products). */
hmx_status hmx_set_tile_config(hmx_hmatrix h, int32_t config);

/* Conjugate gradients for (H + sigma2 I) c = b, the kernel ridge regression
 * / Gaussian process system of Section 1, with H this handle's H-matrix and
 * sigma2 from its params (textbook CG; inner products accumulated in FP64).
 *   b, x : device vectors of n entries, original point order, compute dtype.
 *          x is overwritten; the iteration starts from x = 0.
 *   stops when the recurrence residual |r| / |b| <= rel_tol, after max_iter
 *   iterations, or on breakdown (p.(H + sigma2 I)p <= 0: the shifted
 *   H-matrix is not positive definite to working precision).
 *   iters, rel_res (recurrence), true_rel_res (|b - (H + sigma2 I) x| / |b|,
 *   one extra product at the end): host, optional.
 * Returns HMX_ERR_NOT_CONVERGED when rel_tol was not reached (x holds the
 * last iterate; on breakdown the step that broke down is not taken, so x is
 * the iterate before it, while iters counts that step too).  Host-blocking
 * (one readback per iteration); allocates three work vectors. */
hmx_status hmx_cg_solve(hmx_hmatrix h, const void* b, void* x, double rel_tol, int32_t max_iter,
                        void* stream, int32_t* iters, double* rel_res, double* true_rel_res);

/* hmx_cg_solve for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same solve, the same kernels and the same results bit for bit, with its
 * three work vectors, scalars and partial sums in a fixed device array of
 * HMX_CG_NOALLOC_MAX_BYTES that the library holds on every device it runs on
 * until the process ends.  The work space needs 3 * ceil256(n * e) + 256 +
 * 8256 bytes (e = 8 with F64 arithmetic, else 4; ceil256 rounds up to a
 * multiple of 256), which admits n up to 2^22 + 4736 in FP32 and 2^21 + 2368
 * in FP64; a larger handle returns HMX_ERR_INVALID_ARG before any work.
 * Calls no device allocation or free.  All calls on one device share the
 * array, so calls that overlap on one device (two threads, or two streams
 * without ordering between them) race; the array keeps the last call's
 * contents, every buffer is overwritten before it is read.  b, x, stream and
 * the outputs as for hmx_cg_solve. */
#define HMX_CG_NOALLOC_MAX_BYTES ((size_t)50397184) /* 48 MiB + 64 KiB */
hmx_status hmx_cg_solve_noalloc(hmx_hmatrix h, const void* b, void* x, double rel_tol,
                                int32_t max_iter, void* stream, int32_t* iters, double* rel_res,
                                double* true_rel_res);

/* Copy the ordering and the partition to host memory (any pointer may be
 * NULL to skip it):
 *   codes : n Morton codes in the ORIGINAL point order
 *   perm  : n int32; perm[k] = original index of the k-th point in Morton order
 *   adm, dense : 5 int32 per leaf (tlo, thi, slo, shi, level) in canonical
 *           order (level, position in level); index ranges are half-open in
 *           the Morton order.  *n_adm / *n_dense receive the counts and give
 *           the capacities on input (in leaves); too small -> INVALID_ARG.
 * Synchronises `stream`. */
hmx_status hmx_get_partition(hmx_hmatrix h, uint64_t* codes, int32_t* perm, int32_t* adm,
                             int64_t* n_adm, int32_t* dense, int64_t* n_dense, void* stream);

/* Cluster-tree leaf boxes / any node box: copies the global box (2*d doubles:
 * lo then hi) and, if nodes != NULL, the boxes of the leaf clusters in Morton
 * order (n_tiles x (lo[d], hi[d], first, last+1) as doubles).  Synchronises. */
hmx_status hmx_get_boxes(hmx_hmatrix h, double* global_box, double* leaf_boxes, void* stream);

/* ACA ranks of the admissible leaves in canonical order (n_adm int32), and
 * optionally the factors of one admissible leaf converted to double:
 * U (m x rank, column-major), V (n x rank).  Synchronises. */
hmx_status hmx_get_ranks(hmx_hmatrix h, int32_t* ranks, void* stream);
hmx_status hmx_get_factors(hmx_hmatrix h, int64_t leaf, double* U, double* V, int32_t* rank,
                           void* stream);

hmx_status hmx_get_stats(hmx_hmatrix h, hmx_stats* s);

/* Per-phase matvec timing with HIP events (tracing).  After
 * hmx_profile_begin(h, max_calls) every hmx_matvec on h records events on its
 * stream around its three phases (gather of x, far-field phase 1, row tiles)
 * for the first max_calls calls.  hmx_profile_end synchronises on the last
 * recorded event, writes the summed milliseconds of each phase to ms[0..2]
 * (host) and the number of recorded calls to *calls, and releases the
 * events.  begin allocates the events (host-side HIP objects, no device
 * memory); matvec itself still allocates nothing.  For a handle built with
 * far_recompute the three phases are: the near field (gather and row
 * tiles), the far field (ACA and application of every chunk), and the
 * ranks' bookkeeping; that matvec allocates its chunk scratch. */
hmx_status hmx_profile_begin(hmx_hmatrix h, int32_t max_calls);
hmx_status hmx_profile_end(hmx_hmatrix h, double* ms, int32_t* calls);

/* ---- rank predictor (HMX_RANK_LEARNED) ---- */

/* Create a predictor.  params: host, HMX_MLP_NPARAMS floats (the initial
 * weights; NULL = all zero).  Standardisation starts as the identity
 * (mean 0, scale 1) and the Adam state at zero. */
hmx_status hmx_mlp_create(const float* params, hmx_mlp* out);
hmx_status hmx_mlp_destroy(hmx_mlp m);

/* Host copies of the parameters and the standardisation (8 floats each);
 * any pointer may be NULL.  set resets the Adam state (moments and step). */
hmx_status hmx_mlp_set_params(hmx_mlp m, const float* params, const float* mean,
                              const float* scale);
hmx_status hmx_mlp_get_params(hmx_mlp m, float* params, float* mean, float* scale);

/* Checkpoint of a predictor: hmx_mlp_save writes the parameters, the
 * standardisation and the Adam state (moments and step count) to the file
 * `path` (host string; a little-endian binary record: 8-byte magic
 * "HMXMLP01", int64 parameter count and Adam step, then FP32 parameters,
 * mean, scale, first and second moments).  hmx_mlp_load creates a predictor
 * from such a file; a file of another size, magic or parameter count gives
 * HMX_ERR_INVALID_ARG and no predictor.  Both synchronise the device. */
hmx_status hmx_mlp_save(hmx_mlp m, const char* path);
hmx_status hmx_mlp_load(const char* path, hmx_mlp* out);

/* Set the standardisation from n training samples X (device, n x 8 FP32):
 * mean = sample mean, scale = 1 / population standard deviation (1 where it
 * is below 1e-6), both accumulated in FP64. */
hmx_status hmx_mlp_fit_normalization(hmx_mlp m, const float* X, int64_t n, void* stream);

/* out[b] = MLP(standardised X[b]) for B samples (device X: B x 8, out: B).
 * Asynchronous; allocates activation memory of B * 193 floats. */
hmx_status hmx_mlp_forward(hmx_mlp m, const float* X, int64_t B, float* out, void* stream);

/* Gradient of the mean pinball loss with quantile q in (0, 1) over a batch:
 * X (device, B x 8), y (device, B targets), grad (device, HMX_MLP_NPARAMS,
 * packed like the parameters), loss (host double, optional; synchronises
 * when given).  At y == pred the subgradient q is used. */
hmx_status hmx_mlp_loss_grad(hmx_mlp m, const float* X, const float* y, int64_t B, double q,
                             float* grad, double* loss, void* stream);

/* One Adam step with the given gradient (device): t += 1, then
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
hmx_status hmx_mlp_adam(hmx_mlp m, const float* grad, double lr, double beta1, double beta2,
                        double eps, void* stream);

/* Mini-batch training: for s = 0..steps-1 the batch is the samples
 * batch_idx[s * B .. s * B + B) (device int64 indices into X, y, drawn by
 * the caller; values outside [0, n) are clamped), forward, backward, Adam (beta 0.9 / 0.999, eps 1e-8).
 * X (device n x 8), y (device n).  losses (device double, steps entries,
 * optional) receives each batch's loss before its update.  Asynchronous. */
hmx_status hmx_mlp_train(hmx_mlp m, const float* X, const float* y, int64_t n,
                         const int64_t* batch_idx, int64_t B, int32_t steps, double q, double lr,
                         double* losses, void* stream);

/* Training pairs of a built handle (any rank mode, including aca_only):
 * the features of every admissible leaf in canonical order (device, n_adm x
 * 8 FP32) and, if ranks != NULL, its ACA rank as float (device, n_adm).
 * *n_adm (host) gives the capacity in leaves and receives the count; a too
 * small capacity returns INVALID_ARG.  Asynchronous. */
hmx_status hmx_block_features(hmx_hmatrix h, float* features, float* ranks, int64_t* n_adm,
                              void* stream);

/* The rank predictor's in-build inference on this handle's admissible leaves
 * (the fused kernel HMX_RANK_LEARNED runs before the ACA: features, input
 * standardisation, the four layers, the target clamp), with predictor m:
 *   pred   : device, n_adm floats, the raw network output per leaf (canonical
 *            order), or NULL;
 *   target : device, n_adm int32, clamp(ceil(pred) + 1, 1, min(max_rank, m,
 *            n)) with the handle's max_rank (a NaN output gives the upper
 *            bound), or NULL; at least one of the two is needed.
 * *n_adm (host) gives the capacity in leaves and receives the count; a too
 * small capacity returns INVALID_ARG.  Batched handles: UNSUPPORTED.
 * Asynchronous; allocates nothing. */
hmx_status hmx_rank_predict(hmx_hmatrix h, hmx_mlp m, float* pred, int32_t* target,
                            int64_t* n_adm, void* stream);

/* Release every device buffer of the handle (synchronises the device).  The
 * buffers return to the library's device-block cache, which later builds
 * reuse; hmx_trim gives the cached blocks back to the driver. */
hmx_status hmx_destroy(hmx_hmatrix h);

/* Free the library's cached device blocks (synchronises the device);
 * *released_bytes (optional, host) receives the bytes returned. */
hmx_status hmx_trim(int64_t* released_bytes);

const char* hmx_status_string(hmx_status s);
const char* hmx_last_error(void); /* thread-local message of the last failure */

#ifdef __cplusplus
}
#endif
#endif
