/*
 * hmxo.h -- CPU oracle for the H-matrix construction and H-matrix-vector
 * product of Zaspel, "Algorithmic patterns for H-matrices on many-core
 * processors" (arXiv:1708.09707).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain, FP64 reference
 * that the HIP path is checked against.  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code, no
 * header and no constant with the HIP library.
 *
 * All pointers are host pointers.  Points are row-major (n x d) doubles;
 * "soa" arrays are the Morton-ordered coordinates stored dimension-major
 * (d x n).  Functions return 0 on success and a negative value on bad
 * arguments.
 */
#ifndef HMXO_H
#define HMXO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* kernel kinds; p0 is the kernel parameter */
#define HMXO_GAUSSIAN 0   /* exp(-r^2 / p0)                                */
#define HMXO_MATERN32 1   /* (1 + sqrt(3) r / p0) exp(-sqrt(3) r / p0)      */
#define HMXO_MATERN_NU1 2 /* Section 6.2 Matern, beta - d/2 = 1, length p0:
                             (r/p0) K_1(r/p0) / (2^(beta-1) Gamma(beta)),
                             beta = 1 + d/2                                 */
#define HMXO_CONST    3   /* 1 (rank-one matrix)                            */
#define HMXO_LOWRANK  4   /* (1 + x.y)^2 (rank <= 1 + d + d(d+1)/2)         */

double hmxo_kernel(int kind, double p0, const double* x, const double* y, int d);

/* s K_1(s) for s >= 0 (modified Bessel function of the second kind, order 1;
 * the limit 1 at s = 0) */
double hmxo_xk1(double s);

/* Section 4.4 (Z-order curve) and Algorithm 6 */
int hmxo_global_box(const double* pts, int64_t n, int32_t d, double* lo, double* hi);
int hmxo_morton(const double* pts, int64_t n, int32_t d, const double* lo, const double* hi,
                uint64_t* codes);
int hmxo_sort(const uint64_t* codes, int64_t n, int32_t* perm);
int hmxo_ordered_coords(const double* pts, int64_t n, int32_t d, const int32_t* perm, double* soa);

/* Section 2.1 (cluster tree, cardinality-based clustering on the Z-order).
 * Nodes in breadth-first order; child0[k] = -1 for a leaf, else the two
 * children are child0[k] and child0[k]+1.  Returns the node count, or the
 * required count if cap is too small (arrays untouched). */
int64_t hmxo_cluster_tree(int64_t n, int32_t leaf, int64_t cap, int32_t* lo, int32_t* hi,
                          int32_t* depth, int64_t* child0);
/* Section 2.2: a = min, b = max over the node's points; boxes are d-major per node */
int hmxo_boxes(const double* soa, int64_t n, int32_t d, int64_t nnodes, const int32_t* lo,
               const int32_t* hi, double* bmin, double* bmax);
/* eq. (3) in the squared form (no square roots) */
int hmxo_admissible(const double* amin, const double* amax, const double* bmin,
                    const double* bmax, int32_t d, double eta);

/* Algorithm 1, done level by level as in Algorithm 4.  Leaves are written as
 * (tlo, thi, slo, shi, level) records (5 int32 each) in canonical order
 * (level, position in level).  level_sizes[l] = |V(l)|.  Returns 0, or 1 if a
 * capacity was too small (counts are still reported). */
int hmxo_partition(const double* soa, int64_t n, int32_t d, int32_t leaf, double eta,
                   int64_t cap_adm, int32_t* adm, int64_t* n_adm,
                   int64_t cap_dense, int32_t* dense, int64_t* n_dense,
                   int64_t* level_sizes, int32_t* n_levels);

/* Algorithm 2 on the block tau x sigma = [tlo,thi) x [slo,shi) of the
 * Morton-ordered matrix.  First column: the sigma point nearest to the centre
 * of tau's bounding box; a column without a residual entry above eps0 times
 * the column's own largest |entry| adds no rank, the lowest unused column
 * follows, and kmax such columns end the block.
 * U is m x kmax and V is n x kmax, column-major.  fixed != 0 skips the stopping test (fixed rank).  r_start > 0 selects the
 * one-shot form: exactly min(r_start, R) steps, then the stopping test on the
 * last term; if it fails, continue adaptively.  *steps gets the number of
 * columns evaluated (including skipped ones). */
int hmxo_aca(const double* soa, int64_t n, int32_t d, int32_t kind, double p0,
             int64_t tlo, int64_t thi, int64_t slo, int64_t shi, int32_t kmax,
             double eps, double aca_eta, double eps0, int32_t fixed, int32_t r_start,
             double* U, double* V, int32_t* rank, int32_t* steps);
/* hmxo_aca with a trace (optional, kmax x 5 doubles): for accepted step r,
 * the row pivot i_r and the column j_r (block-local indices), the relative
 * gap between the largest and second largest |residual| over unused rows
 * at the row pivot choice, the stopping test's ratio
 * |u_r| |v_r| / (eps (1 - aca_eta) / (1 + eps) |S_r|_F) (the test passes at
 * <= 1), and the relative gap of the next column pivot's choice.  Used to
 * show that a rank another implementation finds differently was decided by
 * a near-tie. */
int hmxo_aca_traced(const double* soa, int64_t n, int32_t d, int32_t kind, double p0,
                    int64_t tlo, int64_t thi, int64_t slo, int64_t shi, int32_t kmax, double eps,
                    double aca_eta, double eps0, int32_t fixed, int32_t r_start, double* U,
                    double* V, int32_t* rank, int32_t* steps, double* trace);

/* Algorithm 3 in flat form (no-storage mode: every block is built, applied and
 * discarded):  z = alpha * (H x + sigma2 x) + beta * z, vectors in the
 * original point order.  ranks (optional, cap n_adm) gets the ACA ranks in
 * canonical admissible order.  stats (optional, 8 doubles):
 * [n_adm, n_dense, sum rank, dense entries, factor entries, levels, 0, 0]. */
int hmxo_hmvp(const double* pts, int64_t n, int32_t d, int32_t kind, double p0,
              int32_t leaf, double eta, int32_t kmax, double eps, double aca_eta,
              double eps0, int32_t fixed, double sigma2, double alpha, double beta,
              const double* x, double* z, int64_t ranks_cap, int32_t* ranks, double* stats);
/* hmxo_hmvp with the symmetric far field (symmetric = 1): only the
 * admissible leaf with tau before sigma (or tau = sigma) is approximated, its
 * mirror (sigma, tau) applies the transposed factors V U^T; ranks of a
 * mirror are its primary's; stats[4] counts the stored factor entries.
 * Returns -4 if an admissible leaf has no mirror. */
int hmxo_hmvp_ex(const double* pts, int64_t n, int32_t d, int32_t kind, double p0,
                 int32_t leaf, double eta, int32_t kmax, double eps, double aca_eta,
                 double eps0, int32_t fixed, int32_t symmetric, double sigma2, double alpha,
                 double beta, const double* x, double* z, int64_t ranks_cap, int32_t* ranks,
                 double* stats);

/* Rectangular A_{phi, Y1 x Y2} (two point sets, Section 6): each set ordered
 * by its own Morton codes and clustered in its own tree, Algorithm 1 from the
 * block Y1 x Y2.  hmxo_partition_rect: leaves (tlo, thi, slo, shi, level)
 * with rows in Y1's Morton order and columns in Y2's (soa1, soa2: the sets'
 * ordered coordinates), return codes as hmxo_partition.  hmxo_hmvp_rect:
 * z = alpha H x + beta z, x (n2) in Y2's original order, z (n1) in Y1's.
 * hmxo_dense_matvec_rect: z = A x, the plain dense product. */
int hmxo_dense_matvec_rect(const double* pts1, int64_t n1, const double* pts2, int64_t n2,
                           int32_t d, int32_t kind, double p0, const double* x, double* z);
int hmxo_partition_rect(const double* soa1, int64_t n1, const double* soa2, int64_t n2,
                        int32_t d, int32_t leaf, double eta, int64_t cap_adm, int32_t* adm,
                        int64_t* n_adm, int64_t cap_dense, int32_t* dense, int64_t* n_dense,
                        int64_t* level_sizes, int32_t* n_levels);
int hmxo_hmvp_rect(const double* pts1, int64_t n1, const double* pts2, int64_t n2, int32_t d,
                   int32_t kind, double p0, int32_t leaf, double eta, int32_t kmax, double eps,
                   double aca_eta, double eps0, int32_t fixed, double alpha, double beta,
                   const double* x, double* z, int64_t ranks_cap, int32_t* ranks, double* stats);

/* Stored-mode product restricted to the Morton-order rows [row_lo, row_hi):
 * the leaves whose tau meets the range are built (ACA / dense entries),
 * stored and applied; z gets (H x) for those rows in Morton order (no shift).
 * perm_out (optional, n) gets the permutation.  times (5 doubles): order +
 * partition seconds, build seconds, apply seconds, stored entries, blocks. */
int hmxo_hmvp_rows(const double* pts, int64_t n, int32_t d, int32_t kind, double p0,
                   int32_t leaf, double eta, int32_t kmax, double eps, double aca_eta,
                   double eps0, int32_t fixed, int64_t row_lo, int64_t row_hi, const double* x,
                   double* z, int32_t* perm_out, double* times);

/* brute-force dense product z_i = sum_j phi(y_i, y_j) x_j (+ sigma2 x_i) for
 * the listed rows (rows == NULL: all rows; then z has n entries, else nrows). */
int hmxo_dense_matvec(const double* pts, int64_t n, int32_t d, int32_t kind, double p0,
                      double sigma2, const double* x, const int64_t* rows, int64_t nrows,
                      double* z);
/* the dense product for m <= 64 right-hand sides (X n x m, Z rows x m,
 * row-major), each column summed as hmxo_dense_matvec sums it */
int hmxo_dense_matmat(const double* pts, int64_t n, int32_t d, int32_t kind, double p0,
                      double sigma2, const double* X, int32_t m, const int64_t* rows,
                      int64_t nrows, double* Z);

/* Conjugate gradients on the dense system (A + sigma2 I) x = b, x from 0,
 * stopping at |r| / |b| <= tol.  Returns 0 converged, 1 not converged,
 * 2 breakdown (p.Ap <= 0). */
int hmxo_cg_dense(const double* pts, int64_t n, int32_t d, int32_t kind, double p0,
                  double sigma2, const double* b, double* x, double tol, int32_t max_iter,
                  int32_t* iters, double* rel_res);

/* dense block A|tau x sigma of the Morton-ordered matrix, column-major m x n */
int hmxo_dense_block(const double* soa, int64_t n, int32_t d, int32_t kind, double p0,
                     int64_t tlo, int64_t thi, int64_t slo, int64_t shi, double* A);

/* Rank predictor MLP 8 -> 64 -> 64 -> 64 -> 1 (ReLU), parameters packed as
 * W1 (64x8 row-major), b1, W2 (64x64), b2, W3 (64x64), b3, W4 (1x64), b4. */
int hmxo_mlp_nparams(void);
int hmxo_mlp_forward(const double* w, const double* X, int64_t B, double* out);
/* pinball loss (quantile q) averaged over the batch and its gradient */
int hmxo_mlp_loss_grad(const double* w, const double* X, const double* y, int64_t B, double q,
                       double* loss, double* grad);
/* one Adam step (t >= 1) on n parameters */
int hmxo_mlp_adam(double* w, double* m, double* v, const double* g, int64_t n, int64_t t,
                  double lr, double b1, double b2, double eps);
/* the 8 block features from the two cluster boxes */
int hmxo_features(const double* ta, const double* tb, const double* sa, const double* sb, int32_t d,
                  int64_t m, int64_t n, double ell, double* f);

int hmxo_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
