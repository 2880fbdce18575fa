/*
 * hmxo.c -- CPU oracle (TEST INFRASTRUCTURE ONLY) for the H-matrix path of
 * Zaspel, "Algorithmic patterns for H-matrices on many-core processors".
 *
 * Plain, slow, FP64 code written from the paper's definitions.  Only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  Nothing here is shared with the HIP library.
 *
 * Build:  gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared
 * (no FMA contraction: the ordering and the partition must come out of the
 * exact IEEE operation sequence written below).
 */
#include "hmxo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int hmxo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Kernel functions (eq. (2) matrix entries; Section 6.2 model problem with a
 * length scale, and two exactly-low-rank test kernels).                     */
/* ------------------------------------------------------------------------ */
/* s K_1(s), written out from two textbook representations of K_1:
 *  - s <= 2: the power series of K_n at n = 1 (Abramowitz & Stegun 9.6.11),
 *      K_1(s) = 1/s + ln(s/2) I_1(s)
 *               - (s/4) sum_k (psi(k+1) + psi(k+2)) q^k / (k! (k+1)!),
 *      I_1(s) = (s/2) sum_k q^k / (k! (k+1)!),  q = s^2/4,
 *    psi(1) = -Euler's gamma, psi(k+1) = psi(k) + 1/k; the sums run until
 *    their terms no longer change them;
 *  - s > 2: the integral K_1(s) = int_0^inf exp(-s cosh t) cosh t dt
 *    (A&S 9.6.24) by the trapezoidal rule, written as
 *      s K_1(s) = s e^-s int_0^inf exp(-2 s sinh^2(t/2)) cosh t dt
 *    with step h = 0.25 / sqrt(s) (the integrand's width is about 1/sqrt(s)),
 *    summed until a term is below 1e-20 of the sum. */
double hmxo_xk1(double s)
{
    if (s == 0.0) return 1.0;
    if (s <= 2.0) {
        const double euler_gamma = 0.57721566490153286061;
        double q = 0.25 * s * s;
        double a = 1.0, s1 = 0.0, s2 = 0.0;
        double psi1 = -euler_gamma, psi2 = 1.0 - euler_gamma; /* psi(k+1), psi(k+2) */
        for (int k = 0; k < 60; ++k) {
            double n1 = s1 + a, n2 = s2 + (psi1 + psi2) * a;
            if (n1 == s1 && n2 == s2) break;
            s1 = n1;
            s2 = n2;
            a = a * q / ((double)(k + 1) * (double)(k + 2));
            psi1 += 1.0 / (double)(k + 1);
            psi2 += 1.0 / (double)(k + 2);
        }
        /* s K_1(s) = 1 + s ln(s/2) I_1(s) - (s^2/4) S2 with s I_1(s) = 2 q S1 */
        return 1.0 + 2.0 * q * log(0.5 * s) * s1 - q * s2;
    }
    double h = 0.25 / sqrt(s);
    double sum = 0.5; /* the t = 0 term, halved */
    for (int k = 1; k < 100000; ++k) {
        double t = k * h;
        double sh = sinh(0.5 * t);
        double term = exp(-2.0 * s * sh * sh) * cosh(t);
        sum += term;
        if (term < 1e-20 * sum) break;
    }
    return s * exp(-s) * h * sum;
}

double hmxo_kernel(int kind, double p0, const double* x, const double* y, int d)
{
    double r2 = 0.0, dot = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = x[k] - y[k];
        r2 += t * t;
        dot += x[k] * y[k];
    }
    switch (kind) {
    case HMXO_GAUSSIAN:
        return exp(-r2 / p0);
    case HMXO_MATERN32: {
        double s = sqrt(3.0) * sqrt(r2) / p0;
        return (1.0 + s) * exp(-s);
    }
    case HMXO_MATERN_NU1: {
        /* beta = 1 + d/2: the normalisation 2^(beta-1) Gamma(beta) */
        double beta = 1.0 + 0.5 * d;
        return hmxo_xk1(sqrt(r2) / p0) / (pow(2.0, beta - 1.0) * tgamma(beta));
    }
    case HMXO_CONST:
        return 1.0;
    case HMXO_LOWRANK:
        return (1.0 + dot) * (1.0 + dot);
    default:
        return NAN;
    }
}

/* entry (i, j) of the Morton-ordered matrix, coordinates from the d x n SoA */
static double entry(const double* soa, int64_t n, int d, int kind, double p0, int64_t i,
                    int64_t j)
{
    double x[3], y[3];
    for (int k = 0; k < d; ++k) {
        x[k] = soa[(int64_t)k * n + i];
        y[k] = soa[(int64_t)k * n + j];
    }
    return hmxo_kernel(kind, p0, x, y, d);
}

/* ------------------------------------------------------------------------ */
/* Z-order (Section 4.4, Algorithm 6)                                        */
/* ------------------------------------------------------------------------ */
int hmxo_global_box(const double* pts, int64_t n, int32_t d, double* lo, double* hi)
{
    if (n < 1 || d < 1 || d > 3) return -1;
    for (int k = 0; k < d; ++k) {
        lo[k] = pts[k];
        hi[k] = pts[k];
    }
    for (int64_t i = 1; i < n; ++i)
        for (int k = 0; k < d; ++k) {
            double v = pts[i * d + k];
            if (v < lo[k]) lo[k] = v;
            if (v > hi[k]) hi[k] = v;
        }
    return 0;
}

/* bits per dimension of the fixed-point representation */
static int morton_bits(int d)
{
    int b = 64 / d;
    return b < 32 ? b : 32;
}

int hmxo_morton(const double* pts, int64_t n, int32_t d, const double* lo, const double* hi,
                uint64_t* codes)
{
    if (n < 0 || d < 1 || d > 3) return -1;
    const int B = morton_bits(d);
    const double scale = ldexp(1.0, B);           /* 2^B, exact */
    const uint64_t qmax = (B == 64) ? ~0ull : ((1ull << B) - 1ull);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t q[3] = {0, 0, 0};
        for (int k = 0; k < d; ++k) {
            if (hi[k] == lo[k]) {
                q[k] = 0;
                continue;
            }
            /* fixed-point representation relative to the global box */
            double t = (pts[i * d + k] - lo[k]) / (hi[k] - lo[k]);
            double f = floor(t * scale);
            uint64_t v = (f >= (double)qmax) ? qmax : (uint64_t)f;
            q[k] = v;
        }
        /* interleave: bit b of dimension k lands at position b*d + (d-1-k) */
        uint64_t code = 0;
        for (int b = 0; b < B; ++b)
            for (int k = 0; k < d; ++k)
                if ((q[k] >> b) & 1ull) code |= 1ull << (b * d + (d - 1 - k));
        codes[i] = code;
    }
    return 0;
}

typedef struct {
    uint64_t code;
    int32_t idx;
} code_idx;

static int cmp_code_idx(const void* a, const void* b)
{
    const code_idx* x = (const code_idx*)a;
    const code_idx* y = (const code_idx*)b;
    if (x->code < y->code) return -1;
    if (x->code > y->code) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx); /* stable: original order on ties */
}

int hmxo_sort(const uint64_t* codes, int64_t n, int32_t* perm)
{
    if (n < 0) return -1;
    code_idx* a = (code_idx*)malloc(sizeof(code_idx) * (size_t)(n > 0 ? n : 1));
    if (!a) return -2;
    for (int64_t i = 0; i < n; ++i) {
        a[i].code = codes[i];
        a[i].idx = (int32_t)i;
    }
    qsort(a, (size_t)n, sizeof(code_idx), cmp_code_idx);
    for (int64_t i = 0; i < n; ++i) perm[i] = a[i].idx;
    free(a);
    return 0;
}

int hmxo_ordered_coords(const double* pts, int64_t n, int32_t d, const int32_t* perm, double* soa)
{
    for (int k = 0; k < d; ++k)
        for (int64_t i = 0; i < n; ++i) soa[(int64_t)k * n + i] = pts[(int64_t)perm[i] * d + k];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Cluster tree (Section 2.1, (C1)-(C4); split in halves of the Morton order) */
/* ------------------------------------------------------------------------ */
int64_t hmxo_cluster_tree(int64_t n, int32_t leaf, int64_t cap, int32_t* lo, int32_t* hi,
                          int32_t* depth, int64_t* child0)
{
    if (n < 1 || leaf < 1) return -1;
    /* count first: breadth-first expansion of [0, n) */
    int64_t count = 0;
    {
        int64_t qcap = 16, qn = 1, qh = 0;
        int64_t* qlo = (int64_t*)malloc(sizeof(int64_t) * qcap);
        int64_t* qhi = (int64_t*)malloc(sizeof(int64_t) * qcap);
        qlo[0] = 0;
        qhi[0] = n;
        while (qh < qn) {
            int64_t a = qlo[qh], b = qhi[qh];
            ++qh;
            ++count;
            if (b - a > leaf) {
                if (qn + 2 > qcap) {
                    qcap *= 2;
                    qlo = (int64_t*)realloc(qlo, sizeof(int64_t) * qcap);
                    qhi = (int64_t*)realloc(qhi, sizeof(int64_t) * qcap);
                }
                int64_t mid = a + (b - a) / 2;
                qlo[qn] = a;
                qhi[qn] = mid;
                ++qn;
                qlo[qn] = mid;
                qhi[qn] = b;
                ++qn;
            }
        }
        free(qlo);
        free(qhi);
    }
    if (cap < count) return count;
    /* fill in breadth-first order; children of node k appended at the tail */
    int64_t tail = 1;
    lo[0] = 0;
    hi[0] = (int32_t)n;
    depth[0] = 0;
    for (int64_t k = 0; k < count; ++k) {
        int64_t a = lo[k], b = hi[k];
        if (b - a > leaf) {
            int64_t mid = a + (b - a) / 2; /* the first half is the floor half */
            child0[k] = tail;
            lo[tail] = (int32_t)a;
            hi[tail] = (int32_t)mid;
            depth[tail] = depth[k] + 1;
            lo[tail + 1] = (int32_t)mid;
            hi[tail + 1] = (int32_t)b;
            depth[tail + 1] = depth[k] + 1;
            tail += 2;
        } else {
            child0[k] = -1;
        }
    }
    return count;
}

int hmxo_boxes(const double* soa, int64_t n, int32_t d, int64_t nnodes, const int32_t* lo,
               const int32_t* hi, double* bmin, double* bmax)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < nnodes; ++c) {
        for (int k = 0; k < d; ++k) {
            double mn = soa[(int64_t)k * n + lo[c]], mx = mn;
            for (int64_t i = lo[c] + 1; i < hi[c]; ++i) {
                double v = soa[(int64_t)k * n + i];
                if (v < mn) mn = v;
                if (v > mx) mx = v;
            }
            bmin[c * d + k] = mn;
            bmax[c * d + k] = mx;
        }
    }
    return 0;
}

/* eq. (3): min(diam Q_t, diam Q_s) <= eta dist(Q_t, Q_s), squared on both
 * sides (diam, dist >= 0), summed in dimension order. */
int hmxo_admissible(const double* amin, const double* amax, const double* bmin,
                    const double* bmax, int32_t d, double eta)
{
    double dt = 0.0, ds = 0.0, dist2 = 0.0;
    for (int k = 0; k < d; ++k) {
        double w = amax[k] - amin[k];
        dt += w * w;
    }
    for (int k = 0; k < d; ++k) {
        double w = bmax[k] - bmin[k];
        ds += w * w;
    }
    for (int k = 0; k < d; ++k) {
        double g1 = amin[k] - bmax[k];
        double g2 = bmin[k] - amax[k];
        if (g1 < 0.0) g1 = 0.0;
        if (g2 < 0.0) g2 = 0.0;
        double s = g1 * g1 + g2 * g2;
        dist2 += s;
    }
    double dmin = dt < ds ? dt : ds;
    return dmin <= (eta * eta) * dist2;
}

/* ------------------------------------------------------------------------ */
/* Block cluster tree (Algorithm 1) traversed level by level (Algorithm 4)   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t nn;
    int32_t *lo, *hi, *depth;
    int64_t* child0;
    double *bmin, *bmax;
} ctree;

static int ctree_make(ctree* t, const double* soa, int64_t n, int32_t d, int32_t leaf)
{
    int64_t cnt = hmxo_cluster_tree(n, leaf, 0, NULL, NULL, NULL, NULL);
    if (cnt < 1) return -1;
    t->nn = cnt;
    t->lo = (int32_t*)malloc(sizeof(int32_t) * cnt);
    t->hi = (int32_t*)malloc(sizeof(int32_t) * cnt);
    t->depth = (int32_t*)malloc(sizeof(int32_t) * cnt);
    t->child0 = (int64_t*)malloc(sizeof(int64_t) * cnt);
    t->bmin = (double*)malloc(sizeof(double) * cnt * d);
    t->bmax = (double*)malloc(sizeof(double) * cnt * d);
    if (!t->lo || !t->hi || !t->depth || !t->child0 || !t->bmin || !t->bmax) return -2;
    hmxo_cluster_tree(n, leaf, cnt, t->lo, t->hi, t->depth, t->child0);
    hmxo_boxes(soa, n, d, cnt, t->lo, t->hi, t->bmin, t->bmax);
    return 0;
}

static void ctree_free(ctree* t)
{
    free(t->lo);
    free(t->hi);
    free(t->depth);
    free(t->child0);
    free(t->bmin);
    free(t->bmax);
}

typedef struct {
    int64_t n, cap;
    int64_t* a; /* pairs of cluster-node ids */
} pairlist;

static void pl_push(pairlist* p, int64_t t, int64_t s)
{
    if (p->n + 1 > p->cap) {
        p->cap = p->cap ? 2 * p->cap : 64;
        p->a = (int64_t*)realloc(p->a, sizeof(int64_t) * 2 * p->cap);
    }
    p->a[2 * p->n] = t;
    p->a[2 * p->n + 1] = s;
    p->n++;
}

/* leaves with levels, as pairs of node ids */
typedef struct {
    pairlist adm, dense;
    int64_t *adm_level, *dense_level;
    int64_t level_sizes[64];
    int32_t nlev;
} partition;

static void part_free(partition* P)
{
    free(P->adm.a);
    free(P->dense.a);
    free(P->adm_level);
    free(P->dense_level);
}

/* T1: the row tree (tau), T2: the column tree (sigma); a square matrix
 * passes one tree twice */
static int part_make2(partition* P, const ctree* T1, const ctree* T2, int32_t d, int32_t leaf,
                      double eta)
{
    memset(P, 0, sizeof(*P));
    pairlist cur = {0, 0, NULL}, nxt = {0, 0, NULL};
    int64_t acap = 0, dcap = 0;
    pl_push(&cur, 0, 0); /* level 0 holds I x I */
    int lev = 0;
    while (cur.n > 0) {
        if (lev >= 64) return -3;
        P->level_sizes[lev] = cur.n;
        nxt.n = 0;
        for (int64_t q = 0; q < cur.n; ++q) {
            int64_t t = cur.a[2 * q], s = cur.a[2 * q + 1];
            int64_t mt = T1->hi[t] - T1->lo[t], ms = T2->hi[s] - T2->lo[s];
            if (hmxo_admissible(T1->bmin + t * d, T1->bmax + t * d, T2->bmin + s * d,
                                T2->bmax + s * d, d, eta)) {
                pl_push(&P->adm, t, s);
                if (P->adm.n > acap) {
                    acap = P->adm.cap;
                    P->adm_level = (int64_t*)realloc(P->adm_level, sizeof(int64_t) * acap);
                }
                P->adm_level[P->adm.n - 1] = lev;
            } else if (mt > leaf && ms > leaf) {
                /* children in the loop order of Algorithm 1: tau' outer, sigma' inner */
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) pl_push(&nxt, T1->child0[t] + a, T2->child0[s] + b);
            } else {
                pl_push(&P->dense, t, s);
                if (P->dense.n > dcap) {
                    dcap = P->dense.cap;
                    P->dense_level =
                        (int64_t*)realloc(P->dense_level, sizeof(int64_t) * dcap);
                }
                P->dense_level[P->dense.n - 1] = lev;
            }
        }
        pairlist tmp = cur;
        cur = nxt;
        nxt = tmp;
        ++lev;
    }
    P->nlev = lev;
    free(cur.a);
    free(nxt.a);
    return 0;
}

static int part_make(partition* P, const ctree* T, int32_t d, int32_t leaf, double eta)
{
    return part_make2(P, T, T, d, leaf, eta);
}

int hmxo_partition(const double* soa, int64_t n, int32_t d, int32_t leaf, double eta,
                   int64_t cap_adm, int32_t* adm, int64_t* n_adm, int64_t cap_dense,
                   int32_t* dense, int64_t* n_dense, int64_t* level_sizes, int32_t* n_levels)
{
    if (n < 1 || d < 1 || d > 3 || leaf < 1 || !(eta >= 0.0)) return -1;
    ctree T;
    if (ctree_make(&T, soa, n, d, leaf)) return -2;
    partition P;
    if (part_make(&P, &T, d, leaf, eta)) {
        ctree_free(&T);
        return -3;
    }
    *n_adm = P.adm.n;
    *n_dense = P.dense.n;
    *n_levels = P.nlev;
    for (int l = 0; l < P.nlev; ++l) level_sizes[l] = P.level_sizes[l];
    int rc = 0;
    if (P.adm.n > cap_adm || P.dense.n > cap_dense) rc = 1;
    if (rc == 0) {
        for (int64_t q = 0; q < P.adm.n; ++q) {
            int64_t t = P.adm.a[2 * q], s = P.adm.a[2 * q + 1];
            int32_t* o = adm + 5 * q;
            o[0] = T.lo[t];
            o[1] = T.hi[t];
            o[2] = T.lo[s];
            o[3] = T.hi[s];
            o[4] = (int32_t)P.adm_level[q];
        }
        for (int64_t q = 0; q < P.dense.n; ++q) {
            int64_t t = P.dense.a[2 * q], s = P.dense.a[2 * q + 1];
            int32_t* o = dense + 5 * q;
            o[0] = T.lo[t];
            o[1] = T.hi[t];
            o[2] = T.lo[s];
            o[3] = T.hi[s];
            o[4] = (int32_t)P.dense_level[q];
        }
    }
    part_free(&P);
    ctree_free(&T);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Adaptive cross approximation (Algorithm 2), column-first with partial    */
/* pivoting.  Column pivots (left to the implementation by the paper): the  */
/* first column is the sigma point nearest to the centre of tau's bounding  */
/* box; later ones the largest entry of the last row residual among unused  */
/* columns.  A column whose residual has no entry (over unused rows) above */
/* eps0 times the largest |entry| of the column itself adds no rank (the   */
/* residual is zero or rounding noise); the lowest unused column is tried  */
/* next, and after kmax such failed columns the block stops.               */
/* ------------------------------------------------------------------------ */

/* the sigma column whose point is nearest (squared distance, dimension
 * order, FP64) to the centre 0.5 (a + b) of tau's bounding box; lowest
 * index on ties */
static int64_t first_column(const double* soa, int64_t n, int d, int64_t tlo, int64_t thi,
                            int64_t slo, int64_t shi)
{
    double c[3];
    for (int k = 0; k < d; ++k) {
        double a = soa[(int64_t)k * n + tlo], b = a;
        for (int64_t i = tlo + 1; i < thi; ++i) {
            double v = soa[(int64_t)k * n + i];
            if (v < a) a = v;
            if (v > b) b = v;
        }
        c[k] = 0.5 * (a + b);
    }
    int64_t best = 0;
    double bd = INFINITY;
    for (int64_t q = slo; q < shi; ++q) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) {
            double t = soa[(int64_t)k * n + q] - c[k];
            s += t * t;
        }
        if (s < bd) {
            bd = s;
            best = q - slo;
        }
    }
    return best;
}
int hmxo_aca(const double* soa, int64_t n, int32_t d, int32_t kind, double p0, int64_t tlo,
             int64_t thi, int64_t slo, int64_t shi, int32_t kmax, double eps, double aca_eta,
             double eps0, int32_t fixed, int32_t r_start, double* U, double* V, int32_t* rank,
             int32_t* steps)
{
    return hmxo_aca_traced(soa, n, d, kind, p0, tlo, thi, slo, shi, kmax, eps, aca_eta, eps0,
                           fixed, r_start, U, V, rank, steps, NULL);
}

/* relative gap between the largest and the second largest |w_k| over the
 * unmarked k (1 when fewer than two remain): how close an argmax was to a tie */
static double pivot_margin(const double* w, const char* used, int64_t len)
{
    double b1 = -1.0, b2 = -1.0;
    for (int64_t k = 0; k < len; ++k) {
        if (used[k]) continue;
        const double a = fabs(w[k]);
        if (a > b1) {
            b2 = b1;
            b1 = a;
        } else if (a > b2) {
            b2 = a;
        }
    }
    if (b2 < 0.0 || !(b1 > 0.0)) return 1.0;
    return (b1 - b2) / b1;
}

int hmxo_aca_traced(const double* soa, int64_t n, int32_t d, int32_t kind, double p0,
                    int64_t tlo, int64_t thi, int64_t slo, int64_t shi, int32_t kmax, double eps,
                    double aca_eta, double eps0, int32_t fixed, int32_t r_start, double* U,
                    double* V, int32_t* rank, int32_t* steps, double* trace)
{
    const int64_t m = thi - tlo, nc = shi - slo;
    if (m < 1 || nc < 1 || kmax < 1) return -1;
    int64_t R = kmax;
    if (m < R) R = m;
    if (nc < R) R = nc;
    char* used_r = (char*)calloc((size_t)m, 1);
    char* used_c = (char*)calloc((size_t)nc, 1);
    double* uh = (double*)malloc(sizeof(double) * m);
    if (!used_r || !used_c || !uh) return -2;
    const double tol = eps * (1.0 - aca_eta) / (1.0 + eps);
    int64_t r = 0, ncols_used = 0, nfailed = 0;
    int64_t j = first_column(soa, n, d, tlo, thi, slo, shi);
    int32_t nsteps = 0;
    double S2 = 0.0;
    int one_shot = r_start > 0;
    int64_t target = one_shot ? (r_start < R ? r_start : R) : R;
    for (;;) {
        if (r >= target) {
            /* one-shot target reached: judge the last term, continue if it fails */
            if (!one_shot || r >= R) break;
            one_shot = 0;
            target = R;
            /* the test on the last computed term was not yet applied */
            double nu2 = 0.0, nv2 = 0.0;
            for (int64_t i = 0; i < m; ++i) nu2 += U[(r - 1) * m + i] * U[(r - 1) * m + i];
            for (int64_t q = 0; q < nc; ++q) nv2 += V[(r - 1) * nc + q] * V[(r - 1) * nc + q];
            if (sqrt(nu2 * nv2) <= tol * sqrt(S2)) break;
            continue;
        }
        /* residual column u^ = A[:, j] - sum_l u_l (v_l)_j */
        double colmax = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            double a = entry(soa, n, d, kind, p0, tlo + i, slo + j);
            if (fabs(a) > colmax) colmax = fabs(a);
            for (int64_t l = 0; l < r; ++l) a -= U[l * m + i] * V[l * nc + j];
            uh[i] = a;
        }
        used_c[j] = 1;
        ++ncols_used;
        ++nsteps;
        /* row pivot: largest |u^_i| over unused rows, lowest index on ties */
        int64_t ip = -1;
        double best = -1.0;
        for (int64_t i = 0; i < m; ++i)
            if (!used_r[i] && fabs(uh[i]) > best) {
                best = fabs(uh[i]);
                ip = i;
            }
        if (ip < 0 || best <= eps0 * colmax) {
            ++nfailed;
            if (ncols_used >= nc || nfailed >= kmax) break;
            int64_t q = 0;
            while (used_c[q]) ++q;
            j = q;
            continue;
        }
        if (trace) {
            trace[5 * r + 0] = (double)ip;
            trace[5 * r + 1] = (double)j;
            trace[5 * r + 2] = pivot_margin(uh, used_r, m);
            trace[5 * r + 3] = 0.0;
            trace[5 * r + 4] = 1.0;
        }
        const double piv = uh[ip];
        for (int64_t i = 0; i < m; ++i) U[r * m + i] = uh[i] / piv;
        /* residual row v = A[i_r, :]^T - sum_l (u_l)_{i_r} v_l */
        for (int64_t q = 0; q < nc; ++q) {
            double a = entry(soa, n, d, kind, p0, tlo + ip, slo + q);
            for (int64_t l = 0; l < r; ++l) a -= U[l * m + ip] * V[l * nc + q];
            V[r * nc + q] = a;
        }
        used_r[ip] = 1;
        /* ||S_r||_F^2 = ||S_{r-1}||_F^2 + 2 sum_l (u_r.u_l)(v_r.v_l) + |u_r|^2 |v_r|^2 */
        double nu2 = 0.0, nv2 = 0.0, cross = 0.0;
        for (int64_t i = 0; i < m; ++i) nu2 += U[r * m + i] * U[r * m + i];
        for (int64_t q = 0; q < nc; ++q) nv2 += V[r * nc + q] * V[r * nc + q];
        for (int64_t l = 0; l < r; ++l) {
            double du = 0.0, dv = 0.0;
            for (int64_t i = 0; i < m; ++i) du += U[r * m + i] * U[l * m + i];
            for (int64_t q = 0; q < nc; ++q) dv += V[r * nc + q] * V[l * nc + q];
            cross += du * dv;
        }
        S2 += 2.0 * cross + nu2 * nv2;
        if (trace) {
            trace[5 * r + 3] = sqrt(nu2 * nv2) / (tol * sqrt(S2));
            trace[5 * r + 4] = pivot_margin(V + r * nc, used_c, nc);
        }
        ++r;
        if (!fixed && !one_shot && sqrt(nu2 * nv2) <= tol * sqrt(S2)) break;
        /* next column pivot: largest |(v_r)_j| over unused columns */
        int64_t jp = -1;
        double bc = -1.0;
        for (int64_t q = 0; q < nc; ++q)
            if (!used_c[q] && fabs(V[(r - 1) * nc + q]) > bc) {
                bc = fabs(V[(r - 1) * nc + q]);
                jp = q;
            }
        if (jp < 0) break;
        j = jp;
    }
    *rank = (int32_t)r;
    if (steps) *steps = nsteps;
    free(used_r);
    free(used_c);
    free(uh);
    return 0;
}

int hmxo_dense_block(const double* soa, int64_t n, int32_t d, int32_t kind, double p0,
                     int64_t tlo, int64_t thi, int64_t slo, int64_t shi, double* A)
{
    const int64_t m = thi - tlo, nc = shi - slo;
    for (int64_t q = 0; q < nc; ++q)
        for (int64_t i = 0; i < m; ++i)
            A[q * m + i] = entry(soa, n, d, kind, p0, tlo + i, slo + q);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* H-matrix-vector product (Algorithm 3, flat over the leaf lists)           */
/* ------------------------------------------------------------------------ */
int hmxo_hmvp(const double* pts, int64_t n, int32_t d, int32_t kind, double p0, int32_t leaf,
              double eta, int32_t kmax, double eps, double aca_eta, double eps0, int32_t fixed,
              double sigma2, double alpha, double beta, const double* x, double* z,
              int64_t ranks_cap, int32_t* ranks, double* stats)
{
    return hmxo_hmvp_ex(pts, n, d, kind, p0, leaf, eta, kmax, eps, aca_eta, eps0, fixed, 0,
                        sigma2, alpha, beta, x, z, ranks_cap, ranks, stats);
}

/* admissible leaf q of the partition whose (first row, first column) is
 * (r0, c0): the leaves partition I x I, so the pair names one leaf */
typedef struct {
    int64_t r0, c0, q;
} leafkey;

static int leafkey_cmp(const void* a, const void* b)
{
    const leafkey* x = (const leafkey*)a;
    const leafkey* y = (const leafkey*)b;
    if (x->r0 != y->r0) return x->r0 < y->r0 ? -1 : 1;
    if (x->c0 != y->c0) return x->c0 < y->c0 ? -1 : 1;
    return 0;
}

/* symmetric = 1: the kernel matrix is symmetric and so is the partition
 * (Alg. 1 visits (tau, sigma) and (sigma, tau) alike), so only the leaf with
 * tau before sigma (or tau = sigma) is approximated and its mirror (sigma,
 * tau) uses the transposed factors, A|sigma x tau ~ V U^T. */
int hmxo_hmvp_ex(const double* pts, int64_t n, int32_t d, int32_t kind, double p0, int32_t leaf,
                 double eta, int32_t kmax, double eps, double aca_eta, double eps0, int32_t fixed,
                 int32_t symmetric, double sigma2, double alpha, double beta, const double* x,
                 double* z, int64_t ranks_cap, int32_t* ranks, double* stats)
{
    if (n < 1 || d < 1 || d > 3 || leaf < 1 || !(eta >= 0.0) || kmax < 1) return -1;
    double lo[3], hi[3];
    hmxo_global_box(pts, n, d, lo, hi);
    uint64_t* codes = (uint64_t*)malloc(sizeof(uint64_t) * n);
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * n);
    double* soa = (double*)malloc(sizeof(double) * n * d);
    double* xm = (double*)malloc(sizeof(double) * n);
    double* zm = (double*)calloc((size_t)n, sizeof(double));
    if (!codes || !perm || !soa || !xm || !zm) return -2;
    hmxo_morton(pts, n, d, lo, hi, codes);
    hmxo_sort(codes, n, perm);
    hmxo_ordered_coords(pts, n, d, perm, soa);
    for (int64_t k = 0; k < n; ++k) xm[k] = x[perm[k]];

    ctree T;
    if (ctree_make(&T, soa, n, d, leaf)) return -2;
    partition P;
    if (part_make(&P, &T, d, leaf, eta)) return -3;

    double sum_rank = 0.0, dense_entries = 0.0, factor_entries = 0.0;
    int nthr = hmxo_num_threads();
    double* zpriv = (double*)calloc((size_t)nthr * (size_t)n, sizeof(double));
    if (!zpriv) return -2;

#pragma omp parallel reduction(+ : sum_rank, dense_entries, factor_entries)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* zt = zpriv + (int64_t)tid * n;
        /* admissible leaves: z|tau += U (V^T x|sigma); with the symmetric
         * far field a primary leaf also gives its mirror z|sigma += V (U^T x|tau) */
#pragma omp for schedule(dynamic, 1) nowait
        for (int64_t q = 0; q < P.adm.n; ++q) {
            int64_t t = P.adm.a[2 * q], s = P.adm.a[2 * q + 1];
            int64_t tlo = T.lo[t], thi = T.hi[t], slo = T.lo[s], shi = T.hi[s];
            if (symmetric && tlo > slo) continue; /* a mirror: done by its primary */
            int64_t m = thi - tlo, nc = shi - slo;
            int64_t R = kmax;
            double* U = (double*)malloc(sizeof(double) * m * R);
            double* V = (double*)malloc(sizeof(double) * nc * R);
            int32_t rk = 0;
            hmxo_aca(soa, n, d, kind, p0, tlo, thi, slo, shi, kmax, eps, aca_eta, eps0, fixed, 0,
                     U, V, &rk, NULL);
            if (ranks && q < ranks_cap) ranks[q] = rk;
            for (int64_t l = 0; l < rk; ++l) {
                double tl = 0.0;
                for (int64_t jj = 0; jj < nc; ++jj) tl += V[l * nc + jj] * xm[slo + jj];
                for (int64_t i = 0; i < m; ++i) zt[tlo + i] += U[l * m + i] * tl;
            }
            if (symmetric && tlo != slo) {
                for (int64_t l = 0; l < rk; ++l) {
                    double tl = 0.0;
                    for (int64_t i = 0; i < m; ++i) tl += U[l * m + i] * xm[tlo + i];
                    for (int64_t jj = 0; jj < nc; ++jj) zt[slo + jj] += V[l * nc + jj] * tl;
                }
                sum_rank += rk;
            }
            sum_rank += rk;
            factor_entries += (double)rk * (double)(m + nc);
            free(U);
            free(V);
        }
        /* dense leaves: z|tau += A|tau x sigma x|sigma */
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < P.dense.n; ++q) {
            int64_t t = P.dense.a[2 * q], s = P.dense.a[2 * q + 1];
            int64_t tlo = T.lo[t], thi = T.hi[t], slo = T.lo[s], shi = T.hi[s];
            for (int64_t i = tlo; i < thi; ++i) {
                double acc = 0.0;
                for (int64_t jj = slo; jj < shi; ++jj)
                    acc += entry(soa, n, d, kind, p0, i, jj) * xm[jj];
                zt[i] += acc;
            }
            dense_entries += (double)(thi - tlo) * (double)(shi - slo);
        }
    }
    for (int th = 0; th < nthr; ++th)
        for (int64_t k = 0; k < n; ++k) zm[k] += zpriv[(int64_t)th * n + k];
    for (int64_t k = 0; k < n; ++k) {
        int64_t p = perm[k];
        double hz = zm[k] + sigma2 * xm[k];
        z[p] = alpha * hz + (beta != 0.0 ? beta * z[p] : 0.0);
    }
    if (symmetric && ranks && P.adm.n <= ranks_cap && P.adm.n > 0) {
        /* a mirror's rank is its primary's */
        leafkey* K = (leafkey*)malloc(sizeof(leafkey) * P.adm.n);
        if (!K) return -2;
        for (int64_t q = 0; q < P.adm.n; ++q) {
            K[q].r0 = T.lo[P.adm.a[2 * q]];
            K[q].c0 = T.lo[P.adm.a[2 * q + 1]];
            K[q].q = q;
        }
        qsort(K, (size_t)P.adm.n, sizeof(leafkey), leafkey_cmp);
        for (int64_t q = 0; q < P.adm.n; ++q) {
            const int64_t r0 = T.lo[P.adm.a[2 * q]], c0 = T.lo[P.adm.a[2 * q + 1]];
            if (r0 <= c0) continue;
            leafkey want = {c0, r0, 0};
            const leafkey* hit =
                (const leafkey*)bsearch(&want, K, (size_t)P.adm.n, sizeof(leafkey), leafkey_cmp);
            if (!hit) {
                free(K);
                return -4; /* the partition has no mirror for this leaf */
            }
            ranks[q] = ranks[hit->q];
        }
        free(K);
    }
    if (stats) {
        stats[0] = (double)P.adm.n;
        stats[1] = (double)P.dense.n;
        stats[2] = sum_rank;
        stats[3] = dense_entries;
        stats[4] = factor_entries;
        stats[5] = (double)P.nlev;
        stats[6] = 0.0;
        stats[7] = 0.0;
    }
    free(zpriv);
    part_free(&P);
    ctree_free(&T);
    free(codes);
    free(perm);
    free(soa);
    free(xm);
    free(zm);
    return 0;
}

int hmxo_dense_matvec(const double* pts, int64_t n, int32_t d, int32_t kind, double p0,
                      double sigma2, const double* x, const int64_t* rows, int64_t nrows,
                      double* z)
{
    int64_t cnt = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < cnt; ++q) {
        int64_t i = rows ? rows[q] : q;
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) acc += hmxo_kernel(kind, p0, pts + i * d, pts + j * d, d) * x[j];
        z[q] = acc + sigma2 * x[i];
    }
    return 0;
}

/* The same dense product for m right-hand sides at once (X: n x m
 * row-major, Z: rows x m); each matrix entry is evaluated once and every
 * column is summed in the order of hmxo_dense_matvec. */
int hmxo_dense_matmat(const double* pts, int64_t n, int32_t d, int32_t kind, double p0,
                      double sigma2, const double* X, int32_t m, const int64_t* rows,
                      int64_t nrows, double* Z)
{
    if (m < 1 || m > 64) return -1;
    int64_t cnt = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < cnt; ++q) {
        int64_t i = rows ? rows[q] : q;
        double acc[64];
        for (int c = 0; c < m; ++c) acc[c] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double a = hmxo_kernel(kind, p0, pts + i * d, pts + j * d, d);
            for (int c = 0; c < m; ++c) acc[c] += a * X[j * m + c];
        }
        for (int c = 0; c < m; ++c) Z[q * m + c] = acc[c] + sigma2 * X[i * m + c];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Rectangular A_{phi, Y1 x Y2} (the kernel matrix between two point sets,  */
/* Section 6): each set ordered by its own Morton codes (Algorithm 6 in its */
/* own bounding box) and clustered in its own tree; Algorithm 1 from the    */
/* single block Y1 x Y2 with eq. (3).  Leaves report rows in Y1's Morton    */
/* order and columns in Y2's.                                               */
/* ------------------------------------------------------------------------ */

/* z = A_{Y1 x Y2} x, the plain dense product (x: n2 entries, z: n1) */
int hmxo_dense_matvec_rect(const double* pts1, int64_t n1, const double* pts2, int64_t n2,
                           int32_t d, int32_t kind, double p0, const double* x, double* z)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n1; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < n2; ++j)
            acc += hmxo_kernel(kind, p0, pts1 + i * d, pts2 + j * d, d) * x[j];
        z[i] = acc;
    }
    return 0;
}

int hmxo_partition_rect(const double* soa1, int64_t n1, const double* soa2, int64_t n2,
                        int32_t d, int32_t leaf, double eta, int64_t cap_adm, int32_t* adm,
                        int64_t* n_adm, int64_t cap_dense, int32_t* dense, int64_t* n_dense,
                        int64_t* level_sizes, int32_t* n_levels)
{
    if (n1 < 1 || n2 < 1 || d < 1 || d > 3 || leaf < 1 || !(eta >= 0.0)) return -1;
    ctree T1, T2;
    if (ctree_make(&T1, soa1, n1, d, leaf) || ctree_make(&T2, soa2, n2, d, leaf)) return -2;
    partition P;
    if (part_make2(&P, &T1, &T2, d, leaf, eta)) return -3;
    *n_adm = P.adm.n;
    *n_dense = P.dense.n;
    *n_levels = P.nlev;
    for (int l = 0; l < P.nlev; ++l) level_sizes[l] = P.level_sizes[l];
    int rc = (P.adm.n > cap_adm || P.dense.n > cap_dense) ? 1 : 0;
    for (int k = 0; rc == 0 && k < 2; ++k) {
        const pairlist* L = k ? &P.dense : &P.adm;
        const int64_t* lev = k ? P.dense_level : P.adm_level;
        int32_t* out = k ? dense : adm;
        for (int64_t q = 0; q < L->n; ++q) {
            int64_t t = L->a[2 * q], s = L->a[2 * q + 1];
            int32_t* o = out + 5 * q;
            o[0] = T1.lo[t];
            o[1] = T1.hi[t];
            o[2] = T2.lo[s];
            o[3] = T2.hi[s];
            o[4] = (int32_t)lev[q];
        }
    }
    part_free(&P);
    ctree_free(&T1);
    ctree_free(&T2);
    return rc;
}

/* z = alpha H x + beta z for the H-matrix of A_{Y1 x Y2} (x: n2 entries in
 * Y2's original order, z: n1 in Y1's); the ACA runs on the union of the two
 * ordered sets (rows first, columns after them), each block as in
 * hmxo_hmvp_ex */
int hmxo_hmvp_rect(const double* pts1, int64_t n1, const double* pts2, int64_t n2, int32_t d,
                   int32_t kind, double p0, int32_t leaf, double eta, int32_t kmax, double eps,
                   double aca_eta, double eps0, int32_t fixed, double alpha, double beta,
                   const double* x, double* z, int64_t ranks_cap, int32_t* ranks, double* stats)
{
    if (n1 < 1 || n2 < 1 || d < 1 || d > 3 || leaf < 1 || !(eta >= 0.0) || kmax < 1) return -1;
    const int64_t nu = n1 + n2;
    double lo1[3], hi1[3], lo2[3], hi2[3];
    hmxo_global_box(pts1, n1, d, lo1, hi1);
    hmxo_global_box(pts2, n2, d, lo2, hi2);
    uint64_t* c1 = (uint64_t*)malloc(sizeof(uint64_t) * n1);
    uint64_t* c2 = (uint64_t*)malloc(sizeof(uint64_t) * n2);
    int32_t* perm1 = (int32_t*)malloc(sizeof(int32_t) * n1);
    int32_t* perm2 = (int32_t*)malloc(sizeof(int32_t) * n2);
    double* soa1 = (double*)malloc(sizeof(double) * n1 * d);
    double* soa2 = (double*)malloc(sizeof(double) * n2 * d);
    double* soa = (double*)malloc(sizeof(double) * nu * d);
    double* xm = (double*)malloc(sizeof(double) * n2);
    double* zm = (double*)calloc((size_t)n1, sizeof(double));
    if (!c1 || !c2 || !perm1 || !perm2 || !soa1 || !soa2 || !soa || !xm || !zm) return -2;
    hmxo_morton(pts1, n1, d, lo1, hi1, c1);
    hmxo_morton(pts2, n2, d, lo2, hi2, c2);
    hmxo_sort(c1, n1, perm1);
    hmxo_sort(c2, n2, perm2);
    hmxo_ordered_coords(pts1, n1, d, perm1, soa1);
    hmxo_ordered_coords(pts2, n2, d, perm2, soa2);
    for (int k = 0; k < d; ++k) {
        memcpy(soa + (int64_t)k * nu, soa1 + (int64_t)k * n1, sizeof(double) * n1);
        memcpy(soa + (int64_t)k * nu + n1, soa2 + (int64_t)k * n2, sizeof(double) * n2);
    }
    for (int64_t j = 0; j < n2; ++j) xm[j] = x[perm2[j]];

    ctree T1, T2;
    if (ctree_make(&T1, soa1, n1, d, leaf) || ctree_make(&T2, soa2, n2, d, leaf)) return -2;
    partition P;
    if (part_make2(&P, &T1, &T2, d, leaf, eta)) return -3;

    double sum_rank = 0.0, dense_entries = 0.0, factor_entries = 0.0;
    int nthr = hmxo_num_threads();
    double* zpriv = (double*)calloc((size_t)nthr * (size_t)n1, sizeof(double));
    if (!zpriv) return -2;
#pragma omp parallel reduction(+ : sum_rank, dense_entries, factor_entries)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* zt = zpriv + (int64_t)tid * n1;
#pragma omp for schedule(dynamic, 1) nowait
        for (int64_t q = 0; q < P.adm.n; ++q) {
            int64_t t = P.adm.a[2 * q], s = P.adm.a[2 * q + 1];
            int64_t tlo = T1.lo[t], thi = T1.hi[t], slo = T2.lo[s], shi = T2.hi[s];
            int64_t m = thi - tlo, nc = shi - slo;
            double* U = (double*)malloc(sizeof(double) * m * kmax);
            double* V = (double*)malloc(sizeof(double) * nc * kmax);
            int32_t rk = 0;
            hmxo_aca(soa, nu, d, kind, p0, tlo, thi, n1 + slo, n1 + shi, kmax, eps, aca_eta,
                     eps0, fixed, 0, U, V, &rk, NULL);
            if (ranks && q < ranks_cap) ranks[q] = rk;
            for (int64_t l = 0; l < rk; ++l) {
                double tl = 0.0;
                for (int64_t jj = 0; jj < nc; ++jj) tl += V[l * nc + jj] * xm[slo + jj];
                for (int64_t i = 0; i < m; ++i) zt[tlo + i] += U[l * m + i] * tl;
            }
            sum_rank += rk;
            factor_entries += (double)rk * (double)(m + nc);
            free(U);
            free(V);
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < P.dense.n; ++q) {
            int64_t t = P.dense.a[2 * q], s = P.dense.a[2 * q + 1];
            int64_t tlo = T1.lo[t], thi = T1.hi[t], slo = T2.lo[s], shi = T2.hi[s];
            for (int64_t i = tlo; i < thi; ++i) {
                double acc = 0.0;
                for (int64_t jj = slo; jj < shi; ++jj)
                    acc += entry(soa, nu, d, kind, p0, i, n1 + jj) * xm[jj];
                zt[i] += acc;
            }
            dense_entries += (double)(thi - tlo) * (double)(shi - slo);
        }
    }
    for (int th = 0; th < nthr; ++th)
        for (int64_t k = 0; k < n1; ++k) zm[k] += zpriv[(int64_t)th * n1 + k];
    for (int64_t k = 0; k < n1; ++k) {
        int64_t p = perm1[k];
        z[p] = alpha * zm[k] + (beta != 0.0 ? beta * z[p] : 0.0);
    }
    if (stats) {
        stats[0] = (double)P.adm.n;
        stats[1] = (double)P.dense.n;
        stats[2] = sum_rank;
        stats[3] = dense_entries;
        stats[4] = factor_entries;
        stats[5] = (double)P.nlev;
        stats[6] = 0.0;
        stats[7] = 0.0;
    }
    free(zpriv);
    part_free(&P);
    ctree_free(&T1);
    ctree_free(&T2);
    free(c1);
    free(c2);
    free(perm1);
    free(perm2);
    free(soa1);
    free(soa2);
    free(soa);
    free(xm);
    free(zm);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Stored-mode H-matrix-vector product restricted to the Morton-order rows  */
/* [row_lo, row_hi): every leaf whose tau meets the range is built (ACA or  */
/* dense entries) and stored, then applied.  z receives (H x)_k for the     */
/* rows in Morton order.  times: [order+partition s, build s, apply s,      */
/* stored entries, blocks].  Used as a bounded CPU sample of a workload.    */
/* ------------------------------------------------------------------------ */
#include <time.h>

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

typedef struct {
    int64_t tlo, thi, slo, shi, r0, r1; /* block and the rows of it kept */
    int32_t adm, rank;
    double *U, *V, *A;
} stored_block;

int hmxo_hmvp_rows(const double* pts, int64_t n, int32_t d, int32_t kind, double p0,
                   int32_t leaf, double eta, int32_t kmax, double eps, double aca_eta,
                   double eps0, int32_t fixed, int64_t row_lo, int64_t row_hi, const double* x,
                   double* z, int32_t* perm_out, double* times)
{
    if (n < 1 || d < 1 || d > 3 || leaf < 1 || row_lo < 0 || row_hi > n || row_lo >= row_hi)
        return -1;
    double t0 = now_s();
    double lo[3], hi[3];
    hmxo_global_box(pts, n, d, lo, hi);
    uint64_t* codes = (uint64_t*)malloc(sizeof(uint64_t) * n);
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * n);
    double* soa = (double*)malloc(sizeof(double) * n * d);
    double* xm = (double*)malloc(sizeof(double) * n);
    if (!codes || !perm || !soa || !xm) return -2;
    hmxo_morton(pts, n, d, lo, hi, codes);
    hmxo_sort(codes, n, perm);
    hmxo_ordered_coords(pts, n, d, perm, soa);
    for (int64_t k = 0; k < n; ++k) xm[k] = x[perm[k]];
    if (perm_out)
        for (int64_t k = 0; k < n; ++k) perm_out[k] = perm[k];
    ctree T;
    if (ctree_make(&T, soa, n, d, leaf)) return -2;
    partition P;
    if (part_make(&P, &T, d, leaf, eta)) return -3;
    /* blocks meeting the rows */
    int64_t nb = 0;
    stored_block* B = (stored_block*)malloc(sizeof(stored_block) * (P.adm.n + P.dense.n + 1));
    for (int pass = 0; pass < 2; ++pass) {
        pairlist* L = pass == 0 ? &P.adm : &P.dense;
        for (int64_t q = 0; q < L->n; ++q) {
            int64_t t = L->a[2 * q], s = L->a[2 * q + 1];
            int64_t a = T.lo[t], b = T.hi[t];
            if (b <= row_lo || a >= row_hi) continue;
            stored_block* sb = &B[nb++];
            sb->tlo = a;
            sb->thi = b;
            sb->slo = T.lo[s];
            sb->shi = T.hi[s];
            sb->r0 = a > row_lo ? a : row_lo;
            sb->r1 = b < row_hi ? b : row_hi;
            sb->adm = pass == 0;
            sb->rank = 0;
            sb->U = sb->V = sb->A = NULL;
        }
    }
    double t1 = now_s();
    double entries = 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : entries)
    for (int64_t q = 0; q < nb; ++q) {
        stored_block* sb = &B[q];
        int64_t m = sb->thi - sb->tlo, nc = sb->shi - sb->slo, mr = sb->r1 - sb->r0;
        if (sb->adm) {
            double* U = (double*)malloc(sizeof(double) * m * kmax);
            double* V = (double*)malloc(sizeof(double) * nc * kmax);
            int32_t rk = 0;
            hmxo_aca(soa, n, d, kind, p0, sb->tlo, sb->thi, sb->slo, sb->shi, kmax, eps, aca_eta,
                     eps0, fixed, 0, U, V, &rk, NULL);
            /* keep the rows of U in the range */
            sb->U = (double*)malloc(sizeof(double) * (mr * rk + 1));
            for (int64_t l = 0; l < rk; ++l)
                for (int64_t i = 0; i < mr; ++i) sb->U[l * mr + i] = U[l * m + (sb->r0 - sb->tlo) + i];
            sb->V = V;
            sb->rank = rk;
            free(U);
            entries += (double)rk * (double)(mr + nc);
        } else {
            sb->A = (double*)malloc(sizeof(double) * mr * nc);
            for (int64_t jj = 0; jj < nc; ++jj)
                for (int64_t i = 0; i < mr; ++i)
                    sb->A[jj * mr + i] = entry(soa, n, d, kind, p0, sb->r0 + i, sb->slo + jj);
            entries += (double)mr * (double)nc;
        }
    }
    double t2 = now_s();
    const int64_t nr = row_hi - row_lo;
    int nthr = hmxo_num_threads();
    double* zp = (double*)calloc((size_t)nthr * (size_t)nr, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* zt = zp + (int64_t)tid * nr;
#pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < nb; ++q) {
            stored_block* sb = &B[q];
            int64_t nc = sb->shi - sb->slo, mr = sb->r1 - sb->r0, off = sb->r0 - row_lo;
            if (sb->adm) {
                for (int64_t l = 0; l < sb->rank; ++l) {
                    double tl = 0.0;
                    for (int64_t jj = 0; jj < nc; ++jj) tl += sb->V[l * nc + jj] * xm[sb->slo + jj];
                    for (int64_t i = 0; i < mr; ++i) zt[off + i] += sb->U[l * mr + i] * tl;
                }
            } else {
                for (int64_t jj = 0; jj < nc; ++jj) {
                    double xv = xm[sb->slo + jj];
                    for (int64_t i = 0; i < mr; ++i) zt[off + i] += sb->A[jj * mr + i] * xv;
                }
            }
        }
    }
    for (int64_t i = 0; i < nr; ++i) {
        double acc = 0.0;
        for (int th = 0; th < nthr; ++th) acc += zp[(int64_t)th * nr + i];
        z[i] = acc;
    }
    double t3 = now_s();
    if (times) {
        times[0] = t1 - t0;
        times[1] = t2 - t1;
        times[2] = t3 - t2;
        times[3] = entries;
        times[4] = (double)nb;
    }
    for (int64_t q = 0; q < nb; ++q) {
        free(B[q].U);
        free(B[q].V);
        free(B[q].A);
    }
    free(B);
    free(zp);
    part_free(&P);
    ctree_free(&T);
    free(codes);
    free(perm);
    free(soa);
    free(xm);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Conjugate gradients (Hestenes-Stiefel) on the dense system               */
/* (A + sigma2 I) x = b with the brute-force product: the reference for the */
/* kernel ridge regression solve.  x starts at 0; stops when |r|/|b| <= tol */
/* (recurrence residual).  Returns 0 converged, 1 not converged, 2 breakdown */
/* ------------------------------------------------------------------------ */
int hmxo_cg_dense(const double* pts, int64_t n, int32_t d, int32_t kind, double p0,
                  double sigma2, const double* b, double* x, double tol, int32_t max_iter,
                  int32_t* iters, double* rel_res)
{
    double* r = (double*)malloc(sizeof(double) * n);
    double* p = (double*)malloc(sizeof(double) * n);
    double* q = (double*)malloc(sizeof(double) * n);
    if (!r || !p || !q) return -2;
    double bb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        x[i] = 0.0;
        r[i] = b[i];
        p[i] = b[i];
        bb += b[i] * b[i];
    }
    double rr = bb;
    int rc = 1;
    int32_t it = 0;
    double res = bb > 0.0 ? 1.0 : 0.0;
    if (bb == 0.0) rc = 0;
    while (rc == 1 && it < max_iter) {
        hmxo_dense_matvec(pts, n, d, kind, p0, sigma2, p, NULL, 0, q);
        double pq = 0.0;
        for (int64_t i = 0; i < n; ++i) pq += p[i] * q[i];
        ++it;
        if (!(pq > 0.0)) {
            rc = 2;
            break;
        }
        const double alpha = rr / pq;
        double rr2 = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
            rr2 += r[i] * r[i];
        }
        res = sqrt(rr2 / bb);
        if (res <= tol) {
            rc = 0;
            break;
        }
        const double beta = rr2 / rr;
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rr = rr2;
    }
    if (iters) *iters = it;
    if (rel_res) *rel_res = res;
    free(r);
    free(p);
    free(q);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Rank predictor: an MLP 8 -> 64 -> 64 -> 64 -> 1 with ReLU, trained on     */
/* (block features, ACA rank) pairs with the pinball (quantile) loss and    */
/* Adam.  Parameters are packed as W1 (64x8, row-major), b1, W2 (64x64),    */
/* b2, W3 (64x64), b3, W4 (1x64), b4.                                       */
/* ------------------------------------------------------------------------ */
#define MLP_IN 8
#define MLP_H 64
#define MLP_NPARAM (MLP_H * MLP_IN + MLP_H + 2 * (MLP_H * MLP_H + MLP_H) + MLP_H + 1)

int hmxo_mlp_nparams(void) { return MLP_NPARAM; }

typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4;
} mlp_view;

static mlp_view mlp_unpack(const double* w)
{
    mlp_view v;
    v.W1 = w;
    v.b1 = v.W1 + MLP_H * MLP_IN;
    v.W2 = v.b1 + MLP_H;
    v.b2 = v.W2 + MLP_H * MLP_H;
    v.W3 = v.b2 + MLP_H;
    v.b3 = v.W3 + MLP_H * MLP_H;
    v.W4 = v.b3 + MLP_H;
    v.b4 = v.W4 + MLP_H;
    return v;
}

/* one sample: pre-activations z1..z3, activations a1..a3 (64 each), output */
static double mlp_sample(const mlp_view* p, const double* x, double* z1, double* a1, double* z2,
                         double* a2, double* z3, double* a3)
{
    for (int i = 0; i < MLP_H; ++i) {
        double s = p->b1[i];
        for (int k = 0; k < MLP_IN; ++k) s += p->W1[i * MLP_IN + k] * x[k];
        z1[i] = s;
        a1[i] = s > 0.0 ? s : 0.0;
    }
    for (int i = 0; i < MLP_H; ++i) {
        double s = p->b2[i];
        for (int k = 0; k < MLP_H; ++k) s += p->W2[i * MLP_H + k] * a1[k];
        z2[i] = s;
        a2[i] = s > 0.0 ? s : 0.0;
    }
    for (int i = 0; i < MLP_H; ++i) {
        double s = p->b3[i];
        for (int k = 0; k < MLP_H; ++k) s += p->W3[i * MLP_H + k] * a2[k];
        z3[i] = s;
        a3[i] = s > 0.0 ? s : 0.0;
    }
    double o = p->b4[0];
    for (int k = 0; k < MLP_H; ++k) o += p->W4[k] * a3[k];
    return o;
}

int hmxo_mlp_forward(const double* w, const double* X, int64_t B, double* out)
{
    mlp_view p = mlp_unpack(w);
    double z1[MLP_H], a1[MLP_H], z2[MLP_H], a2[MLP_H], z3[MLP_H], a3[MLP_H];
    for (int64_t b = 0; b < B; ++b) out[b] = mlp_sample(&p, X + b * MLP_IN, z1, a1, z2, a2, z3, a3);
    return 0;
}

/* pinball loss rho_q(u) = u (q - [u < 0]) with u = y - prediction, averaged
 * over the batch; grad (packed like the parameters) by back-propagation.
 * At u = 0 the subgradient q is used. */
int hmxo_mlp_loss_grad(const double* w, const double* X, const double* y, int64_t B, double q,
                       double* loss, double* grad)
{
    mlp_view p = mlp_unpack(w);
    memset(grad, 0, sizeof(double) * MLP_NPARAM);
    double *gW1 = grad, *gb1 = gW1 + MLP_H * MLP_IN, *gW2 = gb1 + MLP_H, *gb2 = gW2 + MLP_H * MLP_H;
    double *gW3 = gb2 + MLP_H, *gb3 = gW3 + MLP_H * MLP_H, *gW4 = gb3 + MLP_H, *gb4 = gW4 + MLP_H;
    double L = 0.0;
    double z1[MLP_H], a1[MLP_H], z2[MLP_H], a2[MLP_H], z3[MLP_H], a3[MLP_H];
    double d3[MLP_H], d2[MLP_H], d1[MLP_H];
    for (int64_t b = 0; b < B; ++b) {
        const double* x = X + b * MLP_IN;
        const double o = mlp_sample(&p, x, z1, a1, z2, a2, z3, a3);
        const double u = y[b] - o;
        const double ind = u < 0.0 ? 1.0 : 0.0;
        L += u * (q - ind);
        const double dout = -(q - ind) / (double)B; /* dL/d prediction */
        gb4[0] += dout;
        for (int k = 0; k < MLP_H; ++k) {
            gW4[k] += dout * a3[k];
            d3[k] = z3[k] > 0.0 ? dout * p.W4[k] : 0.0;
        }
        for (int i = 0; i < MLP_H; ++i) {
            gb3[i] += d3[i];
            for (int k = 0; k < MLP_H; ++k) gW3[i * MLP_H + k] += d3[i] * a2[k];
        }
        for (int k = 0; k < MLP_H; ++k) {
            double s = 0.0;
            for (int i = 0; i < MLP_H; ++i) s += p.W3[i * MLP_H + k] * d3[i];
            d2[k] = z2[k] > 0.0 ? s : 0.0;
        }
        for (int i = 0; i < MLP_H; ++i) {
            gb2[i] += d2[i];
            for (int k = 0; k < MLP_H; ++k) gW2[i * MLP_H + k] += d2[i] * a1[k];
        }
        for (int k = 0; k < MLP_H; ++k) {
            double s = 0.0;
            for (int i = 0; i < MLP_H; ++i) s += p.W2[i * MLP_H + k] * d2[i];
            d1[k] = z1[k] > 0.0 ? s : 0.0;
        }
        for (int i = 0; i < MLP_H; ++i) {
            gb1[i] += d1[i];
            for (int k = 0; k < MLP_IN; ++k) gW1[i * MLP_IN + k] += d1[i] * x[k];
        }
    }
    *loss = L / (double)B;
    return 0;
}

/* Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps), t >= 1 */
int hmxo_mlp_adam(double* w, double* m, double* v, const double* g, int64_t n, int64_t t,
                  double lr, double b1, double b2, double eps)
{
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        w[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
    return 0;
}

/* Geometric features of a block tau x sigma (boxes a..b, sizes m, n):
 * [log2 m, log2 n, diam_tau / l, diam_sigma / l, dist / l,
 *  min(diam) / max(dist, 1e-12), d, log10 l^2] with l the kernel length. */
int hmxo_features(const double* ta, const double* tb, const double* sa, const double* sb, int32_t d,
                  int64_t m, int64_t n, double ell, double* f)
{
    double dt = 0.0, ds = 0.0, dist2 = 0.0;
    for (int k = 0; k < d; ++k) {
        dt += (tb[k] - ta[k]) * (tb[k] - ta[k]);
        ds += (sb[k] - sa[k]) * (sb[k] - sa[k]);
        double g1 = ta[k] - sb[k], g2 = sa[k] - tb[k];
        if (g1 < 0.0) g1 = 0.0;
        if (g2 < 0.0) g2 = 0.0;
        dist2 += g1 * g1 + g2 * g2;
    }
    const double Dt = sqrt(dt), Ds = sqrt(ds), dist = sqrt(dist2);
    f[0] = log2((double)m);
    f[1] = log2((double)n);
    f[2] = Dt / ell;
    f[3] = Ds / ell;
    f[4] = dist / ell;
    f[5] = (Dt < Ds ? Dt : Ds) / (dist > 1e-12 ? dist : 1e-12);
    f[6] = (double)d;
    f[7] = log10(ell * ell);
    return 0;
}
