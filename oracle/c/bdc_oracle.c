/*
 * Plain C oracle for the Blahut-Arimoto iteration on the finite-length binary
 * deletion channel BDC_d.  TEST INFRASTRUCTURE ONLY: the GPU library never links
 * or calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it (through oracle/native.py).
 *
 * Conventions (same as oracle/bdc.py): x_0 is the most significant bit of the
 * input index; the output y of length k has rank (2^k - 1) + bits(y) with y_0 most
 * significant.  Arithmetic is FP64, in nats.
 *
 * What each function writes out:
 *   bdc_row_brute     emb(y,x) for every y, by enumerating every position subset
 *                     S of {0..n-1} and counting x_S (Section 2.2, definition of
 *                     the exact deletion channel's numerator).
 *   bdc_csr_*         the channel W(y|x) = emb(y,x) d^(n-k) (1-d)^k stored as a
 *                     sparse matrix, and the BA iteration of Section 2.3 on it.
 *   bdc_product_*     closed forms for a product input law p(x) = prod_i P(x_i):
 *                     r(y) = sum_S prod_j P(x_{s_j} = y_j).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint32_t rank_of(uint32_t bits, int k) { return ((1u << k) - 1u) + bits; }

static void weights(int n, double d, double *w) {
    for (int k = 0; k <= n; ++k) {
        /* 0^0 = 1 at d = 0 or d = 1 */
        double a = (n - k == 0) ? 1.0 : pow(d, (double)(n - k));
        double b = (k == 0) ? 1.0 : pow(1.0 - d, (double)k);
        w[k] = a * b;
    }
}

static inline int length_of_rank(uint32_t r) {
    int k = 0;
    while (((1u << (k + 1)) - 1u) <= r) ++k;
    return k;
}

/* ---- brute-force row over position subsets ------------------------------ */

typedef struct {
    int n;
    uint32_t x;
    uint32_t *dense;   /* counts indexed by rank, all zero on entry and exit */
    uint32_t *touched; /* ranks seen, in first-seen order */
    int ntouched;
} row_state;

/* Position i is either deleted or kept; every subset is visited once. */
static void subsets(row_state *s, int i, uint32_t y, int k) {
    if (i == s->n) {
        uint32_t r = rank_of(y, k);
        if (s->dense[r] == 0) s->touched[s->ntouched++] = r;
        s->dense[r] += 1;
        return;
    }
    subsets(s, i + 1, y, k);
    subsets(s, i + 1, (y << 1) | ((s->x >> (s->n - 1 - i)) & 1u), k + 1);
}

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* Fill (rank, emb) of row x sorted by rank; returns nnz (or -nnz-1 if cap is
 * too small, in which case nothing beyond cap is written). */
static int row_into(int n, uint32_t x, uint32_t *dense, uint32_t *touched,
                    uint32_t *rank_out, uint32_t *emb_out, int cap) {
    row_state s = {n, x, dense, touched, 0};
    subsets(&s, 0, 0u, 0);
    qsort(touched, (size_t)s.ntouched, sizeof(uint32_t), cmp_u32);
    int nnz = s.ntouched;
    for (int i = 0; i < nnz; ++i) {
        uint32_t r = touched[i];
        if (i < cap) {
            rank_out[i] = r;
            emb_out[i] = dense[r];
        }
        dense[r] = 0;
    }
    return nnz <= cap ? nnz : -nnz - 1;
}

static size_t row_cap(int n) { /* distinct subsequences of an n-bit string <= 2^(n+1)-1 */
    return ((size_t)1 << (n + 1)) - 1;
}

int bdc_row_brute(int n, uint32_t x, uint32_t *rank_out, uint32_t *emb_out, int cap) {
    if (n < 0 || n > 24) return -1;
    uint32_t *dense = (uint32_t *)calloc(row_cap(n), sizeof(uint32_t));
    uint32_t *touched = (uint32_t *)malloc(row_cap(n) * sizeof(uint32_t));
    if (!dense || !touched) { free(dense); free(touched); return -2; }
    int r = row_into(n, x, dense, touched, rank_out, emb_out, cap);
    free(dense); free(touched);
    return r;
}

/* Many rows at once (OpenMP over rows).  Row i is written at offset i*cap;
 * nnz_out[i] receives its nnz (negative as above if cap was too small). */
int bdc_rows_brute(int n, const uint32_t *xs, int count, uint32_t *rank_out,
                   uint32_t *emb_out, int cap, int *nnz_out) {
    if (n < 0 || n > 24) return -1;
    int err = 0;
#pragma omp parallel
    {
        uint32_t *dense = (uint32_t *)calloc(row_cap(n), sizeof(uint32_t));
        uint32_t *touched = (uint32_t *)malloc(row_cap(n) * sizeof(uint32_t));
        if (!dense || !touched) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int i = 0; i < count; ++i)
                nnz_out[i] = row_into(n, xs[i], dense, touched, rank_out + (size_t)i * cap,
                                      emb_out + (size_t)i * cap, cap);
        }
        free(dense); free(touched);
    }
    return err;
}

/* ---- CSR channel (n <= 16) ---------------------------------------------- */

/* Pass 1: nnz of every row. */
int bdc_csr_rowcounts(int n, int64_t *indptr) {
    if (n < 0 || n > 16) return -1;
    const uint32_t X = 1u << n;
    int err = 0;
    indptr[0] = 0;
#pragma omp parallel
    {
        uint32_t *dense = (uint32_t *)calloc(row_cap(n), sizeof(uint32_t));
        uint32_t *touched = (uint32_t *)malloc(row_cap(n) * sizeof(uint32_t));
        if (!dense || !touched) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int64_t x = 0; x < (int64_t)X; ++x) {
                row_state s = {n, (uint32_t)x, dense, touched, 0};
                subsets(&s, 0, 0u, 0);
                for (int i = 0; i < s.ntouched; ++i) dense[touched[i]] = 0;
                indptr[x + 1] = s.ntouched;
            }
        }
        free(dense); free(touched);
    }
    if (err) return err;
    for (uint32_t x = 0; x < X; ++x) indptr[x + 1] += indptr[x];
    return 0;
}

/* Pass 2: column ranks and embedding counts, each row sorted by rank. */
int bdc_csr_fill(int n, const int64_t *indptr, uint32_t *indices, uint32_t *emb) {
    if (n < 0 || n > 16) return -1;
    const uint32_t X = 1u << n;
    int err = 0;
#pragma omp parallel
    {
        uint32_t *dense = (uint32_t *)calloc(row_cap(n), sizeof(uint32_t));
        uint32_t *touched = (uint32_t *)malloc(row_cap(n) * sizeof(uint32_t));
        if (!dense || !touched) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int64_t x = 0; x < (int64_t)X; ++x) {
                int cap = (int)(indptr[x + 1] - indptr[x]);
                int r = row_into(n, (uint32_t)x, dense, touched, indices + indptr[x],
                                 emb + indptr[x], cap);
                if (r != cap) {
#pragma omp atomic write
                    err = -3;
                }
            }
        }
        free(dense); free(touched);
    }
    return err;
}

/* One evaluation of Section 2.3 steps 1 and 2(a) at X = exp(lp):
 *   Y(y) = sum_x X(x) W(y|x);  D(x) = sum_y W(y|x) log(W(y|x)/Y(y));
 *   L = log sum_x X(x) e^{D(x)};  U = max_x D(x);  I = sum_x X(x) D(x).
 * lp need not be normalised.  If floor_nats > 0, lp is first raised to at least
 * max(lp) - floor_nats.  Y is accumulated as Y e^{-max lp} to avoid underflow.
 * Outputs: D_out[2^n] (nats), lui[3] = {L, U, I} (nats); q_out (optional,
 * 2^(n+1)-1) receives Y(y) e^{-max lp} of the normalised law. */
int bdc_csr_eval(int n, double d, const int64_t *indptr, const uint32_t *indices,
                 const uint32_t *emb, const double *lp_in, double floor_nats,
                 double *q_out, double *D_out, double *lui) {
    if (n < 0 || n > 16) return -1;
    const int64_t X = (int64_t)1 << n;
    const int64_t Y = ((int64_t)1 << (n + 1)) - 1;
    double w[32];
    weights(n, d, w);
    double *lp = (double *)malloc((size_t)X * sizeof(double));
    double *q = (double *)calloc((size_t)Y, sizeof(double));
    if (!lp || !q) { free(lp); free(q); return -2; }
    /* normalise (and floor) */
    double m = -INFINITY;
    for (int64_t x = 0; x < X; ++x) m = fmax(m, lp_in[x]);
    for (int64_t x = 0; x < X; ++x) lp[x] = (floor_nats > 0) ? fmax(lp_in[x], m - floor_nats) : lp_in[x];
    m = -INFINITY;
    for (int64_t x = 0; x < X; ++x) m = fmax(m, lp[x]);
    double z = 0.0;
    for (int64_t x = 0; x < X; ++x) z += exp(lp[x] - m);
    double lz = m + log(z);
    for (int64_t x = 0; x < X; ++x) lp[x] -= lz;
    m -= lz;
    /* step 1: output law, scaled by e^{-m} */
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double *qpart = (double *)calloc((size_t)nt * (size_t)Y, sizeof(double));
    if (!qpart) { free(lp); free(q); return -2; }
#pragma omp parallel
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        double *qt = qpart + (size_t)t * Y;
#pragma omp for schedule(static)
        for (int64_t x = 0; x < X; ++x) {
            double px = exp(lp[x] - m);
            for (int64_t e = indptr[x]; e < indptr[x + 1]; ++e) {
                uint32_t r = indices[e];
                qt[r] += px * (double)emb[e] * w[length_of_rank(r)];
            }
        }
    }
    for (int t = 0; t < nt; ++t)
        for (int64_t r = 0; r < Y; ++r) q[r] += qpart[(size_t)t * Y + r];
    free(qpart);
    /* step 2(a): D(x), in nats; the scale e^{-m} of q is undone by "- m * rowsum" */
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < X; ++x) {
        double acc = 0.0, rowsum = 0.0;
        for (int64_t e = indptr[x]; e < indptr[x + 1]; ++e) {
            uint32_t r = indices[e];
            double Wv = (double)emb[e] * w[length_of_rank(r)];
            if (Wv > 0.0) {
                acc += Wv * log(Wv / q[r]);
                rowsum += Wv;
            }
        }
        D_out[x] = acc - m * rowsum;
    }
    double am = -INFINITY, U = -INFINITY, I = 0.0;
    for (int64_t x = 0; x < X; ++x) {
        am = fmax(am, lp[x] + D_out[x]);
        U = fmax(U, D_out[x]);
        I += exp(lp[x]) * D_out[x];
    }
    double s = 0.0;
    for (int64_t x = 0; x < X; ++x) s += exp(lp[x] + D_out[x] - am);
    lui[0] = am + log(s);
    lui[1] = U;
    lui[2] = I;
    if (q_out) memcpy(q_out, q, (size_t)Y * sizeof(double));
    free(lp); free(q);
    return 0;
}

/* `iters` BA updates in place: log X <- log X + D - L (Section 2.3 step 2(b)). */
int bdc_csr_iterate(int n, double d, const int64_t *indptr, const uint32_t *indices,
                    const uint32_t *emb, double *lp, int iters) {
    const int64_t X = (int64_t)1 << n;
    double *D = (double *)malloc((size_t)X * sizeof(double));
    if (!D) return -2;
    for (int it = 0; it < iters; ++it) {
        double lui[3];
        int rc = bdc_csr_eval(n, d, indptr, indices, emb, lp, 0.0, NULL, D, lui);
        if (rc) { free(D); return rc; }
        /* bdc_csr_eval normalised a private copy; normalise lp the same way */
        double m = -INFINITY;
        for (int64_t x = 0; x < X; ++x) m = fmax(m, lp[x]);
        double z = 0.0;
        for (int64_t x = 0; x < X; ++x) z += exp(lp[x] - m);
        double lz = m + log(z);
        for (int64_t x = 0; x < X; ++x) lp[x] = lp[x] - lz + D[x] - lui[0];
    }
    free(D);
    return 0;
}

/* ---- product input laws -------------------------------------------------- */

/* r(y) = sum_x p(x) emb(y,x) for p(x) = prod_i P(x_i), P(x_i = 1) = pi1[i]:
 * the sum over position sets S of prod_j P(x_{s_j} = y_j), by the recursion
 * f_i(t) = f_{i-1}(t) + f_{i-1}(t-1) P(x_{i-1} = y_{t-1}). */
double bdc_product_r(int n, const double *pi1, uint32_t ybits, int k) {
    double f[33];
    f[0] = 1.0;
    for (int t = 1; t <= k; ++t) f[t] = 0.0;
    for (int i = 0; i < n; ++i)
        for (int t = k; t >= 1; --t) {
            int yb = (int)((ybits >> (k - t)) & 1u);
            double pb = yb ? pi1[i] : 1.0 - pi1[i];
            f[t] += f[t - 1] * pb;
        }
    return f[k];
}

int bdc_product_r_many(int n, const double *pi1, const uint32_t *ranks, int count, double *out) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < count; ++i) {
        int k = length_of_rank(ranks[i]);
        out[i] = bdc_product_r(n, pi1, ranks[i] - ((1u << k) - 1u), k);
    }
    return 0;
}

/* D(x) = sum_y W(y|x) log(W(y|x)/q(y)) with q(y) = w_k r(y) from the product law
 * (a normalised law, so no rescaling is needed).  Row emb from subsets. */
int bdc_product_D(int n, double d, const double *pi1, const uint32_t *xs, int count,
                  double *D_out, double *Dd_out) {
    if (n < 1 || n > 22) return -1;
    double w[32], sk[32];
    weights(n, d, w);
    for (int k = 0; k <= n; ++k) sk[k] = (d > 0.0 && d < 1.0) ? (n - k) / d - k / (1.0 - d) : 0.0;
    int err = 0;
#pragma omp parallel
    {
        uint32_t *dense = (uint32_t *)calloc(row_cap(n), sizeof(uint32_t));
        uint32_t *touched = (uint32_t *)malloc(row_cap(n) * sizeof(uint32_t));
        uint32_t *rk = (uint32_t *)malloc(row_cap(n) * sizeof(uint32_t));
        uint32_t *em = (uint32_t *)malloc(row_cap(n) * sizeof(uint32_t));
        if (!dense || !touched || !rk || !em) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int i = 0; i < count; ++i) {
                int nnz = row_into(n, xs[i], dense, touched, rk, em, (int)row_cap(n));
                double acc = 0.0, accd = 0.0;
                for (int e = 0; e < nnz; ++e) {
                    int k = length_of_rank(rk[e]);
                    double r = bdc_product_r(n, pi1, rk[e] - ((1u << k) - 1u), k);
                    double Wv = (double)em[e] * w[k];
                    if (Wv > 0.0) {
                        double t = Wv * log(Wv / (w[k] * r));
                        acc += t;
                        accd += sk[k] * t;
                    }
                }
                D_out[i] = acc;
                if (Dd_out) Dd_out[i] = accd;
            }
        }
        free(dense); free(touched); free(rk); free(em);
    }
    return err;
}

int bdc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---- both sweeps of one BA iteration on a sample of input rows ----------- */

/* For each sampled x: its row by brute force over position subsets, then
 *   q_part(y) += p(x) W(y|x)                                 (Section 2.3 step 1)
 *   D(x) = sum_y W(y|x) log(W(y|x) / q(y)), q given in q_full (step 2(a)).
 * q_part has one slice of 2^(n+1)-1 doubles per OpenMP thread (the caller sums
 * them).  Returns the number of nonzeros visited, or a negative error. */
long long bdc_sample_sweeps(int n, double d, const double *p, const uint32_t *xs, int count,
                            const double *q_full, double *q_part, double *D_out) {
    if (n < 1 || n > 22) return -1;
    double w[32];
    weights(n, d, w);
    const size_t Y = row_cap(n);
    long long total = 0;
    int err = 0;
#pragma omp parallel reduction(+ : total)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        double *qt = q_part + (size_t)t * Y;
        uint32_t *dense = (uint32_t *)calloc(Y, sizeof(uint32_t));
        uint32_t *touched = (uint32_t *)malloc(Y * sizeof(uint32_t));
        uint32_t *rk = (uint32_t *)malloc(Y * sizeof(uint32_t));
        uint32_t *em = (uint32_t *)malloc(Y * sizeof(uint32_t));
        if (!dense || !touched || !rk || !em) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int i = 0; i < count; ++i) {
                int nnz = row_into(n, xs[i], dense, touched, rk, em, (int)Y);
                double acc = 0.0;
                const double px = p[xs[i]];
                for (int e = 0; e < nnz; ++e) {
                    const double Wv = (double)em[e] * w[length_of_rank(rk[e])];
                    qt[rk[e]] += px * Wv;
                    if (Wv > 0.0) acc += Wv * log(Wv / q_full[rk[e]]);
                }
                D_out[i] = acc;
                total += nnz;
            }
        }
        free(dense); free(touched); free(rk); free(em);
    }
    return err ? err : total;
}
