/*
 * Plain, serial, obviously-correct CPU oracle for the triangular-solve path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test suite, the smoke check and the CPU baseline
 * leg of the benchmark load it.  It shares no code, header, table or helper
 * with the GPU path.
 *
 * Every routine works on CSR (0-based, int32 indices), in double precision
 * unless its name ends in _f32, in the natural row order, with no blocking,
 * fusion or reordering beyond what the cited definition states.  Build with
 * -O2 -ffp-contract=off so that no fused multiply-add changes the rounding.
 *
 * Return codes: 0 ok, -1 entry on the wrong side of the diagonal, -2 missing
 * diagonal, -3 zero pivot, -4 allocation failure, -5 bad argument.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void orc_free(void *p) { free(p); }

/* ------------------------------------------------------------------------ */
/* Triangular solves: eq. (1) of Section 2, L y = b then U x = y, written as  */
/* plain forward / backward substitution.  Vectors are [n][nrhs], RHS index   */
/* fastest.  Off-diagonal terms are subtracted in ascending column order.     */
/* ------------------------------------------------------------------------ */

int orc_lower_solve(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                    int unit, int32_t nrhs, const double *b, double *x)
{
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0;
        int have_d = 0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] > i) return -1;
            if (ci[p] == i) { d = v[p]; have_d = 1; }
        }
        if (!unit && !have_d) return -2;
        for (int32_t r = 0; r < nrhs; ++r) {
            double s = b[(int64_t)i * nrhs + r];
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
                int32_t j = ci[p];
                if (j < i) s = s - v[p] * x[(int64_t)j * nrhs + r];
            }
            x[(int64_t)i * nrhs + r] = unit ? s : s / d;
        }
    }
    return 0;
}

int orc_upper_solve(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                    int unit, int32_t nrhs, const double *b, double *x)
{
    for (int32_t i = n - 1; i >= 0; --i) {
        double d = 0.0;
        int have_d = 0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < i) return -1;
            if (ci[p] == i) { d = v[p]; have_d = 1; }
        }
        if (!unit && !have_d) return -2;
        for (int32_t r = 0; r < nrhs; ++r) {
            double s = b[(int64_t)i * nrhs + r];
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
                int32_t j = ci[p];
                if (j > i) s = s - v[p] * x[(int64_t)j * nrhs + r];
            }
            x[(int64_t)i * nrhs + r] = unit ? s : s / d;
        }
    }
    return 0;
}

/* Single-precision substitution: FP32 factors, FP32 vectors, FP32 sums.  This
 * is the arithmetic the mixed-precision preconditioner promises. */
int orc_lower_solve_f32(int32_t n, const int32_t *rp, const int32_t *ci, const float *v,
                        int unit, int32_t nrhs, const float *b, float *x)
{
    for (int32_t i = 0; i < n; ++i) {
        float d = 0.0f;
        int have_d = 0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] > i) return -1;
            if (ci[p] == i) { d = v[p]; have_d = 1; }
        }
        if (!unit && !have_d) return -2;
        for (int32_t r = 0; r < nrhs; ++r) {
            float s = b[(int64_t)i * nrhs + r];
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
                int32_t j = ci[p];
                if (j < i) s = s - v[p] * x[(int64_t)j * nrhs + r];
            }
            x[(int64_t)i * nrhs + r] = unit ? s : s / d;
        }
    }
    return 0;
}

int orc_upper_solve_f32(int32_t n, const int32_t *rp, const int32_t *ci, const float *v,
                        int unit, int32_t nrhs, const float *b, float *x)
{
    for (int32_t i = n - 1; i >= 0; --i) {
        float d = 0.0f;
        int have_d = 0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < i) return -1;
            if (ci[p] == i) { d = v[p]; have_d = 1; }
        }
        if (!unit && !have_d) return -2;
        for (int32_t r = 0; r < nrhs; ++r) {
            float s = b[(int64_t)i * nrhs + r];
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
                int32_t j = ci[p];
                if (j > i) s = s - v[p] * x[(int64_t)j * nrhs + r];
            }
            x[(int64_t)i * nrhs + r] = unit ? s : s / d;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Levels, eq. (2) of Section 2.2, by Kahn peeling of the dependency DAG.    */
/* Row i depends on row j when the (off-diagonal) entry (i, j) is stored:     */
/* j < i for a lower, j > i for an upper triangle.  Round 1 takes every row   */
/* with no dependency; removing them, round 2 takes the rows that are then    */
/* free, and so on.  The round number is the row's level, which equals the    */
/* longest-path level of eq. (2) with the diagonal excluded.                  */
/* ------------------------------------------------------------------------ */

int orc_levels_kahn(int32_t n, const int32_t *rp, const int32_t *ci, int upper,
                    int32_t *level, int32_t *nlev_out)
{
    int32_t *indeg = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *sptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    int64_t nnz = rp[n];
    int32_t *succ = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *frontier = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    if (!indeg || !sptr || !succ || !cur || !frontier || !next) {
        free(indeg); free(sptr); free(succ); free(cur); free(frontier); free(next);
        return -4;
    }
    /* dependency counts and successor lists (j -> i) */
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            int32_t j = ci[p];
            if (j == i) continue;
            if ((!upper && j > i) || (upper && j < i)) {
                free(indeg); free(sptr); free(succ); free(cur); free(frontier); free(next);
                return -1;
            }
            indeg[i] += 1;
            sptr[j + 1] += 1;
        }
    }
    for (int32_t j = 0; j < n; ++j) sptr[j + 1] += sptr[j];
    memcpy(cur, sptr, sizeof(int32_t) * (size_t)n);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] != i) succ[cur[ci[p]]++] = i;

    int32_t nf = 0;
    for (int32_t i = 0; i < n; ++i)
        if (indeg[i] == 0) frontier[nf++] = i;
    int32_t round = 0, done = 0;
    while (nf > 0) {
        round += 1;
        int32_t nn = 0;
        for (int32_t f = 0; f < nf; ++f) {
            int32_t j = frontier[f];
            level[j] = round;
            done += 1;
            for (int32_t q = sptr[j]; q < sptr[j + 1]; ++q) {
                int32_t i = succ[q];
                if (--indeg[i] == 0) next[nn++] = i;
            }
        }
        int32_t *t = frontier; frontier = next; next = t;
        nf = nn;
    }
    *nlev_out = round;
    free(indeg); free(sptr); free(succ); free(cur); free(frontier); free(next);
    return done == n ? 0 : -5;
}

/* ------------------------------------------------------------------------ */
/* Sparse matrix-vector product y = A x (multi-RHS), ascending entry order.   */
/* ------------------------------------------------------------------------ */

void orc_spmv(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
              int32_t nrhs, const double *x, double *y)
{
    for (int32_t i = 0; i < n; ++i)
        for (int32_t r = 0; r < nrhs; ++r) {
            double s = 0.0;
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
                s = s + v[p] * x[(int64_t)ci[p] * nrhs + r];
            y[(int64_t)i * nrhs + r] = s;
        }
}

/* ------------------------------------------------------------------------ */
/* SOR sweeps (the Gauss-Seidel smoothers Section 1 lists among the users of  */
/* triangular solves), elementwise textbook form: row by row,                 */
/*   x_i <- (1 - omega) x_i + omega (b_i - sum_{j != i} a_ij x_j) / a_ii,     */
/* in place, so rows before i already hold their new values.  A forward sweep */
/* runs i = 0..n-1; a symmetric sweep follows it with i = n-1..0.             */
/* ------------------------------------------------------------------------ */

static int sor_row(int32_t i, const int32_t *rp, const int32_t *ci, const double *v, double omega,
                   int32_t nrhs, const double *b, double *x)
{
    double d = 0.0;
    int have_d = 0;
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
        if (ci[p] == i) { d = v[p]; have_d = 1; }
    if (!have_d) return -2;
    if (d == 0.0) return -3;
    for (int32_t r = 0; r < nrhs; ++r) {
        double sigma = 0.0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] != i) sigma = sigma + v[p] * x[(int64_t)ci[p] * nrhs + r];
        const double xi = x[(int64_t)i * nrhs + r];
        x[(int64_t)i * nrhs + r] = (1.0 - omega) * xi + omega * (b[(int64_t)i * nrhs + r] - sigma) / d;
    }
    return 0;
}

int orc_sor(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, double omega, int32_t nrhs,
            const double *b, double *x, int32_t sweeps, int symmetric)
{
    if (nrhs < 1 || sweeps < 0) return -5;
    for (int32_t k = 0; k < sweeps; ++k) {
        for (int32_t i = 0; i < n; ++i) {
            int rc = sor_row(i, rp, ci, v, omega, nrhs, b, x);
            if (rc) return rc;
        }
        if (symmetric)
            for (int32_t i = n - 1; i >= 0; --i) {
                int rc = sor_row(i, rp, ci, v, omega, nrhs, b, x);
                if (rc) return rc;
            }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Incomplete factorizations of Section 3 (Saad's textbook forms).           */
/* ------------------------------------------------------------------------ */

/* Numeric IKJ elimination restricted to a given pattern.  `rp/ci` is the
 * factor pattern (rows sorted ascending, diagonal present), `a` holds A's
 * values scattered into that pattern (zero at fill positions) and is
 * overwritten with L (strict lower part, unit diagonal implied) and U (upper
 * part with diagonal).  For each row i and each k < i in ascending order:
 * a_ik /= a_kk, then a_ij -= a_ik * a_kj for every j > k present in both row
 * k and row i. */
static int ikj_numeric(int32_t n, const int32_t *rp, const int32_t *ci, double *a)
{
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *dptr = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!pos || !dptr) { free(pos); free(dptr); return -4; }
    for (int32_t j = 0; j < n; ++j) pos[j] = -1;
    for (int32_t i = 0; i < n; ++i) {
        dptr[i] = -1;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] == i) dptr[i] = p;
        if (dptr[i] < 0) { free(pos); free(dptr); return -2; }
    }
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) pos[ci[p]] = p;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            int32_t k = ci[p];
            if (k >= i) break;
            double piv = a[dptr[k]];
            if (piv == 0.0 || !isfinite(piv)) { free(pos); free(dptr); return -3; }
            a[p] = a[p] / piv;
            for (int32_t q = dptr[k] + 1; q < rp[k + 1]; ++q) {
                int32_t j = ci[q];
                if (pos[j] >= 0) a[pos[j]] = a[pos[j]] - a[p] * a[q];
            }
        }
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) pos[ci[p]] = -1;
        double d = a[dptr[i]];
        if (d == 0.0 || !isfinite(d)) { free(pos); free(dptr); return -3; }
    }
    free(pos);
    free(dptr);
    return 0;
}

/* ILU(0): no fill-in; the factor pattern is A's pattern.  Output values on
 * A's pattern (L strictly below, U on and above the diagonal). */
int orc_ilu0(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, double *lu)
{
    memcpy(lu, v, sizeof(double) * (size_t)rp[n]);
    return ikj_numeric(n, rp, ci, lu);
}

/* ILU(k) symbolic phase by level of fill: an entry of A has level 0; a fill
 * entry (i, j) created through pivot k gets level lev(i,k) + lev(k,j) + 1 and
 * keeps the minimum over all k; entries with level > K are not kept.  Row i's
 * candidates are visited in ascending k, including fill entries created
 * earlier in the same row.  Allocates the factor pattern; the numeric phase
 * then runs IKJ on it.  Outputs malloc'ed arrays (free with orc_free). */
int orc_iluk(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t K,
             int32_t **out_rp, int32_t **out_ci, double **out_v)
{
    int32_t *frp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *lev = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);   /* current row levels */
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *row = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);   /* current row columns */
    int64_t cap = (int64_t)rp[n] * 2 + 16, nz = 0;
    int32_t *fci = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int32_t *flev = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int32_t *fdiag = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!frp || !lev || !mark || !row || !fci || !flev || !fdiag) goto oom;
    for (int32_t j = 0; j < n; ++j) mark[j] = 0;
    frp[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t len = 0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            row[len++] = ci[p];
            mark[ci[p]] = 1;
            lev[ci[p]] = 0;
        }
        if (!mark[i]) { row[len++] = i; mark[i] = 1; lev[i] = 0; }
        /* visit pivots k < i in ascending order; the row set grows */
        int32_t done_k = -1;
        for (;;) {
            int32_t k = n;
            for (int32_t t = 0; t < len; ++t)
                if (row[t] > done_k && row[t] < i && row[t] < k) k = row[t];
            if (k == n) break;
            done_k = k;
            int32_t lik = lev[k];
            for (int64_t q = fdiag[k] + 1; q < frp[k + 1]; ++q) {
                int32_t j = fci[q];
                int32_t nl = lik + flev[q] + 1;
                if (nl > K) continue;
                if (!mark[j]) { mark[j] = 1; lev[j] = nl; row[len++] = j; }
                else if (nl < lev[j]) lev[j] = nl;
            }
        }
        /* sort the row's columns ascending (insertion sort; rows are short) */
        for (int32_t a = 1; a < len; ++a) {
            int32_t c = row[a], b = a - 1;
            while (b >= 0 && row[b] > c) { row[b + 1] = row[b]; --b; }
            row[b + 1] = c;
        }
        if (nz + len > cap) {
            cap = (nz + len) * 2;
            int32_t *t1 = (int32_t *)realloc(fci, sizeof(int32_t) * (size_t)cap);
            if (!t1) goto oom;
            fci = t1;
            int32_t *t2 = (int32_t *)realloc(flev, sizeof(int32_t) * (size_t)cap);
            if (!t2) goto oom;
            flev = t2;
        }
        for (int32_t t = 0; t < len; ++t) {
            fci[nz + t] = row[t];
            flev[nz + t] = lev[row[t]];
            if (row[t] == i) fdiag[i] = (int32_t)(nz + t);
            mark[row[t]] = 0;
        }
        nz += len;
        frp[i + 1] = (int32_t)nz;
    }
    double *fv = (double *)calloc((size_t)nz + 1, sizeof(double));
    if (!fv) goto oom;
    /* scatter A's values into the pattern */
    for (int32_t i = 0; i < n; ++i) {
        int32_t q = frp[i];
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            while (fci[q] < ci[p]) ++q;
            fv[q] = v[p];
        }
    }
    free(lev); free(mark); free(row); free(flev); free(fdiag);
    int rc = ikj_numeric(n, frp, fci, fv);
    *out_rp = frp; *out_ci = fci; *out_v = fv;
    return rc;
oom:
    free(frp); free(lev); free(mark); free(row); free(fci); free(flev); free(fdiag);
    return -4;
}

/* ILUT(p, tau) with dual dropping (Saad's textbook algorithm): for row i,
 * with tau_i = tau * ||a_i||_2, load w = a_i; for k < i in ascending order
 * over the current non-zeros of w: w_k /= u_kk; drop w_k if |w_k| < tau_i,
 * else w -= w_k * u_k (the strict upper part of U's row k).  Then drop every
 * off-diagonal |w_j| < tau_i, keep the p largest magnitudes in the L part and
 * the p largest in the strict U part (ties to the smaller column index), and
 * always keep the diagonal.  Outputs L (strict lower) and U (diagonal first)
 * as separate malloc'ed CSR arrays. */
typedef struct { double mag; int32_t col; } orc_cand;

static int cand_cmp(const void *a, const void *b)
{
    const orc_cand *x = (const orc_cand *)a, *y = (const orc_cand *)b;
    if (x->mag > y->mag) return -1;
    if (x->mag < y->mag) return 1;
    return (x->col < y->col) ? -1 : (x->col > y->col);
}

static int col_cmp(const void *a, const void *b)
{
    const orc_cand *x = (const orc_cand *)a, *y = (const orc_cand *)b;
    return (x->col < y->col) ? -1 : (x->col > y->col);
}

int orc_ilut(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t p,
             double tau, int32_t **lrp, int32_t **lci, double **lv,
             int32_t **urp, int32_t **uci, double **uv)
{
    double *w = (double *)calloc((size_t)n, sizeof(double));
    int32_t *nzf = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    int32_t *lst = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    orc_cand *cand = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)n);
    int64_t lcap = (int64_t)n * (p + 1) + 16, ucap = (int64_t)n * (p + 2) + 16, ln = 0, un = 0;
    int32_t *Lrp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *Urp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *Lci = (int32_t *)malloc(sizeof(int32_t) * (size_t)lcap);
    int32_t *Uci = (int32_t *)malloc(sizeof(int32_t) * (size_t)ucap);
    double *Lv = (double *)malloc(sizeof(double) * (size_t)lcap);
    double *Uv = (double *)malloc(sizeof(double) * (size_t)ucap);
    int rc = 0;
    if (!w || !nzf || !lst || !cand || !Lrp || !Urp || !Lci || !Uci || !Lv || !Uv) { rc = -4; goto out; }
    Lrp[0] = 0;
    Urp[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        double nrm = 0.0;
        int32_t len = 0;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            nrm = nrm + v[q] * v[q];
            w[ci[q]] = v[q];
            if (!nzf[ci[q]]) { nzf[ci[q]] = 1; lst[len++] = ci[q]; }
        }
        if (!nzf[i]) { nzf[i] = 1; w[i] = 0.0; lst[len++] = i; }
        double tau_i = tau * sqrt(nrm);
        int32_t done_k = -1;
        for (;;) {
            int32_t k = n;
            for (int32_t t = 0; t < len; ++t)
                if (lst[t] > done_k && lst[t] < i && lst[t] < k) k = lst[t];
            if (k == n) break;
            done_k = k;
            /* U row k: diagonal first, then strict upper */
            double ukk = Uv[Urp[k]];
            double wk = w[k] / ukk;
            if (fabs(wk) < tau_i) { w[k] = 0.0; continue; }
            w[k] = wk;
            for (int64_t q = Urp[k] + 1; q < Urp[k + 1]; ++q) {
                int32_t j = Uci[q];
                if (!nzf[j]) { nzf[j] = 1; w[j] = 0.0; lst[len++] = j; }
                w[j] = w[j] - wk * Uv[q];
            }
        }
        /* L part: drop small, keep p largest */
        int32_t nc = 0;
        for (int32_t t = 0; t < len; ++t) {
            int32_t j = lst[t];
            if (j < i && w[j] != 0.0 && fabs(w[j]) >= tau_i) { cand[nc].mag = fabs(w[j]); cand[nc].col = j; ++nc; }
        }
        qsort(cand, (size_t)nc, sizeof(orc_cand), cand_cmp);
        if (nc > p) nc = p;
        qsort(cand, (size_t)nc, sizeof(orc_cand), col_cmp);
        for (int32_t t = 0; t < nc; ++t) { Lci[ln] = cand[t].col; Lv[ln] = w[cand[t].col]; ++ln; }
        Lrp[i + 1] = (int32_t)ln;
        /* U part: diagonal always, then p largest of the strict upper part */
        double d = w[i];
        if (d == 0.0 || !isfinite(d)) { rc = -3; goto out; }
        Uci[un] = i; Uv[un] = d; ++un;
        nc = 0;
        for (int32_t t = 0; t < len; ++t) {
            int32_t j = lst[t];
            if (j > i && w[j] != 0.0 && fabs(w[j]) >= tau_i) { cand[nc].mag = fabs(w[j]); cand[nc].col = j; ++nc; }
        }
        qsort(cand, (size_t)nc, sizeof(orc_cand), cand_cmp);
        if (nc > p) nc = p;
        qsort(cand, (size_t)nc, sizeof(orc_cand), col_cmp);
        for (int32_t t = 0; t < nc; ++t) { Uci[un] = cand[t].col; Uv[un] = w[cand[t].col]; ++un; }
        Urp[i + 1] = (int32_t)un;
        for (int32_t t = 0; t < len; ++t) { w[lst[t]] = 0.0; nzf[lst[t]] = 0; }
    }
out:
    free(w); free(nzf); free(lst); free(cand);
    if (rc != 0) { free(Lrp); free(Urp); free(Lci); free(Uci); free(Lv); free(Uv); return rc; }
    *lrp = Lrp; *lci = Lci; *lv = Lv; *urp = Urp; *uci = Uci; *uv = Uv;
    return 0;
}
