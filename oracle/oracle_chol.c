/*
 * ORACLE -- test infrastructure only.  Plain, slow, scalar FP64 reference for the GMRF
 * posterior path; only tests, the smoke check and the CPU-baseline leg of the bench may
 * load it.  It shares no code with the GPU library.
 *
 * Operates on a symmetric positive-definite matrix that the caller has already
 * permuted (B = P Q P^T), given as its lower triangle in CSC (column j holds rows
 * i >= j, sorted ascending, diagonal first).
 *
 *   oc_symbolic : elimination tree and the exact pattern of L (struct(L_j) is
 *                 struct(B_{>=j, j}) united with struct(L_c) \ {c} over the etree
 *                 children c of j).
 *   oc_numeric  : left-looking column Cholesky B = L L^T (Sec. 3.2, sparse Cholesky):
 *                 column j = B_{:,j} - sum_{k<j, L_jk != 0} L_{:,k} L_jk, then scaled by
 *                 the square root of its diagonal.  Returns the 0-based column of the
 *                 first non-positive pivot as -(j+1), else 0.
 *   oc_lsolve / oc_ltsolve : L y = b and L^T x = y (Sec. 3.2: posterior mean needs one
 *                 forward and one backward solve; a sample needs one backward solve).
 *   oc_takahashi: the Takahashi recursion (Sec. 3.2, marginal variances) on pattern(L):
 *                 for j = n-1 .. 0 and i in struct(L_j), i > j:
 *                   S_ij = -(1/L_jj) sum_{k in struct(L_j), k > j} L_kj S_ki
 *                   S_jj = 1/L_jj^2 - (1/L_jj) sum_{k > j} L_kj S_kj
 *                 with S_ki read as S_ik when k < i.  S is returned on pattern(L).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* etree + column counts + row indices of L. Lp has n+1 entries. Caller frees *Li. */
int64_t oc_symbolic(int64_t n, const int64_t *Bp, const int32_t *Bi, int32_t *parent,
                    int64_t *Lp, int32_t **Li_out)
{
    /* elimination tree: parent[j] = min{ i > j : L_ij != 0 } = the smallest row of
       struct(L_j) below the diagonal; computed together with the patterns. */
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *head = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t cap = 0;
    for (int64_t j = 0; j < n; ++j) cap += Bp[j + 1] - Bp[j];
    cap = cap * 2 + 16;
    int32_t *Li = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    for (int64_t j = 0; j < n; ++j) { mark[j] = -1; head[j] = -1; }
    Lp[0] = 0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t start = Lp[j], cnt = 0;
        /* gather rows: diagonal, lower entries of B, and children's rows below j */
        if (start + n - j + 1 > cap) {
            while (start + n - j + 1 > cap) cap *= 2;
            Li = (int32_t *)realloc(Li, sizeof(int32_t) * (size_t)cap);
        }
        mark[j] = (int32_t)j;
        Li[start + cnt++] = (int32_t)j;
        for (int64_t e = Bp[j]; e < Bp[j + 1]; ++e) {
            int32_t i = Bi[e];
            if (i > j && mark[i] != j) { mark[i] = (int32_t)j; Li[start + cnt++] = i; }
        }
        for (int32_t c = head[j]; c != -1; c = next[c]) {
            for (int64_t e = Lp[c] + 1; e < Lp[c + 1]; ++e) {
                int32_t i = Li[e];
                if (i > j && mark[i] != j) { mark[i] = (int32_t)j; Li[start + cnt++] = i; }
            }
        }
        /* sort the below-diagonal rows (insertion sort is fine for a reference) */
        for (int64_t a = start + 2; a < start + cnt; ++a) {
            int32_t v = Li[a]; int64_t b = a - 1;
            while (b > start && Li[b] > v) { Li[b + 1] = Li[b]; --b; }
            Li[b + 1] = v;
        }
        Lp[j + 1] = start + cnt;
        parent[j] = cnt > 1 ? Li[start + 1] : -1;
        if (parent[j] >= 0) { next[j] = head[parent[j]]; head[parent[j]] = (int32_t)j; }
    }
    free(mark); free(head); free(next);
    *Li_out = Li;
    return Lp[n];
}

void oc_free(void *p) { free(p); }

int64_t oc_numeric(int64_t n, const int64_t *Bp, const int32_t *Bi, const double *Bx,
                   const int64_t *Lp, const int32_t *Li, double *Lx)
{
    double *w = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    int64_t *ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *head = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t status = 0;
    for (int64_t j = 0; j < n; ++j) head[j] = -1;
    for (int64_t j = 0; j < n; ++j) {
        /* w = B(:, j), lower part */
        for (int64_t e = Bp[j]; e < Bp[j + 1]; ++e)
            if (Bi[e] >= j) w[Bi[e]] += Bx[e];
        /* subtract every earlier column k with L_jk != 0 (linked by their next row) */
        int32_t k = head[j];
        while (k != -1) {
            int32_t knext = next[k];
            int64_t p = ptr[k];             /* position of row j in column k */
            double ljk = Lx[p];
            for (int64_t e = p; e < Lp[k + 1]; ++e) w[Li[e]] -= Lx[e] * ljk;
            if (p + 1 < Lp[k + 1]) {
                ptr[k] = p + 1;
                int32_t r = Li[p + 1];
                next[k] = head[r]; head[r] = k;
            }
            k = knext;
        }
        double d = w[j];
        if (!(d > 0.0) && status == 0) status = -(j + 1);
        double ljj = sqrt(d > 0.0 ? d : 1.0);
        Lx[Lp[j]] = ljj;
        w[j] = 0.0;
        for (int64_t e = Lp[j] + 1; e < Lp[j + 1]; ++e) {
            Lx[e] = w[Li[e]] / ljj;
            w[Li[e]] = 0.0;
        }
        if (Lp[j + 1] - Lp[j] > 1) {
            ptr[j] = Lp[j] + 1;
            int32_t r = Li[Lp[j] + 1];
            next[j] = head[r]; head[r] = (int32_t)j;
        }
    }
    free(w); free(ptr); free(head); free(next);
    return status;
}

/* forward solve L y = b in place, k right-hand sides, column-major with leading dim n */
void oc_lsolve(int64_t n, const int64_t *Lp, const int32_t *Li, const double *Lx,
               double *x, int64_t k)
{
    for (int64_t r = 0; r < k; ++r) {
        double *v = x + r * n;
        for (int64_t j = 0; j < n; ++j) {
            v[j] /= Lx[Lp[j]];
            double t = v[j];
            for (int64_t e = Lp[j] + 1; e < Lp[j + 1]; ++e) v[Li[e]] -= Lx[e] * t;
        }
    }
}

/* backward solve L^T x = y in place */
void oc_ltsolve(int64_t n, const int64_t *Lp, const int32_t *Li, const double *Lx,
                double *x, int64_t k)
{
    for (int64_t r = 0; r < k; ++r) {
        double *v = x + r * n;
        for (int64_t j = n - 1; j >= 0; --j) {
            double t = v[j];
            for (int64_t e = Lp[j] + 1; e < Lp[j + 1]; ++e) t -= Lx[e] * v[Li[e]];
            v[j] = t / Lx[Lp[j]];
        }
    }
}

/* Takahashi recursion; S has the layout of L (S[e] = Sigma_{Li[e], j}). */
void oc_takahashi(int64_t n, const int64_t *Lp, const int32_t *Li, const double *Lx,
                  double *S)
{
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double *acc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) pos[i] = -1;
    for (int64_t j = n - 1; j >= 0; --j) {
        int64_t b = Lp[j] + 1, e_end = Lp[j + 1], c = e_end - b;   /* rows i > j */
        double ljj = Lx[Lp[j]];
        for (int64_t t = 0; t < c; ++t) { pos[Li[b + t]] = (int32_t)t; acc[t] = 0.0; }
        /* acc[pos(i)] = sum_k S_ik L_kj over k, i in struct(L_j)\{j}; S_ik for i >= k
           lives in column k at row i, and by the closure of the pattern every row of
           struct(L_j) above k is present in column k. */
        for (int64_t t = 0; t < c; ++t) {
            int32_t kcol = Li[b + t];
            double lkj = Lx[b + t];
            for (int64_t e = Lp[kcol]; e < Lp[kcol + 1]; ++e) {
                int32_t i = Li[e];
                int32_t pi = pos[i];
                if (pi < 0) continue;
                double s = S[e];                 /* Sigma_{i, kcol}, i >= kcol */
                acc[pi] += s * lkj;              /* row i gets Sigma_{i,k} L_kj   */
                if (i != kcol) acc[t] += s * Lx[b + pi];  /* row k gets Sigma_{k,i} L_ij */
            }
        }
        double dsum = 0.0;
        for (int64_t t = 0; t < c; ++t) {
            S[b + t] = -acc[t] / ljj;
            dsum += Lx[b + t] * S[b + t];
        }
        S[Lp[j]] = 1.0 / (ljj * ljj) - dsum / ljj;
        for (int64_t t = 0; t < c; ++t) pos[Li[b + t]] = -1;
    }
    free(pos); free(acc);
}
