/*
 * Oracle implicit dual-operator application on the CPU (test infrastructure).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests and by the benchmark's
 * CPU-baseline leg, never by the GPU library, with which it shares no code.
 *
 * It computes q = sum_i D_i^T B~_i K_reg,i^{-1} B~_i^T D_i lambda right to
 * left, as the paper's implicit application (Sec. III, eq. dualop_apply_impl):
 * a sparse scatter, a forward and a backward triangular solve with the
 * Cholesky factor of K_reg,i, and a sparse gather.  The factor is computed
 * here with a plain up-looking sparse Cholesky (row k of L from a sparse
 * triangular solve whose pattern is the elimination-tree reach of column k
 * of A), in the fill-reducing order given by the caller.  FP64 throughout.
 * Subdomains are spread over a pool of threads; the final gather runs in
 * ascending subdomain order so the result does not depend on the threads.
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n, m;
    /* upper triangle of C = P A P^T, column-compressed */
    int *Cp, *Ci;
    double *Cx;
    int *perm;  /* new -> old */
    int *pinv;  /* old -> new */
    int *parent;
    /* factor L, column-compressed, diagonal first in each column */
    int *Lp, *Li;
    double *Lx;
    int *b_new;        /* permuted dof of each local multiplier */
    double *b_sign;
    int *dual_map;
    double *work;      /* n */
    double *qloc;      /* m */
    int status;
} orc_sub;

typedef struct {
    int nsub;
    orc_sub *s;
} orc_handle;

void *orc_create(int nsub)
{
    orc_handle *h = (orc_handle *)calloc(1, sizeof(orc_handle));
    h->nsub = nsub;
    h->s = (orc_sub *)calloc((size_t)nsub, sizeof(orc_sub));
    return h;
}

static void sub_free(orc_sub *s)
{
    free(s->Cp); free(s->Ci); free(s->Cx); free(s->perm); free(s->pinv);
    free(s->parent); free(s->Lp); free(s->Li); free(s->Lx); free(s->b_new);
    free(s->b_sign); free(s->dual_map); free(s->work); free(s->qloc);
    memset(s, 0, sizeof(*s));
}

void orc_destroy(void *hh)
{
    orc_handle *h = (orc_handle *)hh;
    if (!h) return;
    for (int i = 0; i < h->nsub; ++i) sub_free(&h->s[i]);
    free(h->s);
    free(h);
}

/* Store subdomain i: A is the full symmetric CSR of K_reg,i. */
int orc_set_sub(void *hh, int i, int n, const int *Ap, const int *Ai, const double *Ax,
                const int *perm, int m, const int *b_dof, const signed char *b_sign,
                const int *dual_map)
{
    orc_handle *h = (orc_handle *)hh;
    if (i < 0 || i >= h->nsub) return -1;
    orc_sub *s = &h->s[i];
    sub_free(s);
    s->n = n;
    s->m = m;
    s->perm = (int *)malloc(sizeof(int) * (size_t)n);
    s->pinv = (int *)malloc(sizeof(int) * (size_t)n);
    memcpy(s->perm, perm, sizeof(int) * (size_t)n);
    for (int k = 0; k < n; ++k) s->pinv[perm[k]] = k;
    /* count entries of the upper triangle of C, column by column */
    s->Cp = (int *)calloc((size_t)n + 1, sizeof(int));
    for (int r = 0; r < n; ++r)
        for (int p = Ap[r]; p < Ap[r + 1]; ++p) {
            int a = s->pinv[r], b = s->pinv[Ai[p]];
            if (a <= b) s->Cp[b + 1]++;
        }
    for (int k = 0; k < n; ++k) s->Cp[k + 1] += s->Cp[k];
    s->Ci = (int *)malloc(sizeof(int) * (size_t)s->Cp[n]);
    s->Cx = (double *)malloc(sizeof(double) * (size_t)s->Cp[n]);
    int *next = (int *)malloc(sizeof(int) * (size_t)n);
    memcpy(next, s->Cp, sizeof(int) * (size_t)n);
    for (int r = 0; r < n; ++r)
        for (int p = Ap[r]; p < Ap[r + 1]; ++p) {
            int a = s->pinv[r], b = s->pinv[Ai[p]];
            if (a <= b) {
                s->Ci[next[b]] = a;
                s->Cx[next[b]++] = Ax[p];
            }
        }
    free(next);
    s->b_new = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    s->b_sign = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    s->dual_map = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    for (int j = 0; j < m; ++j) {
        s->b_new[j] = s->pinv[b_dof[j]];
        s->b_sign[j] = (double)b_sign[j];
        s->dual_map[j] = dual_map[j];
    }
    s->work = (double *)calloc((size_t)n, sizeof(double));
    s->qloc = (double *)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
    return 0;
}

/* elimination tree of the upper-triangular CSC pattern (path compression) */
static void etree(const orc_sub *s, int *parent, int *anc)
{
    for (int k = 0; k < s->n; ++k) {
        parent[k] = -1;
        anc[k] = -1;
        for (int p = s->Cp[k]; p < s->Cp[k + 1]; ++p) {
            int i = s->Ci[p];
            while (i != -1 && i < k) {
                int nx = anc[i];
                anc[i] = k;
                if (nx == -1) parent[i] = k;
                i = nx;
            }
        }
    }
}

/* Nonzero pattern of row k of L: the reach of column k of the upper
 * triangle in the elimination tree.  Returns top; pattern is stack[top..n-1]
 * in topological order. mark[] must hold values != k on entry. */
static int ereach(const orc_sub *s, int k, const int *parent, int *stack, int *mark)
{
    int n = s->n, top = n;
    mark[k] = k;
    for (int p = s->Cp[k]; p < s->Cp[k + 1]; ++p) {
        int i = s->Ci[p];
        if (i > k) continue;
        int len = 0;
        while (mark[i] != k) {
            stack[len++] = i; /* temporarily at the front */
            mark[i] = k;
            i = parent[i];
        }
        while (len > 0) stack[--top] = stack[--len];
    }
    return top;
}

static int factor_one(orc_sub *s)
{
    int n = s->n;
    int *parent = (int *)malloc(sizeof(int) * (size_t)n);
    int *anc = (int *)malloc(sizeof(int) * (size_t)n);
    int *stack = (int *)malloc(sizeof(int) * (size_t)n);
    int *mark = (int *)malloc(sizeof(int) * (size_t)n);
    int *cnt = (int *)calloc((size_t)n, sizeof(int));
    etree(s, parent, anc);
    /* column counts by a symbolic pass over the row patterns */
    for (int k = 0; k < n; ++k) mark[k] = -1;
    for (int k = 0; k < n; ++k) {
        cnt[k]++; /* diagonal */
        int top = ereach(s, k, parent, stack, mark);
        for (int t = top; t < n; ++t) cnt[stack[t]]++;
    }
    s->Lp = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    s->Lp[0] = 0;
    for (int k = 0; k < n; ++k) s->Lp[k + 1] = s->Lp[k] + cnt[k];
    s->Li = (int *)malloc(sizeof(int) * (size_t)s->Lp[n]);
    s->Lx = (double *)malloc(sizeof(double) * (size_t)s->Lp[n]);
    int *fill = anc; /* reuse: next free slot of each column */
    for (int k = 0; k < n; ++k) mark[k] = -1;
    double *x = s->work;
    int status = 0;
    for (int k = 0; k < n; ++k) {
        int top = ereach(s, k, parent, stack, mark);
        x[k] = 0.0;
        for (int p = s->Cp[k]; p < s->Cp[k + 1]; ++p)
            if (s->Ci[p] <= k) x[s->Ci[p]] = s->Cx[p];
        double d = x[k];
        x[k] = 0.0;
        for (int t = top; t < n; ++t) {
            int j = stack[t];
            double lkj = x[j] / s->Lx[s->Lp[j]];
            x[j] = 0.0;
            for (int p = s->Lp[j] + 1; p < fill[j]; ++p) x[s->Li[p]] -= s->Lx[p] * lkj;
            d -= lkj * lkj;
            s->Li[fill[j]] = k;
            s->Lx[fill[j]++] = lkj;
        }
        if (!(d > 0.0)) { status = -(k + 1); break; }
        s->Li[s->Lp[k]] = k;
        s->Lx[s->Lp[k]] = sqrt(d);
        fill[k] = s->Lp[k] + 1;
    }
    s->parent = parent;
    free(anc); free(stack); free(mark); free(cnt);
    memset(s->work, 0, sizeof(double) * (size_t)n);
    s->status = status;
    return status;
}

/* x <- L^{-T} L^{-1} x, in the permuted order */
static void solve_one(const orc_sub *s, double *x)
{
    int n = s->n;
    for (int j = 0; j < n; ++j) {
        double v = x[j] / s->Lx[s->Lp[j]];
        x[j] = v;
        for (int p = s->Lp[j] + 1; p < s->Lp[j + 1]; ++p) x[s->Li[p]] -= s->Lx[p] * v;
    }
    for (int j = n - 1; j >= 0; --j) {
        double v = x[j];
        for (int p = s->Lp[j] + 1; p < s->Lp[j + 1]; ++p) v -= s->Lx[p] * x[s->Li[p]];
        x[j] = v / s->Lx[s->Lp[j]];
    }
}

typedef struct {
    orc_handle *h;
    int next;
    pthread_mutex_t mu;
    int mode; /* 0 factor, 1 apply */
    const double *lam;
} pool_t;

static void apply_one(orc_sub *s, const double *lam)
{
    double *x = s->work;
    memset(x, 0, sizeof(double) * (size_t)s->n);
    for (int j = 0; j < s->m; ++j) x[s->b_new[j]] += s->b_sign[j] * lam[s->dual_map[j]];
    solve_one(s, x);
    for (int j = 0; j < s->m; ++j) s->qloc[j] = s->b_sign[j] * x[s->b_new[j]];
}

static void *worker(void *arg)
{
    pool_t *P = (pool_t *)arg;
    for (;;) {
        pthread_mutex_lock(&P->mu);
        int i = P->next++;
        pthread_mutex_unlock(&P->mu);
        if (i >= P->h->nsub) break;
        if (P->mode == 0) factor_one(&P->h->s[i]);
        else apply_one(&P->h->s[i], P->lam);
    }
    return NULL;
}

static void run_pool(orc_handle *h, int nthreads, int mode, const double *lam)
{
    pool_t P;
    P.h = h;
    P.next = 0;
    P.mode = mode;
    P.lam = lam;
    pthread_mutex_init(&P.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, worker, &P);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&P.mu);
}

/* Factor every subdomain; returns 0, or -(1+i) for the first failing one. */
int orc_factor_all(void *hh, int nthreads)
{
    orc_handle *h = (orc_handle *)hh;
    run_pool(h, nthreads, 0, NULL);
    for (int i = 0; i < h->nsub; ++i)
        if (h->s[i].status != 0) return -(1 + i);
    return 0;
}

/* q = sum_i D_i^T B~_i K_reg,i^{-1} B~_i^T D_i lam  (q has n_lambda entries) */
void orc_apply(void *hh, const double *lam, double *q, int n_lambda, int nthreads)
{
    orc_handle *h = (orc_handle *)hh;
    run_pool(h, nthreads, 1, lam);
    memset(q, 0, sizeof(double) * (size_t)n_lambda);
    for (int i = 0; i < h->nsub; ++i) {
        const orc_sub *s = &h->s[i];
        for (int j = 0; j < s->m; ++j) q[s->dual_map[j]] += s->qloc[j];
    }
}

long orc_nnz(void *hh, int i)
{
    orc_handle *h = (orc_handle *)hh;
    return h->s[i].Lp ? (long)h->s[i].Lp[h->s[i].n] : -1;
}
