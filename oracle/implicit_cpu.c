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
 *
 * With the same factors it also forms the explicit local dual operators the
 * plain way (eq. localdualoperator: one unit right-hand side per local
 * multiplier, F~_i = B~_i K_reg,i^{-1} B~_i^T column by column, stored dense)
 * and applies them as dense matrix-vector products (eq.
 * dualop_apply_expl); and it estimates ||F~_i||_2 by power iteration and the
 * condition number of K_reg,i by power and inverse iteration, the scales of
 * the rounding bounds the parity tests use.
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
    double *F;         /* explicit F~_i, m x m row-major (after orc_assemble_all) */
    double est;        /* last estimate of orc_opnorm_all / orc_kappa_all */
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
    free(s->b_sign); free(s->dual_map); free(s->work); free(s->qloc); free(s->F);
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

/* y = C x for the symmetric matrix whose upper triangle C holds (permuted order) */
static void symv_upper(const orc_sub *s, const double *x, double *y)
{
    memset(y, 0, sizeof(double) * (size_t)s->n);
    for (int k = 0; k < s->n; ++k)
        for (int p = s->Cp[k]; p < s->Cp[k + 1]; ++p) {
            int i = s->Ci[p];
            y[i] += s->Cx[p] * x[k];
            if (i != k) y[k] += s->Cx[p] * x[i];
        }
}

/* y = F~_i v = B~_i K_reg,i^{-1} B~_i^T v for a local vector v (m entries) */
static void apply_local(orc_sub *s, const double *v, double *y)
{
    double *x = s->work;
    memset(x, 0, sizeof(double) * (size_t)s->n);
    for (int j = 0; j < s->m; ++j) x[s->b_new[j]] += s->b_sign[j] * v[j];
    solve_one(s, x);
    for (int j = 0; j < s->m; ++j) y[j] = s->b_sign[j] * x[s->b_new[j]];
}

static void apply_one(orc_sub *s, const double *lam)
{
    double *x = s->work;
    memset(x, 0, sizeof(double) * (size_t)s->n);
    for (int j = 0; j < s->m; ++j) x[s->b_new[j]] += s->b_sign[j] * lam[s->dual_map[j]];
    solve_one(s, x);
    for (int j = 0; j < s->m; ++j) s->qloc[j] = s->b_sign[j] * x[s->b_new[j]];
}

/* deterministic start vector with no structure: entries in [0.5, 1.5) */
static void start_vector(double *v, int n)
{
    unsigned long long st = 0x9e3779b97f4a7c15ULL;
    for (int k = 0; k < n; ++k) {
        st = st * 6364136223846793005ULL + 1442695040888963407ULL;
        v[k] = 0.5 + (double)(st >> 11) * (1.0 / 9007199254740992.0);
    }
}

static double norm2(const double *v, int n)
{
    double t = 0.0;
    for (int k = 0; k < n; ++k) t += v[k] * v[k];
    return sqrt(t);
}

/* ||F~_i||_2 by power iteration (F~_i is symmetric positive semi-definite):
 * the Rayleigh quotient of the last iterate, a lower estimate */
static void opnorm_one(orc_sub *s, int iters)
{
    int m = s->m;
    double *v = (double *)malloc(sizeof(double) * (size_t)m);
    double *y = (double *)malloc(sizeof(double) * (size_t)m);
    start_vector(v, m);
    double nv = norm2(v, m), est = 0.0;
    for (int k = 0; k < m; ++k) v[k] /= nv;
    for (int it = 0; it < iters; ++it) {
        apply_local(s, v, y);
        est = 0.0;
        for (int k = 0; k < m; ++k) est += v[k] * y[k];
        double ny = norm2(y, m);
        if (!(ny > 0.0)) break;
        for (int k = 0; k < m; ++k) v[k] = y[k] / ny;
    }
    s->est = est;
    free(v);
    free(y);
}

/* condition number of K_reg,i: the largest eigenvalue by power iteration,
 * the smallest by inverse iteration with the factor */
static void kappa_one(orc_sub *s, int iters)
{
    int n = s->n;
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    start_vector(v, n);
    double nv = norm2(v, n), lmax = 0.0, lmin = 0.0;
    for (int k = 0; k < n; ++k) v[k] /= nv;
    for (int it = 0; it < iters; ++it) {
        symv_upper(s, v, y);
        lmax = 0.0;
        for (int k = 0; k < n; ++k) lmax += v[k] * y[k];
        double ny = norm2(y, n);
        for (int k = 0; k < n; ++k) v[k] = y[k] / ny;
    }
    start_vector(v, n);
    nv = norm2(v, n);
    for (int k = 0; k < n; ++k) v[k] /= nv;
    for (int it = 0; it < iters; ++it) {
        memcpy(y, v, sizeof(double) * (size_t)n);
        solve_one(s, y);
        double r = 0.0;
        for (int k = 0; k < n; ++k) r += v[k] * y[k];   /* v^T K^{-1} v -> 1 / lambda_min */
        lmin = 1.0 / r;
        double ny = norm2(y, n);
        for (int k = 0; k < n; ++k) v[k] = y[k] / ny;
    }
    s->est = lmax / lmin;
    free(v);
    free(y);
}

/* explicit F~_i (m x m, row-major): column a is B~ K_reg^{-1} (sign_a e_dof_a) */
static void assemble_one(orc_sub *s)
{
    int m = s->m;
    free(s->F);
    s->F = (double *)malloc(sizeof(double) * (size_t)m * (size_t)m);
    double *x = s->work;
    for (int a = 0; a < m; ++a) {
        memset(x, 0, sizeof(double) * (size_t)s->n);
        x[s->b_new[a]] = s->b_sign[a];
        solve_one(s, x);
        for (int b = 0; b < m; ++b) s->F[(size_t)b * m + a] = s->b_sign[b] * x[s->b_new[b]];
    }
}

/* q~_i = F~_i lambda_i with the stored dense F~_i */
static void apply_dense_one(orc_sub *s, const double *lam)
{
    int m = s->m;
    for (int a = 0; a < m; ++a) {
        const double *row = s->F + (size_t)a * m;
        double t = 0.0;
        for (int b = 0; b < m; ++b) t += row[b] * lam[s->dual_map[b]];
        s->qloc[a] = t;
    }
}

enum { MODE_FACTOR, MODE_APPLY, MODE_OPNORM, MODE_KAPPA, MODE_ASSEMBLE, MODE_APPLY_DENSE };

typedef struct {
    orc_handle *h;
    int next;
    pthread_mutex_t mu;
    int mode;
    int iters;
    const double *lam;
} pool_t;

static void *worker(void *arg)
{
    pool_t *P = (pool_t *)arg;
    for (;;) {
        pthread_mutex_lock(&P->mu);
        int i = P->next++;
        pthread_mutex_unlock(&P->mu);
        if (i >= P->h->nsub) break;
        orc_sub *s = &P->h->s[i];
        switch (P->mode) {
        case MODE_FACTOR: factor_one(s); break;
        case MODE_APPLY: apply_one(s, P->lam); break;
        case MODE_OPNORM: opnorm_one(s, P->iters); break;
        case MODE_KAPPA: kappa_one(s, P->iters); break;
        case MODE_ASSEMBLE: assemble_one(s); break;
        default: apply_dense_one(s, P->lam); break;
        }
    }
    return NULL;
}

static void run_pool(orc_handle *h, int nthreads, int mode, const double *lam, int iters)
{
    pool_t P;
    P.h = h;
    P.next = 0;
    P.mode = mode;
    P.iters = iters;
    P.lam = lam;
    pthread_mutex_init(&P.mu, NULL);
    if (nthreads > h->nsub) nthreads = h->nsub;
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
    run_pool(h, nthreads, MODE_FACTOR, NULL, 0);
    for (int i = 0; i < h->nsub; ++i)
        if (h->s[i].status != 0) return -(1 + i);
    return 0;
}

/* q = sum_i D_i^T B~_i K_reg,i^{-1} B~_i^T D_i lam  (q has n_lambda entries) */
void orc_apply(void *hh, const double *lam, double *q, int n_lambda, int nthreads)
{
    orc_handle *h = (orc_handle *)hh;
    run_pool(h, nthreads, MODE_APPLY, lam, 0);
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

/* ||F~_i||_2 of every subdomain (power iteration, `iters` steps) into out[nsub] */
void orc_opnorm_all(void *hh, int iters, double *out, int nthreads)
{
    orc_handle *h = (orc_handle *)hh;
    run_pool(h, nthreads, MODE_OPNORM, NULL, iters);
    for (int i = 0; i < h->nsub; ++i) out[i] = h->s[i].est;
}

/* condition number estimates of every K_reg,i into out[nsub] */
void orc_kappa_all(void *hh, int iters, double *out, int nthreads)
{
    orc_handle *h = (orc_handle *)hh;
    run_pool(h, nthreads, MODE_KAPPA, NULL, iters);
    for (int i = 0; i < h->nsub; ++i) out[i] = h->s[i].est;
}

/* explicit assembly: the dense F~_i of every subdomain, one unit solve per column */
void orc_assemble_all(void *hh, int nthreads)
{
    orc_handle *h = (orc_handle *)hh;
    run_pool(h, nthreads, MODE_ASSEMBLE, NULL, 0);
}

/* copy F~_i (m x m, row-major, local multiplier order); -1 before assembly */
int orc_get_F(void *hh, int i, double *out)
{
    orc_handle *h = (orc_handle *)hh;
    const orc_sub *s = &h->s[i];
    if (!s->F) return -1;
    memcpy(out, s->F, sizeof(double) * (size_t)s->m * (size_t)s->m);
    return 0;
}

/* q = sum_i D_i^T F~_i D_i lam with the assembled dense F~_i */
void orc_apply_explicit(void *hh, const double *lam, double *q, int n_lambda, int nthreads)
{
    orc_handle *h = (orc_handle *)hh;
    run_pool(h, nthreads, MODE_APPLY_DENSE, lam, 0);
    memset(q, 0, sizeof(double) * (size_t)n_lambda);
    for (int i = 0; i < h->nsub; ++i) {
        const orc_sub *s = &h->s[i];
        for (int j = 0; j < s->m; ++j) q[s->dual_map[j]] += s->qloc[j];
    }
}

/* x <- K_reg,i^{-1} x for a vector in the caller's (unpermuted) DOF order */
int orc_solve(void *hh, int i, double *x)
{
    orc_handle *h = (orc_handle *)hh;
    orc_sub *s = &h->s[i];
    if (!s->Lp || s->status != 0) return -1;
    double *w = (double *)malloc(sizeof(double) * (size_t)s->n);
    for (int k = 0; k < s->n; ++k) w[k] = x[s->perm[k]];
    solve_one(s, w);
    for (int k = 0; k < s->n; ++k) x[s->perm[k]] = w[k];
    free(w);
    return 0;
}
