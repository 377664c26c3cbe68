/* Driver for the sanitizer run of the oracle (tests/test_oracle_sanitize.py): solves a
 * few small SPD systems through oracle_ccg, covering the stop test, a restart, the
 * rank step (duplicate start columns; p not dividing n), re-inflation, the per-step
 * traces and the R / D outputs.  The systems come from a counter hash, not from the method. */
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int status, iters, restarts, p_final, best_agent, deflations;
    double rel_res, rel_res_max;
    int reinflations;
} orc_info;

int oracle_ccg(int n, int p, const double *A, int lda, const double *b, double *X, int ldx,
               double tol, int maxit, double tau, int trace_k, double *ta, double *tb,
               double *R_out, double *D_out, int reinflate_max, orc_info *info);
int oracle_residual(int n, int p, const double *A, int lda, const double *b, const double *X,
                    int ldx, double *T);

static double hash01(unsigned long long x)
{
    x *= 0x9E3779B97F4A7C15ull;
    x ^= x >> 31;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 29;
    return (double)(x & 0xffffff) / 16777216.0 - 0.5;
}

/* symmetric, diagonally dominant with a spread diagonal: SPD */
static void make(int n, int p, int lda, int ldx, double *A, double *b, double *X, double spread)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            int lo = i < j ? i : j, hi = i < j ? j : i;
            double v = hash01((unsigned long long)lo * 7919u + hi);
            A[i + (size_t)j * lda] = (i == j) ? n * (1.0 + spread * i / n) : v;
        }
    for (int i = 0; i < n; ++i) b[i] = hash01(100000u + i);
    for (int j = 0; j < p; ++j)
        for (int i = 0; i < ldx; ++i) X[i + (size_t)j * ldx] = hash01(200000u + i + 1000u * j);
}

static int run(int n, int p, int lda, int ldx, double tol, int maxit, int dup, int reinflate)
{
    double *A = malloc(sizeof(double) * (size_t)lda * n);
    double *b = malloc(sizeof(double) * n);
    double *X = malloc(sizeof(double) * (size_t)ldx * p);
    double *T = malloc(sizeof(double) * (size_t)n * p);
    double *ta = malloc(sizeof(double) * 5 * p * p);
    double *tb = malloc(sizeof(double) * 5 * p * p);
    double *R = malloc(sizeof(double) * (size_t)n * p);
    double *D = malloc(sizeof(double) * (size_t)n * p);
    make(n, p, lda, ldx, A, b, X, 1e3);
    if (dup && p > 1)
        for (int i = 0; i < n; ++i) X[i + (size_t)(p - 1) * ldx] = X[i];
    orc_info info;
    int st = oracle_ccg(n, p, A, lda, b, X, ldx, tol, maxit, 1e-14, 5, ta, tb, R, D, reinflate, &info);
    int st2 = oracle_residual(n, p, A, lda, b, X, ldx, T);
    printf("n=%d p=%d status=%d iters=%d restarts=%d deflations=%d reinflations=%d p_final=%d rel_res=%.3e\n",
           n, p, st, info.iters, info.restarts, info.deflations, info.reinflations, info.p_final, info.rel_res);
    free(A); free(b); free(X); free(T); free(ta); free(tb); free(R); free(D);
    return (st < 0 || st2 != 0) ? 1 : 0;
}

int main(void)
{
    int bad = 0;
    bad |= run(40, 3, 41, 43, 1e-10, 500, 0, 0);
    bad |= run(40, 4, 40, 40, 1e-10, 500, 1, 0);     /* duplicate start columns */
    bad |= run(13, 3, 13, 13, 1e-12, 50, 0, 0);      /* p does not divide n */
    bad |= run(30, 2, 30, 31, 1e-15, 300, 0, 0);     /* below the attainable residual: restarts */
    bad |= run(25, 5, 25, 25, 0.0, 5, 0, 0);         /* fixed step count */
    bad |= run(40, 4, 40, 40, 1e-10, 500, 1, 2);     /* duplicate columns, re-inflated */
    return bad;
}
