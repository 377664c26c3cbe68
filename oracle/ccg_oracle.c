/*
 * Reference (oracle) implementation of cooperative conjugate gradient, plain C.
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code with the HIP path
 * and is written to be read against the paper, not to be fast: every product is a
 * plain loop in the order the definition is written, with no blocking or fusion.
 *
 * Method (Bhaya, Bliman, Niedu, Pazos, "A cooperative conjugate gradient method
 * for linear systems permitting multithread implementation of low complexity"):
 *   - Alg. 2 (cCG, Sec. 3.2): p agents hold the columns of X, R, D (n x p); each
 *     step forms the p x p matrices D^T A D and R^T D, solves for the matrix step
 *     alpha, updates X and R, solves for the matrix beta and updates D.
 *   - Table 1 (Sec. 4): the residual is carried by the recurrence
 *     R_{k+1} = R_k - A D_k alpha (one product A.D per step).
 *   - Alg. 3 (mcCG, Sec. 3.2): when D_k loses rank, keep a full-rank subset J of
 *     the agents and continue with p_k = |J| agents.
 *   - Alg. 4 (Sec. 5): the run stops when the smallest agent residual norm is
 *     below the tolerance.
 *
 * Sign convention.  The paper writes the residual as the gradient A x - b.  Here
 * R = B - A X with B = b 1^T (b in every column).  Both describe the same iterates:
 *     alpha = G^{-1} (D^T R),        X += D alpha,     R -= (A D) alpha,
 *     beta  = -G^{-1} ((A D)^T R),   D  = R + D beta,  G = D^T A D,
 * which is the paper's alpha and beta transposed, with alpha negated (the paper's
 * R and D are the negatives of these).
 *
 * Readings taken where the paper is silent or loose (each is also recorded in the
 * design notes):
 *   - "b 1^T" is read as the n x p matrix with b in every column (Alg. 2 prints
 *     the product in the other order).
 *   - Stop test: relative, min_j ||R_j|| / ||b|| <= tol on the recurrence
 *     residual, confirmed by the explicit residual B - A X; if the explicit one
 *     fails the test, restart with R = B - A X, D = R.
 *   - "D_k full rank" is decided by a greedy pivoted Cholesky of the diagonally
 *     scaled G (unit diagonal).  The largest remaining pivot is taken at each step
 *     (ties: lowest index); a pivot <= tau means the rest is dependent.  J is the
 *     set of pivots taken; the rank of D equals that of G because A is SPD.
 *   - The p x p systems are solved by Cholesky of G restricted to J (the paper uses
 *     Gaussian elimination; the solution is the same up to rounding).
 *   - Dropped agents keep their last iterate in X.
 *
 * Storage: every matrix is column-major.  A is n x n with leading dimension lda;
 * X is n x p with leading dimension ldx.  Internal X, R, D, AD are n x p with
 * leading dimension n, column j = agent j.
 *
 * Precision: every internal value has the type `real`, FP64 (double) by default.
 * Built with -DORC_REAL='long double' (x86 80-bit extended, 64-bit significand)
 * the same code runs the same algorithm with 11 more bits in every operation; the
 * interface stays FP64 (inputs are exact in either type, outputs are rounded to
 * double once at the end).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>

#ifndef ORC_REAL
#define ORC_REAL double
#endif
typedef ORC_REAL real;

/* Rows per share of the products with A.  The default build takes every row in one
 * share.  The all-cores build (-fopenmp -DORC_ROWS=1024) hands shares of rows to
 * threads; each element is still the same sum over k in the same order, so every
 * build gives the same bits. */
#ifndef ORC_ROWS
#define ORC_ROWS 2147483647
#endif

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_ERR_ARG -1
#define ORC_ERR_NONFINITE -2
#define ORC_ERR_NOT_SPD -3
#define ORC_ERR_NOMEM -5

#define ORC_MAXP 64

typedef struct {
    int status;
    int iters;        /* block steps taken (all restarts included) */
    int restarts;     /* explicit-residual restarts */
    int p_final;      /* agents still active at the end */
    int best_agent;   /* argmin_j of the explicit relative residual (ties: lowest j) */
    int deflations;   /* rank-drop events */
    double rel_res;   /* min_j ||b - A x_j|| / ||b|| over all agents */
    double rel_res_max;
    int reinflations; /* re-inflation events (see oracle_ccg) */
} orc_info;

/* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): the state advances by the golden-ratio increment and
 * each output is the state passed through the published 64-bit finaliser. */
static uint64_t splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* The first `count` outputs from `state` (exported so that the tests can hold the
 * generator to its published values). */
void oracle_splitmix64(uint64_t state, int count, uint64_t *out)
{
    for (int i = 0; i < count; ++i) out[i] = splitmix64_next(&state);
}

/* Entry i of the draw of re-inflation event e for agent j: the (i+1)-th SplitMix64
 * output from the state 0x1204 << 48 ^ e << 32 ^ j, mapped to [-1, 1) by its top 53
 * bits (exactly: 2 * (z >> 11) * 2^-53 - 1). */
static uint64_t reinflate_state(int e, int j)
{
    return (0x1204ull << 48) ^ ((uint64_t)e << 32) ^ (uint64_t)j;
}
static double unit_draw(uint64_t z)
{
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

/* ---------- plain dense helpers ---------- */

/* Y = A * M for A n x n (lda) and M n x m (ldm), one agent column at a time:
 * Y[:,j] = sum_k A[:,k] M[k,j]   (Table 1: each agent forms A d_j). */
static void matmat(int n, int m, const double *A, int lda, const real *M, int ldm,
                   real *Y, int ldy)
{
    for (int j = 0; j < m; ++j) {
        real *y = Y + (size_t)j * ldy;
#pragma omp parallel for schedule(static)
        for (int i0 = 0; i0 < n; i0 += (ORC_ROWS < n ? ORC_ROWS : n)) {
            int i1 = n - i0 > ORC_ROWS ? i0 + ORC_ROWS : n;
            for (int i = i0; i < i1; ++i) y[i] = 0.0;
            for (int k = 0; k < n; ++k) {
                real mkj = M[k + (size_t)j * ldm];
                const double *a = A + (size_t)k * lda;
                for (int i = i0; i < i1; ++i) y[i] += a[i] * mkj;
            }
        }
    }
}

/* C = U^T V for U, V n x m (leading dimension n): C[i,j] = sum_r U[r,i] V[r,j].
 * C is m x m, column-major with leading dimension m. */
static void gram(int n, int m, const real *U, const real *V, real *C)
{
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
            real s = 0.0;
            for (int r = 0; r < n; ++r) s += U[r + (size_t)i * n] * V[r + (size_t)j * n];
            C[i + j * m] = s;
        }
}

/* Cholesky G = L L^T (m x m, column-major, lower triangle of L written, upper zero).
 * Returns 0 on success, -1 if a pivot is not positive. */
static int cholesky(int m, const real *G, real *L)
{
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) L[i + j * m] = 0.0;
    for (int j = 0; j < m; ++j) {
        real d = G[j + j * m];
        for (int k = 0; k < j; ++k) d -= L[j + k * m] * L[j + k * m];
        if (!(d > 0.0)) return -1;
        real ljj = sqrt(d);
        L[j + j * m] = ljj;
        for (int i = j + 1; i < m; ++i) {
            real s = G[i + j * m];
            for (int k = 0; k < j; ++k) s -= L[i + k * m] * L[j + k * m];
            L[i + j * m] = s / ljj;
        }
    }
    return 0;
}

/* Solve (L L^T) Z = B for Z (m x q, column-major, leading dimension m). */
static void chol_solve(int m, const real *L, int q, const real *B, real *Z)
{
    for (int c = 0; c < q; ++c) {
        const real *bc = B + (size_t)c * m;
        real *z = Z + (size_t)c * m;
        for (int i = 0; i < m; ++i) {          /* L y = b */
            real s = bc[i];
            for (int k = 0; k < i; ++k) s -= L[i + k * m] * z[k];
            z[i] = s / L[i + i * m];
        }
        for (int i = m - 1; i >= 0; --i) {     /* L^T z = y */
            real s = z[i];
            for (int k = i + 1; k < m; ++k) s -= L[k + i * m] * z[k];
            z[i] = s / L[i + i * m];
        }
    }
}

/* Rank test on G (m x m, SPD or semi-definite): greedy pivoted Cholesky of the
 * diagonally scaled matrix.  Writes the chosen indices, ascending, to keep[] and
 * returns their count.  Returns -1 if a diagonal entry is negative (A not SPD),
 * -2 if a non-finite value is met.  Columns with G_ii == 0 (a zero direction) are
 * never chosen. */
static int rank_select(int m, const real *G, double tau, int *keep)
{
    real H[ORC_MAXP * ORC_MAXP];
    real s[ORC_MAXP];
    int cand[ORC_MAXP], taken[ORC_MAXP];
    int ncand = 0, ntaken = 0;
    for (int i = 0; i < m; ++i) {
        real g = G[i + i * m];
        if (!isfinite(g)) return -2;
        if (g < 0.0) return -1;
        s[i] = sqrt(g);
    }
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
            real g = G[i + j * m];
            if (!isfinite(g)) return -2;
            H[i + j * m] = (s[i] > 0.0 && s[j] > 0.0) ? g / (s[i] * s[j]) : 0.0;
        }
    for (int i = 0; i < m; ++i)
        if (s[i] > 0.0) cand[ncand++] = i;
    while (ncand > 0) {
        int best = 0;
        for (int c = 1; c < ncand; ++c)
            if (H[cand[c] + cand[c] * m] > H[cand[best] + cand[best] * m]) best = c;
        int piv = cand[best];
        real d = H[piv + piv * m];
        if (!(d > tau)) break;
        taken[ntaken++] = piv;
        for (int c = best; c + 1 < ncand; ++c) cand[c] = cand[c + 1];
        --ncand;
        /* Schur complement update of the remaining candidates. */
        real r = sqrt(d);
        real l[ORC_MAXP];
        for (int c = 0; c < ncand; ++c) l[c] = H[cand[c] + piv * m] / r;
        for (int a = 0; a < ncand; ++a)
            for (int c = 0; c < ncand; ++c)
                H[cand[c] + cand[a] * m] -= l[c] * l[a];
    }
    /* ascending order */
    for (int a = 0; a < ntaken; ++a)
        for (int c = a + 1; c < ntaken; ++c)
            if (taken[c] < taken[a]) { int t = taken[a]; taken[a] = taken[c]; taken[c] = t; }
    for (int a = 0; a < ntaken; ++a) keep[a] = taken[a];
    return ntaken;
}

static real norm2(int n, const real *v)
{
    real s = 0.0;
    for (int i = 0; i < n; ++i) s += v[i] * v[i];
    return sqrt(s);
}

/* T = B - A X for the columns listed in cols[0..m) of X (ldx); T is n x m. */
static void explicit_residual(int n, const double *A, int lda, const double *b,
                              const real *X, int ldx, int m, const int *cols, real *T)
{
    for (int c = 0; c < m; ++c) {
        real *t = T + (size_t)c * n;
        const real *x = X + (size_t)cols[c] * ldx;
#pragma omp parallel for schedule(static)
        for (int i0 = 0; i0 < n; i0 += (ORC_ROWS < n ? ORC_ROWS : n)) {
            int i1 = n - i0 > ORC_ROWS ? i0 + ORC_ROWS : n;
            for (int i = i0; i < i1; ++i) t[i] = 0.0;
            for (int k = 0; k < n; ++k) {
                const double *a = A + (size_t)k * lda;
                real xk = x[k];
                for (int i = i0; i < i1; ++i) t[i] += a[i] * xk;
            }
            for (int i = i0; i < i1; ++i) t[i] = b[i] - t[i];
        }
    }
}

/* T = B - A X for all p columns (exported for tests that need the plain residual). */
int oracle_residual(int n, int p, const double *A, int lda, const double *b,
                    const double *X, int ldx, double *T)
{
    if (n < 1 || p < 1 || lda < n || ldx < n) return ORC_ERR_ARG;
    int cols[ORC_MAXP];
    if (p > ORC_MAXP) return ORC_ERR_ARG;
    for (int j = 0; j < p; ++j) cols[j] = j;
    size_t np = (size_t)n * p;
    real *Xr = calloc(np, sizeof(real));
    real *Tr = calloc(np, sizeof(real));
    if (!Xr || !Tr) { free(Xr); free(Tr); return ORC_ERR_NOMEM; }
    for (int j = 0; j < p; ++j)
        for (int i = 0; i < n; ++i) Xr[i + (size_t)j * n] = X[i + (size_t)j * ldx];
    explicit_residual(n, A, lda, b, Xr, n, p, cols, Tr);
    for (size_t i = 0; i < np; ++i) T[i] = (double)Tr[i];
    free(Xr); free(Tr);
    return ORC_OK;
}

/*
 * cCG (Alg. 2 with the Table 1 residual recurrence and the Alg. 3 rank step).
 *
 *   X (in: X0, out: final agents), n x p, column-major, ldx >= n.
 *   tol > 0: relative stop test; tol == 0 runs exactly maxit steps (no stop test,
 *   no confirmation), which the per-step comparisons use.
 *   tau: rank threshold on the scaled pivots.
 *   trace_k > 0 records alpha_k and beta_k (p x p, column-major, in the ORIGINAL
 *   agent numbering, zero rows/columns for dropped agents) for the first trace_k
 *   steps into trace_alpha / trace_beta (each trace_k * p * p doubles).
 *   R_out, D_out (nullable): final R and D (n x p, leading dimension n; zero
 *   columns for dropped agents).
 *   reinflate_max: re-inflation events allowed (0: plain Alg. 3).  A policy beyond
 *   the paper: when the rank step would drop some (not all) agents, each agent outside the kept set
 *   J instead restarts from the iterate of the active agent with the smallest
 *   residual norm (ties: lowest index) plus a uniform draw in [-1, 1) per entry
 *   (SplitMix64, see reinflate_state), and the whole block restarts as Alg. 2 starts
 *   (R = B - A X, D = R, all p agents active), in place of that step.
 */
int oracle_ccg(int n, int p, const double *A, int lda, const double *b,
               double *X, int ldx, double tol, int maxit, double tau,
               int trace_k, double *trace_alpha, double *trace_beta,
               double *R_out, double *D_out, int reinflate_max, orc_info *info)
{
    orc_info inf;
    memset(&inf, 0, sizeof inf);
    inf.best_agent = -1;
    if (n < 1 || p < 1 || p > ORC_MAXP || p > n || lda < n || ldx < n || !(tol >= 0.0) ||
        maxit < 0 || !A || !b || !X) {
        inf.status = ORC_ERR_ARG;
        if (info) *info = inf;
        return ORC_ERR_ARG;
    }
    size_t np = (size_t)n * p;
    real *R = calloc(np, sizeof(real));
    real *D = calloc(np, sizeof(real));
    real *AD = calloc(np, sizeof(real));
    real *T = calloc(np, sizeof(real));
    real *Xa = calloc(np, sizeof(real));
    real *Xr = calloc(np, sizeof(real));   /* the agents, leading dimension n */
    if (!R || !D || !AD || !T || !Xa || !Xr) {
        free(R); free(D); free(AD); free(T); free(Xa); free(Xr);
        inf.status = ORC_ERR_NOMEM;
        if (info) *info = inf;
        return ORC_ERR_NOMEM;
    }
    int act[ORC_MAXP];   /* active agents (original indices), ascending */
    int m = p;
    for (int j = 0; j < p; ++j) act[j] = j;
    real G[ORC_MAXP * ORC_MAXP], S[ORC_MAXP * ORC_MAXP], L[ORC_MAXP * ORC_MAXP];
    real alpha[ORC_MAXP * ORC_MAXP], beta[ORC_MAXP * ORC_MAXP], W[ORC_MAXP * ORC_MAXP];
    int status = ORC_NOT_CONVERGED;
    int k = 0;
    for (int j = 0; j < p; ++j)
        for (int i = 0; i < n; ++i) Xr[i + (size_t)j * n] = X[i + (size_t)j * ldx];

    real nb = 0.0;
    for (int i = 0; i < n; ++i) nb += (real)b[i] * b[i];
    nb = sqrt(nb);
    if (!isfinite(nb)) { status = ORC_ERR_NONFINITE; goto done; }
    if (nb == 0.0) { status = ORC_ERR_ARG; goto done; }

    /* Alg. 2, first lines: R0 = B - A X0, D0 = R0.  Columns of R, D, AD, Xa are
     * stored compactly for the active agents: column c <-> agent act[c]. */
    explicit_residual(n, A, lda, b, Xr, n, m, act, R);
    memcpy(D, R, np * sizeof(real));
    if (trace_k > 0) {
        memset(trace_alpha, 0, (size_t)trace_k * p * p * sizeof(double));
        memset(trace_beta, 0, (size_t)trace_k * p * p * sizeof(double));
    }

    for (;;) {
        if (m == 0) { status = ORC_OK; break; }
        /* Stop test on the recurrence residual (Alg. 4: minimum over agents). */
        if (tol > 0.0) {
            real mn = INFINITY;
            for (int c = 0; c < m; ++c) {
                real r = norm2(n, R + (size_t)c * n) / nb;
                if (!isfinite(r)) { status = ORC_ERR_NONFINITE; goto done; }
                if (r < mn) mn = r;
            }
            if (mn <= tol) {
                /* confirm with the explicit residual */
                explicit_residual(n, A, lda, b, Xr, n, m, act, T);
                real tm = INFINITY;
                for (int c = 0; c < m; ++c) {
                    real r = norm2(n, T + (size_t)c * n) / nb;
                    if (r < tm) tm = r;
                }
                if (tm <= tol) { status = ORC_OK; break; }
                /* restart: R = B - A X, D = R */
                memcpy(R, T, (size_t)n * m * sizeof(real));
                memcpy(D, T, (size_t)n * m * sizeof(real));
                inf.restarts++;
            }
        }
        if (k >= maxit) { status = (tol > 0.0) ? ORC_NOT_CONVERGED : ORC_OK; break; }

        /* A D, then G = D^T A D and S = D^T R (Table 1, first three rows). */
        matmat(n, m, A, lda, D, n, AD, n);
        gram(n, m, D, AD, G);
        gram(n, m, D, R, S);

        /* Rank step (Alg. 3): keep a full-rank subset of the agents. */
        int keep[ORC_MAXP];
        int r = rank_select(m, G, tau, keep);
        if (r == -2) { status = ORC_ERR_NONFINITE; goto done; }
        if (r == -1) { status = ORC_ERR_NOT_SPD; goto done; }
        if (r > 0 && r < m && inf.reinflations < reinflate_max) {
            /* re-inflation (see above) in place of this step */
            int best = act[0];
            real bestn = norm2(n, R);
            for (int c = 1; c < m; ++c) {
                real v = norm2(n, R + (size_t)c * n);
                if (v < bestn) { bestn = v; best = act[c]; }
            }
            int kept[ORC_MAXP];
            for (int j = 0; j < p; ++j) kept[j] = 0;
            for (int q = 0; q < r; ++q) kept[act[keep[q]]] = 1;
            real *xb = T;                        /* the best iterate, copied first */
            for (int i = 0; i < n; ++i) xb[i] = Xr[i + (size_t)best * n];
            for (int j = 0; j < p; ++j) {
                if (kept[j]) continue;
                uint64_t st = reinflate_state(inf.reinflations, j);
                for (int i = 0; i < n; ++i) Xr[i + (size_t)j * n] = xb[i] + unit_draw(splitmix64_next(&st));
            }
            m = p;
            for (int j = 0; j < p; ++j) act[j] = j;
            explicit_residual(n, A, lda, b, Xr, n, m, act, R);
            memcpy(D, R, (size_t)n * m * sizeof(real));
            inf.reinflations++;
            continue;
        }
        if (r < m) {
            inf.deflations++;
            /* restrict columns and the p x p blocks to keep[] */
            real G2[ORC_MAXP * ORC_MAXP], S2[ORC_MAXP * ORC_MAXP];
            for (int b2 = 0; b2 < r; ++b2)
                for (int a2 = 0; a2 < r; ++a2) {
                    G2[a2 + b2 * r] = G[keep[a2] + keep[b2] * m];
                    S2[a2 + b2 * r] = S[keep[a2] + keep[b2] * m];
                }
            memcpy(G, G2, sizeof(real) * r * r);
            memcpy(S, S2, sizeof(real) * r * r);
            for (int c = 0; c < r; ++c) {
                int src = keep[c];
                if (src != c) {
                    memmove(R + (size_t)c * n, R + (size_t)src * n, (size_t)n * sizeof(real));
                    memmove(D + (size_t)c * n, D + (size_t)src * n, (size_t)n * sizeof(real));
                    memmove(AD + (size_t)c * n, AD + (size_t)src * n, (size_t)n * sizeof(real));
                }
                act[c] = act[src];
            }
            m = r;
            if (m == 0) { status = ORC_OK; break; }
        }

        /* alpha = G^{-1} S  (Alg. 2; Sec. 3.1 optimality of the descent step) */
        if (cholesky(m, G, L) != 0) { status = ORC_ERR_NOT_SPD; goto done; }
        chol_solve(m, L, m, S, alpha);

        /* X += D alpha ; R -= (A D) alpha   (Alg. 2 update of X; Table 1 for R) */
        for (int c = 0; c < m; ++c) {
            real *x = Xr + (size_t)act[c] * n;
            real *rr = R + (size_t)c * n;
            for (int l = 0; l < m; ++l) {
                real a = alpha[l + c * m];
                const real *d = D + (size_t)l * n;
                const real *ad = AD + (size_t)l * n;
                for (int i = 0; i < n; ++i) {
                    x[i] += d[i] * a;
                    rr[i] -= ad[i] * a;
                }
            }
        }

        /* beta = -G^{-1} (A D)^T R_{k+1}   (Alg. 2; Sec. 3.1 orthogonalization) */
        gram(n, m, AD, R, W);
        chol_solve(m, L, m, W, beta);
        for (int i = 0; i < m * m; ++i) beta[i] = -beta[i];

        if (k < trace_k) {
            double *ta = trace_alpha + (size_t)k * p * p;
            double *tb = trace_beta + (size_t)k * p * p;
            for (int b2 = 0; b2 < m; ++b2)
                for (int a2 = 0; a2 < m; ++a2) {
                    ta[act[a2] + act[b2] * p] = (double)alpha[a2 + b2 * m];
                    tb[act[a2] + act[b2] * p] = (double)beta[a2 + b2 * m];
                }
        }

        /* D = R + D beta   (Alg. 2 direction update); build into T, then copy. */
        for (int c = 0; c < m; ++c) {
            real *t = T + (size_t)c * n;
            const real *rr = R + (size_t)c * n;
            for (int i = 0; i < n; ++i) t[i] = rr[i];
            for (int l = 0; l < m; ++l) {
                real bb = beta[l + c * m];
                const real *d = D + (size_t)l * n;
                for (int i = 0; i < n; ++i) t[i] += d[i] * bb;
            }
        }
        memcpy(D, T, (size_t)n * m * sizeof(real));
        ++k;
    }

done:
    inf.iters = k;
    inf.p_final = m;
    if (status >= 0) {
        /* explicit residual of every agent; best agent */
        int all[ORC_MAXP];
        for (int j = 0; j < p; ++j) all[j] = j;
        explicit_residual(n, A, lda, b, Xr, n, p, all, Xa);
        real mn = INFINITY, mx = 0.0;
        for (int j = 0; j < p; ++j) {
            real r = norm2(n, Xa + (size_t)j * n) / nb;
            if (r < mn) { mn = r; inf.best_agent = j; }
            if (r > mx) mx = r;
        }
        inf.rel_res = (double)mn;
        inf.rel_res_max = (double)mx;
    }
    for (int j = 0; j < p; ++j)
        for (int i = 0; i < n; ++i) X[i + (size_t)j * ldx] = (double)Xr[i + (size_t)j * n];
    if (R_out || D_out) {
        if (R_out) memset(R_out, 0, np * sizeof(double));
        if (D_out) memset(D_out, 0, np * sizeof(double));
        for (int c = 0; c < m; ++c)
            for (int i = 0; i < n; ++i) {
                if (R_out) R_out[(size_t)act[c] * n + i] = (double)R[(size_t)c * n + i];
                if (D_out) D_out[(size_t)act[c] * n + i] = (double)D[(size_t)c * n + i];
            }
    }
    inf.status = status;
    if (info) *info = inf;
    free(R); free(D); free(AD); free(T); free(Xa); free(Xr);
    return status;
}

/* Textbook CG is the p = 1 case of the routine above (Sec. 3.2); no separate
 * entry point is exported so that the tests compare against an independent one. */
