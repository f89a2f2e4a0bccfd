/*
 * FP64 CPU oracle for augmented preconditioned conjugate gradients (APCG)
 * with Krylov reuse — TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously-correct reference that the HIP
 * library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code with the
 * library: no headers, helpers or kernels.
 *
 * Source: Gosselet, Rey, Pebrel, "Total and selective reuse of Krylov
 * subspaces for the resolution of sequences of nonlinear structural
 * problems" (arXiv 1301.7530).  Each function names the passage it follows.
 *
 * Conventions: CSR matrices with int64 row pointers and int32 columns, dense
 * blocks column-major with an explicit leading dimension, everything in
 * double precision, single thread.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_OK = 0, ORC_MAXIT = 1, ORC_BREAKDOWN = 2, ORC_INVALID = 3, ORC_NOMEM = 4 };
enum { ORC_PC_NONE = 0, ORC_PC_JACOBI = 1, ORC_PC_BLOCK3 = 3 };

/* ---------------------------------------------------------------- basics */

/* y = A x for CSR A. */
/* Accumulation of sums: double (the default), or the x87 extended type
 * (64-bit significand) when an APCG call asks for ORC_OPT_EXTENDED, set for
 * the duration of that call.  Both are faithful evaluations of the same
 * sums; comparing them shows how much rounding alone moves a long run. */
static __thread int g_extended = 0;

void orc_spmv(int64_t n, const int64_t* rp, const int32_t* ci, const double* av, const double* x, double* y) {
    for (int64_t i = 0; i < n; ++i) {
        if (g_extended) {
            long double s = 0.0L;
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s += (long double)av[k] * (long double)x[ci[k]];
            y[i] = (double)s;
        } else {
            double s = 0.0;
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s += av[k] * x[ci[k]];
            y[i] = s;
        }
    }
}

double orc_dot(int64_t n, const double* a, const double* b) {
    if (g_extended) {
        long double s = 0.0L;
        for (int64_t i = 0; i < n; ++i) s += (long double)a[i] * (long double)b[i];
        return (double)s;
    }
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Entry (i, j) of a CSR matrix, 0 if not stored. */
static double csr_entry(const int64_t* rp, const int32_t* ci, const double* av, int64_t i, int64_t j) {
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] == j) return av[k];
    return 0.0;
}

/* ------------------------------------------------------- preconditioner */
/*
 * M is the diagonal of A (Jacobi) or its 3x3 nodal diagonal blocks
 * (dofs 3p..3p+2).  M^{-1} r is obtained by solving M s = r; for the block
 * case each 3x3 block is Cholesky-factored once (Section 2.1: M symmetric
 * positive definite).
 */
typedef struct {
    int kind;
    int64_t n;
    double* f; /* Jacobi: diag; block: 6 Cholesky factor entries per node */
} orc_prec;

static int prec_setup(orc_prec* P, int kind, int64_t n, const int64_t* rp, const int32_t* ci, const double* av) {
    P->kind = kind;
    P->n = n;
    P->f = NULL;
    if (kind == ORC_PC_NONE) return ORC_OK;
    if (kind == ORC_PC_JACOBI) {
        P->f = (double*)malloc(sizeof(double) * (size_t)n);
        if (!P->f) return ORC_NOMEM;
        for (int64_t i = 0; i < n; ++i) {
            P->f[i] = csr_entry(rp, ci, av, i, i);
            if (!(P->f[i] > 0.0)) return ORC_INVALID;
        }
        return ORC_OK;
    }
    if (kind == ORC_PC_BLOCK3) {
        if (n % 3) return ORC_INVALID;
        int64_t nb = n / 3;
        P->f = (double*)malloc(sizeof(double) * 6 * (size_t)nb);
        if (!P->f) return ORC_NOMEM;
        for (int64_t p = 0; p < nb; ++p) {
            double m[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) m[a][b] = csr_entry(rp, ci, av, 3 * p + a, 3 * p + b);
            /* lower Cholesky factor L of the block: l00, l10, l11, l20, l21, l22 */
            double l00 = m[0][0];
            if (!(l00 > 0.0)) return ORC_INVALID;
            l00 = sqrt(l00);
            double l10 = m[1][0] / l00, l20 = m[2][0] / l00;
            double l11 = m[1][1] - l10 * l10;
            if (!(l11 > 0.0)) return ORC_INVALID;
            l11 = sqrt(l11);
            double l21 = (m[2][1] - l20 * l10) / l11;
            double l22 = m[2][2] - l20 * l20 - l21 * l21;
            if (!(l22 > 0.0)) return ORC_INVALID;
            l22 = sqrt(l22);
            double* f = P->f + 6 * p;
            f[0] = l00; f[1] = l10; f[2] = l11; f[3] = l20; f[4] = l21; f[5] = l22;
        }
        return ORC_OK;
    }
    return ORC_INVALID;
}

/* s = M^{-1} r */
static void prec_apply(const orc_prec* P, const double* r, double* s) {
    int64_t n = P->n;
    if (P->kind == ORC_PC_NONE) {
        memcpy(s, r, sizeof(double) * (size_t)n);
    } else if (P->kind == ORC_PC_JACOBI) {
        for (int64_t i = 0; i < n; ++i) s[i] = r[i] / P->f[i];
    } else {
        for (int64_t p = 0; p < n / 3; ++p) {
            const double* f = P->f + 6 * p;
            const double* rr = r + 3 * p;
            /* L y = r */
            double y0 = rr[0] / f[0];
            double y1 = (rr[1] - f[1] * y0) / f[2];
            double y2 = (rr[2] - f[3] * y0 - f[4] * y1) / f[5];
            /* L^T s = y */
            double s2 = y2 / f[5];
            double s1 = (y1 - f[4] * s2) / f[2];
            double s0 = (y0 - f[1] * s1 - f[3] * s2) / f[0];
            s[3 * p] = s0; s[3 * p + 1] = s1; s[3 * p + 2] = s2;
        }
    }
}

static void prec_free(orc_prec* P) { free(P->f); P->f = NULL; }

/* ------------------------------------------------------- coarse problem */
/*
 * Coarse matrix G = C^T A C (Section 2.1, the initialisation/projector pair;
 * Section 2.3 lists its construction and factorisation).  Its Cholesky
 * factor is computed column by column; a column whose pivot falls to
 * guard * max_i G_ii or below is declared dependent and dropped (the paper
 * leaves the full-rank check open, Section 2.3; this rule is the reading
 * adopted here, with guard = 1e-6 by default: the kept coarse matrix then
 * has a condition number of at most about 1e6, so the double-precision
 * projector stays accurate well below a 1e-8 tolerance).  Only the kept
 * columns take part in the projector.
 */
typedef struct {
    int nc, nk;
    int* kept;        /* indices of kept columns, nk of them */
    double* Ck;       /* n x nk, kept columns of C */
    double* Qk;       /* n x nk, A Ck */
    double* L;        /* nk x nk lower Cholesky factor of Ck^T A Ck, column-major */
    double* tmp;      /* nk */
    int64_t n;
} orc_coarse;

/* mu = G^{-1} v using the kept factor (forward then backward substitution). */
static void coarse_solve(const orc_coarse* K, const double* v, double* mu) {
    int nk = K->nk;
    const double* L = K->L;
    for (int i = 0; i < nk; ++i) {
        double s = v[i];
        for (int k = 0; k < i; ++k) s -= L[i + (size_t)k * nk] * mu[k];
        mu[i] = s / L[i + (size_t)i * nk];
    }
    for (int i = nk - 1; i >= 0; --i) {
        double s = mu[i];
        for (int k = i + 1; k < nk; ++k) s -= L[k + (size_t)i * nk] * mu[k];
        mu[i] = s / L[i + (size_t)i * nk];
    }
}

static int coarse_build(orc_coarse* K, int64_t n, const int64_t* rp, const int32_t* ci, const double* av,
                        const double* C, int nc, int64_t ldc, double guard, int* kept_flags) {
    memset(K, 0, sizeof(*K));
    K->n = n;
    K->nc = nc;
    if (nc <= 0) return ORC_OK;
    double* Q = (double*)malloc(sizeof(double) * (size_t)n * nc);
    double* G = (double*)malloc(sizeof(double) * (size_t)nc * nc);
    double* Lfull = (double*)calloc((size_t)nc * nc, sizeof(double));
    int* kept = (int*)malloc(sizeof(int) * nc);
    if (!Q || !G || !Lfull || !kept) { free(Q); free(G); free(Lfull); free(kept); return ORC_NOMEM; }
    for (int c = 0; c < nc; ++c) orc_spmv(n, rp, ci, av, C + (size_t)c * ldc, Q + (size_t)c * n);
    for (int a = 0; a < nc; ++a)
        for (int b = 0; b < nc; ++b) G[a + (size_t)b * nc] = orc_dot(n, C + (size_t)a * ldc, Q + (size_t)b * n);
    /* symmetrise: G <- (G + G^T)/2 */
    for (int a = 0; a < nc; ++a)
        for (int b = a + 1; b < nc; ++b) {
            double s = 0.5 * (G[a + (size_t)b * nc] + G[b + (size_t)a * nc]);
            G[a + (size_t)b * nc] = s;
            G[b + (size_t)a * nc] = s;
        }
    double maxdiag = 0.0;
    for (int a = 0; a < nc; ++a) if (G[a + (size_t)a * nc] > maxdiag) maxdiag = G[a + (size_t)a * nc];
    int nk = 0;
    /* left-looking Cholesky over the kept columns, in column order */
    for (int j = 0; j < nc; ++j) {
        double d = G[j + (size_t)j * nc];
        for (int t = 0; t < nk; ++t) { int k = kept[t]; d -= Lfull[j + (size_t)k * nc] * Lfull[j + (size_t)k * nc]; }
        if (!(d > guard * maxdiag)) { if (kept_flags) kept_flags[j] = 0; continue; }
        double ljj = sqrt(d);
        Lfull[j + (size_t)j * nc] = ljj;
        for (int i = j + 1; i < nc; ++i) {
            double s = G[i + (size_t)j * nc];
            for (int t = 0; t < nk; ++t) { int k = kept[t]; s -= Lfull[i + (size_t)k * nc] * Lfull[j + (size_t)k * nc]; }
            Lfull[i + (size_t)j * nc] = s / ljj;
        }
        kept[nk++] = j;
        if (kept_flags) kept_flags[j] = 1;
    }
    K->nk = nk;
    K->kept = kept;
    K->Ck = (double*)malloc(sizeof(double) * (size_t)n * (nk ? nk : 1));
    K->Qk = (double*)malloc(sizeof(double) * (size_t)n * (nk ? nk : 1));
    K->L = (double*)malloc(sizeof(double) * (size_t)(nk ? nk : 1) * (nk ? nk : 1));
    K->tmp = (double*)malloc(sizeof(double) * (size_t)(nk ? nk : 1));
    if (!K->Ck || !K->Qk || !K->L || !K->tmp) { free(Q); free(G); free(Lfull); return ORC_NOMEM; }
    for (int t = 0; t < nk; ++t) {
        memcpy(K->Ck + (size_t)t * n, C + (size_t)kept[t] * ldc, sizeof(double) * (size_t)n);
        memcpy(K->Qk + (size_t)t * n, Q + (size_t)kept[t] * n, sizeof(double) * (size_t)n);
        for (int u = 0; u < nk; ++u) K->L[u + (size_t)t * nk] = Lfull[kept[u] + (size_t)kept[t] * nc];
    }
    free(Q); free(G); free(Lfull);
    return ORC_OK;
}

/* Replace the kept basis by an A-orthonormal one of the same span:
 * Ck <- Ck L^{-T}, Qk <- Qk L^{-T} (so Ck^T A Ck = L^{-1} G L^{-T} = I) and
 * L <- I.  The projector P = I - C G^{-1} (A C)^T is unchanged in exact
 * arithmetic; its rounding no longer carries the condition number of G. */
static void coarse_orthonormalize(orc_coarse* K) {
    const int nk = K->nk;
    const int64_t n = K->n;
    if (nk <= 0) return;
    /* rows of X L^T = Y solved by forward substitution: for each row i,
     * y_t = (x_t - sum_{k<t} y_k L[t,k]) / L[t,t] */
    double* row = (double*)malloc(sizeof(double) * (size_t)nk);
    double* rq = (double*)malloc(sizeof(double) * (size_t)nk);
    if (!row || !rq) { free(row); free(rq); return; }
    for (int64_t i = 0; i < n; ++i) {
        for (int t = 0; t < nk; ++t) {
            double a = K->Ck[(size_t)t * n + i], q = K->Qk[(size_t)t * n + i];
            for (int k = 0; k < t; ++k) {
                const double l = K->L[t + (size_t)k * nk];
                a -= row[k] * l;
                q -= rq[k] * l;
            }
            row[t] = a / K->L[t + (size_t)t * nk];
            rq[t] = q / K->L[t + (size_t)t * nk];
        }
        for (int t = 0; t < nk; ++t) {
            K->Ck[(size_t)t * n + i] = row[t];
            K->Qk[(size_t)t * n + i] = rq[t];
        }
    }
    for (int a = 0; a < nk; ++a)
        for (int b = 0; b < nk; ++b) K->L[a + (size_t)b * nk] = (a == b) ? 1.0 : 0.0;
    free(row);
    free(rq);
}

static void coarse_free(orc_coarse* K) {
    free(K->kept); free(K->Ck); free(K->Qk); free(K->L); free(K->tmp);
    memset(K, 0, sizeof(*K));
}

/* z = P s = s - C G^{-1} (A C)^T s  (Section 2.1, projector P) */
static void project(const orc_coarse* K, const double* s, double* z, double* mu) {
    int64_t n = K->n;
    memcpy(z, s, sizeof(double) * (size_t)n);
    if (K->nk == 0) return;
    for (int t = 0; t < K->nk; ++t) K->tmp[t] = orc_dot(n, K->Qk + (size_t)t * n, s);
    coarse_solve(K, K->tmp, mu);
    for (int t = 0; t < K->nk; ++t) {
        const double* c = K->Ck + (size_t)t * n;
        double m = mu[t];
        for (int64_t i = 0; i < n; ++i) z[i] -= c[i] * m;
    }
}

/* Gram-Schmidt coefficient of direction i: out[i] = (A w_i, z) / (w_i, A w_i). */
static void mu_h(const double* Qall, const double* gam, int64_t n, int i, const double* z, double* out) {
    out[i] = orc_dot(n, Qall + (size_t)i * n, z) / gam[i];
}

/* ------------------------------------------------------------------ APCG */
/*
 * APCG(A, M, C, b) — Algorithm 1 with the initialisation/projector pair of
 * Section 2.1, written in the standard (Hestenes–Stiefel) form:
 *
 *   x0 = C G^{-1} C^T b,  r0 = b - A x0,  z0 = P M^{-1} r0,  w0 = z0,
 *   rho_j   = (r_j, z_j)
 *   alpha_j = rho_j / (w_j, A w_j)
 *   x_{j+1} = x_j + alpha_j w_j,   r_{j+1} = r_j - alpha_j A w_j
 *   z_{j+1} = P M^{-1} r_{j+1}
 *   beta_{j+1} = rho_{j+1} / rho_j, w_{j+1} = z_{j+1} + beta_{j+1} w_j
 *
 * The algorithm as printed obtains w_{j+1} by A-orthogonalising z_{j+1}
 * against w_j, which in exact arithmetic is the same vector with the sign
 * of beta flipped; orc_apcg_alg1 below keeps that form for cross-checks.
 * The recurrence stops after the first update with ||r|| <= tol ||b||, or
 * after max_iter updates; m is the number of products A w_j performed.
 * With x00 = 0 (Section 2.1).  If r0 already meets the tolerance, m = 0.
 *
 * Outputs (any pointer may be NULL except x):
 *   alpha[j], gamma[j] = (w_j, A w_j), j < m;  rho[j], j <= m-1 (and rho[m]
 *   when a further direction was formed); resn[j] = ||r_j||, j <= m;
 *   Z, W: columns j < m of z_j, w_j (leading dims ldz, ldw);
 *   kept[c] = 1 if column c survived the rank guard.
 *
 * opts (0 = the update above):
 *   ORC_OPT_PROJECT_OLD: the next direction is z_{j+1} + beta P w_j, the
 *     projector applied to the old direction too (P w_j = w_j in exact
 *     arithmetic, so this is the same iteration; it is the library's
 *     default form, kept here to measure what the difference does).
 *   ORC_OPT_ORTHONORMAL: after the guarded Cholesky G = L L^T of the kept
 *     columns, work with the A-orthonormal basis C L^{-T} (same span, same
 *     projector in exact arithmetic) instead of C and the factor.
 *   ORC_OPT_EXTENDED: matrix-vector products and dot products accumulated
 *     in extended precision (then rounded to double).
 *   ORC_OPT_REORTH: full reorthogonalisation, which the paper states APCG
 *     admits (Section 2.1) and uses in every experiment (Section 5.1): the
 *     next direction is z_{j+1} made A-orthogonal to every earlier one,
 *       w_{j+1} = z_{j+1} - sum_{i<=j} ((A w_i, z_{j+1}) / (w_i, A w_i)) w_i
 *     (classical Gram-Schmidt in the A inner product over the stored w_i
 *     and A w_i).  In exact arithmetic only the i = j term is nonzero and it
 *     equals beta_{j+1} w_j.  rho and beta keep their definitions, so the
 *     Lanczos coefficients of Section 4.1 are unchanged.
 */
enum { ORC_OPT_PROJECT_OLD = 1, ORC_OPT_REORTH = 2, ORC_OPT_ORTHONORMAL = 4, ORC_OPT_EXTENDED = 8 };

int orc_apcg(int64_t n, const int64_t* rp, const int32_t* ci, const double* av, int precond,
             const double* C, int nc, int64_t ldc, const double* b, double tol, int max_iter, double guard,
             double* x, double* alpha, double* rho, double* gamma, double* resn,
             double* Z, int64_t ldz, double* W, int64_t ldw, int* kept, int* m_out, double* relres_true,
             int opts) {
    if (n <= 0 || max_iter < 0 || (nc > 0 && (!C || ldc < n))) return ORC_INVALID;
    g_extended = (opts & ORC_OPT_EXTENDED) != 0;
    orc_prec P;
    int st = prec_setup(&P, precond, n, rp, ci, av);
    if (st != ORC_OK) { prec_free(&P); g_extended = 0; return st; }
    orc_coarse K;
    st = coarse_build(&K, n, rp, ci, av, C, nc, ldc, guard, kept);
    if (st != ORC_OK) { prec_free(&P); coarse_free(&K); g_extended = 0; return st; }
    if (opts & ORC_OPT_ORTHONORMAL) coarse_orthonormalize(&K);

    double* r = (double*)malloc(sizeof(double) * (size_t)n);
    double* s = (double*)malloc(sizeof(double) * (size_t)n);
    double* z = (double*)malloc(sizeof(double) * (size_t)n);
    double* w = (double*)malloc(sizeof(double) * (size_t)n);
    double* q = (double*)malloc(sizeof(double) * (size_t)n);
    double* mu = (double*)malloc(sizeof(double) * (size_t)(K.nk > 0 ? K.nk : 1));
    /* every direction and its product with A, for the reorthogonalisation */
    const int reorth = (opts & ORC_OPT_REORTH) != 0;
    const size_t hcols = reorth ? (size_t)max_iter + 1 : 0;
    double* Wall = reorth ? (double*)malloc(sizeof(double) * (size_t)n * hcols) : NULL;
    double* Qall = reorth ? (double*)malloc(sizeof(double) * (size_t)n * hcols) : NULL;
    double* gam = reorth ? (double*)malloc(sizeof(double) * hcols) : NULL;
    double* gsc = reorth ? (double*)malloc(sizeof(double) * hcols) : NULL;
    double* pw = (opts & ORC_OPT_PROJECT_OLD) ? (double*)malloc(sizeof(double) * (size_t)n) : NULL;
    double* pmu = (opts & ORC_OPT_PROJECT_OLD) ? (double*)malloc(sizeof(double) * (size_t)(K.nk > 0 ? K.nk : 1)) : NULL;
    if (!r || !s || !z || !w || !q || !mu || (reorth && (!Wall || !Qall || !gam || !gsc)) ||
        ((opts & ORC_OPT_PROJECT_OLD) && (!pw || !pmu))) { st = ORC_NOMEM; goto out; }

    double bnorm = sqrt(orc_dot(n, b, b));
    /* initialisation: x0 = C G^{-1} C^T b, r0 = b - A C mu0 */
    memset(x, 0, sizeof(double) * (size_t)n);
    memcpy(r, b, sizeof(double) * (size_t)n);
    if (K.nk > 0) {
        for (int t = 0; t < K.nk; ++t) K.tmp[t] = orc_dot(n, K.Ck + (size_t)t * n, b);
        coarse_solve(&K, K.tmp, mu);
        for (int t = 0; t < K.nk; ++t) {
            const double* c = K.Ck + (size_t)t * n;
            const double* aq = K.Qk + (size_t)t * n;
            for (int64_t i = 0; i < n; ++i) { x[i] += c[i] * mu[t]; r[i] -= aq[i] * mu[t]; }
        }
    }
    double rn = sqrt(orc_dot(n, r, r));
    if (resn) resn[0] = rn;
    int m = 0;
    st = ORC_OK;
    if (!(rn > tol * bnorm) || max_iter == 0) {
        if (max_iter == 0 && rn > tol * bnorm) st = ORC_MAXIT;
        goto done;
    }
    prec_apply(&P, r, s);
    project(&K, s, z, mu);
    double rh = orc_dot(n, r, z);
    memcpy(w, z, sizeof(double) * (size_t)n);
    if (rho) rho[0] = rh;
    for (int j = 0;; ++j) {
        if (Z) memcpy(Z + (size_t)j * ldz, z, sizeof(double) * (size_t)n);
        if (W) memcpy(W + (size_t)j * ldw, w, sizeof(double) * (size_t)n);
        orc_spmv(n, rp, ci, av, w, q);
        double g = orc_dot(n, w, q);
        if (gamma) gamma[j] = g;
        if (reorth) {
            memcpy(Wall + (size_t)j * n, w, sizeof(double) * (size_t)n);
            memcpy(Qall + (size_t)j * n, q, sizeof(double) * (size_t)n);
            gam[j] = g;
        }
        if (!(g > 0.0) || !(rh > 0.0)) { m = j; st = ORC_BREAKDOWN; goto done; }
        double a = rh / g;
        if (alpha) alpha[j] = a;
        for (int64_t i = 0; i < n; ++i) { x[i] += a * w[i]; r[i] -= a * q[i]; }
        rn = sqrt(orc_dot(n, r, r));
        if (resn) resn[j + 1] = rn;
        m = j + 1;
        if (!(rn > tol * bnorm)) break;
        if (m == max_iter) { st = ORC_MAXIT; break; }
        prec_apply(&P, r, s);
        project(&K, s, z, mu);
        double rh_new = orc_dot(n, r, z);
        double be = rh_new / rh;
        if (reorth) {
            /* classical Gram-Schmidt in the A inner product: all the
             * coefficients from z, then one update */
            for (int i = 0; i <= j; ++i) mu_h(Qall, gam, n, i, z, gsc);
            memcpy(w, z, sizeof(double) * (size_t)n);
            for (int i = 0; i <= j; ++i) {
                const double c = gsc[i];
                const double* wi = Wall + (size_t)i * n;
                for (int64_t t = 0; t < n; ++t) w[t] -= c * wi[t];
            }
        } else if (opts & ORC_OPT_PROJECT_OLD) {
            project(&K, w, pw, pmu);
            for (int64_t i = 0; i < n; ++i) w[i] = z[i] + be * pw[i];
        } else {
            for (int64_t i = 0; i < n; ++i) w[i] = z[i] + be * w[i];
        }
        rh = rh_new;
        if (rho) rho[j + 1] = rh;
    }
done:
    if (relres_true) {
        orc_spmv(n, rp, ci, av, x, q);
        double t = 0.0;
        for (int64_t i = 0; i < n; ++i) { double d = b[i] - q[i]; t += d * d; }
        *relres_true = bnorm > 0.0 ? sqrt(t) / bnorm : sqrt(t);
    }
    if (m_out) *m_out = m;
out:
    free(r); free(s); free(z); free(w); free(q); free(mu);
    free(Wall); free(Qall); free(gam); free(gsc); free(pw); free(pmu);
    prec_free(&P);
    coarse_free(&K);
    g_extended = 0;
    return st;
}

/*
 * Cross-check of the standard form against the conjugacy conditions that
 * define APCG (Section 2.1), on small inputs.  Each step takes the step
 * length that makes the new residual orthogonal to the current direction,
 *   (r_j - a A w_j, w_j) = 0,
 * and builds the next direction from the projected preconditioned residual
 * by removing its A-component along the current direction,
 *   (z + c w_j, A w_j) = 0.
 * Algorithm 1 prints this Gram-Schmidt form (its coefficient is -c); the
 * standard form replaces the two inner products by rho ratios, equal in
 * exact arithmetic.  Runs exactly `iters` steps with no stopping test and
 * returns the step lengths a_j and the Gram-Schmidt coefficients
 * gs[j] = -c_j (j >= 1; gs[0] unused).
 */
static double conj_step_length(int64_t n, const double* r, const double* w, const double* aw, double waw) {
    return orc_dot(n, r, w) / waw;
}

static double conj_gs_coeff(int64_t n, const double* z, const double* aw, double waw) {
    return orc_dot(n, z, aw) / waw;
}

int orc_apcg_alg1(int64_t n, const int64_t* rp, const int32_t* ci, const double* av, int precond,
                  const double* C, int nc, int64_t ldc, const double* b, int iters, double guard,
                  double* x, double* alpha, double* bgs) {
    orc_prec P;
    int st = prec_setup(&P, precond, n, rp, ci, av);
    if (st != ORC_OK) { prec_free(&P); return st; }
    orc_coarse K;
    st = coarse_build(&K, n, rp, ci, av, C, nc, ldc, guard, NULL);
    if (st != ORC_OK) { prec_free(&P); coarse_free(&K); return st; }
    double* res = (double*)malloc(sizeof(double) * (size_t)n);
    double* pre = (double*)malloc(sizeof(double) * (size_t)n);
    double* dir = (double*)malloc(sizeof(double) * (size_t)n);
    double* adir = (double*)malloc(sizeof(double) * (size_t)n);
    double* zz = (double*)malloc(sizeof(double) * (size_t)n);
    double* cmu = (double*)malloc(sizeof(double) * (size_t)(K.nk > 0 ? K.nk : 1));
    if (!res || !pre || !dir || !adir || !zz || !cmu) { st = ORC_NOMEM; goto fin; }
    /* start: x0 = C G^-1 C^T b and its residual (the initialisation of P) */
    memset(x, 0, sizeof(double) * (size_t)n);
    memcpy(res, b, sizeof(double) * (size_t)n);
    if (K.nk > 0) {
        for (int t = 0; t < K.nk; ++t) K.tmp[t] = orc_dot(n, K.Ck + (size_t)t * n, b);
        coarse_solve(&K, K.tmp, cmu);
        for (int t = 0; t < K.nk; ++t)
            for (int64_t i = 0; i < n; ++i) { x[i] += K.Ck[(size_t)t * n + i] * cmu[t]; res[i] -= K.Qk[(size_t)t * n + i] * cmu[t]; }
    }
    prec_apply(&P, res, pre);
    project(&K, pre, dir, cmu);
    for (int j = 0; j < iters; ++j) {
        orc_spmv(n, rp, ci, av, dir, adir);
        const double waw = orc_dot(n, dir, adir);
        const double a = conj_step_length(n, res, dir, adir, waw);
        alpha[j] = a;
        for (int64_t i = 0; i < n; ++i) x[i] += a * dir[i];
        for (int64_t i = 0; i < n; ++i) res[i] -= a * adir[i];
        if (j + 1 == iters) break;
        prec_apply(&P, res, pre);
        project(&K, pre, zz, cmu);
        const double g = conj_gs_coeff(n, zz, adir, waw);  /* = -c */
        bgs[j + 1] = g;
        for (int64_t i = 0; i < n; ++i) dir[i] = zz[i] - g * dir[i];
    }
fin:
    free(res); free(pre); free(dir); free(adir); free(zz); free(cmu);
    prec_free(&P);
    coarse_free(&K);
    return st;
}

/* ------------------------------------------- Ritz analysis (Section 4.1) */
/*
 * The Lanczos tridiagonal H_m recovered from the CG coefficients has
 *   delta_0 = 1/alpha_0, delta_j = 1/alpha_j + beta_j/alpha_{j-1},
 *   eta_j   = sqrt(beta_{j+1})/alpha_j,
 * with beta_j = rho_j/rho_{j-1} > 0 (the standard, positive coefficient).
 * This is exactly H_m = L D L^T with D = diag(1/alpha_j) and L unit lower
 * bidiagonal with sub-diagonal entries sqrt(beta_{j+1}): expanding L D L^T
 * gives the diagonal d_j + l_{j-1}^2 d_{j-1} and the off-diagonal l_j d_j.
 * The eigenvalues are computed from the factored form (d_j = 1/alpha_j,
 * l_j^2 = beta_{j+1}), which determines them to high relative accuracy,
 * so that the 1e-14 relative stagnation test of Section 4.4 is meaningful
 * also for the small Ritz values.
 */

/* Number of eigenvalues of L D L^T strictly below sigma: the count of
 * negative pivots of L D L^T - sigma I = L+ D+ L+^T (stationary qd form). */
int orc_ldl_count(int m, const double* d, const double* l2, double sigma) {
    int cnt = 0;
    double s = -sigma;
    for (int i = 0; i < m; ++i) {
        double dp = d[i] + s;
        if (dp == 0.0) dp = -DBL_EPSILON * (fabs(d[i]) + fabs(s)) - DBL_MIN;
        if (dp < 0.0) ++cnt;
        if (i + 1 < m) s = (l2[i] * d[i] / dp) * s - sigma;
    }
    return cnt;
}

/*
 * All eigenvalues of L D L^T by bisection on the Sturm count, each to full
 * double-precision resolution, returned in DESCENDING order
 * theta[0] >= theta[1] >= ... (the ordering used by Algorithm 3).
 */
void orc_ldl_eigvals(int m, const double* d, const double* l2, double* theta) {
    if (m <= 0) return;
    /* Gershgorin interval of the explicit tridiagonal */
    double lo = 0.0, hi = 0.0;
    for (int i = 0; i < m; ++i) {
        double diag = d[i] + (i > 0 ? l2[i - 1] * d[i - 1] : 0.0);
        double off = (i > 0 ? sqrt(l2[i - 1]) * fabs(d[i - 1]) : 0.0) + (i + 1 < m ? sqrt(l2[i]) * fabs(d[i]) : 0.0);
        if (i == 0 || diag - off < lo) lo = diag - off;
        if (i == 0 || diag + off > hi) hi = diag + off;
    }
    if (lo > 0.0) lo = 0.0;
    hi = hi * (1.0 + 4.0 * DBL_EPSILON) + DBL_MIN;
    for (int k = 0; k < m; ++k) {
        /* k-th smallest: count(a) <= k < count(b) */
        double a = lo, b = hi;
        for (;;) {
            double mid = 0.5 * (a + b);
            if (mid <= a || mid >= b) break;
            if (orc_ldl_count(m, d, l2, mid) <= k) a = mid; else b = mid;
        }
        theta[m - 1 - k] = 0.5 * (a + b);
    }
}

/*
 * Unit eigenvector of the explicit symmetric tridiagonal (diagonal dg[m],
 * off-diagonal of[m-1]) for an eigenvalue estimate th, by inverse
 * iteration: three solves of (T - th I) v = v_prev with Gaussian
 * elimination and partial pivoting, each followed by normalisation.
 */
void orc_tridiag_eigvec(int m, const double* dg, const double* of, double th, double* v) {
    if (m <= 0) return;
    if (m == 1) { v[0] = 1.0; return; }
    double tn = 0.0;
    for (int i = 0; i < m; ++i) tn = fmax(tn, fabs(dg[i]) + (i ? fabs(of[i - 1]) : 0.0) + (i + 1 < m ? fabs(of[i]) : 0.0));
    double tiny = DBL_EPSILON * (tn > 0 ? tn : 1.0);
    /* banded LU with partial pivoting: U has diagonal u0, first u1, second u2 super-diagonals */
    double* u0 = (double*)malloc(sizeof(double) * m);
    double* u1 = (double*)malloc(sizeof(double) * m);
    double* u2 = (double*)malloc(sizeof(double) * m);
    double* lm = (double*)malloc(sizeof(double) * m);
    int* sw = (int*)malloc(sizeof(int) * m);
    /* factor T - th I */
    double a0 = dg[0] - th, a1 = of[0];
    for (int i = 0; i < m; ++i) {
        /* current row i has entries (a0 at col i, a1 at col i+1, a2 at col i+2) */
        double a2 = 0.0;
        if (i + 1 < m) {
            double b0 = of[i], b1 = dg[i + 1] - th, b2 = (i + 2 < m) ? of[i + 1] : 0.0;
            if (fabs(b0) > fabs(a0)) {
                /* swap rows i and i+1 */
                double t0 = a0, t1 = a1, t2 = a2;
                a0 = b0; a1 = b1; a2 = b2;
                b0 = t0; b1 = t1; b2 = t2;
                sw[i] = 1;
            } else sw[i] = 0;
            if (a0 == 0.0) a0 = tiny;
            double l = b0 / a0;
            lm[i] = l;
            u0[i] = a0; u1[i] = a1; u2[i] = a2;
            a0 = b1 - l * a1;
            a1 = b2 - l * a2;
        } else {
            if (a0 == 0.0) a0 = tiny;
            u0[i] = a0; u1[i] = 0.0; u2[i] = 0.0; sw[i] = 0; lm[i] = 0.0;
        }
    }
    for (int i = 0; i < m; ++i) v[i] = 1.0;
    for (int it = 0; it < 3; ++it) {
        /* apply L^{-1} with the recorded swaps */
        for (int i = 0; i + 1 < m; ++i) {
            if (sw[i]) { double t = v[i]; v[i] = v[i + 1]; v[i + 1] = t; }
            v[i + 1] -= lm[i] * v[i];
        }
        /* back substitution with U */
        for (int i = m - 1; i >= 0; --i) {
            double s = v[i];
            if (i + 1 < m) s -= u1[i] * v[i + 1];
            if (i + 2 < m) s -= u2[i] * v[i + 2];
            v[i] = s / u0[i];
        }
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += v[i] * v[i];
        nrm = sqrt(nrm);
        for (int i = 0; i < m; ++i) v[i] /= nrm;
    }
    /* fix the sign: largest-magnitude component positive */
    int im = 0;
    for (int i = 1; i < m; ++i) if (fabs(v[i]) > fabs(v[im])) im = i;
    if (v[im] < 0) for (int i = 0; i < m; ++i) v[i] = -v[i];
    free(u0); free(u1); free(u2); free(lm); free(sw);
}

/*
 * Dense symmetric eigenvalues by cyclic Jacobi rotations (for small test
 * matrices only): a is n x n column-major, overwritten; eigenvalues are
 * returned ascending.  Used to pin the tridiagonal routines to an
 * independent method.
 */
void orc_jacobi_eigvals(int n, double* a, double* ev) {
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p) for (int q = p + 1; q < n; ++q) off += a[p + q * n] * a[p + q * n];
        if (off < 1e-300) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = a[p + q * n];
                if (apq == 0.0) continue;
                double app = a[p + p * n], aqq = a[q + q * n];
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) {
                    double akp = a[k + p * n], akq = a[k + q * n];
                    a[k + p * n] = c * akp - s * akq;
                    a[k + q * n] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = a[p + k * n], aqk = a[q + k * n];
                    a[p + k * n] = c * apk - s * aqk;
                    a[q + k * n] = s * apk + c * aqk;
                }
            }
    }
    for (int i = 0; i < n; ++i) ev[i] = a[i + i * n];
    /* insertion sort ascending */
    for (int i = 1; i < n; ++i) {
        double v = ev[i];
        int j = i - 1;
        while (j >= 0 && ev[j] > v) { ev[j + 1] = ev[j]; --j; }
        ev[j + 1] = v;
    }
}

/* Dense Cholesky solve of SPD A (n x n column-major) x = b, for pins. */
int orc_dense_cholesky_solve(int n, const double* A, const double* b, double* x) {
    double* L = (double*)calloc((size_t)n * n, sizeof(double));
    if (!L) return ORC_NOMEM;
    for (int j = 0; j < n; ++j) {
        double d = A[j + (size_t)j * n];
        for (int k = 0; k < j; ++k) d -= L[j + (size_t)k * n] * L[j + (size_t)k * n];
        if (!(d > 0.0)) { free(L); return ORC_INVALID; }
        double ljj = sqrt(d);
        L[j + (size_t)j * n] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = A[i + (size_t)j * n];
            for (int k = 0; k < j; ++k) s -= L[i + (size_t)k * n] * L[j + (size_t)k * n];
            L[i + (size_t)j * n] = s / ljj;
        }
    }
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i + (size_t)k * n] * x[k];
        x[i] = s / L[i + (size_t)i * n];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int k = i + 1; k < n; ++k) s -= L[k + (size_t)i * n] * x[k];
        x[i] = s / L[i + (size_t)i * n];
    }
    free(L);
    return ORC_OK;
}
