/*
 * CPU oracle for the conjugate-gradient variants of Chen & Carson,
 * "Predict-and-recompute conjugate gradient variants".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the solver library links, loads or
 * calls this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU path.
 *
 * What it is: a plain, slow, step-by-step FP64 transcription of the
 * algorithms, written for checking by eye against the paper:
 *   - initialize (Appendix D, Alg. "Initializations"),
 *   - HS-CG      (Alg. 1, Hestenes-Stiefel, preconditioned),
 *   - PR-CG      (Alg. 2, predict nu' with eq. nuk_simplified, recompute nu),
 *   - pipe-PR-CG (Alg. 3, recurrences for w, w~, s~; recompute w = A r~),
 *   - M-CG and pipe-PR-M-CG (Appendix D; nu' = -nu + alpha^2 gamma),
 *   - GV-CG      (Appendix D, Ghysels-Vanroose pipelined CG),
 *   - CG-CG      (Appendix D, Chronopoulos-Gear CG),
 *   - two ablations from Section 2: PR-CG without the recompute of nu
 *     (eq. nuk_norecomp) and pipe-PR-CG without the recompute of w,
 *   - PR-CG with the unsimplified four-term prediction of eq. nuk, which
 *     keeps <s~, r> as an inner product of its own instead of taking it
 *     equal to <r~, s> (Appendix C).
 *
 * Arithmetic model (Section 3, eq. fp): every + - * / is rounded separately
 * (built with -ffp-contract=off -fno-fast-math).  A sparse product sums each
 * row sequentially in stored column order starting from 0.0.  An inner
 * product sums fixed 4096-entry chunks sequentially and then adds the chunk
 * sums in index order, so the result does not depend on the thread count.
 * The preconditioner is given by the reciprocal diagonal d (Jacobi,
 * M^{-1} v = d .* v); with no preconditioner every tilde vector is the same
 * array as its plain counterpart (r~ = r, s~ = s, w~ = w, u~ = u).
 *
 * Readings where the paper is silent (stopping, breakdown, scalar order):
 *   - the scalars alpha_{k-1}, nu'_k, beta_k of iteration k are formed as
 *     soon as their inputs exist, i.e. at the end of iteration k-1
 *     (Section 2.2.1 recommends forming them at the start of iteration k;
 *     the values are identical);
 *   - stop at the first k with ||r_k||_2 <= tol * ||b||_2 using the updated
 *     residual r_k (with no preconditioner ||r_k||^2 = nu_k, otherwise an
 *     extra inner product <r_k, r_k> joins the same reduction);
 *   - breakdown: the paper notes the variants break down when nu becomes
 *     negative; here nu_k <= 0, mu_k <= 0 or a non-finite scalar after the
 *     reduction of iteration k stops the solve with status BREAKDOWN and
 *     x = x_k;
 *   - a predicted nu'_{k+1} <= 0 (or non-finite) makes iteration k+1 the
 *     last one: its x and r updates use only alpha_k and are still taken,
 *     beta_{k+1} is replaced by 0, and after its reduction the solve ends as
 *     converged if ||r_{k+1}|| <= tol ||b||, else as BREAKDOWN with
 *     x = x_{k+1}.  (At finite termination nu' approximates ||r_{k+1}||^2 = 0
 *     and may round to a non-positive value; this keeps that step.);
 *   - order of checks after the reduction of iteration k: converged, then
 *     breakdown, then k == maxit, then the scalar step for iteration k+1;
 *   - ||b|| = 0 gives x = 0, 0 iterations, converged.
 * Every exported function is pinned by the CPU tests against something other
 * than itself: dense solves, Krylov-subspace optimality of the iterates,
 * exact rational arithmetic, finite termination, closed forms, the paper's
 * nu'-gap bound and the paper's printed table for its model problem.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    ORC_HS = 0,
    ORC_PR = 1,
    ORC_PIPE_PR = 2,
    ORC_M = 3,
    ORC_PIPE_M = 4,
    ORC_GV = 5,
    ORC_PR_NO_RECOMPUTE = 6,      /* nu'_k from nu'_{k-1}; nu never recomputed */
    ORC_PIPE_PR_NO_W_RECOMPUTE = 7, /* w kept as the predicted w'_k           */
    ORC_CG = 8,                     /* CG-CG (Chronopoulos-Gear, Appendix D)   */
    ORC_PR_UNSIMPLIFIED = 9         /* PR-CG predicting nu' with eq. nuk       */
};

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_BREAKDOWN = 2, ORC_EINVAL = -1, ORC_ENOMEM = -2 };

/* Optional per-iteration diagnostics; every pointer may be NULL.  Arrays
 * hold maxit+1 entries indexed by k.  Entries not defined for a variant are
 * left untouched. */
typedef struct {
    double* nu;        /* nu_k = <r~_k, r_k> (recomputed value)               */
    double* nup;       /* nu'_k, the predicted value used in beta_k (k >= 1)  */
    double* rr;        /* <r_k, r_k>                                          */
    double* mu;        /* mu_k = <p_k, s_k>                                   */
    double* alpha;     /* alpha_k                                             */
    double* beta;      /* beta_k (k >= 1)                                     */
    double* true_res;  /* ||b - A x_k|| / ||b||                               */
    double* err_a;     /* ||x* - x_k||_A (needs xstar)                        */
    double* orth;      /* |<p_{k-1}, s_k>| / (||p_{k-1}|| ||s_k||)  (k >= 1)  */
    const double* xstar;
} orc_diag;

typedef struct {
    int64_t n;
    const int32_t* row_ptr;
    const int32_t* col;
    const double* val;
} orc_csr;

/* ---------------------------------------------------------------- primitives */

/* y = A x: row sums in stored order (Section 3 eq. Ax). */
static void orc_spmv(const orc_csr* A, const double* x, double* y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < A->n; ++i) {
        double acc = 0.0;
        for (int32_t e = A->row_ptr[i]; e < A->row_ptr[i + 1]; ++e)
            acc = acc + A->val[e] * x[A->col[e]];
        y[i] = acc;
    }
}

#define ORC_CHUNK 4096

/* <a, b>: fixed chunks, then chunk sums in index order (Section 3 eq. ip). */
static double orc_dot(int64_t n, const double* a, const double* b)
{
    int64_t nc = (n + ORC_CHUNK - 1) / ORC_CHUNK;
    double* part = (double*)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(double));
    if (!part) abort();
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        int64_t lo = c * ORC_CHUNK, hi = lo + ORC_CHUNK < n ? lo + ORC_CHUNK : n;
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) s = s + a[i] * b[i];
        part[c] = s;
    }
    double s = 0.0;
    for (int64_t c = 0; c < nc; ++c) s = s + part[c];
    free(part);
    return s;
}

/* out = M^{-1} v with M^{-1} = diag(d). */
static void orc_prec(int64_t n, const double* d, const double* v, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = d[i] * v[i];
}

/* y = y + a x  (a plain AXPY; Section 3 eq. axpy) */
static void orc_axpy(int64_t n, double a, const double* x, double* y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = y[i] + a * x[i];
}

/* y = x + a y  (the direction updates p = r~ + beta p, s = w + beta s) */
static void orc_xpay(int64_t n, const double* x, double a, double* y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = x[i] + a * y[i];
}

static int orc_finite(double v) { return isfinite(v) ? 1 : 0; }

/* ||b - A x|| / ||b|| and ||x* - x||_A, recorded in diagnostics mode only. */
static void orc_record_truth(const orc_csr* A, const double* b, const double* x, double bnorm,
                             orc_diag* dg, int64_t k, double* tmp1, double* tmp2)
{
    if (!dg) return;
    int64_t n = A->n;
    if (dg->true_res) {
        orc_spmv(A, x, tmp1);
        for (int64_t i = 0; i < n; ++i) tmp1[i] = b[i] - tmp1[i];
        dg->true_res[k] = sqrt(orc_dot(n, tmp1, tmp1)) / bnorm;
    }
    if (dg->err_a && dg->xstar) {
        for (int64_t i = 0; i < n; ++i) tmp1[i] = dg->xstar[i] - x[i];
        orc_spmv(A, tmp1, tmp2);
        double e = orc_dot(n, tmp1, tmp2);
        dg->err_a[k] = sqrt(e > 0.0 ? e : 0.0);
    }
}

/* ---------------------------------------------------------------- workspace */

typedef struct {
    double *r, *rt, *p, *s, *st, *w, *wt, *u, *ut, *t, *pold, *tmp1, *tmp2;
} orc_ws;

static void orc_ws_free(orc_ws* W)
{
    double** f[] = {&W->r, &W->rt, &W->p, &W->s, &W->st, &W->w, &W->wt,
                    &W->u, &W->ut, &W->t, &W->pold, &W->tmp1, &W->tmp2};
    for (size_t i = 0; i < sizeof(f) / sizeof(f[0]); ++i) {
        free(*f[i]);
        *f[i] = NULL;
    }
}

static int orc_ws_alloc(orc_ws* W, int64_t n, int pre)
{
    memset(W, 0, sizeof(*W));
    size_t bytes = (size_t)n * sizeof(double);
    W->r = malloc(bytes);
    W->p = malloc(bytes);
    W->s = malloc(bytes);
    W->w = malloc(bytes);
    W->u = malloc(bytes);
    W->t = malloc(bytes);
    W->pold = malloc(bytes);
    W->tmp1 = malloc(bytes);
    W->tmp2 = malloc(bytes);
    if (pre) {
        W->rt = malloc(bytes);
        W->st = malloc(bytes);
        W->wt = malloc(bytes);
        W->ut = malloc(bytes);
    } else {
        /* No preconditioner: tilde vectors alias their plain counterparts. */
        W->rt = NULL;
        W->st = NULL;
        W->wt = NULL;
        W->ut = NULL;
    }
    if (!W->r || !W->p || !W->s || !W->w || !W->u || !W->t || !W->pold || !W->tmp1 || !W->tmp2 ||
        (pre && (!W->rt || !W->st || !W->wt || !W->ut))) {
        orc_ws_free(W);
        return ORC_ENOMEM;
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------- solver */

typedef struct {
    orc_csr A;
    const double* dinv;
    const double* b;
    double* x;
    double bnorm;
    double tol;
    int32_t maxit;
    double* hist;
    orc_diag* dg;
    int pre;
    orc_ws W;
} orc_ctx;

/* Record ||r_k|| and the diagnostics of step k; return 1 if converged. */
static int orc_observe(orc_ctx* C, int64_t k, double rr, double nu, const double* r)
{
    double rnorm = sqrt(rr > 0.0 ? rr : 0.0);
    if (C->hist) C->hist[k] = rnorm / C->bnorm;
    if (C->dg) {
        if (C->dg->nu) C->dg->nu[k] = nu;
        if (C->dg->rr) C->dg->rr[k] = orc_dot(C->A.n, r, r);
        orc_record_truth(&C->A, C->b, C->x, C->bnorm, C->dg, k, C->W.tmp1, C->W.tmp2);
    }
    return orc_finite(rr) && rnorm <= C->tol * C->bnorm;
}

static void orc_record_orth(orc_ctx* C, int64_t k, const double* pold, const double* s)
{
    if (!C->dg || !C->dg->orth) return;
    int64_t n = C->A.n;
    double np = sqrt(orc_dot(n, pold, pold)), ns = sqrt(orc_dot(n, s, s));
    C->dg->orth[k] = fabs(orc_dot(n, pold, s)) / (np * ns);
}

/* Alg. 1: HS-CG.  Two reductions per iteration: nu_k, then mu_k. */
static int orc_hs(orc_ctx* C, int64_t* kout)
{
    const int64_t n = C->A.n;
    const int pre = C->pre;
    double* x = C->x;
    double* r = C->W.r;
    double* p = C->W.p;
    double* s = C->W.s;
    double* rt = pre ? C->W.rt : r;
    orc_diag* dg = C->dg;

    /* initialize (Appendix D): r0, r~0, nu0, p0, s0, alpha0 */
    orc_spmv(&C->A, x, r);
    for (int64_t i = 0; i < n; ++i) r[i] = C->b[i] - r[i];     /* r0 = b - A x0     */
    if (pre) orc_prec(n, C->dinv, r, rt);                      /* r~0 = M^-1 r0     */
    double nu = orc_dot(n, r, rt);                             /* nu0 = <r0, r~0>   */
    memcpy(p, rt, (size_t)n * sizeof(double));                 /* p0 = r~0          */
    orc_spmv(&C->A, p, s);                                     /* s0 = A p0         */
    double mu = orc_dot(n, p, s);                              /* <p0, s0>          */
    double rr = pre ? orc_dot(n, r, r) : nu;

    int64_t k = 0;
    int status;
    if (dg && dg->mu) dg->mu[0] = mu;
    /* same order as in the loop: converged, nu breakdown, maxit, mu breakdown */
    if (orc_observe(C, 0, rr, nu, r)) { status = ORC_OK; goto out; }
    if (!orc_finite(nu) || !orc_finite(rr) || !(nu > 0.0)) { status = ORC_BREAKDOWN; goto out; }
    if (k == C->maxit) { status = ORC_NOT_CONVERGED; goto out; }
    if (!orc_finite(mu) || !(mu > 0.0)) { status = ORC_BREAKDOWN; goto out; }
    double alpha = nu / mu;                                    /* alpha0 = nu0 / <p0, s0> */
    if (dg && dg->alpha) dg->alpha[0] = alpha;

    for (;;) {
        ++k;
        orc_axpy(n, alpha, p, x);                              /* x_k = x_{k-1} + alpha_{k-1} p_{k-1} */
        orc_axpy(n, -alpha, s, r);                             /* r_k = r_{k-1} - alpha_{k-1} s_{k-1} */
        if (pre) orc_prec(n, C->dinv, r, rt);                  /* r~_k = M^-1 r_k                     */
        double nu_new = orc_dot(n, rt, r);                     /* nu_k = <r~_k, r_k>                  */
        rr = pre ? orc_dot(n, r, r) : nu_new;
        if (orc_observe(C, k, rr, nu_new, r)) { status = ORC_OK; goto out; }
        if (!orc_finite(nu_new) || !orc_finite(rr) || !(nu_new > 0.0)) { status = ORC_BREAKDOWN; goto out; }
        if (k == C->maxit) { status = ORC_NOT_CONVERGED; goto out; }
        double beta = nu_new / nu;                             /* beta_k = nu_k / nu_{k-1}            */
        nu = nu_new;
        if (dg && dg->beta) dg->beta[k] = beta;
        if (dg && dg->orth) memcpy(C->W.pold, p, (size_t)n * sizeof(double));
        orc_xpay(n, rt, beta, p);                              /* p_k = r~_k + beta_k p_{k-1}         */
        orc_spmv(&C->A, p, s);                                 /* s_k = A p_k                         */
        mu = orc_dot(n, p, s);                                 /* mu_k = <p_k, s_k>                   */
        if (dg && dg->mu) dg->mu[k] = mu;
        orc_record_orth(C, k, C->W.pold, s);
        if (!orc_finite(mu) || !(mu > 0.0)) { status = ORC_BREAKDOWN; goto out; }
        alpha = nu / mu;                                       /* alpha_k = nu_k / mu_k               */
        if (dg && dg->alpha) dg->alpha[k] = alpha;
    }
out:
    *kout = k;
    return status;
}

/* Alg. 2 (PR-CG), Alg. 3 (pipe-PR-CG), their Meurant forms, GV-CG and the
 * two no-recompute ablations.  One reduction per iteration; after it the
 * loop head runs the checks and the scalar step for the next iteration. */
static int orc_one_sync(int variant, orc_ctx* C, int64_t* kout)
{
    const int64_t n = C->A.n;
    const int pre = C->pre;
    const double* dinv = C->dinv;
    double* x = C->x;
    double* r = C->W.r;
    double* p = C->W.p;
    double* s = C->W.s;
    double* w = C->W.w;
    double* u = C->W.u;
    double* t = C->W.t;
    double* rt = pre ? C->W.rt : C->W.r;
    double* st = pre ? C->W.st : C->W.s;
    double* wt = pre ? C->W.wt : C->W.w;
    double* ut = pre ? C->W.ut : C->W.u;
    orc_diag* dg = C->dg;

    const int is_pr = variant == ORC_PR || variant == ORC_M || variant == ORC_PR_NO_RECOMPUTE ||
                      variant == ORC_PR_UNSIMPLIFIED;
    const int unsimplified = variant == ORC_PR_UNSIMPLIFIED;
    const int is_pipe = variant == ORC_PIPE_PR || variant == ORC_PIPE_M || variant == ORC_PIPE_PR_NO_W_RECOMPUTE;
    const int is_gv = variant == ORC_GV;
    const int is_cg = variant == ORC_CG;
    const int meurant = variant == ORC_M || variant == ORC_PIPE_M;

    /* initialize (Appendix D) */
    orc_spmv(&C->A, x, r);
    for (int64_t i = 0; i < n; ++i) r[i] = C->b[i] - r[i];     /* r0 = b - A x0        */
    if (pre) orc_prec(n, dinv, r, rt);                         /* r~0 = M^-1 r0        */
    double nu = orc_dot(n, r, rt);                             /* nu0 = <r0, r~0>      */
    memcpy(p, rt, (size_t)n * sizeof(double));                 /* p0 = r~0             */
    orc_spmv(&C->A, p, s);                                     /* s0 = A p0            */
    double mu = orc_dot(n, p, s);                              /* <p0, s0>             */
    if (pre) orc_prec(n, dinv, s, st);                         /* s~0 = M^-1 s0        */
    double sigma = orc_dot(n, rt, s);                          /* sigma0 = <r~0, s0>   */
    double gamma = orc_dot(n, st, s);                          /* gamma0 = <s~0, s0>   */
    double delta = unsimplified ? orc_dot(n, st, r) : 0.0;     /* delta0 = <s~0, r0>   */
    double eta = 0.0;
    if (is_pipe || is_gv) {
        memcpy(w, s, (size_t)n * sizeof(double));             /* w0 = A r~0 = A p0 = s0 */
        if (pre) orc_prec(n, dinv, w, wt);                     /* w~0 = M^-1 w0        */
        orc_spmv(&C->A, st, u);                                /* u0 = A s~0           */
        if (pre) orc_prec(n, dinv, u, ut);                     /* u~0 = M^-1 u0        */
    }
    double rr = pre ? orc_dot(n, r, r) : nu;
    double nup = nu;      /* nu'_0 := nu_0 (only the no-recompute ablation reads it) */
    double alpha = 0.0, beta = 0.0;
    int64_t k = 0;
    int status;
    int last = 0;         /* set when nu' <= 0: the current iteration is the final one */

    for (;;) {
        /* the reduction of iteration k has produced nu_k, mu_k, sigma_k, gamma_k */
        if (dg && dg->mu) dg->mu[k] = mu;
        if (orc_observe(C, k, rr, nu, r)) { status = ORC_OK; break; }
        if (last || !orc_finite(nu) || !orc_finite(mu) || !orc_finite(rr) || !(nu > 0.0) || !(mu > 0.0)) {
            status = ORC_BREAKDOWN;
            break;
        }
        if (k == C->maxit) { status = ORC_NOT_CONVERGED; break; }

        /* scalar step for iteration k+1 (Section 2.2.1) */
        alpha = nu / mu;                                       /* alpha_k = nu_k / mu_k */
        if (dg && dg->alpha) dg->alpha[k] = alpha;
        if (is_pr || is_pipe) {
            if (variant == ORC_PR_NO_RECOMPUTE)
                nup = nup - 2.0 * alpha * sigma + alpha * alpha * gamma;  /* eq. nuk_norecomp   */
            else if (meurant)
                nup = -nu + alpha * alpha * gamma;                        /* M-CG form           */
            else if (unsimplified)
                nup = nu - alpha * (sigma + delta) + alpha * alpha * gamma; /* eq. nuk            */
            else
                nup = nu - 2.0 * alpha * sigma + alpha * alpha * gamma;   /* eq. nuk_simplified  */
            if (!orc_finite(nup) || !(nup > 0.0)) {
                last = 1;                                      /* take x, r of iteration k+1, then stop */
                beta = 0.0;
            } else {
                beta = nup / nu;                               /* beta_{k+1} = nu'_{k+1} / nu_k */
            }
        }
        ++k;
        if (dg && dg->nup && !is_gv && !is_cg) dg->nup[k] = nup;
        if (dg && dg->beta && !is_gv && !is_cg) dg->beta[k] = beta;
        if (dg && dg->orth) memcpy(C->W.pold, p, (size_t)n * sizeof(double));

        if (is_pr) {
            /* Alg. 2, iteration k */
            orc_axpy(n, alpha, p, x);                          /* x_k = x_{k-1} + alpha p      */
            orc_axpy(n, -alpha, s, r);                         /* r_k = r_{k-1} - alpha s      */
            if (pre) orc_axpy(n, -alpha, st, rt);              /* r~_k = r~_{k-1} - alpha s~   */
            orc_xpay(n, rt, beta, p);                          /* p_k = r~_k + beta_k p_{k-1}  */
            orc_spmv(&C->A, p, s);                             /* s_k = A p_k                  */
            if (pre) orc_prec(n, dinv, s, st);                 /* s~_k = M^-1 s_k              */
            mu = orc_dot(n, p, s);                             /* mu_k    = <p_k, s_k>         */
            sigma = orc_dot(n, rt, s);                         /* sigma_k = <r~_k, s_k>        */
            gamma = orc_dot(n, st, s);                         /* gamma_k = <s~_k, s_k>        */
            if (unsimplified) delta = orc_dot(n, st, r);       /* delta_k = <s~_k, r_k>        */
            if (variant == ORC_PR_NO_RECOMPUTE) {
                nu = nup;                                      /* nu_k is never recomputed     */
                rr = orc_dot(n, r, r);
            } else {
                nu = orc_dot(n, rt, r);                        /* nu_k    = <r~_k, r_k>        */
                rr = pre ? orc_dot(n, r, r) : nu;
            }
        } else if (is_pipe) {
            /* Alg. 3, iteration k; w and w' share one array, as do w~ and w~' */
            orc_axpy(n, alpha, p, x);                          /* x_k = x_{k-1} + alpha p      */
            orc_axpy(n, -alpha, s, r);                         /* r_k = r_{k-1} - alpha s      */
            if (pre) orc_axpy(n, -alpha, st, rt);              /* r~_k = r~_{k-1} - alpha s~   */
            orc_axpy(n, -alpha, u, w);                         /* w'_k = w_{k-1} - alpha u     */
            if (pre) orc_axpy(n, -alpha, ut, wt);              /* w~'_k = w~_{k-1} - alpha u~  */
            orc_xpay(n, rt, beta, p);                          /* p_k = r~_k + beta_k p_{k-1}  */
            orc_xpay(n, w, beta, s);                           /* s_k = w'_k + beta_k s_{k-1}  */
            if (pre) orc_xpay(n, wt, beta, st);                /* s~_k = w~'_k + beta_k s~_{k-1} */
            orc_spmv(&C->A, st, u);                            /* u_k = A s~_k                 */
            if (pre) orc_prec(n, dinv, u, ut);                 /* u~_k = M^-1 u_k              */
            if (variant != ORC_PIPE_PR_NO_W_RECOMPUTE) {
                orc_spmv(&C->A, rt, w);                        /* w_k = A r~_k  (recompute)    */
                if (pre) orc_prec(n, dinv, w, wt);             /* w~_k = M^-1 w_k              */
            }
            mu = orc_dot(n, p, s);                             /* mu_k    = <p_k, s_k>         */
            sigma = orc_dot(n, rt, s);                         /* sigma_k = <r~_k, s_k>        */
            gamma = orc_dot(n, st, s);                         /* gamma_k = <s~_k, s_k>        */
            nu = orc_dot(n, rt, r);                            /* nu_k    = <r~_k, r_k>        */
            rr = pre ? orc_dot(n, r, r) : nu;
        } else if (is_cg) {
            /* CG-CG (Appendix D), iteration k */
            orc_axpy(n, alpha, p, x);                          /* x_k = x_{k-1} + alpha p      */
            orc_axpy(n, -alpha, s, r);                         /* r_k = r_{k-1} - alpha s      */
            if (pre) orc_prec(n, dinv, r, rt);                 /* r~_k = M^-1 r_k              */
            orc_spmv(&C->A, rt, w);                            /* w_k = A r~_k                 */
            double nu_new = orc_dot(n, rt, r);                 /* nu_k  = <r~_k, r_k>          */
            eta = orc_dot(n, rt, w);                           /* eta_k = <r~_k, w_k>          */
            beta = nu_new / nu;                                /* beta_k = nu_k / nu_{k-1}     */
            if (dg && dg->beta) dg->beta[k] = beta;
            orc_xpay(n, rt, beta, p);                          /* p_k = r~_k + beta p_{k-1}    */
            orc_xpay(n, w, beta, s);                           /* s_k = w_k + beta s_{k-1}     */
            mu = eta - (beta / alpha) * nu_new;                /* mu_k = eta_k - (beta_k/alpha_{k-1}) nu_k */
            nu = nu_new;
            rr = pre ? orc_dot(n, r, r) : nu;
        } else {
            /* GV-CG (Appendix D), iteration k */
            orc_axpy(n, alpha, p, x);                          /* x_k = x_{k-1} + alpha p      */
            orc_axpy(n, -alpha, s, r);                         /* r_k = r_{k-1} - alpha s      */
            if (pre) orc_axpy(n, -alpha, st, rt);              /* r~_k = r~_{k-1} - alpha s~   */
            orc_axpy(n, -alpha, u, w);                         /* w_k = w_{k-1} - alpha u      */
            if (pre) orc_prec(n, dinv, w, wt);                 /* w~_k = M^-1 w_k              */
            double nu_new = orc_dot(n, rt, r);                 /* nu_k  = <r~_k, r_k>          */
            eta = orc_dot(n, rt, w);                           /* eta_k = <r~_k, w_k>          */
            orc_spmv(&C->A, wt, t);                            /* t_k = A w~_k                 */
            beta = nu_new / nu;                                /* beta_k = nu_k / nu_{k-1}     */
            if (dg && dg->beta) dg->beta[k] = beta;
            if (dg && dg->nup) dg->nup[k] = nu_new;
            orc_xpay(n, rt, beta, p);                          /* p_k = r~_k + beta p_{k-1}    */
            orc_xpay(n, w, beta, s);                           /* s_k = w_k + beta s_{k-1}     */
            if (pre) orc_xpay(n, wt, beta, st);                /* s~_k = w~_k + beta s~_{k-1}  */
            orc_xpay(n, t, beta, u);                           /* u_k = t_k + beta u_{k-1}     */
            mu = eta - (beta / alpha) * nu_new;                /* mu_k = eta_k - (beta_k/alpha_{k-1}) nu_k */
            nu = nu_new;
            rr = pre ? orc_dot(n, r, r) : nu;
        }
        orc_record_orth(C, k, C->W.pold, s);
    }
    *kout = k;
    return status;
}

/*
 * Solve A x = b.  x holds x_0 on entry and the final iterate on exit.
 * hist (nullable, maxit+1 entries) receives ||r_k|| / ||b|| for k = 0..iters.
 * Returns ORC_OK / ORC_NOT_CONVERGED / ORC_BREAKDOWN, or a negative error.
 */
int orc_solve(int variant, int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
              const double* dinv, const double* b, double* x, double tol, int32_t maxit,
              int32_t* iters_out, double* hist, orc_diag* dg)
{
    if (n < 1 || !row_ptr || !col || !val || !b || !x || !iters_out || !(tol >= 0.0) || maxit < 0)
        return ORC_EINVAL;
    if (variant < ORC_HS || variant > ORC_PR_UNSIMPLIFIED) return ORC_EINVAL;
    *iters_out = 0;

    double bnorm = sqrt(orc_dot(n, b, b));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        if (hist) hist[0] = 0.0;
        return ORC_OK;
    }
    orc_ctx C;
    C.A.n = n;
    C.A.row_ptr = row_ptr;
    C.A.col = col;
    C.A.val = val;
    C.dinv = dinv;
    C.b = b;
    C.x = x;
    C.bnorm = bnorm;
    C.tol = tol;
    C.maxit = maxit;
    C.hist = hist;
    C.dg = dg;
    C.pre = dinv != NULL;
    if (orc_ws_alloc(&C.W, n, C.pre) != ORC_OK) return ORC_ENOMEM;
    int64_t k = 0;
    int status = variant == ORC_HS ? orc_hs(&C, &k) : orc_one_sync(variant, &C, &k);
    *iters_out = (int32_t)k;
    orc_ws_free(&C.W);
    return status;
}

/* Exported primitives, so the tests can pin them on their own. */
void orc_spmv_export(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                     const double* x, double* y)
{
    orc_csr A = {n, row_ptr, col, val};
    orc_spmv(&A, x, y);
}

double orc_dot_export(int64_t n, const double* a, const double* b) { return orc_dot(n, a, b); }

/* d_i = 1 / a_ii; returns ORC_EINVAL if a diagonal entry is missing or not positive. */
int orc_jacobi(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val, double* d)
{
    for (int64_t i = 0; i < n; ++i) {
        double a = 0.0;
        int found = 0;
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            if (col[e] == i) { a = a + val[e]; found = 1; }
        if (!found || !(a > 0.0)) return ORC_EINVAL;
        d[i] = 1.0 / a;
    }
    return ORC_OK;
}

/* Gradient of L = w^T A^{-1} b with respect to every stored entry of A, given
 * x = A^{-1} b and lambda = A^{-1} w (A symmetric):  g_e = -lambda_row(e) * x_col(e). */
void orc_outer_csr(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* lambda,
                   const double* x, double* g)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) g[e] = -lambda[i] * x[col[e]];
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the following calls (timing only: every result is the same
 * for any count, since the inner products sum fixed chunks in index order). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
