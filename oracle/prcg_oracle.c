/*
 * CPU oracle for the conjugate-gradient variants of Chen & Carson,
 * "Predict-and-recompute conjugate gradient variants".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the solver library links, loads or
 * calls this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU path.
 *
 * What it is: a plain, slow FP64 implementation of the algorithms in the
 * paper's notation, written for checking by eye against the paper:
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
 * nu'-gap and residual-gap analysis, its statements about the two
 * ablations and its printed table for its model problem.
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
    double* gap;       /* ||b - A x_k - r_k|| / ||b||, the residual gap       */
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

/* y = x + a y  (the direction updates p = r~ + beta p, s = w + beta s) */
static void orc_xpay(int64_t n, const double* x, double a, double* y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = x[i] + a * y[i];
}

static int orc_finite(double v) { return isfinite(v) ? 1 : 0; }

/* ||b - A x|| / ||b||, the residual gap ||b - A x - r|| / ||b|| (Section
 * 3.1.1, Delta_r) and ||x* - x||_A, recorded in diagnostics mode only. */
static void orc_record_truth(const orc_csr* A, const double* b, const double* x, const double* r, double bnorm,
                             orc_diag* dg, int64_t k, double* tmp1, double* tmp2)
{
    if (!dg) return;
    int64_t n = A->n;
    if (dg->true_res || dg->gap) {
        orc_spmv(A, x, tmp1);
        for (int64_t i = 0; i < n; ++i) tmp1[i] = b[i] - tmp1[i];
        if (dg->true_res) dg->true_res[k] = sqrt(orc_dot(n, tmp1, tmp1)) / bnorm;
        if (dg->gap) {
            for (int64_t i = 0; i < n; ++i) tmp1[i] = tmp1[i] - r[i];
            dg->gap[k] = sqrt(orc_dot(n, tmp1, tmp1)) / bnorm;
        }
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
        orc_record_truth(&C->A, C->b, C->x, r, C->bnorm, C->dg, k, C->W.tmp1, C->W.tmp2);
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

/* The vectors of an iteration.  Without a preconditioner the tilde vectors
 * are the plain arrays themselves (r~ = r, s~ = s, w~ = w, u~ = u). */
typedef struct {
    int64_t n;
    int pre;
    const double* d;
    double *x, *r, *rt, *p, *s, *st, *w, *wt, *u, *ut, *t;
} orc_vecs;

static orc_vecs orc_vecs_of(orc_ctx* C)
{
    orc_vecs v;
    v.n = C->A.n;
    v.pre = C->pre;
    v.d = C->dinv;
    v.x = C->x;
    v.r = C->W.r;
    v.p = C->W.p;
    v.s = C->W.s;
    v.w = C->W.w;
    v.u = C->W.u;
    v.t = C->W.t;
    v.rt = C->pre ? C->W.rt : C->W.r;
    v.st = C->pre ? C->W.st : C->W.s;
    v.wt = C->pre ? C->W.wt : C->W.w;
    v.ut = C->pre ? C->W.ut : C->W.u;
    return v;
}

/* ---- the parts of an iteration --------------------------------------------
 * Section 2.2.1 splits an iteration of a predict-and-recompute method into a
 * scalar step (alpha, nu', beta from the previous reduction), the vector
 * recurrences, the matrix products and one global reduction of all inner
 * products.  Each variant below is written as those parts.  The recurrences
 * act row by row: row i of every vector depends only on row i of the others,
 * so taking all of a row's updates together gives the same values as taking
 * each vector update over all rows in turn. */

/* The predicted nu'_{k+1} (Section 2.1).  PR-CG: eq. nuk_simplified,
 * nu_k - 2 alpha_k sigma_k + alpha_k^2 gamma_k.  M-CG: the Meurant form
 * -nu_k + alpha_k^2 gamma_k (Appendix D).  eq. nuk keeps <s~_k, r_k> = delta_k
 * apart from sigma_k; its two middle terms are grouped as alpha (sigma +
 * delta), which with delta = sigma (M = I) rounds exactly like 2 alpha sigma.
 * The ablation of eq. nuk_norecomp starts from the previous prediction nu'_k
 * instead of the recomputed nu_k. */
enum { FORM_PR, FORM_MEURANT, FORM_NUK, FORM_NORECOMPUTE };

static double orc_predict_nu(int form, double nu, double nup_prev, double alpha, double sigma, double gamma,
                             double delta)
{
    switch (form) {
    case FORM_MEURANT: return -nu + alpha * alpha * gamma;
    case FORM_NUK: return nu - alpha * (sigma + delta) + alpha * alpha * gamma;
    case FORM_NORECOMPUTE: return nup_prev - 2.0 * alpha * sigma + alpha * alpha * gamma;
    default: return nu - 2.0 * alpha * sigma + alpha * alpha * gamma;
    }
}

/* Solution and residual recurrences of every variant:
 *   x_k = x_{k-1} + alpha_{k-1} p_{k-1},   r_k = r_{k-1} - alpha_{k-1} s_{k-1}. */
static inline void orc_xr_row(const orc_vecs* v, int64_t i, double alpha)
{
    v->x[i] = v->x[i] + alpha * v->p[i];
    v->r[i] = v->r[i] - alpha * v->s[i];
}

/* Alg. 2: x, r, the preconditioned residual by its own recurrence
 * r~_k = r~_{k-1} - alpha s~_{k-1} (not recomputed as M^{-1} r_k), and the
 * new direction p_k = r~_k + beta_k p_{k-1}. */
static void orc_pr_recurrences(const orc_vecs* v, double alpha, double beta)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < v->n; ++i) {
        orc_xr_row(v, i, alpha);
        if (v->pre) v->rt[i] = v->rt[i] - alpha * v->st[i];
        v->p[i] = v->rt[i] + beta * v->p[i];
    }
}

/* Alg. 3: besides x, r and r~, the predictions w'_k = w_{k-1} - alpha u_{k-1}
 * and w~'_k = w~_{k-1} - alpha u~_{k-1}, then the directions
 * p_k = r~_k + beta p_{k-1}, s_k = w'_k + beta s_{k-1} and
 * s~_k = w~'_k + beta s~_{k-1}.  w' and w~' overwrite w and w~: they are
 * replaced by the recomputed A r~_k and M^{-1} A r~_k after the products
 * (unless the ablation keeps them). */
static void orc_pipe_recurrences(const orc_vecs* v, double alpha, double beta)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < v->n; ++i) {
        orc_xr_row(v, i, alpha);
        if (v->pre) v->rt[i] = v->rt[i] - alpha * v->st[i];
        v->w[i] = v->w[i] - alpha * v->u[i];
        if (v->pre) v->wt[i] = v->wt[i] - alpha * v->ut[i];
        v->p[i] = v->rt[i] + beta * v->p[i];
        v->s[i] = v->w[i] + beta * v->s[i];
        if (v->pre) v->st[i] = v->wt[i] + beta * v->st[i];
    }
}

/* Several inner products of one reduction, each summed exactly as orc_dot
 * sums it (the same chunks in the same order), so forming them in one sweep
 * changes no bit.  out[q] = <a[q], b[q]> for q < m (m <= 8). */
static void orc_dots(int64_t n, int m, const double* const* a, const double* const* b, double* out)
{
    int64_t nc = (n + ORC_CHUNK - 1) / ORC_CHUNK;
    double* part = (double*)malloc((size_t)(nc > 0 ? nc : 1) * (size_t)m * sizeof(double));
    if (!part) abort();
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        int64_t lo = c * ORC_CHUNK, hi = lo + ORC_CHUNK < n ? lo + ORC_CHUNK : n;
        double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int64_t i = lo; i < hi; ++i)
            for (int q = 0; q < m; ++q) s[q] = s[q] + a[q][i] * b[q][i];
        for (int q = 0; q < m; ++q) part[(size_t)q * (size_t)nc + (size_t)c] = s[q];
    }
    for (int q = 0; q < m; ++q) {
        double s = 0.0;
        for (int64_t c = 0; c < nc; ++c) s = s + part[(size_t)q * (size_t)nc + (size_t)c];
        out[q] = s;
    }
    free(part);
}

/* The reduction of PR-CG and pipe-PR-CG (Alg. 2, Alg. 3; Table 1): mu_k =
 * <p_k, s_k>, sigma_k = <r~_k, s_k>, gamma_k = <s~_k, s_k>, nu_k = <r~_k, r_k>,
 * and where needed <r_k, r_k> (stopping test with M != I) and delta_k =
 * <s~_k, r_k> (eq. nuk).  Returns the values in that order in out[0..5]. */
static void orc_pr_reduction(const orc_vecs* v, int want_rr, int want_delta, double* out)
{
    const double* a[6] = {v->p, v->rt, v->st, v->rt, v->r, v->st};
    const double* b[6] = {v->s, v->s, v->s, v->r, v->r, v->r};
    double t[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    orc_dots(v->n, 4, a, b, t);
    if (want_rr) orc_dots(v->n, 1, a + 4, b + 4, t + 4);
    if (want_delta) orc_dots(v->n, 1, a + 5, b + 5, t + 5);
    for (int q = 0; q < 6; ++q) out[q] = t[q];
}

/* initialize (Appendix D): r_0 = b - A x_0, r~_0 = M^{-1} r_0, p_0 = r~_0,
 * s_0 = A p_0, s~_0 = M^{-1} s_0, and for the pipelined methods w_0 = A r~_0
 * (= A p_0 = s_0), w~_0 = M^{-1} w_0, u_0 = A s~_0, u~_0 = M^{-1} u_0. */
static void orc_initialize(orc_ctx* C, const orc_vecs* v, int pipelined)
{
    const int64_t n = v->n;
    orc_spmv(&C->A, v->x, v->r);
    for (int64_t i = 0; i < n; ++i) v->r[i] = C->b[i] - v->r[i];
    if (v->pre) orc_prec(n, v->d, v->r, v->rt);
    memcpy(v->p, v->rt, (size_t)n * sizeof(double));
    orc_spmv(&C->A, v->p, v->s);
    if (v->pre) orc_prec(n, v->d, v->s, v->st);
    if (pipelined) {
        memcpy(v->w, v->s, (size_t)n * sizeof(double));
        if (v->pre) orc_prec(n, v->d, v->w, v->wt);
        orc_spmv(&C->A, v->st, v->u);
        if (v->pre) orc_prec(n, v->d, v->u, v->ut);
    }
}

/* Alg. 1: HS-CG.  Two reductions per iteration: nu_k after the x and r
 * recurrences, mu_k after the product s_k = A p_k. */
static int orc_hs(orc_ctx* C, int64_t* kout)
{
    const orc_vecs V = orc_vecs_of(C);
    const orc_vecs* v = &V;
    const int64_t n = v->n;
    orc_diag* dg = C->dg;

    orc_initialize(C, v, 0);
    double nu = orc_dot(n, v->r, v->rt);
    double mu = orc_dot(n, v->p, v->s);
    double rr = v->pre ? orc_dot(n, v->r, v->r) : nu;

    int64_t k = 0;
    int status;
    if (dg && dg->mu) dg->mu[0] = mu;
    /* same order as in the loop: converged, nu breakdown, maxit, mu breakdown */
    if (orc_observe(C, 0, rr, nu, v->r)) { status = ORC_OK; goto out; }
    if (!orc_finite(nu) || !orc_finite(rr) || !(nu > 0.0)) { status = ORC_BREAKDOWN; goto out; }
    if (k == C->maxit) { status = ORC_NOT_CONVERGED; goto out; }
    if (!orc_finite(mu) || !(mu > 0.0)) { status = ORC_BREAKDOWN; goto out; }
    double alpha = nu / mu;
    if (dg && dg->alpha) dg->alpha[0] = alpha;

    for (;;) {
        ++k;
        /* x_k, r_k, then the preconditioned residual recomputed as M^{-1} r_k */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) orc_xr_row(v, i, alpha);
        if (v->pre) orc_prec(n, v->d, v->r, v->rt);
        /* first reduction: nu_k = <r~_k, r_k> (and <r_k, r_k>) */
        double nu_new = orc_dot(n, v->rt, v->r);
        rr = v->pre ? orc_dot(n, v->r, v->r) : nu_new;
        if (orc_observe(C, k, rr, nu_new, v->r)) { status = ORC_OK; goto out; }
        if (!orc_finite(nu_new) || !orc_finite(rr) || !(nu_new > 0.0)) { status = ORC_BREAKDOWN; goto out; }
        if (k == C->maxit) { status = ORC_NOT_CONVERGED; goto out; }
        /* beta_k = nu_k / nu_{k-1}; p_k = r~_k + beta_k p_{k-1}; s_k = A p_k */
        double beta = nu_new / nu;
        nu = nu_new;
        if (dg && dg->beta) dg->beta[k] = beta;
        if (dg && dg->orth) memcpy(C->W.pold, v->p, (size_t)n * sizeof(double));
        orc_xpay(n, v->rt, beta, v->p);
        orc_spmv(&C->A, v->p, v->s);
        /* second reduction: mu_k = <p_k, s_k>; alpha_k = nu_k / mu_k */
        mu = orc_dot(n, v->p, v->s);
        if (dg && dg->mu) dg->mu[k] = mu;
        orc_record_orth(C, k, C->W.pold, v->s);
        if (!orc_finite(mu) || !(mu > 0.0)) { status = ORC_BREAKDOWN; goto out; }
        alpha = nu / mu;
        if (dg && dg->alpha) dg->alpha[k] = alpha;
    }
out:
    *kout = k;
    return status;
}

/* The one-reduction variants: PR-CG (Alg. 2) with its nu' forms and the
 * ablation without the recompute of nu, pipe-PR-CG (Alg. 3), pipe-PR-M-CG and
 * the ablation without the recompute of w, GV-CG and CG-CG (Appendix D).  The
 * loop head takes the tests after the reduction of iteration k, then the
 * scalar step of iteration k+1; the body runs that iteration's recurrences,
 * products and reduction. */
static int orc_one_sync(int variant, orc_ctx* C, int64_t* kout)
{
    const orc_vecs V = orc_vecs_of(C);
    const orc_vecs* v = &V;
    const int64_t n = v->n;
    const int pre = v->pre;
    orc_diag* dg = C->dg;

    const int is_pr = variant == ORC_PR || variant == ORC_M || variant == ORC_PR_NO_RECOMPUTE ||
                      variant == ORC_PR_UNSIMPLIFIED;
    const int is_pipe = variant == ORC_PIPE_PR || variant == ORC_PIPE_M || variant == ORC_PIPE_PR_NO_W_RECOMPUTE;
    const int is_gv = variant == ORC_GV;
    const int is_cg = variant == ORC_CG;
    const int form = (variant == ORC_M || variant == ORC_PIPE_M) ? FORM_MEURANT
                     : variant == ORC_PR_UNSIMPLIFIED          ? FORM_NUK
                     : variant == ORC_PR_NO_RECOMPUTE          ? FORM_NORECOMPUTE
                                                               : FORM_PR;
    const int recompute_nu = variant != ORC_PR_NO_RECOMPUTE;
    const int recompute_w = variant != ORC_PIPE_PR_NO_W_RECOMPUTE;

    orc_initialize(C, v, is_pipe || is_gv);
    /* the reduction of initialize: mu_0, sigma_0, gamma_0, nu_0, <r_0, r_0>,
     * delta_0 (eq. nuk) */
    double red[6];
    orc_pr_reduction(v, pre, form == FORM_NUK, red);
    double mu = red[0], sigma = red[1], gamma = red[2], nu = red[3], delta = red[5];
    double rr = pre ? red[4] : nu;
    double nup = nu;      /* nu'_0 := nu_0 (only the no-recompute ablation reads it) */
    double alpha = 0.0, beta = 0.0, eta = 0.0;
    int64_t k = 0;
    int status;
    int last = 0;         /* set when nu' <= 0: the current iteration is the final one */

    for (;;) {
        /* ---- tests after the reduction of iteration k */
        if (dg && dg->mu) dg->mu[k] = mu;
        if (orc_observe(C, k, rr, nu, v->r)) { status = ORC_OK; break; }
        if (last || !orc_finite(nu) || !orc_finite(mu) || !orc_finite(rr) || !(nu > 0.0) || !(mu > 0.0)) {
            status = ORC_BREAKDOWN;
            break;
        }
        if (k == C->maxit) { status = ORC_NOT_CONVERGED; break; }

        /* ---- scalar step for iteration k+1 (Section 2.2.1): alpha_k, and for
         * the predict-and-recompute methods nu'_{k+1} and beta_{k+1} */
        alpha = nu / mu;
        if (dg && dg->alpha) dg->alpha[k] = alpha;
        if (is_pr || is_pipe) {
            nup = orc_predict_nu(form, nu, nup, alpha, sigma, gamma, delta);
            if (!orc_finite(nup) || !(nup > 0.0)) {
                last = 1;                                      /* take x, r of iteration k+1, then stop */
                beta = 0.0;
            } else {
                beta = nup / nu;
            }
        }
        ++k;
        if (dg && dg->nup && !is_gv && !is_cg) dg->nup[k] = nup;
        if (dg && dg->beta && !is_gv && !is_cg) dg->beta[k] = beta;
        if (dg && dg->orth) memcpy(C->W.pold, v->p, (size_t)n * sizeof(double));

        if (is_pr) {
            /* ---- Alg. 2: recurrences; s_k = A p_k, s~_k = M^{-1} s_k; one
             * reduction.  The ablation takes nu_k := nu'_k and uses the inner
             * product of r with itself only for the stopping test. */
            orc_pr_recurrences(v, alpha, beta);
            orc_spmv(&C->A, v->p, v->s);
            if (pre) orc_prec(n, v->d, v->s, v->st);
            orc_pr_reduction(v, pre || !recompute_nu, form == FORM_NUK, red);
            mu = red[0], sigma = red[1], gamma = red[2], delta = red[5];
            nu = recompute_nu ? red[3] : nup;
            rr = (pre || !recompute_nu) ? red[4] : nu;
        } else if (is_pipe) {
            /* ---- Alg. 3: recurrences; u_k = A s~_k and the recompute
             * w_k = A r~_k (both read A: Section 2.2.1 takes them as one
             * product with a block vector), their preconditioned forms; one
             * reduction over the vectors of the recurrences */
            orc_pipe_recurrences(v, alpha, beta);
            orc_spmv(&C->A, v->st, v->u);
            if (pre) orc_prec(n, v->d, v->u, v->ut);
            if (recompute_w) {
                orc_spmv(&C->A, v->rt, v->w);
                if (pre) orc_prec(n, v->d, v->w, v->wt);
            }
            orc_pr_reduction(v, pre, 0, red);
            mu = red[0], sigma = red[1], gamma = red[2], nu = red[3];
            rr = pre ? red[4] : nu;
        } else {
            /* ---- CG-CG and GV-CG (Appendix D): x, r, r~ first; the reduction
             * of nu_k = <r~_k, r_k> and eta_k = <r~_k, w_k>; then
             * beta_k = nu_k / nu_{k-1}, the direction recurrences and
             * mu_k = eta_k - (beta_k / alpha_{k-1}) nu_k.
             *   CG-CG: r~_k = M^{-1} r_k and w_k = A r~_k are recomputed.
             *   GV-CG: r~_k and w_k by recurrence, w~_k = M^{-1} w_k, and the
             *          product t_k = A w~_k feeds u_k = t_k + beta_k u_{k-1}. */
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) {
                orc_xr_row(v, i, alpha);
                if (is_gv) {
                    if (pre) v->rt[i] = v->rt[i] - alpha * v->st[i];
                    v->w[i] = v->w[i] - alpha * v->u[i];
                }
            }
            if (pre) orc_prec(n, v->d, is_gv ? v->w : v->r, is_gv ? v->wt : v->rt);
            if (is_cg) orc_spmv(&C->A, v->rt, v->w);
            const double* a2[2] = {v->rt, v->rt};
            const double* b2[2] = {v->r, v->w};
            double ne[2];
            orc_dots(n, 2, a2, b2, ne);
            const double nu_new = ne[0];
            eta = ne[1];
            if (is_gv) orc_spmv(&C->A, v->wt, v->t);
            beta = nu_new / nu;
            if (dg && dg->beta) dg->beta[k] = beta;
            if (dg && dg->nup && is_gv) dg->nup[k] = nu_new;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) {
                v->p[i] = v->rt[i] + beta * v->p[i];
                v->s[i] = v->w[i] + beta * v->s[i];
                if (is_gv) {
                    if (pre) v->st[i] = v->wt[i] + beta * v->st[i];
                    v->u[i] = v->t[i] + beta * v->u[i];
                }
            }
            mu = eta - (beta / alpha) * nu_new;
            nu = nu_new;
            rr = pre ? orc_dot(n, v->r, v->r) : nu;
        }
        orc_record_orth(C, k, C->W.pold, v->s);
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
