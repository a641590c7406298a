// Iteration kernels of HS-CG (Alg. 1), PR-CG (Alg. 2), pipe-PR-CG (Alg. 3)
// and their Meurant forms (Appendix D), plus the initialisation of
// Appendix D and the exit kernels.
//
// Structure on the GPU.  A global synchronisation of the paper (C_gr, a
// reduction over all rows) becomes a kernel boundary: stage 1 of every
// reduction writes one partial per workgroup, and the kernel that needs the
// totals sums the partials in a fixed order (stage 2), so results are
// bitwise repeatable and no host synchronisation happens per iteration.
// The sparse product needs its input vector complete at neighbouring rows,
// which is a second kernel boundary (the paper's C_mv).
//
//   PR-CG:   [update + stage 2] [SpMV + 5 inner products]
//            stage 2 and the scalar step (alpha_k, nu'_{k+1}, beta_{k+1})
//            run redundantly in every workgroup of the update kernel.
//   pipe-PR: [update + 5 inner products] [SpMV pair (u, w) || stage 2]
//            every vector update and inner product of Alg. 3 depends only
//            on data of the row, so they share one pass; workgroup 0 of the
//            SpMV kernel runs stage 2 while the other workgroups compute
//            u = A s~ and w = A r~ (one pass over A): the overlap of the
//            reduction with the products of Section 2.2.1.  This placement
//            costs nothing and is the default for pipe-PR.
//   HS-CG:   [stage 2 of mu + x, r updates + nu] [stage 2 of nu + p update]
//            [SpMV + mu]: two reductions per iteration, as Alg. 1 needs.
//
// Where stage 2 runs is a choice (Split): redundantly in every workgroup of
// the consuming kernel (above), in a one-workgroup kernel of its own
// (stage2), or in the last workgroup of the producing kernel to finish its
// partials (lastwg; take_last_ticket).  The sums are the same in all three:
// the partials are added in the same fixed order.
//
// Jacobi (M^{-1} = diag(d)): the vectors the algorithms define explicitly
// as M^{-1} v (HS r~, PR s~, pipe u~ and w~) are recomputed as d*v where
// needed instead of being stored; this gives identical bits.  Vectors
// defined by recurrence (PR/pipe r~, pipe s~) are stored.  Without a
// preconditioner every tilde vector is its plain counterpart.
#include <hip/hip_ext.h>

#include "prcg_device.h"
#include "prcg_textbook.h"

namespace prcg {

namespace {

// Launch with optional dispatch timestamps (start/stop events recorded by
// the dispatch itself, so they measure the kernel and nothing else).
template <class K, class... Args>
void launch(K kernel, dim3 grid, dim3 block, hipStream_t st, const LaunchEvents* ev, Args... args)
{
    if (ev && ev->start)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, ev->start, ev->stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

__device__ __forceinline__ bool writer_thread() { return blockIdx.x == 0 && threadIdx.x == 0; }

// ------------------------------------------------------------------ init

// x = x0, r0 = b - A x0, p0 = r~0 = M^{-1} r0 (r~0 stored when it evolves by
// recurrence); partial of <b, b>.
template <int LANES, bool PRE>
__global__ __launch_bounds__(kBlock) void k_init_r(SellView S, CsrView C, Split sp, const double* __restrict__ b,
                                                   const double* __restrict__ x0, Vecs v, int store_rt,
                                                   double* __restrict__ PB)
{
    __shared__ double lds[kWaves * 1];
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    double acc[1] = {0.0};
    for (int64_t g = g0; g < g1; ++g) {
        rows_of_group<LANES, 1>(S, C, g, x0, nullptr, [&](int64_t i, double ax, double) {
            const double bi = b[i];
            const double ri = bi - ax;
            v.x[i] = x0[i];
            v.r[i] = ri;
            const double rti = PRE ? v.d[i] * ri : ri;
            if (PRE && store_rt) v.rt[i] = rti;
            v.p[i] = rti;
            acc[0] = fma(bi, bi, acc[0]);
        });
    }
    write_partials<1>(acc, PB, sp.Gs, blockIdx.x, lds);
}

// s0 = A p0 (s~0 = M^{-1} s0 stored when it evolves by recurrence);
// partials of mu0, sigma0, gamma0 (to PS) and nu0, <r0, r0> (to PN), and,
// when PD is given (PR-CG with eq. nuk), of delta0 = <s~0, r0> (to PD).
template <int LANES, bool PRE>
__global__ __launch_bounds__(kBlock) void k_init_s(SellView S, CsrView C, Split sp, Vecs v, int store_st,
                                                   double* __restrict__ PS, double* __restrict__ PN,
                                                   double* __restrict__ PD)
{
    __shared__ double lds[kWaves * 5];
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double dacc[1] = {0.0};
    for (int64_t g = g0; g < g1; ++g) {
        rows_of_group<LANES, 1>(S, C, g, v.p, nullptr, [&](int64_t i, double si, double) {
            v.s[i] = si;
            const double ri = v.r[i];
            const double di = PRE ? v.d[i] : 1.0;
            const double sti = PRE ? di * si : si;
            const double rti = PRE ? di * ri : ri;
            if (PRE && store_st) v.st[i] = sti;
            acc[0] = fma(v.p[i], si, acc[0]);  // mu0    = <p0, s0>
            acc[1] = fma(rti, si, acc[1]);     // sigma0 = <r~0, s0>
            acc[2] = fma(sti, si, acc[2]);     // gamma0 = <s~0, s0>
            acc[3] = fma(rti, ri, acc[3]);     // nu0    = <r~0, r0>
            acc[4] = fma(ri, ri, acc[4]);      // <r0, r0>
            dacc[0] = fma(sti, ri, dacc[0]);   // delta0 = <s~0, r0>
        });
    }
    write_partials_at<5, 3>(acc, PS, PN, sp.Gs, blockIdx.x, lds);
    if (PD) write_partials<1>(dacc, PD, sp.Gs, blockIdx.x, lds);
}

// pipe-PR-CG and GV-CG: w0 = A r~0 = A p0 = s0 (copied) and u0 = A s~0; the
// block vectors (s~0, r~0) and (u0, w0) are filled as well.  gv = 1 (GV-CG)
// also keeps t := u0 and w~0 = M^{-1} w0 = s~0, so that its first direction
// update (beta = 0) reproduces p0, s0, s~0 and u0; gv = 2 (pipe-PR-CG
// without the recompute of w) keeps w~0 only.
template <int LANES, bool PRE>
__global__ __launch_bounds__(kBlock) void k_init_u(SellView S, CsrView C, Split sp, Vecs v, int gv)
{
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    const double* st = PRE ? v.st : v.s;
    const double* rt = PRE ? v.rt : v.r;
    for (int64_t g = g0; g < g1; ++g) {
        rows_of_group<LANES, 1>(S, C, g, st, nullptr, [&](int64_t i, double ui, double) {
            const double si = v.s[i];
            v.u[i] = ui;
            v.w[i] = si;
            v.uw[i] = make_double2(ui, si);
            v.zr[i] = make_double2(st[i], rt[i]);
            if (gv & 1) v.t[i] = ui;
            if (gv && PRE) v.wt[i] = st[i];  // w~0 = M^{-1} w0 = s~0
        });
    }
}

// One workgroup: ||b||, the b = 0 case, and the first scalar step where the
// variant's first iteration kernel does not perform it.
// step0: 1 when this kernel performs the scalar step of k = 0 (pipe-PR
// two-pass and HS; PR when the iteration's own step runs at the end of the
// product kernel); otherwise the first iteration kernel does.  HS with
// step0 = 2 also forms alpha_0 from mu_0.
template <bool PRE>
__global__ __launch_bounds__(kStage2Block) void k_init_finish(int variant, int step0, Split sp, const double* __restrict__ PB,
                                                        const double* __restrict__ PS, const double* __restrict__ PN,
                                                        const double* __restrict__ PD, State* __restrict__ out,
                                                        double* __restrict__ hist, double tol, int maxit)
{
    __shared__ double lds[kStage2Waves * 5];
    double bb[1];
    reduce_partials<1, true>(PB, sp.G, sp.Gs, bb, lds);
    double t[5];
    reduce_partials_at<5, 3, true>(PS, PN, sp.G, sp.Gs, t, lds);
    double dd[1] = {t[1]};  // delta0 = sigma0 without a preconditioner
    if (PD) reduce_partials<1, true>(PD, sp.G, sp.Gs, dd, lds);
    State st = {};
    st.bnorm = sqrt(bb[0]);
    st.tol = tol;
    st.maxit = maxit;
    st.k = -1;
    st.status = kNotConverged;
    const bool w = threadIdx.x == 0;
    if (bb[0] == 0.0) {
        st.k = 0;
        st.done = 1;
        st.status = kOK;
        st.zero_x = 1;
        st.rr = 0.0;
        if (w) hist[0] = 0.0;
    } else if (variant == kHS) {
        step_hs_nu(st, t[3], PRE ? t[4] : t[3], hist, w);
        if (step0 == 2 && !st.done) step_hs_mu(st, t[0]);
    } else if (variant == kGV || variant == kCG) {
        step_gv_first(st, t, PRE, hist, w);
    } else if (step0) {
        step_one_reduction(st, t, PRE, nu_form(variant), hist, w, dd[0]);
    }
    // otherwise the first iteration kernel performs the step for k = 0
    if (w) store_state(out, st);
}

// ------------------------------------------------------------------ PR-CG

__device__ __forceinline__ void row_range(const Split& sp, int64_t g0, int64_t g1, int64_t& i0, int64_t& i1)
{
    i0 = g0 * kGroupRows + threadIdx.x;
    i1 = g1 * kGroupRows < sp.n ? g1 * kGroupRows : sp.n;
}

// Stage 2 of a PR-CG reduction in kWaves workgroups: the sums of the lane
// groups of mu, sigma, gamma (PS) and nu, <r, r> (PN), to W; the update
// kernel adds them and performs the scalar step in every workgroup.  Same
// bits as a one-workgroup stage 2, at a quarter of its loads per workgroup.
__global__ __launch_bounds__(kWaveBlock) void k_stage2_waves(Split sp, const double* __restrict__ PS,
                                                             const double* __restrict__ PN, double* __restrict__ W)
{
    wave_partial_sums<5, 3>(PS, PN, sp.G, sp.Gs, W);
}

// Stage 2 of iteration k + scalar step, then the vector updates of
// iteration k+1 (Alg. 2): x += alpha p; r -= alpha s; r~ -= alpha s~;
// p = r~ + beta p.
// RED: how the state of iteration k is reached.  0: already advanced (a
// one-workgroup kernel, or the last workgroup of the product kernel) and
// `in` is the current state; 1: every workgroup sums all partials of PS
// (mu, sigma, gamma) and PN (nu, <r, r>); 2: every workgroup adds the lane
// group sums W of k_stage2_waves.  With RED != 0 every workgroup performs
// the scalar step (`in` -> `out`, written by workgroup 0).
// NUDOT (Jacobi, RED != 1): this kernel also writes the partials of
// nu_{k+1} = <r~, r> and <r, r> of the rows it has just updated to PN, so
// the product kernel need not read r again.
// PD (nullable, RED = 1): the partials of delta_k = <s~_k, r_k> (eq. nuk
// with a preconditioner), reduced together with the others.
template <bool PRE, int RED, bool NUDOT>
__global__ __launch_bounds__(kBlock) void k_pr_update(Split sp, const State* __restrict__ in,
                                                      State* __restrict__ out, double* __restrict__ hist,
                                                      const double* __restrict__ PS, double* __restrict__ PN,
                                                      const double* __restrict__ PD, const double* __restrict__ W,
                                                      int form, Vecs v)
{
    static_assert(!(RED == 1 && NUDOT), "PN is read by every workgroup when RED = 1");
    static_assert(PRE || !NUDOT, "without a preconditioner the product kernel reads r anyway");
    __shared__ double lds[kWaves * 5];
    int64_t g0, g1, i0, i1;
    // rows in the opposite order to the product kernel's (see
    // reverse_block): slot is the workgroup that owns them in that order
    const int slot = reverse_block(blockIdx.x, sp.G);
    chunk_of(slot, sp.G, sp.ngroups, g0, g1);
    row_range(sp, g0, g1, i0, i1);
    double* __restrict__ x = v.x;
    double* __restrict__ r = v.r;
    double* __restrict__ rt = v.rt;
    double* __restrict__ p = v.p;
    const double* __restrict__ s = v.s;
    const double* __restrict__ d = v.d;
    // two rows per step (i and i + kBlock), every load issued before the
    // first store
    struct Rows {
        double s[2], p[2], x[2], r[2], rt[2], d[2];
    };
    auto load = [&](int64_t i, Rows& q) {
        const int64_t j = i + kBlock;
        const int64_t jj = j < i1 ? j : i;
        q.s[0] = s[i], q.s[1] = s[jj];
        q.p[0] = p[i], q.p[1] = p[jj];
        q.x[0] = x[i], q.x[1] = x[jj];
        q.r[0] = r[i], q.r[1] = r[jj];
        if (PRE) {
            q.rt[0] = rt[i], q.rt[1] = rt[jj];
            q.d[0] = d[i], q.d[1] = d[jj];
        } else {
            q.rt[0] = q.rt[1] = q.d[0] = q.d[1] = 0.0;
        }
    };
    // the first step's rows are loaded before the state is examined (row 0
    // when this thread has none; every index stays below i1 <= n), so that
    // their latency overlaps the stage-2 sums and the scalar step
    Rows q;
    load(i0 < i1 ? i0 : 0, q);
    State st = load_state(in);
    if (RED != 0) {
        if (st.done) {
            if (writer_thread()) store_state(out, st);
            return;
        }
        double t[5];
        double dd[1];
        if (RED == 1) {
            reduce_partials_at<5, 3>(PS, PN, sp.G, sp.Gs, t, lds);
            dd[0] = t[1];
            if (PD) reduce_partials<1>(PD, sp.G, sp.Gs, dd, lds);
        } else {
            sum_wave_sums<5>(W, t);
            dd[0] = t[1];
        }
        step_one_reduction(st, t, PRE, form, hist, writer_thread(), dd[0]);
        if (writer_thread()) store_state(out, st);
    }
    if (st.done) return;
    const double alpha = st.alpha, beta = st.beta;
    double acc[2] = {0.0, 0.0};
    for (int64_t i = i0; i < i1; i += 2 * kBlock) {
        if (i != i0) load(i, q);
        const int64_t j = i + kBlock;
        const bool two = j < i1;
        double rn[2], rtn[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            rn[u] = fma(-alpha, q.s[u], q.r[u]);
            rtn[u] = PRE ? fma(-alpha, q.d[u] * q.s[u], q.rt[u]) : rn[u];
        }
        x[i] = fma(alpha, q.p[0], q.x[0]);
        r[i] = rn[0];
        if (PRE) rt[i] = rtn[0];
        p[i] = fma(beta, q.p[0], rtn[0]);
        if (NUDOT) {
            acc[0] = fma(rtn[0], rn[0], acc[0]);
            acc[1] = fma(rn[0], rn[0], acc[1]);
        }
        if (two) {
            x[j] = fma(alpha, q.p[1], q.x[1]);
            r[j] = rn[1];
            if (PRE) rt[j] = rtn[1];
            p[j] = fma(beta, q.p[1], rtn[1]);
            if (NUDOT) {
                acc[0] = fma(rtn[1], rn[1], acc[0]);
                acc[1] = fma(rn[1], rn[1], acc[1]);
            }
        }
    }
    if (NUDOT) write_partials<2>(acc, PN, sp.Gs, slot, lds);
}

// One workgroup: stage 2 of iteration k and the scalar step of a
// one-reduction variant (PR, M, pipe-PR, pipe-M), when neither the consuming
// kernel nor the producing kernel reduces the partials itself.
template <bool PRE>
__global__ __launch_bounds__(kStage2Block) void k_finish_one(Split sp, const State* __restrict__ in,
                                                      State* __restrict__ out, double* __restrict__ hist,
                                                      const double* __restrict__ PS, const double* __restrict__ PN,
                                                      const double* __restrict__ PD, int form)
{
    __shared__ double lds[kStage2Waves * 5];
    // the partials are read whether or not the solve has ended (the loads
    // stay in bounds), so their latency overlaps that of the state
    State st = load_state(in);
    double t[5];
    reduce_partials_at<5, 3, true>(PS, PN, sp.G, sp.Gs, t, lds);
    double dd[1] = {t[1]};  // delta = sigma without a preconditioner
    if (PD) reduce_partials<1, true>(PD, sp.G, sp.Gs, dd, lds);
    if (!st.done) step_one_reduction(st, t, PRE, form, hist, threadIdx.x == 0, dd[0]);
    if (threadIdx.x == 0) store_state(out, st);
}

// One workgroup: stage 2 of HS-CG's mu_k (alpha_k) or nu_k (tests, beta_k).
__global__ __launch_bounds__(kStage2Block) void k_hs_finish_mu(Split sp, const State* __restrict__ in,
                                                         State* __restrict__ out, const double* __restrict__ PS)
{
    __shared__ double lds[kStage2Waves * 1];
    State st = load_state(in);
    double t[1];
    reduce_partials<1, true>(PS, sp.G, sp.Gs, t, lds);  // read whether or not the solve has ended
    if (!st.done) step_hs_mu(st, t[0]);
    if (threadIdx.x == 0) store_state(out, st);
}

template <bool PRE>
__global__ __launch_bounds__(kStage2Block) void k_hs_finish_nu(Split sp, const State* __restrict__ in,
                                                         State* __restrict__ out, double* __restrict__ hist,
                                                         const double* __restrict__ PU)
{
    __shared__ double lds[kStage2Waves * 2];
    State st = load_state(in);
    double t[2];
    reduce_partials<2, true>(PU, sp.G, sp.Gs, t, lds);  // read whether or not the solve has ended
    if (!st.done) step_hs_nu(st, t[0], PRE ? t[1] : t[0], hist, threadIdx.x == 0);
    if (threadIdx.x == 0) store_state(out, st);
}

// s_k = A p_k, s~_k = M^{-1} s_k, and the inner products of Alg. 2
// mu = <p, s>, sigma = <r~, s>, gamma = <s~, s> (to PS) and, with NUDOT,
// nu = <r~, r> (+ <r, r>) (to PN; otherwise the update kernel wrote them).
// DELTA (eq. nuk with a preconditioner): also delta = <s~, r> (to PD).
// LAST: the last workgroup also runs stage 2 and the scalar step, advancing
// the state from `in` to `out`.
// Occupancy of the product kernels: at least 7 wavefronts per SIMD (at most
// 72 registers; measured on MI355X, PR-CG's product is 1.5 us faster at
// 128^3 than with the 78 registers the compiler would take), pipe-PR-CG's
// paired product at least 6.
constexpr int kSpmvWaves = 7;
constexpr int kPipeSpmvWaves = 6;

template <int LANES, bool PRE, bool LAST, bool NUDOT, bool DELTA = false>
__global__ __launch_bounds__(kBlock, kSpmvWaves) void k_pr_spmv(SellView S, CsrView C, Split sp, const State* __restrict__ in,
                                                    State* __restrict__ out, double* __restrict__ hist,
                                                    double* __restrict__ PS, double* __restrict__ PN,
                                                    double* __restrict__ PD, int form, int* ticket, Vecs v)
{
    static_assert(PRE || NUDOT, "without a preconditioner nu = <r, r> is formed here");
    static_assert(PRE || !DELTA, "without a preconditioner delta = sigma");
    constexpr int NV = NUDOT ? 5 : 3;
    __shared__ double lds[kWaves * 5];
    if (in->done) {
        if (LAST && writer_thread()) store_state(out, load_state(in));
        return;
    }
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    double dacc[1] = {0.0};
    for (int64_t g = g0; g < g1; ++g) {
        rows_of_group<LANES, 1>(S, C, g, v.p, nullptr, [&](int64_t i, double si, double) {
            v.s[i] = si;
            const double rti = PRE ? v.rt[i] : v.r[i];
            const double sti = PRE ? v.d[i] * si : si;
            acc[0] = fma(v.p[i], si, acc[0]);
            acc[1] = fma(rti, si, acc[1]);
            acc[2] = fma(sti, si, acc[2]);
            if constexpr (NUDOT || DELTA) {
                const double ri = PRE ? v.r[i] : rti;
                if constexpr (NUDOT) {
                    acc[3] = fma(rti, ri, acc[3]);
                    if (PRE) acc[4] = fma(ri, ri, acc[4]);
                }
                if constexpr (DELTA) dacc[0] = fma(sti, ri, dacc[0]);
            }
        });
    }
    write_partials_at<NV, 3>(acc, PS, PN, sp.Gs, blockIdx.x, lds);
    if (DELTA) write_partials<1>(dacc, PD, sp.Gs, blockIdx.x, lds);
    if (LAST && take_last_ticket(ticket, sp.G)) {
        State st = load_state(in);
        double t[5];
        reduce_partials_at<5, 3>(PS, PN, sp.G, sp.Gs, t, lds);
        double dd[1] = {t[1]};
        if (DELTA) reduce_partials<1>(PD, sp.G, sp.Gs, dd, lds);
        step_one_reduction(st, t, PRE, form, hist, threadIdx.x == 0, dd[0]);
        if (threadIdx.x == 0) store_state(out, st);
    }
}

// ------------------------------------------------------------------ pipe-PR-CG

// All vector updates of iteration k (Alg. 3) in one pass, then the four
// (five) inner products of the same iteration from the updated rows:
//   x += alpha p; r -= alpha s; r~ -= alpha s~; w' = w - alpha u;
//   w~' = w~ - alpha u~; p = r~ + beta p; s = w' + beta s; s~ = w~' + beta s~.
// w' and w~' live only in registers (Section 2.2.1: w and w' need not be
// stored separately; w is recomputed by the next kernel).
// LAST: the last workgroup also runs stage 2 and the scalar step of
// iteration k (`in` -> `out`); the product kernel then only multiplies.
// NOW: the ablation of Section 2 that never recomputes w: w'_k (and, with
// a preconditioner, w~'_k = w~_{k-1} - alpha u~) is stored and is the next
// iteration's w (w~), instead of A r~ (M^{-1} A r~).
template <bool PRE, bool LAST, bool NOW = false>
__global__ __launch_bounds__(kBlock) void k_pipe_update(Split sp, const State* __restrict__ in,
                                                        State* __restrict__ out, double* __restrict__ hist,
                                                        double* __restrict__ PS, int form, int* ticket, Vecs v)
{
    __shared__ double lds[kWaves * 5];
    const State st = load_state(in);
    if (st.done) {
        if (LAST && writer_thread()) store_state(out, st);
        return;
    }
    const double alpha = st.alpha, beta = st.beta;
    int64_t g0, g1, i0, i1;
    // rows in the opposite order to the product kernel's (reverse_block)
    const int slot = reverse_block(blockIdx.x, sp.G);
    chunk_of(slot, sp.G, sp.ngroups, g0, g1);
    row_range(sp, g0, g1, i0, i1);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double* __restrict__ x = v.x;
    double* __restrict__ r = v.r;
    double* __restrict__ p = v.p;
    double* __restrict__ s = v.s;
    double2* __restrict__ zr = v.zr;
    double2* __restrict__ uw = v.uw;
    double* __restrict__ wt = v.wt;
    const double* __restrict__ d = v.d;
    for (int64_t i = i0; i < i1; i += kBlock) {
        const double pi = p[i], xi = x[i];
        const double2 zri = zr[i], uwi = uw[i];
        const double ui = uwi.x, wi = uwi.y;
        const double si = PRE ? s[i] : zri.x;
        const double ri = PRE ? r[i] : zri.y;
        const double rn = fma(-alpha, si, ri);                 // r_k
        const double wn = fma(-alpha, ui, wi);                 // w'_k
        const double snew = fma(beta, si, wn);                 // s_k = w'_k + beta s_{k-1}
        double rti = rn, sti = snew;
        if (PRE) {
            const double di = d[i];
            rti = fma(-alpha, zri.x, zri.y);                   // r~_k = r~_{k-1} - alpha s~_{k-1}
            // w~'_k = w~_{k-1} - alpha u~ (w~ = M^{-1} w when w is recomputed)
            const double wtn = fma(-alpha, di * ui, NOW ? wt[i] : di * wi);
            sti = fma(beta, zri.x, wtn);                       // s~_k = w~'_k + beta s~_{k-1}
            if (NOW) wt[i] = wtn;
        }
        if (NOW) uw[i].y = wn;
        const double pnew = fma(beta, pi, rti);                // p_k
        x[i] = fma(alpha, pi, xi);
        p[i] = pnew;
        if (PRE) {
            r[i] = rn;
            s[i] = snew;
        }
        zr[i] = make_double2(sti, rti);
        acc[0] = fma(pnew, snew, acc[0]);                      // mu_k    = <p_k, s_k>
        acc[1] = fma(rti, snew, acc[1]);                       // sigma_k = <r~_k, s_k>
        acc[2] = fma(sti, snew, acc[2]);                       // gamma_k = <s~_k, s_k>
        acc[3] = fma(rti, rn, acc[3]);                         // nu_k    = <r~_k, r_k>
        if (PRE) acc[4] = fma(rn, rn, acc[4]);
    }
    write_partials<5>(acc, PS, sp.Gs, slot, lds);
    if (LAST && take_last_ticket(ticket, sp.G)) {
        State nx = st;
        double t[5];
        reduce_partials<5>(PS, sp.G, sp.Gs, t, lds);
        step_one_reduction(nx, t, PRE, form, hist, threadIdx.x == 0);
        if (threadIdx.x == 0) store_state(out, nx);
    }
}

// u_k = A s~_k and w_k = A r~_k (the recompute) in one pass over A with the
// block vector (s~, r~).  REDUCE: workgroup 0 first reduces the inner
// products of iteration k and performs the scalar step, then takes its
// share of the product, while the other workgroups multiply (Section 2.2.1:
// the reduction proceeds during the products).  Reducing first keeps the
// reduction off the kernel's tail: done after the product, it lengthened
// the kernel by 9-12 us on MI355X.
// REDUCE = false: the update kernel or a one-workgroup kernel advances the
// state instead.  NOW (no recompute of w): only u = A s~ is stored; w keeps
// the update kernel's w'.
template <int LANES, bool PRE, bool REDUCE, bool NOW = false>
__global__ __launch_bounds__(kBlock, kPipeSpmvWaves) void k_pipe_spmv(SellView S, CsrView C, Split sp, const State* __restrict__ in,
                                                      State* __restrict__ out, double* __restrict__ hist,
                                                      const double* __restrict__ PS, int form, Vecs v)
{
    __shared__ double lds[kWaves * 5];
    const State st = load_state(in);
    if (REDUCE && blockIdx.x == 0) {
        State nx = st;
        if (!st.done) {
            double t[5];
            reduce_partials<5>(PS, sp.G, sp.Gs, t, lds);
            step_one_reduction(nx, t, PRE, form, hist, threadIdx.x == 0);
        }
        if (threadIdx.x == 0) store_state(out, nx);
    }
    if (st.done) return;
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    double2* __restrict__ uw = v.uw;
    for (int64_t g = g0; g < g1; ++g) {
        rows_of_group_pair<LANES>(S, C, g, v.zr, [&](int64_t i, double ui, double wi) {
            if (NOW)
                uw[i].x = ui;
            else
                uw[i] = make_double2(ui, wi);
        });
    }
}

// ------------------------------------------------------------------ GV-CG

// GV-CG (Appendix D) in two kernels per iteration.  This one first finishes
// iteration k-1's direction updates with beta_{k-1} (they wait for the
// reduction of iteration k-1) and then takes iteration k's updates with
// alpha_{k-1}; every operation is row-local:
//   p = r~ + beta p; s = w + beta s; s~ = w~ + beta s~; u = t + beta u;
//   x += alpha p; r -= alpha s; r~ -= alpha s~; w -= alpha u; w~ = M^{-1} w;
// then the partials of nu_k = <r~, r>, eta_k = <r~, w> (+ <r, r>).
template <bool PRE>
__global__ __launch_bounds__(kBlock) void k_gv_update(Split sp, const State* __restrict__ cur,
                                                      double* __restrict__ PS, Vecs v)
{
    __shared__ double lds[kWaves * 3];
    const State st = load_state(cur);
    if (st.done) return;
    const double alpha = st.alpha, beta = st.beta;
    int64_t g0, g1, i0, i1;
    // rows in the opposite order to the product kernel's (reverse_block)
    const int slot = reverse_block(blockIdx.x, sp.G);
    chunk_of(slot, sp.G, sp.ngroups, g0, g1);
    row_range(sp, g0, g1, i0, i1);
    double* __restrict__ x = v.x;
    double* __restrict__ r = v.r;
    double* __restrict__ rt = v.rt;
    double* __restrict__ p = v.p;
    double* __restrict__ s = v.s;
    double* __restrict__ stl = v.st;
    double* __restrict__ w = v.w;
    double* __restrict__ u = v.u;
    double* __restrict__ wt = v.wt;
    const double* __restrict__ t = v.t;
    const double* __restrict__ d = v.d;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t i = i0; i < i1; i += kBlock) {
        const double pi = p[i], si = s[i], ui = u[i], ti = t[i], wi = w[i], xi = x[i], ri = r[i];
        double rti = ri, sti = si, di = 1.0;
        if (PRE) {
            rti = rt[i];
            sti = stl[i];
            di = d[i];
        }
        const double pn = fma(beta, pi, rti);                     // p_{k-1}
        const double sn = fma(beta, si, wi);                      // s_{k-1}
        const double stn = PRE ? fma(beta, sti, di * wi) : sn;    // s~_{k-1} = w~_{k-1} + beta s~_{k-2}
        const double un = fma(beta, ui, ti);                      // u_{k-1}
        const double rn = fma(-alpha, sn, ri);                    // r_k
        const double rtn = PRE ? fma(-alpha, stn, rti) : rn;      // r~_k
        const double wn = fma(-alpha, un, wi);                    // w_k
        x[i] = fma(alpha, pn, xi);                                // x_k
        r[i] = rn;
        p[i] = pn;
        s[i] = sn;
        u[i] = un;
        w[i] = wn;
        if (PRE) {
            rt[i] = rtn;
            stl[i] = stn;
            wt[i] = di * wn;                                      // w~_k = M^{-1} w_k
        }
        acc[0] = fma(rtn, rn, acc[0]);                            // nu_k  = <r~_k, r_k>
        acc[1] = fma(rtn, wn, acc[1]);                            // eta_k = <r~_k, w_k>
        if (PRE) acc[2] = fma(rn, rn, acc[2]);
    }
    write_partials<3>(acc, PS, sp.Gs, slot, lds);
}

// t_k = A w~_k.  Workgroup 0 first reduces nu_k, eta_k (+ <r_k, r_k>) and
// performs the scalar step (beta_k, mu_k, tests, alpha_k), then takes its
// share of the product: the reduction overlaps the product, as GV-CG is
// designed for.
template <int LANES, bool PRE>
__global__ __launch_bounds__(kBlock, kSpmvWaves) void k_gv_spmv(SellView S, CsrView C, Split sp, const State* __restrict__ in,
                                                    State* __restrict__ out, double* __restrict__ hist,
                                                    const double* __restrict__ PS, Vecs v)
{
    __shared__ double lds[kWaves * 3];
    const State st = load_state(in);
    if (blockIdx.x == 0) {
        State nx = st;
        if (!st.done) {
            double t[3];
            reduce_partials<3>(PS, sp.G, sp.Gs, t, lds);
            step_gv(nx, t, PRE, hist, threadIdx.x == 0);
        }
        if (threadIdx.x == 0) store_state(out, nx);
    }
    if (st.done) return;
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    double* __restrict__ t = v.t;
    for (int64_t g = g0; g < g1; ++g)
        rows_of_group<LANES, 1>(S, C, g, PRE ? v.wt : v.w, nullptr, [&](int64_t i, double ti, double) { t[i] = ti; });
}

// ------------------------------------------------------------------ CG-CG

// w0 = s0 for CG-CG (w0 = A r~0 = A p0, p0 = r~0), so that its first
// direction update (beta = 0) reproduces p0 and s0.
__global__ __launch_bounds__(kBlock) void k_init_w(Split sp, Vecs v)
{
    int64_t g0, g1, i0, i1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    row_range(sp, g0, g1, i0, i1);
    for (int64_t i = i0; i < i1; i += kBlock) v.w[i] = v.s[i];
}

// CG-CG (Appendix D) in three kernels per iteration.  This one finishes
// iteration k-1's direction updates with beta_{k-1} and takes iteration k's
// updates with alpha_{k-1}, all row-local:
//   p = r~ + beta p; s = w + beta s; x += alpha p; r -= alpha s;
//   r~ = M^{-1} r (stored for the product),
// and writes the partials of nu_k = <r~_k, r_k> (+ <r_k, r_k>) to PN.
// r~_{k-1} is recomputed as d * r_{k-1} (it is defined as M^{-1} r).
template <bool PRE>
__global__ __launch_bounds__(kBlock) void k_cg_update(Split sp, const State* __restrict__ cur,
                                                      double* __restrict__ PN, Vecs v)
{
    __shared__ double lds[kWaves * 2];
    const State st = load_state(cur);
    if (st.done) return;
    const double alpha = st.alpha, beta = st.beta;
    int64_t g0, g1, i0, i1;
    // rows in the opposite order to the product kernel's (reverse_block)
    const int slot = reverse_block(blockIdx.x, sp.G);
    chunk_of(slot, sp.G, sp.ngroups, g0, g1);
    row_range(sp, g0, g1, i0, i1);
    double* __restrict__ x = v.x;
    double* __restrict__ r = v.r;
    double* __restrict__ rt = v.rt;
    double* __restrict__ p = v.p;
    double* __restrict__ s = v.s;
    const double* __restrict__ w = v.w;
    const double* __restrict__ d = v.d;
    double acc[2] = {0.0, 0.0};
    for (int64_t i = i0; i < i1; i += kBlock) {
        const double pi = p[i], si = s[i], wi = w[i], xi = x[i], ri = r[i];
        const double di = PRE ? d[i] : 1.0;
        const double rti = PRE ? di * ri : ri;                  // r~_{k-1}
        const double pn = fma(beta, pi, rti);                   // p_{k-1}
        const double sn = fma(beta, si, wi);                    // s_{k-1}
        const double rn = fma(-alpha, sn, ri);                  // r_k
        const double rtn = PRE ? di * rn : rn;                  // r~_k = M^{-1} r_k
        x[i] = fma(alpha, pn, xi);                              // x_k
        r[i] = rn;
        p[i] = pn;
        s[i] = sn;
        if (PRE) rt[i] = rtn;
        acc[0] = fma(rtn, rn, acc[0]);                          // nu_k
        if (PRE) acc[1] = fma(rn, rn, acc[1]);
    }
    write_partials<2>(acc, PN, sp.Gs, slot, lds);
}

// w_k = A r~_k and the partials of eta_k = <r~_k, w_k>.
template <int LANES, bool PRE>
__global__ __launch_bounds__(kBlock, kSpmvWaves) void k_cg_spmv(SellView S, CsrView C, Split sp, const State* __restrict__ cur,
                                                    double* __restrict__ PS, Vecs v)
{
    __shared__ double lds[kWaves * 1];
    if (cur->done) return;
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    const double* __restrict__ rt = PRE ? v.rt : v.r;
    double* __restrict__ w = v.w;
    double acc[1] = {0.0};
    for (int64_t g = g0; g < g1; ++g) {
        rows_of_group<LANES, 1>(S, C, g, rt, nullptr, [&](int64_t i, double wi, double) {
            w[i] = wi;
            acc[0] = fma(rt[i], wi, acc[0]);
        });
    }
    write_partials<1>(acc, PS, sp.Gs, blockIdx.x, lds);
}

// One workgroup: stage 2 of eta_k (PS) and nu_k, <r_k, r_k> (PN), then
// beta_k, mu_k = eta_k - (beta_k / alpha_{k-1}) nu_k, the tests and alpha_k
// (the scalar step GV-CG shares).
template <bool PRE>
__global__ __launch_bounds__(kStage2Block) void k_cg_finish(Split sp, const State* __restrict__ in,
                                                      State* __restrict__ out, double* __restrict__ hist,
                                                      const double* __restrict__ PS, const double* __restrict__ PN)
{
    __shared__ double lds[kStage2Waves * 3];
    State st = load_state(in);
    double t[3];
    reduce_partials_at<3, 1, true>(PS, PN, sp.G, sp.Gs, t, lds);  // eta, nu, rr; read whether or not the solve has ended
    if (!st.done) {
        const double q[3] = {t[1], t[0], t[2]};  // nu, eta, rr
        step_gv(st, q, PRE, hist, threadIdx.x == 0);
    }
    if (threadIdx.x == 0) store_state(out, st);
}

// ------------------------------------------------------------------ HS-CG

// Stage 2 of mu_{k-1} (alpha_{k-1}), then x += alpha p, r -= alpha s and the
// partials of nu_k = <r~_k, r_k> (+ <r_k, r_k>), r~_k = M^{-1} r_k.
// REDUCE = false: a one-workgroup kernel or the product kernel has already
// done the step and `in` is the current state.
// LAST: the last workgroup reduces nu_k and runs its step (`in` -> `out`).
template <bool PRE, bool REDUCE, bool LAST>
__global__ __launch_bounds__(kBlock) void k_hs_xr(Split sp, const State* __restrict__ in, State* __restrict__ out,
                                                  double* __restrict__ hist, const double* __restrict__ PS,
                                                  double* __restrict__ PU, int* ticket, Vecs v)
{
    static_assert(!(REDUCE && LAST), "one state transition per kernel");
    __shared__ double lds[kWaves * 2];
    State st = load_state(in);
    if (REDUCE) {
        if (st.done) {
            if (writer_thread()) store_state(out, st);
            return;
        }
        double t[1];
        reduce_partials<1>(PS, sp.G, sp.Gs, t, lds);
        step_hs_mu(st, t[0]);
        if (writer_thread()) store_state(out, st);
    }
    if (st.done) {
        if (LAST && writer_thread()) store_state(out, st);
        return;
    }
    const double alpha = st.alpha;
    int64_t g0, g1, i0, i1;
    // rows in the opposite order to the product kernel's (reverse_block)
    const int slot = reverse_block(blockIdx.x, sp.G);
    chunk_of(slot, sp.G, sp.ngroups, g0, g1);
    row_range(sp, g0, g1, i0, i1);
    double acc[2] = {0.0, 0.0};
    double* __restrict__ x = v.x;
    double* __restrict__ r = v.r;
    const double* __restrict__ p = v.p;
    const double* __restrict__ s = v.s;
    const double* __restrict__ d = v.d;
    for (int64_t i = i0; i < i1; i += kBlock) {
        const double pi = p[i], si = s[i], xi = x[i], ri = r[i];
        const double di = PRE ? d[i] : 1.0;
        const double rn = fma(-alpha, si, ri);
        x[i] = fma(alpha, pi, xi);
        r[i] = rn;
        const double rti = PRE ? di * rn : rn;
        acc[0] = fma(rti, rn, acc[0]);
        if (PRE) acc[1] = fma(rn, rn, acc[1]);
    }
    write_partials<2>(acc, PU, sp.Gs, slot, lds);
    if (LAST && take_last_ticket(ticket, sp.G)) {
        double t[2];
        reduce_partials<2>(PU, sp.G, sp.Gs, t, lds);
        step_hs_nu(st, t[0], PRE ? t[1] : t[0], hist, threadIdx.x == 0);
        if (threadIdx.x == 0) store_state(out, st);
    }
}

// Stage 2 of nu_k (convergence test, beta_k), then p_k = r~_k + beta_k p_{k-1}.
template <bool PRE, bool REDUCE>
__global__ __launch_bounds__(kBlock) void k_hs_p(Split sp, const State* __restrict__ in, State* __restrict__ out,
                                                 double* __restrict__ hist, const double* __restrict__ PU, Vecs v)
{
    __shared__ double lds[kWaves * 2];
    State st = load_state(in);
    if (REDUCE) {
        if (st.done) {
            if (writer_thread()) store_state(out, st);
            return;
        }
        double t[2];
        reduce_partials<2>(PU, sp.G, sp.Gs, t, lds);
        step_hs_nu(st, t[0], PRE ? t[1] : t[0], hist, writer_thread());
        if (writer_thread()) store_state(out, st);
    }
    if (st.done) return;
    const double beta = st.beta;
    int64_t g0, g1, i0, i1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    row_range(sp, g0, g1, i0, i1);
    const double* __restrict__ r = v.r;
    const double* __restrict__ d = v.d;
    double* __restrict__ p = v.p;
    for (int64_t i = i0; i < i1; i += 2 * kBlock) {
        const int64_t j = i + kBlock;
        const bool two = j < i1;
        const int64_t jj = two ? j : i;
        const double r0 = r[i], r1 = r[jj], p0 = p[i], p1 = p[jj];
        const double rt0 = PRE ? d[i] * r0 : r0;
        const double rt1 = PRE ? d[jj] * r1 : r1;
        p[i] = fma(beta, p0, rt0);
        if (two) p[j] = fma(beta, p1, rt1);
    }
}

// s_k = A p_k and the partials of mu_k = <p_k, s_k>.  LAST: the last
// workgroup also reduces mu_k and forms alpha_k (`in` -> `out`).
template <int LANES, bool LAST>
__global__ __launch_bounds__(kBlock, kSpmvWaves) void k_hs_spmv(SellView S, CsrView C, Split sp, const State* __restrict__ in,
                                                    State* __restrict__ out, double* __restrict__ PS, int* ticket,
                                                    Vecs v)
{
    __shared__ double lds[kWaves * 1];
    if (in->done) {
        if (LAST && writer_thread()) store_state(out, load_state(in));
        return;
    }
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    double acc[1] = {0.0};
    for (int64_t g = g0; g < g1; ++g) {
        rows_of_group<LANES, 1>(S, C, g, v.p, nullptr, [&](int64_t i, double si, double) {
            v.s[i] = si;
            acc[0] = fma(v.p[i], si, acc[0]);
        });
    }
    write_partials<1>(acc, PS, sp.Gs, blockIdx.x, lds);
    if (LAST && take_last_ticket(ticket, sp.G)) {
        State st = load_state(in);
        double t[1];
        reduce_partials<1>(PS, sp.G, sp.Gs, t, lds);
        step_hs_mu(st, t[0]);
        if (threadIdx.x == 0) store_state(out, st);
    }
}

// ------------------------------------------------------------------ exit

// x_out = x (or 0 when b = 0) and the partials of ||b - A x_out||^2.
template <int LANES>
__global__ __launch_bounds__(kBlock) void k_final_res(SellView S, CsrView C, Split sp, const State* __restrict__ cur,
                                                      const double* __restrict__ b, const double* __restrict__ x,
                                                      double* __restrict__ xout, double* __restrict__ PB)
{
    __shared__ double lds[kWaves * 1];
    const int zero = cur->zero_x;
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    double acc[1] = {0.0};
    for (int64_t g = g0; g < g1; ++g) {
        rows_of_group<LANES, 1>(S, C, g, x, nullptr, [&](int64_t i, double ax, double) {
            const double bi = b[i];
            const double ti = zero ? bi : bi - ax;
            xout[i] = zero ? 0.0 : x[i];
            acc[0] = fma(ti, ti, acc[0]);
        });
    }
    write_partials<1>(acc, PB, sp.Gs, blockIdx.x, lds);
}

__global__ __launch_bounds__(kStage2Block) void k_final_reduce(Split sp, const double* __restrict__ PB, State* __restrict__ st)
{
    __shared__ double lds[kStage2Waves * 1];
    double t[1];
    reduce_partials<1, true>(PB, sp.G, sp.Gs, t, lds);
    if (threadIdx.x == 0) {
        const double bn = st->bnorm;
        st->relres_true = bn > 0.0 ? sqrt(t[0]) / bn : 0.0;
    }
}

// y = A x
template <int LANES>
__global__ __launch_bounds__(kBlock) void k_spmv(SellView S, CsrView C, Split sp, const double* __restrict__ x,
                                                 double* __restrict__ y)
{
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    for (int64_t g = g0; g < g1; ++g)
        rows_of_group<LANES, 1>(S, C, g, x, nullptr, [&](int64_t i, double yi, double) { y[i] = yi; });
}

// ------------------------------------------------------------------ host dispatch

template <class F>
hipError_t with_lanes(int lanes, F&& f)
{
    switch (lanes) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 16: return f(std::integral_constant<int, 16>{});
    case 32: return f(std::integral_constant<int, 32>{});
    case 64: return f(std::integral_constant<int, 64>{});
    default: return hipErrorInvalidValue;
    }
}

template <class F>
hipError_t with_pre(int pre, F&& f)
{
    return pre ? f(std::true_type{}) : f(std::false_type{});
}

SellView sell_or_empty(const SellView* s)
{
    return s ? *s : SellView{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0};
}
CsrView csr_or_empty(const CsrView* c) { return c ? *c : CsrView{nullptr, nullptr, nullptr, 0}; }

// With a preconditioner and stage 2 outside the update kernel, PR's update
// kernel forms nu and <r, r> (in PN); otherwise the product kernel forms all
// five inner products, and PN is the tail of PS.
bool nu_in_update(int variant, int pre, const Split& sp)
{
    return pre && is_pr_family(variant) && !uses_fused(variant, sp) && (stage2_of(sp, kPR) || sp.lastwg);
}

// The partials of delta = <s~, r> (PR-CG with eq. nuk and a preconditioner;
// without one delta = sigma and no partials are formed).
double* pd_of(int variant, int pre, const Bufs& B) { return variant == kPRUnsimplified && pre ? B.PD : nullptr; }

double* pn_of(int variant, int pre, const Split& sp, const Bufs& B)
{
    return nu_in_update(variant, pre, sp) ? B.PN : B.PS + 3 * (int64_t)sp.Gs;
}

}  // namespace

hipError_t launch_init(int variant, int pre, const SellView* sell, const CsrView* csr, const Split& sp,
                       const Vecs& v, const Bufs& B, const double* b, const double* x0, double tol, int32_t maxit,
                       hipStream_t st)
{
    const SellView S = sell_or_empty(sell);
    const CsrView C = csr_or_empty(csr);
    const bool pipe = is_pipe(variant);
    const int store_rt = variant != kHS;  // r~ evolves by recurrence in PR and pipe-PR
    const int gv = variant == kGV ? 1 : (variant == kPipeNoWRecompute ? 2 : 0);
    const int store_st = pipe || gv;      // s~ evolves by recurrence in pipe-PR and GV
    hipError_t e = with_lanes(sp.lanes, [&](auto L) {
        return with_pre(pre, [&](auto P) {
            hipLaunchKernelGGL((k_init_r<decltype(L)::value, decltype(P)::value>), dim3(sp.G), dim3(kBlock), 0, st,
                               S, C, sp, b, x0, v, store_rt, B.PB);
            hipLaunchKernelGGL((k_init_s<decltype(L)::value, decltype(P)::value>), dim3(sp.G), dim3(kBlock), 0, st,
                               S, C, sp, v, store_st, B.PS, pn_of(variant, pre, sp, B), pd_of(variant, pre, B));
            if (pipe || gv)
                hipLaunchKernelGGL((k_init_u<decltype(L)::value, decltype(P)::value>), dim3(sp.G), dim3(kBlock), 0,
                                   st, S, C, sp, v, gv);
            if (variant == kCG) hipLaunchKernelGGL(k_init_w, dim3(sp.G), dim3(kBlock), 0, st, sp, v);
            return hipGetLastError();
        });
    });
    if (e != hipSuccess) return e;
    return with_pre(pre, [&](auto P) {
        const bool pipe2 = is_pipe(variant) && !uses_fused(variant, sp);
        const int step0 = variant == kHS ? (sp.lastwg ? 2 : 1) : (pipe2 || sp.lastwg ? 1 : 0);
        hipLaunchKernelGGL((k_init_finish<decltype(P)::value>), dim3(1), dim3(kStage2Block), 0, st, variant, step0, sp,
                           B.PB, B.PS, pn_of(variant, pre, sp, B), (const double*)pd_of(variant, pre, B), B.S[0],
                           B.hist, tol, (int)maxit);
        return hipGetLastError();
    });
}

int iter_kernel_count(int variant, const Split& sp)
{
    if (variant == kGV) return 2;  // one structure for GV-CG
    if (variant == kCG) return 3;  // and one for CG-CG
    if (sp.textbook && variant == kHS) return textbook_kernel_count(sp.textbook_pre);
    if (uses_fused(variant, sp)) return variant == kHS ? 2 : 1;
    if (variant == kHS) return stage2_of(sp, kHS) ? 5 : 3;
    if (variant != kHS && stage2_of(sp, variant)) return 3;
    return 2;
}

const char* iter_kernel_name(int variant, const Split& sp, int j)
{
    if (variant == kGV) return j == 0 ? "k_gv_update" : "k_gv_spmv";
    if (variant == kCG) return j == 0 ? "k_cg_update" : (j == 1 ? "k_cg_spmv" : "k_cg_finish");
    if (sp.textbook && variant == kHS) return textbook_kernel_name(sp.textbook_pre, j);
    if (uses_fused(variant, sp)) {
        if (variant == kHS) return j == 0 ? "k_hs_xr" : "k_hs_fused";
        return (variant == kPipePR || variant == kPipeM) ? "k_pipe_fused" : "k_pr_fused";
    }
    if (variant == kHS && stage2_of(sp, kHS)) {
        static const char* n5[] = {"k_hs_finish_mu", "k_hs_xr", "k_hs_finish_nu", "k_hs_p", "k_hs_spmv"};
        return n5[j];
    }
    switch (variant) {
    case kHS: return j == 0 ? "k_hs_xr" : (j == 1 ? "k_hs_p" : "k_hs_spmv");
    case kPR:
    case kM:
    case kPRNoRecompute:
    case kPRUnsimplified:
        if (stage2_of(sp, kPR))
            return j == 0 ? (variant == kPRUnsimplified && sp.textbook_pre ? "k_finish_one" : "k_stage2_waves")
                          : (j == 1 ? "k_pr_update" : "k_pr_spmv");
        return j == 0 ? "k_pr_update" : "k_pr_spmv";
    default:
        if (stage2_of(sp, variant)) return j == 0 ? "k_pipe_update" : (j == 1 ? "k_pipe_spmv" : "k_finish_one");
        return j == 0 ? "k_pipe_update" : "k_pipe_spmv";
    }
}

hipError_t launch_iter_kernel(int variant, int pre, int j, int& cur, const SellView* sell, const CsrView* csr,
                              const Split& sp, const Vecs& v, const Bufs& B, hipStream_t st, const LaunchEvents* ev,
                              int)
{
    const SellView S = sell_or_empty(sell);
    const CsrView C = csr_or_empty(csr);
    const dim3 grid(sp.G), block(kBlock);
    const int nxt = 1 - cur;
    const int form = nu_form(variant);
    hipError_t e = with_lanes(sp.lanes, [&](auto L) {
        return with_pre(pre, [&](auto P) {
            constexpr int LL = decltype(L)::value;
            constexpr bool PP = decltype(P)::value;
            int* tk = B.ticket;
            const bool s2 = stage2_of(sp, variant);
            switch (variant) {
            case kCG:
                if (j == 0) {
                    launch(k_cg_update<PP>, grid, block, st, ev, sp, (const State*)B.S[cur], B.PN, v);
                } else if (j == 1) {
                    launch(k_cg_spmv<LL, PP>, grid, block, st, ev, S, C, sp, (const State*)B.S[cur], B.PS, v);
                } else {
                    launch(k_cg_finish<PP>, dim3(1), dim3(kStage2Block), st, ev, sp, (const State*)B.S[cur], B.S[nxt], B.hist,
                           (const double*)B.PS, (const double*)B.PN);
                    cur = nxt;
                }
                break;
            case kGV:
                if (j == 0) {
                    launch(k_gv_update<PP>, grid, block, st, ev, sp, (const State*)B.S[cur], B.PS, v);
                } else {
                    launch(k_gv_spmv<LL, PP>, grid, block, st, ev, S, C, sp, (const State*)B.S[cur], B.S[nxt],
                           B.hist, (const double*)B.PS, v);
                    cur = nxt;
                }
                break;
            case kPR:
            case kM:
            case kPRNoRecompute:
            case kPRUnsimplified: {
                double* PN = pn_of(variant, pre, sp, B);
                double* PD = pd_of(variant, pre, B);
                const bool nu_up = nu_in_update(variant, pre, sp);
                // stage 2 split over kWaves workgroups, the scalar step in every
                // workgroup of the update kernel (PD, eq. nuk with a
                // preconditioner, keeps the one-workgroup stage 2)
                const bool waves = s2 && !PD;
                // the update kernel (RED 0: no reduction, 2: the wave sums),
                // forming nu when nu_up
                auto update = [&](auto red) {
                    constexpr int RD = decltype(red)::value;
                    if constexpr (PP) {
                        if (nu_up) {
                            launch(k_pr_update<PP, RD, true>, grid, block, st, ev, sp, (const State*)B.S[cur],
                                   B.S[nxt], B.hist, (const double*)B.PS, PN, (const double*)PD,
                                   (const double*)B.PW, form, v);
                            return;
                        }
                    }
                    launch(k_pr_update<PP, RD, false>, grid, block, st, ev, sp, (const State*)B.S[cur], B.S[nxt],
                           B.hist, (const double*)B.PS, PN, (const double*)PD, (const double*)B.PW, form, v);
                };
                // the product kernel (LAST: with the reduction in its last
                // workgroup; with delta's partials when PD)
                auto product = [&](auto last) {
                    constexpr bool LA = decltype(last)::value;
                    if constexpr (PP) {
                        if (nu_up && PD) {
                            launch(k_pr_spmv<LL, PP, LA, false, true>, grid, block, st, ev, S, C, sp,
                                   (const State*)B.S[cur], B.S[nxt], B.hist, B.PS, PN, PD, form, tk, v);
                            return;
                        }
                        if (PD) {
                            launch(k_pr_spmv<LL, PP, LA, true, true>, grid, block, st, ev, S, C, sp,
                                   (const State*)B.S[cur], B.S[nxt], B.hist, B.PS, PN, PD, form, tk, v);
                            return;
                        }
                        if (nu_up) {
                            launch(k_pr_spmv<LL, PP, LA, false>, grid, block, st, ev, S, C, sp,
                                   (const State*)B.S[cur], B.S[nxt], B.hist, B.PS, PN, PD, form, tk, v);
                            return;
                        }
                    }
                    launch(k_pr_spmv<LL, PP, LA, true>, grid, block, st, ev, S, C, sp, (const State*)B.S[cur],
                           B.S[nxt], B.hist, B.PS, PN, PD, form, tk, v);
                };
                if (sp.lastwg) {
                    if (j == 0) {
                        update(std::integral_constant<int, 0>{});
                    } else {
                        product(std::true_type{});
                        cur = nxt;
                    }
                } else if (waves && j == 0) {
                    launch(k_stage2_waves, dim3(kWaves), dim3(kWaveBlock), st, ev, sp, (const double*)B.PS,
                           (const double*)PN, B.PW);
                } else if (waves && j == 1) {
                    update(std::integral_constant<int, 2>{});
                    cur = nxt;
                } else if (s2 && j == 0) {
                    launch(k_finish_one<PP>, dim3(1), dim3(kStage2Block), st, ev, sp, (const State*)B.S[cur], B.S[nxt], B.hist,
                           (const double*)B.PS, (const double*)PN, (const double*)PD, form);
                    cur = nxt;
                } else if (s2 && j == 1) {
                    update(std::integral_constant<int, 0>{});
                } else if (j == 0) {
                    launch(k_pr_update<PP, 1, false>, grid, block, st, ev, sp, (const State*)B.S[cur], B.S[nxt],
                           B.hist, (const double*)B.PS, PN, (const double*)PD, (const double*)B.PW, form, v);
                    cur = nxt;
                } else {
                    product(std::false_type{});
                }
                break;
            }
            case kPipePR:
            case kPipeM:
            case kPipeNoWRecompute: {
                auto pipe = [&](auto now) {
                    constexpr bool NW = decltype(now)::value;
                    if (sp.lastwg) {
                        if (j == 0) {
                            launch(k_pipe_update<PP, true, NW>, grid, block, st, ev, sp, (const State*)B.S[cur],
                                   B.S[nxt], B.hist, B.PS, form, tk, v);
                            cur = nxt;
                        } else {
                            launch(k_pipe_spmv<LL, PP, false, NW>, grid, block, st, ev, S, C, sp,
                                   (const State*)B.S[cur], B.S[nxt], B.hist, (const double*)B.PS, form, v);
                        }
                    } else if (j == 0) {
                        launch(k_pipe_update<PP, false, NW>, grid, block, st, ev, sp, (const State*)B.S[cur],
                               B.S[nxt], B.hist, B.PS, form, tk, v);
                    } else if (s2 && j == 1) {
                        launch(k_pipe_spmv<LL, PP, false, NW>, grid, block, st, ev, S, C, sp, (const State*)B.S[cur],
                               B.S[nxt], B.hist, (const double*)B.PS, form, v);
                    } else if (s2) {
                        launch(k_finish_one<PP>, dim3(1), dim3(kStage2Block), st, ev, sp, (const State*)B.S[cur], B.S[nxt],
                               B.hist, (const double*)B.PS, (const double*)(B.PS + 3 * (int64_t)sp.Gs),
                               (const double*)nullptr, form);
                        cur = nxt;
                    } else {
                        launch(k_pipe_spmv<LL, PP, true, NW>, grid, block, st, ev, S, C, sp, (const State*)B.S[cur],
                               B.S[nxt], B.hist, (const double*)B.PS, form, v);
                        cur = nxt;
                    }
                };
                if (variant == kPipeNoWRecompute)
                    pipe(std::true_type{});
                else
                    pipe(std::false_type{});
                break;
            }
            default:  // HS
                if (sp.lastwg) {
                    if (j == 0) {
                        launch(k_hs_xr<PP, false, true>, grid, block, st, ev, sp, (const State*)B.S[cur], B.S[nxt],
                               B.hist, (const double*)B.PS, B.PU, tk, v);
                        cur = nxt;
                    } else if (j == 1) {
                        launch(k_hs_p<PP, false>, grid, block, st, ev, sp, (const State*)B.S[cur], B.S[nxt],
                               B.hist, (const double*)B.PU, v);
                    } else {
                        launch(k_hs_spmv<LL, true>, grid, block, st, ev, S, C, sp, (const State*)B.S[cur], B.S[nxt],
                               B.PS, tk, v);
                        cur = nxt;
                    }
                } else if (s2 && j == 0) {
                    launch(k_hs_finish_mu, dim3(1), dim3(kStage2Block), st, ev, sp, (const State*)B.S[cur], B.S[nxt],
                           (const double*)B.PS);
                    cur = nxt;
                } else if (s2 && j == 1) {
                    launch(k_hs_xr<PP, false, false>, grid, block, st, ev, sp, (const State*)B.S[cur], B.S[nxt],
                           B.hist, (const double*)B.PS, B.PU, tk, v);
                } else if (s2 && j == 2) {
                    launch(k_hs_finish_nu<PP>, dim3(1), dim3(kStage2Block), st, ev, sp, (const State*)B.S[cur], B.S[nxt],
                           B.hist, (const double*)B.PU);
                    cur = nxt;
                } else if (s2 && j == 3) {
                    launch(k_hs_p<PP, false>, grid, block, st, ev, sp, (const State*)B.S[cur], B.S[nxt], B.hist,
                           (const double*)B.PU, v);
                } else if (j == 0) {
                    launch(k_hs_xr<PP, true, false>, grid, block, st, ev, sp, (const State*)B.S[cur], B.S[nxt],
                           B.hist, (const double*)B.PS, B.PU, tk, v);
                    cur = nxt;
                } else if (j == 1) {
                    launch(k_hs_p<PP, true>, grid, block, st, ev, sp, (const State*)B.S[cur], B.S[nxt], B.hist,
                           (const double*)B.PU, v);
                    cur = nxt;
                } else {
                    launch(k_hs_spmv<LL, false>, grid, block, st, ev, S, C, sp, (const State*)B.S[cur], B.S[nxt],
                           B.PS, tk, v);
                }
                break;
            }
            return hipGetLastError();
        });
    });
    return e;
}

hipError_t launch_final(const SellView* sell, const CsrView* csr, const Split& sp, const Vecs& v, const Bufs& B,
                        int cur, const double* b, double* xout, hipStream_t st)
{
    const SellView S = sell_or_empty(sell);
    const CsrView C = csr_or_empty(csr);
    hipError_t e = with_lanes(sp.lanes, [&](auto L) {
        hipLaunchKernelGGL((k_final_res<decltype(L)::value>), dim3(sp.G), dim3(kBlock), 0, st, S, C, sp, B.S[cur], b,
                           v.x, xout, B.PB);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_final_reduce, dim3(1), dim3(kStage2Block), 0, st, sp, B.PB, B.S[cur]);
    return hipGetLastError();
}

hipError_t launch_spmv(const SellView* sell, const CsrView* csr, const Split& sp, const double* x, double* y,
                       hipStream_t st)
{
    const SellView S = sell_or_empty(sell);
    const CsrView C = csr_or_empty(csr);
    return with_lanes(sp.lanes, [&](auto L) {
        hipLaunchKernelGGL((k_spmv<decltype(L)::value>), dim3(sp.G), dim3(kBlock), 0, st, S, C, sp, x, y);
        return hipGetLastError();
    });
}

}  // namespace prcg
