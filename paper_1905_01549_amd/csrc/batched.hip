// Batched solve: many independent systems (one block-diagonal matrix) in one
// persistent launch.  Not part of the paper; each system runs exactly the
// single-system algorithm (Alg. 1, Alg. 2 or Alg. 3 with the initialisation of
// Appendix D, same tests and scalar step), but inside one workgroup:
// every reduction is a workgroup reduction (wavefront butterfly + LDS, fixed
// order), and the kernel boundaries of the single-system path become
// workgroup barriers.  No grid-wide synchronisation is needed because
// systems are independent.
//
// Work distribution: workgroups take systems from a queue (an atomic
// counter over a largest-first order) until it is empty; every workgroup
// leaves once the counter passes the number of systems.
#include "batched.h"
#include "prcg_device.h"

namespace prcg {

namespace {

// Products of the rows of Q offset-aligned slices of the same width W at
// once (their value, offset and gather loads all in flight together), each
// row's entries summed in stored order from 0.0 as in sell_row.  Zero slots
// read a column clamped into the system's own rows [lo, hi].
template <int W, int NX, int Q>
__device__ __forceinline__ void aligned_group(const SellView& A, const int64_t (&base)[Q], const int32_t* const (&off)[Q],
                                              int lane, const int64_t (&row)[Q], int lo, int hi,
                                              const double* __restrict__ x0, const double* __restrict__ x1,
                                              double (&y0)[Q], double (&y1)[Q])
{
    int c[Q][W];
    double a[Q][W], g0[Q][W], g1[Q][W];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int u = 0; u < W; ++u) c[q][u] = min(max((int)row[q] + off[q][u], lo), hi);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int u = 0; u < W; ++u) {
            a[q][u] = A.val[base[q] + (int64_t)u * 64 + lane];
            g0[q][u] = x0[c[q][u]];
            if (NX == 2) g1[q][u] = x1[c[q][u]];
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int u = 0; u < W; ++u) {
            a0 = fma(a[q][u], g0[q][u], a0);
            if (NX == 2) a1 = fma(a[q][u], g1[q][u], a1);
        }
        y0[q] = a0;
        y1[q] = a1;
    }
}

// Calls f(row, y0, y1) for every row of the system's slices [sl0, sl1)
// (the system's rows are [lo, hi]; zero slots never read past them):
// wavefront w takes slices sl0 + w, sl0 + w + NW, ... in that order, Q at a
// time; Q offset-aligned slices of equal width (every slice of a stencil
// matrix) are multiplied with all their loads in flight together, so a
// workgroup that runs a system on its own waits about one memory round trip
// per Q slices instead of three per slice.  Q (1 or 2) is a choice of the
// batched autotuner (measured on the batched workload: pairs 21% faster
// than single slices; Q = 4 no faster than pairs, with more registers).
// The rows reach f in the same order for every Q.
template <int NT, int NX, int Q, class F>
__device__ __forceinline__ void sys_spmv(const BatchView& B, int64_t sl0, int64_t sl1, int lo, int hi,
                                         const double* __restrict__ x0, const double* __restrict__ x1, F&& f)
{
    constexpr int NW = NT / 64;
    constexpr int kWMax = NX == 2 ? 5 : 8;  // widest slice grouped (registers)
    const SellView& A = B.A;
    const int w = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // the metadata of the next group of slices is loaded while the current
    // group is multiplied
    struct Meta {
        int64_t base[Q], row0[Q];
        int meta[Q], nrows[Q], shape[Q];
    };
    auto load_meta = [&](int64_t s0, Meta& m) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int64_t sq = s0 + (int64_t)q * NW;
            m.base[q] = A.slice_ptr[sq];
            m.shape[q] = A.slice_shape[sq];
            m.meta[q] = A.slice_meta[sq];
            m.row0[q] = B.slice_row0[sq];
            m.nrows[q] = B.slice_nrows[sq];
        }
    };
    int64_t sl = sl0 + w;
    Meta cur;
    if (sl + (int64_t)(Q - 1) * NW < sl1) load_meta(sl, cur);
    for (; sl + (int64_t)(Q - 1) * NW < sl1; sl += (int64_t)Q * NW) {
        Meta nxt = cur;
        const int64_t sn = sl + (int64_t)Q * NW;
        if (sn + (int64_t)(Q - 1) * NW < sl1) load_meta(sn, nxt);
        int64_t sq[Q], row[Q];
        int width[Q];
        bool valid[Q];
        bool group = true;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            sq[q] = sl + (int64_t)q * NW;
            width[q] = shape_width(cur.shape[q]);
            row[q] = cur.row0[q] + lane;
            valid[q] = lane < cur.nrows[q];
            // (slices stored singly: slot stride 64, as aligned_group reads them)
            group = group && cur.meta[q] >= 0 && width[q] == width[0] && shape_stride(cur.shape[q]) == kSlice;
        }
        group = group && width[0] >= 1 && width[0] <= kWMax;
        double y0[Q], y1[Q];
        if (group) {
            const int32_t* off[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) off[q] = A.soff + cur.meta[q];
            const int32_t* const(&co)[Q] = off;
            const int64_t(&base)[Q] = cur.base;
            switch (width[0]) {
            case 1: aligned_group<1, NX, Q>(A, base, co, lane, row, lo, hi, x0, x1, y0, y1); break;
            case 2: aligned_group<2, NX, Q>(A, base, co, lane, row, lo, hi, x0, x1, y0, y1); break;
            case 3: aligned_group<3, NX, Q>(A, base, co, lane, row, lo, hi, x0, x1, y0, y1); break;
            case 4: aligned_group<4, NX, Q>(A, base, co, lane, row, lo, hi, x0, x1, y0, y1); break;
            case 5: aligned_group<5, NX, Q>(A, base, co, lane, row, lo, hi, x0, x1, y0, y1); break;
            case 6: aligned_group<kWMax < 6 ? 1 : 6, NX, Q>(A, base, co, lane, row, lo, hi, x0, x1, y0, y1); break;
            case 7: aligned_group<kWMax < 7 ? 1 : 7, NX, Q>(A, base, co, lane, row, lo, hi, x0, x1, y0, y1); break;
            default: aligned_group<kWMax < 8 ? 1 : 8, NX, Q>(A, base, co, lane, row, lo, hi, x0, x1, y0, y1); break;
            }
        } else {
#pragma unroll
            for (int q = 0; q < Q; ++q) sell_row<NX>(A, sq[q], lane, row[q], x0, x1, y0[q], y1[q], lo, hi);
        }
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (valid[q]) f(row[q], y0[q], y1[q]);
        cur = nxt;
    }
    for (; sl < sl1; sl += NW) {
        const int64_t row = B.slice_row0[sl] + lane;
        const bool valid = lane < B.slice_nrows[sl];
        double y0, y1;
        sell_row<NX>(A, sl, lane, row, x0, x1, y0, y1, lo, hi);
        if (valid) f(row, y0, y1);
    }
}

// The vectors are parameters of their own, marked restrict (distinct
// arrays), so that loads of one row may be issued ahead of stores to
// another.  rt and stv are accessed only with a preconditioner.
template <int NT, bool PRE, int KIND, int Q>
__device__ __forceinline__ void solve_system(const BatchView& B, double* __restrict__ x, double* __restrict__ r,
                             double* __restrict__ rt, double* __restrict__ p, double* __restrict__ s,
                             double* __restrict__ stv, double* __restrict__ w, double* __restrict__ u,
                             const double* __restrict__ d, const double* __restrict__ b, double tol, int maxit,
                             int form, int sys, int32_t* __restrict__ iters_out, int32_t* __restrict__ status_out,
                             double* lds)
{
    constexpr int NW = NT / 64;
    // rows per thread whose loads are in flight together in the vector
    // updates (1024-thread workgroups have half the registers per thread)
    constexpr int kRowsAtOnce = NT >= 1024 ? 2 : 4;
    const int64_t r0 = B.sys_row0[sys], r1 = B.sys_row0[sys + 1];
    const int64_t sl0 = B.sys_slice0[sys], sl1 = B.sys_slice0[sys + 1];
    const int lo = (int)r0, hi = (int)r1 - 1;

    // ---- initialize (Appendix D): r0 = b - A x0, r~0 = M^{-1} r0, p0 = r~0
    double bb[1] = {0.0};
    sys_spmv<NT, 1, Q>(B, sl0, sl1, lo, hi, x, nullptr, [&](int64_t i, double ax, double) {
        const double bi = b[i];
        const double ri = bi - ax;
        r[i] = ri;
        const double rti = PRE ? d[i] * ri : ri;
        if (PRE && KIND != 0) rt[i] = rti;
        p[i] = rti;
        bb[0] = fma(bi, bi, bb[0]);
    });
    __syncthreads();
    // s0 = A p0 and mu0, sigma0, gamma0, nu0, <r0, r0>, <b, b>
    double t[6] = {0.0, 0.0, 0.0, 0.0, 0.0, bb[0]};
    sys_spmv<NT, 1, Q>(B, sl0, sl1, lo, hi, p, nullptr, [&](int64_t i, double si, double) {
        s[i] = si;
        const double ri = r[i];
        const double di = PRE ? d[i] : 1.0;
        const double sti = PRE ? di * si : si;
        const double rti = PRE ? di * ri : ri;
        if (PRE && KIND == 2) stv[i] = sti;
        t[0] = fma(p[i], si, t[0]);
        t[1] = fma(rti, si, t[1]);
        t[2] = fma(sti, si, t[2]);
        t[3] = fma(rti, ri, t[3]);
        t[4] = fma(ri, ri, t[4]);
    });
    block_sum<6, NW>(t, lds);
    State st = {};
    st.bnorm = sqrt(t[5]);
    st.tol = tol;
    st.maxit = maxit;
    st.k = -1;
    st.status = kNotConverged;
    if (t[5] == 0.0) {
        for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) x[i] = 0.0;
        st.k = 0;
        st.status = kOK;
        st.done = 1;
    } else if (KIND == 0) {
        step_hs_nu(st, t[3], PRE ? t[4] : t[3], nullptr, false);
        if (!st.done) step_hs_mu(st, t[0]);
    } else {
        double t5[5] = {t[0], t[1], t[2], t[3], t[4]};
        if (KIND == 2) {
            // w0 = A r~0 = s0; u0 = A s~0
            for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) w[i] = s[i];
            sys_spmv<NT, 1, Q>(B, sl0, sl1, lo, hi, PRE ? stv : s, nullptr, [&](int64_t i, double ui, double) { u[i] = ui; });
            __syncthreads();
        }
        step_one_reduction(st, t5, PRE, form, nullptr, false);
    }

    while (!st.done) {
        const double alpha = st.alpha, beta = st.beta;
        if (KIND == 1) {
            // Alg. 2: vector updates, then s = A p and the four (five) inner products
            #pragma unroll kRowsAtOnce
            for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
                const double si = s[i], pi = p[i], xi = x[i], ri = r[i];
                const double rn = fma(-alpha, si, ri);
                const double rtn = PRE ? fma(-alpha, d[i] * si, rt[i]) : rn;
                x[i] = fma(alpha, pi, xi);
                r[i] = rn;
                if (PRE) rt[i] = rtn;
                p[i] = fma(beta, pi, rtn);
            }
            __syncthreads();
            double q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            sys_spmv<NT, 1, Q>(B, sl0, sl1, lo, hi, p, nullptr, [&](int64_t i, double si, double) {
                s[i] = si;
                const double ri = r[i];
                const double rti = PRE ? rt[i] : ri;
                const double sti = PRE ? d[i] * si : si;
                q[0] = fma(p[i], si, q[0]);
                q[1] = fma(rti, si, q[1]);
                q[2] = fma(sti, si, q[2]);
                q[3] = fma(rti, ri, q[3]);
                if (PRE) q[4] = fma(ri, ri, q[4]);
            });
            block_sum<5, NW>(q, lds);
            step_one_reduction(st, q, PRE, form, nullptr, false);
        } else if (KIND == 2) {
            // Alg. 3: all vector updates and the inner products in one pass
            double q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            #pragma unroll kRowsAtOnce
            for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
                const double pi = p[i], si = s[i], wi = w[i], ui = u[i], xi = x[i], ri = r[i];
                const double rn = fma(-alpha, si, ri);
                const double wpi = fma(-alpha, ui, wi);
                const double snew = fma(beta, si, wpi);
                double rti = rn, sti = snew;
                if (PRE) {
                    const double di = d[i], sto = stv[i];
                    rti = fma(-alpha, sto, rt[i]);
                    sti = fma(beta, sto, fma(-alpha, di * ui, di * wi));
                    rt[i] = rti;
                    stv[i] = sti;
                }
                const double pnew = fma(beta, pi, rti);
                x[i] = fma(alpha, pi, xi);
                r[i] = rn;
                p[i] = pnew;
                s[i] = snew;
                q[0] = fma(pnew, snew, q[0]);
                q[1] = fma(rti, snew, q[1]);
                q[2] = fma(sti, snew, q[2]);
                q[3] = fma(rti, rn, q[3]);
                if (PRE) q[4] = fma(rn, rn, q[4]);
            }
            block_sum<5, NW>(q, lds);  // its barriers also publish the updated vectors
            step_one_reduction(st, q, PRE, form, nullptr, false);
            if (st.done) break;
            // u = A s~, w = A r~ (one pass over the system's matrix)
            sys_spmv<NT, 2, Q>(B, sl0, sl1, lo, hi, PRE ? stv : s, PRE ? rt : r, [&](int64_t i, double ui, double wi) {
                u[i] = ui;
                w[i] = wi;
            });
            __syncthreads();
        } else {
            // Alg. 1: x, r, nu; then beta and p; then s = A p and mu
            double q[2] = {0.0, 0.0};
            #pragma unroll kRowsAtOnce
            for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
                const double rn = fma(-alpha, s[i], r[i]);
                x[i] = fma(alpha, p[i], x[i]);
                r[i] = rn;
                const double rti = PRE ? d[i] * rn : rn;
                q[0] = fma(rti, rn, q[0]);
                if (PRE) q[1] = fma(rn, rn, q[1]);
            }
            block_sum<2, NW>(q, lds);
            step_hs_nu(st, q[0], PRE ? q[1] : q[0], nullptr, false);
            if (st.done) break;
            const double bk = st.beta;
            #pragma unroll kRowsAtOnce
            for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
                const double ri = r[i];
                p[i] = fma(bk, p[i], PRE ? d[i] * ri : ri);
            }
            __syncthreads();
            double m[1] = {0.0};
            sys_spmv<NT, 1, Q>(B, sl0, sl1, lo, hi, p, nullptr, [&](int64_t i, double si, double) {
                s[i] = si;
                m[0] = fma(p[i], si, m[0]);
            });
            block_sum<1, NW>(m, lds);
            step_hs_mu(st, m[0]);
        }
    }
    if (threadIdx.x == 0) {
        iters_out[sys] = st.k < 0 ? 0 : st.k;
        status_out[sys] = st.status;
    }
    __syncthreads();
}

template <int NT, bool PRE, int KIND, int Q>
__global__ __launch_bounds__(NT) void k_batch(BatchView B, Vecs v, const double* __restrict__ b, double tol,
                                              int maxit, int form, int32_t* __restrict__ queue,
                                              int32_t* __restrict__ iters_out, int32_t* __restrict__ status_out)
{
    __shared__ double lds[(NT / 64) * 6];
    __shared__ int s_next;
    for (;;) {
        if (threadIdx.x == 0) s_next = atomicAdd(queue, 1);
        __syncthreads();
        const int q = s_next;
        __syncthreads();
        if (q >= B.nsys) return;  // the queue only grows: every workgroup reaches this
        solve_system<NT, PRE, KIND, Q>(B, v.x, v.r, v.rt, v.p, v.s, v.st, v.w, v.u, v.d, b, tol, maxit, form, B.order[q],
                                    iters_out, status_out, lds);
    }
}

__global__ void k_batch_reset(int32_t* queue) { *queue = 0; }

// Batched PR-CG and M-CG in lockstep: every iteration is three launches over
// the row groups of all systems that are still running (the vector update,
// the product with its inner products, and one workgroup per system for
// stage 2 and the scalar step), so every compute unit works on the batch's
// rows whatever their systems.  Not part of the paper; each system runs
// exactly the single-system algorithm (Alg. 2 with the initialisation of
// Appendix D, same tests and scalar step as the persistent batched kernel)
// with its reductions split in two stages as in the single-system two-pass
// structure: one partial per row group, summed by the system's stage-2
// workgroup in a fixed order.
//
// A row group is up to kLockstepSlices consecutive slices of one system; a
// system that has finished (its state says done) costs each of its groups
// one load of the flag per launch.

// Product of a uniform row group (Group: offset-aligned slices of width W
// with one list of column offsets, stored one after another): wave w takes
// slices w, w + kWaves, ... of the group, R of them (the group holds
// kWaves R slices), in rounds of RR slices (RR W <= 20 value loads, to bound the
// registers): a round issues the loads of its values, of the W offsets, of
// each row's own entry x[row] and of each row's other entries (pre(i, row))
// together, before any gather, so a round costs two memory round trips.
// D0 >= 0: slot D0 holds offset 0 and slots D0 - 1 and D0 + 1 offsets -1 and
// +1; slot D0 then takes x[row] and its two neighbours x[row -+ 1] from the
// neighbouring lanes (cross-lane moves, no memory request) and the slice's
// two boundary entries, so a 5-point row gathers two entries instead of
// five.  D0 < 0: every slot is gathered.  Slices past the group's end are
// clamped to its last slice (their loads stay inside the group; their rows
// are skipped).  Columns are clamped into the system's rows [lo, hi] as in
// sell_row, and each row's slots are summed in stored order from 0.0: the
// same operands in the same order.  Calls f(i, row, y, x[row]) for the valid
// rows in slice order.  The group's width wg may be below W (a kernel
// compiled for the widest group of a table): slots wg .. W - 1 are skipped
// by wavefront-uniform branches.
constexpr int kLsRoundLoads = 20;  // value loads per round of uniform_group
template <int W, int D0, int R, class Pre, class F>
__device__ __forceinline__ void uniform_group(const SellView& A, const Group& G, const int wg,
                                              const double* __restrict__ x, Pre&& pre, F&& f)
{
    constexpr int RR = W * R <= kLsRoundLoads ? R : (W * R / 2 <= kLsRoundLoads ? R / 2 : 1);
    constexpr bool SHIFT = D0 >= 1 && D0 + 1 < W;
    const int w = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    int o[W];
#pragma unroll
    for (int u = 0; u < W; ++u) o[u] = G.o[u];
    // slot u reads the row's own entry or a lane neighbour's instead of memory
    constexpr auto local_slot = [](int u) { return SHIFT && (u == D0 - 1 || u == D0 || u == D0 + 1); };
    const double* __restrict__ vb = A.val + (int64_t)G.vrow * kSlice + lane;
#pragma unroll
    for (int i0 = 0; i0 < R; i0 += RR) {
        int row[RR];
        bool valid[RR];
        double a[RR][W], xs[RR], below[RR], above[RR];
#pragma unroll
        for (int j = 0; j < RR; ++j) {
            const int sl = w + kWaves * (i0 + j);
            const int slc = min(sl, G.nsl - 1);
            const int local = slc * kSlice + lane;
            valid[j] = sl < G.nsl && local < G.nrows;
            row[j] = G.row0 + min(local, G.nrows - 1);
#pragma unroll
            for (int u = 0; u < W; ++u)
                if (u < wg) a[j][u] = vb[(int64_t)(slc * wg + u) * kSlice];
            xs[j] = x[row[j]];
            if constexpr (SHIFT) {
                // the entries next to the slice, clamped into the system
                const int first = G.row0 + slc * kSlice;
                below[j] = x[max(first - 1, G.lo)];
                above[j] = x[min(first + kSlice, G.hi)];
            }
            pre(i0 + j, row[j]);
        }
        double g[RR][W];
#pragma unroll
        for (int j = 0; j < RR; ++j) {
#pragma unroll
            for (int u = 0; u < W; ++u) {
                if (u < wg && !local_slot(u)) g[j][u] = x[min(max(row[j] + o[u], G.lo), G.hi)];
            }
        }
#pragma unroll
        for (int j = 0; j < RR; ++j) {
            if constexpr (SHIFT) {
                double xm = __shfl_up(xs[j], 1, 64);
                double xp = __shfl_down(xs[j], 1, 64);
                if (lane == 0) xm = below[j];
                if (lane == kSlice - 1) xp = above[j];
                g[j][D0 - 1] = xm;
                g[j][D0] = xs[j];
                g[j][D0 + 1] = xp;
            }
            double y = 0.0;
#pragma unroll
            for (int u = 0; u < W; ++u)
                if (u < wg) y = fma(a[j][u], g[j][u], y);
            // y in a register here, outside the valid rows' branch: otherwise
            // the compiler moves a slice's loads into that branch, behind
            // the wait for the cross-lane moves, and they no longer overlap
            // with the other slices' loads
            asm volatile("" : "+v"(y));
            if (valid[j]) f(i0 + j, row[j], y, xs[j]);
        }
    }
}

// Occupancy floor of the lockstep product (wavefronts per SIMD: at most
// 128 registers per thread; with a preconditioner, whose rows carry two more
// entries, one wavefront less).
constexpr int kLockstepSpmvWaves = 4;

// PHASE 1: r0 = b - A x0, r~0 = M^{-1} r0, p0 = r~0 and the <b, b> partial.
// PHASE 2: s0 = A p0 and the partials of mu, sigma, gamma, nu, <r, r>.
// PHASE 0: the same product for an iteration of a system still running.
// The group's slices go through sys_spmv (two slices per wavefront with
// their loads in flight together).
// UW > 0: every group of the table is uniform, of width at most UW (the
// kernel then holds that one product and needs fewer registers, so more
// workgroups fit on a compute unit).
template <bool PRE, int PHASE, int SPW, int UW = 0>
__global__ __launch_bounds__(kBlock, PRE ? kLockstepSpmvWaves - 1 : kLockstepSpmvWaves) void k_ls_spmv(BatchView B, GroupView gv, const State* __restrict__ S, Vecs v,
                                                    const double* __restrict__ b, double* __restrict__ P)
{
    __shared__ double lds[kWaves * 5];
    const int64_t g = blockIdx.x;
    if (PHASE == 0 && gv.gdone[g]) return;  // the whole workgroup
    const Group G = gv.grp[g];
    double* __restrict__ r = v.r;
    double* __restrict__ rt = v.rt;
    double* __restrict__ p = v.p;
    double* __restrict__ s = v.s;
    const double* __restrict__ d = v.d;
    constexpr int NV = PHASE == 1 ? 1 : 5;
    double q[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) q[i] = 0.0;
    // the row's contribution once y = (A x)_row is known; e0 .. e3 hold the
    // row's own entries (PHASE 1: b; else p, r, r~, d)
    auto row_done = [&](int64_t row, double y0, double e0, double e1, double e2, double e3) {
        if constexpr (PHASE == 1) {
            const double bi = e0;
            const double ri = bi - y0;
            const double rti = PRE ? e3 * ri : ri;
            r[row] = ri;
            if (PRE) rt[row] = rti;
            p[row] = rti;
            q[0] = fma(bi, bi, q[0]);
        } else {
            s[row] = y0;
            const double ri = e1;
            const double rti = PRE ? e2 : ri;
            const double sti = PRE ? e3 * y0 : y0;
            q[0] = fma(e0, y0, q[0]);
            q[1] = fma(rti, y0, q[1]);
            q[2] = fma(sti, y0, q[2]);
            q[3] = fma(rti, ri, q[3]);
            if (PRE) q[4] = fma(ri, ri, q[4]);
        }
    };
    const double* __restrict__ xin = PHASE == 1 ? v.x : p;
    constexpr int R = SPW;
    double e0[R], e1[R], e2[R], e3[R];
    // the product of a uniform group
    auto uniform_product = [&]() {
        auto pre = [&](int i, int row) {
            if constexpr (PHASE == 1) {
                e0[i] = b[row];
                e1[i] = e2[i] = 0.0;
                e3[i] = PRE ? d[row] : 1.0;
            } else {
                e1[i] = r[row];
                e2[i] = PRE ? rt[row] : 0.0;
                e3[i] = PRE ? d[row] : 1.0;
            }
        };
        // PHASE 0 and 2 multiply p, so p[row] is the row's own entry
        auto f = [&](int i, int row, double y, double xrow) {
            row_done(row, y, PHASE == 1 ? e0[i] : xrow, e1[i], e2[i], e3[i]);
        };
        // stencils whose sorted offsets put 0 in the middle slot, flanked by
        // -1 and +1, take the neighbours from the lanes
        auto go = [&](auto Wc) {
            constexpr int W = decltype(Wc)::value;
            const int wg = UW > 0 ? G.width : W;
            if (W >= 3 && (G.flags & kGroupShift) && G.diag == W / 2)
                uniform_group<W, W / 2, R>(B.A, G, wg, xin, pre, f);
            else
                uniform_group<W, -1, R>(B.A, G, wg, xin, pre, f);
        };
        if constexpr (UW > 0) {
            go(std::integral_constant<int, UW>{});
        } else {
            switch (G.width) {
            case 1: go(std::integral_constant<int, 1>{}); break;
            case 2: go(std::integral_constant<int, 2>{}); break;
            case 3: go(std::integral_constant<int, 3>{}); break;
            case 4: go(std::integral_constant<int, 4>{}); break;
            case 5: go(std::integral_constant<int, 5>{}); break;
            case 6: go(std::integral_constant<int, 6>{}); break;
            case 7: go(std::integral_constant<int, 7>{}); break;
            default: go(std::integral_constant<int, kUniformMaxWidth>{}); break;
            }
        }
    };
    if constexpr (UW > 0) {
        uniform_product();
    } else if (G.off >= 0) {
        uniform_product();
    } else {
        sys_spmv<kBlock, 1, 2>(B, G.slice0, G.slice0 + G.nsl, G.lo, G.hi, xin, nullptr,
                            [&](int64_t row, double y0, double) {
                                if constexpr (PHASE == 1)
                                    row_done(row, y0, b[row], 0.0, 0.0, PRE ? d[row] : 1.0);
                                else
                                    row_done(row, y0, p[row], r[row], PRE ? rt[row] : 0.0, PRE ? d[row] : 1.0);
                            });
    }
    block_sum<NV, kWaves>(q, lds);
    if (threadIdx.x == 0) {
        const int64_t ng = gv.ngroups;
        if (PHASE == 1)
            P[5 * ng + g] = q[0];
        else
#pragma unroll
            for (int i = 0; i < NV; ++i) P[i * ng + g] = q[i];
    }
}

// x_{k+1} = x_k + alpha p_k, r_{k+1} = r_k - alpha s_k, r~_{k+1} = r~_k -
// alpha M^{-1} s_k, p_{k+1} = r~_{k+1} + beta p_k (Alg. 2); the loads of
// several rows per thread in flight together.
template <bool PRE>
__global__ __launch_bounds__(kBlock) void k_ls_update(GroupView gv, const State* __restrict__ S, Vecs v)
{
    // the groups in the order opposite to k_ls_spmv's, so each kernel
    // starts on the groups the other touched last (still in the last-level
    // cache); the flag and the record load together, the state's scalars
    // with the rows (they are needed only for the arithmetic)
    const int64_t g = gv.ngroups - 1 - blockIdx.x;
    if (gv.gdone[g]) return;
    const Group G = gv.grp[g];
    const double alpha = S[G.sys].alpha, beta = S[G.sys].beta;
    double* __restrict__ x = v.x;
    double* __restrict__ r = v.r;
    double* __restrict__ rt = v.rt;
    double* __restrict__ p = v.p;
    const double* __restrict__ s = v.s;
    const double* __restrict__ d = v.d;
    const int64_t i1 = G.row0 + G.nrows;
#pragma unroll 4
    for (int64_t i = G.row0 + threadIdx.x; i < i1; i += kBlock) {
        const double si = s[i], pi = p[i], xi = x[i], ri = r[i];
        const double rn = fma(-alpha, si, ri);
        const double rtn = PRE ? fma(-alpha, d[i] * si, rt[i]) : rn;
        x[i] = fma(alpha, pi, xi);
        r[i] = rn;
        if (PRE) rt[i] = rtn;
        p[i] = fma(beta, pi, rtn);
    }
}

// Stage 2 and the scalar step of one running system by one workgroup:
// thread t adds the partials of groups g0 + t, g0 + t + kBlock, ... in that
// order from 0.0, the thread sums go through block_sum, then the scalar
// step; the groups' done flags are set when the system ends.
// COHERENT: the partials were written in the same launch, by workgroups on
// other XCDs, with agent-scope atomic stores; they are read the same way.
template <bool PRE, bool COHERENT = false>
__device__ __forceinline__ void finish_system(const GroupView& gv, State* __restrict__ S,
                                              const double* __restrict__ P, int sys, int form,
                                              int32_t* __restrict__ iters, int32_t* __restrict__ status)
{
    __shared__ double lds[kWaves * 5];
    State st = load_state(S + sys);
    if (st.done) return;
    const int64_t g0 = gv.sys_grp0[sys], g1 = gv.sys_grp0[sys + 1], ng = gv.ngroups;
    double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kBlock) {
#pragma unroll
        for (int i = 0; i < 5; ++i)
            t[i] += COHERENT ? __hip_atomic_load(P + i * ng + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                             : P[i * ng + g];
    }
    block_sum<5, kWaves>(t, lds);
    step_one_reduction(st, t, PRE, form, nullptr, false);
    if (threadIdx.x == 0) {
        store_state(S + sys, st);
        iters[sys] = st.k < 0 ? 0 : st.k;
        status[sys] = st.status;
    }
    if (st.done) {
        for (int64_t g = g0 + threadIdx.x; g < g1; g += kBlock) gv.gdone[g] = 1;
    }
}

// One lockstep iteration of a uniform group with the update and the product
// in one pass (PR-CG, M-CG).  k_ls_update followed by k_ls_spmv moves ten
// vector words per row without a preconditioner (x, r, p, s read; x, r, p
// written; p, r read again; s written); this kernel moves eight (x, r, p, s
// read; x, r', p', s' written; with Jacobi also r~ and d read and r~'
// written).  The product s' = A p' needs p' at every column the group's
// rows reach, which extends past the group by the stencil's span (within
// the system): the workgroup recomputes p' there from r~, s and p (and d),
// which its neighbouring groups read as their own rows at about the same
// time (the workgroup-to-group map keeps neighbouring groups on one XCD, so
// these reads are served by its L2).  Reads r~, p, s from `in` and writes
// r~', p', s' to `out`: other workgroups still read the old values.  x (and
// r, with a preconditioner) is updated in place.  Every row's arithmetic
// and the order of every sum are those of k_ls_update then
// k_ls_spmv<PRE, 0, SPW>, and the last workgroup of each system (by a
// ticket) then runs the stage 2 and scalar step of k_ls_finish: the results
// agree bit for bit with those three launches.  (The other workgroups of
// the system have read alpha and beta before they took their tickets, so
// the state may change then.)
//   window: LDS, p' at the rows [wlo, whi] (the clamped columns of the
//           group's rows); then r' and (PRE) r~' at the group's own rows.
constexpr int kWindowRows = 4;  // window rows per thread whose loads k_ls_fused issues together
template <bool PRE, int SPW, int W>
__global__ __launch_bounds__(kBlock) void k_ls_fused(BatchView B, GroupView gv, State* __restrict__ S,
                                                     double* __restrict__ x, const double* __restrict__ d,
                                                     LsVecs in, LsVecs out, double* __restrict__ P, int form,
                                                     int32_t* __restrict__ iters, int32_t* __restrict__ status,
                                                     int reverse)
{
    extern __shared__ double window[];
    __shared__ double lds[kWaves * 5];
    // XCD x (workgroups b with b mod 8 = x) takes a contiguous range of
    // groups, in increasing order, or decreasing on every other iteration
    // (reverse): an iteration then starts on the groups the previous one
    // touched last, whose vectors may still be in the last-level cache
    const int64_t gp = gridDim.x;  // a multiple of 8
    const int64_t pos = blockIdx.x / 8;
    const int64_t g = (blockIdx.x % 8) * (gp / 8) + (reverse ? gp / 8 - 1 - pos : pos);
    if (g >= gv.ngroups || gv.gdone[g]) return;  // the whole workgroup
    const Group G = gv.grp[g];
    const double alpha = S[G.sys].alpha, beta = S[G.sys].beta;
    const int w = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // the window holds the group's own rows and every column they reach;
    // slots wg .. W - 1 (a group narrower than the table's widest) are
    // skipped by wavefront-uniform branches
    const int wg = G.width;
    int o[W];
    int omin = 0, omax = 0;
#pragma unroll
    for (int u = 0; u < W; ++u) {
        o[u] = u < wg ? G.o[u] : 0;
        omin = min(omin, o[u]);
        omax = max(omax, o[u]);
    }
    const int last = G.row0 + G.nrows - 1;
    const int wlo = min(max(G.row0 + omin, G.lo), G.hi);
    const int whi = max(min(last + omax, G.hi), G.lo);
    double* __restrict__ rown = window + (whi - wlo + 1);  // r' of the group's rows
    double* __restrict__ rtown = rown + G.nrows;           // with PRE: r~' of the group's rows
    // the product's values first: they do not depend on the update
    const double* __restrict__ vb = B.A.val + (int64_t)G.vrow * kSlice + lane;
    double a[SPW][W], dr[SPW];
    int row[SPW];
    bool valid[SPW];
#pragma unroll
    for (int j = 0; j < SPW; ++j) {
        const int sl = w + kWaves * j;
        const int slc = min(sl, G.nsl - 1);
        const int local = slc * kSlice + lane;
        valid[j] = sl < G.nsl && local < G.nrows;
        row[j] = G.row0 + min(local, G.nrows - 1);
#pragma unroll
        for (int u = 0; u < W; ++u)
            if (u < wg) a[j][u] = __builtin_nontemporal_load(&vb[(int64_t)(slc * wg + u) * kSlice]);
        dr[j] = PRE ? d[row[j]] : 1.0;
    }
    // p' over the window (r', r~' and x as well at the group's own rows);
    // the two buffer sets never overlap.  Without a preconditioner p' is
    // formed from r (= r~), which alternates between the sets; with one,
    // from r~ and d, which alternate, while r is read and written at the
    // group's own rows only and stays in place (r_io).
    const double* __restrict__ in_t = PRE ? in.rt : in.r;  // r~ (old)
    const double* __restrict__ in_p = in.p;
    const double* __restrict__ in_s = in.s;
    double* __restrict__ out_t = PRE ? out.rt : out.r;     // r~ (new)
    double* __restrict__ out_p = out.p;
    double* __restrict__ out_s = out.s;
    double* __restrict__ r_io = in.r;                      // PRE: r, updated in place
    // kWindowRows rows per thread at a time: their loads are issued
    // together (rows past the window load its last row and are skipped)
    constexpr int U = kWindowRows;
    for (int i0 = wlo + (int)threadIdx.x; i0 <= whi; i0 += U * kBlock) {
        double sv[U], pv[U], tv[U], xv[U], dv[U], rv[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int i = min(i0 + k * kBlock, whi);
            const bool own = i >= G.row0 && i <= last;
            sv[k] = in_s[i];
            pv[k] = in_p[i];
            tv[k] = in_t[i];
            xv[k] = own ? x[i] : 0.0;
            dv[k] = PRE ? d[i] : 1.0;
            rv[k] = PRE && own ? r_io[i] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int i = i0 + k * kBlock;
            if (i > whi) break;
            // k_ls_update's expressions: r' = r - alpha s, r~' = r~ - alpha
            // d s (= r' without a preconditioner), p' = r~' + beta p
            const double tn = PRE ? fma(-alpha, dv[k] * sv[k], tv[k]) : fma(-alpha, sv[k], tv[k]);
            const double pn = fma(beta, pv[k], tn);
            window[i - wlo] = pn;
            if (i >= G.row0 && i <= last) {
                __builtin_nontemporal_store(fma(alpha, pv[k], xv[k]), &x[i]);
                __builtin_nontemporal_store(tn, &out_t[i]);
                __builtin_nontemporal_store(pn, &out_p[i]);
                if constexpr (PRE) {
                    const double rn = fma(-alpha, sv[k], rv[k]);
                    __builtin_nontemporal_store(rn, &r_io[i]);
                    rown[i - G.row0] = rn;
                    rtown[i - G.row0] = tn;
                } else {
                    rown[i - G.row0] = tn;
                }
            }
        }
    }
    __syncthreads();
    double q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < SPW; ++j) {
        double y = 0.0;
#pragma unroll
        for (int u = 0; u < W; ++u)
            if (u < wg) y = fma(a[j][u], window[min(max(row[j] + o[u], G.lo), G.hi) - wlo], y);
        if (valid[j]) {
            // k_ls_spmv's inner products: <p, s>, <r~, s>, <s~, s>, <r~, r>
            // and, with a preconditioner, <r, r>
            const double pi = window[row[j] - wlo], ri = rown[row[j] - G.row0];
            const double ti = PRE ? rtown[row[j] - G.row0] : ri;
            const double sti = PRE ? dr[j] * y : y;
            __builtin_nontemporal_store(y, &out_s[row[j]]);
            q[0] = fma(pi, y, q[0]);
            q[1] = fma(ti, y, q[1]);
            q[2] = fma(sti, y, q[2]);
            q[3] = fma(ti, ri, q[3]);
            if (PRE) q[4] = fma(ri, ri, q[4]);
        }
    }
    block_sum<5, kWaves>(q, lds);
    // The system's last workgroup to finish takes its stage 2 and scalar
    // step.  The partials go out as agent-scope atomic stores (coherent
    // across the XCDs' L2 caches) and thread 0 waits for them to complete
    // before it takes its ticket, so the workgroup that draws the last
    // ticket reads every partial of its system with agent-scope atomic
    // loads; no fence has to write back an L2.
    __shared__ int is_last;
    const int sys = G.sys;
    if (threadIdx.x == 0) {
        const int64_t ng = gv.ngroups;
#pragma unroll
        for (int i = 0; i < 5; ++i) __hip_atomic_store(P + i * ng + g, q[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0);
        const int nsg = (int)(gv.sys_grp0[sys + 1] - gv.sys_grp0[sys]);
        const int t = __hip_atomic_fetch_add(gv.ticket + sys, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        is_last = t == nsg - 1;
        if (is_last) __hip_atomic_store(gv.ticket + sys, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (is_last) finish_system<PRE, true>(gv, S, P, sys, form, iters, status);
}

// Stage 2 and the scalar step of one system (one workgroup per system):
// thread t adds the partials of groups g0 + t, g0 + t + kBlock, ... in that
// order from 0.0, and the thread sums go through block_sum.  INIT also sets
// up the state (||b||, tol, maxit) and handles b = 0 (x = 0, converged).
template <bool PRE, bool INIT>
__global__ __launch_bounds__(kBlock) void k_ls_finish(BatchView B, GroupView gv, State* __restrict__ S,
                                                      const double* __restrict__ P, double* __restrict__ x, double tol,
                                                      int maxit, int form, int32_t* __restrict__ iters,
                                                      int32_t* __restrict__ status)
{
    const int sys = blockIdx.x;
    if constexpr (!INIT) {
        finish_system<PRE>(gv, S, P, sys, form, iters, status);
    } else {
        constexpr int NV = 6;
        __shared__ double lds[kWaves * NV];
        State st = State{};
        st.tol = tol;
        st.maxit = maxit;
        st.k = -1;
        st.status = kNotConverged;
        const int64_t g0 = gv.sys_grp0[sys], g1 = gv.sys_grp0[sys + 1], ng = gv.ngroups;
        double t[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) t[i] = 0.0;
        for (int64_t g = g0 + threadIdx.x; g < g1; g += kBlock) {
#pragma unroll
            for (int i = 0; i < NV; ++i) t[i] += P[i * ng + g];
        }
        block_sum<NV, kWaves>(t, lds);
        const double t5[5] = {t[0], t[1], t[2], t[3], t[4]};
        st.bnorm = sqrt(t[NV - 1]);
        if (t[NV - 1] == 0.0) {
            for (int64_t i = B.sys_row0[sys] + threadIdx.x; i < B.sys_row0[sys + 1]; i += kBlock) x[i] = 0.0;
            st.k = 0;
            st.status = kOK;
            st.done = 1;
        } else {
            step_one_reduction(st, t5, PRE, form, nullptr, false);
        }
        if (threadIdx.x == 0) {
            store_state(S + sys, st);
            iters[sys] = st.k < 0 ? 0 : st.k;
            status[sys] = st.status;
            gv.ticket[sys] = 0;  // the fused iteration's stage-2 ticket
        }
        // the groups' copies of the flag (the next kernels read them instead
        // of the state, with no load before)
        for (int64_t g = g0 + threadIdx.x; g < g1; g += kBlock) gv.gdone[g] = st.done;
    }
}

// Number of systems still running (one workgroup).
__global__ __launch_bounds__(kBlock) void k_ls_count(const State* __restrict__ S, int nsys, int32_t* __restrict__ active)
{
    __shared__ double lds[kWaves];
    double c[1] = {0.0};
    for (int q = threadIdx.x; q < nsys; q += kBlock) c[0] += S[q].done ? 0.0 : 1.0;
    block_sum<1, kWaves>(c, lds);
    if (threadIdx.x == 0) *active = (int32_t)c[0];
}


template <int NT, class F>
hipError_t with_kind(int kind, int pre, int q, F&& f)
{
    auto go = [&](auto P, auto Q) -> hipError_t {
        switch (kind) {
        case 0: return f(std::integral_constant<int, NT>{}, P, std::integral_constant<int, 0>{}, Q);
        case 1: return f(std::integral_constant<int, NT>{}, P, std::integral_constant<int, 1>{}, Q);
        default: return f(std::integral_constant<int, NT>{}, P, std::integral_constant<int, 2>{}, Q);
        }
    };
    auto goq = [&](auto P) -> hipError_t {
        return q == 1 ? go(P, std::integral_constant<int, 1>{}) : go(P, std::integral_constant<int, 2>{});
    };
    return pre ? goq(std::true_type{}) : goq(std::false_type{});
}

// Calls f(std::integral_constant<int, SPW>) for the group view's slices per
// wavefront.
template <class F>
hipError_t with_spw(const GroupView& gv, F&& f)
{
    switch (gv.spw) {
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 8: return f(std::integral_constant<int, 8>{});
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_batch(const BatchView& B, const Vecs& v, const double* b, double tol, int maxit, int variant,
                        int pre, int nt, int grid, int q, int32_t* queue, int32_t* iters, int32_t* status,
                        hipStream_t st)
{
    const int kind = variant == kHS ? 0 : (variant == kPR || variant == kM) ? 1 : 2;
    const int form = nu_form(variant);
    if (q != 1 && q != 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, st, queue);
    auto body = [&](auto NTc, auto P, auto Kc, auto Qc) -> hipError_t {
        constexpr int T = decltype(NTc)::value;
        hipLaunchKernelGGL((k_batch<T, decltype(P)::value, decltype(Kc)::value, decltype(Qc)::value>), dim3(grid),
                           dim3(T), 0, st, B, v, b, tol, maxit, form, queue, iters, status);
        return hipGetLastError();
    };
    switch (nt) {
    case 256: return with_kind<256>(kind, pre, q, body);
    case 512: return with_kind<512>(kind, pre, q, body);
    case 1024: return with_kind<1024>(kind, pre, q, body);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lockstep_init(const BatchView& B, const GroupView& gv, const Vecs& v, const double* b, State* S,
                                double* P, double tol, int maxit, int variant, int pre, int32_t* iters,
                                int32_t* status, hipStream_t st)
{
    const int form = nu_form(variant);
    const dim3 grid((unsigned)gv.ngroups), nsys((unsigned)B.nsys), blk(kBlock);
    return with_spw(gv, [&](auto SPWc) -> hipError_t {
        constexpr int SPW = decltype(SPWc)::value;
        if (pre) {
            hipLaunchKernelGGL((k_ls_spmv<true, 1, SPW>), grid, blk, 0, st, B, gv, S, v, b, P);
            hipLaunchKernelGGL((k_ls_spmv<true, 2, SPW>), grid, blk, 0, st, B, gv, S, v, b, P);
            hipLaunchKernelGGL((k_ls_finish<true, true>), nsys, blk, 0, st, B, gv, S, P, v.x, tol, maxit, form, iters,
                               status);
        } else {
            hipLaunchKernelGGL((k_ls_spmv<false, 1, SPW>), grid, blk, 0, st, B, gv, S, v, b, P);
            hipLaunchKernelGGL((k_ls_spmv<false, 2, SPW>), grid, blk, 0, st, B, gv, S, v, b, P);
            hipLaunchKernelGGL((k_ls_finish<false, true>), nsys, blk, 0, st, B, gv, S, P, v.x, tol, maxit, form,
                               iters, status);
        }
        return hipGetLastError();
    });
}

hipError_t launch_lockstep_iterations(const BatchView& B, const GroupView& gv, const Vecs& v, State* S, double* P,
                                      int iterations, int variant, int pre, bool fused, int32_t* iters,
                                      int32_t* status, int32_t* active, hipStream_t st)
{
    const int form = nu_form(variant);
    const dim3 grid((unsigned)gv.ngroups), nsys((unsigned)B.nsys), blk(kBlock);
    if (fused) {
        if (iterations % 2 != 0 || (gv.spw != 2 && gv.spw != 4) ||
            (gv.uwidth != 3 && gv.uwidth != 5 && gv.uwidth != 7))
            return hipErrorInvalidValue;
        const dim3 fgrid((unsigned)((gv.ngroups + 7) / 8 * 8));
        const size_t lds = sizeof(double) * (size_t)fused_lds_doubles(kWaves * gv.spw * kSlice, gv.span, pre != 0);
        if (lds > sizeof(double) * (size_t)kFuseLdsDoubles) return hipErrorInvalidValue;
        // the two buffer sets: r (without a preconditioner), r~ (with one),
        // p and s alternate; with one, r stays in place
        const LsVecs A = pre ? LsVecs{v.r, v.p, v.s, v.rt} : LsVecs{v.r, v.p, v.s, nullptr};
        const LsVecs A2 = pre ? LsVecs{v.r, v.u, v.st, v.w} : LsVecs{v.w, v.u, v.st, nullptr};
        auto go = [&](auto SPWc, auto Wc) -> hipError_t {
            constexpr int SPW = decltype(SPWc)::value, W = decltype(Wc)::value;
            for (int k = 0; k < iterations; ++k) {
                if (pre)
                    hipLaunchKernelGGL((k_ls_fused<true, SPW, W>), fgrid, blk, lds, st, B, gv, S, v.x, v.d,
                                       k % 2 ? A2 : A, k % 2 ? A : A2, P, form, iters, status, k % 2);
                else
                    hipLaunchKernelGGL((k_ls_fused<false, SPW, W>), fgrid, blk, lds, st, B, gv, S, v.x, v.d,
                                       k % 2 ? A2 : A, k % 2 ? A : A2, P, form, iters, status, k % 2);
            }
            return hipGetLastError();
        };
        auto gow = [&](auto SPWc) -> hipError_t {
            switch (gv.uwidth) {
            case 3: return go(SPWc, std::integral_constant<int, 3>{});
            case 5: return go(SPWc, std::integral_constant<int, 5>{});
            default: return go(SPWc, std::integral_constant<int, 7>{});
            }
        };
        hipError_t e = gv.spw == 2 ? gow(std::integral_constant<int, 2>{}) : gow(std::integral_constant<int, 4>{});
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_ls_count, dim3(1), blk, 0, st, S, B.nsys, active);
        return hipGetLastError();
    }
    hipError_t e = with_spw(gv, [&](auto SPWc) -> hipError_t {
        constexpr int SPW = decltype(SPWc)::value;
        for (int k = 0; k < iterations; ++k) {
            if (pre) {
                hipLaunchKernelGGL((k_ls_update<true>), grid, blk, 0, st, gv, S, v);
                hipLaunchKernelGGL((k_ls_spmv<true, 0, SPW>), grid, blk, 0, st, B, gv, S, v, nullptr, P);
                hipLaunchKernelGGL((k_ls_finish<true, false>), nsys, blk, 0, st, B, gv, S, P, v.x, 0.0, 0, form,
                                   iters, status);
            } else {
                hipLaunchKernelGGL((k_ls_update<false>), grid, blk, 0, st, gv, S, v);
                switch (gv.uwidth) {
                case 3: hipLaunchKernelGGL((k_ls_spmv<false, 0, SPW, 3>), grid, blk, 0, st, B, gv, S, v, nullptr, P); break;
                case 5: hipLaunchKernelGGL((k_ls_spmv<false, 0, SPW, 5>), grid, blk, 0, st, B, gv, S, v, nullptr, P); break;
                case 7: hipLaunchKernelGGL((k_ls_spmv<false, 0, SPW, 7>), grid, blk, 0, st, B, gv, S, v, nullptr, P); break;
                default: hipLaunchKernelGGL((k_ls_spmv<false, 0, SPW>), grid, blk, 0, st, B, gv, S, v, nullptr, P); break;
                }
                hipLaunchKernelGGL((k_ls_finish<false, false>), nsys, blk, 0, st, B, gv, S, P, v.x, 0.0, 0, form,
                                   iters, status);
            }
        }
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ls_count, dim3(1), blk, 0, st, S, B.nsys, active);
    return hipGetLastError();
}

}  // namespace prcg
