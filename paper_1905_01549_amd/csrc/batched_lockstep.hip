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
// A row group is up to four consecutive slices of one system (kGroupRows
// rows); a system that has finished (its state says done) costs its groups
// one load of the flag per launch.
#include "batched.h"
#include "prcg_device.h"

namespace prcg {

namespace {

// PHASE 1: r0 = b - A x0, r~0 = M^{-1} r0, p0 = r~0 and the <b, b> partial.
// PHASE 2: s0 = A p0 and the partials of mu, sigma, gamma, nu, <r, r>.
// PHASE 0: the same product for an iteration of a system still running.
template <bool PRE, int PHASE>
__global__ __launch_bounds__(kBlock) void k_ls_spmv(BatchView B, GroupView gv, const State* __restrict__ S, Vecs v,
                                                    const double* __restrict__ b, double* __restrict__ P)
{
    __shared__ double lds[kWaves * 5];
    const int64_t g = blockIdx.x;
    const int sys = gv.grp_sys[g];
    if (PHASE == 0 && S[sys].done) return;  // the whole workgroup
    const int w = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t sl = gv.grp_slice0[g] + w;
    constexpr int NV = PHASE == 1 ? 1 : 5;
    double q[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) q[i] = 0.0;
    if (sl < B.sys_slice0[sys + 1]) {
        const int64_t row = B.slice_row0[sl] + lane;
        const bool valid = lane < B.slice_nrows[sl];
        double y0, y1;
        sell_row<1>(B.A, sl, lane, row, PHASE == 1 ? v.x : v.p, nullptr, y0, y1);
        if (valid) {
            if constexpr (PHASE == 1) {
                const double bi = b[row];
                const double ri = bi - y0;
                const double rti = PRE ? v.d[row] * ri : ri;
                v.r[row] = ri;
                if (PRE) v.rt[row] = rti;
                v.p[row] = rti;
                q[0] = bi * bi;
            } else {
                v.s[row] = y0;
                const double ri = v.r[row];
                const double rti = PRE ? v.rt[row] : ri;
                const double sti = PRE ? v.d[row] * y0 : y0;
                q[0] = v.p[row] * y0;
                q[1] = rti * y0;
                q[2] = sti * y0;
                q[3] = rti * ri;
                q[4] = PRE ? ri * ri : 0.0;
            }
        }
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
// alpha M^{-1} s_k, p_{k+1} = r~_{k+1} + beta p_k (Alg. 2).
template <bool PRE>
__global__ __launch_bounds__(kBlock) void k_ls_update(BatchView B, GroupView gv, const State* __restrict__ S, Vecs v)
{
    const int64_t g = blockIdx.x;
    const int sys = gv.grp_sys[g];
    if (S[sys].done) return;
    const double alpha = S[sys].alpha, beta = S[sys].beta;
    const int64_t sl = gv.grp_slice0[g] + uniform(threadIdx.x >> 6);
    if (sl >= B.sys_slice0[sys + 1]) return;
    const int lane = threadIdx.x & 63;
    if (lane >= B.slice_nrows[sl]) return;
    const int64_t i = B.slice_row0[sl] + lane;
    const double si = v.s[i], pi = v.p[i], xi = v.x[i], ri = v.r[i];
    const double rn = fma(-alpha, si, ri);
    const double rtn = PRE ? fma(-alpha, v.d[i] * si, v.rt[i]) : rn;
    v.x[i] = fma(alpha, pi, xi);
    v.r[i] = rn;
    if (PRE) v.rt[i] = rtn;
    v.p[i] = fma(beta, pi, rtn);
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
    constexpr int NV = INIT ? 6 : 5;
    __shared__ double lds[kWaves * NV];
    const int sys = blockIdx.x;
    State st;
    if (INIT) {
        st = State{};
        st.tol = tol;
        st.maxit = maxit;
        st.k = -1;
        st.status = kNotConverged;
    } else {
        st = load_state(S + sys);
        if (st.done) return;
    }
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
    if (INIT) {
        st.bnorm = sqrt(t[NV - 1]);
        if (t[NV - 1] == 0.0) {
            for (int64_t i = B.sys_row0[sys] + threadIdx.x; i < B.sys_row0[sys + 1]; i += kBlock) x[i] = 0.0;
            st.k = 0;
            st.status = kOK;
            st.done = 1;
        } else {
            step_one_reduction(st, t5, PRE, form, nullptr, false);
        }
    } else {
        step_one_reduction(st, t5, PRE, form, nullptr, false);
    }
    if (threadIdx.x == 0) {
        store_state(S + sys, st);
        iters[sys] = st.k < 0 ? 0 : st.k;
        status[sys] = st.status;
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

}  // namespace

hipError_t launch_lockstep_init(const BatchView& B, const GroupView& gv, const Vecs& v, const double* b, State* S,
                                double* P, double tol, int maxit, int variant, int pre, int32_t* iters,
                                int32_t* status, hipStream_t st)
{
    const int form = nu_form(variant);
    const dim3 grid((unsigned)gv.ngroups), nsys((unsigned)B.nsys), blk(kBlock);
    if (pre) {
        hipLaunchKernelGGL((k_ls_spmv<true, 1>), grid, blk, 0, st, B, gv, S, v, b, P);
        hipLaunchKernelGGL((k_ls_spmv<true, 2>), grid, blk, 0, st, B, gv, S, v, b, P);
        hipLaunchKernelGGL((k_ls_finish<true, true>), nsys, blk, 0, st, B, gv, S, P, v.x, tol, maxit, form, iters,
                           status);
    } else {
        hipLaunchKernelGGL((k_ls_spmv<false, 1>), grid, blk, 0, st, B, gv, S, v, b, P);
        hipLaunchKernelGGL((k_ls_spmv<false, 2>), grid, blk, 0, st, B, gv, S, v, b, P);
        hipLaunchKernelGGL((k_ls_finish<false, true>), nsys, blk, 0, st, B, gv, S, P, v.x, tol, maxit, form, iters,
                           status);
    }
    return hipGetLastError();
}

hipError_t launch_lockstep_iterations(const BatchView& B, const GroupView& gv, const Vecs& v, State* S, double* P,
                                      int iterations, int variant, int pre, int32_t* iters, int32_t* status,
                                      int32_t* active, hipStream_t st)
{
    const int form = nu_form(variant);
    const dim3 grid((unsigned)gv.ngroups), nsys((unsigned)B.nsys), blk(kBlock);
    for (int k = 0; k < iterations; ++k) {
        if (pre) {
            hipLaunchKernelGGL((k_ls_update<true>), grid, blk, 0, st, B, gv, S, v);
            hipLaunchKernelGGL((k_ls_spmv<true, 0>), grid, blk, 0, st, B, gv, S, v, nullptr, P);
            hipLaunchKernelGGL((k_ls_finish<true, false>), nsys, blk, 0, st, B, gv, S, P, v.x, 0.0, 0, form, iters,
                               status);
        } else {
            hipLaunchKernelGGL((k_ls_update<false>), grid, blk, 0, st, B, gv, S, v);
            hipLaunchKernelGGL((k_ls_spmv<false, 0>), grid, blk, 0, st, B, gv, S, v, nullptr, P);
            hipLaunchKernelGGL((k_ls_finish<false, false>), nsys, blk, 0, st, B, gv, S, P, v.x, 0.0, 0, form, iters,
                               status);
        }
    }
    hipLaunchKernelGGL(k_ls_count, dim3(1), blk, 0, st, S, B.nsys, active);
    return hipGetLastError();
}

}  // namespace prcg
