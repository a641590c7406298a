// Textbook HS-CG: one kernel per line of Alg. 1, the way the iteration is
// written with separate BLAS-1 and sparse-product calls.  This is the
// unfused baseline ("plain HS-CG"): every AXPY, the preconditioner, every
// inner product and the product are kernels of their own, and each
// reduction ends in a one-workgroup kernel.  Scalars stay on the device.
#include <hip/hip_ext.h>

#include "prcg_device.h"
#include "prcg_textbook.h"

namespace prcg {

namespace {

template <class F>
__device__ __forceinline__ void for_rows(const Split& sp, F&& f)
{
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    const int64_t i1 = g1 * kGroupRows < sp.n ? g1 * kGroupRows : sp.n;
    for (int64_t i = g0 * kGroupRows + threadIdx.x; i < i1; i += kBlock) f(i);
}

// y += sign * alpha * x
__global__ __launch_bounds__(kBlock) void k_tb_axpy(Split sp, const State* __restrict__ st, double sign,
                                                    const double* __restrict__ x, double* __restrict__ y)
{
    if (st->done) return;
    const double a = sign * st->alpha;
    for_rows(sp, [&](int64_t i) { y[i] = fma(a, x[i], y[i]); });
}

// y = x + beta * y
__global__ __launch_bounds__(kBlock) void k_tb_xpay(Split sp, const State* __restrict__ st,
                                                    const double* __restrict__ x, double* __restrict__ y)
{
    if (st->done) return;
    const double b = st->beta;
    for_rows(sp, [&](int64_t i) { y[i] = fma(b, y[i], x[i]); });
}

// y = M^{-1} x = d .* x
__global__ __launch_bounds__(kBlock) void k_tb_prec(Split sp, const State* __restrict__ st,
                                                    const double* __restrict__ d, const double* __restrict__ x,
                                                    double* __restrict__ y)
{
    if (st->done) return;
    for_rows(sp, [&](int64_t i) { y[i] = d[i] * x[i]; });
}

// partial sums of <a, b> into P[slot * Gs + workgroup]
__global__ __launch_bounds__(kBlock) void k_tb_dot(Split sp, const State* __restrict__ st,
                                                   const double* __restrict__ a, const double* __restrict__ b,
                                                   double* __restrict__ P, int slot)
{
    __shared__ double lds[kWaves];
    if (st->done) return;
    double acc[1] = {0.0};
    for_rows(sp, [&](int64_t i) { acc[0] = fma(a[i], b[i], acc[0]); });
    write_partials<1>(acc, P + (size_t)slot * sp.Gs, sp.Gs, blockIdx.x, lds);
}

// y = A x
template <int LANES>
__global__ __launch_bounds__(kBlock) void k_tb_spmv(SellView S, CsrView C, Split sp, const State* __restrict__ st,
                                                    const double* __restrict__ x, double* __restrict__ y)
{
    if (st->done) return;
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    for (int64_t g = g0; g < g1; ++g)
        rows_of_group<LANES, 1>(S, C, g, x, nullptr, [&](int64_t i, double yi, double) { y[i] = yi; });
}

// one workgroup: stage 2 of nu_k (and <r, r>), convergence test, beta_k
template <bool PRE>
__global__ __launch_bounds__(kStage2Block) void k_tb_nu(Split sp, const State* __restrict__ in, State* __restrict__ out,
                                                  double* __restrict__ hist, const double* __restrict__ PU)
{
    __shared__ double lds[kStage2Waves * 2];
    State st = load_state(in);
    double t[2];
    reduce_partials<2, true>(PU, sp.G, sp.Gs, t, lds);  // read whether or not the solve has ended
    if (!st.done) step_hs_nu(st, t[0], PRE ? t[1] : t[0], hist, threadIdx.x == 0);
    if (threadIdx.x == 0) store_state(out, st);
}

// one workgroup: stage 2 of mu_k, alpha_k
__global__ __launch_bounds__(kStage2Block) void k_tb_mu(Split sp, const State* __restrict__ in, State* __restrict__ out,
                                                  const double* __restrict__ PS)
{
    __shared__ double lds[kStage2Waves * 1];
    State st = load_state(in);
    double t[1];
    reduce_partials<1, true>(PS, sp.G, sp.Gs, t, lds);  // read whether or not the solve has ended
    if (!st.done) step_hs_mu(st, t[0]);
    if (threadIdx.x == 0) store_state(out, st);
}

template <class K, class... Args>
hipError_t go(K kernel, dim3 grid, hipStream_t st, const LaunchEvents* ev, Args... args)
{
    if (ev && ev->start)
        hipExtLaunchKernelGGL(kernel, grid, dim3(kBlock), 0, st, ev->start, ev->stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, dim3(kBlock), 0, st, args...);
    return hipGetLastError();
}

// one-workgroup reduction kernels (kStage2Block threads)
template <class K, class... Args>
hipError_t go1(K kernel, hipStream_t st, const LaunchEvents* ev, Args... args)
{
    if (ev && ev->start)
        hipExtLaunchKernelGGL(kernel, dim3(1), dim3(kStage2Block), 0, st, ev->start, ev->stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, dim3(1), dim3(kStage2Block), 0, st, args...);
    return hipGetLastError();
}

const char* kNames[] = {"k_tb_mu", "k_tb_axpy_x", "k_tb_axpy_r", "k_tb_prec", "k_tb_dot_nu",
                        "k_tb_dot_rr", "k_tb_nu", "k_tb_xpay_p", "k_tb_spmv", "k_tb_dot_mu"};

}  // namespace

int textbook_kernel_count(int pre) { return pre ? 10 : 8; }

const char* textbook_kernel_name(int pre, int j)
{
    // without a preconditioner the prec and <r, r> kernels are skipped
    static const int map_none[] = {0, 1, 2, 4, 6, 7, 8, 9};
    return kNames[pre ? j : map_none[j]];
}

hipError_t launch_textbook_kernel(int pre, int j, int& cur, const SellView* sell, const CsrView* csr,
                                  const Split& sp, const Vecs& v, const Bufs& B, hipStream_t st,
                                  const LaunchEvents* ev)
{
    static const int map_none[] = {0, 1, 2, 4, 6, 7, 8, 9};
    const int k = pre ? j : map_none[j];
    const dim3 grid(sp.G);
    const int nxt = 1 - cur;
    const State* S = B.S[cur];
    double* rt = pre ? v.rt : v.r;
    const SellView SV = sell ? *sell : SellView{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0};
    const CsrView CV = csr ? *csr : CsrView{nullptr, nullptr, nullptr, 0};
    hipError_t e = hipSuccess;
    switch (k) {
    case 0:  // alpha_{k-1} = nu_{k-1} / mu_{k-1}
        e = go1(k_tb_mu, st, ev, sp, S, B.S[nxt], (const double*)B.PS);
        cur = nxt;
        break;
    case 1: e = go(k_tb_axpy, grid, st, ev, sp, S, 1.0, (const double*)v.p, v.x); break;   // x += alpha p
    case 2: e = go(k_tb_axpy, grid, st, ev, sp, S, -1.0, (const double*)v.s, v.r); break;  // r -= alpha s
    case 3: e = go(k_tb_prec, grid, st, ev, sp, S, v.d, (const double*)v.r, v.rt); break;  // r~ = M^-1 r
    case 4: e = go(k_tb_dot, grid, st, ev, sp, S, (const double*)rt, (const double*)v.r, B.PU, 0); break;
    case 5: e = go(k_tb_dot, grid, st, ev, sp, S, (const double*)v.r, (const double*)v.r, B.PU, 1); break;
    case 6:  // nu_k, tests, beta_k
        e = pre ? go1(k_tb_nu<true>, st, ev, sp, S, B.S[nxt], B.hist, (const double*)B.PU)
                : go1(k_tb_nu<false>, st, ev, sp, S, B.S[nxt], B.hist, (const double*)B.PU);
        cur = nxt;
        break;
    case 7: e = go(k_tb_xpay, grid, st, ev, sp, S, (const double*)rt, v.p); break;  // p = r~ + beta p
    case 8:                                                                        // s = A p
        switch (sp.lanes) {
        case 1: e = go(k_tb_spmv<1>, grid, st, ev, SV, CV, sp, S, (const double*)v.p, v.s); break;
        case 8: e = go(k_tb_spmv<8>, grid, st, ev, SV, CV, sp, S, (const double*)v.p, v.s); break;
        case 16: e = go(k_tb_spmv<16>, grid, st, ev, SV, CV, sp, S, (const double*)v.p, v.s); break;
        case 32: e = go(k_tb_spmv<32>, grid, st, ev, SV, CV, sp, S, (const double*)v.p, v.s); break;
        default: e = go(k_tb_spmv<64>, grid, st, ev, SV, CV, sp, S, (const double*)v.p, v.s); break;
        }
        break;
    default: e = go(k_tb_dot, grid, st, ev, sp, S, (const double*)v.p, (const double*)v.s, B.PS, 0); break;
    }
    return e;
}

}  // namespace prcg
