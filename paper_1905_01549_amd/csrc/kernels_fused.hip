// Fused iterations on the SELL-64 layout: one kernel per iteration of PR-CG
// and of pipe-PR-CG, two per iteration of HS-CG.
//
// The sparse product of an iteration needs the iteration's new direction
// (PR: p_k; pipe-PR: s~_k and r~_k; HS: p_k) at neighbouring rows, which other
// workgroups produce in the same kernel.  Instead of a kernel boundary, each
// row recomputes those neighbour entries from the previous iteration's
// vectors with exactly the owner's expression (same operations, same
// order, so the same bits), and the vectors involved are double-buffered:
// iteration k reads copy k mod 2 and writes copy (k+1) mod 2, so no row ever
// reads an entry another row is overwriting.  Vectors read only at the own
// row (x always; p, r, s where no neighbour needs them) are updated in place.
//
// Every kernel starts with stage 2 of the previous reduction (every
// workgroup sums the partials in the same fixed order) and the scalar step;
// the partial buffers are double-buffered as well.
#include <hip/hip_ext.h>

#include "prcg_device.h"
#include "prcg_fused.h"

namespace prcg {

namespace {

__device__ __forceinline__ bool writer() { return blockIdx.x == 0 && threadIdx.x == 0; }

// Start of a one-reduction kernel: stage 2 + scalar step; false if done.
template <bool PRE, int M>
__device__ __forceinline__ bool enter_one_reduction(const Split& sp, const State* __restrict__ in,
                                                    State* __restrict__ out, double* __restrict__ hist,
                                                    const double* __restrict__ Pin, int form, State& st,
                                                    double (&lds)[M])
{
    st = load_state(in);
    if (st.done) {
        if (writer()) store_state(out, st);
        return false;
    }
    double t[5];
    reduce_partials<5>(Pin, sp.G, sp.Gs, t, lds);
    step_one_reduction(st, t, PRE, form, hist, writer());
    if (writer()) store_state(out, st);
    return !st.done;
}

// Offset-aligned or packed slot j of a SELL row: column and value.
struct SlotIter {
    const int32_t* off;   // aligned: slice offsets, else nullptr
    const int32_t* col;   // packed: column of the first slot of this lane
    const double* val;
    int row, last;
    int stride;  // elements between consecutive slots of a row
};

__device__ __forceinline__ SlotIter slots_of(const SellView& A, int64_t slice, int lane, int64_t row, int& width)
{
    const int64_t base = A.slice_ptr[slice];
    const int32_t shape = A.slice_shape[slice];
    width = shape_width(shape);
    const int meta = A.slice_meta[slice];
    SlotIter it;
    it.stride = shape_stride(shape);
    it.off = meta >= 0 ? A.soff + meta : nullptr;
    it.col = A.col + base + lane;
    it.val = A.val + base + lane;
    it.row = (int)row;
    it.last = (int)A.n - 1;
    return it;
}

// Calls f(c, a) for the slots of a SELL-64 row in stored order, with the
// slot's column c and value a.  Aligned and packed slices take separate
// code (one uniform branch per slice), and the slots go in pieces of
// kFusedPiece whose columns (an aligned piece's offsets in one scalar load)
// and values are loaded before the first call, so the gathers of a piece are
// in flight together.
constexpr int kFusedPiece = 4;

// UNIT: every slice is stored singly (slot stride 64, a constant the loads
// fold into their offsets), as in the matrices the fused structure is chosen
// for by default; the kernels are built both ways and the launcher picks
// (measured: a runtime stride made the fused PR-CG iteration of the
// 884,736-row problem 7% slower).
template <int K, bool ALIGNED, bool UNIT, class F>
__device__ __forceinline__ void fused_piece(const SlotIter& it, int j0, F&& f)
{
    const int64_t stride = UNIT ? kSlice : it.stride;
    int c[K];
    double a[K];
    if constexpr (ALIGNED) {
        int o[K];
#pragma unroll
        for (int u = 0; u < K; ++u) o[u] = it.off[j0 + u];
#pragma unroll
        for (int u = 0; u < K; ++u) c[u] = min(max(it.row + o[u], 0), it.last);
    } else {
#pragma unroll
        for (int u = 0; u < K; ++u) c[u] = it.col[(j0 + u) * stride];
    }
#pragma unroll
    for (int u = 0; u < K; ++u) a[u] = it.val[(j0 + u) * stride];
#pragma unroll
    for (int u = 0; u < K; ++u) f(c[u], a[u]);
}

template <bool ALIGNED, bool UNIT, class F>
__device__ __forceinline__ void fused_slots_of(const SlotIter& it, int width, F&& f)
{
    int j0 = 0;
    for (; j0 + kFusedPiece <= width; j0 += kFusedPiece) fused_piece<kFusedPiece, ALIGNED, UNIT>(it, j0, f);
    switch (width - j0) {
    case 1: fused_piece<1, ALIGNED, UNIT>(it, j0, f); break;
    case 2: fused_piece<2, ALIGNED, UNIT>(it, j0, f); break;
    case 3: fused_piece<3, ALIGNED, UNIT>(it, j0, f); break;
    default: break;
    }
}

template <bool UNIT, class F>
__device__ __forceinline__ void fused_slots(const SlotIter& it, int width, F&& f)
{
    if (it.off)
        fused_slots_of<true, UNIT>(it, width, f);
    else
        fused_slots_of<false, UNIT>(it, width, f);
}

// PR-CG, one kernel per iteration (Alg. 2):
//   x += alpha p; r -= alpha s; r~ -= alpha s~ (s~ = d s); p' = r~ + beta p;
//   s' = A p' with p' at neighbour j recomputed from p, s, r~ (and d);
//   partials of mu, sigma, gamma, nu (+ <r, r>) for the next kernel.
// Double-buffered: p, s, r~ (r~ is r without a preconditioner).
template <bool PRE, bool UNIT>
__global__ __launch_bounds__(kBlock) void k_pr_fused(SellView S, Split sp, const State* __restrict__ in,
                                                     State* __restrict__ out, double* __restrict__ hist,
                                                     const double* __restrict__ Pin, double* __restrict__ Pout,
                                                     int form, FusedVecs f, int q)
{
    __shared__ double lds[kWaves * 5];
    State st;
    if (!enter_one_reduction<PRE>(sp, in, out, hist, Pin, form, st, lds)) return;
    const double alpha = st.alpha, beta = st.beta;
    const double* __restrict__ p_o = f.p[q];
    double* __restrict__ p_n = f.p[1 - q];
    const double* __restrict__ s_o = f.s[q];
    double* __restrict__ s_n = f.s[1 - q];
    const double* __restrict__ t_o = PRE ? f.rt[q] : f.r[q];   // r~ (old)
    double* __restrict__ t_n = PRE ? f.rt[1 - q] : f.r[1 - q];  // r~ (new)
    double* __restrict__ r = f.r[0];                            // r in place (with a preconditioner)
    double* __restrict__ x = f.x;
    const double* __restrict__ d = f.d;
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int w = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (int64_t g = g0; g < g1; ++g) {
        const int64_t slice = g * kWaves + w;
        if (slice >= S.nslices) break;
        const int64_t i = slice * kSlice + lane;
        const bool own = i < S.n;
        // own row: the vector updates
        double pn = 0.0, rn = 0.0, tn = 0.0, di = 0.0;
        if (own) {
            const double pi = p_o[i], si = s_o[i], ti = t_o[i], xi = x[i];
            const double ri = PRE ? r[i] : ti;
            di = PRE ? d[i] : 1.0;
            rn = fma(-alpha, si, ri);
            tn = PRE ? fma(-alpha, di * si, ti) : rn;
            pn = fma(beta, pi, tn);
            x[i] = fma(alpha, pi, xi);
            if (PRE) {
                r[i] = rn;
                t_n[i] = tn;
            } else {
                t_n[i] = rn;
            }
            p_n[i] = pn;
        }
        // s' = A p', p' at neighbours from the previous vectors
        int width;
        const SlotIter it = slots_of(S, slice, lane, i, width);
        double sn = 0.0;
        fused_slots<UNIT>(it, width, [&](int c, double a) {
            const double sc = s_o[c];
            const double tc = t_o[c];
            const double pc = p_o[c];
            const double dc = PRE ? d[c] : 1.0;
            const double tnc = PRE ? fma(-alpha, dc * sc, tc) : fma(-alpha, sc, tc);
            sn = fma(a, fma(beta, pc, tnc), sn);
        });
        if (own) {
            s_n[i] = sn;
            const double stn = PRE ? di * sn : sn;
            acc[0] = fma(pn, sn, acc[0]);   // mu    = <p, s>
            acc[1] = fma(tn, sn, acc[1]);   // sigma = <r~, s>
            acc[2] = fma(stn, sn, acc[2]);  // gamma = <s~, s>
            acc[3] = fma(tn, rn, acc[3]);   // nu    = <r~, r>
            if (PRE) acc[4] = fma(rn, rn, acc[4]);
        }
    }
    write_partials<5>(acc, Pout, sp.Gs, blockIdx.x, lds);
}

// pipe-PR-CG, one kernel per iteration (Alg. 3): all vector updates of the
// own row, the inner products, then u' = A s~' and w' = A r~' with s~' and
// r~' at neighbour j recomputed from r~, s~, w, u (and d).  Double-buffered:
// r~, s~, w, u (r~ = r and s~ = s without a preconditioner).
template <bool PRE, bool UNIT>
__global__ __launch_bounds__(kBlock) void k_pipe_fused(SellView S, Split sp, const State* __restrict__ in,
                                                       State* __restrict__ out, double* __restrict__ hist,
                                                       const double* __restrict__ Pin, double* __restrict__ Pout,
                                                       int form, FusedVecs f, int q)
{
    __shared__ double lds[kWaves * 5];
    State st;
    if (!enter_one_reduction<PRE>(sp, in, out, hist, Pin, form, st, lds)) return;
    const double alpha = st.alpha, beta = st.beta;
    const double* __restrict__ t_o = PRE ? f.rt[q] : f.r[q];
    double* __restrict__ t_n = PRE ? f.rt[1 - q] : f.r[1 - q];
    const double* __restrict__ z_o = PRE ? f.st[q] : f.s[q];    // s~ (old)
    double* __restrict__ z_n = PRE ? f.st[1 - q] : f.s[1 - q];
    const double* __restrict__ w_o = f.w[q];
    double* __restrict__ w_n = f.w[1 - q];
    const double* __restrict__ u_o = f.u[q];
    double* __restrict__ u_n = f.u[1 - q];
    double* __restrict__ r = f.r[0];
    double* __restrict__ s = f.s[0];
    double* __restrict__ p = f.p[0];
    double* __restrict__ x = f.x;
    const double* __restrict__ d = f.d;
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int w = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (int64_t g = g0; g < g1; ++g) {
        const int64_t slice = g * kWaves + w;
        if (slice >= S.nslices) break;
        const int64_t i = slice * kSlice + lane;
        const bool own = i < S.n;
        if (own) {
            const double pi = p[i], xi = x[i], wi = w_o[i], ui = u_o[i], ti = t_o[i], zi = z_o[i];
            const double si = PRE ? s[i] : zi;
            const double ri = PRE ? r[i] : ti;
            const double rn = fma(-alpha, si, ri);                 // r_k
            const double sn = fma(beta, si, fma(-alpha, ui, wi));  // s_k = w'_k + beta s_{k-1}
            double tn = rn, zn = sn;
            if (PRE) {
                const double di = d[i];
                tn = fma(-alpha, zi, ti);                                // r~_k
                zn = fma(beta, zi, fma(-alpha, di * ui, di * wi));       // s~_k
            }
            const double pn = fma(beta, pi, tn);                   // p_k
            x[i] = fma(alpha, pi, xi);
            p[i] = pn;
            if (PRE) {
                r[i] = rn;
                s[i] = sn;
            }
            t_n[i] = tn;
            z_n[i] = zn;
            acc[0] = fma(pn, sn, acc[0]);
            acc[1] = fma(tn, sn, acc[1]);
            acc[2] = fma(zn, sn, acc[2]);
            acc[3] = fma(tn, rn, acc[3]);
            if (PRE) acc[4] = fma(rn, rn, acc[4]);
        }
        int width;
        const SlotIter it = slots_of(S, slice, lane, i, width);
        double un = 0.0, wn = 0.0;
        fused_slots<UNIT>(it, width, [&](int c, double a) {
            const double tc = t_o[c], zc = z_o[c], wc = w_o[c], uc = u_o[c];
            double tnc, znc;
            if (PRE) {
                const double dc = d[c];
                tnc = fma(-alpha, zc, tc);
                znc = fma(beta, zc, fma(-alpha, dc * uc, dc * wc));
            } else {
                tnc = fma(-alpha, zc, tc);
                znc = fma(beta, zc, fma(-alpha, uc, wc));
            }
            un = fma(a, znc, un);
            wn = fma(a, tnc, wn);
        });
        if (own) {
            u_n[i] = un;
            w_n[i] = wn;
        }
    }
    write_partials<5>(acc, Pout, sp.Gs, blockIdx.x, lds);
}

// HS-CG, second kernel of an iteration: stage 2 of nu (beta, tests), then
// s = A p' with p' = r~ + beta p at neighbours from r (final in this kernel)
// and the previous p; writes p' (double-buffered) and s; partials of mu.
template <bool PRE, bool UNIT>
__global__ __launch_bounds__(kBlock) void k_hs_fused(SellView S, Split sp, const State* __restrict__ in,
                                                     State* __restrict__ out, double* __restrict__ hist,
                                                     const double* __restrict__ PU, double* __restrict__ PS,
                                                     FusedVecs f, int q)
{
    __shared__ double lds[kWaves * 2];
    State st = load_state(in);
    if (st.done) {
        if (writer()) store_state(out, st);
        return;
    }
    double t[2];
    reduce_partials<2>(PU, sp.G, sp.Gs, t, lds);
    step_hs_nu(st, t[0], PRE ? t[1] : t[0], hist, writer());
    if (writer()) store_state(out, st);
    if (st.done) return;
    const double beta = st.beta;
    const double* __restrict__ p_o = f.p[q];
    double* __restrict__ p_n = f.p[1 - q];
    const double* __restrict__ r = f.r[0];
    double* __restrict__ s = f.s[0];
    const double* __restrict__ d = f.d;
    int64_t g0, g1;
    chunk_of(blockIdx.x, sp.G, sp.ngroups, g0, g1);
    double acc[1] = {0.0};
    const int w = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (int64_t g = g0; g < g1; ++g) {
        const int64_t slice = g * kWaves + w;
        if (slice >= S.nslices) break;
        const int64_t i = slice * kSlice + lane;
        const bool own = i < S.n;
        double pn = 0.0;
        if (own) {
            const double ri = r[i];
            pn = fma(beta, p_o[i], PRE ? d[i] * ri : ri);
            p_n[i] = pn;
        }
        int width;
        const SlotIter it = slots_of(S, slice, lane, i, width);
        double sn = 0.0;
        fused_slots<UNIT>(it, width, [&](int c, double a) {
            const double rc = r[c];
            sn = fma(a, fma(beta, p_o[c], PRE ? d[c] * rc : rc), sn);
        });
        if (own) {
            s[i] = sn;
            acc[0] = fma(pn, sn, acc[0]);
        }
    }
    write_partials<1>(acc, PS, sp.Gs, blockIdx.x, lds);
}

}  // namespace

hipError_t launch_fused_kernel(int variant, int pre, int j, int it, int& cur, const SellView& S, const Split& sp,
                               const FusedVecs& f, const Bufs& B, double* PS2, hipStream_t st,
                               const LaunchEvents* ev)
{
    const dim3 grid(sp.G), block(kBlock);
    const int q = it & 1;
    const int nxt = 1 - cur;
    const int form = nu_form(variant);
    double* Pq[2] = {B.PS, PS2};
    auto go = [&](auto kernel, auto... args) {
        if (ev && ev->start)
            hipExtLaunchKernelGGL(kernel, grid, block, 0, st, ev->start, ev->stop, 0, args...);
        else
            hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
        return hipGetLastError();
    };
    hipError_t e = hipSuccess;
    const bool unit = S.runs == 0;
    auto pick = [&](auto P, auto U) -> hipError_t {
        constexpr bool PR = decltype(P)::value, UN = decltype(U)::value;
        if (is_pr_family(variant))
            return go(k_pr_fused<PR, UN>, S, sp, (const State*)B.S[cur], B.S[nxt], B.hist, (const double*)Pq[q],
                      Pq[1 - q], form, f, q);
        if (variant == kPipePR || variant == kPipeM)
            return go(k_pipe_fused<PR, UN>, S, sp, (const State*)B.S[cur], B.S[nxt], B.hist, (const double*)Pq[q],
                      Pq[1 - q], form, f, q);
        // HS: the first kernel is the two-pass k_hs_xr on the current buffers
        return go(k_hs_fused<PR, UN>, S, sp, (const State*)B.S[cur], B.S[nxt], B.hist, (const double*)B.PU, B.PS,
                  f, q);
    };
    if (!is_pr_family(variant) && variant != kPipePR && variant != kPipeM && j == 0) return hipErrorInvalidValue;
    using T = std::true_type;
    using F = std::false_type;
    e = pre ? (unit ? pick(T{}, T{}) : pick(T{}, F{})) : (unit ? pick(F{}, T{}) : pick(F{}, F{}));
    cur = nxt;
    return e;
}

}  // namespace prcg
