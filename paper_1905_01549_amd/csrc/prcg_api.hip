// libprcg host runtime: the C ABI of include/prcg.h.
//
// A matrix handle owns device copies of the CSR arrays, the SpMV layout
// (SELL-64 for short rows, vector CSR for long ones), the Jacobi diagonal,
// the solver vectors, the partial-sum buffers, two copies of the scalar
// state and one instantiated HIP graph per variant.  A graph holds K
// iterations of the variant's kernels; a solve runs the initialisation,
// replays the graph until the device-side state says the solve ended (every
// kernel returns at once after that), then computes the true residual.  The
// host reads the state once per replay, overlapped with the next replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/prcg.h"
#include "batched.h"
#include "prcg_common.h"
#include "prcg_fused.h"
#include "prcg_textbook.h"

using namespace prcg;

namespace {

thread_local std::string g_last_error;

prcg_status fail(prcg_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? PRCG_ENOMEM : PRCG_EDEVICE,                    \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                        \
    } while (0)

constexpr int kGraphIters = 16;  // iterations per graph replay (even: the state copy returns to 0)

bool is_device_pointer(const void* p)
{
    if (!p) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// Words of the partial-sum buffers: PS | PU | PB | PS2 | PN | PD | PW, each
// reduction value a row of kMaxGrid doubles.
constexpr int64_t kPartialWords = (int64_t)(2 * kMaxDots + 7) * kMaxGrid;

// The reduction buffers of a solve laid out over `partials` (kPartialWords
// doubles), two state copies, the residual history and the ticket counter.
Bufs bufs_at(double* partials, State* S, double* hist, int* ticket)
{
    Bufs B;
    B.S[0] = S;
    B.S[1] = S + 1;
    B.hist = hist;
    B.PS = partials;
    B.PU = partials + (size_t)kMaxDots * kMaxGrid;
    B.PB = partials + (size_t)(kMaxDots + 2) * kMaxGrid;
    B.PS2 = partials + (size_t)(kMaxDots + 3) * kMaxGrid;
    B.PN = partials + (size_t)(2 * kMaxDots + 3) * kMaxGrid;
    B.PD = partials + (size_t)(2 * kMaxDots + 5) * kMaxGrid;
    B.PW = partials + (size_t)(2 * kMaxDots + 6) * kMaxGrid;
    B.ticket = ticket;
    return B;
}

// Offset-aligned slices whose column-offset lists are equal are pointed at
// one copy of the list (meta[q] rewritten; the other copies stay unused), so
// that the products' scalar loads of the offsets hit the scalar cache
// instead of missing once per slice.
void share_offsets(const std::vector<int32_t>& soff, const std::vector<int32_t>& width, std::vector<int32_t>& meta)
{
    std::map<std::vector<int32_t>, int32_t> first;
    for (size_t q = 0; q < meta.size(); ++q) {
        if (meta[q] < 0) continue;
        std::vector<int32_t> key(soff.begin() + meta[q], soff.begin() + meta[q] + width[q]);
        auto it = first.emplace(std::move(key), meta[q]).first;
        meta[q] = it->second;
    }
}

}  // namespace

struct prcg_matrix_s {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;
    int64_t n = 0, nnz = 0;
    int precond = 0;
    // CSR copies (the adjoint's outer product and value updates use them)
    int32_t* row_ptr = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
    // SELL-64 layout (when lanes == 1)
    int64_t* slice_ptr = nullptr;
    int32_t* slice_meta = nullptr;
    int32_t* slice_shape = nullptr;
    int32_t* soff = nullptr;
    int32_t* scol = nullptr;
    double* sval = nullptr;
    int64_t nslices = 0;
    int64_t stream_from = INT64_MAX;  // first slice past the cacheable values (cached_value_bytes)
    int32_t runs = 0;            // 1 when some slice is stored in a run of more than one
    int64_t stored = 0;          // value slots, padding included
    int64_t stored_packed = 0;   // slots of packed slices (they also read a column index)
    int64_t stored_streamed = 0; // slots read with nontemporal loads
    int64_t noffsets = 0;        // offsets of aligned slices
    double* d = nullptr;
    Split sp{};
    // solver workspace
    double* vecs = nullptr;  // x r rt p s st w u spare | second copies r rt p s st w u
    int kernels_mode = 0;    // PRCG_KERNELS_*
    double2* pairs = nullptr;  // pipe-PR block vectors: (s~, r~) then (u, w)
    int grid_opt = 0;        // largest workgroup count (0: chosen by size)
    State* S = nullptr;      // two copies
    double* hist = nullptr;
    int64_t hist_cap = 0;
    double* partials = nullptr;  // PS | PU | PB | PS2 | PN | PD | PW
    int32_t* dflags = nullptr;   // [0..3] setup flags, [4] reduction ticket
    State* hstate = nullptr;     // pinned, two slots
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipGraphExec_t graph[kNumVariants] = {};

    SellView sell() const
    {
        SellView s{slice_ptr, slice_meta, slice_shape, soff, scol, sval, n, nslices};
        s.stream_from = stream_from;
        s.runs = runs;
        return s;
    }
    CsrView csr() const { return CsrView{row_ptr, col, val, n}; }
    const SellView* sellp() const { return sp.lanes == 1 ? &sell_storage : nullptr; }
    const CsrView* csrp() const { return sp.lanes == 1 ? nullptr : &csr_storage; }
    SellView sell_storage{};
    CsrView csr_storage{};

    Vecs vecs_view() const
    {
        const size_t n8 = (size_t)n;
        Vecs v;
        v.x = vecs + 0 * n8;
        v.r = vecs + 1 * n8;
        v.rt = vecs + 2 * n8;
        v.p = vecs + 3 * n8;
        v.s = vecs + 4 * n8;
        v.st = vecs + 5 * n8;
        v.w = vecs + 6 * n8;
        v.u = vecs + 7 * n8;
        v.d = d;
        v.zr = pairs;
        v.uw = pairs + n8;
        // GV-CG uses two of the fused structure's second copies
        v.t = vecs + 9 * n8;
        v.wt = vecs + 10 * n8;
        return v;
    }
    double* spare() const { return vecs + 8 * (size_t)n; }

    FusedVecs fused_view() const
    {
        const size_t n8 = (size_t)n;
        FusedVecs f;
        f.x = vecs;
        double** two[] = {f.r, f.rt, f.p, f.s, f.st, f.w, f.u};
        for (int q = 0; q < 7; ++q) {
            two[q][0] = vecs + (size_t)(1 + q) * n8;
            two[q][1] = vecs + (size_t)(9 + q) * n8;
        }
        f.d = d;
        return f;
    }

    Bufs bufs() const { return bufs_at(partials, S, hist, dflags + 4); }
};

struct prcg_batch_s {
    prcg_matrix A = nullptr;
    int32_t nsys = 0;
    int64_t nslices = 0;
    int64_t stored = 0;
    int64_t stored_packed = 0;  // slots of packed slices (they also read a column index)
    int64_t noffsets = 0;       // offsets of aligned slices
    int num_cus = 256;
    int64_t* slice_row0 = nullptr;
    int32_t* slice_nrows = nullptr;
    int64_t* sys_row0 = nullptr;
    int64_t* sys_slice0 = nullptr;
    int32_t* order = nullptr;
    int64_t* slice_ptr = nullptr;
    int32_t* slice_meta = nullptr;
    int32_t* slice_shape = nullptr;
    int32_t* soff = nullptr;
    int32_t* scol = nullptr;
    double* sval = nullptr;
    double* vecs = nullptr;  // x r rt p s st w u b
    int32_t* queue = nullptr;
    int32_t* iters = nullptr;
    int32_t* status = nullptr;
    // persistent launch per kind (HS, PR/M, pipe): threads per workgroup,
    // workgroups, slices multiplied together per wavefront (0: not tuned)
    int tuned_nt[3] = {0, 0, 0};
    int tuned_grid[3] = {0, 0, 0};
    int tuned_q[3] = {0, 0, 0};
    // configuration fixed by prcg_batch_set_config (0: autotuned)
    int force_nt = 0, force_per_cu = 0, force_q = 0, force_group = 0;
    int force_fusion = PRCG_BATCH_FUSION_AUTO;
    hipGraphExec_t graph[kNumVariants] = {};
    double graph_tol[kNumVariants] = {};
    int32_t graph_maxit[kNumVariants] = {};
    int64_t stream_from = INT64_MAX;  // first slice past the cacheable values (cached_value_bytes)
    // lockstep solver (PR-CG, M-CG): row groups of 8, 16 and 32 slices
    // (tables 0, 1, 2: 2, 4, 8 slices per wavefront), per-system states,
    // partials
    struct GroupTable {
        int64_t ngroups = 0;
        int64_t uniform_groups = 0;
        Group* grp = nullptr;
        int64_t* sys_grp0 = nullptr;
        int32_t* gdone = nullptr;
        int32_t spw = 0;
        int32_t uwidth = 0;  // every group uniform: 3, 5 or 7 slots, the least at or above the widest; else 0
        bool fuse_ok = false;  // iterations may run fused (launch_lockstep_iterations)
        int32_t span = 0;      // the largest stencil span of a uniform group
    };
    static constexpr int kTables = 3;
    GroupTable tab[kTables];
    int ls_table = -1;         // table in use (-1: not tuned yet)
    bool ls_fused = false;     // its iterations run fused
    State* lstate = nullptr;
    double* lpart = nullptr;   // 6 * the largest table's ngroups
    int32_t* lactive = nullptr;
    int32_t* lticket = nullptr;  // [nsys]: stage-2 tickets of the fused lockstep iteration
    int32_t* hactive = nullptr;  // pinned, two slots
    hipEvent_t lev[2] = {nullptr, nullptr};
    hipGraphExec_t ls_graph[kNumVariants] = {};
    int32_t mode_req = PRCG_BATCH_AUTO;
    int32_t mode[3] = {0, 0, 0};  // per kind: 0 undecided, else PRCG_BATCH_PERSISTENT / _LOCKSTEP

    GroupView groups(int t) const
    {
        return GroupView{tab[t].grp, tab[t].sys_grp0, tab[t].ngroups, tab[t].gdone, tab[t].spw, tab[t].uwidth,
                         lticket, tab[t].span};
    }

    Vecs vecs_view() const
    {
        const size_t n8 = (size_t)A->n;
        Vecs v;
        v.x = vecs;
        v.r = vecs + n8;
        v.rt = vecs + 2 * n8;
        v.p = vecs + 3 * n8;
        v.s = vecs + 4 * n8;
        v.st = vecs + 5 * n8;
        v.w = vecs + 6 * n8;
        v.u = vecs + 7 * n8;
        v.d = A->d;
        v.zr = nullptr;
        v.uw = nullptr;
        v.t = nullptr;
        v.wt = nullptr;
        return v;
    }
    BatchView view() const
    {
        BatchView b;
        b.A = SellView{slice_ptr, slice_meta, slice_shape, soff, scol, sval, A->n, nslices};
        b.A.stream_from = stream_from;
        b.slice_row0 = slice_row0;
        b.slice_nrows = slice_nrows;
        b.sys_row0 = sys_row0;
        b.sys_slice0 = sys_slice0;
        b.order = order;
        b.nsys = nsys;
        return b;
    }
};

namespace {

void free_batch(prcg_batch B)
{
    if (!B) return;
    (void)hipSetDevice(B->A->device);
    for (auto& g : B->graph)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto& g : B->ls_graph)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto& e : B->lev)
        if (e) (void)hipEventDestroy(e);
    if (B->hactive) (void)hipHostFree(B->hactive);
    void* dev[] = {B->slice_row0, B->slice_nrows, B->sys_row0, B->sys_slice0, B->order, B->slice_ptr,
                   B->slice_meta, B->slice_shape, B->soff, B->scol, B->sval, B->vecs, B->queue, B->iters, B->status,
                   B->lstate, B->lpart, B->lactive, B->lticket};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    for (auto& t : B->tab) {
        void* td[] = {t.grp, t.sys_grp0, t.gdone};
        for (void* p : td)
            if (p) (void)hipFree(p);
    }
    delete B;
}

void free_matrix(prcg_matrix A)
{
    if (!A) return;
    (void)hipSetDevice(A->device);
    for (auto& g : A->graph)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto& e : A->ev)
        if (e) (void)hipEventDestroy(e);
    void* dev[] = {A->row_ptr, A->col, A->val, A->slice_ptr, A->slice_meta, A->slice_shape, A->soff, A->scol, A->sval, A->d,
                   A->vecs, A->pairs, A->S, A->hist, A->partials, A->dflags};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    if (A->hstate) (void)hipHostFree(A->hstate);
    if (A->capture) (void)hipStreamDestroy(A->capture);
    delete A;
}

void invalidate_graphs(prcg_matrix A)
{
    for (auto& g : A->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

// Choose the work split: G workgroups (multiple of 8 when G >= 8, so every
// XCD gets the same number), at most gmax_opt (PRCG_OPT_GRID), or by size
// when gmax_opt is 0 (the default): from kBigGroups 256-row groups up, one
// group per workgroup (at most kMaxGrid workgroups), below that at most 1024
// workgroups.  Measured on MI355X: at 128^3 8192 workgroups run PR-CG 1.7%
// and HS-CG 2% faster per iteration than 4096 (1536 and 2048 are slower);
// at 160^3 (27-point) 8192 are 2-4% faster than 4096; problems of 1-4k
// groups run best at 1024.
constexpr int64_t kBigGroups = 8192;
//
// Stage-2 placement of the default two-pass structure.  The redundant form
// costs every workgroup of the consuming kernel a read of all partials
// (G^2 reads of the same few cache lines per reduction); a one-workgroup
// kernel costs one launch and one memory round trip (4-5 us on MI355X).
// Measured: at 1024 workgroups the redundant form is 1-4 us per reduction
// faster than the separate kernel, at 4096 it is 8-22 us slower.  HS-CG and
// PR-CG therefore take the separate kernel from kStage2MinGrid workgroups
// up.  pipe-PR-CG reduces in one workgroup of its product kernel before
// that workgroup's share of the product, which hides the reduction.
// AUTO also picks the fused structure (SELL-64 only) below kStage2MinGrid:
// at 1024 workgroups it is the fastest for HS-CG and PR-CG on the 262k-,
// 885k- and 1M-row problems (PR-CG 15.1 / 28.5 / 18.3 us per iteration
// against 19.1 / 29.8 / 24.1 two-pass), at 4096 it is 1.5x slower.
constexpr int kStage2MinGrid = 2048;
constexpr int kPipeFusedMaxGrid = 64;
Split make_split(int64_t n, int lanes, int gmax_opt, int kernels_mode)
{
    Split sp{};
    sp.n = n;
    sp.lanes = lanes;
    sp.ngroups = (n + kGroupRows - 1) / kGroupRows;
    int64_t gmax = gmax_opt > 0 ? std::min(kMaxGrid, std::max(8, gmax_opt))
                                : (sp.ngroups >= kBigGroups ? std::min<int64_t>(kMaxGrid, sp.ngroups) : 1024);
    int64_t G = std::min<int64_t>(sp.ngroups, gmax);
    if (G >= 8) G -= G % 8;
    sp.G = (int)std::max<int64_t>(G, 1);
    sp.Gs = (sp.G + 63) / 64 * 64;
    // AUTO: the fused structure for problems of fewer than kStage2MinGrid
    // workgroups, two-pass above
    const bool small = sp.G < kStage2MinGrid;
    // (pipe-PR-CG only below kPipeFusedMaxGrid: its two-pass product kernel
    // already hides the reduction, and its fused form gathers five vectors
    // per entry; 16.0 against 17.5 us per iteration at 1024 workgroups, but
    // 8.7 against 9.7 at 16)
    const bool tiny = sp.G < kPipeFusedMaxGrid;
    sp.fused = lanes != 1                                               ? 0
               : kernels_mode == PRCG_KERNELS_FUSED                     ? 3
               : kernels_mode == PRCG_KERNELS_AUTO && tiny              ? 3
               : kernels_mode == PRCG_KERNELS_AUTO && small             ? 1
                                                                         : 0;
    if (kernels_mode == PRCG_KERNELS_TWO_PASS_STAGE2) {
        sp.stage2 = 7;
    } else if (kernels_mode == PRCG_KERNELS_TWO_PASS || kernels_mode == PRCG_KERNELS_TEXTBOOK ||
               kernels_mode == PRCG_KERNELS_AUTO) {
        sp.stage2 = sp.G >= kStage2MinGrid ? 3 : 0;
    }
    sp.lastwg = kernels_mode == PRCG_KERNELS_TWO_PASS_LAST ? 1 : 0;
    sp.textbook = kernels_mode == PRCG_KERNELS_TEXTBOOK ? 1 : 0;
    return sp;
}

prcg_status read_flags(prcg_matrix A, int32_t* host_flags, int nflags)
{
    HIP_TRY(hipMemcpyAsync(host_flags, A->dflags, sizeof(int32_t) * nflags, hipMemcpyDeviceToHost, A->stream));
    HIP_TRY(hipStreamSynchronize(A->stream));
    return PRCG_OK;
}

prcg_status ensure_hist(prcg_matrix A, int64_t need)
{
    if (A->hist_cap >= need) return PRCG_OK;
    int64_t cap = std::max<int64_t>(need, 1024);
    if (A->hist) HIP_TRY(hipFree(A->hist));
    A->hist = nullptr;
    A->hist_cap = 0;
    HIP_TRY(hipMalloc(&A->hist, sizeof(double) * cap));
    A->hist_cap = cap;
    invalidate_graphs(A);  // the graphs hold the history pointer
    return PRCG_OK;
}

// Kernel j of the iteration at position `it` (its parity selects the buffer
// copies of the fused kernels).
hipError_t launch_iteration(prcg_matrix A, const Bufs& B, int variant, int j, int it, int& cur, hipStream_t st,
                            const LaunchEvents* ev = nullptr)
{
    if (A->sp.textbook && variant == kHS)
        return launch_textbook_kernel(A->precond, j, cur, A->sellp(), A->csrp(), A->sp, A->vecs_view(), B, st, ev);
    if (uses_fused(variant, A->sp)) {
        const FusedVecs f = A->fused_view();
        if (variant == kHS && j == 0) {
            Vecs v = A->vecs_view();
            v.p = f.p[it & 1];
            return launch_iter_kernel(variant, A->precond, 0, cur, A->sellp(), A->csrp(), A->sp, v, B, st, ev);
        }
        return launch_fused_kernel(variant, A->precond, j, it, cur, A->sell_storage, A->sp, f, B, B.PS2, st, ev);
    }
    return launch_iter_kernel(variant, A->precond, j, cur, A->sellp(), A->csrp(), A->sp, A->vecs_view(), B, st, ev);
}

prcg_status build_graph(prcg_matrix A, int variant)
{
    if (A->graph[variant]) return PRCG_OK;
    HIP_TRY(hipStreamBeginCapture(A->capture, hipStreamCaptureModeThreadLocal));
    int cur = 0;
    hipError_t err = hipSuccess;
    for (int it = 0; it < kGraphIters && err == hipSuccess; ++it)
        for (int j = 0; j < iter_kernel_count(variant, A->sp) && err == hipSuccess; ++j)
            err = launch_iteration(A, A->bufs(), variant, j, it, cur, A->capture);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(A->capture, &g);
    if (err != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(PRCG_EDEVICE, std::string("graph capture: ") + hipGetErrorString(err));
    }
    HIP_TRY(e2);
    if (cur != 0) {
        (void)hipGraphDestroy(g);
        return fail(PRCG_EDEVICE, "internal: state copy does not return to 0 after a replay");
    }
    hipError_t e3 = hipGraphInstantiate(&A->graph[variant], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(e3);
    return PRCG_OK;
}

// One chunk of kGraphIters iterations: a replay of the variant's graph, or
// (graph == nullptr) the same launches, in the same order, made one by one.
prcg_status launch_chunk(prcg_matrix A, const Bufs& B, int variant, hipGraphExec_t graph)
{
    if (graph) {
        HIP_TRY(hipGraphLaunch(graph, A->stream));
        return PRCG_OK;
    }
    int cur = 0;
    const int nk = iter_kernel_count(variant, A->sp);
    for (int it = 0; it < kGraphIters; ++it)
        for (int j = 0; j < nk; ++j) HIP_TRY(launch_iteration(A, B, variant, j, it, cur, A->stream));
    if (cur != 0) return fail(PRCG_EDEVICE, "internal: state copy does not return to 0 after a chunk");
    return PRCG_OK;
}

// A complete solve on the handle's stream with the reduction buffers B:
// the initialisation, chunks of kGraphIters iterations until the
// device-side state says the solve ended (the host reads the state once per
// chunk, overlapped with the next chunk), then the true residual.  x0
// (device) may be the spare zero vector; xout receives the result.
prcg_status solve_loop(prcg_matrix A, const Bufs& B, int variant, hipGraphExec_t graph, const double* b,
                       const double* x0, double* xout, double tol, int32_t maxit, State* final_state)
{
    const Vecs v = A->vecs_view();
    HIP_TRY(launch_init(variant, A->precond, A->sellp(), A->csrp(), A->sp, v, B, b, x0, tol, maxit, A->stream));
    // transitions needed <= maxit + 2; each chunk performs kGraphIters (HS: 2 per iteration)
    const int64_t max_chunks = ((int64_t)maxit + 2) / kGraphIters + 3;
    int64_t launched = 0;
    int pending = -1;  // slot whose copy is in flight
    bool done = false;
    while (!done) {
        if (launched > max_chunks)
            return fail(PRCG_EDEVICE, "internal: solve did not finish within the expected number of chunks");
        prcg_status s = launch_chunk(A, B, variant, graph);
        if (s != PRCG_OK) return s;
        const int slot = (int)(launched & 1);
        HIP_TRY(hipMemcpyAsync(&A->hstate[slot], B.S[0], sizeof(State), hipMemcpyDeviceToHost, A->stream));
        HIP_TRY(hipEventRecord(A->ev[slot], A->stream));
        ++launched;
        if (pending >= 0) {
            HIP_TRY(hipEventSynchronize(A->ev[pending]));
            done = A->hstate[pending].done != 0;
        }
        pending = slot;
    }
    HIP_TRY(launch_final(A->sellp(), A->csrp(), A->sp, v, B, 0, b, xout, A->stream));
    HIP_TRY(hipMemcpyAsync(&A->hstate[0], B.S[0], sizeof(State), hipMemcpyDeviceToHost, A->stream));
    HIP_TRY(hipStreamSynchronize(A->stream));
    *final_state = A->hstate[0];
    return PRCG_OK;
}

// A complete solve with the handle's own buffers and graph.
prcg_status run_solve(prcg_matrix A, int variant, const double* b, const double* x0, double* xout, double tol,
                      int32_t maxit, State* final_state)
{
    prcg_status s = ensure_hist(A, (int64_t)maxit + 1);
    if (s != PRCG_OK) return s;
    s = build_graph(A, variant);
    if (s != PRCG_OK) return s;
    return solve_loop(A, A->bufs(), variant, A->graph[variant], b, x0, xout, tol, maxit, final_state);
}

prcg_status check_variant(int v)
{
    if (v < PRCG_HS || v > PRCG_PR_UNSIMPLIFIED) return fail(PRCG_EINVAL, "unknown variant");
    return PRCG_OK;
}

// The batched solver runs HS, PR, pipe-PR and their Meurant forms.
prcg_status check_batch_variant(int v)
{
    if (check_variant(v) != PRCG_OK) return PRCG_EINVAL;
    if (v > PRCG_PIPE_M) return fail(PRCG_EINVAL, "the batched solver runs HS, PR, pipe-PR, M and pipe-M only");
    return PRCG_OK;
}

void fill_info(const State& st, prcg_info* info)
{
    if (!info) return;
    info->iters = st.k < 0 ? 0 : st.k;
    info->status = st.status;
    info->relres_updated = st.bnorm > 0.0 ? std::sqrt(st.rr > 0.0 ? st.rr : 0.0) / st.bnorm : 0.0;
    info->relres_true = st.relres_true;
}

// ---- scratch of the no-allocation solve ----
// prcg_solve_noalloc takes its partial sums, two state copies, the reduction
// ticket and the residual history from one file-scope device array, so that
// a solve allocates nothing.  Every device that runs the library holds its
// own copy (at its own address) until the process ends; every call on a
// device shares that device's copy.  Host code never uses the array's name
// as an address: the device address comes from hipGetSymbolAddress, taken
// once per device with that device current.
constexpr int64_t kStateWords = (int64_t)(2 * sizeof(State) / sizeof(double));
constexpr int64_t kTicketWords = 16;  // 128 bytes: the history stays 128-byte aligned
constexpr int64_t kScratchWords = kPartialWords + kStateWords + kTicketWords + PRCG_NOALLOC_MAX_ITERS + 1;
static_assert(kPartialWords % 16 == 0, "the state copies stay 128-byte aligned");

static __device__ __align__(256) double scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch[kMaxDevices] = {};

// Device address of the calling device's scratch (the device must be current).
prcg_status scratch_of(int device, double** out)
{
    if (device < 0 || device >= kMaxDevices) return fail(PRCG_EDEVICE, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PRCG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[device] = static_cast<double*>(p);
    }
    *out = g_scratch[device];
    return PRCG_OK;
}

// The last-workgroup reduction expects its ticket counter at zero between
// kernels; the scratch keeps whatever the previous call left.
__global__ void k_clear_ticket(int* ticket) { *ticket = 0; }

}  // namespace

extern "C" {

const char* prcg_last_error(void) { return g_last_error.c_str(); }

prcg_status prcg_create_csr(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                            const double* values, prcg_precond precond, void* hip_stream, prcg_matrix* out)
{
    if (!out) return fail(PRCG_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n >= (int64_t)1 << 31) return fail(PRCG_EINVAL, "n must satisfy 1 <= n < 2^31");
    if (nnz < 0 || nnz >= (int64_t)1 << 31) return fail(PRCG_EINVAL, "nnz must satisfy 0 <= nnz < 2^31");
    if (precond != PRCG_PRECOND_NONE && precond != PRCG_PRECOND_JACOBI) return fail(PRCG_EINVAL, "unknown precond");
    if (!is_device_pointer(row_ptr) || (nnz > 0 && (!is_device_pointer(col_idx) || !is_device_pointer(values))))
        return fail(PRCG_EINVAL, "row_ptr, col_idx and values must be device pointers");

    prcg_matrix A = new prcg_matrix_s();
    auto bail = [&](prcg_status s) {
        free_matrix(A);
        return s;
    };
#define TRY(expr)                                       \
    do {                                                \
        prcg_status s_ = (expr);                        \
        if (s_ != PRCG_OK) return bail(s_);             \
    } while (0)
#define HTRY(expr)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return bail(fail(e_ == hipErrorOutOfMemory ? PRCG_ENOMEM : PRCG_EDEVICE,                \
                             std::string(#expr) + ": " + hipGetErrorString(e_)));                   \
    } while (0)

    HTRY(hipGetDevice(&A->device));
    A->stream = (hipStream_t)hip_stream;
    A->n = n;
    A->nnz = nnz;
    A->precond = precond;
    HTRY(hipStreamCreateWithFlags(&A->capture, hipStreamNonBlocking));
    HTRY(hipMalloc(&A->row_ptr, sizeof(int32_t) * (n + 1)));
    HTRY(hipMalloc(&A->col, sizeof(int32_t) * std::max<int64_t>(nnz, 1)));
    HTRY(hipMalloc(&A->val, sizeof(double) * std::max<int64_t>(nnz, 1)));
    HTRY(hipMalloc(&A->dflags, sizeof(int32_t) * 8));
    HTRY(hipHostMalloc(&A->hstate, sizeof(State) * 2, hipHostMallocDefault));
    HTRY(hipEventCreateWithFlags(&A->ev[0], hipEventDisableTiming));
    HTRY(hipEventCreateWithFlags(&A->ev[1], hipEventDisableTiming));
    HTRY(hipMemcpyAsync(A->row_ptr, row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, A->stream));
    if (nnz > 0) {
        HTRY(hipMemcpyAsync(A->col, col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, A->stream));
        HTRY(hipMemcpyAsync(A->val, values, sizeof(double) * nnz, hipMemcpyDeviceToDevice, A->stream));
    }

    // validate the structure (flags[0]) and find the longest row (flags[1])
    HTRY(hipMemsetAsync(A->dflags, 0, sizeof(int32_t) * 8, A->stream));
    HTRY(launch_validate(n, nnz, A->row_ptr, A->col, A->dflags, A->dflags + 1, A->stream));
    int32_t hf[4];
    TRY(read_flags(A, hf, 4));
    if (hf[0] & 1) return bail(fail(PRCG_EINVAL, "row_ptr[0] must be 0"));
    if (hf[0] & 2) return bail(fail(PRCG_EINVAL, "row_ptr must be non-decreasing within [0, nnz]"));
    if (hf[0] & 4) return bail(fail(PRCG_EINVAL, "row_ptr[n] must equal nnz"));
    if (hf[0] & 8) return bail(fail(PRCG_EINVAL, "column index out of range"));
    const int32_t maxlen = hf[1];

    if (precond == PRCG_PRECOND_JACOBI) {
        HTRY(hipMalloc(&A->d, sizeof(double) * n));
        HTRY(launch_jacobi(n, A->row_ptr, A->col, A->val, A->d, A->dflags, A->stream));
        TRY(read_flags(A, hf, 1));
        if (hf[0] & 16) return bail(fail(PRCG_EINVAL, "Jacobi needs every diagonal entry present and > 0"));
    }

    // SELL-64 plan: per-slice slot counts and layout (offset-aligned or packed)
    A->nslices = (n + kSlice - 1) / kSlice;
    std::vector<int32_t> width((size_t)A->nslices), aligned((size_t)A->nslices);
    {
        int32_t* dplan = nullptr;
        HTRY(hipMalloc(&dplan, sizeof(int32_t) * 2 * A->nslices));
        hipError_t e1 = launch_slice_plan(n, A->nslices, A->row_ptr, A->col, nullptr, nullptr, dplan,
                                          dplan + A->nslices, A->stream);
        if (e1 == hipSuccess)
            e1 = hipMemcpyAsync(width.data(), dplan, sizeof(int32_t) * A->nslices, hipMemcpyDeviceToHost, A->stream);
        if (e1 == hipSuccess)
            e1 = hipMemcpyAsync(aligned.data(), dplan + A->nslices, sizeof(int32_t) * A->nslices,
                                hipMemcpyDeviceToHost, A->stream);
        if (e1 == hipSuccess) e1 = hipStreamSynchronize(A->stream);
        (void)hipFree(dplan);
        HTRY(e1);
    }
    // runs of up to kRunSlices consecutive slices of one width and kind,
    // each stored slot-major, for matrices whose default grid gives every
    // workgroup at least one 256-row group (from kBigGroups groups up);
    // smaller ones keep single slices (measured on MI355X: runs take 6% off
    // the 27-point 160^3 product at 8192 workgroups, but slow the fused
    // PR-CG iteration of an 884,736-row problem at 1024 workgroups by 7%)
    const int64_t run_max = (n + kGroupRows - 1) / kGroupRows >= kBigGroups ? kRunSlices : 1;
    std::vector<int64_t> hptr((size_t)A->nslices + 1);
    std::vector<int32_t> hmeta((size_t)A->nslices), hshape((size_t)A->nslices);
    int64_t total = 0;  // value slots of the whole matrix
    for (int64_t q = 0; q < A->nslices; ++q) total += (int64_t)kSlice * width[q];
    const int64_t cached = cached_value_bytes(total * (int64_t)sizeof(double));
    int64_t pos = 0;
    for (int64_t q0 = 0; q0 < A->nslices;) {
        int64_t len = 1;
        while (len < run_max && q0 + len < A->nslices && width[q0 + len] == width[q0] &&
               aligned[q0 + len] == aligned[q0])
            ++len;
        for (int64_t i = 0; i < len; ++i) {
            hptr[q0 + i] = pos + (int64_t)kSlice * i;
            hshape[q0 + i] = width[q0] | (int32_t)(len << 16);
        }
        if (len > 1) A->runs = 1;
        pos += (int64_t)kSlice * len * width[q0];
        if (A->stream_from == INT64_MAX && pos * (int64_t)sizeof(double) > cached)
            A->stream_from = q0 + len;  // the next run
        q0 += len;
    }
    hptr[A->nslices] = pos;
    for (int64_t q = 0; q < A->nslices; ++q) {
        if (aligned[q]) {
            hmeta[q] = (int32_t)A->noffsets;
            A->noffsets += width[q];
        } else {
            hmeta[q] = -1;
            A->stored_packed += (int64_t)kSlice * width[q];
        }
        if (aligned[q] && q >= A->stream_from) A->stored_streamed += (int64_t)kSlice * width[q];
        // every slot of every slice lies inside the storage (widths of 2^16
        // and more do not fit the shape word: SELL-64 is refused for them below)
        if (width[q] > 0 && width[q] <= 0xffff &&
            hptr[q] + (int64_t)(width[q] - 1) * shape_stride(hshape[q]) + kSlice > pos)
            return bail(fail(PRCG_EDEVICE, "internal error: SELL layout out of bounds"));
    }
    A->stored = pos;
    int lanes = 1;
    const char* fmt = std::getenv("PRCG_FORMAT");
    const double mean = (double)nnz / (double)n;
    if (fmt && std::strncmp(fmt, "csr", 3) == 0) {
        lanes = std::atoi(fmt + 3);
        if (lanes != 8 && lanes != 16 && lanes != 32 && lanes != 64) lanes = 8;
    } else if (!(fmt && std::strcmp(fmt, "sell") == 0)) {
        // vector CSR when padding would inflate the SELL storage or rows are long
        const bool sell_ok = (double)A->stored <= 1.5 * (double)nnz + 64.0 * (double)A->nslices && maxlen <= 256;
        if (!sell_ok) lanes = mean >= 96 ? 64 : mean >= 48 ? 32 : mean >= 24 ? 16 : 8;
    }
    if (lanes == 1) {
        // the slice shape word holds widths below 2^16
        if (maxlen > 0xffff)
            return bail(fail(PRCG_EINVAL, "SELL-64 holds rows of at most 65535 entries; use vector CSR"));
        HTRY(hipMalloc(&A->slice_ptr, sizeof(int64_t) * (A->nslices + 1)));
        HTRY(hipMalloc(&A->slice_meta, sizeof(int32_t) * A->nslices));
        HTRY(hipMalloc(&A->slice_shape, sizeof(int32_t) * A->nslices));
        HTRY(hipMalloc(&A->soff, sizeof(int32_t) * std::max<int64_t>(A->noffsets, 1)));
        HTRY(hipMalloc(&A->scol, sizeof(int32_t) * std::max<int64_t>(A->stored, 1)));
        HTRY(hipMalloc(&A->sval, sizeof(double) * std::max<int64_t>(A->stored, 1)));
        HTRY(hipMemcpyAsync(A->slice_ptr, hptr.data(), sizeof(int64_t) * (A->nslices + 1), hipMemcpyHostToDevice,
                            A->stream));
        HTRY(hipMemcpyAsync(A->slice_meta, hmeta.data(), sizeof(int32_t) * A->nslices, hipMemcpyHostToDevice,
                            A->stream));
        HTRY(hipMemcpyAsync(A->slice_shape, hshape.data(), sizeof(int32_t) * A->nslices, hipMemcpyHostToDevice,
                            A->stream));
        HTRY(launch_fill_sell(n, A->nslices, A->row_ptr, A->col, A->val, nullptr, nullptr, A->slice_ptr,
                              A->slice_meta, A->slice_shape, A->soff, A->scol, A->sval, 1, A->stream));
        HTRY(hipStreamSynchronize(A->stream));  // host vectors above must outlive the copies
        if (A->noffsets > 0) {
            std::vector<int32_t> hso((size_t)A->noffsets);
            HTRY(hipMemcpy(hso.data(), A->soff, sizeof(int32_t) * A->noffsets, hipMemcpyDeviceToHost));
            share_offsets(hso, width, hmeta);
            HTRY(hipMemcpy(A->slice_meta, hmeta.data(), sizeof(int32_t) * A->nslices, hipMemcpyHostToDevice));
        }
    }
    A->kernels_mode = PRCG_KERNELS_AUTO;
    A->grid_opt = 0;
    A->sp = make_split(n, lanes, A->grid_opt, A->kernels_mode);
    A->sp.textbook_pre = precond;
    A->sell_storage = A->sell();
    A->csr_storage = A->csr();

    HTRY(hipMalloc(&A->vecs, sizeof(double) * 16 * (size_t)n));
    HTRY(hipMemsetAsync(A->vecs, 0, sizeof(double) * 16 * (size_t)n, A->stream));
    HTRY(hipMalloc(&A->pairs, sizeof(double2) * 2 * (size_t)n));
    HTRY(hipMalloc(&A->S, sizeof(State) * 2));
    HTRY(hipMemsetAsync(A->S, 0, sizeof(State) * 2, A->stream));
    // partials sized for the largest grid, so the grid can change later
    HTRY(hipMalloc(&A->partials, sizeof(double) * (size_t)kPartialWords));
    HTRY(hipStreamSynchronize(A->stream));
    TRY(ensure_hist(A, 1024));
    *out = A;
    return PRCG_OK;
#undef TRY
#undef HTRY
}

prcg_status prcg_set_option(prcg_matrix A, int32_t option, int32_t value)
{
    if (!A) return fail(PRCG_EINVAL, "null handle");
    if (option == PRCG_OPT_KERNELS) {
        if (value < PRCG_KERNELS_FUSED || value > PRCG_KERNELS_AUTO)
            return fail(PRCG_EINVAL, "unknown kernel structure");
        A->kernels_mode = value;
    } else if (option == PRCG_OPT_GRID) {
        if (value != 0 && (value < 8 || value > kMaxGrid))
            return fail(PRCG_EINVAL, "grid must be 0 (by size) or in [8, 16384]");
        A->grid_opt = value;
    } else {
        return fail(PRCG_EINVAL, "unknown option");
    }
    HIP_TRY(hipSetDevice(A->device));
    HIP_TRY(hipStreamSynchronize(A->stream));
    A->sp = make_split(A->n, A->sp.lanes, A->grid_opt, A->kernels_mode);
    A->sp.textbook_pre = A->precond;
    invalidate_graphs(A);
    return PRCG_OK;
}

prcg_status prcg_set_stream(prcg_matrix A, void* hip_stream)
{
    if (!A) return fail(PRCG_EINVAL, "null handle");
    A->stream = (hipStream_t)hip_stream;
    return PRCG_OK;
}

prcg_status prcg_set_values(prcg_matrix A, const double* values)
{
    if (!A) return fail(PRCG_EINVAL, "null handle");
    if (A->nnz > 0 && !is_device_pointer(values)) return fail(PRCG_EINVAL, "values must be a device pointer");
    HIP_TRY(hipSetDevice(A->device));
    if (A->nnz > 0)
        HIP_TRY(hipMemcpyAsync(A->val, values, sizeof(double) * A->nnz, hipMemcpyDeviceToDevice, A->stream));
    if (A->sp.lanes == 1)
        HIP_TRY(launch_fill_sell(A->n, A->nslices, A->row_ptr, A->col, A->val, nullptr, nullptr, A->slice_ptr,
                                 A->slice_meta, A->slice_shape, A->soff, A->scol, A->sval, 0, A->stream));
    if (A->precond == PRCG_PRECOND_JACOBI) {
        HIP_TRY(hipMemsetAsync(A->dflags, 0, sizeof(int32_t), A->stream));
        HIP_TRY(launch_jacobi(A->n, A->row_ptr, A->col, A->val, A->d, A->dflags, A->stream));
        int32_t hf[1];
        prcg_status s = read_flags(A, hf, 1);
        if (s != PRCG_OK) return s;
        if (hf[0] & 16) return fail(PRCG_EINVAL, "Jacobi needs every diagonal entry present and > 0");
    }
    HIP_TRY(hipStreamSynchronize(A->stream));
    return PRCG_OK;
}

prcg_status prcg_spmv(prcg_matrix A, const double* x, double* y)
{
    if (!A) return fail(PRCG_EINVAL, "null handle");
    if (!is_device_pointer(x) || !is_device_pointer(y)) return fail(PRCG_EINVAL, "x and y must be device pointers");
    if (x == y) return fail(PRCG_EINVAL, "x and y must not overlap");
    HIP_TRY(hipSetDevice(A->device));
    HIP_TRY(launch_spmv(A->sellp(), A->csrp(), A->sp, x, y, A->stream));
    HIP_TRY(hipStreamSynchronize(A->stream));
    return PRCG_OK;
}

prcg_status prcg_solve(prcg_matrix A, prcg_variant v, const double* b, double* x, double tol, int32_t maxit,
                       prcg_info* info, double* history)
{
    if (!A) return fail(PRCG_EINVAL, "null handle");
    if (check_variant(v) != PRCG_OK) return PRCG_EINVAL;
    if (!(tol >= 0.0)) return fail(PRCG_EINVAL, "tol must be >= 0");
    if (maxit < 0) return fail(PRCG_EINVAL, "maxit must be >= 0");
    if (!is_device_pointer(b) || !is_device_pointer(x)) return fail(PRCG_EINVAL, "b and x must be device pointers");
    HIP_TRY(hipSetDevice(A->device));
    State st;
    prcg_status s = run_solve(A, v, b, x, x, tol, maxit, &st);
    if (s != PRCG_OK) return s;
    if (history) {
        const int32_t k = st.k < 0 ? 0 : st.k;
        HIP_TRY(hipMemcpy(history, A->hist, sizeof(double) * (k + 1), hipMemcpyDeviceToHost));
    }
    fill_info(st, info);
    return (prcg_status)st.status;
}

prcg_status prcg_solve_noalloc(prcg_matrix A, prcg_variant v, const double* b, double* x, double tol,
                               int32_t maxit, prcg_info* info, double* history)
{
    if (!A) return fail(PRCG_EINVAL, "null handle");
    if (check_variant(v) != PRCG_OK) return PRCG_EINVAL;
    if (!(tol >= 0.0)) return fail(PRCG_EINVAL, "tol must be >= 0");
    if (maxit < 0) return fail(PRCG_EINVAL, "maxit must be >= 0");
    if (maxit > PRCG_NOALLOC_MAX_ITERS)
        return fail(PRCG_EINVAL, "maxit exceeds PRCG_NOALLOC_MAX_ITERS: the residual history lives in a fixed "
                                 "device array of PRCG_NOALLOC_MAX_ITERS + 1 entries");
    if (A->sp.G > kMaxGrid) return fail(PRCG_EINVAL, "more workgroups than the scratch holds partial sums for");
    if (!is_device_pointer(b) || !is_device_pointer(x)) return fail(PRCG_EINVAL, "b and x must be device pointers");
    HIP_TRY(hipSetDevice(A->device));
    double* base = nullptr;
    prcg_status s = scratch_of(A->device, &base);
    if (s != PRCG_OK) return s;
    State* S = reinterpret_cast<State*>(base + kPartialWords);
    int* ticket = reinterpret_cast<int*>(base + kPartialWords + kStateWords);
    double* hist = base + kPartialWords + kStateWords + kTicketWords;
    const Bufs B = bufs_at(base, S, hist, ticket);
    hipLaunchKernelGGL(k_clear_ticket, dim3(1), dim3(1), 0, A->stream, ticket);
    HIP_TRY(hipGetLastError());
    State st;
    s = solve_loop(A, B, v, nullptr, b, x, x, tol, maxit, &st);
    if (s != PRCG_OK) return s;
    if (history) {
        const int32_t k = st.k < 0 ? 0 : st.k;
        HIP_TRY(hipMemcpy(history, hist, sizeof(double) * (k + 1), hipMemcpyDeviceToHost));
    }
    fill_info(st, info);
    return (prcg_status)st.status;
}

prcg_status prcg_get_props(prcg_matrix A, prcg_matrix_props* props)
{
    if (!A || !props) return fail(PRCG_EINVAL, "null argument");
    props->n = A->n;
    props->nnz = A->nnz;
    props->format = A->sp.lanes == 1 ? 0 : 1;
    props->lanes_per_row = A->sp.lanes;
    props->stored_entries = A->sp.lanes == 1 ? A->stored : A->nnz;
    props->grid = A->sp.G;
    props->kernels = A->sp.fused ? PRCG_KERNELS_FUSED
                                 : (A->kernels_mode == PRCG_KERNELS_AUTO ? PRCG_KERNELS_TWO_PASS : A->kernels_mode);
    props->stage2 = A->sp.stage2;
    props->block = kBlock;
    // bytes one product reads: values, the column indices of packed slices,
    // the offsets of aligned slices and the per-slice metadata
    props->matrix_bytes = A->sp.lanes == 1
                              ? 8 * A->stored + 4 * A->stored_packed + 4 * A->noffsets + 16 * A->nslices
                              : 12 * A->nnz + 4 * (A->n + 1);
    props->aligned_slices_frac = 0.0;
    if (A->sp.lanes == 1 && A->nslices > 0)
        props->aligned_slices_frac = 1.0 - (double)A->stored_packed / (double)std::max<int64_t>(A->stored, 1);
    props->streamed_entries = A->sp.lanes == 1 ? A->stored_streamed : 0;
    return PRCG_OK;
}

prcg_status prcg_time_kernels(prcg_matrix A, prcg_variant v, int32_t iters, double* ms_per_launch,
                              char (*names)[48], int32_t capacity, int32_t* nkernels)
{
    if (!A || !ms_per_launch || !nkernels) return fail(PRCG_EINVAL, "null argument");
    if (check_variant(v) != PRCG_OK) return PRCG_EINVAL;
    if (iters < 1) return fail(PRCG_EINVAL, "iters must be >= 1");
    if (capacity < iter_kernel_count(v, A->sp))
        return fail(PRCG_EINVAL, "capacity is smaller than the number of kernels per iteration");
    HIP_TRY(hipSetDevice(A->device));
    prcg_status s = ensure_hist(A, (int64_t)iters + 2);
    if (s != PRCG_OK) return s;
    const Vecs vv = A->vecs_view();
    const Bufs B = A->bufs();
    // The timed launches go to the handle's own non-blocking stream (after
    // the caller's stream has drained): dispatch timestamps on a
    // non-blocking stream measure the kernel alone.
    HIP_TRY(hipStreamSynchronize(A->stream));
    hipStream_t ts = A->capture;
    // right-hand side: the spare vector filled with ones; x0 = 0 (vector x)
    const int nk = iter_kernel_count(v, A->sp);
    std::vector<double> ones((size_t)A->n, 1.0);
    double* bvec = A->spare();
    HIP_TRY(hipMemcpyAsync(bvec, ones.data(), sizeof(double) * A->n, hipMemcpyHostToDevice, ts));
    HIP_TRY(hipMemsetAsync(vv.x, 0, sizeof(double) * A->n, ts));
    HIP_TRY(launch_init(v, A->precond, A->sellp(), A->csrp(), A->sp, vv, B, bvec, vv.x, 0.0, iters + 1, ts));
    std::vector<hipEvent_t> ev((size_t)2 * nk * iters, nullptr);
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    int cur = 0;
    hipError_t err = hipSuccess;
    for (int it = 0; it < iters && err == hipSuccess; ++it)
        for (int j = 0; j < nk && err == hipSuccess; ++j) {
            const size_t q = (size_t)2 * (it * nk + j);
            const LaunchEvents le{ev[q], ev[q + 1]};
            err = launch_iteration(A, B, v, j, it, cur, ts, &le);
        }
    if (err == hipSuccess) err = hipStreamSynchronize(ts);
    std::vector<double> tot((size_t)nk, 0.0);
    for (int it = 0; it < iters && err == hipSuccess; ++it)
        for (int j = 0; j < nk && err == hipSuccess; ++j) {
            const size_t q = (size_t)2 * (it * nk + j);
            float ms = 0.f;
            err = hipEventElapsedTime(&ms, ev[q], ev[q + 1]);
            tot[j] += ms;
        }
    for (auto& e : ev) (void)hipEventDestroy(e);
    HIP_TRY(err);
    State st;
    HIP_TRY(hipMemcpy(&st, A->S + cur, sizeof(State), hipMemcpyDeviceToHost));
    if (st.done && st.k < iters)
        return fail(PRCG_EDEVICE, "timing run ended early (breakdown); times would be diluted");
    *nkernels = nk;
    for (int j = 0; j < nk; ++j) {
        ms_per_launch[j] = tot[j] / iters;
        if (names) {
            std::snprintf(names[j], 48, "%s", iter_kernel_name(v, A->sp, j));
        }
    }
    return PRCG_OK;
}

prcg_status prcg_adjoint(prcg_matrix A, prcg_variant v, const double* x, const double* gx, double* gb, double* gvals,
                         double tol, int32_t maxit, prcg_info* info)
{
    if (!A) return fail(PRCG_EINVAL, "null handle");
    if (check_variant(v) != PRCG_OK) return PRCG_EINVAL;
    if (!(tol >= 0.0) || maxit < 0) return fail(PRCG_EINVAL, "tol must be >= 0 and maxit >= 0");
    if (!is_device_pointer(x) || !is_device_pointer(gx)) return fail(PRCG_EINVAL, "x and gx must be device pointers");
    if ((gb && !is_device_pointer(gb)) || (gvals && !is_device_pointer(gvals)))
        return fail(PRCG_EINVAL, "gb and gvals must be device pointers");
    HIP_TRY(hipSetDevice(A->device));
    // lambda = A^{-1} gx from x0 = 0 (the spare vector, zeroed); the result
    // goes to gb, or to the spare vector itself when gb is NULL (the
    // initialisation has copied x0 before the result is written).
    double* x0 = A->spare();
    double* lam = gb ? gb : x0;
    HIP_TRY(hipMemsetAsync(x0, 0, sizeof(double) * A->n, A->stream));
    State st;
    prcg_status s = run_solve(A, v, gx, x0, lam, tol, maxit, &st);
    if (s != PRCG_OK) return s;
    if (gvals && A->nnz > 0) {
        HIP_TRY(launch_outer_csr(A->n, A->row_ptr, A->col, lam, x, gvals, (double)A->nnz / (double)A->n, A->stream));
        HIP_TRY(hipStreamSynchronize(A->stream));
    }
    fill_info(st, info);
    return (prcg_status)st.status;
}

void prcg_destroy(prcg_matrix A) { free_matrix(A); }

prcg_status prcg_create_batch(prcg_matrix A, int32_t nsys, const int64_t* sys_row_offset, prcg_batch* out)
{
    if (!out) return fail(PRCG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!A || nsys < 1 || !sys_row_offset) return fail(PRCG_EINVAL, "need a matrix, nsys >= 1 and offsets");
    if (sys_row_offset[0] != 0 || sys_row_offset[nsys] != A->n)
        return fail(PRCG_EINVAL, "sys_row_offset must start at 0 and end at n");
    for (int32_t q = 0; q < nsys; ++q)
        if (sys_row_offset[q + 1] <= sys_row_offset[q])
            return fail(PRCG_EINVAL, "sys_row_offset must be strictly increasing");
    HIP_TRY(hipSetDevice(A->device));
    prcg_batch B = new prcg_batch_s();
    B->A = A;
    B->nsys = nsys;
    auto bail = [&](prcg_status st) {
        free_batch(B);
        return st;
    };
#define BTRY(expr)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return bail(fail(e_ == hipErrorOutOfMemory ? PRCG_ENOMEM : PRCG_EDEVICE,                \
                             std::string(#expr) + ": " + hipGetErrorString(e_)));                   \
    } while (0)
    const int64_t n = A->n;
    hipStream_t st = A->stream;
    // block structure: no column may leave its system
    {
        std::vector<int32_t> row_sys((size_t)n);
        for (int32_t q = 0; q < nsys; ++q)
            for (int64_t i = sys_row_offset[q]; i < sys_row_offset[q + 1]; ++i) row_sys[(size_t)i] = q;
        int32_t* drs = nullptr;
        int64_t* doff = nullptr;
        BTRY(hipMalloc(&drs, sizeof(int32_t) * n));
        hipError_t e = hipMalloc(&doff, sizeof(int64_t) * (nsys + 1));
        if (e == hipSuccess) e = hipMemcpyAsync(drs, row_sys.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(doff, sys_row_offset, sizeof(int64_t) * (nsys + 1), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemsetAsync(A->dflags, 0, sizeof(int32_t), st);
        if (e == hipSuccess) e = launch_block_check(n, A->row_ptr, A->col, drs, doff, A->dflags, st);
        int32_t hf = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&hf, A->dflags, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        (void)hipFree(drs);
        if (doff) (void)hipFree(doff);
        BTRY(e);
        if (hf & 32) return bail(fail(PRCG_EINVAL, "a column index leaves its system's block"));
    }
    // slice geometry: slices restart at every system
    std::vector<int64_t> sys_slice0((size_t)nsys + 1), slice_row0;
    std::vector<int32_t> slice_nrows;
    sys_slice0[0] = 0;
    for (int32_t q = 0; q < nsys; ++q) {
        for (int64_t r0 = sys_row_offset[q]; r0 < sys_row_offset[q + 1]; r0 += kSlice) {
            slice_row0.push_back(r0);
            slice_nrows.push_back((int32_t)std::min<int64_t>(kSlice, sys_row_offset[q + 1] - r0));
        }
        sys_slice0[q + 1] = (int64_t)slice_row0.size();
    }
    const int64_t ns = (int64_t)slice_row0.size();
    B->nslices = ns;
    BTRY(hipMalloc(&B->slice_row0, sizeof(int64_t) * ns));
    BTRY(hipMalloc(&B->slice_nrows, sizeof(int32_t) * ns));
    BTRY(hipMalloc(&B->sys_row0, sizeof(int64_t) * (nsys + 1)));
    BTRY(hipMalloc(&B->sys_slice0, sizeof(int64_t) * (nsys + 1)));
    BTRY(hipMemcpyAsync(B->slice_row0, slice_row0.data(), sizeof(int64_t) * ns, hipMemcpyHostToDevice, st));
    BTRY(hipMemcpyAsync(B->slice_nrows, slice_nrows.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, st));
    BTRY(hipMemcpyAsync(B->sys_row0, sys_row_offset, sizeof(int64_t) * (nsys + 1), hipMemcpyHostToDevice, st));
    BTRY(hipMemcpyAsync(B->sys_slice0, sys_slice0.data(), sizeof(int64_t) * (nsys + 1), hipMemcpyHostToDevice, st));
    // plan and fill the slices (offset-aligned or packed, as for a single matrix)
    std::vector<int32_t> width((size_t)ns), aligned((size_t)ns);
    {
        int32_t* dplan = nullptr;
        BTRY(hipMalloc(&dplan, sizeof(int32_t) * 2 * ns));
        hipError_t e = launch_slice_plan(n, ns, A->row_ptr, A->col, B->slice_row0, B->slice_nrows, dplan, dplan + ns,
                                         st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(width.data(), dplan, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(aligned.data(), dplan + ns, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        (void)hipFree(dplan);
        BTRY(e);
    }
    for (int64_t q = 0; q < ns; ++q)
        if (width[q] > 0xffff) return bail(fail(PRCG_EINVAL, "a batched system has a row of more than 65535 entries"));
    // slices of a batch are stored singly (run length 1, slot stride 64),
    // as the persistent kernel's paired product reads them
    std::vector<int64_t> hptr((size_t)ns + 1);
    std::vector<int32_t> hmeta((size_t)ns), hshape((size_t)ns);
    int64_t noff = 0;
    hptr[0] = 0;
    for (int64_t q = 0; q < ns; ++q) {
        hptr[q + 1] = hptr[q] + (int64_t)kSlice * width[q];
        hmeta[q] = aligned[q] ? (int32_t)noff : -1;
        hshape[q] = width[q] | (1 << 16);
        if (aligned[q]) noff += width[q];
    }
    B->stored = hptr[ns];
    B->noffsets = noff;
    for (int64_t q = 0; q < ns; ++q)
        if (!aligned[q]) B->stored_packed += (int64_t)kSlice * width[q];
    const int64_t cached = cached_value_bytes(hptr[ns] * (int64_t)sizeof(double));
    for (int64_t q = 0; q < ns; ++q)
        if (hptr[q + 1] * (int64_t)sizeof(double) > cached) {
            B->stream_from = q + 1;
            break;
        }
    BTRY(hipMalloc(&B->slice_ptr, sizeof(int64_t) * (ns + 1)));
    BTRY(hipMalloc(&B->slice_meta, sizeof(int32_t) * ns));
    BTRY(hipMalloc(&B->slice_shape, sizeof(int32_t) * ns));
    BTRY(hipMalloc(&B->soff, sizeof(int32_t) * std::max<int64_t>(noff, 1)));
    BTRY(hipMalloc(&B->scol, sizeof(int32_t) * std::max<int64_t>(B->stored, 1)));
    BTRY(hipMalloc(&B->sval, sizeof(double) * std::max<int64_t>(B->stored, 1)));
    BTRY(hipMemcpyAsync(B->slice_ptr, hptr.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, st));
    BTRY(hipMemcpyAsync(B->slice_meta, hmeta.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, st));
    BTRY(hipMemcpyAsync(B->slice_shape, hshape.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, st));
    BTRY(launch_fill_sell(n, ns, A->row_ptr, A->col, A->val, B->slice_row0, B->slice_nrows, B->slice_ptr,
                          B->slice_meta, B->slice_shape, B->soff, B->scol, B->sval, 1, st));
    // Row groups of the lockstep solver: runs of up to 8, 16 or 32 slices
    // of one system (the autotuner picks the size).  Offset-aligned slices of one width (at most
    // kUniformMaxWidth) with the same column offsets form uniform groups,
    // which the product multiplies with all their value loads issued at
    // once; every other run of slices forms a general group.
    std::vector<int32_t> hsoff((size_t)std::max<int64_t>(noff, 1));
    if (noff > 0) {
        BTRY(hipMemcpyAsync(hsoff.data(), B->soff, sizeof(int32_t) * noff, hipMemcpyDeviceToHost, st));
        BTRY(hipStreamSynchronize(st));
        share_offsets(hsoff, width, hmeta);
        BTRY(hipMemcpy(B->slice_meta, hmeta.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice));
    }
    auto uniform_slice = [&](int64_t q) {
        return aligned[q] && width[q] >= 1 && width[q] <= kUniformMaxWidth && hptr[q] / kSlice < INT32_MAX;
    };
    auto same_key = [&](int64_t q, int64_t t) {
        if (uniform_slice(q) != uniform_slice(t)) return false;
        if (!uniform_slice(q)) return true;
        if (width[q] != width[t]) return false;
        for (int32_t u = 0; u < width[q]; ++u)
            if (hsoff[(size_t)hmeta[q] + u] != hsoff[(size_t)hmeta[t] + u]) return false;
        return true;
    };
    // one table per group size; the host arrays stay alive until the copies
    // have run (the stream is synchronised below)
    std::vector<Group> grp[prcg_batch_s::kTables];
    std::vector<int64_t> sys_grp0[prcg_batch_s::kTables];
    int64_t max_groups = 1;
    for (int t = 0; t < prcg_batch_s::kTables; ++t) {
        const int spw = 2 << t;  // 2, 4, 8 slices per wavefront
        const int gslices = kWaves * spw;
        sys_grp0[t].assign((size_t)nsys + 1, 0);
        for (int32_t q = 0; q < nsys; ++q) {
            sys_grp0[t][q] = (int64_t)grp[t].size();
            for (int64_t s0 = sys_slice0[q]; s0 < sys_slice0[q + 1];) {
                int64_t len = 1;
                while (len < gslices && s0 + len < sys_slice0[q + 1] && same_key(s0, s0 + len)) ++len;
                Group G{};
                G.slice0 = (int32_t)s0;
                G.nsl = (int32_t)len;
                G.row0 = (int32_t)slice_row0[(size_t)s0];
                const int64_t last = s0 + len - 1;
                G.nrows = (int32_t)(slice_row0[(size_t)last] + slice_nrows[(size_t)last] - G.row0);
                G.sys = q;
                G.lo = (int32_t)sys_row_offset[q];
                G.hi = (int32_t)(sys_row_offset[q + 1] - 1);
                G.off = uniform_slice(s0) ? hmeta[s0] : -1;
                G.width = width[s0];
                G.vrow = (int32_t)(hptr[s0] / kSlice);
                G.diag = -1;
                G.flags = 0;
                if (G.off >= 0) {
                    const int32_t* o = hsoff.data() + G.off;
                    for (int32_t u = 0; u < G.width; ++u) {
                        G.o[u] = o[u];
                        if (o[u] == 0) G.diag = u;
                    }
                    if (G.diag >= 1 && G.diag + 1 < G.width && o[G.diag - 1] == -1 && o[G.diag + 1] == 1)
                        G.flags |= kGroupShift;
                }
                grp[t].push_back(G);
                s0 += len;
            }
        }
        sys_grp0[t][nsys] = (int64_t)grp[t].size();
        auto& T = B->tab[t];
        T.spw = spw;
        T.ngroups = sys_grp0[t][nsys];
        for (const Group& G : grp[t]) T.uniform_groups += G.off >= 0;
        // every group uniform: the lockstep product (and the fused
        // iteration) launch the kernel compiled for the least of 3, 5, 7
        // slots at or above the widest group
        int32_t wmax = 0;
        for (const Group& G : grp[t]) wmax = std::max(wmax, G.width);
        T.uwidth = 0;
        if (T.ngroups > 0 && T.uniform_groups == T.ngroups)
            T.uwidth = wmax <= 3 ? 3 : wmax <= 5 ? 5 : wmax <= 7 ? 7 : 0;
        T.span = 0;
        for (const Group& G : grp[t]) {
            if (G.off < 0) continue;
            int omin = 0, omax = 0;  // the span includes offset 0 (the group's own rows)
            for (int u = 0; u < G.width; ++u) {
                omin = std::min(omin, G.o[u]);
                omax = std::max(omax, G.o[u]);
            }
            T.span = std::max(T.span, omax - omin);
        }
        T.fuse_ok = T.uwidth > 0 && (spw == 2 || spw == 4) &&
                    fused_lds_doubles(kWaves * spw * kSlice, T.span, true) <= kFuseLdsDoubles;
        max_groups = std::max(max_groups, T.ngroups);
        BTRY(hipMalloc(&T.grp, sizeof(Group) * T.ngroups));
        BTRY(hipMalloc(&T.sys_grp0, sizeof(int64_t) * (nsys + 1)));
        BTRY(hipMalloc(&T.gdone, sizeof(int32_t) * T.ngroups));
        BTRY(hipMemcpyAsync(T.grp, grp[t].data(), sizeof(Group) * T.ngroups, hipMemcpyHostToDevice, st));
        BTRY(hipMemcpyAsync(T.sys_grp0, sys_grp0[t].data(), sizeof(int64_t) * (nsys + 1), hipMemcpyHostToDevice,
                            st));
    }
    BTRY(hipMalloc(&B->lstate, sizeof(State) * nsys));
    BTRY(hipMalloc(&B->lpart, sizeof(double) * 6 * max_groups));
    BTRY(hipMalloc(&B->lactive, sizeof(int32_t) * 4));
    BTRY(hipMalloc(&B->lticket, sizeof(int32_t) * nsys));
    BTRY(hipMemsetAsync(B->lticket, 0, sizeof(int32_t) * nsys, st));
    BTRY(hipHostMalloc(&B->hactive, sizeof(int32_t) * 2, hipHostMallocDefault));
    BTRY(hipEventCreateWithFlags(&B->lev[0], hipEventDisableTiming));
    BTRY(hipEventCreateWithFlags(&B->lev[1], hipEventDisableTiming));
    // largest systems first
    std::vector<int32_t> order((size_t)nsys);
    for (int32_t q = 0; q < nsys; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return sys_row_offset[a + 1] - sys_row_offset[a] > sys_row_offset[b + 1] - sys_row_offset[b];
    });
    BTRY(hipMalloc(&B->order, sizeof(int32_t) * nsys));
    BTRY(hipMemcpyAsync(B->order, order.data(), sizeof(int32_t) * nsys, hipMemcpyHostToDevice, st));
    BTRY(hipMalloc(&B->vecs, sizeof(double) * 9 * (size_t)n));
    // zero slots read the vectors at clamped columns of their own system
    // before every entry has been written once: start from finite values
    BTRY(hipMemsetAsync(B->vecs, 0, sizeof(double) * 9 * (size_t)n, st));
    BTRY(hipMalloc(&B->queue, sizeof(int32_t) * 4));
    BTRY(hipMalloc(&B->iters, sizeof(int32_t) * nsys));
    BTRY(hipMalloc(&B->status, sizeof(int32_t) * nsys));
    BTRY(hipStreamSynchronize(st));  // the host vectors above must outlive the copies
    hipDeviceProp_t prop;
    BTRY(hipGetDeviceProperties(&prop, A->device));
    B->num_cus = prop.multiProcessorCount;
    *out = B;
    return PRCG_OK;
#undef BTRY
}

prcg_status prcg_solve_batched(prcg_batch B, prcg_variant v, const double* b, double* x, double tol, int32_t maxit,
                               int32_t* iters, int32_t* status)
{
    if (!B) return fail(PRCG_EINVAL, "null batch");
    if (check_batch_variant(v) != PRCG_OK) return PRCG_EINVAL;
    if (!(tol >= 0.0) || maxit < 0) return fail(PRCG_EINVAL, "tol must be >= 0 and maxit >= 0");
    if (!is_device_pointer(b) || !is_device_pointer(x)) return fail(PRCG_EINVAL, "b and x must be device pointers");
    prcg_matrix A = B->A;
    HIP_TRY(hipSetDevice(A->device));
    hipStream_t st = A->stream;
    const size_t nb = sizeof(double) * (size_t)A->n;
    double* bvec = B->vecs + 8 * (size_t)A->n;
    const Vecs vv = B->vecs_view();
    const BatchView view = B->view();
    const int kind = v == PRCG_HS ? 0 : (v == PRCG_PR || v == PRCG_M) ? 1 : 2;
    HIP_TRY(hipMemcpyAsync(bvec, b, nb, hipMemcpyDeviceToDevice, st));
    // lockstep solve of the batch in vv.x (PR-CG, M-CG): the initialisation,
    // then graphs of kLockstepChunk iterations until no system is running;
    // the count of a chunk is read while the next chunk runs.  Every system
    // is done after maxit iterations, so the chunk count is bounded.
    constexpr int kLockstepChunk = 16;
    auto run_lockstep = [&]() -> hipError_t {
        const GroupView gv = B->groups(B->ls_table);
        hipError_t e = launch_lockstep_init(view, gv, vv, bvec, B->lstate, B->lpart, tol, maxit, v, A->precond,
                                            B->iters, B->status, st);
        if (e != hipSuccess) return e;
        if (!B->ls_graph[v]) {
            e = hipStreamBeginCapture(A->capture, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return e;
            hipError_t e1 = launch_lockstep_iterations(view, gv, vv, B->lstate, B->lpart, kLockstepChunk, v,
                                                       A->precond, B->ls_fused, B->iters, B->status, B->lactive,
                                                       A->capture);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(A->capture, &g);
            hipError_t e3 = (e1 == hipSuccess && e2 == hipSuccess) ? hipGraphInstantiate(&B->ls_graph[v], g, nullptr,
                                                                                         nullptr, 0)
                                                                   : (e1 != hipSuccess ? e1 : e2);
            if (g) (void)hipGraphDestroy(g);
            if (e3 != hipSuccess) {
                B->ls_graph[v] = nullptr;
                return e3;
            }
        }
        const int64_t chunks = (int64_t)maxit / kLockstepChunk + 2;
        for (int64_t c = 0; c < chunks; ++c) {
            if ((e = hipGraphLaunch(B->ls_graph[v], st)) != hipSuccess) return e;
            if ((e = hipMemcpyAsync(B->hactive + (c & 1), B->lactive, sizeof(int32_t), hipMemcpyDeviceToHost, st)) !=
                hipSuccess)
                return e;
            if ((e = hipEventRecord(B->lev[c & 1], st)) != hipSuccess) return e;
            if (c > 0) {
                if ((e = hipEventSynchronize(B->lev[(c - 1) & 1])) != hipSuccess) return e;
                if (B->hactive[(c - 1) & 1] == 0) break;
            }
        }
        return hipSuccess;
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto elapsed = [&](auto&& work, float& ms) -> prcg_status {
        if (!e0) {
            HIP_TRY(hipEventCreate(&e0));
            HIP_TRY(hipEventCreate(&e1));
        }
        HIP_TRY(hipMemcpyAsync(vv.x, x, nb, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipEventRecord(e0, st));
        HIP_TRY(work());
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        return PRCG_OK;
    };
    auto release_events = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        e0 = e1 = nullptr;
    };
    // Autotune once per kind the persistent launch: threads per workgroup x
    // workgroups per compute unit x slices multiplied together per
    // wavefront, each candidate timed on a short run of this batch (tol = 0,
    // a few iterations per system).  Dimensions fixed by
    // prcg_batch_set_config (or PRCG_BATCH_CONFIG="threads,per_cu") are not
    // searched.
    if (B->tuned_nt[kind] == 0) {
        int fnt = B->force_nt, fper = B->force_per_cu;
        const char* env = std::getenv("PRCG_BATCH_CONFIG");
        int ent = 0, eper = 0;
        if (!fnt && env && std::sscanf(env, "%d,%d", &ent, &eper) == 2 && (ent == 256 || ent == 512 || ent == 1024) &&
            eper >= 1 && eper <= 8) {
            fnt = ent;
            fper = eper;
        }
        const int nts[] = {256, 512, 1024};
        const int pers[] = {1, 2, 4, 8};
        const int qs[] = {1, 2};
        float best = 1e30f;
        const int trial_it = std::min<int32_t>(maxit, 12);
        bool single = true;  // a single candidate needs no trial
        int ncand = 0;
        for (int nt : nts)
            for (int per : pers)
                for (int q : qs) {
                    if ((fnt && nt != fnt) || (fper && per != fper) || (B->force_q && q != B->force_q)) continue;
                    if (nt * per > 2048) continue;  // threads per compute unit
                    ++ncand;
                }
        single = ncand == 1;
        for (int nt : nts)
            for (int per : pers)
                for (int q : qs) {
                    if ((fnt && nt != fnt) || (fper && per != fper) || (B->force_q && q != B->force_q)) continue;
                    if (nt * per > 2048) continue;
                    const int grid = (int)std::min<int64_t>(B->nsys, (int64_t)B->num_cus * per);
                    float ms = 0.f;
                    if (!single) {
                        prcg_status s = elapsed(
                            [&] {
                                return launch_batch(view, vv, bvec, 0.0, trial_it, v, A->precond, nt, grid, q,
                                                    B->queue, B->iters, B->status, st);
                            },
                            ms);
                        if (s != PRCG_OK) {
                            release_events();
                            return s;
                        }
                    }
                    if (ms < best) {
                        best = ms;
                        B->tuned_nt[kind] = nt;
                        B->tuned_grid[kind] = grid;
                        B->tuned_q[kind] = q;
                    }
                }
        if (B->tuned_nt[kind] == 0) {
            release_events();
            return fail(PRCG_EINVAL, "no persistent launch shape satisfies the fixed configuration");
        }
    }
    // Lockstep group size (PR-CG and M-CG): groups of 8, 16 and 32 slices,
    // each with three launches per iteration and, where the table allows,
    // with the fused iteration; each candidate
    // timed on the initialisation and 32 iterations of this batch (tol = 0).
    // The group size is fixed by prcg_batch_set_config, the fusion by
    // prcg_batch_set_fusion.
    if (kind == 1 && B->mode_req != PRCG_BATCH_PERSISTENT && B->ls_table < 0) {
        float best = 1e30f;
        int ncand = 0;
        for (int t = 0; t < prcg_batch_s::kTables; ++t) {
            if (B->force_group && kWaves * B->tab[t].spw != B->force_group) continue;
            for (int f = 0; f < 2; ++f) {
                const bool fused = f == 1;
                if (fused && (!B->tab[t].fuse_ok || B->force_fusion == PRCG_BATCH_FUSION_OFF)) continue;
                if (!fused && B->force_fusion == PRCG_BATCH_FUSION_ON) continue;
                ++ncand;
                float ms = 0.f;
                const GroupView gv = B->groups(t);
                prcg_status s = elapsed(
                    [&] {
                        hipError_t e = launch_lockstep_init(view, gv, vv, bvec, B->lstate, B->lpart, 0.0,
                                                            std::min<int32_t>(maxit, 32), v, A->precond, B->iters,
                                                            B->status, st);
                        if (e == hipSuccess)
                            e = launch_lockstep_iterations(view, gv, vv, B->lstate, B->lpart, 32, v, A->precond,
                                                           fused, B->iters, B->status, B->lactive, st);
                        return e;
                    },
                    ms);
                if (s != PRCG_OK) {
                    release_events();
                    return s;
                }
                if (ms < best) {
                    best = ms;
                    B->ls_table = t;
                    B->ls_fused = fused;
                }
            }
        }
        if (ncand == 0) {
            release_events();
            return fail(PRCG_EINVAL, "no lockstep group table allows the fused iteration with this configuration");
        }
        for (auto& g : B->ls_graph) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    }
    // persistent or lockstep: PR-CG and M-CG time one whole solve of each on
    // this batch (the persistent kernel's tail, where a few large systems
    // run on one workgroup each, is what lockstep avoids)
    if (B->mode[kind] == 0) {
        if (kind != 1 || B->mode_req == PRCG_BATCH_PERSISTENT) {
            B->mode[kind] = PRCG_BATCH_PERSISTENT;
        } else if (B->mode_req == PRCG_BATCH_LOCKSTEP) {
            B->mode[kind] = PRCG_BATCH_LOCKSTEP;
        } else {
            float ms[2] = {0.f, 0.f};
            for (int m = 0; m < 2; ++m) {
                prcg_status s = elapsed(
                    [&] {
                        if (m == 0)
                            return launch_batch(view, vv, bvec, tol, maxit, v, A->precond, B->tuned_nt[kind],
                                                B->tuned_grid[kind], B->tuned_q[kind], B->queue, B->iters, B->status,
                                                st);
                        return run_lockstep();
                    },
                    ms[m]);
                if (s != PRCG_OK) {
                    release_events();
                    return s;
                }
            }
            B->mode[kind] = ms[1] < ms[0] ? PRCG_BATCH_LOCKSTEP : PRCG_BATCH_PERSISTENT;
        }
    }
    release_events();
    if (B->mode[kind] == PRCG_BATCH_LOCKSTEP) {
        HIP_TRY(hipMemcpyAsync(vv.x, x, nb, hipMemcpyDeviceToDevice, st));
        HIP_TRY(run_lockstep());
    } else {
        // one graph per (kind, variant, tol, maxit): reset the queue + persistent kernel
        if (!B->graph[v] || B->graph_tol[v] != tol || B->graph_maxit[v] != maxit) {
            if (B->graph[v]) (void)hipGraphExecDestroy(B->graph[v]);
            B->graph[v] = nullptr;
            HIP_TRY(hipStreamBeginCapture(A->capture, hipStreamCaptureModeThreadLocal));
            hipError_t err = launch_batch(view, vv, bvec, tol, maxit, v, A->precond, B->tuned_nt[kind],
                                          B->tuned_grid[kind], B->tuned_q[kind], B->queue, B->iters, B->status,
                                          A->capture);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(A->capture, &g);
            if (err != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail(PRCG_EDEVICE, "batched graph capture failed");
            }
            hipError_t e3 = hipGraphInstantiate(&B->graph[v], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIP_TRY(e3);
            B->graph_tol[v] = tol;
            B->graph_maxit[v] = maxit;
        }
        HIP_TRY(hipMemcpyAsync(vv.x, x, nb, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipGraphLaunch(B->graph[v], st));
    }
    HIP_TRY(hipMemcpyAsync(x, vv.x, nb, hipMemcpyDeviceToDevice, st));
    std::vector<int32_t> hst((size_t)B->nsys);
    HIP_TRY(hipMemcpyAsync(hst.data(), B->status, sizeof(int32_t) * B->nsys, hipMemcpyDeviceToHost, st));
    if (iters) HIP_TRY(hipMemcpyAsync(iters, B->iters, sizeof(int32_t) * B->nsys, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (status) std::memcpy(status, hst.data(), sizeof(int32_t) * B->nsys);
    int worst = PRCG_OK;
    for (int32_t q = 0; q < B->nsys; ++q) worst = std::max(worst, (int)hst[q]);
    return (prcg_status)worst;
}

prcg_status prcg_batch_config(prcg_batch B, prcg_variant v, int32_t* threads, int32_t* grid)
{
    if (!B || !threads || !grid) return fail(PRCG_EINVAL, "null argument");
    if (check_batch_variant(v) != PRCG_OK) return PRCG_EINVAL;
    const int kind = v == PRCG_HS ? 0 : (v == PRCG_PR || v == PRCG_M) ? 1 : 2;
    *threads = B->tuned_nt[kind];
    *grid = B->tuned_grid[kind];
    return PRCG_OK;
}

prcg_status prcg_batch_set_config(prcg_batch B, int32_t threads, int32_t per_cu, int32_t slices_in_flight,
                                  int32_t group_slices)
{
    if (!B) return fail(PRCG_EINVAL, "null batch");
    if (threads != 0 && threads != 256 && threads != 512 && threads != 1024)
        return fail(PRCG_EINVAL, "threads must be 0, 256, 512 or 1024");
    if (per_cu < 0 || per_cu > 8 || (threads && per_cu && threads * per_cu > 2048))
        return fail(PRCG_EINVAL, "per_cu must be in 0..8 with threads x per_cu <= 2048");
    if (slices_in_flight < 0 || slices_in_flight > 2) return fail(PRCG_EINVAL, "slices_in_flight must be 0, 1 or 2");
    if (group_slices != 0 && group_slices != 8 && group_slices != 16 && group_slices != 32)
        return fail(PRCG_EINVAL, "group_slices must be 0, 8, 16 or 32");
    HIP_TRY(hipSetDevice(B->A->device));
    HIP_TRY(hipStreamSynchronize(B->A->stream));
    B->force_nt = threads;
    B->force_per_cu = per_cu;
    B->force_q = slices_in_flight;
    B->force_group = group_slices;
    for (int k = 0; k < 3; ++k) B->tuned_nt[k] = B->tuned_grid[k] = B->tuned_q[k] = 0;
    B->ls_table = -1;
    for (auto& m : B->mode) m = 0;
    for (auto& g : B->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    for (auto& g : B->ls_graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    return PRCG_OK;
}

prcg_status prcg_batch_get_props(prcg_batch B, prcg_variant v, prcg_batch_props* props)
{
    if (!B || !props) return fail(PRCG_EINVAL, "null argument");
    if (check_batch_variant(v) != PRCG_OK) return PRCG_EINVAL;
    const int kind = v == PRCG_HS ? 0 : (v == PRCG_PR || v == PRCG_M) ? 1 : 2;
    prcg_batch_props p{};
    p.n = B->A->n;
    p.nsys = B->nsys;
    p.stored_entries = B->stored;
    // values, the column indices of packed slices, the offsets of aligned
    // slices and the per-slice metadata
    p.matrix_bytes = 8 * B->stored + 4 * B->stored_packed + 4 * B->noffsets + 16 * B->nslices;
    p.mode = B->mode[kind];
    p.threads = B->tuned_nt[kind];
    p.grid = B->tuned_grid[kind];
    p.slices_in_flight = B->tuned_q[kind];
    const int t = kind == 1 ? B->ls_table : -1;
    p.group_slices = t >= 0 ? kWaves * B->tab[t].spw : 0;
    p.groups = t >= 0 ? B->tab[t].ngroups : 0;
    p.uniform_groups = t >= 0 ? B->tab[t].uniform_groups : 0;
    p.fused = t >= 0 && B->ls_fused ? 1 : 0;
    *props = p;
    return PRCG_OK;
}

prcg_status prcg_batch_set_fusion(prcg_batch B, int32_t fusion)
{
    if (!B) return fail(PRCG_EINVAL, "null batch");
    if (fusion < PRCG_BATCH_FUSION_AUTO || fusion > PRCG_BATCH_FUSION_ON)
        return fail(PRCG_EINVAL, "unknown fusion setting");
    HIP_TRY(hipSetDevice(B->A->device));
    HIP_TRY(hipStreamSynchronize(B->A->stream));
    B->force_fusion = fusion;
    B->ls_table = -1;
    B->ls_fused = false;
    for (auto& m : B->mode) m = 0;
    for (auto& g : B->ls_graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    return PRCG_OK;
}

prcg_status prcg_batch_set_mode(prcg_batch B, int32_t mode)
{
    if (!B) return fail(PRCG_EINVAL, "null batch");
    if (mode < PRCG_BATCH_AUTO || mode > PRCG_BATCH_LOCKSTEP) return fail(PRCG_EINVAL, "unknown batch mode");
    B->mode_req = mode;
    for (auto& m : B->mode) m = 0;
    return PRCG_OK;
}

prcg_status prcg_batch_mode(prcg_batch B, prcg_variant v, int32_t* mode)
{
    if (!B || !mode) return fail(PRCG_EINVAL, "null argument");
    if (check_batch_variant(v) != PRCG_OK) return PRCG_EINVAL;
    *mode = B->mode[v == PRCG_HS ? 0 : (v == PRCG_PR || v == PRCG_M) ? 1 : 2];
    return PRCG_OK;
}

void prcg_batch_destroy(prcg_batch B) { free_batch(B); }

}  // extern "C"
