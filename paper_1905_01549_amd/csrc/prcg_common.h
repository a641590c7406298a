// Internal declarations shared by the libprcg translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace prcg {

constexpr int kBlock = 256;     // threads per workgroup of every row-parallel kernel
constexpr int kWaves = kBlock / 64;
constexpr int kSlice = 64;      // SELL slice height: one wavefront, one row per lane
constexpr int kGroupRows = kBlock;  // rows handled by one workgroup step (4 slices)
constexpr int kMaxDots = 5;
constexpr int kMaxGrid = 16384;  // largest workgroup count of the row-parallel kernels

enum Variant {
    kHS = 0,
    kPR = 1,
    kPipePR = 2,
    kM = 3,
    kPipeM = 4,
    kGV = 5,
    kPRNoRecompute = 6,
    kPipeNoWRecompute = 7,
    kCG = 8,
    kPRUnsimplified = 9
};
constexpr int kNumVariants = 10;

__host__ __device__ inline bool is_pipe(int variant)
{
    return variant == kPipePR || variant == kPipeM || variant == kPipeNoWRecompute;
}

// How a one-reduction variant forms nu and nu' (step_one_reduction):
// 0 PR (eq. nuk_simplified), 1 Meurant (nu' = -nu + alpha^2 gamma),
// 2 PR without the recompute (nu_k := nu'_k, eq. nuk_norecomp),
// 3 PR with the four-term eq. nuk (delta = <s~, r> of its own).
enum NuForm { kFormPR = 0, kFormMeurant = 1, kFormNoRecompute = 2, kFormUnsimplified = 3 };
__host__ __device__ inline int nu_form(int variant)
{
    if (variant == kM || variant == kPipeM) return kFormMeurant;
    if (variant == kPRUnsimplified) return kFormUnsimplified;
    return variant == kPRNoRecompute ? kFormNoRecompute : kFormPR;
}

// The variants that run PR-CG's kernels (Alg. 2 with one nu' form or another).
__host__ __device__ inline bool is_pr_family(int variant)
{
    return variant == kPR || variant == kM || variant == kPRNoRecompute || variant == kPRUnsimplified;
}
enum Status { kOK = 0, kNotConverged = 1, kBreakdown = 2 };

// Scalar state of a solve, resident in device memory.  Two copies are kept
// and each kernel that advances the state reads one and writes the other, so
// no workgroup ever reads a copy that another workgroup of the same kernel
// is writing.
struct alignas(128) State {
    double alpha;        // alpha_k (used by the vector updates of iteration k+1)
    double beta;         // beta_{k+1}
    double nu;           // nu_k (the recomputed value)
    double mu, sigma, gamma, rr;
    double nup;          // nu'_{k+1}
    double bnorm;        // ||b||
    double tol;
    double relres_true;  // ||b - A x|| / ||b||, filled at exit
    int32_t k;           // index of the last reduction processed
    int32_t done;        // 1 once the solve has ended
    int32_t status;      // Status
    int32_t last;        // 1 when nu' <= 0 made the next iteration the final one
    int32_t maxit;
    int32_t zero_x;      // b = 0: the returned x is 0
    int32_t spare0, spare1;
    double spare2;  // no padding: every byte is a scalar field, so copies of
                    // the state stay in registers
};
static_assert(sizeof(State) == 128, "State fills its 128-byte alignment");

// SELL-64 matrix: rows are cut into slices of 64 (one wavefront, one row
// per lane); slot j of row 64 s + l is at slice_ptr[s] + j stride_s + l.
// Consecutive slices of one width and kind are stored as runs of up to
// kRunSlices slices, slot-major: slot j of every slice of the run side by
// side, so the slices that run at the same time read neighbouring memory;
// slice_shape[s] = width | (run length << 16), stride_s = 64 x run length.
// An offset-aligned slice (slice_meta[s] >= 0)
// stores no column indices: slot j of row r holds the entry at column
// r + soff[slice_meta[s] + j] or a zero.  A packed slice (slice_meta[s] < 0)
// holds each row's j-th entry in slot j with its column in col; short rows
// are padded with zeros whose column is the row itself.
struct SellView {
    const int64_t* slice_ptr;    // [nslices + 1]
    const int32_t* slice_meta;   // [nslices]
    const int32_t* slice_shape;  // [nslices]
    const int32_t* soff;
    const int32_t* col;
    const double* val;
    int64_t n;
    int64_t nslices;
    // Offset-aligned slices from stream_from on are read with nontemporal
    // value loads, so that a matrix larger than the last-level cache streams
    // past it and the first kCachedValueBytes of values stay resident from
    // one product to the next (nslices or more: every slice is cached).
    int64_t stream_from = INT64_MAX;
    int32_t runs = 0;  // 1 when some slice is stored in a run of more than one
};

// Matrix values kept cacheable before loads turn nontemporal: all of them
// up to kCachedValueBytes, half of the MI355X's 256 MB last-level cache, so
// the vectors of an iteration fit beside them; of a larger matrix, only the
// first kCachedPrefixBytes (measured on a 27-point matrix of 885 MB:
// prefixes of 64, 128 and 192 MB gave products of 205, 199 and 217 us
// against 230 us with every load cached and 213 us with none; once the
// update kernel swept the rows in reverse, a 96 MB prefix gave PR-CG 215
// against 218 us per iteration with 128 MB, while the 118 MB matrix of the
// 128^3 problem ran 11% slower when only 96 MB of it were cached).
constexpr int64_t kCachedValueBytes = (int64_t)128 << 20;
constexpr int64_t kCachedPrefixBytes = (int64_t)96 << 20;
// The cacheable prefix of a matrix whose values take `total` bytes.
inline int64_t cached_value_bytes(int64_t total)
{
    return total <= kCachedValueBytes ? total : kCachedPrefixBytes;
}

// Slices per run of the SELL-64 layout (measured on MI355X, streaming the
// 885 MB of a 27-point matrix: runs of 64 slices 6% faster than single
// slices, runs of 640 or more slower than single slices).  Matrices of
// fewer than kMaxGrid row groups keep single slices.
constexpr int kRunSlices = 64;
__host__ __device__ inline int shape_width(int32_t sh) { return sh & 0xffff; }
__host__ __device__ inline int shape_stride(int32_t sh) { return (sh >> 16) * kSlice; }

// Vector-CSR matrix for long rows: L lanes per row, CSR arrays as given.
struct CsrView {
    const int32_t* row_ptr;
    const int32_t* col;
    const double* val;
    int64_t n;
};

// Work split of the row-parallel kernels: G workgroups; workgroup b owns a
// contiguous run of 256-row groups.  Runs are assigned so that the
// workgroups an XCD receives (b mod 8) own neighbouring runs.
struct Split {
    int64_t n;      // rows
    int G;          // workgroups (partial sums per reduction)
    int Gs;         // stride between reduction values in a partials buffer
    int64_t ngroups;
    int lanes;      // 1 = SELL-64, else lanes per row of vector CSR
    int stage2;     // two-pass, per variant (bit 0: HS, 1: PR/M, 2: pipe): a
                    // one-workgroup kernel reduces the partials before the
                    // kernel that needs the totals
    int lastwg;     // two-pass: the last workgroup of the kernel that writes
                    // the partials reduces them (ticket counter)
                    // (neither: every workgroup of the consuming kernel
                    // reduces them redundantly)
    int fused;      // fused kernels (SELL-64 only): bit 0 HS/PR forms, bit 1 pipe-PR forms; 0 = two-pass
    int textbook;   // 1 = HS-CG as one kernel per algorithm line
    int textbook_pre;  // preconditioned (the textbook kernel list depends on it)
};

inline bool stage2_of(const Split& sp, int variant)
{
    const int bit = variant == kHS ? 1 : (is_pipe(variant) ? 4 : 2);
    return (sp.stage2 & bit) != 0;
}

// The fused structure covers HS, PR, pipe-PR and their forms; GV-CG, CG-CG,
// the no-w-recompute ablation and PR-CG with eq. nuk always run two-pass.
// sp.fused bit 0: HS-CG and the PR-CG forms fused; bit 1: pipe-PR-CG too.
inline bool uses_fused(int variant, const Split& sp)
{
    if (!sp.fused || variant == kGV || variant == kPipeNoWRecompute || variant == kCG || variant == kPRUnsimplified)
        return false;
    return is_pipe(variant) ? (sp.fused & 2) != 0 : (sp.fused & 1) != 0;
}

// ---- setup kernels (kernels_setup.hip) ----
hipError_t launch_validate(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                           int32_t* flags, int32_t* maxlen, hipStream_t st);
hipError_t launch_jacobi(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                         double* d, int32_t* flags, hipStream_t st);
// Slice planning / filling.  row0/nrows (nullable) give each slice's first
// row and row count; when null, slice s covers rows 64 s .. 64 s + 63.
hipError_t launch_slice_plan(int64_t n, int64_t nslices, const int32_t* row_ptr, const int32_t* col,
                             const int64_t* row0, const int32_t* nrows, int32_t* width, int32_t* aligned,
                             hipStream_t st);
hipError_t launch_fill_sell(int64_t n, int64_t nslices, const int32_t* row_ptr, const int32_t* col,
                            const double* val, const int64_t* row0, const int32_t* nrows,
                            const int64_t* slice_ptr, const int32_t* slice_meta, const int32_t* slice_shape,
                            int32_t* soff, int32_t* scol, double* sval, int write_cols, hipStream_t st);
hipError_t launch_block_check(int64_t n, const int32_t* row_ptr, const int32_t* col,
                              const int32_t* row_sys, const int64_t* sys_off, int32_t* flags, hipStream_t st);
hipError_t launch_outer_csr(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* lam,
                            const double* x, double* g, double mean_row, hipStream_t st);
hipError_t launch_spmv(const SellView* sell, const CsrView* csr, const Split& sp, const double* x,
                       double* y, hipStream_t st);

// ---- iteration kernels (kernels_iter.hip) ----
struct Vecs {
    double *x, *r, *rt, *p, *s, *st, *w, *u;
    const double* d;  // Jacobi reciprocal diagonal or nullptr
    // pipe-PR-CG block vectors (two-pass kernels): zr[i] = (s~_i, r~_i) and
    // uw[i] = (u_i, w_i), so that the pair of products [A s~, A r~] gathers
    // one 16-byte entry per stored matrix entry (Section 5 reads A once for
    // the block vector [s, r]).
    double2* zr;
    double2* uw;
    // GV-CG: t = A w~ and the stored w~ = M^{-1} w (the product's input);
    // pipe-PR-CG without the recompute of w keeps its recurrence w~' in wt
    double *t, *wt;
};

struct Bufs {
    State* S[2];
    double* hist;
    double* PS;   // [mu, sigma, gamma, nu, rr] partials
    double* PN;   // [nu, rr] partials when PR's update kernel produces them
    double* PD;   // [delta] partials (PR-CG with eq. nuk and a preconditioner)
    double* PW;   // [value][kWaves] lane-group sums of a split stage 2
    double* PU;   // [nu, rr] partials (HS)
    double* PB;   // [bb] or [tt] partials
    double* PS2;  // second copy of PS (fused kernels alternate between the two)
    int* ticket;  // workgroup counter of the last-workgroup reduction (0 between kernels)
};

hipError_t launch_init(int variant, int pre, const SellView* sell, const CsrView* csr, const Split& sp,
                       const Vecs& v, const Bufs& B, const double* b, const double* x0, double tol,
                       int32_t maxit, hipStream_t st);
// Number of kernels per iteration and their launch; `cur` is the state copy
// that holds the current state and is updated.
int iter_kernel_count(int variant, const Split& sp);
const char* iter_kernel_name(int variant, const Split& sp, int j);
// Optional dispatch timestamps for one launch.
struct LaunchEvents {
    hipEvent_t start;
    hipEvent_t stop;
};
hipError_t launch_iter_kernel(int variant, int pre, int j, int& cur, const SellView* sell,
                              const CsrView* csr, const Split& sp, const Vecs& v, const Bufs& B,
                              hipStream_t st, const LaunchEvents* ev = nullptr, int p_copy = 0);
hipError_t launch_final(const SellView* sell, const CsrView* csr, const Split& sp, const Vecs& v,
                        const Bufs& B, int cur, const double* b, double* xout, hipStream_t st);

}  // namespace prcg
