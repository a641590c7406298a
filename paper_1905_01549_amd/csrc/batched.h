// Batched persistent solver: layout and launcher.
#pragma once

#include "prcg_common.h"

namespace prcg {

// Slices of the batched layout never cross a system boundary: system s owns
// slices [sys_slice0[s], sys_slice0[s+1]); slice q starts at row
// slice_row0[q] and holds slice_nrows[q] <= 64 rows.
struct BatchView {
    SellView A;
    const int64_t* slice_row0;
    const int32_t* slice_nrows;
    const int64_t* sys_row0;    // [nsys + 1]
    const int64_t* sys_slice0;  // [nsys + 1]
    const int32_t* order;       // systems, largest first
    int32_t nsys;
};

// Row groups of the lockstep solver: up to kWaves spw consecutive
// slices (rows row0 .. row0 + nrows - 1) of one system, whose rows are
// lo .. hi; system s owns groups [sys_grp0[s], sys_grp0[s+1]).  A uniform
// group (off >= 0) holds offset-aligned slices of one width (1 ..
// kUniformMaxWidth) and one list of column offsets, o[0 .. width - 1] (also
// at soff[off ..]), stored one after another from value slot 64 vrow: the
// product reads everything about it from this record, so its gathers need
// no other load first.  Other groups (off < 0) hold any slices and take the
// general slice-by-slice product.  (Rows, slices and value slots / 64 fit
// int32: column indices are int32.)
constexpr int kLockstepSlices = 16;  // the default group: 4 slices per wavefront
constexpr int kUniformMaxWidth = 8;
struct Group {
    int32_t slice0;
    int32_t row0;
    int32_t sys;
    int32_t nsl;
    int32_t nrows;
    int32_t lo;
    int32_t hi;
    int32_t off;    // uniform groups: first of the slices' common offsets in soff; -1 otherwise
    int32_t width;  // uniform groups: slots per row
    int32_t vrow;   // uniform groups: the first slice's values start at slot 64 vrow
    int32_t diag;   // uniform groups: the slot whose offset is 0, or -1
    int32_t flags;  // uniform groups: kGroupShift when slots diag - 1 and diag + 1 hold offsets -1 and +1
    int32_t o[kUniformMaxWidth];  // uniform groups: the column offsets
};
constexpr int32_t kGroupShift = 1;
static_assert(sizeof(Group) == 80, "five 16-byte loads per group");
struct GroupView {
    const Group* grp;          // [ngroups]
    const int64_t* sys_grp0;   // [nsys + 1]
    int64_t ngroups;
    int32_t* gdone;            // [ngroups]: 1 once the group's system has finished
    int32_t spw;               // slices per wavefront (2, 4 or 8): groups hold kWaves spw slices
    int32_t uwidth;            // every group uniform: 3, 5 or 7, the least at or above the widest; else 0
    int32_t* ticket;           // [nsys]: the fused iteration's stage-2 tickets (0 between launches)
    int32_t span;              // the largest stencil span of a group (offset 0 included)
};

// The lockstep vectors one fused iteration reads or writes besides x
// (rt: r~, with a preconditioner only).
struct LsVecs {
    double* r;
    double* p;
    double* s;
    double* rt;
};
// LDS of one fused workgroup, in doubles: the window of p' (the group's
// rows plus the table's largest stencil span, i.e. largest minus smallest
// column offset of a group, offset 0 included) and r' (and r~' with a
// preconditioner) of the group's rows.  A table may run fused when this
// fits the 64 KB a workgroup may hold with a preconditioner.
__host__ __device__ constexpr int fused_lds_doubles(int group_rows, int span, bool pre)
{
    return group_rows * (pre ? 3 : 2) + span;
}
constexpr int kFuseLdsDoubles = 65536 / 8;

// Lockstep PR-CG / M-CG (variant kPR or kM): the initialisation (three
// launches), then `iterations` iterations of three launches each and the
// count of running systems into *active.  P: 6 * ngroups doubles; S: nsys
// states.  All launches go on `st` and may be captured in a graph.
hipError_t launch_lockstep_init(const BatchView& B, const GroupView& gv, const Vecs& v, const double* b, State* S,
                                double* P, double tol, int maxit, int variant, int pre, int32_t* iters,
                                int32_t* status, hipStream_t st);
// fused: each iteration as one launch of k_ls_fused, whose last workgroup
// of each system takes the system's stage 2 (uniform groups (uwidth > 0)
// whose window fits kFuseLdsDoubles, 2 or 4 slices per wavefront, an even number
// of iterations: r (r~ with a preconditioner, r then staying in place), p
// and s alternate between (v.r or v.rt, v.p, v.s) and (v.w, v.u, v.st), and
// the initialisation leaves them in the first).
hipError_t launch_lockstep_iterations(const BatchView& B, const GroupView& gv, const Vecs& v, State* S, double* P,
                                      int iterations, int variant, int pre, bool fused, int32_t* iters,
                                      int32_t* status, int32_t* active, hipStream_t st);

// Reset the queue and launch the persistent kernel (nt threads per
// workgroup: 256, 512 or 1024; grid workgroups; q = 1 or 2 slices
// multiplied together per wavefront).  Both launches go on `st` and may be
// captured in a graph.
hipError_t launch_batch(const BatchView& B, const Vecs& v, const double* b, double tol, int maxit, int variant,
                        int pre, int nt, int grid, int q, int32_t* queue, int32_t* iters, int32_t* status,
                        hipStream_t st);

}  // namespace prcg
