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

// Reset the queue and launch the persistent kernel (nt threads per
// workgroup: 256, 512 or 1024; grid workgroups).  Both launches go on `st`
// and may be captured in a graph.
hipError_t launch_batch(const BatchView& B, const Vecs& v, const double* b, double tol, int maxit, int variant,
                        int pre, int nt, int grid, int32_t* queue, int32_t* iters, int32_t* status, hipStream_t st);

}  // namespace prcg
