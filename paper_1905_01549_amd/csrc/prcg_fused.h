// Fused iteration kernels (SELL-64 layout): double-buffered vectors.
#pragma once

#include "prcg_common.h"

namespace prcg {

// Copies [0] and [1] of the vectors the fused kernels double-buffer;
// iteration k reads copy k mod 2 and writes the other.  Vectors updated in
// place use copy [0].
struct FusedVecs {
    double* x;
    double* r[2];
    double* rt[2];
    double* p[2];
    double* s[2];
    double* st[2];
    double* w[2];
    double* u[2];
    const double* d;
};

// Launch kernel j of a fused iteration (PR, pipe-PR: j = 0 only; HS: j = 1,
// the first HS kernel is the two-pass k_hs_xr).  `it` is the iteration's
// position (its parity selects the buffer copies); PS2 is the second copy
// of the partials buffer.
hipError_t launch_fused_kernel(int variant, int pre, int j, int it, int& cur, const SellView& S, const Split& sp,
                               const FusedVecs& f, const Bufs& B, double* PS2, hipStream_t st,
                               const LaunchEvents* ev);

}  // namespace prcg
