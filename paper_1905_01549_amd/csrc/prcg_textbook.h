// Textbook (kernel-per-line) HS-CG: the unfused baseline.
#pragma once

#include "prcg_common.h"

namespace prcg {

int textbook_kernel_count(int pre);
const char* textbook_kernel_name(int pre, int j);
hipError_t launch_textbook_kernel(int pre, int j, int& cur, const SellView* sell, const CsrView* csr,
                                  const Split& sp, const Vecs& v, const Bufs& B, hipStream_t st,
                                  const LaunchEvents* ev);

}  // namespace prcg
