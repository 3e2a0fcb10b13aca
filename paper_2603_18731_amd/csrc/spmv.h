// Matrix-free SpMV launch for one key width (Methods, Matrix evaluation, matrix-free).  Each
// width's kernels are instantiated in a translation unit of their own (spmv_w*.hip).
#pragma once

#include "common.h"

namespace qsd {
// Launches Y = H X for nvec (1..16; 1..4 complex) interleaved vectors of element type ET on
// an operator whose keys have Wp padded words.
template <int Wp, class ET, bool CPLX>
void spmv_dispatch(const qsd_ham *h, const void *x, int64_t ldx, void *y, int64_t ldy, int nvec, hipStream_t st);
}  // namespace qsd
