// Device-side constants and cross-file declarations of the HIP kernels' drivers.
#pragma once

#include "hf_internal.h"

namespace hf {

constexpr int PANEL_NB = 32;  // pivots per panel of the F11 factorization

template <class T>
void step1(hf_ctx* ctx, const double* values, hipStream_t s);

// inverses of the 64x64 diagonal blocks of L11, needed by precond_apply
template <class T>
void prepare_solve(hf_ctx* ctx, hipStream_t s);

// Q^{-1} of Sec. 3.2: Y = (L D L^T)^{-1} R on the moderate part, R and Y row-major
// n x m in elimination order, FP64; factors in T.
template <class T>
void precond_apply(hf_ctx* ctx, int m, const double* R, double* Y, hipStream_t s);

}  // namespace hf
