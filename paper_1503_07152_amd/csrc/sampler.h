// Built-in sampling operators (kernel matrix on points, dense matrix) on MFMA.
#pragma once
#include "common.h"

namespace hm {

constexpr int SMP_MAXC = 128;       // columns per sampler launch, F64 / F32 forms
constexpr int SMP_MAXC_BF16 = 288;  // BF16 form (entries evaluated once for all columns)
constexpr int SMP_NARROW_BF16 = 128;  // widest BF16 call of the narrow form (split over K)

int sampler_max_cols(int mode);

int sampler_bk(int mode);
size_t sampler_pack_bytes(int mode, int64_t n, int c);
// Y(0:n, 0:c) = A X.  mode: 0 F64, 1 F32, 2 BF16.  src: 0 log kernel,
// 1 near-singular kernel 1/(|x-y| + kp), 2 dense matrix Ad, 3 dense Ad^T
// (dense: FP64 only).
// work: sampler_pack_bytes(mode, n, c) bytes.  c <= sampler_max_cols(mode).
void sampler_apply(int mode, int src, int64_t n, int c, const double* pts, double kp,
                   const double* Ad, int64_t lda, const double* X, int64_t ldx, double* Y,
                   int64_t ldy, void* work, hipStream_t s);

}  // namespace hm
