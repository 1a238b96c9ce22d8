// Backward of the compressed apply (generator gradients from expansions).
#pragma once
#include "common.h"

namespace hm {

// X, GY: inputs (N x c); QH/UH: forward outgoing/incoming expansions per node
// (R x c, ld R); GU/GQ: adjoint-apply expansions of GY (g(uh), g(qh)).
// Outputs in the flat heap-indexed layout (any may be null): gU, gV (N x R,
// ld), gUt, gVt (blocks 2R x R), gB (blocks R x R), gD (N x nmax, ldd).
template <class T>
void launch_grad(const Node* d_nodes, const int32_t* leaves, int nleaves, int64_t max_leaf,
                 int nmax, const int32_t* nodes_list, int nlist, int R, int c, const T* X,
                 int64_t ldx, const T* GY, int64_t ldgy, const T* QH, const T* UH, const T* GU,
                 const T* GQ, T* gU, T* gV, T* gUt, T* gVt, T* gB, T* gD, int64_t ld, int64_t ldd,
                 hipStream_t s);

}  // namespace hm
