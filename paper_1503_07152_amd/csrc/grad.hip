// Backward of the compressed apply y = A_H x (not in the paper; the
// derivative of Fig. 7 + D with respect to its inputs).
//
// With the forward expansions qh_v (outgoing) and uh_v (incoming) and the
// expansions of the adjoint apply of gy -- whose upward pass yields
// g(uh)_v = U^T-side accumulations and whose downward pass yields g(qh)_v --
// every generator gradient is an outer product over the right-hand sides:
//   gD_t  = gy_t x_t^T                     gU_t = gy_t uh_t^T     (leaves)
//   gV_t  = x_t g(qh)_t^T                  gB[v] = g(uh)_sib(v) qh_v^T
//   gUt_t(child a) = g(uh)_a uh_t^T        gVt_t(child a) = qh_a g(qh)_t^T
// and gx = A_H^* gy is the adjoint apply itself.
#include "grad.h"
#include "tile_mfma.h"

namespace hm {

constexpr int GM = MF_T, GN = MF_T;

// Leaves: row tiles of gU, gV and gD.
template <class T>
__global__ __launch_bounds__(256) void k_grad_leaf(const Node* nodes, const int32_t* leaves,
                                                   int R, int c, const T* X, int64_t ldx,
                                                   const T* GY, int64_t ldgy, const T* UH,
                                                   const T* GQ, T* gU, T* gV, T* gD, int64_t ld,
                                                   int64_t ldd) {
  __shared__ T smem[mf_smem_elems<T>()];
  const int g = leaves[blockIdx.y];
  const Node nd = nodes[g];
  const int64_t i0 = nd.lo + (int64_t)blockIdx.x * GM;
  if (i0 >= nd.hi) return;
  const int M = (int)min<int64_t>(GM, nd.hi - i0);
  const int nt = (int)(nd.hi - nd.lo);
  const int part = blockIdx.z;  // 0: gU, 1: gV, 2..: column tiles of gD
  MfAcc<T> acc;
  acc.zero();
  if (part == 0) {
    if (!gU || nd.level == 0) return;
    // gU(rows) = GY(rows, :) UH_g^T  (UH_g is R x c, ld R)
    mf_tile<T>(M, R, c, GY + i0, 1, ldgy, UH + (int64_t)g * R * c, R, 1, acc, smem);
    mf_store_lds<T>(M, R, gU + i0, ld, acc, T(1), T(0), smem);
  } else if (part == 1) {
    if (!gV || nd.level == 0) return;
    mf_tile<T>(M, R, c, X + i0, 1, ldx, GQ + (int64_t)g * R * c, R, 1, acc, smem);
    mf_store_lds<T>(M, R, gV + i0, ld, acc, T(1), T(0), smem);
  } else {
    if (!gD) return;
    const int j0 = (part - 2) * GN;
    if (j0 >= nt) return;
    // gD(rows, j) = sum_c GY(row, c) X(lo + j, c)
    mf_tile<T>(M, nt - j0, c, GY + i0, 1, ldgy, X + nd.lo + j0, ldx, 1, acc, smem);
    mf_store_lds<T>(M, min(GN, nt - j0), gD + i0 + (int64_t)j0 * ldd, ldd, acc, T(1), T(0), smem);
  }
}

// Nodes: gB for every non-root node, gUt / gVt halves for children of internal nodes.
// Output blocks are heap-indexed in the flat layout: node g -> block g + 1 of
// its tree (single-tree handles).  The blocks no node owns (gB of the root,
// gUt / gVt of the root and of the leaves, and block 0) are written as zeros.
template <class T>
__global__ __launch_bounds__(256) void k_grad_node(const Node* nodes, const int32_t* list, int R,
                                                   int c, const T* QH, const T* UH,
                                                   const T* GU, const T* GQ, T* gB, T* gUt,
                                                   T* gVt) {
  __shared__ T smem[mf_smem_elems<T>()];
  const int v = list[blockIdx.x];
  const Node nd = nodes[v];
  const int part = blockIdx.y;
  const int64_t blk = (int64_t)v + 1;
  MfAcc<T> acc;
  acc.zero();
  const T* qh = QH + (int64_t)v * R * c;
  if (part == 0) {
    if (!gB) return;
    if (nd.parent < 0) {
      mf_store<T>(R, R, gB + blk * R * R, R, acc, T(1), T(0));
      mf_store<T>(R, R, gB, R, acc, T(1), T(0));
      return;
    }
    // gB[v] = g(uh)_sib qh_v^T
    mf_tile<T>(R, R, c, GU + (int64_t)nd.sib * R * c, 1, R, qh, R, 1, acc, smem);
    mf_store<T>(R, R, gB + blk * R * R, R, acc, T(1), T(0));
  } else {
    // part 1: gUt half of child (side 0/1), part 3/4: gVt half
    const bool want_u = part <= 2;
    const int side = (part - 1) % 2;
    if (want_u ? !gUt : !gVt) return;
    if (nd.left < 0 || nd.parent < 0) {
      T* gt = want_u ? gUt : gVt;
      mf_store<T>(R, R, gt + blk * 2 * R * R + side * R, 2 * R, acc, T(1), T(0));
      if (nd.parent < 0) mf_store<T>(R, R, gt + side * R, 2 * R, acc, T(1), T(0));
      return;
    }
    const int a = side == 0 ? nd.left : nd.right;
    if (want_u) {
      mf_tile<T>(R, R, c, GU + (int64_t)a * R * c, 1, R, UH + (int64_t)v * R * c, R, 1,
                         acc, smem);
      mf_store<T>(R, R, gUt + blk * 2 * R * R + side * R, 2 * R, acc, T(1), T(0));
    } else {
      mf_tile<T>(R, R, c, QH + (int64_t)a * R * c, 1, R, GQ + (int64_t)v * R * c, R, 1,
                         acc, smem);
      mf_store<T>(R, R, gVt + blk * 2 * R * R + side * R, 2 * R, acc, T(1), T(0));
    }
  }
}

template <class T>
void launch_grad(const Node* d_nodes, const int32_t* leaves, int nleaves, int64_t max_leaf,
                 int nmax, const int32_t* nodes_list, int nlist, int R, int c, const T* X,
                 int64_t ldx, const T* GY, int64_t ldgy, const T* QH, const T* UH, const T* GU,
                 const T* GQ, T* gU, T* gV, T* gUt, T* gVt, T* gB, T* gD, int64_t ld, int64_t ldd,
                 hipStream_t s) {
  if (nleaves > 0) {
    const int parts = 2 + (nmax + GN - 1) / GN;
    hipLaunchKernelGGL(k_grad_leaf<T>, dim3((unsigned)((max_leaf + GM - 1) / GM), nleaves, parts),
                       dim3(256), 0, s, d_nodes, leaves, R, c, X, ldx, GY, ldgy, UH, GQ, gU, gV,
                       gD, ld, ldd);
    KCHK();
  }
  if (nlist > 0 && R > 0) {
    hipLaunchKernelGGL(k_grad_node<T>, dim3(nlist, 5), dim3(256), 0, s, d_nodes, nodes_list, R, c,
                       QH, UH, GU, GQ, gB, gUt, gVt);
    KCHK();
  }
}

#define INST(T)                                                                                 \
  template void launch_grad<T>(const Node*, const int32_t*, int, int64_t, int, const int32_t*,  \
                               int, int, int, const T*, int64_t, const T*, int64_t, const T*,   \
                               const T*, const T*, const T*, T*, T*, T*, T*, T*, T*, int64_t,   \
                               int64_t, hipStream_t);
INST(double)
INST(float)

}  // namespace hm
