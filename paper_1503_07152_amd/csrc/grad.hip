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
// One wave per (node, part) product out = a b^T (a, b: R x c, column-major,
// ld R), with no LDS and no barrier: NT x NT tiles of 16 x 16 held in
// registers, the operands of each 4-deep K-step read straight from global
// memory (16 consecutive entries per lane group).
template <class T, int NT>
__global__ __launch_bounds__(256) void k_grad_node(const Node* nodes, const int32_t* list,
                                                   int nlist, int R, int c, const T* QH,
                                                   const T* UH, const T* GU, const T* GQ, T* gB,
                                                   T* gUt, T* gVt) {
  typedef MfTraits<T> Tr;
  const int lane = threadIdx.x & 63;
  const int64_t prod = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (prod >= (int64_t)nlist * 5) return;
  const int v = list[prod / 5];
  const int part = (int)(prod % 5);
  const Node nd = nodes[v];
  const int64_t blk = (int64_t)v + 1;
  T* out = nullptr;    // the product's block
  T* out0 = nullptr;   // the root's block 0 (zeros)
  int64_t ld = R;
  const T* a = nullptr;   // null: a zero block
  const T* b = nullptr;
  if (part == 0) {
    if (!gB) return;
    // gB[v] = g(uh)_sib qh_v^T
    out = gB + blk * R * R;
    if (nd.parent < 0) {
      out0 = gB;
    } else {
      a = GU + (int64_t)nd.sib * R * c;
      b = QH + (int64_t)v * R * c;
    }
  } else {
    // parts 1 / 2: gUt half of child (side 0 / 1), parts 3 / 4: gVt half
    const bool want_u = part <= 2;
    const int side = (part - 1) % 2;
    T* gt = want_u ? gUt : gVt;
    if (!gt) return;
    out = gt + blk * 2 * R * R + side * R;
    ld = 2 * R;
    if (nd.parent < 0) out0 = gt + side * R;
    if (nd.left >= 0 && nd.parent >= 0) {
      const int ch = side == 0 ? nd.left : nd.right;
      a = (want_u ? GU : QH) + (int64_t)ch * R * c;
      b = (want_u ? UH : GQ) + (int64_t)v * R * c;
    }
  }
  typename Tr::acc_t acc[NT][NT];
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) acc[ti][tj] = typename Tr::acc_t{0, 0, 0, 0};
  const int li = lane & 15, lk = lane >> 4;
  if (a) {
    // four K-steps per round: every load of the round (at clamped, always
    // valid indices; entries outside R x c zeroed after the load) is issued
    // before its MFMAs, so that they are in flight together
    constexpr int KS = 4;
    for (int k0 = 0; k0 < c; k0 += 4 * KS) {
      T av[KS][NT], bv[KS][NT];
#pragma unroll
      for (int s4 = 0; s4 < KS; ++s4) {
        const int k = k0 + 4 * s4 + lk;
        const int kc = min(k, c - 1);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int ic = min(16 * t + li, R - 1);
          av[s4][t] = a[ic + (int64_t)kc * R];
          bv[s4][t] = b[ic + (int64_t)kc * R];
        }
      }
#pragma unroll
      for (int s4 = 0; s4 < KS; ++s4) {
        const int k = k0 + 4 * s4 + lk;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const bool ok = 16 * t + li < R && k < c;
          av[s4][t] = ok ? av[s4][t] : T(0);
          bv[s4][t] = ok ? bv[s4][t] : T(0);
        }
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
          for (int tj = 0; tj < NT; ++tj)
            acc[ti][tj] = Tr::step(av[s4][ti], bv[s4][tj], acc[ti][tj]);
      }
    }
  }
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 16 * ti + Tr::row(lane, q), j = 16 * tj + li;
        if (i < R && j < R) {
          out[i + (int64_t)j * ld] = acc[ti][tj][q];
          if (out0) out0[i + (int64_t)j * ld] = T(0);
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
    const dim3 grid((unsigned)(((int64_t)nlist * 5 + 3) / 4));
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, d_nodes, nodes_list, nlist, R, c, QH, UH,
                         GU, GQ, gB, gUt, gVt);
      KCHK();
    };
    if (R <= 16) go(k_grad_node<T, 1>);
    else if (R <= 32) go(k_grad_node<T, 2>);
    else if (R <= 48) go(k_grad_node<T, 3>);
    else HM_THROW(HM_ERR_UNSUPPORTED, "backward: padded rank %d > 48", R);
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
