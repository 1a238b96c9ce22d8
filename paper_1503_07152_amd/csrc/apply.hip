// Forest apply of A^(m) (Fig. 7) and the segmented transposed products.
#include <algorithm>

#include "apply.h"
#include "tile_mfma.h"

namespace hm {

void build_apply_lists(const Forest& f, const std::vector<int>& m, ApplyLists& out,
                       hipStream_t s) {
  std::vector<int32_t> front;
  std::vector<TreeOp> lvl1;
  int mmax = 0;
  for (int i = 0; i < (int)f.inst.size(); ++i) mmax = std::max(mmax, m[i]);
  std::vector<std::vector<TreeOp>> inter(std::max(mmax, 1));
  int64_t maxr = 0;
  for (int g = 0; g < (int)f.nodes.size(); ++g) {
    const Node& nd = f.nodes[g];
    const int mi = m[nd.inst];
    if (mi < 0) continue;
    if (nd.level == mi) {
      front.push_back(g);
      maxr = std::max<int64_t>(maxr, nd.hi - nd.lo);
    }
    const TreeOp op{g, nd.left, nd.right, nd.sib};
    if (nd.level >= 1 && nd.level < mi) inter[nd.level].push_back(op);
    if (nd.level == 1 && mi >= 1) lvl1.push_back(op);
  }
  out.nfront = (int)front.size();
  out.frontier = upload(front, s);
  out.max_rows = maxr;
  out.chunks = (int)std::max<int64_t>(1, (maxr + APPLY_CHUNK - 1) / APPLY_CHUNK);
  out.mmax = mmax;
  out.internal.clear();
  out.ninternal.assign(std::max(mmax, 1), 0);
  out.internal.resize(std::max(mmax, 1));
  for (int l = 1; l < mmax; ++l) {
    out.ninternal[l] = (int)inter[l].size();
    out.internal[l] = upload(inter[l], s);
  }
  out.nlevel1 = (int)lvl1.size();
  out.level1 = upload(lvl1, s);
}

constexpr int TM = MF_T, TN = MF_T;   // output tile of the MFMA products

template <class T>
__global__ __launch_bounds__(256) void k_leaf_up(const Node* nodes, const int32_t* front,
                                                 int chunks, const T* V, int64_t ldl, int R,
                                                 const T* X, int64_t ldx, int c, T* QH, T* P) {
  __shared__ T smem[mf_smem_elems<T>()];
  const int ch = blockIdx.x, fi = blockIdx.y, j0 = blockIdx.z * TN;
  const int g = front[fi];
  const Node nd = nodes[g];
  const int64_t r0 = nd.lo + (int64_t)ch * APPLY_CHUNK;
  const int K = (int)max<int64_t>(0, min<int64_t>(APPLY_CHUNK, nd.hi - r0));
  MfAcc<T> acc;
  acc.zero();
  if (nd.level > 0 && K > 0)
    mf_tile<T>(R, c - j0, K, V + r0, ldl, 1, X + r0 + (int64_t)j0 * ldx, 1, ldx, acc,
                       smem);
  T* out = chunks == 1 ? QH + (int64_t)g * R * c : P + ((int64_t)fi * chunks + ch) * R * c;
  mf_store<T>(R, c - j0, out + (int64_t)j0 * R, R, acc, T(1), T(0));
}

template <class T>
__global__ void k_chunk_reduce(const int32_t* front, int chunks, const T* P, int64_t n, T* QH,
                               T alpha, T beta, int64_t out_stride) {
  const int fi = blockIdx.y;
  const int g = front[fi];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    T s = T(0);
    for (int ch = 0; ch < chunks; ++ch) s += P[((int64_t)fi * chunks + ch) * n + e];
    T* o = QH + (int64_t)g * out_stride + e;
    *o = beta == T(0) ? alpha * s : alpha * s + beta * *o;
  }
}

// ---- tree sweeps ------------------------------------------------------------
// One node (and a tile of TRC columns) per workgroup: out (R x TRC) = A1 B1 +
// A2 B2 with R x R coefficient blocks A_h (strided: A_h(i, k) = a_h[i sai +
// k sak]) and expansions B_h (R x TRC, ld R), R <= HM_MAX_SAMPLES.  Every
// operand is staged in LDS in one round (no K loop over global memory: K <=
// 2 R_max), so a level costs one global round trip; K is padded with zeros
// to a multiple of 8 and the product runs 8 K-steps per batch of LDS loads.
// Thread (ti, tj) holds rows ti + 16 u and columns 2 tj, 2 tj + 1.
constexpr int TRM = HM_MAX_SAMPLES;   // largest padded rank
constexpr int TRC = 32;               // columns per workgroup
constexpr int TRK = 8;                // K-steps per batch

template <class T>
struct TreeSmem {
  T a[2 * TRM][TRM + 1];   // A(i, k) at a[k][i] (both halves stacked along k)
  T b[2 * TRM][TRC];       // B(k, j)
};

// Staging loops run over fixed trip counts (R <= 64 along the unit stride,
// four rows per pass of 256 threads): all of a thread's global loads are
// issued before the first LDS store, so a stage costs one memory latency
// rather than one per element.
template <class T>
__device__ __forceinline__ void stage_coef(int R, int k0, const T* a, int64_t sai, int64_t sak,
                                           TreeSmem<T>& sm) {
  static_assert(TRM <= 64, "one 64-lane row per coefficient column");
  const int tid = threadIdx.x;
  const int lo = tid & 63, hi = tid >> 6;
  constexpr int NQ = TRM / 4;
  T v[NQ];
  if (sai == 1) {   // i along the unit stride: lane lo takes row i = lo of columns k
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = hi + 4 * q;
      v[q] = (lo < R && k < R) ? a[lo + (int64_t)k * sak] : T(0);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = hi + 4 * q;
      if (lo < R && k < R) sm.a[k0 + k][lo] = v[q];
    }
  } else {          // k along the unit stride
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = hi + 4 * q;
      v[q] = (lo < R && i < R) ? a[(int64_t)i * sai + (int64_t)lo * sak] : T(0);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = hi + 4 * q;
      if (lo < R && i < R) sm.a[k0 + lo][i] = v[q];
    }
  }
}

template <class T, int NU>
__device__ __forceinline__ void tree_mac(int Kp, int ti, int tj, const TreeSmem<T>& sm,
                                         T (&acc)[3][2]) {
  for (int k0 = 0; k0 < Kp; k0 += TRK) {
    T av[TRK][NU], bv[TRK][2];
#pragma unroll
    for (int q = 0; q < TRK; ++q) {
#pragma unroll
      for (int u = 0; u < NU; ++u) av[q][u] = sm.a[k0 + q][ti + 16 * u];
      bv[q][0] = sm.b[k0 + q][2 * tj];
      bv[q][1] = sm.b[k0 + q][2 * tj + 1];
    }
#pragma unroll
    for (int q = 0; q < TRK; ++q)
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        acc[u][0] = fma(av[q][u], bv[q][0], acc[u][0]);
        acc[u][1] = fma(av[q][u], bv[q][1], acc[u][1]);
      }
  }
}

template <class T>
__device__ __forceinline__ void tree_product(int R, int nc, int nparts, const T* a1, int64_t sai1,
                                             int64_t sak1, const T* b1, const T* a2,
                                             int64_t sai2, int64_t sak2, const T* b2, T* out,
                                             TreeSmem<T>& sm) {
  const int tid = threadIdx.x;
  const int K = nparts * R;
  const int Kp = (K + TRK - 1) / TRK * TRK;
  stage_coef<T>(R, 0, a1, sai1, sak1, sm);
  if (nparts == 2) stage_coef<T>(R, R, a2, sai2, sak2, sm);
  for (int e = tid; e < (Kp - K) * TRM; e += 256) sm.a[K + e / TRM][e % TRM] = T(0);
  {
    // B (Kp x TRC, Kp <= 2 TRM = 96): lane kl = tid % 32 takes k = kl + 32 h,
    // column j = tid / 32 + 8 w
    static_assert(2 * TRM <= 96 && TRC == 32, "B staging covers 96 x 32");
    const int kl = tid & 31, jl = tid >> 5;
    T bv[3][4];
#pragma unroll
    for (int h = 0; h < 3; ++h)
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int k = kl + 32 * h, j = jl + 8 * w;
        const bool second = k >= R;
        const int kk = second ? k - R : k;
        T v = T(0);
        if (k < K && j < nc) v = second ? b2[kk + (int64_t)j * R] : b1[kk + (int64_t)j * R];
        bv[h][w] = v;
      }
#pragma unroll
    for (int h = 0; h < 3; ++h)
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int k = kl + 32 * h;
        if (k < Kp) sm.b[k][jl + 8 * w] = bv[h][w];
      }
  }
  __syncthreads();
  const int ti = tid & 15, tj = tid >> 4;
  T acc[3][2];
#pragma unroll
  for (int u = 0; u < 3; ++u) acc[u][0] = acc[u][1] = T(0);
  const int nu = (R + 15) / 16;
  if (nu == 3) tree_mac<T, 3>(Kp, ti, tj, sm, acc);
  else if (nu == 2) tree_mac<T, 2>(Kp, ti, tj, sm, acc);
  else tree_mac<T, 1>(Kp, ti, tj, sm, acc);
#pragma unroll
  for (int u = 0; u < 3; ++u)
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const int i = ti + 16 * u, j = 2 * tj + w;
      if (u < nu && i < R && j < nc) out[i + (int64_t)j * R] = acc[u][w];
    }
}

// Upward pass, one level: qh_t = Vt_t^T [qh_left; qh_right].
template <class T>
__global__ __launch_bounds__(256) void k_tree_up(const TreeOp* list, const T* Vt, int R, T* QH,
                                                 int c) {
  __shared__ TreeSmem<T> sm;
  const TreeOp op = list[blockIdx.x];
  const int j0 = blockIdx.y * TRC;
  const T* vt = Vt + (int64_t)op.t * 2 * R * R;
  tree_product<T>(R, min(TRC, c - j0), 2, vt, 2 * R, 1,
                  QH + (int64_t)op.left * R * c + (int64_t)j0 * R, vt + R, 2 * R, 1,
                  QH + (int64_t)op.right * R * c + (int64_t)j0 * R,
                  QH + (int64_t)op.t * R * c + (int64_t)j0 * R, sm);
}

// Incoming expansion of node a from its sibling s's outgoing one: forward
// uh_a = B[s] qh_s, adjoint uh_a = B[a]^T qh_s; below level 1 plus the
// parent's term Ut_t(half of a) uh_t.
template <class T>
__global__ __launch_bounds__(256) void k_root(const TreeOp* list, const T* B, int R, const T* QH,
                                              T* UH, int c, int adjoint) {
  __shared__ TreeSmem<T> sm;
  const TreeOp op = list[blockIdx.x];
  const int a = op.t, s = op.sib;
  const int j0 = blockIdx.y * TRC;
  const T* bm = adjoint ? B + (int64_t)a * R * R : B + (int64_t)s * R * R;
  tree_product<T>(R, min(TRC, c - j0), 1, bm, adjoint ? R : 1, adjoint ? 1 : R,
                  QH + (int64_t)s * R * c + (int64_t)j0 * R, bm, 0, 0, nullptr,
                  UH + (int64_t)a * R * c + (int64_t)j0 * R, sm);
}

template <class T>
__global__ __launch_bounds__(256) void k_tree_down(const TreeOp* list, const T* Ut, const T* B,
                                                   int R, const T* QH, T* UH, int c,
                                                   int adjoint) {
  __shared__ TreeSmem<T> sm;
  const TreeOp op = list[blockIdx.x];
  const int side = blockIdx.y;  // 0: left child, 1: right child
  const int j0 = blockIdx.z * TRC;
  const int a = side == 0 ? op.left : op.right, s = side == 0 ? op.right : op.left;
  const T* bm = adjoint ? B + (int64_t)a * R * R : B + (int64_t)s * R * R;
  tree_product<T>(R, min(TRC, c - j0), 2, Ut + (int64_t)op.t * 2 * R * R + side * R, 1, 2 * R,
                  UH + (int64_t)op.t * R * c + (int64_t)j0 * R, bm, adjoint ? R : 1,
                  adjoint ? 1 : R, QH + (int64_t)s * R * c + (int64_t)j0 * R,
                  UH + (int64_t)a * R * c + (int64_t)j0 * R, sm);
}

template <class T>
__global__ __launch_bounds__(256) void k_leaf_down(const Node* nodes, const int32_t* front,
                                                   const T* U, int64_t ldl, int R, const T* UH,
                                                   int c, const T* D, int64_t ldd, int adjoint,
                                                   const T* X, int64_t ldx, T* Y, int64_t ldy,
                                                   T alpha, T beta) {
  __shared__ T smem[mf_smem_elems<T>()];
  const int g = front[blockIdx.y];
  const Node nd = nodes[g];
  const int64_t i0 = nd.lo + (int64_t)blockIdx.x * TM;
  if (i0 >= nd.hi) return;
  const int M = (int)min<int64_t>(TM, nd.hi - i0);
  const int j0 = blockIdx.z * TN;
  const int N = c - j0;
  MfAcc<T> acc;
  acc.zero();
  if (nd.level > 0)
    mf_tile<T>(M, N, R, U + i0, 1, ldl, UH + (int64_t)g * R * c + (int64_t)j0 * R, 1, R,
                       acc, smem);
  if (D) {
    const int nt = (int)(nd.hi - nd.lo);
    const T* xb = X + nd.lo + (int64_t)j0 * ldx;
    if (!adjoint)
      mf_tile<T>(M, N, nt, D + i0, 1, ldd, xb, 1, ldx, acc, smem);
    else
      mf_tile<T>(M, N, nt, D + nd.lo + (i0 - nd.lo) * ldd, ldd, 1, xb, 1, ldx, acc, smem);
  }
  mf_store<T>(M, N, Y + i0 + (int64_t)j0 * ldy, ldy, acc, alpha, beta);
}

template <class T>
size_t apply_work_bytes(const Forest& f, const ApplyLists& al, int R, int c) {
  const size_t per = (size_t)R * c * sizeof(T);
  size_t b = 2 * per * f.nodes.size();
  if (al.chunks > 1) b += per * (size_t)al.nfront * al.chunks;
  return b + 256;
}

template <class T>
void apply_forest(const Node* d_nodes, const ApplyLists& al, const HbsView<T>& h, bool adjoint,
                  int c, const T* X, int64_t ldx, T* Y, int64_t ldy, T alpha, T beta, void* work,
                  size_t nnodes, hipStream_t s, bool expansions_only) {
  if (al.nfront == 0 || c <= 0) return;
  const int R = h.R;
  if (R > TRM) HM_THROW(HM_ERR_UNSUPPORTED, "apply: padded rank %d > %d", R, TRM);
  T* QH = static_cast<T*>(work);
  T* UH = QH + (size_t)R * c * nnodes;
  T* P = UH + (size_t)R * c * nnodes;
  const int ct = (c + TN - 1) / TN;
  const int ctt = (c + TRC - 1) / TRC;
  const T* Uin = adjoint ? h.Vlong : h.Ulong;  // incoming long basis
  const T* Vout = adjoint ? h.Ulong : h.Vlong; // outgoing long basis
  const T* Tin = adjoint ? h.Vt : h.Ut;
  const T* Tout = adjoint ? h.Ut : h.Vt;
  const int* front = al.frontier.as<int32_t>();
  if (al.mmax >= 1 && R > 0) {
    hipLaunchKernelGGL(k_leaf_up<T>, dim3(al.chunks, al.nfront, ct), dim3(256), 0, s, d_nodes,
                       front, al.chunks, Vout, h.ldl, R, X, ldx, c, QH, P);
    KCHK();
    if (al.chunks > 1) {
      const int64_t n = (int64_t)R * c;
      hipLaunchKernelGGL(k_chunk_reduce<T>, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 64),
                                                 al.nfront),
                         dim3(256), 0, s, front, al.chunks, P, n, QH, T(1), T(0), n);
      KCHK();
    }
    for (int l = al.mmax - 1; l >= 1; --l) {
      if (al.ninternal[l] == 0) continue;
      hipLaunchKernelGGL(k_tree_up<T>, dim3(al.ninternal[l], ctt), dim3(256), 0, s,
                         al.internal[l].as<TreeOp>(), Tout, R, QH, c);
      KCHK();
    }
    if (al.nlevel1 > 0) {
      hipLaunchKernelGGL(k_root<T>, dim3(al.nlevel1, ctt), dim3(256), 0, s,
                         al.level1.as<TreeOp>(), h.B, R, QH, UH, c, adjoint ? 1 : 0);
      KCHK();
    }
    for (int l = 1; l < al.mmax; ++l) {
      if (al.ninternal[l] == 0) continue;
      hipLaunchKernelGGL(k_tree_down<T>, dim3(al.ninternal[l], 2, ctt), dim3(256), 0, s,
                         al.internal[l].as<TreeOp>(), Tin, h.B, R, QH, UH, c, adjoint ? 1 : 0);
      KCHK();
    }
  }
  if (expansions_only) return;
  const int rt = (int)((al.max_rows + TM - 1) / TM);
  hipLaunchKernelGGL(k_leaf_down<T>, dim3(rt, al.nfront, ct), dim3(256), 0, s, d_nodes, front,
                     Uin, h.ldl, R, UH, c, h.D, h.ldd, adjoint ? 1 : 0, X, ldx, Y, ldy, alpha,
                     beta);
  KCHK();
}

// ------------------------------------------------------------ HODLR level --
template <class T>
__global__ void k_sib_diag(const Node* nodes, const int32_t* front, int R, const T* S,
                           const T* QH, T* UH, int c, int adjoint) {
  const int a = front[blockIdx.x];
  const int b = nodes[a].sib;
  // forward: uh_a = diag(s[b]) qh_b ; adjoint: uh_a = diag(s[a]) qh_b
  const T* sv = S + (int64_t)(adjoint ? a : b) * R;
  const T* q = QH + (int64_t)b * R * c;
  T* u = UH + (int64_t)a * R * c;
  for (int e = threadIdx.x; e < R * c; e += blockDim.x) u[e] = sv[e % R] * q[e];
}

template <class T>
void hodlr_level_apply(const Node* d_nodes, const ApplyLists& al, const T* U, const T* V,
                       int64_t ldl, int R, const T* S, bool adjoint, int c, const T* X,
                       int64_t ldx, T* Y, int64_t ldy, T alpha, T beta, void* work,
                       size_t nnodes, hipStream_t s) {
  if (al.nfront == 0 || c <= 0) return;
  T* QH = static_cast<T*>(work);
  T* UH = QH + (size_t)R * c * nnodes;
  T* P = UH + (size_t)R * c * nnodes;
  const int ct = (c + TN - 1) / TN;
  const int* front = al.frontier.as<int32_t>();
  const T* Vout = adjoint ? U : V;
  const T* Uin = adjoint ? V : U;
  hipLaunchKernelGGL(k_leaf_up<T>, dim3(al.chunks, al.nfront, ct), dim3(256), 0, s, d_nodes, front,
                     al.chunks, Vout, ldl, R, X, ldx, c, QH, P);
  KCHK();
  if (al.chunks > 1) {
    const int64_t n = (int64_t)R * c;
    hipLaunchKernelGGL(k_chunk_reduce<T>,
                       dim3((unsigned)std::min<int64_t>((n + 255) / 256, 64), al.nfront),
                       dim3(256), 0, s, front, al.chunks, P, n, QH, T(1), T(0), n);
    KCHK();
  }
  hipLaunchKernelGGL(k_sib_diag<T>, dim3(al.nfront), dim3(256), 0, s, d_nodes, front, R, S, QH, UH,
                     c, adjoint ? 1 : 0);
  KCHK();
  const int rt = (int)((al.max_rows + TM - 1) / TM);
  hipLaunchKernelGGL(k_leaf_down<T>, dim3(rt, al.nfront, ct), dim3(256), 0, s, d_nodes, front, Uin,
                     ldl, R, UH, c, (const T*)nullptr, (int64_t)0, 0, X, ldx, Y, ldy, alpha, beta);
  KCHK();
}

// ------------------------------------------------------------ seg_tn ------
template <class T>
__global__ __launch_bounds__(256) void k_seg_tn(const Node* nodes, const int32_t* list,
                                                int chunks, int rows, int cols, const T* A,
                                                int64_t lda, const T* B, int64_t ldb, T* P) {
  __shared__ T smem[mf_smem_elems<T>()];
  const int ch = blockIdx.x, li = blockIdx.y;
  const int i0 = (blockIdx.z % ((rows + TM - 1) / TM)) * TM;
  const int j0 = (blockIdx.z / ((rows + TM - 1) / TM)) * TN;
  const Node nd = nodes[list[li]];
  const int64_t r0 = nd.lo + (int64_t)ch * APPLY_CHUNK;
  const int K = (int)max<int64_t>(0, min<int64_t>(APPLY_CHUNK, nd.hi - r0));
  MfAcc<T> acc;
  acc.zero();
  if (K > 0)
    mf_tile<T>(rows - i0, cols - j0, K, A + r0 + (int64_t)i0 * lda, lda, 1,
                       B + r0 + (int64_t)j0 * ldb, 1, ldb, acc, smem);
  T* out = P + ((int64_t)li * chunks + ch) * rows * cols;
  mf_store<T>(rows - i0, cols - j0, out + i0 + (int64_t)j0 * rows, rows, acc, T(1),
                        T(0));
}

template <class T>
__global__ void k_seg_reduce(const Node* nodes, const int32_t* list, int chunks, int rows,
                             int cols, const T* P, T* out, int64_t out_stride, int64_t ldo,
                             T alpha, T beta, int to_parent) {
  const int li = blockIdx.y;
  int g = list[li];
  int64_t off = 0;
  if (to_parent) {
    off = nodes[g].is_left ? 0 : rows;
    g = nodes[g].parent;
  }
  const int64_t n = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    T s = T(0);
    for (int ch = 0; ch < chunks; ++ch) s += P[((int64_t)li * chunks + ch) * n + e];
    const int i = (int)(e % rows), j = (int)(e / rows);
    T* o = out + (int64_t)g * out_stride + off + i + (int64_t)j * ldo;
    *o = beta == T(0) ? alpha * s : alpha * s + beta * *o;
  }
}

template <class T>
size_t seg_tn_work_bytes(int nlist, int64_t max_rows, int rows, int cols) {
  const int64_t chunks = std::max<int64_t>(1, (max_rows + APPLY_CHUNK - 1) / APPLY_CHUNK);
  return (size_t)nlist * chunks * rows * cols * sizeof(T) + 256;
}

template <class T>
void seg_tn(const Node* d_nodes, const int32_t* list, int nlist, int64_t max_rows, int rows,
            int cols, const T* A, int64_t lda, const T* B, int64_t ldb, T* out,
            int64_t out_stride, int64_t ldo, T alpha, T beta, void* work, hipStream_t s,
            int to_parent) {
  if (nlist == 0 || rows == 0 || cols == 0) return;
  const int chunks = (int)std::max<int64_t>(1, (max_rows + APPLY_CHUNK - 1) / APPLY_CHUNK);
  const int tiles = ((rows + TM - 1) / TM) * ((cols + TN - 1) / TN);
  T* P = static_cast<T*>(work);
  hipLaunchKernelGGL(k_seg_tn<T>, dim3(chunks, nlist, tiles), dim3(256), 0, s, d_nodes, list,
                     chunks, rows, cols, A, lda, B, ldb, P);
  KCHK();
  const int64_t n = (int64_t)rows * cols;
  hipLaunchKernelGGL(k_seg_reduce<T>, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 64), nlist),
                     dim3(256), 0, s, d_nodes, list, chunks, rows, cols, P, out, out_stride, ldo,
                     alpha, beta, to_parent);
  KCHK();
}

#define INST(T)                                                                                \
  template void hodlr_level_apply<T>(const Node*, const ApplyLists&, const T*, const T*, int64_t, \
                                     int, const T*, bool, int, const T*, int64_t, T*, int64_t, T, \
                                     T, void*, size_t, hipStream_t);                              \
  template size_t apply_work_bytes<T>(const Forest&, const ApplyLists&, int, int);            \
  template void apply_forest<T>(const Node*, const ApplyLists&, const HbsView<T>&, bool, int,  \
                                const T*, int64_t, T*, int64_t, T, T, void*, size_t,           \
                                hipStream_t, bool);                                            \
  template void seg_tn<T>(const Node*, const int32_t*, int, int64_t, int, int, const T*,       \
                          int64_t, const T*, int64_t, T*, int64_t, int64_t, T, T, void*,       \
                          hipStream_t, int);                                                   \
  template size_t seg_tn_work_bytes<T>(int, int64_t, int, int);
INST(double)
INST(float)

}  // namespace hm
