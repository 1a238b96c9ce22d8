// Fig. 7 ("Application of A^(m) in the HBS framework") on a forest:
// outgoing expansions from long bases on the frontier level, upward pass with
// short transfers, sibling matrices at the root's children, downward pass
// over levels 1 .. m-1 (coarse to fine), incoming expansions through the long
// bases; optionally plus the diagonal blocks D (the full apply, m = L).
#pragma once
#include "common.h"

namespace hm {

// Node lists of one apply: the frontier (each active instance's nodes on its
// level m_i) and the tree sweeps over the internal nodes (levels 1 .. m_i - 1,
// ancestors of frontier nodes) cut into bands of levels.  Built once on the
// host, kept on the device.
// A subtree of a tree sweep taken by one workgroup of a band kernel: its
// nodes in breadth-first order (ids[0] the subtree root, the children of
// entry b at 2b + 1 and 2b + 2) down to `depth` levels below the root;
// info = depth | has_parent << 8 (down sweep: the root's own incoming
// expansion contributes).  Unused ids are -1.
constexpr int BAND_DMAX = 3;
struct BandJob {
  int32_t info;
  int32_t ids[(2 << BAND_DMAX) - 1];
};
struct BandRange {
  int off, n;   // jobs [off, off + n) of one launch
  int depth;    // the largest job depth among them (sizes the launch's LDS)
};

struct ApplyLists {
  DevBuf frontier;
  int nfront = 0;
  int64_t max_rows = 0;     // largest frontier node
  int chunks = 1;           // row chunks per frontier node for the V^T x reduction
  int mmax = 0;
  // Band launches for band depths D = 1 .. BAND_DMAX (index D), in launch
  // order: up = finest band first, down = the roots' band first; all jobs in
  // one device array.
  DevBuf bands;
  std::vector<BandRange> up_band[BAND_DMAX + 1], down_band[BAND_DMAX + 1];
};

constexpr int APPLY_CHUNK = 256;

// m[i] = frontier level of instance i (-1: instance not involved).
void build_apply_lists(const Forest& f, const std::vector<int>& m, ApplyLists& out,
                       hipStream_t s);

template <class T>
struct HbsView {
  const T* Ulong = nullptr;  // N x R long bases on the frontier (incoming)
  const T* Vlong = nullptr;  // N x R (outgoing)
  int64_t ldl = 0;
  const T* Ut = nullptr;     // per node 2R x R (global node id stride 2R*R)
  const T* Vt = nullptr;
  const T* B = nullptr;      // per node R x R: B[v] = B_{sib(v), v}
  const T* D = nullptr;      // N x nmax, or null (partial apply)
  int64_t ldd = 0;
  int R = 0;
};

// Workspace of an apply with c columns: expansions per node and chunk partials.
template <class T>
size_t apply_work_bytes(const Forest& f, const ApplyLists& al, int R, int c);

// Y = beta Y + alpha (A^(m) X [+ D X]); adjoint applies (A^(m))^* [+ D^*].
// The expansions stay in `work`: outgoing at work, incoming at
// work + R*c*nnodes (per node R x c, ld R).  expansions_only skips Y.
template <class T>
void apply_forest(const Node* d_nodes, const ApplyLists& al, const HbsView<T>& h, bool adjoint,
                  int c, const T* X, int64_t ldx, T* Y, int64_t ldy, T alpha, T beta, void* work,
                  size_t nnodes, hipStream_t s, bool expansions_only = false);

// The expansions of the forward apply of X (as apply_forest with
// expansions_only, at work_x) and the adjoint apply Y = A_H^* G with its
// expansions (at work_g), the tree sweeps of both in the same launches.
template <class T>
void apply_forest_pair(const Node* d_nodes, const ApplyLists& al, const HbsView<T>& h, int c,
                       const T* X, int64_t ldx, void* work_x, const T* G, int64_t ldg, T* Y,
                       int64_t ldy, void* work_g, size_t nnodes, hipStream_t s);

// One level of a HODLR apply (Sec. 2.8): for the frontier nodes v (one tree
// level), Y(I_a) = beta Y(I_a) + alpha U(I_a) diag(s[b]) V(I_b)^T X(I_b) with
// b = sib(a); adjoint: Y(I_b) += alpha V(I_b) diag(s[b]) U(I_a)^T X(I_a).
template <class T>
void hodlr_level_apply(const Node* d_nodes, const ApplyLists& al, const T* U, const T* V,
                       int64_t ldl, int R, const T* S, bool adjoint, int c, const T* X,
                       int64_t ldx, T* Y, int64_t ldy, T alpha, T beta, void* work,
                       size_t nnodes, hipStream_t s);

// Segmented transposed product used for the long-K reductions of the
// compression: for every node v in `list`, OUT_v (rows x cols) = alpha *
// A(I_v, 0:rows)^T B(I_v, 0:cols) (+ beta OUT_v), OUT_v at out + v*out_stride
// with leading dim ldo; with to_parent, OUT_v is the block of v's parent
// p at out + p*out_stride, offset by `rows` rows for a right child (the
// child's half of a transfer matrix).  Partials of APPLY_CHUNK rows are
// reduced in `work`.
template <class T>
void seg_tn(const Node* d_nodes, const int32_t* list, int nlist, int64_t max_rows, int rows,
            int cols, const T* A, int64_t lda, const T* B, int64_t ldb, T* out,
            int64_t out_stride, int64_t ldo, T alpha, T beta, void* work, hipStream_t s,
            int to_parent = 0);
template <class T>
size_t seg_tn_work_bytes(int nlist, int64_t max_rows, int rows, int cols);
// The same for A = B (Gram matrices of node blocks, FP64, c <= 96 columns):
// OUT_v = A(I_v, 0:c)^T A(I_v, 0:c), only the 16 x 16 tiles on and above the
// diagonal multiplied (each written with its mirror); work as
// seg_tn_work_bytes(nlist, max_rows, c, c).
void seg_gram(const Node* d_nodes, const int32_t* list, int nlist, int64_t max_rows, int c,
              const double* A, int64_t lda, double* out, int64_t out_stride, void* work,
              hipStream_t s);

}  // namespace hm
