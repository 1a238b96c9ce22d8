// Node factorisations of the peeling step: Householder QR of tall node blocks
// by a tree of LDS-resident panels (TSQR), one-sided Jacobi SVD of the final
// triangle, reflector application that writes the basis directly, and the
// column-pivoted QR behind the interpolative decomposition (Sec. 2.2-2.4).
#pragma once
#include "common.h"

namespace hm {

constexpr int FAC_CMAX = 2 * HM_MAX_SAMPLES;  // columns of a node block
constexpr int FAC_PMAX = 2 * FAC_CMAX;        // rows of a panel (two stacked triangles)
constexpr int FAC_LDMAX = FAC_PMAX + 1;
constexpr int QR_NB = 16;                     // strip width of the blocked QR
constexpr int QR_TMAX = FAC_CMAX / QR_NB;     // strips per panel

struct PanelDesc {
  double* A;        // panel (global, column-major): rows x cols, factored in place
  int64_t ld;
  int32_t rows, cols;
  double* tau;      // min(rows, cols) reflector scalars
  double* T;        // compact WY factors, QR_NB x QR_NB per strip (row-major);
                    // written by the QR, read by the apply
  double* Rout;     // R (min(rows,cols) x cols, zeros below the diagonal)
  int64_t ldR;
  const double* Cin;  // apply: h x ncol input (h = min(rows, cols))
  int64_t ldCin;
  double* Cout;     // apply: rows x ncol output  Q [Cin; 0]
  int64_t ldCout;
  int32_t ncol;
  int32_t trans;    // QR: the panel is the transpose of A (A stored cols x rows);
                    // the factored panel is written back untransposed, ld ld
  const int32_t* dyn_cols;  // optional (device): the panel has min(cols, *dyn_cols)
                            // columns, known only on the device (a revealed rank)
  const int32_t* perm;      // optional (device): apply writes row i of the result
                            // to row perm[i] of Cout
  int32_t cin_full;         // apply: Cin holds all `rows` rows (Cout = Q Cin)
                            // instead of the first min(rows, cols)
  int32_t pad_;
};

struct SvdDesc {
  const double* R;  // h x c (h <= c), leading dim ldR; c x h when trans
  int64_t ldR;
  int32_t h, c;
  double* W;        // left singular vectors, wrows x kout (descending singular values)
  int64_t ldW;
  double* sv;       // kout singular values
  double* X;        // right singular vectors, xrows x kout (may be null)
  int64_t ldX;
  int32_t kout;     // columns of W / X written
  int32_t trans;    // 1: factor R^T (R stored c x h)
  int32_t* sweeps;  // optional: atomic max of the Jacobi sweeps used
  const int32_t* dyn;  // optional (device): h = c = min(c, *dyn), a revealed rank
  int32_t wrows, xrows;  // frames the singular vectors are embedded in (>= h, >= c):
                         // rows beyond h (c) are zero, and output columns
                         // j >= c get the unit vector e_j (zero if j >= wrows /
                         // xrows) with singular value 0, an orthonormal completion
  int32_t xscaled;       // 1: X receives X diag(s) = T^T W (needs trans = 0), formed
                         // from the converged left vectors; no rotations accumulated
  int32_t gram;          // Gram form: T is the pivoted Cholesky factor L of M^T M
                         // (h rows in pivoted order, c = min(c, *dyn) columns); the
                         // converged columns a_j = s_j u_j give the right singular
                         // vectors x_j = P u_j of M: X receives X diag(s), W receives
                         // X diag(1/s^2) (so M W = U), rows scattered by perm; W
                         // columns kout .. wrows - 1 are set to zero
  const int32_t* perm;
};

// Column-pivoted Householder QR of A = R^T (c x h, R stored h x c) that stops
// at the numerical rank rho: the first step k >= kmin whose largest remaining
// column norm is <= eta times the largest initial one (or any step at an
// exactly zero remainder).  A P = Q2 [R2; *] with the dropped trailing block.
struct QrcpDesc {
  double* R;        // in: h x c, ld ldR; out: the reflectors of A (column k in
                    // rows k+1 .. c-1, unit diagonal implied), c x h, ld ldR
  int64_t ldR;
  int32_t c, h;
  double* tau;      // rho reflector scalars
  double* T;        // compact WY factors per QR_NB strip (as PanelDesc.T)
  double* R2;       // rho x h, upper trapezoidal (zero below the diagonal), ld ldR2
  int64_t ldR2;
  int32_t* perm;    // h: column j of A P is column perm[j] of A
  int32_t* rho;     // the numerical rank
  double eta;       // relative threshold (<= 0: max(c, h) eps)
  int32_t kmin;     // steps taken whatever the threshold (stops only at a zero column)
  int32_t pad_;
};
void launch_qrcp(const QrcpDesc* d, int n, hipStream_t s);

// Pivoted Cholesky of a symmetric positive semidefinite c x c matrix (the
// Gram matrix M^T M of a node block), c <= 96: P^T G P = L L^T with L (c x
// rho) lower trapezoidal, rows in pivoted order.  Diagonal pivoting; stops at
// the first step k >= kneed whose largest remaining pivot is <= eta^2 times
// the largest initial one.  A step k < kneed whose pivot is <= tau^2 times it
// (a direction the Gram matrix cannot resolve) sets *short_flag and stops.
struct PcholDesc {
  const double* G;  // c x c, ld ldG (only read)
  int64_t ldG;
  int32_t c, kneed;
  double eta, tau;
  double* L;        // c x rho, ld ldL (rows in pivoted order)
  int64_t ldL;
  int32_t* perm;    // c: pivoted row i is row perm[i] of G
  int32_t* rho;
  int32_t* short_flag;
  int32_t pad_;
};
void launch_pchol(const PcholDesc* d, int n, hipStream_t s);

void launch_panel_qr(const PanelDesc* d, int n, hipStream_t s);
void launch_apply_q(const PanelDesc* d, int n, hipStream_t s);
// gram_only: every descriptor is in Gram form (smaller LDS footprint).
void launch_jacobi_svd(const SvdDesc* d, int n, hipStream_t s, bool gram_only = false);

// Node block of the peeling step (Fig. 4): for each child v (list), rows I_v of
// M get [S(I_v, off : off + r), Lpar(I_v, 0:r) diag(w_parent)] with off = 0 for
// a left child, R for a right child; the second half is omitted under the root.
void launch_build_node_block(const Node* nodes, const Instance* inst, const int32_t* kids,
                             int nkids, int64_t max_rows, int R, const double* S, int64_t lds,
                             const double* Lpar, int64_t ldl, const double* w, double* M,
                             int64_t ldm, hipStream_t s, int first_half_only = 0);
// B[v] = X_v(0:r, 0:r) diag(z_v) (zero-padded to R x R); X_v at X + v*2R*R, ld 2R.
// z == nullptr: X already holds X diag(z).
void launch_form_b(const Node* nodes, const Instance* inst, const int32_t* kids, int nkids, int R,
                   const double* X, const double* z, double* B, hipStream_t s);

// Interpolative decomposition by column-pivoted QR of W^* (Sec. 2.4, eq.
// buildTJ): for each node of `list`, the candidate rows of W = Src diag(w):
//  leaf mode   : rows I_t of Src (N x R, ld lds); skeleton ids lo + i
//  parent mode : Src block t (2R x R, ld 2R); candidate i maps to skeleton
//                skel[left][i] (i < R) or skel[right][i - R]
// Outputs: interpolation basis P (leaf: rows I_t of an N x R array, ld ldp;
// parent: block t of 2R x R), samp_t = Src(J, :) (R x R, rows >= k zero),
// rank_t, skel_t (R entries, -1 padded).  Truncation: k steps or the first
// residual norm <= tol * |R_11| (tol > 0), never beyond r or a zero residual.
void launch_cpqr_id(const Node* nodes, const Instance* inst, const int32_t* list, int nlist,
                    int parent_mode, int R, const double* Src, int64_t lds, const double* w,
                    double* P, int64_t ldp, double* samp, int32_t* rank, int32_t* skel,
                    int32_t* saturated, hipStream_t s);
// The whole Fig. 5 sweep (both sides, every level and instance) in one
// persistent launch: items (node, side) in order of decreasing level; a
// workgroup takes items from *next until none is left, a parent item after
// both children of its side are done (done[2 node + side] set).  done (2 *
// nodes int32) and *next must be zero at launch; *err is set if a wait ran
// past its limit (the sweep's results are then invalid).  Per side: leaf
// interpolation bases into P (rows I_t, ld ldb), parent transfers into Pt
// (block t, 2R x R), samp_t, rank_t, skel_t as launch_cpqr_id.
struct IdItem {
  int32_t node, side;
};
struct IdSide {
  const double* basis;   // leaf long bases (N x R, ld ldb)
  const double* w;       // per-node weights (y or z), R each
  const double* told;    // transfers of the orthonormal form (2R x R per node)
  double* P;             // leaf interpolation bases (N x R, ld ldb)
  double* Pt;            // parent interpolation transfers (2R x R per node)
  double* samp;          // samp_t (R x R per node)
  int32_t* rank;
  int32_t* skel;
};
void launch_id_sweep(const Node* nodes, const Instance* inst, const IdItem* items, int nitems,
                     const IdSide& u, const IdSide& v, int R, int64_t ldb, int32_t* done,
                     int32_t* next, int32_t* err, int32_t* saturated, int workgroups,
                     hipStream_t s);
// Utmp_t(side R + i, :) = samp_child(i, :) Tr_t(side R : side R + R, :)  (Fig. 5)
void launch_utmp(const Node* nodes, const int32_t* list, int nlist, int R, const double* samp,
                 const double* Tr, double* Utmp, hipStream_t s);
// Bnew[v] = sampU[sib(v)] Bold[v] sampV[v]^T  (eq. ben0-ben2)
void launch_bskel(const Node* nodes, const int32_t* list, int nlist, int R, const double* sampU,
                  const double* sampV, const double* Bold, double* Bnew, hipStream_t s);

// out(I_v, 0:N) = A(I_v, 0:K) Bn_w  for v in list, w = v (or sib(v) if
// from_sibling); Bn_w at Bn + w*bstride (K x N, ld ldb).
void launch_node_nn(const Node* nodes, const int32_t* list, int nlist, int64_t max_rows, int K,
                    int N, const double* A, int64_t lda, const double* Bn, int64_t bstride,
                    int64_t ldb, double* out, int64_t ldo, hipStream_t s, int from_sibling = 0);
// Truncation of the HODLR Z-side SVD (Fig. 2 svd(., eps)): per node keep
// k_v = #{s_j > tol s_1} (tol > 0) capped at k, or k (tol == 0); zero the rest of
// the columns of Vl(I_v, :), sv_v and X_v; rank[v] = k_v.
void launch_truncate(const Node* nodes, const Instance* inst, const int32_t* kids, int nkids,
                     int64_t max_rows, int R, double* Vl, int64_t ldv, double* sv, double* X,
                     int32_t* rank, int32_t* saturated, hipStream_t s);

}  // namespace hm
