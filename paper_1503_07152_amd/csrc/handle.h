// Handles and host-side helpers shared by the compress / apply entry points.
#pragma once
#include <cstring>
#include <deque>
#include <memory>

#include "apply.h"
#include "common.h"
#include "factor.h"
#include "sampler.h"

// HBS representation on the device, zero-padded to a uniform rank R:
//   U, V   N x R        rows I_t of leaf t hold its (long) basis
//   Ut, Vt per node 2R x R (global node id g = heap - 1); rows 0..R-1 couple
//          to the left child, R..2R-1 to the right child
//   B      per node R x R: B[v] = B_{sib(v), v}
//   D      N x nmax     rows I_t of leaf t hold D_t in columns 0..n_t-1
struct hm_hbs_s {
  hm::Forest f;
  hm::DevBuf d_nodes, d_inst;
  int R = 0;
  int dtype = HM_F64;
  int is_id = 0;
  hm::DevBuf U, V, Ut, Vt, B, D;
  std::vector<int32_t> rank_u, rank_v;      // per node
  std::vector<int32_t> skel_in, skel_out;   // per node x R (instance-local rows), -1 padded
  hm::ApplyLists full;                      // frontier = leaves
  hm::DevBuf grad_leaves, grad_nodes;       // leaf list and all-node list (backward)
  hm_info info{};

  template <class T>
  hm::HbsView<T> view() const {
    hm::HbsView<T> v;
    v.Ulong = U.as<T>(); v.Vlong = V.as<T>(); v.ldl = f.n_total;
    v.Ut = Ut.as<T>(); v.Vt = Vt.as<T>(); v.B = B.as<T>();
    v.D = D.as<T>(); v.ldd = f.n_total; v.R = R;
    return v;
  }
};

// HODLR representation: per level l = 1..L long bases U_l, V_l (N x R),
// diagonal sibling matrices s (per node R), D (N x nmax).
struct hm_hodlr_s {
  hm::Forest f;
  hm::DevBuf d_nodes, d_inst;
  int R = 0;
  std::vector<hm::DevBuf> U, V;   // index l - 1
  hm::DevBuf S, D;
  std::vector<int32_t> rank;      // per node (B_{sib(v), v} rank)
  std::vector<hm::ApplyLists> lvl;  // per level l: frontier = nodes on level l
  hm::ApplyLists full;
  hm_info info{};
};

namespace hm {

// Keeps host tables alive and their device copies until the owner is
// destroyed (after the stream has been synchronised), so asynchronous copies
// never race.
struct Keeper {
  std::deque<std::vector<char>> host;
  std::vector<DevBuf> dev;
  template <class T>
  T* put(const std::vector<T>& v, hipStream_t s) {
    const size_t b = v.size() * sizeof(T);
    host.emplace_back(b + 16);
    if (b) std::memcpy(host.back().data(), v.data(), b);
    dev.emplace_back(b + 16);
    if (b) HIPCHK(hipMemcpyAsync(dev.back().p, host.back().data(), b, hipMemcpyHostToDevice, s));
    return dev.back().as<T>();
  }
};

// Growable device workspace handed out by offsets; grow() synchronises.
struct Workspace {
  DevBuf buf;
  void ensure(size_t bytes, hipStream_t s) {
    if (buf.bytes >= bytes) return;
    HIPCHK(hipStreamSynchronize(s));
    buf.alloc(bytes + bytes / 4);
  }
  char* base() const { return static_cast<char*>(buf.p); }
};

// Black-box operator wrapper: dispatch, timing (hipEvents), call counts.
struct OpRunner {
  hm_operator op{};
  const hm_hbs_s* hbs = nullptr;     // HM_OP_HBS
  hipStream_t s = nullptr;
  Workspace work;
  std::vector<hipEvent_t> ev;        // pairs around each call
  int calls = 0;
  int64_t columns = 0;
  ~OpRunner();
  void apply(bool adjoint, int64_t n, int c, const double* X, int64_t ldx, double* Y, int64_t ldy);
  double elapsed_ms();               // after stream synchronisation
};

// Leading left singular vectors of node blocks: for each job, the block
// M(lo : lo+rows, 0 : cols) is factored by Householder TSQR, its triangle by
// one-sided Jacobi, and the leading kout left singular vectors are written to
// Uout(lo.., 0:kout) (other columns untouched), singular values to
// sv[node*R ..], right singular vectors to X[node*2R*R ..] (ld 2R) if X.
// qr_only: Uout gets the first min(rows, kout) columns of Q instead.
struct SvdJob {
  int32_t node;
  int32_t rows, cols, kout;
  int64_t lo;
};
void node_svd(const std::vector<SvdJob>& jobs, double* M, int64_t ldm, double* Uout, int64_t ldu,
              double* sv, double* X, int R, bool qr_only, Workspace& ws, Keeper& kp,
              hipStream_t s, int32_t* sweeps = nullptr);

hm_hbs_s* hbs_compress_forest(Forest f, std::vector<OpRunner*>& ops, int32_t flags, hipStream_t s,
                              int* status);
hm_hodlr_s* hodlr_compress_forest(Forest f, OpRunner& op, hipStream_t s, int* status);
void hodlr_apply_full(const hm_hodlr_s* h, bool adjoint, int c, const double* X, int64_t ldx,
                      double* Y, int64_t ldy, hipStream_t s);

void finish_handle_info(hm_hbs_s* h);
// Block-diagonal forest operator from single-tree FP64 handles; one handle per
// instance of a forest handle.
hm_hbs_s* merge_hbs(const std::vector<const hm_hbs_s*>& hs, hipStream_t s);
std::vector<hm_hbs_s*> split_hbs(const hm_hbs_s* src, hipStream_t s);

}  // namespace hm
