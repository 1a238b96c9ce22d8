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

struct hm_frontal_s;   // frontal.hip

namespace hm {

// Frontal-matrix black box (frontal.hip): Y = A X for ncols columns, with a
// work block of frontal_work_bytes(f, ncols) bytes.
void frontal_apply(const hm_frontal_s* f, int64_t ncols, const double* X, int64_t ldx, double* Y,
                   int64_t ldy, void* work, hipStream_t s);
size_t frontal_work_bytes(const hm_frontal_s* f, int64_t ncols);
int64_t frontal_n(const hm_frontal_s* f);

// Device copies of small per-call tables (node lists, descriptors): device
// blocks, bump-allocated, filled through the pinned staging of stage_h2d, so
// the copies stay asynchronous and no allocation happens per table.  Nothing
// is released before the Keeper is destroyed; its owner synchronises the
// stream first.
struct Keeper {
  std::vector<DevBuf> dblk;
  size_t dused = 0;
  Keeper() = default;
  Keeper(const Keeper&) = delete;
  Keeper& operator=(const Keeper&) = delete;
  template <class T>
  T* put(const std::vector<T>& v, hipStream_t s) {
    const size_t b = (v.size() * sizeof(T) + 255) / 256 * 256 + 256;
    if (dblk.empty() || dused + b > dblk.back().bytes) {
      dblk.emplace_back(std::max<size_t>(b, (size_t)4 << 20));
      dused = 0;
    }
    char* dp = dblk.back().as<char>() + dused;
    dused += b;
    if (!v.empty()) stage_h2d(dp, v.data(), v.size() * sizeof(T), s);
    return reinterpret_cast<T*>(dp);
  }
};

// Growable device workspace handed out by offsets.  Growth does not wait for
// the stream: the outgrown buffer may still be in use by enqueued kernels, so
// it is kept until the workspace is destroyed.
struct Workspace {
  DevBuf buf;
  std::vector<DevBuf> old;
  void ensure(size_t bytes, hipStream_t) {
    if (buf.bytes >= bytes) return;
    if (buf.p) old.push_back(std::move(buf));
    buf = DevBuf(bytes + bytes / 4);
  }
  char* base() const { return static_cast<char*>(buf.p); }
};

// Black-box operator wrapper: dispatch, timing (hipEvents), call counts.
struct OpRunner {
  hm_operator op{};
  const hm_hbs_s* hbs = nullptr;     // HM_OP_HBS
  hipStream_t s = nullptr;
  Workspace work;
  Workspace cvt;                     // callback blocks in the sample type
  std::vector<hipEvent_t> ev;        // pairs around each call (created once, reused)
  size_t nev = 0;                    // events recorded since the last reset
  int calls = 0;
  int64_t columns = 0;
  ~OpRunner();
  void apply(bool adjoint, int64_t n, int c, const double* X, int64_t ldx, double* Y, int64_t ldy);
  double elapsed_ms();               // after stream synchronisation
  void reset_stats();                // forget earlier calls (a compress that starts over)
};

// Internal flag of hbs_compress_forest (beside the HM_FLAG_* bits): node
// SVDs on the Householder path only.
constexpr int32_t HM_FLAG_INTERNAL_NO_GRAM = 1 << 30;
// Internal flag: no Householder rerun after a node the Gram matrix cannot
// resolve (timing runs of the tuner).
constexpr int32_t HM_FLAG_INTERNAL_NO_FALLBACK = 1 << 29;

// Leading left singular vectors of node blocks: for each job, the block
// M(lo : lo+rows, 0 : cols) is factored by Householder TSQR, its triangle by
// a rank-revealing pivoted QR (per job: relative threshold eta, at least kmin
// directions) and one-sided Jacobi, and the leading kout left singular
// vectors are written to Uout(lo.., 0:kout) (other columns untouched),
// singular values to sv[node*R ..], right singular vectors to X[node*2R*R ..]
// (ld 2R) if X -- scaled by the singular values if x_scaled.  Directions
// below the threshold get singular value 0 and orthonormal completions.
// qr_only: Uout gets the first min(rows, kout) columns of Q instead.
struct SvdJob {
  int32_t node;
  int32_t rows, cols, kout;
  int64_t lo;
  int32_t kmin;     // directions kept whatever their size (the rank k of the instance)
  double eta;       // relative rank threshold (<= 0: the FP64 rounding level)
};
void node_svd(const std::vector<SvdJob>& jobs, double* M, int64_t ldm, double* Uout, int64_t ldu,
              double* sv, double* X, int R, bool qr_only, Workspace& ws, Keeper& kp,
              hipStream_t s, int32_t* sweeps = nullptr, bool x_scaled = false);
// Relative rank threshold of the node factorisations for samples computed in
// `dtype` (an HM_* sample type): singular values below it are not resolved by
// the samples.  FP64: 0 (the kernels use max(c, h) eps); FP32: 2^-24 / 16;
// BF16: 2^-11, an eighth of the BF16 unit roundoff u = 2^-8 (entries and test
// matrix are both rounded to BF16, each with a relative error uniform in
// [-u, u], so a sample against a Gaussian column carries noise of about
// u sqrt(2/3) = 3.2e-3 times the norm of the sampled row block).
double sample_rank_eta(int dtype);

hm_hbs_s* hbs_compress_forest(Forest f, std::vector<OpRunner*>& ops, int32_t flags, hipStream_t s,
                              int* status);
// Key of the tuning table for a compression of forest f (after forest_finish)
// with padded rank R; bf16_kernel: every operator is the built-in kernel
// sampled in BF16 (the schedules the tuner chooses between exist only then).
TuneKey tune_key(const Forest& f, bool bf16_kernel, int R);
hm_hodlr_s* hodlr_compress_forest(Forest f, OpRunner& op, hipStream_t s, int* status);
void hodlr_apply_full(const hm_hodlr_s* h, bool adjoint, int c, const double* X, int64_t ldx,
                      double* Y, int64_t ldy, hipStream_t s);

void finish_handle_info(hm_hbs_s* h);
// Block-diagonal forest operator from single-tree FP64 handles; one handle per
// instance of an FP64 forest handle, stored in `dtype` (HM_F64 / HM_F32).
hm_hbs_s* merge_hbs(const std::vector<const hm_hbs_s*>& hs, hipStream_t s);
std::vector<hm_hbs_s*> split_hbs(const hm_hbs_s* src, hipStream_t s, int dtype = HM_F64);
// Copy of a handle with generators stored in `dtype` (HM_F64 / HM_F32); the
// copy is complete once the stream has passed the call (sync: waits for it).
// The source must stay alive until then.
hm_hbs_s* convert_hbs(const hm_hbs_s* src, int dtype, hipStream_t s, bool sync = true);

}  // namespace hm
