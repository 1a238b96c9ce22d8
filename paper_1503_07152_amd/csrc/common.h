// Internal declarations shared by the host orchestration and the HIP kernels
// of libhbspeel.  Not part of the public ABI (include/hbspeel.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/hbspeel.h"

namespace hm {

// ---------------------------------------------------------------- errors --
void set_error(const char* fmt, ...);
const char* get_error();

struct Error {
  int code;
};

#define HM_THROW(code, ...)      \
  do {                           \
    ::hm::set_error(__VA_ARGS__); \
    throw ::hm::Error{code};     \
  } while (0)

#define HIPCHK(expr)                                                        \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      HM_THROW(HM_ERR_HIP, "%s failed: %s (%s:%d)", #expr,                  \
               hipGetErrorString(e_), __FILE__, __LINE__);                  \
  } while (0)

#define KCHK() HIPCHK(hipGetLastError())

// ------------------------------------------------------------ forest --------
// A forest of binary index trees (Sec. 2.7) over one global row space: one
// tree per instance (a single compression is a forest of one tree).  Every
// node carries global row bounds and explicit parent/child/sibling ids, so
// kernels take node lists instead of heap arithmetic.
struct Node {
  int64_t lo, hi;      // global rows [lo, hi)
  int32_t parent;      // -1 for a root
  int32_t left, right; // -1 for a leaf
  int32_t sib;         // -1 for a root
  int32_t level;       // depth in its tree (root 0)
  int32_t inst;        // instance
  int32_t heap;        // heap number inside its tree (root 1, children 2t, 2t+1)
  int32_t is_left;     // 1 if left child
  int32_t pad_;
};

struct Instance {
  int64_t row0, n, leaf;
  int32_t L;           // depth of its leaves
  int32_t r;           // samples per level (= rank + oversample)
  int32_t k;           // rank (fixed) or rank cap (tol mode)
  int32_t p;           // oversampling
  double tol;
  uint64_t seed;
  int32_t root;        // global id of its root
  int32_t nmax;        // largest leaf
};

struct Forest {
  std::vector<Node> nodes;
  std::vector<Instance> inst;
  int64_t n_total = 0;
  int32_t max_levels = 0;           // max over instances of L
  // lists of global node ids
  std::vector<std::vector<int32_t>> level;  // all nodes with level == l
  std::vector<int32_t> leaves;
  int32_t nmax = 0;                 // largest leaf over all instances
  int32_t heap_size(int i) const { return 1 << (inst[i].L + 1); }
};

void forest_add_tree(Forest& f, int64_t n, int64_t leaf, int32_t r, int32_t k,
                     int32_t p, double tol, uint64_t seed);
void forest_finish(Forest& f);

// ------------------------------------------------------------- memory -------
// Device memory comes from the library's cache of hipMalloc'd blocks (see
// DevBuf::alloc), or from the caller's allocator once hm_set_allocator has
// installed one.  Every buffer remembers the allocator that made it and the
// stream it was made for, and goes back to that allocator on that stream, even
// if the allocator has been changed since.
struct AllocHook {
  hm_alloc_fn alloc = nullptr;
  hm_free_fn free = nullptr;
  void* ctx = nullptr;
};
AllocHook alloc_hook();
void set_alloc_hook(const AllocHook& h);

// Stream of the entry point running on this thread, handed to the caller's
// allocator (set for the extent of a call by StreamScope; default NULL).
hipStream_t alloc_stream();
struct StreamScope {
  hipStream_t prev;
  explicit StreamScope(void* s);
  ~StreamScope();
  StreamScope(const StreamScope&) = delete;
  StreamScope& operator=(const StreamScope&) = delete;
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  size_t cap = 0;             // size of the block (default allocator's cache class)
  AllocHook hook;             // allocator that made p (alloc == nullptr: the library's cache)
  hipStream_t stream = nullptr;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept
      : p(o.p), bytes(o.bytes), cap(o.cap), hook(o.hook), stream(o.stream) {
    o.p = nullptr;
    o.bytes = 0;
    o.cap = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    release();
    p = o.p; bytes = o.bytes; cap = o.cap; hook = o.hook; stream = o.stream;
    o.p = nullptr; o.bytes = 0; o.cap = 0;
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t b);
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Per-call scratch ordered on a stream: hipMallocAsync / hipFreeAsync, or the
// caller's allocator.
struct StreamBuf {
  void* p = nullptr;
  AllocHook hook;
  hipStream_t stream = nullptr;
  StreamBuf(size_t b, hipStream_t s);
  ~StreamBuf();
  StreamBuf(const StreamBuf&) = delete;
  StreamBuf& operator=(const StreamBuf&) = delete;
};

// ------------------------------------------------------------- tuning -----
// Schedule and tile choices of a compression that do not change what it
// computes (only the order of FP32 sums in the BF16 sampler): picked by
// hm_autotune per workload shape, used by later compressions of that shape.
struct TuneParams {
  int32_t gfirst = 0;   // most levels whose first products share a call (0: sampler width)
  int32_t ride = -1;    // most later first products a second-product call carries (-1: all that fit)
  int32_t ksplit = 0;   // K-splits of the narrow BF16 sampler (0: built-in default)
};
struct TuneKey {
  int64_t n;
  int32_t r, levels, nmax, instances, sampler;   // sampler: 1 = BF16 kernel operator
  bool operator<(const TuneKey& o) const;
};
bool tune_lookup(const TuneKey& k, TuneParams* out);
void tune_store(const TuneKey& k, const TuneParams& p);
// Parameters in effect on this thread (set for the extent of a compression).
const TuneParams& tune_current();
struct TuneScope {
  TuneParams prev;
  explicit TuneScope(const TuneParams& p);
  ~TuneScope();
  TuneScope(const TuneScope&) = delete;
  TuneScope& operator=(const TuneScope&) = delete;
};

// Frees the default allocator's cached device blocks (waits for the device).
void release_cached_memory();

// Host-to-device copy through pinned staging memory, enqueued on `s`
// without waiting for it: `src` may be reused as soon as the call returns.
// Staging chunks are kept for the process and reused once the copy out of
// them has completed.
void stage_h2d(void* dst, const void* src, size_t bytes, hipStream_t s);
// device -> host reads gathered in one pinned staging chunk; returns after
// the stream has drained (the reads are the stream's last work)
struct D2HRead {
  void* dst;
  const void* src;
  size_t bytes;
};
void read_d2h(const std::vector<D2HRead>& items, hipStream_t s);

// Upload a host vector into a fresh device buffer (enqueued on s; the host
// vector may be freed on return).
template <class T>
DevBuf upload(const std::vector<T>& v, hipStream_t s) {
  DevBuf b(v.size() * sizeof(T) + 16);
  if (!v.empty()) stage_h2d(b.p, v.data(), v.size() * sizeof(T), s);
  return b;
}

// ------------------------------------------------------------ kernels -------
// Gaussian stream (Philox4x32-10 + Box-Muller), see hm_gauss.
void launch_gauss_raw(uint64_t seed, int level, int phase, int64_t row0, int64_t nrows,
                      int ncols, double* out, int64_t ld, hipStream_t s);
// Structured test matrix [Omega_2 | Omega_1] for forest level `level`:
// for every child node v in `kids` (nodes on level+1), rows I_v get the
// instance's Gaussian G_level(i - row0, j), j < r, in columns [0, r) if v is a
// right child, [R, R + r) if a left child.  Other columns of those rows are 0.
void launch_gauss_masked(const Node* nodes, const Instance* inst, const int32_t* kids,
                         int nkids, int64_t max_rows, int level, int R, double* Om,
                         int64_t ld, hipStream_t s);
// Same masking with a given long basis instead of Gaussians (Psi of Fig. 2/4):
// rows I_v get U(I_v, 0:r) in the half chosen by the side of v.
void launch_mask_basis(const Node* nodes, const Instance* inst, const int32_t* kids,
                       int nkids, int64_t max_rows, int R, const double* U, int64_t ldu,
                       double* Om, int64_t ld, hipStream_t s);
// Block identity of the diagonal extraction: Om(I_t, 0:n_t) = I for leaves t,
// n_max columns; or only its columns j0 .. j0 + nc - 1 (nc < 0: to n_max),
// written to columns 0 .. nc - 1 of Om.
void launch_block_eye(const Node* nodes, const int32_t* leaves, int nleaves,
                      int64_t max_rows, int nmax, double* Om, int64_t ld, hipStream_t s,
                      int j0 = 0, int nc = -1);

// Zero D(I_t, n_t : nmax) of leaves smaller than nmax.
void launch_zero_dpad(const Node* nodes, const int32_t* leaves, int nleaves, int64_t max_rows,
                      int nmax, double* D, int64_t ld, hipStream_t s);
void launch_fill(double* p, int64_t rows, int64_t cols, int64_t ld, double v, hipStream_t s);
// out[2j] = ||A(:,j) - B(:,j)||^2 and out[2j+1] = ||A(:,j)||^2 (device, FP64)
void launch_col_err2(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t rows,
                     int cols, double* out, hipStream_t s);
// dst (rows x cols, type ddt, ld ldd) = src (type sdt, ld lds); HM_F64 / HM_F32
// sources, HM_F64 / HM_F32 / HM_BF16 destinations.
void launch_convert(const void* src, int sdt, int64_t lds, void* dst, int ddt, int64_t ldd,
                    int64_t rows, int64_t cols, hipStream_t s);
void launch_fill_f(float* p, int64_t count, float v, hipStream_t s);
void launch_nonfinite_check(const double* p, int64_t rows, int64_t cols, int64_t ld,
                            int* flag, hipStream_t s);

// Small-matrix kernels used by apply and compress live in their own headers
// (apply.h, factor.h, sampler.h).

}  // namespace hm
