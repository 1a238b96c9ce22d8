// Test-matrix generation (Sec. 2.5 randn of Fig. 2/4), masking of test
// matrices to the children of a level, block identity of the diagonal
// extraction, fills, the non-finite check, forest construction, errors and
// device buffers.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>

#include "common.h"

namespace hm {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}
const char* get_error() { return g_err.c_str(); }

// ------------------------------------------------------------------ memory
static std::mutex g_hook_mu;
static AllocHook g_hook;
static thread_local hipStream_t g_alloc_stream = nullptr;

AllocHook alloc_hook() {
  std::lock_guard<std::mutex> lk(g_hook_mu);
  return g_hook;
}
void set_alloc_hook(const AllocHook& h) {
  std::lock_guard<std::mutex> lk(g_hook_mu);
  g_hook = h;
}
hipStream_t alloc_stream() { return g_alloc_stream; }
StreamScope::StreamScope(void* s) : prev(g_alloc_stream) { g_alloc_stream = (hipStream_t)s; }
StreamScope::~StreamScope() { g_alloc_stream = prev; }

// Device memory cache of the default allocator (no caller allocator
// installed): a released buffer is kept, by device, stream and rounded size,
// and handed out again to an allocation of that size made for the same
// stream, which stream order makes safe.  Sizes round up to a power of two
// below 1 MiB and to a multiple of 2 MiB above.  When hipMalloc fails, the
// cached blocks are freed (after a device synchronisation) and it is retried.
namespace {
struct CacheKey {
  int dev;
  hipStream_t s;
  size_t bytes;
  bool operator<(const CacheKey& o) const {
    if (dev != o.dev) return dev < o.dev;
    if (s != o.s) return s < o.s;
    return bytes < o.bytes;
  }
};
std::mutex g_cache_mu;
std::map<CacheKey, std::vector<void*>> g_cache;

size_t cache_round(size_t b) {
  if (b >= ((size_t)1 << 20)) {
    const size_t m = (size_t)2 << 20;
    return (b + m - 1) / m * m;
  }
  size_t r = 256;
  while (r < b) r <<= 1;
  return r;
}

void cache_trim() {   // caller holds g_cache_mu
  if (g_cache.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto& kv : g_cache)
    for (void* p : kv.second) (void)hipFree(p);
  g_cache.clear();
}
}  // namespace

void DevBuf::alloc(size_t b) {
  release();
  if (b == 0) b = 16;
  hook = alloc_hook();
  stream = g_alloc_stream;
  if (hook.alloc) {
    p = hook.alloc(hook.ctx, b, stream);
    if (!p) HM_THROW(HM_ERR_ALLOC, "caller's allocator returned NULL for %zu bytes", b);
    bytes = b;
    return;
  }
  const size_t rb = cache_round(b);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_cache.find(CacheKey{dev, stream, rb});
  if (it != g_cache.end() && !it->second.empty()) {
    p = it->second.back();
    it->second.pop_back();
    bytes = b;
    cap = rb;
    return;
  }
  hipError_t e = hipMalloc(&p, rb);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    cache_trim();
    e = hipMalloc(&p, rb);
  }
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    HM_THROW(HM_ERR_ALLOC, "hipMalloc(%zu bytes) failed: %s", rb, hipGetErrorString(e));
  }
  bytes = b;
  cap = rb;
}

void DevBuf::release() {
  if (p) {
    if (hook.alloc) {
      hook.free(hook.ctx, p, stream);
    } else {
      int dev = 0;
      if (hipGetDevice(&dev) != hipSuccess) dev = 0;
      std::lock_guard<std::mutex> lk(g_cache_mu);
      g_cache[CacheKey{dev, stream, cap}].push_back(p);
    }
  }
  p = nullptr;
  bytes = 0;
  cap = 0;
}

void release_cached_memory() {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  cache_trim();
}

StreamBuf::StreamBuf(size_t b, hipStream_t s) : hook(alloc_hook()), stream(s) {
  if (b == 0) b = 16;
  if (hook.alloc) {
    p = hook.alloc(hook.ctx, b, s);
    if (!p) HM_THROW(HM_ERR_ALLOC, "caller's allocator returned NULL for %zu bytes", b);
  } else {
    hipError_t e = hipMallocAsync(&p, b, s);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      HM_THROW(HM_ERR_ALLOC, "hipMallocAsync(%zu bytes) failed: %s", b, hipGetErrorString(e));
    }
  }
}

StreamBuf::~StreamBuf() {
  if (!p) return;
  if (hook.alloc)
    hook.free(hook.ctx, p, stream);
  else
    (void)hipFreeAsync(p, stream);
}

// ------------------------------------------------------------- tuning -----
bool TuneKey::operator<(const TuneKey& o) const {
  if (n != o.n) return n < o.n;
  if (r != o.r) return r < o.r;
  if (levels != o.levels) return levels < o.levels;
  if (nmax != o.nmax) return nmax < o.nmax;
  if (instances != o.instances) return instances < o.instances;
  return sampler < o.sampler;
}

namespace {
std::mutex g_tune_mu;
std::map<TuneKey, TuneParams> g_tune;
thread_local TuneParams g_tune_cur;
}  // namespace

bool tune_lookup(const TuneKey& k, TuneParams* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(k);
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}
void tune_store(const TuneKey& k, const TuneParams& p) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[k] = p;
}
const TuneParams& tune_current() { return g_tune_cur; }
TuneScope::TuneScope(const TuneParams& p) : prev(g_tune_cur) { g_tune_cur = p; }
TuneScope::~TuneScope() { g_tune_cur = prev; }

// ------------------------------------------------------------ staging ------
namespace {
constexpr size_t kPinChunk = (size_t)64 << 10;
struct PinChunk {
  char* p = nullptr;
  void* dp = nullptr;   // the chunk as the device addresses it (null: copy engine only)
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  int dev = -1;
};

// A new pinned chunk of at least `bytes` on device `dev`.
PinChunk new_pin_chunk(size_t bytes, int dev) {
  PinChunk c;
  c.cap = std::max(kPinChunk, (bytes + kPinChunk - 1) / kPinChunk * kPinChunk);
  c.dev = dev;
  HIPCHK(hipHostMalloc((void**)&c.p, c.cap, hipHostMallocDefault));
  const hipError_t e = hipEventCreateWithFlags(&c.ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipHostFree(c.p);
    HM_THROW(HM_ERR_HIP, "hipEventCreate failed: %s", hipGetErrorString(e));
  }
  if (hipHostGetDevicePointer(&c.dp, c.p, 0) != hipSuccess) {
    (void)hipGetLastError();
    c.dp = nullptr;
  }
  return c;
}

// Host -> device copy by a kernel reading the pinned chunk: it runs in the
// stream's own queue, so the kernels around it do not wait for a copy
// engine to take over and hand back (~20 us per copy at the fine levels).
__global__ void k_stage_copy(char* __restrict__ dst, const char* __restrict__ src,
                             int64_t bytes) {
  const int64_t n16 = ((uintptr_t)dst % 16 == 0 && (uintptr_t)src % 16 == 0) ? bytes / 16 : 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < n16; i += stride)
    reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
  for (int64_t i = n16 * 16 + t0; i < bytes; i += stride) dst[i] = src[i];
}
std::mutex g_pin_mu;
std::deque<PinChunk> g_pin_busy;   // copies in flight, in order of use
std::vector<PinChunk> g_pin_free;
}  // namespace

void stage_h2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_pin_mu);
  while (!g_pin_busy.empty() && hipEventQuery(g_pin_busy.front().ev) == hipSuccess) {
    g_pin_free.push_back(g_pin_busy.front());
    g_pin_busy.pop_front();
  }
  (void)hipGetLastError();   // hipEventQuery's hipErrorNotReady
  PinChunk c;
  for (size_t i = 0; i < g_pin_free.size(); ++i)
    if (g_pin_free[i].cap >= bytes && g_pin_free[i].dev == dev) {
      c = g_pin_free[i];
      g_pin_free[i] = g_pin_free.back();
      g_pin_free.pop_back();
      break;
    }
  if (!c.p) c = new_pin_chunk(bytes, dev);
  std::memcpy(c.p, src, bytes);
  g_pin_busy.push_back(c);   // from here the chunk is owned by the queue
  if (c.dp) {
    const int64_t n16 = (int64_t)(bytes + 15) / 16;
    const int blocks = (int)std::min<int64_t>((n16 + 255) / 256, 64);
    hipLaunchKernelGGL(k_stage_copy, dim3(blocks), dim3(256), 0, s, static_cast<char*>(dst),
                       static_cast<const char*>(c.dp), (int64_t)bytes);
    HIPCHK(hipGetLastError());
  } else {
    HIPCHK(hipMemcpyAsync(dst, c.p, bytes, hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipEventRecord(c.ev, s));
}

// Several device -> host reads through one pinned chunk of the staging pool,
// then a wait for the stream: copies into pageable memory are staged by the
// runtime one at a time, each with its own host round trip.
void read_d2h(const std::vector<D2HRead>& items, hipStream_t s) {
  size_t total = 0;
  for (const D2HRead& it : items) total += (it.bytes + 255) / 256 * 256;
  if (total == 0) {
    HIPCHK(hipStreamSynchronize(s));
    return;
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  PinChunk c;
  {
    std::lock_guard<std::mutex> lock(g_pin_mu);
    for (size_t i = 0; i < g_pin_free.size(); ++i)
      if (g_pin_free[i].cap >= total && g_pin_free[i].dev == dev) {
        c = g_pin_free[i];
        g_pin_free[i] = g_pin_free.back();
        g_pin_free.pop_back();
        break;
      }
  }
  if (!c.p) c = new_pin_chunk(total, dev);
  // the chunk goes back to the pool whatever happens below, once the stream
  // is idle
  struct Return {
    PinChunk& c;
    hipStream_t s;
    ~Return() {
      (void)hipStreamSynchronize(s);   // no copy into the chunk is still in flight
      (void)hipGetLastError();
      std::lock_guard<std::mutex> lock(g_pin_mu);
      g_pin_free.push_back(c);
    }
  } ret{c, s};
  size_t off = 0;
  for (const D2HRead& it : items) {
    if (it.bytes)
      HIPCHK(hipMemcpyAsync(c.p + off, it.src, it.bytes, hipMemcpyDeviceToHost, s));
    off += (it.bytes + 255) / 256 * 256;
  }
  HIPCHK(hipStreamSynchronize(s));
  off = 0;
  for (const D2HRead& it : items) {
    if (it.bytes) std::memcpy(it.dst, c.p + off, it.bytes);
    off += (it.bytes + 255) / 256 * 256;
  }
}

// ------------------------------------------------------------------ forest
void forest_add_tree(Forest& f, int64_t n, int64_t leaf, int32_t r, int32_t k, int32_t p,
                     double tol, uint64_t seed) {
  Instance in{};
  in.row0 = f.n_total;
  in.n = n;
  in.leaf = leaf;
  in.L = 0;
  if (n > leaf) in.L = (int32_t)std::ceil(std::log2((double)n / (double)leaf) - 1e-12);
  while ((((n + (1ll << in.L) - 1) >> in.L)) > leaf) in.L++;  // guard log2 rounding
  in.r = r;
  in.k = k;
  in.p = p;
  in.tol = tol;
  in.seed = seed;
  in.root = (int32_t)f.nodes.size();
  const int id = (int)f.inst.size();
  // heap numbering inside the tree; global ids are base + heap - 1
  const int base = in.root;
  const int hs = 1 << (in.L + 1);
  for (int t = 1; t < hs; ++t) {
    Node nd{};
    nd.inst = id;
    nd.heap = t;
    nd.level = 31 - __builtin_clz((unsigned)t);
    nd.parent = t == 1 ? -1 : base + t / 2 - 1;
    nd.left = (t < (1 << in.L)) ? base + 2 * t - 1 : -1;
    nd.right = (t < (1 << in.L)) ? base + 2 * t : -1;
    nd.sib = t == 1 ? -1 : base + (t ^ 1) - 1;
    nd.is_left = (t > 1 && (t & 1) == 0) ? 1 : 0;
    f.nodes.push_back(nd);
  }
  // intervals: root [row0, row0+n); left child takes ceil(n/2)
  f.nodes[base].lo = in.row0;
  f.nodes[base].hi = in.row0 + n;
  for (int t = 1; t < (1 << in.L); ++t) {
    Node& P = f.nodes[base + t - 1];
    const int64_t mid = P.lo + (P.hi - P.lo + 1) / 2;
    f.nodes[base + 2 * t - 1].lo = P.lo;
    f.nodes[base + 2 * t - 1].hi = mid;
    f.nodes[base + 2 * t].lo = mid;
    f.nodes[base + 2 * t].hi = P.hi;
  }
  in.nmax = 0;
  for (int t = 1 << in.L; t < hs; ++t) {
    const Node& nd = f.nodes[base + t - 1];
    in.nmax = std::max<int32_t>(in.nmax, (int32_t)(nd.hi - nd.lo));
  }
  f.inst.push_back(in);
  f.n_total += n;
}

void forest_finish(Forest& f) {
  f.max_levels = 0;
  f.nmax = 0;
  for (auto& in : f.inst) {
    f.max_levels = std::max(f.max_levels, in.L);
    f.nmax = std::max(f.nmax, in.nmax);
  }
  f.level.assign(f.max_levels + 1, {});
  f.leaves.clear();
  for (int g = 0; g < (int)f.nodes.size(); ++g) {
    const Node& nd = f.nodes[g];
    f.level[nd.level].push_back(g);
    if (nd.left < 0) f.leaves.push_back(g);
  }
}

// -------------------------------------------------------------- Philox + BM
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += W0; k1 += W1;
  }
}

// Two Gaussians (columns 2*jp and 2*jp+1) of row i of the stream.
__device__ __forceinline__ void gauss_pair(uint64_t seed, int level, int phase, uint64_t i,
                                           uint32_t jp, double& z0, double& z1) {
  uint32_t c[4] = {(uint32_t)i, jp, (uint32_t)level, (uint32_t)phase};
  philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  const uint64_t m1 = (uint64_t)(c[0] >> 5) * 67108864ull + (uint64_t)(c[1] >> 6);
  const uint64_t m2 = (uint64_t)(c[2] >> 5) * 67108864ull + (uint64_t)(c[3] >> 6);
  const double u1 = ((double)m1 + 1.0) * 0x1.0p-53;
  const double u2 = (double)m2 * 0x1.0p-53;
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 2.0 * M_PI * u2;
  z0 = rad * cos(ang);
  z1 = rad * sin(ang);
}

__global__ void k_gauss_raw(uint64_t seed, int level, int phase, int64_t row0, int64_t nrows,
                            int ncols, double* out, int64_t ld) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  for (int jp = 0; 2 * jp < ncols; ++jp) {
    double z0, z1;
    gauss_pair(seed, level, phase, (uint64_t)(row0 + i), (uint32_t)jp, z0, z1);
    out[i + (int64_t)(2 * jp) * ld] = z0;
    if (2 * jp + 1 < ncols) out[i + (int64_t)(2 * jp + 1) * ld] = z1;
  }
}

void launch_gauss_raw(uint64_t seed, int level, int phase, int64_t row0, int64_t nrows,
                      int ncols, double* out, int64_t ld, hipStream_t s) {
  if (nrows <= 0 || ncols <= 0) return;
  const int nt = 256;
  hipLaunchKernelGGL(k_gauss_raw, dim3((unsigned)((nrows + nt - 1) / nt)), dim3(nt), 0, s, seed,
                     level, phase, row0, nrows, ncols, out, ld);
  KCHK();
}

__global__ void k_gauss_masked(const Node* nodes, const Instance* inst, const int32_t* kids,
                               int level, int R, double* Om, int64_t ld) {
  const Node nd = nodes[kids[blockIdx.y]];
  const Instance in = inst[nd.inst];
  const int64_t i = nd.lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nd.hi) return;
  const int off = nd.is_left ? R : 0;     // left child -> Omega_1 half
  const int oth = nd.is_left ? 0 : R;
  for (int j = 0; j < R; ++j) Om[i + (int64_t)(oth + j) * ld] = 0.0;
  for (int j = in.r; j < R; ++j) Om[i + (int64_t)(off + j) * ld] = 0.0;
  for (int jp = 0; 2 * jp < in.r; ++jp) {
    double z0, z1;
    gauss_pair(in.seed, level, 0, (uint64_t)(i - in.row0), (uint32_t)jp, z0, z1);
    Om[i + (int64_t)(off + 2 * jp) * ld] = z0;
    if (2 * jp + 1 < in.r) Om[i + (int64_t)(off + 2 * jp + 1) * ld] = z1;
  }
}

void launch_gauss_masked(const Node* nodes, const Instance* inst, const int32_t* kids, int nkids,
                         int64_t max_rows, int level, int R, double* Om, int64_t ld,
                         hipStream_t s) {
  if (nkids <= 0) return;
  const int nt = 256;
  hipLaunchKernelGGL(k_gauss_masked, dim3((unsigned)((max_rows + nt - 1) / nt), nkids), dim3(nt),
                     0, s, nodes, inst, kids, level, R, Om, ld);
  KCHK();
}

__global__ void k_mask_basis(const Node* nodes, const Instance* inst, const int32_t* kids, int R,
                             const double* U, int64_t ldu, double* Om, int64_t ld) {
  const Node nd = nodes[kids[blockIdx.y]];
  const int r = inst[nd.inst].r;
  const int64_t i = nd.lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nd.hi) return;
  const int off = nd.is_left ? R : 0;
  const int oth = nd.is_left ? 0 : R;
  for (int j = 0; j < R; ++j) Om[i + (int64_t)(oth + j) * ld] = 0.0;
  // fixed trip count (R <= HM_MAX_SAMPLES): every load in flight before the stores
  double v[HM_MAX_SAMPLES];
#pragma unroll
  for (int j = 0; j < HM_MAX_SAMPLES; ++j) v[j] = j < r ? U[i + (int64_t)j * ldu] : 0.0;
#pragma unroll
  for (int j = 0; j < HM_MAX_SAMPLES; ++j)
    if (j < R) Om[i + (int64_t)(off + j) * ld] = v[j];
}

void launch_mask_basis(const Node* nodes, const Instance* inst, const int32_t* kids, int nkids,
                       int64_t max_rows, int R, const double* U, int64_t ldu, double* Om,
                       int64_t ld, hipStream_t s) {
  if (nkids <= 0) return;
  const int nt = 256;
  hipLaunchKernelGGL(k_mask_basis, dim3((unsigned)((max_rows + nt - 1) / nt), nkids), dim3(nt), 0,
                     s, nodes, inst, kids, R, U, ldu, Om, ld);
  KCHK();
}

__global__ void k_block_eye(const Node* nodes, const int32_t* leaves, int j0, int nc, double* Om,
                            int64_t ld) {
  const Node nd = nodes[leaves[blockIdx.y]];
  const int64_t i = nd.lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nd.hi) return;
  const int64_t li = i - nd.lo;
  for (int j = 0; j < nc; ++j) Om[i + (int64_t)j * ld] = (j0 + j == li) ? 1.0 : 0.0;
}

void launch_block_eye(const Node* nodes, const int32_t* leaves, int nleaves, int64_t max_rows,
                      int nmax, double* Om, int64_t ld, hipStream_t s, int j0, int nc) {
  if (nleaves <= 0) return;
  if (nc < 0) nc = nmax - j0;
  if (j0 < 0 || nc <= 0 || j0 + nc > nmax) return;
  const int nt = 256;
  hipLaunchKernelGGL(k_block_eye, dim3((unsigned)((max_rows + nt - 1) / nt), nleaves), dim3(nt),
                     0, s, nodes, leaves, j0, nc, Om, ld);
  KCHK();
}

__global__ void k_zero_dpad(const Node* nodes, const int32_t* leaves, int nmax, double* D,
                            int64_t ld) {
  const Node nd = nodes[leaves[blockIdx.y]];
  const int64_t i = nd.lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nd.hi) return;
  for (int j = (int)(nd.hi - nd.lo); j < nmax; ++j) D[i + (int64_t)j * ld] = 0.0;
}

void launch_zero_dpad(const Node* nodes, const int32_t* leaves, int nleaves, int64_t max_rows,
                      int nmax, double* D, int64_t ld, hipStream_t s) {
  if (nleaves <= 0) return;
  const int nt = 256;
  hipLaunchKernelGGL(k_zero_dpad, dim3((unsigned)((max_rows + nt - 1) / nt), nleaves), dim3(nt),
                     0, s, nodes, leaves, nmax, D, ld);
  KCHK();
}

__global__ void k_fill(double* p, int64_t rows, int64_t cols, int64_t ld, double v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= rows) return;
  for (int64_t j = 0; j < cols; ++j) p[i + j * ld] = v;
}

void launch_fill(double* p, int64_t rows, int64_t cols, int64_t ld, double v, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  const int nt = 256;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((rows + nt - 1) / nt)), dim3(nt), 0, s, p, rows,
                     cols, ld, v);
  KCHK();
}

__global__ void k_fill_f(float* p, int64_t count, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_fill_f(float* p, int64_t count, float v, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill_f, dim3(1024), dim3(256), 0, s, p, count, v);
  KCHK();
}

// Element type conversion of a column-major block: FP64 <-> FP32, and FP64 ->
// BF16 (round to nearest even on the FP32 value's bits; NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ void k_convert(const void* src, int sdt, int64_t lds, void* dst, int ddt, int64_t ldd,
                          int64_t rows, int64_t cols) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= rows) return;
  for (int64_t j = blockIdx.y; j < cols; j += gridDim.y) {
    double v;
    if (sdt == HM_F64) v = static_cast<const double*>(src)[i + j * lds];
    else v = (double)static_cast<const float*>(src)[i + j * lds];
    if (ddt == HM_F64) static_cast<double*>(dst)[i + j * ldd] = v;
    else if (ddt == HM_F32) static_cast<float*>(dst)[i + j * ldd] = (float)v;
    else static_cast<uint16_t*>(dst)[i + j * ldd] = f32_to_bf16_bits((float)v);
  }
}

void launch_convert(const void* src, int sdt, int64_t lds, void* dst, int ddt, int64_t ldd,
                    int64_t rows, int64_t cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  if (sdt == HM_BF16) HM_THROW(HM_ERR_ARG, "convert: BF16 is an output type only");
  const int nt = 256;
  hipLaunchKernelGGL(k_convert,
                     dim3((unsigned)((rows + nt - 1) / nt), (unsigned)std::min<int64_t>(cols, 64)),
                     dim3(nt), 0, s, src, sdt, lds, dst, ddt, ldd, rows, cols);
  KCHK();
}

// out[2j] = ||a_j - b_j||^2, out[2j + 1] = ||a_j||^2 for the columns of two
// rows x cols blocks: one workgroup per column
__global__ __launch_bounds__(256) void k_col_err2(const double* A, int64_t lda, const double* B,
                                                  int64_t ldb, int64_t rows, double* out) {
  __shared__ double sd[256], sa[256];
  const int j = blockIdx.x;
  double d2 = 0.0, a2 = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += 256) {
    const double a = A[i + j * lda], d = a - B[i + j * ldb];
    d2 = fma(d, d, d2);
    a2 = fma(a, a, a2);
  }
  sd[threadIdx.x] = d2;
  sa[threadIdx.x] = a2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sd[threadIdx.x] += sd[threadIdx.x + w];
      sa[threadIdx.x] += sa[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * j] = sd[0];
    out[2 * j + 1] = sa[0];
  }
}

void launch_col_err2(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t rows,
                     int cols, double* out, hipStream_t s) {
  if (cols <= 0) return;
  hipLaunchKernelGGL(k_col_err2, dim3(cols), dim3(256), 0, s, A, lda, B, ldb, rows, out);
  KCHK();
}

// one thread per row and group of NF_COLS columns (independent loads in flight)
constexpr int NF_COLS = 8;
__global__ void k_nonfinite(const double* p, int64_t rows, int64_t cols, int64_t ld, int* flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const int64_t j0 = (int64_t)blockIdx.y * NF_COLS;
  bool bad = false;
#pragma unroll
  for (int q = 0; q < NF_COLS; ++q)
    if (j0 + q < cols) bad |= !isfinite(p[i + (j0 + q) * ld]);
  if (bad) atomicOr(flag, 1);
}

void launch_nonfinite_check(const double* p, int64_t rows, int64_t cols, int64_t ld, int* flag,
                            hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  const int nt = 256;
  hipLaunchKernelGGL(k_nonfinite,
                     dim3((unsigned)((rows + nt - 1) / nt), (unsigned)((cols + NF_COLS - 1) / NF_COLS)),
                     dim3(nt), 0, s, p, rows, cols, ld, flag);
  KCHK();
}

}  // namespace hm
