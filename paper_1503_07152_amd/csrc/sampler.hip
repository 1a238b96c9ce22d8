// Built-in black-box operators Y = A X for the sampling step (the T_mult of
// Sec. 1): a kernel matrix A(i,j) = K(x_i, x_j) on 2-D points evaluated tile
// by tile on the fly (never stored), or an explicit dense matrix.  The
// contraction runs on MFMA:
//   F64  : v_mfma_f64_16x16x4f64, entries in FP64
//   F32  : v_mfma_f32_16x16x4f32, entries in FP32 (coordinate differences in FP64)
//   BF16 : v_mfma_f32_16x16x32_bf16, entries rounded to BF16, FP32 accumulation
// X is first packed K-tile-major in the contraction type, and a bitmask per
// K-tile records which 16-column groups are nonzero: the structured test
// matrices of Fig. 2/4 (half of every row zero) and the block identity of the
// diagonal step then skip the MFMAs of zero groups.
#include <hip/hip_bf16.h>

#include "sampler.h"

namespace hm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Block shape per form.  BF16 up to 12 column tiles (72 to 90 VGPRs): 8
// waves of one 16-row tile each.  The widest BF16 form (18 column tiles, ~207
// VGPRs, two waves per SIMD): 8 waves of two 16-row tiles, 256 rows per
// block, which halves the X tiles each CU streams per row and lets every B
// operand read from LDS feed two MFMAs (4-6 % faster than one row tile per
// wave at 288 columns; two row tiles with 4 waves gain nothing, and the
// narrower forms lose by it).  FP32 (FP32 and FP64 accumulators, ~420
// registers with the AGPRs) and FP64 (~190): 4 waves of two 16-row tiles.
template <int MODE, int CT>
struct SmpShape {
  static constexpr int WAVES = MODE == 2 ? 8 : 4;
  static constexpr int RT = (MODE == 2 && CT <= 12) ? 1 : 2;    // 16-row tiles per wave
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int ROWS = WAVES * 16 * RT;    // rows per block
};

template <int MODE> struct ModeT;
template <> struct ModeT<0> { typedef double T; static constexpr int BK = 16; };
template <> struct ModeT<1> { typedef float T; static constexpr int BK = 16; };
template <> struct ModeT<2> { typedef __bf16 T; static constexpr int BK = 64; };

int sampler_bk(int mode) { return mode == 2 ? 64 : 16; }
int sampler_max_cols(int mode) { return mode == 2 ? SMP_MAXC_BF16 : SMP_MAXC; }

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// K-splits of the narrow BF16 form (see run_sampler).  Split counts that
// divide 8 map onto XCD groups (k_sampler); measured at 96 columns that cuts
// the sampler's fetch from 183 to 160 MB per call at equal time, and three
// splits stay the fastest default.
constexpr int SMP_KSPLIT = 3;
static int sampler_ksplit(int mode, int64_t n, int c) {
  const int64_t nkt = (n + sampler_bk(mode) - 1) / sampler_bk(mode);
  const int ks = tune_current().ksplit > 0 ? tune_current().ksplit : SMP_KSPLIT;
  return (mode == 2 && c <= 128) ? (int)std::min<int64_t>(ks, nkt) : 1;
}

size_t sampler_pack_bytes(int mode, int64_t n, int c) {
  const int bk = sampler_bk(mode);
  const int64_t kt = (n + bk - 1) / bk;
  const int cp = ((c + 15) / 16) * 16;
  const size_t es = mode == 0 ? 8 : (mode == 1 ? 4 : 2);
  const int ks = sampler_ksplit(mode, n, c);
  return align256((size_t)kt * bk * cp * es) + align256((size_t)kt * 4) +
         (ks > 1 ? align256((size_t)ks * n * c * 4) : 0) + 512;
}

// Pack: F64/F32 tiles [kt][k][col]; BF16 tiles [kt][col][k].
template <int MODE>
__global__ void k_pack(int64_t n, int c, int cp, const double* X, int64_t ldx,
                       typename ModeT<MODE>::T* Xp, uint32_t* mask) {
  typedef typename ModeT<MODE>::T T;
  constexpr int BK = ModeT<MODE>::BK;
  __shared__ uint32_t m;
  const int64_t kt = blockIdx.x;
  if (threadIdx.x == 0) m = 0;
  __syncthreads();
  uint32_t mine = 0;
  T* tile = Xp + kt * (int64_t)BK * cp;
  for (int e = threadIdx.x; e < BK * cp; e += blockDim.x) {
    int k, col;
    if (MODE == 2) { k = e % BK; col = e / BK; } else { col = e % cp; k = e / cp; }
    const int64_t row = kt * BK + k;
    double v = 0.0;
    if (row < n && col < c) v = X[row + (int64_t)col * ldx];
    if (v != 0.0) mine |= 1u << (col / 16);
    tile[e] = (T)v;
  }
  if (mine) atomicOr(&m, mine);
  __syncthreads();
  if (threadIdx.x == 0) mask[kt] = m;
}

// FP64 entry.  Near kernel: sqrt(d2) and 1 / (r + kp) from the hardware
// reciprocal (square root) estimates, each refined by Newton steps in
// residual form (within an ulp or two of the IEEE results, a fraction of the
// instruction count of the IEEE sequences); d2 = 0 gives r = 0.
template <int SRC>
__device__ __forceinline__ double entry_f64(double xi, double yi, double xj, double yj, int64_t gi,
                                            int64_t gj, double kp) {
  const double dx = xi - xj, dy = yi - yj;
  const double d2 = fma(dx, dx, dy * dy);
  if (SRC == 0) return gi == gj ? 1.0 : 0.5 * log(d2);
  double t = __builtin_amdgcn_rsq(d2);   // 1 / sqrt(d2)
#pragma unroll
  for (int it = 0; it < 2; ++it) t = fma(t, fma(-0.5 * d2 * t, t, 0.5), t);
  double r = d2 * t;
  r = fma(0.5 * t, fma(-r, r, d2), r);
  r = d2 > 0.0 ? r : 0.0;
  const double den = r + kp;
  double y = __builtin_amdgcn_rcp(den);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(y, fma(-den, y, 1.0), y);
  return y;
}

template <int SRC>
__device__ __forceinline__ float entry_f32(double xi, double yi, double xj, double yj, int64_t gi,
                                           int64_t gj, float kp) {
  const float dx = (float)(xi - xj), dy = (float)(yi - yj);
  const float d2 = fmaf(dx, dx, dy * dy);
  if (SRC == 0) return gi == gj ? 1.0f : 0.34657359027997264f * __builtin_amdgcn_logf(d2);
  return __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(d2) + kp);
}

// FP32 entry from FP32 coordinates (BF16 form: the coordinate rounding,
// ~6e-8 absolute, stays far below BF16 resolution of the entry).
template <int SRC>
__device__ __forceinline__ float entry_f32c(float xi, float yi, float xj, float yj, int64_t gi,
                                            int64_t gj, float kp) {
  const float dx = xi - xj, dy = yi - yj;
  const float d2 = fmaf(dx, dx, dy * dy);
  if (SRC == 0) return gi == gj ? 1.0f : 0.34657359027997264f * __builtin_amdgcn_logf(d2);
  return __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(d2) + kp);
}

// K-tiles between flushes of the FP32 MFMA accumulators into FP64 (FP32 form)
constexpr int SMP_FLUSH = 32;
// Column tiles handled together: their B operands are read from LDS back to
// back, then their MFMAs issued, so one LDS latency serves SMP_GS MFMAs.  The
// nonzero mask is tested per group (a group with any nonzero tile multiplies
// all of its tiles, the zero ones included; the structured test matrices
// switch whole halves of 3 tiles on and off when r = 48).  Tiles past c hold
// stale LDS data and feed accumulators that are never stored.
constexpr int SMP_GS = 3;
// (depends on col % 16 only, so the LDS offsets of all column tiles differ by
// constants)
__device__ __forceinline__ int swz(int col) { return (col ^ ((col >> 3) & 1)) & 7; }

// SRC: 0 log kernel, 1 near-singular kernel, 2 dense matrix, 3 its transpose (F64 only).
// One block = SmpShape<MODE, CT>::WAVES waves x RT 16-row tiles; X is streamed
// through LDS in K-tiles (the K-tiles of split sp), double-buffered,
// the next tile in flight (registers for F64 / F32, global_load_lds for BF16)
// while the current one feeds the MFMAs.
// CT column tiles of 16 are held in the accumulators (c <= 16 CT); the BF16
// form takes up to 18, so one pass over the entries serves several sample
// blocks at once.
// The FP32 form is held to two waves per SIMD (244 VGPRs, no spills): left
// to itself the compiler took 300 registers and one wave per SIMD, 1.6x slower.
template <int MODE, int SRC, int CT>
__global__ __launch_bounds__((SmpShape<MODE, CT>::THREADS))
__attribute__((amdgpu_waves_per_eu(MODE == 1 ? 2
                                   : (MODE == 2 && CT > 12 ? 2 : (MODE == 2 && CT > 8 ? 4 : 1)))))
void k_sampler(
    int64_t n, int c, int cp, const double* __restrict__ pts, double kp,
    const double* __restrict__ Ad, int64_t lda, const typename ModeT<MODE>::T* __restrict__ Xp,
    const uint32_t* __restrict__ mask, double* __restrict__ Y, int64_t ldy, int64_t kt_chunk,
    float* __restrict__ Ypart) {
  typedef typename ModeT<MODE>::T T;
  constexpr int BK = ModeT<MODE>::BK;
  constexpr int SMP_THREADS = SmpShape<MODE, CT>::THREADS;
  constexpr int SMP_ROWS = SmpShape<MODE, CT>::ROWS;
  constexpr int SMP_RT = SmpShape<MODE, CT>::RT;
  constexpr int SMP_CT = CT;
  constexpr int TILE_BYTES = BK * 16 * CT * (int)sizeof(T);
  constexpr int NV = (TILE_BYTES + SMP_THREADS * 16 - 1) / (SMP_THREADS * 16);  // uint4 per thread
  // BF16 tiles are column-major (BK = 64 contiguous k per column, eight
  // 16-byte chunks); chunk q of column col sits at slot q ^ swz(col).  A
  // B-operand read takes chunk q of 16 consecutive columns: swz is one-to-one
  // on any 8 consecutive columns (one 128-byte bank row each) and on the even
  // and on the odd ones of 16 (two columns per 256-byte bank row), so the
  // reads spread over all banks with 32 or with 64 banks of 4 bytes.
  static_assert(MODE != 2 || BK == 64, "BF16 swizzle assumes 8 chunks per column");
  // two separate arrays, not one of two buffers: the waits that the compiler
  // puts before LDS reads for outstanding global_load_lds writes are skipped
  // only when the write and the read provably address different objects
  __shared__ __attribute__((aligned(16))) T sX0[BK * 16 * CT + 16];
  __shared__ __attribute__((aligned(16))) T sX1[BK * 16 * CT + 16];
  // point coordinates of the K-tile: FP64 (FP64 / FP32 forms), FP32 (BF16 form)
  __shared__ double sP[2][MODE == 2 ? 1 : 2 * BK];
  __shared__ __attribute__((aligned(8))) float sPf[2][MODE == 2 ? 2 * BK : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // Row block rb and K-split sp of this workgroup.  Workgroups go to the 8
  // XCDs round-robin by linear id; when the split count divides 8, the linear
  // id is mapped so that every block of split sp runs on the XCDs x = sp
  // (mod splits), whose L2s then stream only that split's part of X.
  int rb = blockIdx.x, sp = blockIdx.y;
  if (gridDim.y > 1 && 8 % gridDim.y == 0 && (gridDim.x * gridDim.y) % 8 == 0) {
    const int ks = gridDim.y, L = blockIdx.x + blockIdx.y * gridDim.x;
    const int x = L & 7, q = L >> 3;
    sp = x % ks;
    rb = q * (8 / ks) + x / ks;
  }
  const int64_t row0 = (int64_t)rb * SMP_ROWS + wave * 16 * SMP_RT;
  const int ct_n = cp / 16;
  const int tile_u4 = BK * cp * (int)sizeof(T) / 16;
  double xi[SMP_RT], yi[SMP_RT];
  float xif[SMP_RT], yif[SMP_RT];
  int64_t gi[SMP_RT];
#pragma unroll
  for (int rt = 0; rt < SMP_RT; ++rt) {
    gi[rt] = row0 + rt * 16 + (lane & 15);
    const int64_t ii = gi[rt] < n ? gi[rt] : n - 1;
    if (SRC < 2) {
      xi[rt] = pts[2 * ii]; yi[rt] = pts[2 * ii + 1];
      xif[rt] = (float)xi[rt]; yif[rt] = (float)yi[rt];
    }
  }
  typedef typename std::conditional<MODE == 0, d4, f4>::type acc_t;
  acc_t acc[SMP_RT][SMP_CT];
  d4 acc64[MODE == 1 ? SMP_RT : 1][MODE == 1 ? SMP_CT : 1];
#pragma unroll
  for (int rt = 0; rt < SMP_RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < SMP_CT; ++ct) acc[rt][ct] = acc_t{0, 0, 0, 0};
  if constexpr (MODE == 1) {
#pragma unroll
    for (int rt = 0; rt < SMP_RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < SMP_CT; ++ct) acc64[rt][ct] = d4{0, 0, 0, 0};
  }
  const int64_t nkt = (n + BK - 1) / BK;
  // F64 / F32: prefetch registers for the next K-tile (plain statements, not
  // a lambda capture, so the array stays in VGPRs).  BF16: the next tile goes
  // from global memory straight into its LDS buffer (global_load_lds, 16
  // bytes per lane; lane l of a wave fills slot base + l, so it fetches the
  // global chunk that the swizzle puts there), waited for before the barrier
  // that publishes it; no registers held across the MFMAs.
  uint4 pre[MODE == 2 ? 1 : NV];
  double pp = 0.0;
#define HM_SMP_FETCH(KT, BUF)                                                         \
  {                                                                                   \
    const uint4* src_ = reinterpret_cast<const uint4*>(Xp + (KT) * (int64_t)BK * cp); \
    if constexpr (MODE == 2) {                                                        \
      uint4* dst_ = reinterpret_cast<uint4*>((BUF) ? sX1 : sX0);                      \
      _Pragma("unroll") for (int v = 0; v < NV; ++v) {                                \
        const int base_ = (v * (SMP_THREADS / 64) + wave) * 64;                       \
        if (base_ < tile_u4) {                                                        \
          const int d_ = base_ + lane;                                                \
          const int e_ = (d_ & ~7) | ((d_ ^ swz(d_ >> 3)) & 7);                       \
          __builtin_amdgcn_global_load_lds(                                           \
              (const void*)(src_ + e_),                                               \
              (__attribute__((address_space(3))) void*)(dst_ + base_), 16, 0, 0);     \
        }                                                                             \
      }                                                                               \
    } else {                                                                          \
      _Pragma("unroll") for (int v = 0; v < NV; ++v) {                                \
        const int e = tid + v * SMP_THREADS;                                          \
        pre[v] = e < tile_u4 ? src_[e] : uint4{0, 0, 0, 0};                           \
      }                                                                               \
    }                                                                                 \
    if (SRC < 2 && tid < 2 * BK) {                                                    \
      const int64_t j_ = (KT) * BK + tid / 2;                                         \
      pp = j_ < n ? pts[2 * j_ + (tid & 1)] : (MODE == 2 ? 1e15 : 0.0);               \
    }                                                                                 \
  }
#define HM_SMP_STASH(BUF)                                                             \
  {                                                                                   \
    if constexpr (MODE == 2) {                                                        \
      __builtin_amdgcn_s_waitcnt(0x0F70); /* vmcnt(0): this wave's tile loads */     \
    } else {                                                                          \
      uint4* dst_ = reinterpret_cast<uint4*>((BUF) ? sX1 : sX0);                      \
      _Pragma("unroll") for (int v = 0; v < NV; ++v) {                                \
        const int e = tid + v * SMP_THREADS;                                          \
        if (e < tile_u4) dst_[e] = pre[v];                                            \
      }                                                                               \
    }                                                                                 \
    if (SRC < 2 && tid < 2 * BK) {                                                    \
      if constexpr (MODE == 2) sPf[BUF][tid] = (float)pp;                             \
      else sP[BUF][tid] = pp;                                                         \
    }                                                                                 \
  }
  // the nonzero mask of a K-tile is read with its tile, one iteration ahead:
  // a load issued after the prefetch and waited for at once would also wait
  // for the prefetch (loads complete in order)
  // K-tiles kt_beg .. kt_end - 1 of this split (sp); kk counts them
  const int64_t kt_beg = (int64_t)sp * kt_chunk;
  const int64_t kt_end = min(nkt, kt_beg + kt_chunk);
  const int64_t nkk = max(kt_end - kt_beg, (int64_t)0);
  uint32_t msk_nx = 0;
  if (nkk > 0) {
    msk_nx = mask[kt_beg];
    HM_SMP_FETCH(kt_beg, 0)
    HM_SMP_STASH(0)
  }
  __syncthreads();
  // unrolled by two so that the buffer of each copy is known statically
#pragma unroll 2
  for (int64_t kk = 0; kk < nkk; ++kk) {
    const int64_t kt = kt_beg + kk;
    const int buf = (int)(kk & 1);
    const uint32_t msk = msk_nx;
    if (kk + 1 < nkk) {
      msk_nx = mask[kt + 1];
      HM_SMP_FETCH(kt + 1, buf ^ 1)
    }
    const T* xs = buf ? sX1 : sX0;
    const double* ps = sP[buf];
    if (msk != 0) {
      if constexpr (MODE == 0 || MODE == 1) {
#pragma unroll
        for (int s = 0; s < BK / 4; ++s) {
          const int jl = 4 * s + (lane >> 4);
          const int64_t gj = kt * BK + jl;
          T a[SMP_RT];
#pragma unroll
          for (int rt = 0; rt < SMP_RT; ++rt) {
            T v = T(0);
            if (gj < n) {
              if constexpr (SRC == 2 || SRC == 3) {
                const int64_t ii = gi[rt] < n ? gi[rt] : n - 1;
                v = SRC == 2 ? (T)Ad[ii + gj * lda] : (T)Ad[gj + ii * lda];
              } else if constexpr (MODE == 0) {
                v = (T)entry_f64<SRC>(xi[rt], yi[rt], ps[2 * jl], ps[2 * jl + 1], gi[rt], gj, kp);
              } else {
                v = (T)entry_f32<SRC>(xi[rt], yi[rt], ps[2 * jl], ps[2 * jl + 1], gi[rt], gj,
                                      (float)kp);
              }
            }
            a[rt] = v;
          }
#pragma unroll
          for (int g0 = 0; g0 < SMP_CT; g0 += SMP_GS) {
            if (g0 >= ct_n || !((msk >> g0) & ((1u << SMP_GS) - 1))) continue;
            T b[SMP_GS];
#pragma unroll
            for (int t = 0; t < SMP_GS; ++t)
              if (g0 + t < SMP_CT) b[t] = xs[jl * cp + (g0 + t) * 16 + (lane & 15)];
#pragma unroll
            for (int t = 0; t < SMP_GS; ++t)
#pragma unroll
              for (int rt = 0; rt < SMP_RT; ++rt) {
                const int ct = g0 + t;
                if (ct >= SMP_CT) continue;
                if constexpr (MODE == 0)
                  acc[rt][ct] =
                      __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt], b[t], acc[rt][ct], 0, 0, 0);
                else
                  acc[rt][ct] =
                      __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt], b[t], acc[rt][ct], 0, 0, 0);
              }
          }
        }
      } else {
        // BF16: per 32-row K-step s, lane holds A(row, 32 s + 8*(lane/16) + e),
        // e = 0..7, and X(32 s + 8*(lane/16) + e, col).  Points past n sit at
        // 1e15 (finite entries against zero rows of X), so no bounds test.
        const int kb = 8 * (lane >> 4);
        const float* psf = sPf[buf];
#pragma unroll
        for (int s = 0; s < BK / 32; ++s) {
          bf8 a[SMP_RT];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int jl = 32 * s + kb + e;
            const float2 pj = *reinterpret_cast<const float2*>(&psf[2 * jl]);
#pragma unroll
            for (int rt = 0; rt < SMP_RT; ++rt) {
              float v;
              if constexpr (SRC >= 2) {
                const int64_t gj = kt * BK + jl;
                v = gj < n ? entry_f32c<1>(xif[rt], yif[rt], pj.x, pj.y, gi[rt], gj, (float)kp) : 0.0f;
              } else {
                v = entry_f32c<SRC>(xif[rt], yif[rt], pj.x, pj.y, gi[rt], kt * BK + jl, (float)kp);
              }
              a[rt][e] = (__bf16)v;
            }
          }
#pragma unroll
          for (int g0 = 0; g0 < SMP_CT; g0 += SMP_GS) {
            if (g0 >= ct_n || !((msk >> g0) & ((1u << SMP_GS) - 1))) continue;
            bf8 b[SMP_GS];
#pragma unroll
            for (int t = 0; t < SMP_GS; ++t) {
              const int col = (g0 + t) * 16 + (lane & 15);
              const int q = 4 * s + (lane >> 4);
              if (g0 + t < SMP_CT)
                b[t] = *reinterpret_cast<const bf8*>(&xs[col * BK + 8 * (q ^ swz(col))]);
            }
#pragma unroll
            for (int t = 0; t < SMP_GS; ++t)
#pragma unroll
              for (int rt = 0; rt < SMP_RT; ++rt)
                if (g0 + t < SMP_CT)
                  acc[rt][g0 + t] =
                      __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt], b[t], acc[rt][g0 + t], 0, 0, 0);
          }
        }
      }
    }
    if constexpr (MODE == 1) {
      if ((kk % SMP_FLUSH) == SMP_FLUSH - 1 || kk + 1 == nkk) {
#pragma unroll
        for (int rt = 0; rt < SMP_RT; ++rt)
#pragma unroll
          for (int ct = 0; ct < SMP_CT; ++ct) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[rt][ct][v] += (double)acc[rt][ct][v];
            acc[rt][ct] = acc_t{0, 0, 0, 0};
          }
      }
    }
    if (kk + 1 < nkk) HM_SMP_STASH(buf ^ 1)
    __syncthreads();
  }
  // one split writes Y; several (BF16 form only) write their FP32 partial
  // sums, added in FP64 in split order by k_sum_parts
  const bool part = gridDim.y > 1;
  float* Yq = part ? Ypart + (int64_t)sp * n * c : nullptr;
  // Accumulator layout (column lane % 16 of each 16 x 16 tile): item v of lane
  // l holds row 4*(l/16) + v for the FP32-accumulating instructions and row
  // l/16 + 4*v for v_mfma_f64_16x16x4f64 (checked on gfx950 with identity inputs).
#pragma unroll
  for (int rt = 0; rt < SMP_RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < SMP_CT; ++ct) {
      const int col = ct * 16 + (lane & 15);
      if (ct >= ct_n || col >= c) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = MODE == 0 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
        const int64_t row = row0 + rt * 16 + rr;
        if (row >= n) continue;
        if constexpr (MODE == 1) {
          Y[row + (int64_t)col * ldy] = acc64[rt][ct][v];
        } else if constexpr (MODE == 2) {
          if (part) Yq[row + (int64_t)col * n] = acc[rt][ct][v];
          else Y[row + (int64_t)col * ldy] = (double)acc[rt][ct][v];
        } else {
          Y[row + (int64_t)col * ldy] = acc[rt][ct][v];
        }
      }
    }
}

// Y = sum of the ks FP32 partial products (n x c each, ld n), in FP64, in
// split order
__global__ void k_sum_parts(int64_t n, int c, int ks, const float* __restrict__ Yp,
                            double* __restrict__ Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int64_t i = e % n, j = e / n;
  double v = (double)Yp[e];
  for (int q = 1; q < ks; ++q) v += (double)Yp[(int64_t)q * n * c + e];
  Y[i + j * ldy] = v;
}

#undef HM_SMP_FETCH
#undef HM_SMP_STASH

template <int MODE, int SRC>
static void run_sampler(int64_t n, int c, const double* pts, double kp, const double* Ad,
                        int64_t lda, const double* X, int64_t ldx, double* Y, int64_t ldy,
                        void* work, hipStream_t s) {
  typedef typename ModeT<MODE>::T T;
  constexpr int BK = ModeT<MODE>::BK;
  const int cp = ((c + 15) / 16) * 16;
  const int64_t nkt = (n + BK - 1) / BK;
  T* Xp = static_cast<T*>(work);
  const size_t xbytes = align256((size_t)nkt * BK * cp * sizeof(T));
  uint32_t* mask = reinterpret_cast<uint32_t*>(static_cast<char*>(work) + xbytes);
  hipLaunchKernelGGL(k_pack<MODE>, dim3((unsigned)nkt), dim3(256), 0, s, n, c, cp, X, ldx, Xp,
                     mask);
  KCHK();
  // The narrow BF16 form (72 VGPRs: seven waves per SIMD) splits the K-tiles
  // in SMP_KSPLIT parts (or the tuned count), one block row each: 65536 rows
  // give 512 blocks of 8 waves, four per SIMD, which the split raises to what
  // the registers allow.  The wider forms are held to fewer waves per SIMD by
  // their registers, which 512 (256) blocks already fill.
  const int ks = sampler_ksplit(MODE, n, c);
  const int64_t kt_chunk = (nkt + ks - 1) / ks;
  float* Yp = ks > 1 ? reinterpret_cast<float*>(static_cast<char*>(work) + xbytes +
                                                align256((size_t)nkt * 4))
                     : nullptr;
  auto launch = [&](auto kern, auto shape) {
    typedef decltype(shape) Sh;
    const dim3 grid((unsigned)((n + Sh::ROWS - 1) / Sh::ROWS), (unsigned)ks), block(Sh::THREADS);
    hipLaunchKernelGGL(kern, grid, block, 0, s, n, c, cp, pts, kp, Ad, lda, Xp, mask, Y, ldy,
                       kt_chunk, Yp);
    KCHK();
  };
  constexpr int CT12 = MODE == 2 ? 12 : 8, CT18 = MODE == 2 ? 18 : 8;
  if (MODE != 2 || c <= 128)
    launch(k_sampler<MODE, SRC, 8>, SmpShape<MODE, 8>());
  else if (c <= 192)
    launch(k_sampler<MODE, SRC, CT12>, SmpShape<MODE, CT12>());
  else
    launch(k_sampler<MODE, SRC, CT18>, SmpShape<MODE, CT18>());
  if (ks > 1) {
    const int64_t tot = n * c;
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, c, ks,
                       Yp, Y, ldy);
    KCHK();
  }
}

void sampler_apply(int mode, int src, int64_t n, int c, const double* pts, double kp,
                   const double* Ad, int64_t lda, const double* X, int64_t ldx, double* Y,
                   int64_t ldy, void* work, hipStream_t s) {
  if (n <= 0 || c <= 0) return;
  if (c > sampler_max_cols(mode))
    HM_THROW(HM_ERR_UNSUPPORTED, "sampler: %d columns > %d", c, sampler_max_cols(mode));
  if (src >= 2 && mode != 0) HM_THROW(HM_ERR_ARG, "dense operator samples in FP64 only");
#define CASE(M, S) \
  if (mode == M && src == S) return run_sampler<M, S>(n, c, pts, kp, Ad, lda, X, ldx, Y, ldy, work, s);
  CASE(0, 0) CASE(0, 1) CASE(0, 2) CASE(0, 3) CASE(1, 0) CASE(1, 1) CASE(2, 0) CASE(2, 1)
#undef CASE
  HM_THROW(HM_ERR_ARG, "sampler: bad mode %d / source %d", mode, src);
}

}  // namespace hm
