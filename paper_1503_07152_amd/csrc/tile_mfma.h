// 64 x 64 output tiles on the matrix cores (FP32 MFMA 16x16x4 for float, FP64
// MFMA 16x16x4 for double) for the apply, gradient and segmented-product
// kernels: a 256-thread workgroup, wave w owns rows 16 w .. 16 w + 15 of the
// tile and all four 16-column tiles (four accumulators).  Operands are read
// through strides like the LDS tile of tile.h (op(A)(i, k) = A[i sai + k sak],
// op(B)(k, j) = B[k sbk + j sbj]) and staged in LDS in K-chunks of MF_KC,
// each in the layout that keeps both its global loads and its MFMA reads
// cheap: an operand whose unit stride runs along the output index is stored
// K-major, one whose unit stride runs along K is stored index-major.
//
// Operand layout of both MFMAs (checked on the device): A(i, k) comes from
// lane i + 16 k, B(k, j) from lane j + 16 k.  Accumulator item v of lane l
// holds row 4 (l / 16) + v (FP32) or row l / 16 + 4 v (FP64), column l % 16.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hm {

constexpr int MF_T = 64;    // tile rows and columns
constexpr int MF_KC = 32;   // K-chunk staged per round
constexpr int MF_PK = MF_T + 16;   // pitch of a K-major operand row (bank spread)
constexpr int MF_PI = MF_KC + 1;   // pitch of an index-major operand row

typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef double mf_d4 __attribute__((ext_vector_type(4)));

template <class T> struct MfTraits;
template <> struct MfTraits<float> {
  typedef mf_f4 acc_t;
  __device__ static acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct MfTraits<double> {
  typedef mf_d4 acc_t;
  __device__ static acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <class T>
struct MfAcc {
  typename MfTraits<T>::acc_t v[4];
  __device__ void zero() {
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = typename MfTraits<T>::acc_t{0, 0, 0, 0};
  }
};

// LDS elements of one mf_tile call (A and B chunk buffers).
template <class T>
constexpr int mf_smem_elems() {
  return 2 * (MF_KC * MF_PK > MF_T * MF_PI ? MF_KC * MF_PK : MF_T * MF_PI);
}

// One operand's share of a K-chunk: each thread moves MF_R = 64 * MF_KC / 256
// elements (idx, k) -> LDS.  kmajor (unit stride along idx): consecutive
// threads take consecutive idx and the chunk is stored buf[k * MF_PK + idx];
// otherwise consecutive threads take consecutive k, stored buf[idx * MF_PI + k].
constexpr int MF_R = MF_T * MF_KC / 256;

template <class T>
struct MfStager {
  const T* base;      // X(0, 0)
  int64_t s_idx, s_k;
  int nidx, K;
  bool kmajor;
  int i0, kk0, di, dk;   // element r of this thread: (i0 + r di, kk0 + r dk)
  __device__ void init(const T* X, int64_t si, int64_t sk, int ni, int KK, bool km) {
    base = X; s_idx = si; s_k = sk; nidx = ni; K = KK; kmajor = km;
    const int tid = threadIdx.x;
    if (km) { i0 = tid % MF_T; kk0 = tid / MF_T; di = 0; dk = 256 / MF_T; }
    else { kk0 = tid % MF_KC; i0 = tid / MF_KC; dk = 0; di = 256 / MF_KC; }
  }
  // global -> registers for the chunk starting at k0 (zero outside)
  __device__ void load(int k0, T (&reg)[MF_R]) const {
#pragma unroll
    for (int r = 0; r < MF_R; ++r) {
      const int i = i0 + r * di, k = k0 + kk0 + r * dk;
      reg[r] = (i < nidx && k < K) ? base[(int64_t)i * s_idx + (int64_t)k * s_k] : T(0);
    }
  }
  __device__ void store(const T (&reg)[MF_R], T* buf) const {
#pragma unroll
    for (int r = 0; r < MF_R; ++r) {
      const int i = i0 + r * di, k = kk0 + r * dk;
      buf[kmajor ? k * MF_PK + i : i * MF_PI + k] = reg[r];
    }
  }
};

// acc += op(A)(0:M, 0:K) op(B)(0:K, 0:N) for a tile with M, N <= 64; rows
// >= M and columns >= N read as zero.  The next chunk's global loads are in
// flight while the current one is multiplied.
template <class T>
__device__ __forceinline__ void mf_tile(int M, int N, int K, const T* __restrict__ A, int64_t sai,
                                        int64_t sak, const T* __restrict__ B, int64_t sbk,
                                        int64_t sbj, MfAcc<T>& acc, T* smem) {
  typedef MfTraits<T> Tr;
  T* sA = smem;
  T* sB = smem + mf_smem_elems<T>() / 2;
  const bool akm = sai == 1;   // A stored K-major (unit stride along rows)
  const bool bkm = sbj == 1;   // B stored K-major (unit stride along columns)
  MfStager<T> ga, gb;
  ga.init(A, sai, sak, M, K, akm);
  gb.init(B, sbj, sbk, N, K, bkm);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ia = 16 * w + li;
  T ra[MF_R], rb[MF_R];
  if (K > 0) {
    ga.load(0, ra);
    gb.load(0, rb);
  }
  for (int k0 = 0; k0 < K; k0 += MF_KC) {
    ga.store(ra, sA);
    gb.store(rb, sB);
    __syncthreads();
    if (k0 + MF_KC < K) {
      ga.load(k0 + MF_KC, ra);
      gb.load(k0 + MF_KC, rb);
    }
#pragma unroll
    for (int s = 0; s < MF_KC / 4; ++s) {
      const int k = 4 * s + lk;
      const T a = akm ? sA[k * MF_PK + ia] : sA[ia * MF_PI + k];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int jb = 16 * t + li;
        const T b = bkm ? sB[k * MF_PK + jb] : sB[jb * MF_PI + k];
        acc.v[t] = Tr::step(a, b, acc.v[t]);
      }
    }
    __syncthreads();
  }
}

// C(0:M, 0:N) = alpha acc + beta C; beta == 0 never reads C.
template <class T>
__device__ __forceinline__ void mf_store(int M, int N, T* C, int64_t ldc, const MfAcc<T>& acc,
                                         T alpha, T beta) {
  typedef MfTraits<T> Tr;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * w + Tr::row(lane, v), j = 16 * t + (lane & 15);
      if (i < M && j < N) {
        T* c = C + i + (int64_t)j * ldc;
        *c = beta == T(0) ? alpha * acc.v[t][v] : alpha * acc.v[t][v] + beta * *c;
      }
    }
}

// As mf_store, through LDS: the accumulators go to a 64 x 64 tile in smem
// (at least mf_smem_elems<T>() elements; callers pass the smem of their
// mf_tile, which ends with a barrier), then each column is written by
// consecutive threads (contiguous, coalesced), instead of each lane's 16
// scattered elements.  All threads of the block must call it.
template <class T>
__device__ __forceinline__ void mf_store_lds(int M, int N, T* C, int64_t ldc, const MfAcc<T>& acc,
                                             T alpha, T beta, T* smem) {
  typedef MfTraits<T> Tr;
  constexpr int LD = MF_T + 1;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * w + Tr::row(lane, v), j = 16 * t + (lane & 15);
      smem[i + j * LD] = acc.v[t][v];
    }
  __syncthreads();
  for (int e = threadIdx.x; e < MF_T * MF_T; e += 256) {
    const int i = e % MF_T, j = e / MF_T;
    if (i < M && j < N) {
      T* c = C + i + (int64_t)j * ldc;
      const T a = smem[i + j * LD];
      *c = beta == T(0) ? alpha * a : alpha * a + beta * *c;
    }
  }
  __syncthreads();
}

}  // namespace hm
