// LDS-tiled block-level matrix product used by the small, structure-aware
// kernels (apply sweeps, transfers, interaction matrices).  256 threads form
// a 16 x 16 grid; thread (tx, ty) owns rows tx + 16u and columns ty + 16v of
// a TM x TN output tile.  Operands are addressed by strides, so transposes
// cost nothing:  op(A)(i,k) = A[i*sai + k*sak],  op(B)(k,j) = B[k*sbk + j*sbj].
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hm {

constexpr int TILE_BK = 16;

template <class T, int TM, int TN>
struct TileAcc {
  T v[TM / 16][TN / 16];
  __device__ void zero() {
#pragma unroll
    for (int u = 0; u < TM / 16; ++u)
#pragma unroll
      for (int w = 0; w < TN / 16; ++w) v[u][w] = T(0);
  }
};

// Shared-memory footprint (elements of T) of one mm_tile call.
template <int TM, int TN>
constexpr int tile_smem_elems() {
  return TILE_BK * (TM + 1) + TILE_BK * (TN + 1);
}

// acc += op(A)(i0 : i0+TM, 0:K) * op(B)(0:K, j0 : j0+TN), rows >= M and
// columns >= N read as zero.  A and B already point at row i0 / column j0.
template <class T, int TM, int TN>
__device__ __forceinline__ void mm_tile(int M, int N, int K, const T* __restrict__ A,
                                        int64_t sai, int64_t sak, const T* __restrict__ B,
                                        int64_t sbk, int64_t sbj, TileAcc<T, TM, TN>& acc,
                                        T* smem) {
  T* sA = smem;                       // [BK][TM+1]
  T* sB = smem + TILE_BK * (TM + 1);  // [BK][TN+1]
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  for (int k0 = 0; k0 < K; k0 += TILE_BK) {
    // stage op(A) tile, coalesced along whichever index has unit stride
    for (int idx = tid; idx < TM * TILE_BK; idx += 256) {
      int i, k;
      if (sai == 1) { i = idx % TM; k = idx / TM; } else { k = idx % TILE_BK; i = idx / TILE_BK; }
      T v = T(0);
      if (i < M && k0 + k < K) v = A[(int64_t)i * sai + (int64_t)(k0 + k) * sak];
      sA[k * (TM + 1) + i] = v;
    }
    for (int idx = tid; idx < TN * TILE_BK; idx += 256) {
      int j, k;
      if (sbk == 1) { k = idx % TILE_BK; j = idx / TILE_BK; } else { j = idx % TN; k = idx / TN; }
      T v = T(0);
      if (j < N && k0 + k < K) v = B[(int64_t)(k0 + k) * sbk + (int64_t)j * sbj];
      sB[k * (TN + 1) + j] = v;
    }
    __syncthreads();
    const int kk = min(TILE_BK, K - k0);
    for (int k = 0; k < kk; ++k) {
      T a[TM / 16], b[TN / 16];
#pragma unroll
      for (int u = 0; u < TM / 16; ++u) a[u] = sA[k * (TM + 1) + tx + 16 * u];
#pragma unroll
      for (int w = 0; w < TN / 16; ++w) b[w] = sB[k * (TN + 1) + ty + 16 * w];
#pragma unroll
      for (int u = 0; u < TM / 16; ++u)
#pragma unroll
        for (int w = 0; w < TN / 16; ++w) acc.v[u][w] = fma(a[u], b[w], acc.v[u][w]);
    }
    __syncthreads();
  }
}

// C(i0.., j0..) = alpha * acc + beta * C for the valid part of the tile.
// beta == 0 never reads C.
template <class T, int TM, int TN>
__device__ __forceinline__ void store_tile(int M, int N, T* C, int64_t ldc,
                                           const TileAcc<T, TM, TN>& acc, T alpha, T beta) {
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int u = 0; u < TM / 16; ++u)
#pragma unroll
    for (int w = 0; w < TN / 16; ++w) {
      const int i = tx + 16 * u, j = ty + 16 * w;
      if (i < M && j < N) {
        T* c = C + i + (int64_t)j * ldc;
        *c = beta == T(0) ? alpha * acc.v[u][w] : alpha * acc.v[u][w] + beta * *c;
      }
    }
}

}  // namespace hm
