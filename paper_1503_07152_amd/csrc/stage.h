// LDS staging helpers of the apply and gradient kernels: a high-multiply
// division for index maps and a batched global -> LDS copy with 16-byte loads.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hm {

// e / d for 0 <= e < 2^32 / d (d <= 2^16): one high multiply.
struct FastDiv {
  uint32_t m;
  __device__ explicit FastDiv(uint32_t d) : m(0xFFFFFFFFu / d + 1u) {}
  __device__ __forceinline__ int div(int e) const { return (int)__umulhi((uint32_t)e, m); }
};

template <class T, int V>
struct alignas(sizeof(T) * V) BandVec {
  T v[V];
};

// Chunks e in [0, n) of V consecutive source elements: map(e, p, d0, ds) gives
// the source address and the LDS offsets d0, d0 + ds, ... of the chunk's
// elements.  NB chunks per thread (NTH threads) are loaded before any is stored.
template <class T, int V, int NB, int NTH = 256, class Map>
__device__ __forceinline__ void band_stage(int n, T* lds, Map map) {
  for (int base = 0; base < n; base += NTH * NB) {
    BandVec<T, V> v[NB];
    int d0[NB], ds[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = base + q * NTH + (int)threadIdx.x;
      d0[q] = -1;
      ds[q] = 0;
      if (e < n) {
        const T* p;
        map(e, p, d0[q], ds[q]);
        v[q] = *reinterpret_cast<const BandVec<T, V>*>(p);
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q)
      if (d0[q] >= 0)
#pragma unroll
        for (int t = 0; t < V; ++t) lds[d0[q] + t * ds[q]] = v[q].v[t];
  }
}

}  // namespace hm
