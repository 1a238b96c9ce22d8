// Forest apply of A^(m) (Fig. 7) and the segmented transposed products.
#include <algorithm>

#include "apply.h"
#include "stage.h"
#include "tile_mfma.h"

namespace hm {

void build_apply_lists(const Forest& f, const std::vector<int>& m, ApplyLists& out,
                       hipStream_t s) {
  std::vector<int32_t> front;
  int mmax = 0;
  for (int i = 0; i < (int)f.inst.size(); ++i) mmax = std::max(mmax, m[i]);
  int64_t maxr = 0;
  for (int g = 0; g < (int)f.nodes.size(); ++g) {
    const Node& nd = f.nodes[g];
    const int mi = m[nd.inst];
    if (mi >= 0 && nd.level == mi) {
      front.push_back(g);
      maxr = std::max<int64_t>(maxr, nd.hi - nd.lo);
    }
  }
  out.nfront = (int)front.size();
  out.frontier = upload(front, s);
  out.max_rows = maxr;
  out.chunks = (int)std::max<int64_t>(1, (maxr + APPLY_CHUNK - 1) / APPLY_CHUNK);
  out.mmax = mmax;
  // Bands.  Up: levels [lo, hi] from the deepest internal level M = mmax - 1
  // upwards, one job per internal node on level lo, down to min(hi, m_i - 1)
  // (its children below are inputs).  Down: jobs rooted on levels 0, D, 2D ...
  // (instance roots or internal nodes), each computing the incoming
  // expansions of its descendants down to D levels below (at most to m_i).
  std::vector<BandJob> jobs;
  auto job = [&](int g, int d, int info) {
    BandJob jb;
    jb.info = info;
    for (int32_t& x : jb.ids) x = -1;
    jb.ids[0] = g;
    for (int b = 0; b < (1 << d) - 1; ++b) {
      const Node& nd = f.nodes[jb.ids[b]];
      jb.ids[2 * b + 1] = nd.left;
      jb.ids[2 * b + 2] = nd.right;
    }
    jobs.push_back(jb);
  };
  const int M = mmax - 1;
  for (int D = 1; D <= BAND_DMAX; ++D) {
    out.up_band[D].clear();
    out.down_band[D].clear();
    for (int hi = M; hi >= 1; hi -= D) {
      const int lo = std::max(1, hi - D + 1);
      BandRange br{(int)jobs.size(), 0, 0};
      for (int g : f.level[lo]) {
        const int mi = m[f.nodes[g].inst];
        if (mi < 0 || lo >= mi) continue;
        const int d = std::min(hi, mi - 1) - lo + 1;
        job(g, d, d);
        br.depth = std::max(br.depth, d);
      }
      br.n = (int)jobs.size() - br.off;
      if (br.n > 0) out.up_band[D].push_back(br);
    }
    for (int lo = 0; lo <= M; lo += D) {
      BandRange br{(int)jobs.size(), 0, 0};
      for (int g : f.level[lo]) {
        const int mi = m[f.nodes[g].inst];
        if (mi < 1 || lo >= mi) continue;
        const int d = std::min(D, mi - lo);
        job(g, d, d | (lo >= 1 ? 1 << 8 : 0));
        br.depth = std::max(br.depth, d);
      }
      br.n = (int)jobs.size() - br.off;
      if (br.n > 0) out.down_band[D].push_back(br);
    }
  }
  out.bands = upload(jobs, s);
}

constexpr int TM = MF_T, TN = MF_T;   // output tile of the MFMA products

template <class T>
__global__ __launch_bounds__(256) void k_leaf_up(const Node* nodes, const int32_t* front,
                                                 int chunks, const T* V, int64_t ldl, int R,
                                                 const T* X, int64_t ldx, int c, T* QH, T* P) {
  __shared__ T smem[mf_smem_elems<T>()];
  const int ch = blockIdx.x, fi = blockIdx.y, j0 = blockIdx.z * TN;
  const int g = front[fi];
  const Node nd = nodes[g];
  const int64_t r0 = nd.lo + (int64_t)ch * APPLY_CHUNK;
  const int K = (int)max<int64_t>(0, min<int64_t>(APPLY_CHUNK, nd.hi - r0));
  MfAcc<T> acc;
  acc.zero();
  if (nd.level > 0 && K > 0)
    mf_tile<T>(R, c - j0, K, V + r0, ldl, 1, X + r0 + (int64_t)j0 * ldx, 1, ldx, acc,
                       smem);
  T* out = chunks == 1 ? QH + (int64_t)g * R * c : P + ((int64_t)fi * chunks + ch) * R * c;
  mf_store<T>(R, c - j0, out + (int64_t)j0 * R, R, acc, T(1), T(0));
}

template <class T>
__global__ void k_chunk_reduce(const int32_t* front, int chunks, const T* P, int64_t n, T* QH,
                               T alpha, T beta, int64_t out_stride) {
  const int fi = blockIdx.y;
  const int g = front[fi];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    T s = T(0);
    for (int ch = 0; ch < chunks; ++ch) s += P[((int64_t)fi * chunks + ch) * n + e];
    T* o = QH + (int64_t)g * out_stride + e;
    *o = beta == T(0) ? alpha * s : alpha * s + beta * *o;
  }
}

// ---- tree sweeps: band kernels ---------------------------------------------
// Several tree levels per launch.  A workgroup takes one subtree (BandJob) and
// a tile of BC columns, stages every operand it needs in LDS in one round
// (coefficient blocks as A(i, k) at k * RP + i, expansions as (k, j) at
// k * VP + j, rows padded with zeros to R4 = a multiple of 4), then runs the
// node products level by level out of LDS on the matrix cores (16 x 16 output
// tiles, MFMA 16x16x4; the tiles of one level's products spread over the
// four waves), writing each result to global memory (for the other sweep and
// the leaves) and, when a product above needs it, to LDS.
// Up: qh_t = Vt_t^T [qh_a; qh_b].  Down: for child a of t with sibling s,
// uh_a = Ut_t(half of a) uh_t + B[s] qh_s (forward) or B[a]^T qh_s (adjoint);
// the children of a root take only the second term.
constexpr int TRM = HM_MAX_SAMPLES;   // largest padded rank

template <class T> struct BandCfg;
template <> struct BandCfg<float> { static constexpr int BC = 32; };
template <> struct BandCfg<double> { static constexpr int BC = 16; };

// LDS elements of an up band / a down band of depth d (rows R4 per block).
constexpr int band_up_elems(int R4, int BC, int d) {
  return ((2 << d) - 1) * R4 * (BC + 1) + ((1 << d) - 1) * 2 * R4 * (R4 + 1);
}
constexpr int band_down_elems(int R4, int BC, int d) {
  return 2 * ((2 << d) - 1) * R4 * (BC + 1) + ((2 << d) - 2) * 2 * R4 * (R4 + 1);
}
constexpr int BAND_LDS_MAX = 158 * 1024;   // of the 160 KiB per workgroup
constexpr int BAND_SLACK = 64;             // tile rows read past the last block
template <class T>
constexpr int band_depth_up(int RC) {
  int d = BAND_DMAX;
  while (d > 1 &&
         (band_up_elems(RC, BandCfg<T>::BC, d) + BAND_SLACK) * (int)sizeof(T) > BAND_LDS_MAX)
    --d;
  return d;
}
template <class T>
constexpr int band_depth_down(int RC) {
  int d = BAND_DMAX;
  while (d > 1 &&
         (band_down_elems(RC, BandCfg<T>::BC, d) + BAND_SLACK) * (int)sizeof(T) > BAND_LDS_MAX)
    --d;
  return d;
}

// acc += A(r0 + 0..15, 0:4 nk4) B(0:4 nk4, c0 + 0..15) on the matrix cores:
// a = &A(r0, 0) with A(i, k) at k * RP + i; b = &B(0, c0) with B(k, j) at
// k * VP + j.
template <class T>
__device__ __forceinline__ void band_tile(int nk4, int RP, int VP, const T* a, const T* b,
                                          typename MfTraits<T>::acc_t& acc) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  a += lk * RP + li;
  b += lk * VP + li;
  int s = 0;
  for (; s + 4 <= nk4; s += 4) {
    T av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = a[u * 4 * RP];
      bv[u] = b[u * 4 * VP];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = MfTraits<T>::step(av[u], bv[u], acc);
    a += 16 * RP;
    b += 16 * VP;
  }
  for (; s < nk4; ++s) {
    acc = MfTraits<T>::step(a[0], b[0], acc);
    a += 4 * RP;
    b += 4 * VP;
  }
}

// Tile (rt, ct) of a product: rows rt*16 + ..., columns ct*16 + ... of the
// node's R x nc block (global, ld R) and, if lds_blk, of its LDS block.
template <class T>
__device__ __forceinline__ void band_put(const typename MfTraits<T>::acc_t& acc, int rt, int ct,
                                         int R, int nc, T* out, T* lds_blk, int VP) {
  const int lane = threadIdx.x & 63;
  const int j = ct * 16 + (lane & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = rt * 16 + MfTraits<T>::row(lane, v);
    if (i < R && j < nc) {
      out[i + (int64_t)j * R] = acc[v];
      if (lds_blk) lds_blk[i * VP + j] = acc[v];
    }
  }
}

// Zero rows R .. R4-1 of nblk blocks of `rows` rows (pitch P) at lds, block
// stride bs; rows_off: first padded row of each half (up to two halves).
template <class T>
__device__ __forceinline__ void band_zero_pad(T* lds, int nblk, int bs, int P, int R, int R4,
                                              int halves) {
  const int pr = R4 - R;
  if (pr == 0) return;
  const int per = halves * pr * P;
  for (int e = threadIdx.x; e < nblk * per; e += 256) {
    const int q = e / per, r = e - q * per;
    const int h = r / (pr * P), r2 = r - h * pr * P;
    const int row = h * R4 + R + r2 / P, col = r2 % P;
    lds[q * bs + row * P + col] = T(0);
  }
}

template <class T, int RC, int V, int DM>
__global__ __launch_bounds__(256) void k_band_up(const BandJob* jobs, const T* Tout, int R,
                                                 T* QH, int c, const T* Tout2, T* QH2) {
  typedef MfTraits<T> Tr;
  if (blockIdx.z) {   // the second sweep of a pair (same tree, other operands)
    Tout = Tout2;
    QH = QH2;
  }
  constexpr int BC = BandCfg<T>::BC, CT = BC / 16;
  static_assert(DM >= 1 && DM <= band_depth_up<T>(RC), "band depth beyond the LDS");
  __shared__ T lds[band_up_elems(RC, BC, DM) + BAND_SLACK];
  __shared__ int sids[16];
  const int tid = threadIdx.x, wave = tid >> 6;
  if (tid < 16) sids[tid] = tid == 0 ? jobs[blockIdx.x].info : jobs[blockIdx.x].ids[tid - 1];
  __syncthreads();
  const int d = sids[0] & 0xff;
  const int* ids = sids + 1;
  const int j0 = blockIdx.y * BC, nc = min(BC, c - j0);
  const int R4 = (R + 3) & ~3, VP = BC + 1, RP = R4 + 1;
  const int nprod = (1 << d) - 1, nnode = (2 << d) - 1;
  T* vals = lds;                         // node b: R4 x VP at b * R4 * VP
  T* cf = lds + nnode * R4 * VP;         // product p: 2 R4 x RP at p * 2 R4 * RP
  band_zero_pad(vals, nnode, R4 * VP, VP, R, R4, 1);
  band_zero_pad(cf, nprod, 2 * R4 * RP, RP, R, R4, 2);
  {
    // the qh blocks of the children below the band (R x nc, contiguous), then
    // the transfer blocks Tout_t (2R x R, ld 2R) as A(i, k) = Tout_t(k, i)
    const int cin = R * nc / V, ccf = 2 * R * R / V;
    const int n1 = (nnode - nprod) * cin;
    const FastDiv din(cin), dcf(ccf), dr(R), d2r(2 * R);
    band_stage<T, V, 24>(n1 + nprod * ccf, lds, [&](int e, const T*& p, int& d0, int& ds) {
      if (e < n1) {
        const int q = din.div(e), rem = (e - q * cin) * V;
        const int jj = dr.div(rem), i = rem - jj * R;
        p = QH + (int64_t)ids[nprod + q] * R * c + (int64_t)j0 * R + rem;
        d0 = (nprod + q) * R4 * VP + i * VP + jj;
        ds = VP;
      } else {
        const int e2 = e - n1, q = dcf.div(e2), rem = (e2 - q * ccf) * V;
        const int i = d2r.div(rem), k = rem - i * 2 * R;
        const int kk = k < R ? k : k - R + R4;
        p = Tout + (int64_t)ids[q] * 2 * R * R + rem;
        d0 = nnode * R4 * VP + q * 2 * R4 * RP + kk * RP + i;
        ds = RP;
      }
    });
  }
  __syncthreads();
  const int NT = (R + 15) / 16, tiles = NT * CT;
  for (int j = d - 1; j >= 0; --j) {
    const int p0 = (1 << j) - 1, ntile = (1 << j) * tiles;
    for (int q = wave; q < ntile; q += 4) {
      const int p = p0 + q / tiles, r = q % tiles, rt = r / CT, ct = r % CT;
      typename Tr::acc_t acc = {0, 0, 0, 0};
      band_tile<T>(2 * R4 / 4, RP, VP, cf + p * 2 * R4 * RP + rt * 16,
                   vals + (2 * p + 1) * R4 * VP + ct * 16, acc);
      band_put<T>(acc, rt, ct, R, nc, QH + (int64_t)ids[p] * R * c + (int64_t)j0 * R,
                  j > 0 ? vals + p * R4 * VP : nullptr, VP);
    }
    __syncthreads();
  }
}

template <class T, int RC, int V, int DM>
__global__ __launch_bounds__(256) void k_band_down(const BandJob* jobs, const T* Tin,
                                                   const T* B, int R, const T* QH, T* UH, int c,
                                                   int adjoint, const T* Tin2, const T* QH2,
                                                   T* UH2, int adjoint2) {
  typedef MfTraits<T> Tr;
  if (blockIdx.z) {   // the second sweep of a pair
    Tin = Tin2;
    QH = QH2;
    UH = UH2;
    adjoint = adjoint2;
  }
  constexpr int BC = BandCfg<T>::BC, CT = BC / 16;
  static_assert(DM >= 1 && DM <= band_depth_down<T>(RC), "band depth beyond the LDS");
  __shared__ T lds[band_down_elems(RC, BC, DM) + BAND_SLACK];
  __shared__ int sids[16];
  const int tid = threadIdx.x, wave = tid >> 6;
  if (tid < 16) sids[tid] = tid == 0 ? jobs[blockIdx.x].info : jobs[blockIdx.x].ids[tid - 1];
  __syncthreads();
  const int d = sids[0] & 0xff;
  const bool has_parent = (sids[0] >> 8) & 1;
  const int* ids = sids + 1;
  const int j0 = blockIdx.y * BC, nc = min(BC, c - j0);
  const int R4 = (R + 3) & ~3, VP = BC + 1, RP = R4 + 1;
  const int nnode = (2 << d) - 1;
  T* uhv = lds;                          // node b: R4 x VP
  T* qhv = lds + nnode * R4 * VP;        // node b: R4 x VP
  T* cf = lds + 2 * nnode * R4 * VP;     // node b >= 1: 2 R4 x RP at (b - 1) * 2 R4 * RP
  band_zero_pad(uhv, 2 * nnode, R4 * VP, VP, R, R4, 1);
  band_zero_pad(cf, nnode - 1, 2 * R4 * RP, RP, R, R4, 2);
  {
    // uh of the root (if it has a parent), qh of every node below it (each is
    // a sibling), per node b >= 1 the parent's transfer half (A rows 0..R-1)
    // and the sibling coupling (A rows R4 ..)
    const int cin = R * nc / V, crr = R * R / V;
    const int n0 = has_parent ? cin : 0;
    const int n1 = n0 + (nnode - 1) * cin, n2 = n1 + (nnode - 1) * crr;
    const int n3 = n2 + (nnode - 1) * crr;
    const FastDiv din(cin), drr(crr), dr(R);
    const int cfo = 2 * nnode * R4 * VP;
    band_stage<T, V, 24>(n3, lds, [&](int e, const T*& p, int& d0, int& ds) {
      if (e < n1) {
        const int e1 = e < n0 ? e : e - n0;
        const int q = e < n0 ? 0 : din.div(e1), rem = (e1 - q * cin) * V;
        const int jj = dr.div(rem), i = rem - jj * R;
        const int b = e < n0 ? 0 : 1 + q;
        p = (e < n0 ? (const T*)UH : QH) + (int64_t)ids[b] * R * c + (int64_t)j0 * R + rem;
        d0 = (e < n0 ? 0 : nnode * R4 * VP + b * R4 * VP) + i * VP + jj;
        ds = VP;
      } else if (e < n2) {
        const int e2 = e - n1, q = drr.div(e2), rem = (e2 - q * crr) * V;
        const int k = dr.div(rem), i = rem - k * R;
        const int b = 1 + q, side = (b & 1) ? 0 : 1;
        p = Tin + (int64_t)ids[(b - 1) >> 1] * 2 * R * R + side * R + i + (int64_t)k * 2 * R;
        d0 = cfo + q * 2 * R4 * RP + k * RP + i;
        ds = 1;
      } else {
        const int e3 = e - n2, q = drr.div(e3), rem = (e3 - q * crr) * V;
        const int hi = dr.div(rem), lo = rem - hi * R;
        const int b = 1 + q, sib = (b & 1) ? b + 1 : b - 1;
        // forward A(i, k) = B[sib](i, k) = B[sib][i + k R]; adjoint A(i, k) = B[b][k + i R]
        p = B + (int64_t)ids[adjoint ? b : sib] * R * R + rem;
        d0 = cfo + q * 2 * R4 * RP + (adjoint ? (R4 + lo) * RP + hi : (R4 + hi) * RP + lo);
        ds = adjoint ? RP : 1;
      }
    });
  }
  __syncthreads();
  const int NT = (R + 15) / 16, tiles = NT * CT;
  for (int j = 1; j <= d; ++j) {
    const bool up_term = j >= 2 || has_parent;
    const int b0 = (1 << j) - 1, ntile = (1 << j) * tiles;
    for (int q = wave; q < ntile; q += 4) {
      const int b = b0 + q / tiles, r = q % tiles, rt = r / CT, ct = r % CT;
      const int par = (b - 1) >> 1, sib = (b & 1) ? b + 1 : b - 1;
      const T* cb = cf + (b - 1) * 2 * R4 * RP + rt * 16;
      typename Tr::acc_t acc = {0, 0, 0, 0};
      if (up_term) band_tile<T>(R4 / 4, RP, VP, cb, uhv + par * R4 * VP + ct * 16, acc);
      band_tile<T>(R4 / 4, RP, VP, cb + R4 * RP, qhv + sib * R4 * VP + ct * 16, acc);
      band_put<T>(acc, rt, ct, R, nc, UH + (int64_t)ids[b] * R * c + (int64_t)j0 * R,
                  j < d ? uhv + b * R4 * VP : nullptr, VP);
    }
    __syncthreads();
  }
}

// The sweeps of one apply, or of two applies on the same tree side by side
// (pair: the second as blockIdx.z = 1 of the same launches).
template <class T>
struct BandSweep {
  bool adjoint;
  T* QH;
  T* UH;
};

template <class T, int RC, int V>
void run_bands(const ApplyLists& al, const HbsView<T>& h, int c, const BandSweep<T>& a,
               const BandSweep<T>* b, hipStream_t s) {
  constexpr int BC = BandCfg<T>::BC;
  constexpr int DU = band_depth_up<T>(RC), DD = band_depth_down<T>(RC);
  const int ctt = (c + BC - 1) / BC;
  const BandJob* jobs = al.bands.as<BandJob>();
  auto tin = [&](const BandSweep<T>& w) { return w.adjoint ? h.Vt : h.Ut; };
  auto tout = [&](const BandSweep<T>& w) { return w.adjoint ? h.Ut : h.Vt; };
  const BandSweep<T>& b2 = b ? *b : a;
  const unsigned nz = b ? 2 : 1;
  // each launch sized to its band's depth (a shallow band, such as the last
  // downward one, takes less LDS and runs more workgroups per CU)
  auto up = [&](auto kern, const BandRange& r) {
    hipLaunchKernelGGL(kern, dim3(r.n, ctt, nz), dim3(256), 0, s, jobs + r.off, tout(a), h.R,
                       a.QH, c, tout(b2), b2.QH);
    KCHK();
  };
  auto down = [&](auto kern, const BandRange& r) {
    hipLaunchKernelGGL(kern, dim3(r.n, ctt, nz), dim3(256), 0, s, jobs + r.off, tin(a), h.B, h.R,
                       (const T*)a.QH, a.UH, c, a.adjoint ? 1 : 0, tin(b2), (const T*)b2.QH,
                       b2.UH, b2.adjoint ? 1 : 0);
    KCHK();
  };
  for (const BandRange& r : al.up_band[DU]) {
    if (r.depth <= 1) up(k_band_up<T, RC, V, 1>, r);
    else if (r.depth == 2 || DU == 2) up(k_band_up<T, RC, V, DU >= 2 ? 2 : 1>, r);
    else up(k_band_up<T, RC, V, DU>, r);
  }
  for (const BandRange& r : al.down_band[DD]) {
    if (r.depth <= 1) down(k_band_down<T, RC, V, 1>, r);
    else if (r.depth == 2 || DD == 2) down(k_band_down<T, RC, V, DD >= 2 ? 2 : 1>, r);
    else down(k_band_down<T, RC, V, DD>, r);
  }
}

// Vector staging (16-byte loads) needs R a multiple of the vector width and
// 16-byte aligned operand arrays.
template <class T>
void run_bands_any(const ApplyLists& al, const HbsView<T>& h, int c, const BandSweep<T>& a,
                   const BandSweep<T>* b, hipStream_t s) {
  constexpr int V = 16 / sizeof(T);
  auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  bool vec = h.R % V == 0 && al16(a.QH) && al16(a.UH) && al16(h.Ut) && al16(h.Vt) && al16(h.B);
  if (b) vec = vec && al16(b->QH) && al16(b->UH);
  if (h.R <= 32) {
    if (vec) run_bands<T, 32, V>(al, h, c, a, b, s);
    else run_bands<T, 32, 1>(al, h, c, a, b, s);
  } else {
    if (vec) run_bands<T, TRM, V>(al, h, c, a, b, s);
    else run_bands<T, TRM, 1>(al, h, c, a, b, s);
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_leaf_down(const Node* nodes, const int32_t* front,
                                                   const T* U, int64_t ldl, int R, const T* UH,
                                                   int c, const T* D, int64_t ldd, int adjoint,
                                                   const T* X, int64_t ldx, T* Y, int64_t ldy,
                                                   T alpha, T beta) {
  __shared__ T smem[mf_smem_elems<T>()];
  const int g = front[blockIdx.y];
  const Node nd = nodes[g];
  const int64_t i0 = nd.lo + (int64_t)blockIdx.x * TM;
  if (i0 >= nd.hi) return;
  const int M = (int)min<int64_t>(TM, nd.hi - i0);
  const int j0 = blockIdx.z * TN;
  const int N = c - j0;
  MfAcc<T> acc;
  acc.zero();
  if (nd.level > 0)
    mf_tile<T>(M, N, R, U + i0, 1, ldl, UH + (int64_t)g * R * c + (int64_t)j0 * R, 1, R,
                       acc, smem);
  if (D) {
    const int nt = (int)(nd.hi - nd.lo);
    const T* xb = X + nd.lo + (int64_t)j0 * ldx;
    if (!adjoint)
      mf_tile<T>(M, N, nt, D + i0, 1, ldd, xb, 1, ldx, acc, smem);
    else
      mf_tile<T>(M, N, nt, D + nd.lo + (i0 - nd.lo) * ldd, ldd, 1, xb, 1, ldx, acc, smem);
  }
  mf_store_lds<T>(M, N, Y + i0 + (int64_t)j0 * ldy, ldy, acc, alpha, beta, smem);
}

// ---- forward leaf product, one workgroup per (frontier node, column tile) ---
// For frontier nodes of at most LEAF_MAX rows: the B operand of the whole
// product (UH_g stacked over X(I_g, :)) is staged in LDS in one round with
// 16-byte loads where aligned; wave w of eight takes rows 16 w .. 16 w + 15 of
// the node and every column of the tile, reading its A operand (U and D rows,
// 16 consecutive rows per lane group) straight from global memory with the
// next 64 K-values in flight while the current ones feed the MFMAs; the result
// goes through LDS so that the stores run along the rows.
constexpr int LEAF_MAX = 128;
template <class T> struct LeafCfg;
template <> struct LeafCfg<float> { static constexpr int BN = 64, BP = 80; };
template <> struct LeafCfg<double> { static constexpr int BN = 32, BP = 40; };
constexpr int LEAF_KMAX = ((HM_MAX_SAMPLES + LEAF_MAX + 31) / 32) * 32;
constexpr int LEAF_CP = LEAF_MAX + 4;   // pitch of the column-major result tile

// acc[t] += A(16 w + .., 0:K) B(0:K, 16 t + ..) for wave w of 8; A(i, k) from
// aload(i, k) (zero for i >= m or k >= K), B(k, j) = sB[k * BP + j] with rows
// up to K rounded to 32 zero-filled.  The A values of the next two groups of
// 32 K are in flight while a group feeds the MFMAs.
template <class T, int CT, int BP, class ALoad>
__device__ __forceinline__ void leaf_mma(int m, int K, const T* sB, ALoad aload,
                                         typename MfTraits<T>::acc_t (&acc)[CT]) {
  typedef MfTraits<T> Tr;
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int i = 16 * (threadIdx.x >> 6) + li;
  T a0[8], a1[8], a2[8];
  auto fetch = [&](int kg, T (&a)[8]) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = kg + 4 * s + lk;
      a[s] = (i < m && k < K) ? aload(i, k) : T(0);
    }
  };
  fetch(0, a0);
  fetch(32, a1);
  for (int kg = 0; kg < K; kg += 32) {
    fetch(kg + 64, a2);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const T* b = sB + (kg + 4 * s + lk) * BP + li;
      T bv[CT];
#pragma unroll
      for (int t = 0; t < CT; ++t) bv[t] = b[16 * t];
#pragma unroll
      for (int t = 0; t < CT; ++t) acc[t] = Tr::step(a0[s], bv[t], acc[t]);
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      a0[s] = a1[s];
      a1[s] = a2[s];
    }
  }
}

// Y(I_g, j0 + 0:nc) = alpha (U(I_g, :) UH_g + D_g X(I_g, :)) + beta Y (the U
// term for non-root nodes, the D term if D; D is not transposed here).
template <class T>
__global__ __launch_bounds__(512) void k_leaf_down2(const Node* nodes, const int32_t* front,
                                                    const T* U, int64_t ldl, int R, const T* UH,
                                                    int c, const T* D, int64_t ldd,
                                                    const T* X, int64_t ldx, T* Y, int64_t ldy,
                                                    T alpha, T beta) {
  typedef MfTraits<T> Tr;
  constexpr int BN = LeafCfg<T>::BN, BP = LeafCfg<T>::BP, CT = BN / 16;
  constexpr int V = 16 / sizeof(T);
  constexpr int LDS_ELEMS = LEAF_KMAX * BP > BN * LEAF_CP ? LEAF_KMAX * BP : BN * LEAF_CP;
  __shared__ __attribute__((aligned(16))) T sB[LDS_ELEMS];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = front[blockIdx.x];
  const Node nd = nodes[g];
  const int64_t lo = nd.lo;
  const int nt = (int)(nd.hi - nd.lo);
  const int j0 = blockIdx.y * BN, nc = min(BN, c - j0);
  const int KU = (nd.level > 0 && R > 0) ? R : 0, KD = D ? nt : 0, K = KU + KD;
  const int KP = (K + 31) & ~31;
  // stage B: rows 0..KU-1 = UH_g(:, tile), rows KU..K-1 = X(I_g, tile), zero to KP
  for (int e = tid; e < (KP - K) * BP; e += 512) sB[K * BP + e] = T(0);
  const bool vec = ((uintptr_t)X & 15) == 0 && ((uintptr_t)UH & 15) == 0 && lo % V == 0 &&
                   ldx % V == 0 && nt % V == 0 && R % V == 0;
  if (vec) {
    const int cu = KU / V, cx = KD / V;   // chunks per column
    const int n1 = cu * nc, n2 = n1 + cx * nc;
    const FastDiv du(cu > 0 ? cu : 1), dx(cx > 0 ? cx : 1);
    band_stage<T, V, 8, 512>(n2, sB, [&](int e, const T*& p, int& d0, int& ds) {
      if (e < n1) {
        const int j = du.div(e), k = (e - j * cu) * V;
        p = UH + (int64_t)g * R * c + (int64_t)(j0 + j) * R + k;
        d0 = k * BP + j;
      } else {
        const int e2 = e - n1, j = dx.div(e2), k = (e2 - j * cx) * V;
        p = X + lo + k + (int64_t)(j0 + j) * ldx;
        d0 = (KU + k) * BP + j;
      }
      ds = BP;
    });
  } else {
    const int n1 = KU * nc, n2 = n1 + KD * nc;
    const FastDiv du(KU > 0 ? KU : 1), dx(KD > 0 ? KD : 1);
    band_stage<T, 1, 16, 512>(n2, sB, [&](int e, const T*& p, int& d0, int& ds) {
      if (e < n1) {
        const int j = du.div(e), k = e - j * KU;
        p = UH + (int64_t)g * R * c + (int64_t)(j0 + j) * R + k;
        d0 = k * BP + j;
      } else {
        const int e2 = e - n1, j = dx.div(e2), k = e2 - j * KD;
        p = X + lo + k + (int64_t)(j0 + j) * ldx;
        d0 = (KU + k) * BP + j;
      }
      ds = 0;
    });
  }
  __syncthreads();
  typename Tr::acc_t acc[CT];
#pragma unroll
  for (int t = 0; t < CT; ++t) acc[t] = typename Tr::acc_t{0, 0, 0, 0};
  if (16 * w < nt && K > 0) {
    const T* Ul = U + lo;
    const T* Dl = D + lo;
    leaf_mma<T, CT, BP>(nt, K, sB, [&](int i, int k) {
      return k < KU ? Ul[i + (int64_t)k * ldl] : Dl[i + (int64_t)(k - KU) * ldd];
    }, acc);
  }
  __syncthreads();
  // result tile, column-major in LDS, then stores along the rows
  T* sC = sB;
#pragma unroll
  for (int t = 0; t < CT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * w + Tr::row(lane, v), j = 16 * t + (lane & 15);
      sC[j * LEAF_CP + i] = acc[t][v];
    }
  __syncthreads();
  const int i = tid & 127;
  if (i < nt)
    for (int j = tid >> 7; j < nc; j += 4) {
      T* y = Y + lo + i + (int64_t)(j0 + j) * ldy;
      const T r = alpha * sC[j * LEAF_CP + i];
      *y = beta == T(0) ? r : r + beta * *y;
    }
}

template <class T>
size_t apply_work_bytes(const Forest& f, const ApplyLists& al, int R, int c) {
  const size_t per = (size_t)R * c * sizeof(T);
  size_t b = 2 * per * f.nodes.size();
  if (al.chunks > 1) b += per * (size_t)al.nfront * al.chunks;
  return b + 256;
}

// Outgoing expansions on the frontier: QH_v = V_v^T X(I_v) (chunk partials
// for frontier nodes of more than APPLY_CHUNK rows reduced into QH).
template <class T>
static void leaf_up_launch(const Node* d_nodes, const ApplyLists& al, const T* Vout,
                           int64_t ldl, int R, int c, const T* X, int64_t ldx, T* QH, T* P,
                           hipStream_t s) {
  const int ct = (c + TN - 1) / TN;
  const int* front = al.frontier.as<int32_t>();
  hipLaunchKernelGGL(k_leaf_up<T>, dim3(al.chunks, al.nfront, ct), dim3(256), 0, s, d_nodes,
                     front, al.chunks, Vout, ldl, R, X, ldx, c, QH, P);
  KCHK();
  if (al.chunks > 1) {
    const int64_t n = (int64_t)R * c;
    hipLaunchKernelGGL(k_chunk_reduce<T>, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 64),
                                               al.nfront),
                       dim3(256), 0, s, front, al.chunks, P, n, QH, T(1), T(0), n);
    KCHK();
  }
}

// Y(I_v) = beta Y + alpha (U_v UH_v + D_v X(I_v)) on the frontier (D_v^T with
// adjoint).
template <class T>
static void leaf_down_launch(const Node* d_nodes, const ApplyLists& al, const HbsView<T>& h,
                             bool adjoint, const T* Uin, int c, const T* UH, const T* X,
                             int64_t ldx, T* Y, int64_t ldy, T alpha, T beta, hipStream_t s) {
  const int* front = al.frontier.as<int32_t>();
  // the transposed D reads of the adjoint are uncoalesced from global memory:
  // that case stays on the K-chunked LDS tiles of k_leaf_down
  if (al.max_rows <= LEAF_MAX && !(adjoint && h.D)) {
    constexpr int BN = LeafCfg<T>::BN;
    hipLaunchKernelGGL(k_leaf_down2<T>, dim3(al.nfront, (c + BN - 1) / BN), dim3(512), 0, s,
                       d_nodes, front, Uin, h.ldl, h.R, UH, c, h.D, h.ldd, X, ldx, Y, ldy, alpha,
                       beta);
    KCHK();
    return;
  }
  const int ct = (c + TN - 1) / TN;
  const int rt = (int)((al.max_rows + TM - 1) / TM);
  hipLaunchKernelGGL(k_leaf_down<T>, dim3(rt, al.nfront, ct), dim3(256), 0, s, d_nodes, front,
                     Uin, h.ldl, h.R, UH, c, h.D, h.ldd, adjoint ? 1 : 0, X, ldx, Y, ldy, alpha,
                     beta);
  KCHK();
}

template <class T>
static void apply_checks(const ApplyLists& al, int R) {
  if (R > TRM) HM_THROW(HM_ERR_UNSUPPORTED, "apply: padded rank %d > %d", R, TRM);
  if (al.mmax >= 1 && al.bands.bytes == 0)
    HM_THROW(HM_ERR_ARG, "apply: band lists missing");
}

template <class T>
void apply_forest(const Node* d_nodes, const ApplyLists& al, const HbsView<T>& h, bool adjoint,
                  int c, const T* X, int64_t ldx, T* Y, int64_t ldy, T alpha, T beta, void* work,
                  size_t nnodes, hipStream_t s, bool expansions_only) {
  if (al.nfront == 0 || c <= 0) return;
  const int R = h.R;
  apply_checks<T>(al, R);
  T* QH = static_cast<T*>(work);
  T* UH = QH + (size_t)R * c * nnodes;
  T* P = UH + (size_t)R * c * nnodes;
  const T* Uin = adjoint ? h.Vlong : h.Ulong;  // incoming long basis
  const T* Vout = adjoint ? h.Ulong : h.Vlong; // outgoing long basis
  if (al.mmax >= 1 && R > 0) {
    leaf_up_launch<T>(d_nodes, al, Vout, h.ldl, R, c, X, ldx, QH, P, s);
    run_bands_any<T>(al, h, c, BandSweep<T>{adjoint, QH, UH}, nullptr, s);
  }
  if (expansions_only) return;
  leaf_down_launch<T>(d_nodes, al, h, adjoint, Uin, c, UH, X, ldx, Y, ldy, alpha, beta, s);
}

template <class T>
void apply_forest_pair(const Node* d_nodes, const ApplyLists& al, const HbsView<T>& h, int c,
                       const T* X, int64_t ldx, void* work_x, const T* G, int64_t ldg, T* Y,
                       int64_t ldy, void* work_g, size_t nnodes, hipStream_t s) {
  if (al.nfront == 0 || c <= 0) return;
  const int R = h.R;
  apply_checks<T>(al, R);
  const size_t blk = (size_t)R * c * nnodes;
  T* QX = static_cast<T*>(work_x);
  T* QG = static_cast<T*>(work_g);
  if (al.mmax >= 1 && R > 0) {
    leaf_up_launch<T>(d_nodes, al, h.Vlong, h.ldl, R, c, X, ldx, QX, QX + 2 * blk, s);
    leaf_up_launch<T>(d_nodes, al, h.Ulong, h.ldl, R, c, G, ldg, QG, QG + 2 * blk, s);
    const BandSweep<T> adj{true, QG, QG + blk};
    run_bands_any<T>(al, h, c, BandSweep<T>{false, QX, QX + blk}, &adj, s);
  }
  leaf_down_launch<T>(d_nodes, al, h, true, h.Vlong, c, QG + blk, G, ldg, Y, ldy, T(1), T(0), s);
}

// ------------------------------------------------------------ HODLR level --
template <class T>
__global__ void k_sib_diag(const Node* nodes, const int32_t* front, int R, const T* S,
                           const T* QH, T* UH, int c, int adjoint) {
  const int a = front[blockIdx.x];
  const int b = nodes[a].sib;
  // forward: uh_a = diag(s[b]) qh_b ; adjoint: uh_a = diag(s[a]) qh_b
  const T* sv = S + (int64_t)(adjoint ? a : b) * R;
  const T* q = QH + (int64_t)b * R * c;
  T* u = UH + (int64_t)a * R * c;
  for (int e = threadIdx.x; e < R * c; e += blockDim.x) u[e] = sv[e % R] * q[e];
}

template <class T>
void hodlr_level_apply(const Node* d_nodes, const ApplyLists& al, const T* U, const T* V,
                       int64_t ldl, int R, const T* S, bool adjoint, int c, const T* X,
                       int64_t ldx, T* Y, int64_t ldy, T alpha, T beta, void* work,
                       size_t nnodes, hipStream_t s) {
  if (al.nfront == 0 || c <= 0) return;
  T* QH = static_cast<T*>(work);
  T* UH = QH + (size_t)R * c * nnodes;
  T* P = UH + (size_t)R * c * nnodes;
  const int ct = (c + TN - 1) / TN;
  const int* front = al.frontier.as<int32_t>();
  const T* Vout = adjoint ? U : V;
  const T* Uin = adjoint ? V : U;
  hipLaunchKernelGGL(k_leaf_up<T>, dim3(al.chunks, al.nfront, ct), dim3(256), 0, s, d_nodes, front,
                     al.chunks, Vout, ldl, R, X, ldx, c, QH, P);
  KCHK();
  if (al.chunks > 1) {
    const int64_t n = (int64_t)R * c;
    hipLaunchKernelGGL(k_chunk_reduce<T>,
                       dim3((unsigned)std::min<int64_t>((n + 255) / 256, 64), al.nfront),
                       dim3(256), 0, s, front, al.chunks, P, n, QH, T(1), T(0), n);
    KCHK();
  }
  hipLaunchKernelGGL(k_sib_diag<T>, dim3(al.nfront), dim3(256), 0, s, d_nodes, front, R, S, QH, UH,
                     c, adjoint ? 1 : 0);
  KCHK();
  const int rt = (int)((al.max_rows + TM - 1) / TM);
  hipLaunchKernelGGL(k_leaf_down<T>, dim3(rt, al.nfront, ct), dim3(256), 0, s, d_nodes, front, Uin,
                     ldl, R, UH, c, (const T*)nullptr, (int64_t)0, 0, X, ldx, Y, ldy, alpha, beta);
  KCHK();
}

// ------------------------------------------------------------ seg_tn ------
template <class T>
__global__ __launch_bounds__(256) void k_seg_tn(const Node* nodes, const int32_t* list,
                                                int chunks, int rows, int cols, const T* A,
                                                int64_t lda, const T* B, int64_t ldb, T* P) {
  __shared__ T smem[mf_smem_elems<T>()];
  const int ch = blockIdx.x, li = blockIdx.y;
  const int i0 = (blockIdx.z % ((rows + TM - 1) / TM)) * TM;
  const int j0 = (blockIdx.z / ((rows + TM - 1) / TM)) * TN;
  const Node nd = nodes[list[li]];
  const int64_t r0 = nd.lo + (int64_t)ch * APPLY_CHUNK;
  const int K = (int)max<int64_t>(0, min<int64_t>(APPLY_CHUNK, nd.hi - r0));
  MfAcc<T> acc;
  acc.zero();
  if (K > 0)
    mf_tile<T>(rows - i0, cols - j0, K, A + r0 + (int64_t)i0 * lda, lda, 1,
                       B + r0 + (int64_t)j0 * ldb, 1, ldb, acc, smem);
  T* out = P + ((int64_t)li * chunks + ch) * rows * cols;
  mf_store<T>(rows - i0, cols - j0, out + i0 + (int64_t)j0 * rows, rows, acc, T(1),
                        T(0));
}

template <class T>
__global__ void k_seg_reduce(const Node* nodes, const int32_t* list, int chunks, int rows,
                             int cols, const T* P, T* out, int64_t out_stride, int64_t ldo,
                             T alpha, T beta, int to_parent) {
  const int li = blockIdx.y;
  int g = list[li];
  int64_t off = 0;
  if (to_parent) {
    off = nodes[g].is_left ? 0 : rows;
    g = nodes[g].parent;
  }
  const int64_t n = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    T s = T(0);
    for (int ch = 0; ch < chunks; ++ch) s += P[((int64_t)li * chunks + ch) * n + e];
    const int i = (int)(e % rows), j = (int)(e / rows);
    T* o = out + (int64_t)g * out_stride + off + i + (int64_t)j * ldo;
    *o = beta == T(0) ? alpha * s : alpha * s + beta * *o;
  }
}

// Gram partials of one APPLY_CHUNK-row chunk of one node: the chunk goes
// through LDS in SG_K-row slices, column-major with pitch SG_P (the MFMA
// operand reads, 16 columns x 4 rows per instruction, then touch every bank
// at most twice; the staging writes run down a column), the next slice in
// registers while the current one feeds the MFMAs.  The SG_NT (SG_NT + 1) / 2
// tiles on and above the diagonal go to the four waves round-robin.
constexpr int SG_K = 32, SG_P = SG_K + 4, SG_C = 96, SG_NT = SG_C / 16;
constexpr int SG_TW = (SG_NT * (SG_NT + 1) / 2 + 3) / 4;   // tiles per wave
__global__ __launch_bounds__(256) void k_seg_gram(const Node* nodes, const int32_t* list,
                                                  int chunks, int c, const double* A,
                                                  int64_t lda, double* P) {
  typedef MfTraits<double> Tr;
  __shared__ double sM[2][SG_C * SG_P];
  const int ch = blockIdx.x, li = blockIdx.y;
  const Node nd = nodes[list[li]];
  const int64_t r0 = nd.lo + (int64_t)ch * APPLY_CHUNK;
  const int K = (int)max<int64_t>(0, min<int64_t>(APPLY_CHUNK, nd.hi - r0));
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nt = (c + 15) / 16;
  Tr::acc_t acc[SG_TW];
#pragma unroll
  for (int q = 0; q < SG_TW; ++q) acc[q] = Tr::acc_t{0, 0, 0, 0};
  // staging: thread t moves row t % SG_K of columns t / SG_K + 8 u
  constexpr int SU = SG_C * SG_K / 256;
  const int sk = tid % SG_K, sc = tid / SG_K;
  double pre[SU];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int col = sc + 8 * u;
      pre[u] = (col < c && k0 + sk < K) ? A[r0 + k0 + sk + (int64_t)col * lda] : 0.0;
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int u = 0; u < SU; ++u) sM[b][(sc + 8 * u) * SG_P + sk] = pre[u];
  };
  const int ns = (K + SG_K - 1) / SG_K;
  if (ns > 0) {
    fetch(0);
    stash(0);
  }
  __syncthreads();
  const int li16 = lane & 15, lk = lane >> 4;
  for (int sl = 0; sl < ns; ++sl) {
    const int b = sl & 1;
    if (sl + 1 < ns) fetch((sl + 1) * SG_K);
    const double* m = sM[b];
    int t = 0;
#pragma unroll
    for (int ti = 0; ti < SG_NT; ++ti)
#pragma unroll
      for (int tj = ti; tj < SG_NT; ++tj, ++t) {
        if ((t & 3) != wave || tj >= nt) continue;
        const double* pa = m + (16 * ti + li16) * SG_P + lk;
        const double* pb = m + (16 * tj + li16) * SG_P + lk;
#pragma unroll
        for (int kk = 0; kk < SG_K / 4; ++kk)
          acc[t >> 2] = Tr::step(pa[4 * kk], pb[4 * kk], acc[t >> 2]);
      }
    if (sl + 1 < ns) stash(b ^ 1);
    __syncthreads();
  }
  double* out = P + ((int64_t)li * chunks + ch) * c * c;
  int t = 0;
#pragma unroll
  for (int ti = 0; ti < SG_NT; ++ti)
#pragma unroll
    for (int tj = ti; tj < SG_NT; ++tj, ++t) {
      if ((t & 3) != wave || tj >= nt) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * ti + Tr::row(lane, v), j = 16 * tj + li16;
        if (i < c && j < c) {
          out[i + (int64_t)j * c] = acc[t >> 2][v];
          out[j + (int64_t)i * c] = acc[t >> 2][v];
        }
      }
    }
}

void seg_gram(const Node* d_nodes, const int32_t* list, int nlist, int64_t max_rows, int c,
              const double* A, int64_t lda, double* out, int64_t out_stride, void* work,
              hipStream_t s) {
  if (nlist == 0 || c == 0) return;
  if (c > SG_C) HM_THROW(HM_ERR_ARG, "seg_gram: %d columns > %d", c, SG_C);
  const int chunks = (int)std::max<int64_t>(1, (max_rows + APPLY_CHUNK - 1) / APPLY_CHUNK);
  double* P = static_cast<double*>(work);
  hipLaunchKernelGGL(k_seg_gram, dim3(chunks, nlist), dim3(256), 0, s, d_nodes, list, chunks, c,
                     A, lda, P);
  KCHK();
  const int64_t n = (int64_t)c * c;
  hipLaunchKernelGGL(k_seg_reduce<double>,
                     dim3((unsigned)std::min<int64_t>((n + 255) / 256, 64), nlist), dim3(256), 0, s,
                     d_nodes, list, chunks, c, c, P, out, out_stride, (int64_t)c, 1.0, 0.0, 0);
  KCHK();
}

template <class T>
size_t seg_tn_work_bytes(int nlist, int64_t max_rows, int rows, int cols) {
  const int64_t chunks = std::max<int64_t>(1, (max_rows + APPLY_CHUNK - 1) / APPLY_CHUNK);
  return (size_t)nlist * chunks * rows * cols * sizeof(T) + 256;
}

template <class T>
void seg_tn(const Node* d_nodes, const int32_t* list, int nlist, int64_t max_rows, int rows,
            int cols, const T* A, int64_t lda, const T* B, int64_t ldb, T* out,
            int64_t out_stride, int64_t ldo, T alpha, T beta, void* work, hipStream_t s,
            int to_parent) {
  if (nlist == 0 || rows == 0 || cols == 0) return;
  const int chunks = (int)std::max<int64_t>(1, (max_rows + APPLY_CHUNK - 1) / APPLY_CHUNK);
  const int tiles = ((rows + TM - 1) / TM) * ((cols + TN - 1) / TN);
  T* P = static_cast<T*>(work);
  hipLaunchKernelGGL(k_seg_tn<T>, dim3(chunks, nlist, tiles), dim3(256), 0, s, d_nodes, list,
                     chunks, rows, cols, A, lda, B, ldb, P);
  KCHK();
  const int64_t n = (int64_t)rows * cols;
  hipLaunchKernelGGL(k_seg_reduce<T>, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 64), nlist),
                     dim3(256), 0, s, d_nodes, list, chunks, rows, cols, P, out, out_stride, ldo,
                     alpha, beta, to_parent);
  KCHK();
}

#define INST(T)                                                                                \
  template void hodlr_level_apply<T>(const Node*, const ApplyLists&, const T*, const T*, int64_t, \
                                     int, const T*, bool, int, const T*, int64_t, T*, int64_t, T, \
                                     T, void*, size_t, hipStream_t);                              \
  template size_t apply_work_bytes<T>(const Forest&, const ApplyLists&, int, int);            \
  template void apply_forest<T>(const Node*, const ApplyLists&, const HbsView<T>&, bool, int,  \
                                const T*, int64_t, T*, int64_t, T, T, void*, size_t,           \
                                hipStream_t, bool);                                            \
  template void apply_forest_pair<T>(const Node*, const ApplyLists&, const HbsView<T>&, int,    \
                                     const T*, int64_t, void*, const T*, int64_t, T*, int64_t, \
                                     void*, size_t, hipStream_t);                               \
  template void seg_tn<T>(const Node*, const int32_t*, int, int64_t, int, int, const T*,       \
                          int64_t, const T*, int64_t, T*, int64_t, int64_t, T, T, void*,       \
                          hipStream_t, int);                                                   \
  template size_t seg_tn_work_bytes<T>(int, int64_t, int, int);
INST(double)
INST(float)

}  // namespace hm
