// Direct solver for an HBS matrix held in a handle: a factorisation of its
// inverse, built level by level from the leaves up, and the solve of A x = b
// with it (the fast direct solvers the paper names as the consumer of the
// compressed form; the algorithm is the one of Gillman, Young and
// Martinsson for HBS matrices in interpolative form).
//
// With A = D + U A~ V^* at a level (D block diagonal, U and V the nodes'
// bases, A~ the couplings of the next coarser level), per node
//   Dh = (V^* D^-1 U)^-1,  E = D^-1 U Dh,  F^* = Dh V^* D^-1,
//   G  = D^-1 - D^-1 U Dh V^* D^-1,
// and A^-1 = E (Dh + A~)^-1 F^* + G.  Dh + A~ is again HBS, one level up:
// a parent's "D" is [Dh_a  B_ab; B_ba  Dh_b] and its bases are its transfer
// matrices; at the root that block is inverted outright.  The solve takes the
// expansions b^_t = F_t^* b_t up the tree and x^_t = E_t x^_parent + G_t b^
// down it.  Every node block is small (leaves n_t x n_t, parents 2k x 2k):
// batched Gauss-Jordan inversions in LDS and batched MFMA products, one
// launch per level and step.
#include <algorithm>

#include "handle.h"
#include "tile_mfma.h"

namespace hm {

// ---- batched inversion --------------------------------------------------------
// In-place Gauss-Jordan with partial pivoting of one m x m matrix (m <= 128)
// per 256-thread workgroup, in LDS: at step k the row with the largest |a_ik|
// (i >= k, lowest index on ties) is swapped into row k, row k is scaled by
// 1 / a_kk with a_kk replaced by 1 first, and every other row i takes
// a_ij -= a_ik a_kj with a_ik replaced by 0 first; the row swaps are undone
// on the columns at the end, in reverse order.  A zero or non-finite pivot
// sets *singular.
struct InvDesc {
  const double* A;
  int64_t lda;
  double* out;
  int64_t ldo;
  int32_t m;
  int32_t pad_;
};

constexpr int INV_MMAX = 128;
constexpr int INV_LD = INV_MMAX + 1;

__global__ __launch_bounds__(256) void k_ginv(const InvDesc* descs, int32_t* singular) {
  __shared__ double sA[INV_MMAX * INV_LD];   // sA[i + j * INV_LD] = A(i, j)
  __shared__ double fcol[INV_MMAX];
  __shared__ int perm[INV_MMAX];
  __shared__ int s_p;
  const InvDesc d = descs[blockIdx.x];
  const int m = d.m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < m * m; e += 256) {
    const int i = e % m, j = e / m;
    sA[i + j * INV_LD] = d.A[i + (int64_t)j * d.lda];
  }
  __syncthreads();
  bool bad = false;
  for (int k = 0; k < m; ++k) {
    if (wave == 0) {
      // pivot: largest |a_ik|, i >= k; lanes take rows lane and lane + 64
      double best = -1.0;
      int bi = m;
      for (int i = k + lane; i < m; i += 64) {
        const double v = fabs(sA[i + k * INV_LD]);
        if (v > best) { best = v; bi = i; }
      }
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) {
        s_p = bi < m ? bi : k;
        perm[k] = s_p;
      }
    }
    __syncthreads();
    const int p = s_p;
    if (p != k)
      for (int j = tid; j < m; j += 256) {
        const double t = sA[k + j * INV_LD];
        sA[k + j * INV_LD] = sA[p + j * INV_LD];
        sA[p + j * INV_LD] = t;
      }
    __syncthreads();
    const double piv = sA[k + k * INV_LD];
    if (!(fabs(piv) > 0.0) || !isfinite(piv)) bad = true;
    const double rp = 1.0 / piv;
    // multipliers of the other rows, then row k scaled (a_kk -> 1 first)
    for (int i = tid; i < m; i += 256) fcol[i] = i == k ? 0.0 : sA[i + k * INV_LD];
    __syncthreads();
    for (int j = tid; j < m; j += 256) {
      const double v = j == k ? 1.0 : sA[k + j * INV_LD];
      sA[k + j * INV_LD] = v * rp;
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += 256) {
      const int i = e % m, j = e / m;
      if (i == k) continue;
      const double a = j == k ? 0.0 : sA[i + j * INV_LD];
      sA[i + j * INV_LD] = fma(-fcol[i], sA[k + j * INV_LD], a);
    }
    __syncthreads();
  }
  // undo the row swaps on the columns, last swap first; every row on its own
  for (int i = tid; i < m; i += 256)
    for (int k = m - 1; k >= 0; --k) {
      const int p = perm[k];
      if (p != k) {
        const double t = sA[i + k * INV_LD];
        sA[i + k * INV_LD] = sA[i + p * INV_LD];
        sA[i + p * INV_LD] = t;
      }
    }
  __syncthreads();
  for (int e = tid; e < m * m; e += 256) {
    const int i = e % m, j = e / m;
    d.out[i + (int64_t)j * d.ldo] = sA[i + j * INV_LD];
  }
  if (bad && tid == 0) atomicOr(singular, 1);
}

// ---- batched products -----------------------------------------------------------
// C = alpha op(A) op(B) + beta C per descriptor, op(A)(i, k) = A[i sai + k sak],
// op(B)(k, j) = B[k sbk + j sbj]; one 64 x 64 output tile per workgroup on
// FP64 MFMA (mf_tile).
struct GemmDesc {
  const double* A;
  int64_t sai, sak;
  const double* B;
  int64_t sbk, sbj;
  double* C;
  int64_t ldc;
  int32_t M, N, K, pad_;
  double alpha, beta;
};

__global__ __launch_bounds__(256) void k_bgemm(const GemmDesc* descs) {
  __shared__ double smem[mf_smem_elems<double>()];
  const GemmDesc d = descs[blockIdx.y];
  const int tm = (d.M + MF_T - 1) / MF_T, tn = (d.N + MF_T - 1) / MF_T;
  const int t = blockIdx.x;
  if (t >= tm * tn) return;
  const int i0 = (t % tm) * MF_T, j0 = (t / tm) * MF_T;
  MfAcc<double> acc;
  acc.zero();
  mf_tile<double>(d.M - i0, d.N - j0, d.K, d.A + (int64_t)i0 * d.sai, d.sai, d.sak,
                  d.B + (int64_t)j0 * d.sbj, d.sbk, d.sbj, acc, smem);
  mf_store<double>(d.M - i0, d.N - j0, d.C + i0 + (int64_t)j0 * d.ldc, d.ldc, acc, d.alpha,
                   d.beta);
}

// ---- parent blocks ---------------------------------------------------------------
// For parent t with children a, b (rank k each): Dp = [Dh_a B[b]; B[a] Dh_b]
// (2k x 2k; B[v] = B_{sib(v), v}), Up = rows (0:k, R:R+k) of the transfer Ut_t,
// Vp likewise; Dh at dh + node * k * k (ld k).
struct PackDesc {
  int32_t t, a, b, pad_;
  double* Dp;
  double* Up;
  double* Vp;
};

__global__ __launch_bounds__(256) void k_pack_parent(const PackDesc* descs, int k, int R,
                                                     const double* dh, const double* B,
                                                     const double* Ut, const double* Vt) {
  const PackDesc d = descs[blockIdx.x];
  const int k2 = 2 * k;
  const int tid = threadIdx.x;
  for (int e = tid; e < k2 * k2; e += 256) {
    const int i = e % k2, j = e / k2;
    double v;
    if (i < k && j < k) v = dh[(int64_t)d.a * k * k + i + j * k];
    else if (i >= k && j >= k) v = dh[(int64_t)d.b * k * k + (i - k) + (j - k) * k];
    else if (i < k) v = B[(int64_t)d.b * R * R + i + (int64_t)(j - k) * R];   // B_ab
    else v = B[(int64_t)d.a * R * R + (i - k) + (int64_t)j * R];              // B_ba
    d.Dp[i + (int64_t)j * k2] = v;
  }
  if (!d.Up) return;
  for (int e = tid; e < k2 * k; e += 256) {
    const int i = e % k2, j = e / k2;
    const int ri = i < k ? i : R + (i - k);
    d.Up[i + (int64_t)j * k2] = Ut[(int64_t)d.t * 2 * R * R + ri + (int64_t)j * 2 * R];
    d.Vp[i + (int64_t)j * k2] = Vt[(int64_t)d.t * 2 * R * R + ri + (int64_t)j * 2 * R];
  }
}

namespace {

void run_inv(const std::vector<InvDesc>& v, int32_t* singular, Keeper& kp, hipStream_t s) {
  if (v.empty()) return;
  for (const InvDesc& d : v)
    if (d.m > INV_MMAX) HM_THROW(HM_ERR_UNSUPPORTED, "solver: block of %d > %d", d.m, INV_MMAX);
  hipLaunchKernelGGL(k_ginv, dim3((unsigned)v.size()), dim3(256), 0, s, kp.put(v, s), singular);
  KCHK();
}

void run_gemm(const std::vector<GemmDesc>& v, Keeper& kp, hipStream_t s) {
  if (v.empty()) return;
  int tiles = 1;
  for (const GemmDesc& d : v)
    tiles = std::max(tiles, ((d.M + MF_T - 1) / MF_T) * ((d.N + MF_T - 1) / MF_T));
  hipLaunchKernelGGL(k_bgemm, dim3((unsigned)tiles, (unsigned)v.size()), dim3(256), 0, s,
                     kp.put(v, s));
  KCHK();
}

GemmDesc gemm(const double* A, int64_t sai, int64_t sak, const double* B, int64_t sbk,
              int64_t sbj, double* C, int64_t ldc, int M, int N, int K, double alpha,
              double beta) {
  GemmDesc d{};
  d.A = A; d.sai = sai; d.sak = sak;
  d.B = B; d.sbk = sbk; d.sbj = sbj;
  d.C = C; d.ldc = ldc;
  d.M = M; d.N = N; d.K = K;
  d.alpha = alpha; d.beta = beta;
  return d;
}

}  // namespace

}  // namespace hm

using namespace hm;

// Factor storage, node g = global node id, uniform rank k:
//   leaves   E, F (N x k, ld N), G (N x nmax, ld N, rows I_t, columns 0..n_t-1)
//   non-root Dh (k x k at g k^2)
//   internal non-root E, F (2k x k at g 2k^2), G (2k x 2k at g 4k^2)
//   root     G (2k x 2k)
struct hm_hbs_factor_s {
  Forest f;
  int k = 0;
  int64_t n = 0;
  DevBuf E, F, G;                 // leaves
  DevBuf Dh;                      // non-root nodes
  DevBuf Ep, Fp, Gp;              // internal non-root nodes
  DevBuf Groot;
};

extern "C" {

int hbs_factor(const hm_hbs* h, void* stream, hm_hbs_factor** out) {
  if (out) *out = nullptr;
  try {
    set_error("%s", "");
    StreamScope scope(stream);
    if (!h || !out) HM_THROW(HM_ERR_ARG, "factor: bad arguments");
    if (h->dtype != HM_F64) HM_THROW(HM_ERR_ARG, "factor: FP64 handles only (hm_hbs_convert)");
    const Forest& f = h->f;
    if (f.inst.size() != 1) HM_THROW(HM_ERR_ARG, "factor: single-tree handles only");
    const int L = f.inst[0].L;
    if (L < 1) HM_THROW(HM_ERR_ARG, "factor: the tree has no levels (invert D directly)");
    const int nn = (int)f.nodes.size();
    int k = -1;
    for (int g = 0; g < nn; ++g) {
      if (f.nodes[g].parent < 0) continue;
      const int ku = h->rank_u[g], kv = h->rank_v[g];
      if (k < 0) k = ku;
      if (ku != k || kv != k)
        HM_THROW(HM_ERR_UNSUPPORTED, "factor: node ranks must all equal (node %d: %d, %d; k %d)",
                 g, ku, kv, k);
    }
    if (k < 1) HM_THROW(HM_ERR_ARG, "factor: rank 0");
    for (const Node& nd : f.nodes)
      if (nd.left >= 0 && nd.right != nd.left + 1)
        HM_THROW(HM_ERR_ARG, "factor: sibling ids not consecutive");
    for (int g : f.leaves)
      if (f.nodes[g].hi - f.nodes[g].lo > INV_MMAX)
        HM_THROW(HM_ERR_UNSUPPORTED, "factor: leaves of more than %d rows", INV_MMAX);
    const int R = h->R;
    const int64_t N = f.n_total;
    const int nmax = f.nmax;
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<hm_hbs_factor_s> F(new hm_hbs_factor_s());
    F->f = f;
    F->k = k;
    F->n = N;
    const int k2 = 2 * k;
    F->E = DevBuf((size_t)N * k * 8);
    F->F = DevBuf((size_t)N * k * 8);
    F->G = DevBuf((size_t)N * nmax * 8);
    F->Dh = DevBuf((size_t)nn * k * k * 8);
    F->Ep = DevBuf((size_t)nn * k2 * k * 8);
    F->Fp = DevBuf((size_t)nn * k2 * k * 8);
    F->Gp = DevBuf((size_t)nn * k2 * k2 * 8);
    F->Groot = DevBuf((size_t)k2 * k2 * 8);
    // work: leaf W1, W2 (N x k); per node M (k x k), parent Dp (2k x 2k),
    // Up, Vp, W1p, W2p (2k x k)
    DevBuf W1((size_t)N * k * 8), W2((size_t)N * k * 8), M((size_t)nn * k * k * 8);
    DevBuf Dp((size_t)nn * k2 * k2 * 8), Up((size_t)nn * k2 * k * 8), Vp((size_t)nn * k2 * k * 8);
    DevBuf W1p((size_t)nn * k2 * k * 8), W2p((size_t)nn * k2 * k * 8);
    DevBuf sing(16);
    HIPCHK(hipMemsetAsync(sing.p, 0, 16, s));
    if (nmax > 0) HIPCHK(hipMemsetAsync(F->G.p, 0, F->G.bytes, s));
    Keeper kp;
    double* Dh = F->Dh.as<double>();
    double* Mm = M.as<double>();
    // ---- leaves: G first holds D^-1 ----
    {
      std::vector<InvDesc> inv;
      std::vector<GemmDesc> g1, g2, g3, g4;
      for (int g : f.leaves) {
        const Node& nd = f.nodes[g];
        const int m = (int)(nd.hi - nd.lo);
        const int64_t lo = nd.lo;
        double* Di = F->G.as<double>() + lo;
        inv.push_back(InvDesc{h->D.as<double>() + lo, N, Di, N, m, 0});
        const double* U = h->U.as<double>() + lo;
        const double* V = h->V.as<double>() + lo;
        double* w1 = W1.as<double>() + lo;
        double* w2 = W2.as<double>() + lo;
        // W1 = D^-1 U, W2 = D^-T V
        g1.push_back(gemm(Di, 1, N, U, 1, N, w1, N, m, k, m, 1.0, 0.0));
        g1.push_back(gemm(Di, N, 1, V, 1, N, w2, N, m, k, m, 1.0, 0.0));
        // M = V^T W1
        g2.push_back(gemm(V, N, 1, w1, 1, N, Mm + (int64_t)g * k * k, k, k, k, m, 1.0, 0.0));
        // E = W1 Dh, F = W2 Dh^T
        const double* dh = Dh + (int64_t)g * k * k;
        g3.push_back(gemm(w1, 1, N, dh, 1, k, F->E.as<double>() + lo, N, m, k, k, 1.0, 0.0));
        g3.push_back(gemm(w2, 1, N, dh, k, 1, F->F.as<double>() + lo, N, m, k, k, 1.0, 0.0));
        // G = D^-1 - E W2^T
        g4.push_back(gemm(F->E.as<double>() + lo, 1, N, w2, N, 1, Di, N, m, m, k, -1.0, 1.0));
      }
      run_inv(inv, sing.as<int32_t>(), kp, s);
      run_gemm(g1, kp, s);
      run_gemm(g2, kp, s);
      std::vector<InvDesc> invm;
      for (int g : f.leaves)
        invm.push_back(InvDesc{Mm + (int64_t)g * k * k, k, Dh + (int64_t)g * k * k, k, k, 0});
      run_inv(invm, sing.as<int32_t>(), kp, s);
      run_gemm(g3, kp, s);
      run_gemm(g4, kp, s);
    }
    // ---- internal non-root levels, finest first ----
    for (int l = L - 1; l >= 1; --l) {
      std::vector<PackDesc> pk;
      std::vector<InvDesc> inv, invm;
      std::vector<GemmDesc> g1, g2, g3, g4;
      for (int g : f.level[l]) {
        const Node& nd = f.nodes[g];
        if (nd.left < 0) continue;
        double* dp = Dp.as<double>() + (int64_t)g * k2 * k2;
        double* up = Up.as<double>() + (int64_t)g * k2 * k;
        double* vp = Vp.as<double>() + (int64_t)g * k2 * k;
        pk.push_back(PackDesc{g, nd.left, nd.right, 0, dp, up, vp});
        double* Di = F->Gp.as<double>() + (int64_t)g * k2 * k2;
        inv.push_back(InvDesc{dp, k2, Di, k2, k2, 0});
        double* w1 = W1p.as<double>() + (int64_t)g * k2 * k;
        double* w2 = W2p.as<double>() + (int64_t)g * k2 * k;
        g1.push_back(gemm(Di, 1, k2, up, 1, k2, w1, k2, k2, k, k2, 1.0, 0.0));
        g1.push_back(gemm(Di, k2, 1, vp, 1, k2, w2, k2, k2, k, k2, 1.0, 0.0));
        g2.push_back(gemm(vp, k2, 1, w1, 1, k2, Mm + (int64_t)g * k * k, k, k, k, k2, 1.0, 0.0));
        invm.push_back(InvDesc{Mm + (int64_t)g * k * k, k, Dh + (int64_t)g * k * k, k, k, 0});
        const double* dh = Dh + (int64_t)g * k * k;
        double* ep = F->Ep.as<double>() + (int64_t)g * k2 * k;
        double* fp = F->Fp.as<double>() + (int64_t)g * k2 * k;
        g3.push_back(gemm(w1, 1, k2, dh, 1, k, ep, k2, k2, k, k, 1.0, 0.0));
        g3.push_back(gemm(w2, 1, k2, dh, k, 1, fp, k2, k2, k, k, 1.0, 0.0));
        g4.push_back(gemm(ep, 1, k2, w2, k2, 1, Di, k2, k2, k2, k, -1.0, 1.0));
      }
      if (pk.empty()) continue;
      hipLaunchKernelGGL(k_pack_parent, dim3((unsigned)pk.size()), dim3(256), 0, s, kp.put(pk, s),
                         k, R, (const double*)Dh, h->B.as<double>(), h->Ut.as<double>(),
                         h->Vt.as<double>());
      KCHK();
      run_inv(inv, sing.as<int32_t>(), kp, s);
      run_gemm(g1, kp, s);
      run_gemm(g2, kp, s);
      run_inv(invm, sing.as<int32_t>(), kp, s);
      run_gemm(g3, kp, s);
      run_gemm(g4, kp, s);
    }
    // ---- root: invert [Dh_a B_ab; B_ba Dh_b] ----
    {
      const int root = f.inst[0].root;
      const Node& nd = f.nodes[root];
      std::vector<PackDesc> pk{PackDesc{root, nd.left, nd.right, 0, Dp.as<double>(), nullptr,
                                        nullptr}};
      hipLaunchKernelGGL(k_pack_parent, dim3(1), dim3(256), 0, s, kp.put(pk, s), k, R,
                         (const double*)Dh, h->B.as<double>(), h->Ut.as<double>(),
                         h->Vt.as<double>());
      KCHK();
      run_inv({InvDesc{Dp.as<double>(), k2, F->Groot.as<double>(), k2, k2, 0}},
              sing.as<int32_t>(), kp, s);
    }
    int hs[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(hs, sing.p, 16, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hs[0]) HM_THROW(HM_ERR_SINGULAR, "factor: a zero or non-finite pivot (singular block)");
    *out = F.release();
    return HM_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HM_ERR_ALLOC;
  } catch (...) {
    set_error("unexpected exception");
    return HM_ERR_HIP;
  }
}

int hbs_solve(const hm_hbs_factor* F, int64_t nrhs, const double* b, int64_t ldb, double* x,
              int64_t ldx, void* stream) {
  try {
    set_error("%s", "");
    StreamScope scope(stream);
    if (!F || !b || !x || nrhs < 0) HM_THROW(HM_ERR_ARG, "solve: bad arguments");
    const Forest& f = F->f;
    const int64_t N = F->n;
    if (ldb < N || ldx < N) HM_THROW(HM_ERR_ARG, "solve: ld < n");
    if (nrhs == 0) return HM_OK;
    hipStream_t s = (hipStream_t)stream;
    const int k = F->k, k2 = 2 * k, L = f.inst[0].L;
    const int nn = (int)f.nodes.size();
    Keeper kp;
    for (int64_t c0 = 0; c0 < nrhs; c0 += 128) {
      const int c = (int)std::min<int64_t>(128, nrhs - c0);
      const double* bb = b + c0 * ldb;
      double* xx = x + c0 * ldx;
      // expansions of every node as rows g k .. g k + k - 1 of an (nn k) x c
      // array, so that siblings (consecutive ids) form one 2k-row block
      const int64_t le = (int64_t)nn * k;
      DevBuf BH((size_t)le * c * 8), XH((size_t)le * c * 8);
      double* bh = BH.as<double>();
      double* xh = XH.as<double>();
      // up: leaves b^ = F^T b, parents b^ = F^T [b^_a; b^_b]
      std::vector<GemmDesc> up;
      for (int g : f.leaves) {
        const Node& nd = f.nodes[g];
        const int m = (int)(nd.hi - nd.lo);
        up.push_back(gemm(F->F.as<double>() + nd.lo, N, 1, bb + nd.lo, 1, ldb,
                          bh + (int64_t)g * k, le, k, c, m, 1.0, 0.0));
      }
      run_gemm(up, kp, s);
      for (int l = L - 1; l >= 1; --l) {
        std::vector<GemmDesc> v;
        for (int g : f.level[l]) {
          const Node& nd = f.nodes[g];
          if (nd.left < 0) continue;
          v.push_back(gemm(F->Fp.as<double>() + (int64_t)g * k2 * k, k2, 1,
                           bh + (int64_t)nd.left * k, 1, le, bh + (int64_t)g * k, le, k, c, k2,
                           1.0, 0.0));
        }
        run_gemm(v, kp, s);
      }
      // root: [x^_a; x^_b] = G_root [b^_a; b^_b]
      {
        const Node& nd = f.nodes[f.inst[0].root];
        run_gemm({gemm(F->Groot.as<double>(), 1, k2, bh + (int64_t)nd.left * k, 1, le,
                       xh + (int64_t)nd.left * k, le, k2, c, k2, 1.0, 0.0)},
                 kp, s);
      }
      // down: [x^_a; x^_b] = E x^_t + G [b^_a; b^_b]
      for (int l = 1; l < L; ++l) {
        std::vector<GemmDesc> v1, v2;
        for (int g : f.level[l]) {
          const Node& nd = f.nodes[g];
          if (nd.left < 0) continue;
          double* o = xh + (int64_t)nd.left * k;
          v1.push_back(gemm(F->Ep.as<double>() + (int64_t)g * k2 * k, 1, k2, xh + (int64_t)g * k,
                            1, le, o, le, k2, c, k, 1.0, 0.0));
          v2.push_back(gemm(F->Gp.as<double>() + (int64_t)g * k2 * k2, 1, k2,
                            bh + (int64_t)nd.left * k, 1, le, o, le, k2, c, k2, 1.0, 1.0));
        }
        run_gemm(v1, kp, s);
        run_gemm(v2, kp, s);
      }
      // leaves: x_t = E x^_t + G b_t
      std::vector<GemmDesc> v1, v2;
      for (int g : f.leaves) {
        const Node& nd = f.nodes[g];
        const int m = (int)(nd.hi - nd.lo);
        v1.push_back(gemm(F->E.as<double>() + nd.lo, 1, N, xh + (int64_t)g * k, 1, le,
                          xx + nd.lo, ldx, m, c, k, 1.0, 0.0));
        v2.push_back(gemm(F->G.as<double>() + nd.lo, 1, N, bb + nd.lo, 1, ldb, xx + nd.lo, ldx, m,
                          c, m, 1.0, 1.0));
      }
      run_gemm(v1, kp, s);
      run_gemm(v2, kp, s);
      // BH, XH and the tables go back to the library's cache for stream s (or
      // to the caller's allocator, stream-ordered): reuse is ordered after
      // this work
    }
    return HM_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HM_ERR_ALLOC;
  } catch (...) {
    set_error("unexpected exception");
    return HM_ERR_HIP;
  }
}

void hm_hbs_factor_free(hm_hbs_factor* F) { delete F; }

}  // extern "C"
