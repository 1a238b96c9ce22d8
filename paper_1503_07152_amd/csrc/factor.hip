// Node factorisations: TSQR panels, reflector application, Jacobi SVD,
// node-block gather, interaction matrices, column-pivoted QR / ID.
#include <cfloat>

#include "factor.h"
#include "tile.h"

namespace hm {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

constexpr int FT = 1024;
constexpr int FW = FT / 64;

// Sum of the FW per-wave partials p[0], p[S], p[2 S], ... as a balanced tree
// (short dependency chain).
template <int S>
__device__ __forceinline__ double sum_waves(const double* p) {
  double v[FW];
#pragma unroll
  for (int w = 0; w < FW; ++w) v[w] = p[w * S];
#pragma unroll
  for (int h = FW / 2; h >= 1; h >>= 1)
#pragma unroll
    for (int w = 0; w < h; ++w) v[w] += v[w + h];
  return v[0];
}

// ------------------------------------------------------------ panel QR ----
// The node factorisations keep a whole panel in LDS (up to ~150 KB), so only
// one workgroup fits on a CU; 1024 threads (4 waves per SIMD) hide the LDS
// and FP64 latencies within that workgroup.

// Unblocked Householder QR (H_j = I - tau_j v_j v_j^T, v_j(j) = 1) of one
// panel held in LDS.  Reflectors are stored below the diagonal, R on and above.
// Per column j, one reduction gives g_k = sum_{i>=j} A(i,j) A(i,k) for all
// k > j and, for k = j, the squared norm below the diagonal.  With
// beta = -sign(x0) |A(j:,j)| and v = [1; A(j+1:,j)/(x0 - beta)] one has
// v^T A(j:,k) = (g_k - beta A(j,k)) / (x0 - beta), so the update needs no
// second reduction.  The scaling of column j into v is deferred to the next
// step (which never reads column j): three barriers per column.
__global__ __launch_bounds__(FT) void k_panel_qr(const PanelDesc* descs) {
  __shared__ double sA[FAC_LDMAX * FAC_CMAX];
  __shared__ double part[FW][FAC_CMAX];
  __shared__ double sw[FAC_CMAX];
  __shared__ double sc[4];
  const PanelDesc d = descs[blockIdx.x];
  const int m = d.rows, n = d.cols;
  const int lds = (m & 1) ? m : m + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int idx = tid; idx < m * n; idx += FT) {
    const int i = idx % m, j = idx / m;
    sA[i + j * lds] = d.trans ? d.A[j + (int64_t)i * d.ld] : d.A[i + (int64_t)j * d.ld];
  }
  if (tid == 0) { sc[0] = 0.0; sc[1] = 0.0; sc[2] = 0.0; sc[3] = -1.0; }
  __syncthreads();
  const int h = min(m, n);
  for (int j = 0; j < h; ++j) {
    // deferred scaling of the previous reflector column
    const int jp = (int)sc[3];
    if (jp >= 0) {
      const double scl = sc[2], bet = sc[0];
      if (sc[1] != 0.0)
        for (int i = jp + 1 + tid; i < m; i += FT) sA[i + jp * lds] *= scl;
      if (tid == 0) sA[jp + jp * lds] = bet;
    }
    // partial inner products of column j with columns j..n-1 over this wave's
    // rows; fixed trip counts (rows outside the panel weigh zero, their reads
    // are clamped into it) so the LDS reads issue back to back
    const int rows = m - j;
    const int q = (rows + FW - 1) / FW;
    const int ib = j + wave * q, ie = min(m, ib + q);
    double cj[FAC_PMAX / FW];
#pragma unroll
    for (int t = 0; t < FAC_PMAX / FW; ++t) {
      const int i = ib + t;
      cj[t] = i < ie ? sA[i + j * lds] : 0.0;
    }
    for (int kb = 0; kb < n - j; kb += 64) {
      const int kk = kb + lane;
      const int k = j + min(kk, n - j - 1);
      double bv[FAC_PMAX / FW];
#pragma unroll
      for (int t = 0; t < FAC_PMAX / FW; ++t) bv[t] = sA[min(ib + t, m - 1) + k * lds];
      // the diagonal term is left out of the norm below the diagonal (k = j)
      double s0 = ((wave == 0 && kk == 0) ? 0.0 : cj[0]) * bv[0], s1 = cj[1] * bv[1],
             s2 = cj[2] * bv[2], s3 = cj[3] * bv[3];
#pragma unroll
      for (int t = 4; t < FAC_PMAX / FW; t += 4) {
        s0 = fma(cj[t], bv[t], s0);
        s1 = fma(cj[t + 1], bv[t + 1], s1);
        s2 = fma(cj[t + 2], bv[t + 2], s2);
        s3 = fma(cj[t + 3], bv[t + 3], s3);
      }
      if (kk < n - j) part[wave][kk] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
    // combine: reflector scalars and w_k = v^T A(j:, k)
    {
      const double x0 = sA[j + j * lds];
      const double sig = sum_waves<FAC_CMAX>(&part[0][0]);
      double beta = x0, tau = 0.0, scl = 0.0;
      if (sig != 0.0) {
        beta = -copysign(sqrt(fma(x0, x0, sig)), x0);
        tau = (beta - x0) / beta;
        scl = 1.0 / (x0 - beta);
      }
      for (int kk = 1 + tid; kk < n - j; kk += FT) {
        const int k = j + kk;
        const double g = sum_waves<FAC_CMAX>(&part[0][kk]);
        sw[k] = (g - beta * sA[j + k * lds]) * scl;
      }
      if (tid == 0) {
        sc[0] = beta; sc[1] = tau; sc[2] = scl; sc[3] = (double)j;
        d.tau[j] = tau;
      }
    }
    __syncthreads();
    const double tau = sc[1], scl = sc[2];
    if (tau != 0.0) {
      // lanes walk the rows (j + lane + 64 t), waves the columns (j + 1 + wave + 16 u)
      double vr[FAC_PMAX / 64];
#pragma unroll
      for (int t = 0; t < FAC_PMAX / 64; ++t) {
        const int i = j + lane + 64 * t;
        vr[t] = i < m ? (i == j ? 1.0 : sA[i + j * lds] * scl) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < FAC_CMAX / FW; ++u) {
        const int k = j + 1 + wave + FW * u;
        if (k < n) {
          const double tw = tau * sw[k];
#pragma unroll
          for (int t = 0; t < FAC_PMAX / 64; ++t) {
            const int i = j + lane + 64 * t;
            if (i < m) sA[i + k * lds] -= tw * vr[t];
          }
        }
      }
    }
    __syncthreads();
  }
  if (h > 0) {
    const int jp = h - 1;
    const double scl = sc[2], bet = sc[0];
    if (sc[1] != 0.0)
      for (int i = jp + 1 + tid; i < m; i += FT) sA[i + jp * lds] *= scl;
    if (tid == 0) sA[jp + jp * lds] = bet;
  }
  __syncthreads();
  for (int idx = tid; idx < m * n; idx += FT) {
    const int i = idx % m, j = idx / m;
    d.A[i + (int64_t)j * d.ld] = sA[i + j * lds];
  }
  if (d.Rout)
    for (int idx = tid; idx < h * n; idx += FT) {
      const int i = idx % h, j = idx / h;
      d.Rout[i + (int64_t)j * d.ldR] = (i <= j) ? sA[i + j * lds] : 0.0;
    }
}

void launch_panel_qr(const PanelDesc* d, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_panel_qr, dim3(n), dim3(FT), 0, s, d);
  KCHK();
}

// Cout = H_0 H_1 ... H_{h-1} [Cin; 0].  The next reflector is prefetched from
// global memory into registers while the current one is applied.
constexpr int APQ_NMAX = HM_MAX_SAMPLES;
__global__ __launch_bounds__(FT) void k_apply_q(const PanelDesc* descs) {
  __shared__ double sO[FAC_LDMAX * APQ_NMAX];
  __shared__ double sv[2][FAC_PMAX];
  __shared__ double part[FW][64];
  __shared__ double sw[64];
  const PanelDesc d = descs[blockIdx.x];
  const int m = d.rows, h = min(d.rows, d.cols), nc = d.ncol;
  const int ldo = (m & 1) ? m : m + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int idx = tid; idx < m * nc; idx += FT) {
    const int i = idx % m, c = idx / m;
    sO[i + c * ldo] = (i < h) ? d.Cin[i + (int64_t)c * d.ldCin] : 0.0;
  }
  auto vload = [&](int j) -> double {
    if (j < 0 || tid >= m || tid < j) return 0.0;
    return tid == j ? 1.0 : d.A[tid + (int64_t)j * d.ld];
  };
  if (h > 0 && tid < m) sv[0][tid] = vload(h - 1);
  __syncthreads();
  int buf = 0;
  for (int j = h - 1; j >= 0; --j) {
    const double vnext = vload(j - 1);
    const double tau = d.tau[j];
    if (tau != 0.0) {
      const int rows = m - j, q = (rows + FW - 1) / FW;
      const int ib = j + wave * q, ie = min(m, ib + q);
      const int cl = max(min(lane, nc - 1), 0);
      double av[FAC_PMAX / FW], bv[FAC_PMAX / FW];
#pragma unroll
      for (int t = 0; t < FAC_PMAX / FW; ++t) {
        const int i = ib + t;
        av[t] = i < ie ? sv[buf][i] : 0.0;
        bv[t] = sO[min(i, m - 1) + cl * ldo];
      }
      double s0 = av[0] * bv[0], s1 = av[1] * bv[1], s2 = av[2] * bv[2], s3 = av[3] * bv[3];
#pragma unroll
      for (int t = 4; t < FAC_PMAX / FW; t += 4) {
        s0 = fma(av[t], bv[t], s0);
        s1 = fma(av[t + 1], bv[t + 1], s1);
        s2 = fma(av[t + 2], bv[t + 2], s2);
        s3 = fma(av[t + 3], bv[t + 3], s3);
      }
      part[wave][lane] = lane < nc ? (s0 + s1) + (s2 + s3) : 0.0;
      __syncthreads();
      if (wave == 0) sw[lane] = sum_waves<64>(&part[0][lane]);
      __syncthreads();
      double vr[FAC_PMAX / 64];
#pragma unroll
      for (int t = 0; t < FAC_PMAX / 64; ++t) {
        const int i = j + lane + 64 * t;
        vr[t] = i < m ? sv[buf][i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < (APQ_NMAX + FW - 1) / FW; ++u) {
        const int cc = wave + FW * u;
        if (cc < nc) {
          const double tw = tau * sw[cc];
#pragma unroll
          for (int t = 0; t < FAC_PMAX / 64; ++t) {
            const int i = j + lane + 64 * t;
            if (i < m) sO[i + cc * ldo] -= tw * vr[t];
          }
        }
      }
    }
    if (tid < m) sv[buf ^ 1][tid] = vnext;
    buf ^= 1;
    __syncthreads();
  }
  for (int idx = tid; idx < m * nc; idx += FT) {
    const int i = idx % m, c = idx / m;
    d.Cout[i + (int64_t)c * d.ldCout] = sO[i + c * ldo];
  }
}

void launch_apply_q(const PanelDesc* d, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_apply_q, dim3(n), dim3(FT), 0, s, d);
  KCHK();
}

// ------------------------------------------------------------ Jacobi SVD --
// One-sided (Hestenes) Jacobi on the columns of an h x c matrix T (T = R, or
// T = R^T when the descriptor asks for the transpose): T Z = W diag(s).  Pairs
// follow a round-robin tournament; each 16-lane group rotates one pair, so a
// 1024-thread workgroup treats every pair of a round (c <= 96) at once.  The
// pair's two squared norms and inner product are reduced across the group by
// DPP row operations (no LDS round trip), which leaves the same sum in every
// lane.
constexpr int JAC_LD = FAC_CMAX + 1;
constexpr int JAC_GROUPS = FT / 16;
constexpr int JAC_RPL = FAC_CMAX / 16;  // rows per lane of a 16-lane group

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// sum over the 16 lanes of a row: lane pairs (xor 1, xor 2 by quad permutes),
// then the mirrored quad of each half-row, then the mirrored half-row
__device__ __forceinline__ double sum16(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return v;
}

__global__ __launch_bounds__(FT) void k_jacobi(const SvdDesc* descs) {
  __shared__ double sA[FAC_CMAX * JAC_LD];
  __shared__ double sZ[FAC_CMAX * JAC_LD];
  __shared__ double snorm[FAC_CMAX];
  __shared__ int srank[FAC_CMAX];
  __shared__ int flag;
  const SvdDesc d = descs[blockIdx.x];
  const int h = d.h, c = d.c;
  const bool wantX = d.X != nullptr;
  const int tid = threadIdx.x;
  const int grp = tid >> 4, gl = tid & 15;
  for (int idx = tid; idx < h * c; idx += FT) {
    const int i = idx % h, j = idx / h;
    sA[i + j * JAC_LD] = d.trans ? d.R[j + (int64_t)i * d.ldR] : d.R[i + (int64_t)j * d.ldR];
  }
  if (wantX)
    for (int idx = tid; idx < c * c; idx += FT) {
      const int i = idx % c, j = idx / c;
      sZ[i + j * JAC_LD] = (i == j) ? 1.0 : 0.0;
    }
  __syncthreads();
  const int n2 = c + (c & 1);
  const int hm1 = max(h - 1, 0);
  const double tol = (double)max(h, 1) * DBL_EPSILON;
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    if (tid == 0) flag = 0;
    __syncthreads();
    for (int t = 0; t < n2 - 1; ++t) {
      for (int pi = grp; pi < n2 / 2; pi += JAC_GROUPS) {
        const int a = pi, b = n2 - 1 - pi;
        const int pa = a == 0 ? 0 : 1 + (a - 1 + t) % (n2 - 1);
        const int pb = b == 0 ? 0 : 1 + (b - 1 + t) % (n2 - 1);
        const int p = min(pa, pb), q = max(pa, pb);
        if (q >= c) continue;
        // the group's rows gl + 16 u (fixed trip count; rows past h weigh zero)
        double xv[JAC_RPL], yv[JAC_RPL];
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int u = 0; u < JAC_RPL; ++u) {
          const int i = gl + 16 * u;
          const int ic = min(i, hm1);
          const double w = i < h ? 1.0 : 0.0;
          xv[u] = w * sA[ic + p * JAC_LD];
          yv[u] = w * sA[ic + q * JAC_LD];
          al = fma(xv[u], xv[u], al);
          be = fma(yv[u], yv[u], be);
          ga = fma(xv[u], yv[u], ga);
        }
        al = sum16(al);
        be = sum16(be);
        ga = sum16(ga);
        if (ga != 0.0 && fabs(ga) > tol * sqrt(al) * sqrt(be)) {
          // rotation zeroing the pair's inner product: t = tan(theta) is the
          // smaller root of t^2 ga + t (be - al) - ga = 0
          const double dd = be - al;
          const double q2 = fma(dd, dd, 4.0 * ga * ga);
          double tt, cs;
          if (q2 > 1e-280 && q2 < 1e280) {
            // hardware reciprocal (square root) estimates refined by Newton
            // steps: one for t (its accuracy only sets how far the pair's
            // inner product drops), two for cs, so that cs^2 + sn^2 = 1 to
            // rounding without bias and the accumulated rotations stay
            // orthogonal
            double r = __builtin_amdgcn_rsq(q2);
            r = r * fma(-0.5 * q2 * r, r, 1.5);
            const double den = fabs(dd) + q2 * r;
            double rd = __builtin_amdgcn_rcp(den);
            rd = fma(rd, fma(-den, rd, 1.0), rd);
            tt = 2.0 * ga * (dd >= 0.0 ? 1.0 : -1.0) * rd;
            const double u1 = fma(tt, tt, 1.0);
            // residual form e = 1/2 - (u1 cs / 2) cs, cs += cs e: unlike
            // cs (3/2 - u1 cs^2 / 2) it reaches cs = 1 exactly when u1 = 1
            // (tiny angles), so the rotations do not shrink systematically
            cs = __builtin_amdgcn_rsq(u1);
#pragma unroll
            for (int it = 0; it < 2; ++it) cs = fma(cs, fma(-0.5 * u1 * cs, cs, 0.5), cs);
          } else {
            tt = 2.0 * ga * (dd >= 0.0 ? 1.0 : -1.0) / (fabs(dd) + sqrt(q2));
            cs = rsqrt(fma(tt, tt, 1.0));
          }
          const double sn = cs * tt;
#pragma unroll
          for (int u = 0; u < JAC_RPL; ++u) {
            const int i = gl + 16 * u;
            if (i < h) {
              sA[i + p * JAC_LD] = cs * xv[u] - sn * yv[u];
              sA[i + q * JAC_LD] = sn * xv[u] + cs * yv[u];
            }
          }
          if (wantX) {
#pragma unroll
            for (int u = 0; u < JAC_RPL; ++u) {
              const int i = gl + 16 * u;
              const int ic = min(i, c - 1);
              const double x = sZ[ic + p * JAC_LD], y = sZ[ic + q * JAC_LD];
              if (i < c) {
                sZ[i + p * JAC_LD] = cs * x - sn * y;
                sZ[i + q * JAC_LD] = sn * x + cs * y;
              }
            }
          }
          if (gl == 0) flag = 1;
        }
      }
      __syncthreads();
    }
    if (flag == 0) break;
    __syncthreads();  // every thread has read flag before it is reset
  }
  if (tid == 0 && d.sweeps) atomicMax(d.sweeps, sweep + 1);
  for (int j = tid; j < c; j += FT) {
    double s = 0.0;
    for (int i = 0; i < h; ++i) s += sA[i + j * JAC_LD] * sA[i + j * JAC_LD];
    snorm[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < c; j += FT) {
    const double sj = snorm[j];
    int rk = 0;
    for (int i2 = 0; i2 < c; ++i2) rk += (snorm[i2] > sj) || (snorm[i2] == sj && i2 < j);
    srank[j] = rk;
  }
  __syncthreads();
  // column j goes to position srank[j] (descending norms, ties by index);
  // positions c .. kout - 1 (a matrix with fewer columns than asked) are zero
  const int rows = max(h, c);
  for (int e = tid; e < c * rows; e += FT) {
    const int i = e % rows, j = e / rows;
    const int rk = srank[j];
    if (rk >= d.kout) continue;
    const double sj = snorm[j];
    if (i == 0) d.sv[rk] = sj;
    if (i < h) d.W[i + (int64_t)rk * d.ldW] = sj > 0.0 ? sA[i + j * JAC_LD] / sj : 0.0;
    if (wantX && i < c) d.X[i + (int64_t)rk * d.ldX] = sZ[i + j * JAC_LD];
  }
  for (int e = tid; e < (d.kout - c) * rows; e += FT) {
    const int i = e % rows, rk = c + e / rows;
    if (i == 0) d.sv[rk] = 0.0;
    if (i < h) d.W[i + (int64_t)rk * d.ldW] = 0.0;
    if (wantX && i < c) d.X[i + (int64_t)rk * d.ldX] = 0.0;
  }
}

void launch_jacobi_svd(const SvdDesc* d, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_jacobi, dim3(n), dim3(FT), 0, s, d);
  KCHK();
}

// ------------------------------------------------------------ gathers -----
__global__ void k_build_node_block(const Node* nodes, const Instance* inst, const int32_t* kids,
                                   int R, const double* S, int64_t lds, const double* Lpar,
                                   int64_t ldl, const double* w, double* M, int64_t ldm,
                                   int first_half_only) {
  const Node nd = nodes[kids[blockIdx.y]];
  const int64_t i = nd.lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nd.hi) return;
  const int r = inst[nd.inst].r;
  const int off = nd.is_left ? 0 : R;
  for (int j = 0; j < r; ++j) M[i + (int64_t)j * ldm] = S[i + (int64_t)(off + j) * lds];
  if (!first_half_only && nodes[nd.parent].parent >= 0) {
    const double* wp = w + (int64_t)nd.parent * R;
    for (int j = 0; j < r; ++j) M[i + (int64_t)(r + j) * ldm] = Lpar[i + (int64_t)j * ldl] * wp[j];
  }
}

void launch_build_node_block(const Node* nodes, const Instance* inst, const int32_t* kids,
                             int nkids, int64_t max_rows, int R, const double* S, int64_t lds,
                             const double* Lpar, int64_t ldl, const double* w, double* M,
                             int64_t ldm, hipStream_t s, int first_half_only) {
  if (nkids <= 0) return;
  const int nt = 256;
  hipLaunchKernelGGL(k_build_node_block, dim3((unsigned)((max_rows + nt - 1) / nt), nkids),
                     dim3(nt), 0, s, nodes, inst, kids, R, S, lds, Lpar, ldl, w, M, ldm,
                     first_half_only);
  KCHK();
}

__global__ void k_form_b(const Node* nodes, const Instance* inst, const int32_t* kids, int R,
                         const double* X, const double* z, double* B) {
  const int v = kids[blockIdx.x];
  const int r = inst[nodes[v].inst].r;
  const double* Xv = X + (int64_t)v * 2 * R * R;
  const double* zv = z + (int64_t)v * R;
  double* Bv = B + (int64_t)v * R * R;
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    const int i = e % R, j = e / R;
    Bv[e] = (i < r && j < r) ? Xv[i + j * 2 * R] * zv[j] : 0.0;
  }
}

void launch_form_b(const Node* nodes, const Instance* inst, const int32_t* kids, int nkids, int R,
                   const double* X, const double* z, double* B, hipStream_t s) {
  if (nkids <= 0) return;
  hipLaunchKernelGGL(k_form_b, dim3(nkids), dim3(256), 0, s, nodes, inst, kids, R, X, z, B);
  KCHK();
}

// ------------------------------------------------------------ CPQR / ID ---
constexpr int ID_NMAX = 256;  // candidates per node (leaf rows or 2R)
__global__ __launch_bounds__(256) void k_cpqr_id(const Node* nodes, const Instance* inst,
                                                 const int32_t* list, int parent_mode, int R,
                                                 const double* Src, int64_t lds, const double* w,
                                                 double* P, int64_t ldp, double* samp,
                                                 int32_t* rank, int32_t* skel, int32_t* saturated) {
  __shared__ double sM[(HM_MAX_SAMPLES + 1) * ID_NMAX];  // M = W^T, R x n, ld R+1
  __shared__ double snrm[ID_NMAX];
  __shared__ int sperm[ID_NMAX];
  __shared__ double sv[HM_MAX_SAMPLES];
  __shared__ double sc[4];
  __shared__ int sk[2];
  const int g = list[blockIdx.x];
  const Node nd = nodes[g];
  const Instance in = inst[nd.inst];
  const int tid = threadIdx.x;
  const int ldm = R + 1;
  const int n = parent_mode ? 2 * R : (int)(nd.hi - nd.lo);
  const double* src = parent_mode ? Src + (int64_t)g * 2 * R * R : Src + nd.lo;
  const int64_t ls = parent_mode ? 2 * R : lds;
  const double* wv = w + (int64_t)g * R;
  for (int idx = tid; idx < n * R; idx += 256) {
    const int b = idx % n, a = idx / n;  // candidate b, sample dim a
    sM[a + b * ldm] = src[b + (int64_t)a * ls] * wv[a];
  }
  for (int b = tid; b < n; b += 256) sperm[b] = b;
  __syncthreads();
  const int kcap = min(min(in.k, in.r), min(R, n));
  int k = 0;
  double ref = 0.0;
  for (int j = 0; j < kcap; ++j) {
    for (int b = j + tid; b < n; b += 256) {
      double s = 0.0;
      for (int a = j; a < R; ++a) s += sM[a + b * ldm] * sM[a + b * ldm];
      snrm[b] = s;
    }
    __syncthreads();
    if (tid == 0) {
      int p = j;
      double best = snrm[j];
      for (int b = j + 1; b < n; ++b)
        if (snrm[b] > best) { best = snrm[b]; p = b; }
      sk[0] = p;
      sc[0] = sqrt(best);
    }
    __syncthreads();
    const int p = sk[0];
    const double nrm = sc[0];
    if (j == 0) ref = nrm;
    if (nrm == 0.0 || (in.tol > 0.0 && nrm <= in.tol * ref)) break;
    if (p != j) {
      for (int a = tid; a < R; a += 256) {
        const double t = sM[a + j * ldm];
        sM[a + j * ldm] = sM[a + p * ldm];
        sM[a + p * ldm] = t;
      }
      if (tid == 0) {
        const int t = sperm[j]; sperm[j] = sperm[p]; sperm[p] = t;
      }
    }
    __syncthreads();
    // Householder reflector zeroing M(j+1:R, j): v = x - alpha e1, H = I - 2 v v^T / (v^T v)
    if (tid == 0) {
      double s = 0.0;
      for (int a = j; a < R; ++a) s += sM[a + j * ldm] * sM[a + j * ldm];
      const double x0 = sM[j + j * ldm];
      const double alpha = -copysign(sqrt(s), x0);
      for (int a = j; a < R; ++a) sv[a] = sM[a + j * ldm];
      sv[j] = x0 - alpha;
      const double vn = s - x0 * x0 + sv[j] * sv[j];
      sc[1] = alpha;
      sc[2] = vn > 0.0 ? 2.0 / vn : 0.0;
    }
    __syncthreads();
    const double f = sc[2];
    for (int b = j + 1 + tid; b < n; b += 256) {
      double s = 0.0;
      for (int a = j; a < R; ++a) s += sv[a] * sM[a + b * ldm];
      s *= f;
      for (int a = j; a < R; ++a) sM[a + b * ldm] -= s * sv[a];
    }
    __syncthreads();
    if (tid == 0) {
      sM[j + j * ldm] = sc[1];
      for (int a = j + 1; a < R; ++a) sM[a + j * ldm] = 0.0;
    }
    __syncthreads();
    k = j + 1;
  }
  // T = R11^{-1} R12, column by column (back substitution); stored in place of R12.
  for (int b = k + tid; b < n; b += 256) {
    for (int a = k - 1; a >= 0; --a) {
      double s = sM[a + b * ldm];
      for (int c2 = a + 1; c2 < k; ++c2) s -= sM[a + c2 * ldm] * sM[c2 + b * ldm];
      sM[a + b * ldm] = s / sM[a + a * ldm];
    }
  }
  __syncthreads();
  // P (n x R): row perm[b] = e_b (b < k) or T(:, b)^T (b >= k); columns >= k zero.
  double* Pout = parent_mode ? P + (int64_t)g * 2 * R * R : P + nd.lo;
  const int64_t lp = parent_mode ? 2 * R : ldp;
  for (int idx = tid; idx < n * R; idx += 256) {
    const int b = idx % n, col = idx / n;
    double v = 0.0;
    if (col < k) v = (b < k) ? (b == col ? 1.0 : 0.0) : sM[col + b * ldm];
    Pout[sperm[b] + (int64_t)col * lp] = v;
  }
  double* sp = samp + (int64_t)g * R * R;
  for (int idx = tid; idx < R * R; idx += 256) {
    const int i = idx % R, a = idx / R;
    sp[idx] = (i < k) ? src[sperm[i] + (int64_t)a * ls] : 0.0;
  }
  int32_t* sk_out = skel + (int64_t)g * R;
  for (int i = tid; i < R; i += 256) {
    int id = -1;
    if (i < k) {
      const int cnd = sperm[i];
      if (!parent_mode) id = (int)(nd.lo - in.row0) + cnd;
      else id = cnd < R ? skel[(int64_t)nd.left * R + cnd] : skel[(int64_t)nd.right * R + cnd - R];
    }
    sk_out[i] = id;
  }
  if (tid == 0) {
    rank[g] = k;
    if (in.tol > 0.0 && k >= in.r - in.p && saturated) atomicAdd(saturated, 1);
  }
}

void launch_cpqr_id(const Node* nodes, const Instance* inst, const int32_t* list, int nlist,
                    int parent_mode, int R, const double* Src, int64_t lds, const double* w,
                    double* P, int64_t ldp, double* samp, int32_t* rank, int32_t* skel,
                    int32_t* saturated, hipStream_t s) {
  if (nlist <= 0) return;
  hipLaunchKernelGGL(k_cpqr_id, dim3(nlist), dim3(256), 0, s, nodes, inst, list, parent_mode, R,
                     Src, lds, w, P, ldp, samp, rank, skel, saturated);
  KCHK();
}

constexpr int STM = 64, STN = 64;
__global__ __launch_bounds__(256) void k_utmp(const Node* nodes, const int32_t* list, int R,
                                              const double* samp, const double* Tr,
                                              double* Utmp) {
  __shared__ double smem[tile_smem_elems<STM, STN>()];
  const int t = list[blockIdx.x];
  const int side = blockIdx.y;
  const Node nd = nodes[t];
  const int ch = side == 0 ? nd.left : nd.right;
  TileAcc<double, STM, STN> acc;
  acc.zero();
  mm_tile<double, STM, STN>(R, R, R, samp + (int64_t)ch * R * R, 1, R,
                            Tr + (int64_t)t * 2 * R * R + side * R, 1, 2 * R, acc, smem);
  store_tile<double, STM, STN>(R, R, Utmp + (int64_t)t * 2 * R * R + side * R, 2 * R, acc, 1.0,
                               0.0);
}

void launch_utmp(const Node* nodes, const int32_t* list, int nlist, int R, const double* samp,
                 const double* Tr, double* Utmp, hipStream_t s) {
  if (nlist <= 0) return;
  hipLaunchKernelGGL(k_utmp, dim3(nlist, 2), dim3(256), 0, s, nodes, list, R, samp, Tr, Utmp);
  KCHK();
}

__global__ __launch_bounds__(256) void k_bskel(const Node* nodes, const int32_t* list, int R,
                                               const double* sampU, const double* sampV,
                                               const double* Bold, double* Bnew) {
  __shared__ double smem[tile_smem_elems<STM, STN>()];
  __shared__ double sT[STM * STN];
  const int v = list[blockIdx.x];
  const int sb = nodes[v].sib;
  TileAcc<double, STM, STN> acc;
  acc.zero();
  // T1 = Bold[v] sampV[v]^T  (R x R)
  mm_tile<double, STM, STN>(R, R, R, Bold + (int64_t)v * R * R, 1, R, sampV + (int64_t)v * R * R,
                            R, 1, acc, smem);
  store_tile<double, STM, STN>(R, R, sT, STM, acc, 1.0, 0.0);
  __syncthreads();
  acc.zero();
  mm_tile<double, STM, STN>(R, R, R, sampU + (int64_t)sb * R * R, 1, R, sT, 1, STM, acc, smem);
  store_tile<double, STM, STN>(R, R, Bnew + (int64_t)v * R * R, R, acc, 1.0, 0.0);
}

void launch_bskel(const Node* nodes, const int32_t* list, int nlist, int R, const double* sampU,
                  const double* sampV, const double* Bold, double* Bnew, hipStream_t s) {
  if (nlist <= 0) return;
  hipLaunchKernelGGL(k_bskel, dim3(nlist), dim3(256), 0, s, nodes, list, R, sampU, sampV, Bold,
                     Bnew);
  KCHK();
}

__global__ __launch_bounds__(256) void k_node_nn(const Node* nodes, const int32_t* list, int K,
                                                 int N, const double* A, int64_t lda,
                                                 const double* Bn, int64_t bstride, int64_t ldb,
                                                 double* out, int64_t ldo, int from_sibling) {
  __shared__ double smem[tile_smem_elems<STM, STN>()];
  const int g = list[blockIdx.y];
  const int gb = from_sibling ? nodes[g].sib : g;
  const Node nd = nodes[g];
  const int64_t i0 = nd.lo + (int64_t)blockIdx.x * STM;
  if (i0 >= nd.hi) return;
  const int M = (int)min<int64_t>(STM, nd.hi - i0);
  const int j0 = blockIdx.z * STN;
  TileAcc<double, STM, STN> acc;
  acc.zero();
  mm_tile<double, STM, STN>(M, N - j0, K, A + i0, 1, lda, Bn + (int64_t)gb * bstride + j0 * ldb,
                            1, ldb, acc, smem);
  store_tile<double, STM, STN>(M, N - j0, out + i0 + (int64_t)j0 * ldo, ldo, acc, 1.0, 0.0);
}

void launch_node_nn(const Node* nodes, const int32_t* list, int nlist, int64_t max_rows, int K,
                    int N, const double* A, int64_t lda, const double* Bn, int64_t bstride,
                    int64_t ldb, double* out, int64_t ldo, hipStream_t s, int from_sibling) {
  if (nlist <= 0 || N <= 0) return;
  hipLaunchKernelGGL(k_node_nn,
                     dim3((unsigned)((max_rows + STM - 1) / STM), nlist, (N + STN - 1) / STN),
                     dim3(256), 0, s, nodes, list, K, N, A, lda, Bn, bstride, ldb, out, ldo,
                     from_sibling);
  KCHK();
}

__global__ void k_truncate(const Node* nodes, const Instance* inst, const int32_t* kids, int R,
                           double* Vl, int64_t ldv, double* sv, double* X, int32_t* rank,
                           int32_t* saturated) {
  const int v = kids[blockIdx.y];
  const Node nd = nodes[v];
  const Instance in = inst[nd.inst];
  const double* s = sv + (int64_t)v * R;
  int k = min(in.k, in.r);
  if (in.tol > 0.0) {
    int kk = 0;
    for (int j = 0; j < in.r; ++j) kk += (s[0] > 0.0 && s[j] > in.tol * s[0]);
    k = min(kk, k);
  }
  const int64_t i = nd.lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < nd.hi)
    for (int j = k; j < R; ++j) Vl[i + (int64_t)j * ldv] = 0.0;
  if (blockIdx.x == 0) {
    __syncthreads();
    double* Xv = X + (int64_t)v * 2 * R * R;
    for (int e = threadIdx.x; e < 2 * R * R; e += blockDim.x)
      if (e / (2 * R) >= k) Xv[e] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int j = k; j < R; ++j) sv[(int64_t)v * R + j] = 0.0;
      rank[v] = k;
      if (in.tol > 0.0 && k >= in.r - in.p && saturated) atomicAdd(saturated, 1);
    }
  }
}

void launch_truncate(const Node* nodes, const Instance* inst, const int32_t* kids, int nkids,
                     int64_t max_rows, int R, double* Vl, int64_t ldv, double* sv, double* X,
                     int32_t* rank, int32_t* saturated, hipStream_t s) {
  if (nkids <= 0) return;
  const int nt = 256;
  hipLaunchKernelGGL(k_truncate, dim3((unsigned)((max_rows + nt - 1) / nt), nkids), dim3(nt), 0,
                     s, nodes, inst, kids, R, Vl, ldv, sv, X, rank, saturated);
  KCHK();
}

}  // namespace hm
