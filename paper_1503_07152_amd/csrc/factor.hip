// Node factorisations: TSQR panels, reflector application, Jacobi SVD,
// node-block gather, interaction matrices, column-pivoted QR / ID.
#include <cfloat>

#include "factor.h"
#include "tile.h"
#include "tile_mfma.h"

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
// Blocked Householder QR (compact WY form, Schreiber-Van Loan) of one panel
// of <= 192 x 96 held in LDS; strips of QR_NB = 16 columns.
//
// Strip factorisation: wave w keeps strip column j0 + w in registers (rows
// lane + 64 t), reduces over the column with DPP / permlane operations, and
// publishes its reflector into the panel in LDS; the other strip waves apply
// it to their columns (and the earlier ones form the V^T V entries of T).
// One barrier per column; the columns of T (H_j0 ... H_j0+15 = I - V T V^T,
// T upper triangular) are formed one iteration behind.  Then the trailing
// update A <- A - V T^T (V^T A) on FP64 MFMA 16x16x4, two to sixteen waves per
// 16-column tile of the trailing block.
//
// Outputs: reflectors below the diagonal (v_j(j) = 1 implied), R on and
// above, tau_j, the T factor of every strip (QR_NB x QR_NB, row-major by
// strip: T + strip * QR_NB * QR_NB, entry (i, c) at i * QR_NB + c), and R.

typedef double d4 __attribute__((ext_vector_type(4)));

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
// sum over the whole wave, the same value in every lane: rows by sum16, then
// the gfx950 row swaps (rows 0<->1, 2<->3, then halves)
__device__ __forceinline__ double sum64(double v) {
  v = sum16(v);
  {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
    v = __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
  }
  {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
    v = __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
  }
  return v;
}

constexpr int QR_RT = FAC_PMAX / 64;  // row slots per lane

__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// 1/a from the hardware estimate and two Newton steps in residual form
// (e = 1 - a r, r += r e): within an ulp or two for normal a
__device__ __forceinline__ double recip_nr(double a) {
  double r = __builtin_amdgcn_rcp(a);
#pragma unroll
  for (int it = 0; it < 2; ++it) r = fma(r, fma(-a, r, 1.0), r);
  return r;
}

// Householder scalars for the column with diagonal x0 and squared norm sig
// below it: beta = -sign(x0) sqrt(x0^2 + sig), tau = (beta - x0) / beta,
// scl = 1 / (x0 - beta).  The square root and reciprocals come from hardware
// estimates refined by Newton steps (a short dependency chain); outside the
// range where the estimates are safe, IEEE operations are used.
__device__ __forceinline__ void householder_scalars(double x0, double sig, double& beta,
                                                    double& tau, double& scl) {
  const double q = fma(x0, x0, sig);
  if (q > 1e-290 && q < 1e290) {
    double r = __builtin_amdgcn_rsq(q);          // 1/sqrt(q)
#pragma unroll
    for (int it = 0; it < 2; ++it) r = fma(r, fma(-0.5 * q * r, r, 0.5), r);
    double nrm = q * r;
    nrm = fma(0.5 * r, fma(-nrm, nrm, q), nrm);  // one Newton step on sqrt(q)
    beta = -copysign(nrm, x0);
    const double d1 = x0 - beta;                 // |x0| + nrm in magnitude: no cancellation
    scl = recip_nr(d1);
    tau = -d1 * recip_nr(beta);
  } else {
    beta = -copysign(sqrt(q), x0);
    tau = (beta - x0) / beta;
    scl = 1.0 / (x0 - beta);
  }
}

// Column c of the compact WY factor (Schreiber-Van Loan): T(c, c) = tau_c,
// T(i, c) = -tau_c sum_{l = i}^{c-1} T(i, l) (v_l^T v_c) for i < c, zero below;
// lane i of the calling wave writes row i.
__device__ __forceinline__ void t_column(double (*sT)[QR_NB + 1], const double (*sVV)[QR_NB + 1],
                                         const double* sTau, int c, int lane) {
  if (lane >= QR_NB) return;
  double acc = 0.0;
#pragma unroll
  for (int l = 0; l < QR_NB - 1; ++l)
    if (l >= lane && l < c) acc = fma(sT[lane][l], sVV[l][c], acc);
  const double tc = sTau[c];
  sT[lane][c] = lane == c ? tc : (lane < c ? -tc * acc : 0.0);
}

__global__ __launch_bounds__(FT) void k_panel_qr(const PanelDesc* descs) {
  __shared__ double sA[FAC_LDMAX * FAC_CMAX];
  __shared__ double sTau[QR_NB];
  __shared__ double sVV[QR_NB][QR_NB + 1];
  __shared__ double sT[QR_NB][QR_NB + 1];
  const PanelDesc d = descs[blockIdx.x];
  const int m = d.rows, n = d.dyn_cols ? max(0, min(d.cols, *d.dyn_cols)) : d.cols;
  const int lds = (m & 1) ? m : m + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int idx = tid; idx < m * n; idx += FT) {
    const int i = idx % m, j = idx / m;
    sA[i + j * lds] = d.trans ? d.A[j + (int64_t)i * d.ld] : d.A[i + (int64_t)j * d.ld];
  }
  __syncthreads();
  const int h = min(m, n);
  // V(r, j) of the stored panel: 1 on the diagonal, 0 above, LDS below
  auto vget = [&](int r, int j) -> double {
    const double x = sA[min(r, m - 1) + j * lds];
    return r == j ? 1.0 : (r > j && r < m ? x : 0.0);
  };
  for (int j0 = 0; j0 < h; j0 += QR_NB) {
    const int nbs = min(QR_NB, h - j0);
    // ---- strip factorisation ------------------------------------------------
    double x[QR_RT];
    const bool mine = wave < nbs;
    const int cw = j0 + wave;
#pragma unroll
    for (int t = 0; t < QR_RT; ++t) {
      const int r = lane + 64 * t;
      x[t] = (mine && r < m) ? sA[r + cw * lds] : 0.0;
    }
    for (int jj = 0; jj < nbs; ++jj) {
      const int j = j0 + jj;
      if (wave == jj) {
        double s2 = 0.0, xj = 0.0;
#pragma unroll
        for (int t = 0; t < QR_RT; ++t) {
          const int r = lane + 64 * t;
          s2 = (r > j) ? fma(x[t], x[t], s2) : s2;   // rows >= m hold zero
          xj = (t == (j >> 6)) ? x[t] : xj;
        }
        const double x0 = readlane_d(xj, j & 63);   // A(j, j), from the lane holding row j
        const double sig = sum64(s2);
        double beta = x0, tau = 0.0, scl = 0.0;
        if (sig != 0.0) householder_scalars(x0, sig, beta, tau, scl);
#pragma unroll
        for (int t = 0; t < QR_RT; ++t) {
          const int r = lane + 64 * t;
          const double nv = r < j ? x[t] : (r == j ? beta : x[t] * scl);
          if (r < m) sA[r + j * lds] = nv;
          x[t] = r == j ? 1.0 : (r > j ? x[t] * scl : 0.0);   // keep v_j
        }
        if (lane == 0) {
          sTau[jj] = tau;
          d.tau[j] = tau;
        }
      }
      __syncthreads();
      if (mine && wave != jj) {
        double vj[QR_RT];
#pragma unroll
        for (int t = 0; t < QR_RT; ++t) vj[t] = vget(lane + 64 * t, j);
        double p = 0.0;
#pragma unroll
        for (int t = 0; t < QR_RT; ++t) p = fma(vj[t], x[t], p);
        p = sum64(p);
        if (wave > jj) {
          // apply H_j to this wave's column
          const double tp = sTau[jj] * p;
#pragma unroll
          for (int t = 0; t < QR_RT; ++t) x[t] = fma(-tp, vj[t], x[t]);
        } else if (lane == 0) {
          sVV[wave][jj] = p;   // v_wave^T v_j (x holds v_wave)
        }
      }
      // T column jj - 1 (its V^T v entries and the earlier columns are final)
      if (jj >= 1 && wave == jj - 1) t_column(sT, sVV, sTau, jj - 1, lane);
    }
    __syncthreads();
    if (wave == 0) {
      t_column(sT, sVV, sTau, nbs - 1, lane);
      if (lane < QR_NB)
#pragma unroll
        for (int c = nbs; c < QR_NB; ++c) sT[lane][c] = 0.0;
    }
    __syncthreads();
    if (d.T && tid < QR_NB * QR_NB)
      d.T[(int64_t)(j0 / QR_NB) * QR_NB * QR_NB + tid] = sT[tid / QR_NB][tid % QR_NB];
    // ---- trailing update A <- A - V T^T (V^T A), columns j0 + nbs .. n-1 ------------
    // FW / tiles waves per 16-column tile: each forms the whole W = V^T A(:, tile)
    // (two accumulators, operands loaded four K-steps ahead), then updates
    // its share of the 16-row tiles.
    const int ntile = (n - j0 - nbs + 15) / 16;   // <= 6
    const int wpt = ntile > 0 ? max(1, FW / ntile) : FW;   // waves per tile
    const int tile = wave / wpt, sub = wave % wpt;
    const int c0 = j0 + nbs + 16 * tile;
    const bool active = tile < ntile;
    const int cl = c0 + (lane & 15);
    const int clc = min(cl, n - 1);
    const int kq = lane >> 4;
    const int bl = lane & 15;
    d4 w2 = {0.0, 0.0, 0.0, 0.0};
    if (active) {
      const int nks = (m - j0 + 3) / 4;      // 4-row K-steps over rows j0 .. m-1
      // W = V^T A(rows, tile): A-operand V^T(i = lane % 16, k), B-operand A(k, j = lane % 16)
      d4 w0 = {0.0, 0.0, 0.0, 0.0}, w1 = {0.0, 0.0, 0.0, 0.0};
      for (int s = 0; s < nks; s += 4) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = j0 + 4 * (s + u) + kq;
          a[u] = bl < nbs ? vget(r, j0 + bl) : 0.0;
          const double x = sA[min(r, m - 1) + clc * lds];
          b[u] = (r < m && cl < n) ? x : 0.0;
        }
        w0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], w0, 0, 0, 0);
        w1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], w1, 0, 0, 0);
        w0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2], b[2], w0, 0, 0, 0);
        w1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3], b[3], w1, 0, 0, 0);
      }
      const d4 w = w0 + w1;
      // W2 = T^T W: A-operand T^T(i, k) = T(k, i); the B-operand of step s is w[s]
#pragma unroll
      for (int s = 0; s < 4; ++s)
        w2 = __builtin_amdgcn_mfma_f64_16x16x4f64(sT[4 * s + kq][bl], w[s], w2, 0, 0, 0);
    }
    __syncthreads();   // every W is formed before any tile changes
    if (active) {
      // A(rows, tile) -= V W2 on this wave's 16-row tiles; A-operand V(i, k = 4 s + lane / 16)
      const int nrt = (m - j0 + 15) / 16;
      for (int rt = sub; rt < nrt; rt += wpt) {
        const int rb = j0 + 16 * rt;
        double a[4], c[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int b = 4 * s + kq;
          a[s] = b < nbs ? vget(rb + bl, j0 + b) : 0.0;
          c[s] = sA[min(rb + kq + 4 * s, m - 1) + clc * lds];
        }
        d4 u = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) u = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], w2[s], u, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = rb + kq + 4 * v;
          if (r < m && cl < n) sA[r + cl * lds] = c[v] - u[v];
        }
      }
    }
    __syncthreads();
  }
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

// Cout = H_0 H_1 ... H_{h-1} [Cin; 0] = (I - V_0 T_0 V_0^T) ... [Cin; 0], the
// strips applied last to first.  One wave per 16-column tile of C, which stays
// in MFMA accumulator registers (row tile rt, item v of lane l = row
// 16 rt + l/16 + 4 v, column l % 16): W = V_b^T C (the B-operand of K-step s is
// item s % 4 of row tile s / 4), W2 = T_b W, C -= V_b W2.  Each strip's
// reflectors (unit diagonal and zeros made explicit) and T_b are staged in LDS
// by the whole workgroup.
constexpr int APQ_NMAX = HM_MAX_SAMPLES;
constexpr int APQ_WAVES = 4;
__global__ __launch_bounds__(64 * APQ_WAVES) void k_apply_q(const PanelDesc* descs, int tiles) {
  __shared__ double sV[FAC_PMAX * QR_NB];
  __shared__ double sTb[QR_NB * QR_NB];
  const PanelDesc d = descs[blockIdx.x / tiles];
  const int tile = (blockIdx.x % tiles) * APQ_WAVES + (threadIdx.x >> 6);
  const int ncols = d.dyn_cols ? max(0, min(d.cols, *d.dyn_cols)) : d.cols;
  const int m = d.rows, h = min(d.rows, ncols), nc = d.ncol;
  const int hin = d.cin_full ? m : h;   // rows of Cin
  const int tid = threadIdx.x, lane = tid & 63, kq = lane >> 4, bl = lane & 15;
  const int cl = 16 * tile + bl;
  const bool act = 16 * tile < nc;
  d4 cacc[FAC_PMAX / 16];
#pragma unroll
  for (int rt = 0; rt < FAC_PMAX / 16; ++rt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * rt + kq + 4 * v;
      cacc[rt][v] = (act && r < hin && cl < nc) ? d.Cin[r + (int64_t)cl * d.ldCin] : 0.0;
    }
  auto vs = [&](int r, int b) -> double { return r < m ? sV[r + b * FAC_PMAX] : 0.0; };
  const int nstrips = (h + QR_NB - 1) / QR_NB;
  for (int sb = nstrips - 1; sb >= 0; --sb) {
    const int j0 = sb * QR_NB;
    const int rt0 = j0 / 16;
    __syncthreads();   // the previous strip's operands are consumed
    for (int idx = tid; idx < m * QR_NB; idx += 64 * APQ_WAVES) {
      const int r = idx % m, b = idx / m, j = j0 + b;
      double v = 0.0;
      if (j < h && r >= j) v = r == j ? 1.0 : d.A[r + (int64_t)j * d.ld];
      sV[r + b * FAC_PMAX] = v;
    }
    sTb[tid] = d.T[(int64_t)sb * QR_NB * QR_NB + tid];
    __syncthreads();
    if (!act) continue;
    // W = V_b^T C over rows j0 .. m-1
    d4 w0 = {0.0, 0.0, 0.0, 0.0}, w1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int rt = 0; rt < FAC_PMAX / 16; ++rt) {
      if (rt >= rt0 && 16 * rt < m) {
        double a[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) a[v] = vs(16 * rt + 4 * v + kq, bl);
        w0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], cacc[rt][0], w0, 0, 0, 0);
        w1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], cacc[rt][1], w1, 0, 0, 0);
        w0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2], cacc[rt][2], w0, 0, 0, 0);
        w1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3], cacc[rt][3], w1, 0, 0, 0);
      }
    }
    const d4 w = w0 + w1;
    // W2 = T_b W
    d4 w2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s)
      w2 = __builtin_amdgcn_mfma_f64_16x16x4f64(sTb[bl * QR_NB + 4 * s + kq], w[s], w2, 0, 0, 0);
    // C -= V_b W2
#pragma unroll
    for (int rt = 0; rt < FAC_PMAX / 16; ++rt) {
      if (rt >= rt0 && 16 * rt < m) {
        double a[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) a[s] = vs(16 * rt + bl, 4 * s + kq);
        d4 u = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) u = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], w2[s], u, 0, 0, 0);
        cacc[rt] -= u;
      }
    }
  }
  if (!act) return;
#pragma unroll
  for (int rt = 0; rt < FAC_PMAX / 16; ++rt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * rt + kq + 4 * v;
      if (r < m && cl < nc) d.Cout[(d.perm ? d.perm[r] : r) + (int64_t)cl * d.ldCout] = cacc[rt][v];
    }
}

void launch_apply_q(const PanelDesc* d, int n, hipStream_t s) {
  if (n <= 0) return;
  const int tiles = (APQ_NMAX + 16 * APQ_WAVES - 1) / (16 * APQ_WAVES);
  hipLaunchKernelGGL(k_apply_q, dim3(n * tiles), dim3(64 * APQ_WAVES), 0, s, d, tiles);
  KCHK();
}

// ------------------------------------------------------------ pivoted QR --
// Householder QR with column pivoting (Businger-Golub) of A = R^T, c x h <= 96
// x 96 in LDS, stopped at the numerical rank: a step whose largest remaining
// squared column norm is <= (max(c, h) eps)^2 times the largest initial one
// ends the factorisation, and the trailing block (below that threshold) is
// dropped.  Column swaps are logical (a column map in LDS); remaining column
// norms are recomputed exactly at every step, so no downdating is involved.
// One barrier per step between the reflector (wave 0) and its application to
// the trailing columns (all waves, one column per wave at a time), one after.
constexpr int QP_LD = FAC_CMAX + 1;
constexpr int QP_RPL = FAC_CMAX / 16;   // rows per lane of a 16-lane group

__device__ __forceinline__ double max64(double v) {
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  v = fmax(v, dpp_d<0x140>(v));
  {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
    v = fmax(__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1]));
  }
  {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
    v = fmax(__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1]));
  }
  return v;
}

__global__ __launch_bounds__(FT) void k_qrcp(const QrcpDesc* descs) {
  __shared__ double sA[QP_LD * FAC_CMAX];
  __shared__ double snrm[FAC_CMAX];
  __shared__ int scol[FAC_CMAX];
  __shared__ double sTau[FAC_CMAX];
  __shared__ double sVV[QR_TMAX][QR_NB][QR_NB + 1];
  __shared__ double sT[QR_TMAX][QR_NB][QR_NB + 1];
  const QrcpDesc d = descs[blockIdx.x];
  const int c = d.c, h = d.h;   // A = R^T: c rows, h columns
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int idx = tid; idx < c * h; idx += FT) {
    const int i = idx % c, j = idx / c;
    sA[i + j * QP_LD] = d.R[j + (int64_t)i * d.ldR];
  }
  for (int j = tid; j < h; j += FT) scol[j] = j;
  __syncthreads();
  for (int j = wave; j < h; j += FW) {
    double s2 = 0.0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int r = lane + 64 * t;
      const double a = r < c ? sA[r + j * QP_LD] : 0.0;
      s2 = fma(a, a, s2);
    }
    s2 = sum64(s2);
    if (lane == 0) snrm[j] = s2;
  }
  __syncthreads();
  const int kmax = min(c, h);
  const double eta = d.eta > 0.0 ? d.eta : (double)max(c, h) * DBL_EPSILON;
  double thr2 = 0.0;
  int rho = kmax;
  for (int k = 0; k < kmax; ++k) {
    // pivot: the largest remaining squared norm, the lowest index on ties
    // (every wave finds the same one)
    const int j1 = k + lane, j2 = k + lane + 64;
    const double v1 = j1 < h ? snrm[j1] : -1.0;
    const double v2 = j2 < h ? snrm[j2] : -1.0;
    const double vmax = max64(fmax(v1, v2));
    const uint64_t m1 = __ballot(v1 == vmax), m2 = __ballot(v2 == vmax);
    const int p = m1 ? k + __ffsll((unsigned long long)m1) - 1
                     : k + 64 + __ffsll((unsigned long long)m2) - 1;
    if (k == 0) thr2 = eta * eta * vmax;
    if (!(vmax > 0.0) || (k >= d.kmin && !(vmax > thr2))) {   // numerical rank reached
      rho = k;
      break;
    }
    const int pk = scol[p], pp = scol[k];   // physical columns entering positions k and p
    if (wave == 0) {
      double x[2], s2 = 0.0, xk = 0.0;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int r = lane + 64 * t;
        x[t] = r < c ? sA[r + pk * QP_LD] : 0.0;
        s2 = r > k ? fma(x[t], x[t], s2) : s2;
        xk = t == (k >> 6) ? x[t] : xk;
      }
      const double x0 = readlane_d(xk, k & 63);
      const double sig = sum64(s2);
      double beta = x0, tau = 0.0, scl = 0.0;
      if (sig != 0.0) householder_scalars(x0, sig, beta, tau, scl);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int r = lane + 64 * t;
        if (r == k) sA[r + pk * QP_LD] = beta;
        else if (r > k && r < c) sA[r + pk * QP_LD] = x[t] * scl;
      }
      if (lane == 0) sTau[k] = tau;
    }
    __syncthreads();
    if (tid == 0) {
      scol[k] = pk;
      scol[p] = pp;
    }
    // trailing columns: a 16-lane group per column, QP_RPL rows per lane
    const double tk = sTau[k];
    const int grp = tid >> 4, gl = tid & 15;
    if (k + 1 + grp < h) {
      double v[QP_RPL];
#pragma unroll
      for (int u = 0; u < QP_RPL; ++u) {
        const int r = gl + 16 * u;
        v[u] = r == k ? 1.0 : ((r > k && r < c) ? sA[r + pk * QP_LD] : 0.0);
      }
      for (int j = k + 1 + grp; j < h; j += FT / 16) {
        const int pj = j == p ? pp : scol[j];   // scol[p] is being rewritten
        double a[QP_RPL], w = 0.0;
#pragma unroll
        for (int u = 0; u < QP_RPL; ++u) {
          const int r = gl + 16 * u;
          a[u] = (r >= k && r < c) ? sA[r + pj * QP_LD] : 0.0;
          w = fma(v[u], a[u], w);
        }
        const double tw = tk * sum16(w);
        double n2 = 0.0;
#pragma unroll
        for (int u = 0; u < QP_RPL; ++u) {
          const int r = gl + 16 * u;
          a[u] = fma(-tw, v[u], a[u]);
          if (r >= k && r < c) sA[r + pj * QP_LD] = a[u];
          n2 = r > k ? fma(a[u], a[u], n2) : n2;
        }
        n2 = sum16(n2);
        if (gl == 0) snrm[j] = n2;
      }
    }
    __syncthreads();
  }
  __syncthreads();
  // V^T V inside each strip of QR_NB reflectors, then the strip's T factor
  const int nstr = (rho + QR_NB - 1) / QR_NB;
  for (int e = wave; e < nstr * QR_NB * QR_NB; e += FW) {
    const int b = e / (QR_NB * QR_NB), i = (e / QR_NB) % QR_NB, cc = e % QR_NB;
    const int gi = QR_NB * b + i, gc = QR_NB * b + cc;
    if (i >= cc || gc >= rho) continue;
    const int ci = scol[gi], cj = scol[gc];
    double s2 = 0.0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int r = lane + 64 * t;
      const double vi = r == gi ? 1.0 : ((r > gi && r < c) ? sA[r + ci * QP_LD] : 0.0);
      const double vc = r == gc ? 1.0 : ((r > gc && r < c) ? sA[r + cj * QP_LD] : 0.0);
      s2 = fma(vi, vc, s2);
    }
    s2 = sum64(s2);
    if (lane == 0) sVV[b][i][cc] = s2;
  }
  __syncthreads();
  if (wave < nstr) {
    const int nbs = min(QR_NB, rho - QR_NB * wave);
    for (int cc = 0; cc < nbs; ++cc) t_column(sT[wave], sVV[wave], sTau + QR_NB * wave, cc, lane);
    if (lane < QR_NB)
      for (int cc = nbs; cc < QR_NB; ++cc) sT[wave][lane][cc] = 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < nstr * QR_NB * QR_NB; idx += FT)
    d.T[idx] = sT[idx / (QR_NB * QR_NB)][(idx / QR_NB) % QR_NB][idx % QR_NB];
  for (int j = tid; j < h; j += FT) d.perm[j] = scol[j];
  if (tid == 0) *d.rho = rho;
  for (int k = tid; k < rho; k += FT) d.tau[k] = sTau[k];
  for (int idx = tid; idx < rho * h; idx += FT) {
    const int k = idx % rho, j = idx / rho;
    d.R2[k + (int64_t)j * d.ldR2] = j >= k ? sA[k + scol[j] * QP_LD] : 0.0;
  }
  // reflectors in pivoted order over the input (read into LDS above)
  for (int idx = tid; idx < c * rho; idx += FT) {
    const int r = idx % c, k = idx / c;
    if (r > k) d.R[r + (int64_t)k * d.ldR] = sA[r + scol[k] * QP_LD];
  }
}

void launch_qrcp(const QrcpDesc* d, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_qrcp, dim3(n), dim3(FT), 0, s, d);
  KCHK();
}

// ------------------------------------------------------------ pivoted Cholesky --
// Diagonal-pivoted Cholesky of a c x c PSD matrix (the Gram matrix of a node
// block), stopped at the numerical rank; one step per column.  The matrix
// stays in registers in its original (physical) order: thread (tx, ty) of the
// 32 x 32 workgroup holds entries (tx + 32 a, ty + 32 b), a, b < 3.  Swaps are
// logical (a map in LDS).  Per step every wave finds the pivot (largest
// remaining diagonal, lowest logical index on ties), the threads holding the
// pivot column publish it scaled by 1 / l_kk, zero on rows already pivoted,
// and every thread applies the rank-one Schur update to its nine entries
// (rows already pivoted see a zero factor and keep their values).
__global__ __launch_bounds__(FT) void k_pchol(const PcholDesc* descs) {
  static_assert(FT == 1024 && FAC_CMAX <= 96, "32 x 32 threads, 3 x 3 entries each");
  __shared__ double sStage[QP_LD * FAC_CMAX];   // final row permutation of L
  __shared__ double sdg[FAC_CMAX];              // diagonal, physical order
  __shared__ double sl[FAC_CMAX];               // scaled pivot column, physical order
  __shared__ int scol[FAC_CMAX];                // logical -> physical
  __shared__ int sact[FAC_CMAX];                // physical index not yet pivoted
  const PcholDesc d = descs[blockIdx.x];
  const int c = d.c;
  const int tid = threadIdx.x, lane = tid & 63;
  const int tx = tid & 31, ty = tid >> 5;
  double g[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int pi = tx + 32 * a, pj = ty + 32 * b;
      g[a][b] = (pi < c && pj < c) ? d.G[pi + (int64_t)pj * d.ldG] : 0.0;
    }
  for (int j = tid; j < c; j += FT) {
    scol[j] = j;
    sact[j] = 1;
    sdg[j] = d.G[j + (int64_t)j * d.ldG];
  }
  __syncthreads();
  double thr = 0.0, thr_short = 0.0;
  int rho = c;
  for (int k = 0; k < c; ++k) {
    const int j1 = k + lane, j2 = k + lane + 64;
    const double v1 = j1 < c ? sdg[scol[j1]] : -1.0;
    const double v2 = j2 < c ? sdg[scol[j2]] : -1.0;
    const double vmax = max64(fmax(v1, v2));
    const uint64_t m1 = __ballot(v1 == vmax), m2 = __ballot(v2 == vmax);
    const int p = m1 ? k + __ffsll((unsigned long long)m1) - 1
                     : k + 64 + __ffsll((unsigned long long)m2) - 1;
    if (k == 0) {
      thr = d.eta * d.eta * vmax;
      thr_short = d.tau * d.tau * vmax;
    }
    if (k < d.kneed && !(vmax > thr_short)) {   // not resolvable: the caller falls back
      if (tid == 0) atomicOr(d.short_flag, 1);
      rho = k;
      break;
    }
    if (k >= d.kneed && !(vmax > thr)) {
      rho = k;
      break;
    }
    const int pk = scol[p], pp = scol[k];
    const double lkk = sqrt(vmax);
    const double inv = 1.0 / lkk;
    // the pivot column, scaled, on the rows still to be pivoted
    if (ty == (pk & 31)) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int pi = tx + 32 * a;
        double gv = 0.0;
#pragma unroll
        for (int b = 0; b < 3; ++b)
          if (b == (pk >> 5)) gv = g[a][b];
        if (pi < c) sl[pi] = (sact[pi] && pi != pk) ? gv * inv : 0.0;
      }
    }
    __syncthreads();
    if (tid == 0) {
      scol[k] = pk;
      scol[p] = pp;
      sact[pk] = 0;
    }
    // column k of L by physical row (the rows are put in pivot order at the end)
    for (int i = tid; i < c; i += FT) d.L[i + (int64_t)k * d.ldL] = i == pk ? lkk : sl[i];
    // Schur complement: g(i, j) -= l_i l_j (zero factor on pivoted rows)
    double li[3], lj[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      li[a] = tx + 32 * a < c ? sl[tx + 32 * a] : 0.0;
      lj[a] = ty + 32 * a < c ? sl[ty + 32 * a] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        g[a][b] = fma(-li[a], lj[b], g[a][b]);
        if (tx + 32 * a == ty + 32 * b && tx + 32 * a < c) sdg[tx + 32 * a] = g[a][b];
      }
    __syncthreads();
  }
  __syncthreads();
  // rows of L into the final pivoted order (through LDS)
  for (int e = tid; e < c * rho; e += FT) {
    const int i = e % c, k = e / c;
    sStage[i + k * QP_LD] = d.L[scol[i] + (int64_t)k * d.ldL];
  }
  __syncthreads();
  for (int e = tid; e < c * rho; e += FT) {
    const int i = e % c, k = e / c;
    d.L[i + (int64_t)k * d.ldL] = sStage[i + k * QP_LD];
  }
  for (int i = tid; i < c; i += FT) d.perm[i] = scol[i];
  if (tid == 0) *d.rho = rho;
}

void launch_pchol(const PcholDesc* d, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pchol, dim3(n), dim3(FT), 0, s, d);
  KCHK();
}

// ------------------------------------------------------------ Jacobi SVD --
// One-sided (Hestenes) Jacobi on the columns of an h x c matrix T (T = R, or
// T = R^T when the descriptor asks for the transpose): T Z = W diag(s).  Pairs
// follow a round-robin tournament; each 16-lane group rotates one pair, so a
// 1024-thread workgroup treats every pair of a round (c <= 96) at once.  The
// squared column norms are kept in LDS: computed at the start of each sweep
// and, after a rotation by t = tan(theta), updated as |x|^2 - t g and
// |y|^2 + t g (g = x.y; exact for the t that zeroes the pair's inner
// product), so a pair needs only its inner product, reduced across the group
// by DPP row operations (no LDS round trip).  Each lane holds RPL = ceil(h /
// 16) rows of the pair in registers.
constexpr int JAC_LD = FAC_CMAX + 1;
constexpr int JAC_G = 16;                      // lanes per pair
constexpr int JAC_FT = FT;
constexpr int JAC_RPL = FAC_CMAX / JAC_G;      // most rows per lane
static_assert(JAC_FT / JAC_G >= FAC_CMAX / 2, "one group per pair of a round");

// JFT threads: JFT / 16 groups, each taking the pairs grp, grp + JFT / 16, ..
// of a round in turn (the pairs of a round are disjoint)
// A pair is rotated while |x.y| > tol |x| |y|.  With stop > 0 the sweeps also
// end after a sweep in which no pair had |x.y| > stop |x| |y|: cyclic Jacobi
// converges quadratically, so the next sweep would start from inner products
// of order stop^2 (the check sweep that finds no rotation is saved).
template <int RPL, int JFT>
__device__ __forceinline__ int jacobi_sweeps(double* sA, double* sZ, double* sN, int h, int c,
                                             bool wantX, int* flag, double tol, double stop) {
  constexpr int JAC_GROUPS = JFT / JAC_G;
  const int tid = threadIdx.x;
  const int grp = tid / JAC_G, gl = tid % JAC_G;
  const int n2 = c + (c & 1);
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    if (tid == 0) flag[0] = flag[1] = 0;
    // squared column norms, fresh each sweep (the updates drift by rounding)
    for (int j = grp; j < c; j += JAC_GROUPS) {
      double nn = 0.0;
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const double v = sA[gl + JAC_G * u + j * JAC_LD];
        nn = fma(v, v, nn);
      }
      nn = sum16(nn);
      if (gl == 0) sN[j] = nn;
    }
    __syncthreads();
    for (int t = 0; t < n2 - 1; ++t) {
      for (int pi = grp; pi < n2 / 2; pi += JAC_GROUPS) {
        const int a = pi, b = n2 - 1 - pi;
        // tournament positions 1 + (a - 1 + t) mod (n2 - 1), a - 1 + t < 2 (n2 - 1)
        int xa = a - 1 + t, xb = b - 1 + t;
        if (xa >= n2 - 1) xa -= n2 - 1;
        if (xb >= n2 - 1) xb -= n2 - 1;
        const int pa = a == 0 ? 0 : 1 + xa;
        const int pb = b == 0 ? 0 : 1 + xb;
        const int p = min(pa, pb), q = max(pa, pb);
        if (q >= c) continue;
        // the group's rows gl + 16 u (fixed trip count; rows h .. 16 RPL - 1
        // hold zeros, which the rotations keep)
        double xv[RPL], yv[RPL];
        double ga = 0.0;
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
          const int i = gl + JAC_G * u;
          xv[u] = sA[i + p * JAC_LD];
          yv[u] = sA[i + q * JAC_LD];
          ga = fma(xv[u], yv[u], ga);
        }
        ga = sum16(ga);
        const double al = sN[p], be = sN[q];
        // |ga| > tol |x| |y|, from the hardware reciprocal square roots (a
        // threshold needs no correct rounding)
        const double ratio = (ga != 0.0 && al > 0.0 && be > 0.0)
                                 ? fabs(ga) * __builtin_amdgcn_rsq(al) * __builtin_amdgcn_rsq(be)
                                 : 0.0;
        if (ratio > stop && stop > 0.0 && gl == 0) flag[1] = 1;
        if (ratio > tol) {
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
          for (int u = 0; u < RPL; ++u) {
            const int i = gl + JAC_G * u;
            sA[i + p * JAC_LD] = cs * xv[u] - sn * yv[u];
            sA[i + q * JAC_LD] = sn * xv[u] + cs * yv[u];
          }
          if (wantX) {
            // rows of Z: c <= JAC_G JAC_RPL
#pragma unroll
            for (int u = 0; u < JAC_RPL; ++u) {
              const int i = gl + JAC_G * u;
              if (JAC_G * u < c) {
                const int ic = min(i, c - 1);
                const double x = sZ[ic + p * JAC_LD], y = sZ[ic + q * JAC_LD];
                if (i < c) {
                  sZ[i + p * JAC_LD] = cs * x - sn * y;
                  sZ[i + q * JAC_LD] = sn * x + cs * y;
                }
              }
            }
          }
          if (gl == 0) {
            sN[p] = fma(-tt, ga, al);
            sN[q] = fma(tt, ga, be);
            flag[0] = 1;
          }
        }
      }
      __syncthreads();
    }
    if (flag[0] == 0 || (stop > 0.0 && flag[1] == 0)) break;
    __syncthreads();  // every thread has read the flags before they are reset
  }
  return sweep + 1;
}

// NEED_Z: the descriptors may accumulate rotations or form T^T W (a second
// LDS matrix); without it (the Gram route) a workgroup takes half the LDS and
// 512 threads (pairs beyond 32 in a second pass per round), so that two
// workgroups fit a CU: the leaf level has more nodes than the GPU has CUs.
template <bool NEED_Z>
constexpr int jacobi_threads() { return NEED_Z ? JAC_FT : JAC_FT / 2; }

template <bool NEED_Z>
__global__ __launch_bounds__(jacobi_threads<NEED_Z>()) void k_jacobi(const SvdDesc* descs) {
  constexpr int JFT = jacobi_threads<NEED_Z>();
  __shared__ double sA[FAC_CMAX * JAC_LD];
  __shared__ double sZ[NEED_Z ? FAC_CMAX * JAC_LD : 1];
  __shared__ double snorm[FAC_CMAX];
  __shared__ double sN[FAC_CMAX];
  __shared__ int srank[FAC_CMAX];
  __shared__ int flag[2];
  const SvdDesc d = descs[blockIdx.x];
  int h = d.h, c = d.c;
  if (d.dyn) {
    const int r = max(0, min(d.c, *d.dyn));
    if (!d.gram) h = min(h, r);
    c = r;
  }
  const bool wantX = d.X != nullptr;
  const bool accZ = NEED_Z && wantX && !d.xscaled && !d.gram;   // accumulate the rotations
  const int tid = threadIdx.x;
  for (int idx = tid; idx < h * c; idx += JFT) {
    const int i = idx % h, j = idx / h;
    sA[i + j * JAC_LD] = d.trans ? d.R[j + (int64_t)i * d.ldR] : d.R[i + (int64_t)j * d.ldR];
  }
  // rows h .. FAC_CMAX - 1 are zero: the sweeps read and rotate whole groups
  // of 16 rows without tests
  for (int idx = tid; idx < (FAC_CMAX - h) * c; idx += JFT) {
    const int i = h + idx % (FAC_CMAX - h), j = idx / (FAC_CMAX - h);
    sA[i + j * JAC_LD] = 0.0;
  }
  if (accZ)
    for (int idx = tid; idx < c * c; idx += JFT) {
      const int i = idx % c, j = idx / c;
      sZ[i + j * JAC_LD] = (i == j) ? 1.0 : 0.0;
    }
  __syncthreads();
  // Householder route: rotate to rounding level.  Gram route (samples with
  // BF16 noise, ~1e-3): the columns of U = M Z diag(1/s) are orthonormal to
  // the rotation tolerance (U^T U - I = the scaled off-diagonal of Z^T G Z),
  // so 1e-12 is ample; sweeps stop once the largest inner product met in a
  // sweep is below 1e-6.
  const double tol = d.gram ? 1e-12 : (double)max(h, 1) * DBL_EPSILON;
  const double stop = d.gram ? 1e-6 : 0.0;
  int sweeps = 0;
  switch ((h + JAC_G - 1) / JAC_G) {
    case 1: sweeps = jacobi_sweeps<1, JFT>(sA, sZ, sN, h, c, accZ, flag, tol, stop); break;
    case 2: sweeps = jacobi_sweeps<2, JFT>(sA, sZ, sN, h, c, accZ, flag, tol, stop); break;
    case 3: sweeps = jacobi_sweeps<3, JFT>(sA, sZ, sN, h, c, accZ, flag, tol, stop); break;
    case 4: sweeps = jacobi_sweeps<4, JFT>(sA, sZ, sN, h, c, accZ, flag, tol, stop); break;
    case 5: sweeps = jacobi_sweeps<5, JFT>(sA, sZ, sN, h, c, accZ, flag, tol, stop); break;
    case 6: sweeps = jacobi_sweeps<6, JFT>(sA, sZ, sN, h, c, accZ, flag, tol, stop); break;
    default: break;   // h = 0: nothing to rotate
  }
  if (tid == 0 && d.sweeps) atomicMax(d.sweeps, sweeps);
  for (int j = tid; j < c; j += JFT) {
    double s = 0.0;
    for (int i = 0; i < h; ++i) s += sA[i + j * JAC_LD] * sA[i + j * JAC_LD];
    snorm[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < c; j += JFT) {
    const double sj = snorm[j];
    int rk = 0;
    for (int i2 = 0; i2 < c; ++i2) rk += (snorm[i2] > sj) || (snorm[i2] == sj && i2 < j);
    srank[j] = rk;
  }
  if (NEED_Z && wantX && !accZ && !d.gram)   // T (h x c) for X diag(s) = T^T W
    for (int idx = tid; idx < h * c; idx += JFT) {
      const int i = idx % h, j = idx / h;
      sZ[i + j * JAC_LD] = d.R[i + (int64_t)j * d.ldR];
    }
  __syncthreads();
  // column j goes to position srank[j] (descending norms, ties by index),
  // embedded in the wrows (xrows) frame; positions c .. kout - 1 get unit
  // vectors e_j and singular value 0
  if (d.gram) {
    // x_j = P u_j: W(perm[i], rk) = a_j(i) / s_j^2, X(perm[i], rk) = a_j(i)
    for (int e = tid; e < c * h; e += JFT) {
      const int i = e % h, j = e / h;
      const int rk = srank[j];
      if (rk >= d.kout) continue;
      const double sj = snorm[j];
      if (i == 0) d.sv[rk] = sj;
      const double a = sA[i + j * JAC_LD];
      const int pi = d.perm[i];
      d.W[pi + (int64_t)rk * d.ldW] = sj > 0.0 ? a / (sj * sj) : 0.0;
      if (wantX) d.X[pi + (int64_t)rk * d.ldX] = a;
    }
    for (int e = tid; e < (d.kout - c) * h; e += JFT) {
      const int i = e % h, rk = c + e / h;
      if (i == 0) d.sv[rk] = 0.0;
      d.W[i + (int64_t)rk * d.ldW] = 0.0;
      if (wantX) d.X[i + (int64_t)rk * d.ldX] = 0.0;
    }
    // W columns kout .. wrows - 1 (a wider product shared with other nodes) are zero
    for (int e = tid; e < (d.wrows - d.kout) * h; e += JFT)
      d.W[e % h + (int64_t)(d.kout + e / h) * d.ldW] = 0.0;
    return;
  }
  const int rows = max(d.wrows, wantX ? d.xrows : 0);
  for (int e = tid; e < c * rows; e += JFT) {
    const int i = e % rows, j = e / rows;
    const int rk = srank[j];
    if (rk >= d.kout) continue;
    const double sj = snorm[j];
    if (i == 0) d.sv[rk] = sj;
    if (i < d.wrows)
      d.W[i + (int64_t)rk * d.ldW] = (i < h && sj > 0.0) ? sA[i + j * JAC_LD] / sj : 0.0;
    if (wantX && i < d.xrows) {
      double xv = 0.0;
      if (i < c) {
        if (accZ) {
          xv = sZ[i + j * JAC_LD];
        } else if (NEED_Z && sj > 0.0) {
          // (T^T w_j)_i with w_j = T z_j / s_j the converged column j
          for (int l = 0; l < h; ++l) xv = fma(sZ[l + i * JAC_LD], sA[l + j * JAC_LD], xv);
          xv /= sj;
        }
      }
      d.X[i + (int64_t)rk * d.ldX] = xv;
    }
  }
  for (int e = tid; e < (d.kout - c) * rows; e += JFT) {
    const int i = e % rows, rk = c + e / rows;
    if (i == 0) d.sv[rk] = 0.0;
    if (i < d.wrows) d.W[i + (int64_t)rk * d.ldW] = i == rk ? 1.0 : 0.0;
    if (wantX && i < d.xrows) d.X[i + (int64_t)rk * d.ldX] = (accZ && i == rk) ? 1.0 : 0.0;
  }
}

void launch_jacobi_svd(const SvdDesc* d, int n, hipStream_t s, bool gram_only) {
  if (n <= 0) return;
  if (gram_only)
    hipLaunchKernelGGL(k_jacobi<false>, dim3(n), dim3(jacobi_threads<false>()), 0, s, d);
  else
    hipLaunchKernelGGL(k_jacobi<true>, dim3(n), dim3(jacobi_threads<true>()), 0, s, d);
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
  // fixed trip counts (r <= HM_MAX_SAMPLES): every load in flight before the stores
  double v[HM_MAX_SAMPLES];
#pragma unroll
  for (int j = 0; j < HM_MAX_SAMPLES; ++j) v[j] = j < r ? S[i + (int64_t)(off + j) * lds] : 0.0;
#pragma unroll
  for (int j = 0; j < HM_MAX_SAMPLES; ++j)
    if (j < r) M[i + (int64_t)j * ldm] = v[j];
  if (!first_half_only && nodes[nd.parent].parent >= 0) {
    const double* wp = w + (int64_t)nd.parent * R;
#pragma unroll
    for (int j = 0; j < HM_MAX_SAMPLES; ++j) v[j] = j < r ? Lpar[i + (int64_t)j * ldl] * wp[j] : 0.0;
#pragma unroll
    for (int j = 0; j < HM_MAX_SAMPLES; ++j)
      if (j < r) M[i + (int64_t)(r + j) * ldm] = v[j];
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
    Bv[e] = (i < r && j < r) ? Xv[i + j * 2 * R] * (z ? zv[j] : 1.0) : 0.0;
  }
}

void launch_form_b(const Node* nodes, const Instance* inst, const int32_t* kids, int nkids, int R,
                   const double* X, const double* z, double* B, hipStream_t s) {
  if (nkids <= 0) return;
  hipLaunchKernelGGL(k_form_b, dim3(nkids), dim3(256), 0, s, nodes, inst, kids, R, X, z, B);
  KCHK();
}

// ------------------------------------------------------------ CPQR / ID ---
// Threads NT: four lanes per candidate column, so at most NT / 4 candidates
// per node: 1024 for leaves (rows, at most 256), 384 for parents (2R <= 96
// candidates; fewer waves meet at each of the ID's barriers)
constexpr int ID_T_LEAF = 1024;
constexpr int ID_T_PARENT = 4 * 2 * HM_MAX_SAMPLES;
static_assert(HM_MAX_SAMPLES <= 48, "12 rows per lane");
// sum over the four lanes of a quad (the lanes of one candidate column)
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  return v;
}
// LDS of one node's ID with ID_T threads (at most ID_T / 4 candidates)
template <int ID_T>
struct IdShared {
  double M[(HM_MAX_SAMPLES + 1) * (ID_T / 4)];  // M = W^T, R x n, ld R+1
  double nrm[ID_T / 4];
  int perm[ID_T / 4];
  double v[HM_MAX_SAMPLES];
  double c[4];
};

// The ID of one node from its weighted candidate matrix, already in sm.M
// (candidate b, sample dimension a at a + b (R + 1); sm.perm the identity):
// column-pivoted Householder QR of W^* in LDS, T = R11^-1 R12, outputs as
// launch_cpqr_id describes.  src / ls: the unweighted candidate rows (global
// or LDS), read for samp_t.  All ID_T threads of the workgroup call it.
template <int ID_T>
__device__ void id_core(double* sM, double* snrm, int* sperm, double* sv, double* sc,
                        const Node& nd, const Instance& in, int g, int parent_mode, int R, int n,
                        const double* src, int64_t ls, double* P, int64_t ldp, double* samp,
                        int32_t* rank, int32_t* skel, int32_t* saturated) {
  constexpr int ID_NMAX = ID_T / 4;
  const int tid = threadIdx.x;
  const int ldm = R + 1;
  const int kcap = min(min(in.k, in.r), min(R, n));
  const int lane = tid & 63, wave = tid >> 6;
  // squared norms of the candidate columns: lane q of column b's quad takes
  // rows q, q + 4, ...
  {
    const int b = tid >> 2, q = tid & 3;
    double s2 = 0.0;
#pragma unroll
    for (int i = 0; i < HM_MAX_SAMPLES / 4; ++i) {
      const int a = q + 4 * i;
      const double x = (b < n && a < R) ? sM[a + b * ldm] : 0.0;
      s2 = fma(x, x, s2);
    }
    s2 = quad_sum(s2);
    if (b < n && q == 0) snrm[b] = s2;
  }
  __syncthreads();
  int k = 0;
  double ref = 0.0;
  for (int j = 0; j < kcap; ++j) {
    // pivot: largest remaining norm, lowest index on ties (every wave alike)
    double bv = -1.0;
    int bi = n;
#pragma unroll
    for (int q = 0; q < (ID_NMAX + 63) / 64; ++q) {
      const int b = j + lane + 64 * q;
      if (b < n && snrm[b] > bv) { bv = snrm[b]; bi = b; }
    }
    const double vmax = max64(bv);
    // no candidate left with a comparable norm (all NaN: non-finite samples,
    // reported by the caller) stops the factorisation here: p would be n
    if (!(vmax >= 0.0)) break;
    const int p = (int)(-max64(bv == vmax ? -(double)bi : -1e9));
    const double nrm = sqrt(vmax);
    if (j == 0) ref = nrm;
    if (nrm == 0.0 || (in.tol > 0.0 && nrm <= in.tol * ref)) break;
    __syncthreads();   // every wave has read the norms
    if (wave == 0) {
      // Householder reflector of the pivot column (v = x - alpha e_j, H = I - f v v^T),
      // written into position j in its final form; old column j goes to p
      const bool in_r = lane < R;
      const double x = in_r ? sM[lane + p * ldm] : 0.0;
      const double y = in_r ? sM[lane + j * ldm] : 0.0;
      const double x0 = readlane_d(x, j);
      const double s2 = sum64(lane >= j ? x * x : 0.0);
      const double alpha = -copysign(sqrt(s2), x0);
      const double vj = x0 - alpha;
      const double vn = s2 - x0 * x0 + vj * vj;
      if (in_r) {
        sv[lane] = lane == j ? vj : (lane > j ? x : 0.0);
        sM[lane + j * ldm] = lane < j ? x : (lane == j ? alpha : 0.0);
        if (p != j) sM[lane + p * ldm] = y;
      }
      if (lane == 0) {
        sc[2] = vn > 0.0 ? 2.0 / vn : 0.0;
        const int t = sperm[j]; sperm[j] = sperm[p]; sperm[p] = t;
      }
    }
    __syncthreads();
    // apply H to the remaining candidates, then their norms below row j: a
    // quad per candidate, lane q on rows j + q, j + q + 4, ... (at most 12),
    // the partial sums added across the quad
    const double f = sc[2];
    {
      const int b = j + 1 + (tid >> 2), q = tid & 3;
      const bool colok = b < n;
      double xs[HM_MAX_SAMPLES / 4];
      double s2 = 0.0;
#pragma unroll
      for (int i = 0; i < HM_MAX_SAMPLES / 4; ++i) {
        const int a = j + q + 4 * i;
        const bool act = colok && a < R;
        xs[i] = act ? sM[a + b * ldm] : 0.0;
        s2 = fma(act ? sv[a] : 0.0, xs[i], s2);
      }
      s2 = quad_sum(s2) * f;
      double n2 = 0.0;
#pragma unroll
      for (int i = 0; i < HM_MAX_SAMPLES / 4; ++i) {
        const int a = j + q + 4 * i;
        if (colok && a < R) {
          const double v = fma(-s2, sv[a], xs[i]);
          sM[a + b * ldm] = v;
          if (a > j) n2 = fma(v, v, n2);
        }
      }
      n2 = quad_sum(n2);
      if (colok && q == 0) snrm[b] = n2;
    }
    __syncthreads();
    k = j + 1;
  }
  // T = R11^{-1} R12, column by column (back substitution); stored in place of R12.
  for (int b = k + tid; b < n; b += ID_T) {
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
  for (int idx = tid; idx < n * R; idx += ID_T) {
    const int b = idx % n, col = idx / n;
    double v = 0.0;
    if (col < k) v = (b < k) ? (b == col ? 1.0 : 0.0) : sM[col + b * ldm];
    Pout[sperm[b] + (int64_t)col * lp] = v;
  }
  double* sp = samp + (int64_t)g * R * R;
  for (int idx = tid; idx < R * R; idx += ID_T) {
    const int i = idx % R, a = idx / R;
    sp[idx] = (i < k) ? src[sperm[i] + (int64_t)a * ls] : 0.0;
  }
  int32_t* sk_out = skel + (int64_t)g * R;
  for (int i = tid; i < R; i += ID_T) {
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

template <int ID_T>
__global__ __launch_bounds__(ID_T) void k_cpqr_id(const Node* nodes, const Instance* inst,
                                                 const int32_t* list, int parent_mode, int R,
                                                 const double* Src, int64_t lds, const double* w,
                                                 double* P, int64_t ldp, double* samp,
                                                 int32_t* rank, int32_t* skel, int32_t* saturated) {
  __shared__ IdShared<ID_T> sm;
  const int g = list[blockIdx.x];
  const Node nd = nodes[g];
  const Instance in = inst[nd.inst];
  const int tid = threadIdx.x;
  const int ldm = R + 1;
  const int n = parent_mode ? 2 * R : (int)(nd.hi - nd.lo);
  const double* src = parent_mode ? Src + (int64_t)g * 2 * R * R : Src + nd.lo;
  const int64_t ls = parent_mode ? 2 * R : lds;
  const double* wv = w + (int64_t)g * R;
  for (int idx = tid; idx < n * R; idx += ID_T) {
    const int b = idx % n, a = idx / n;  // candidate b, sample dim a
    sm.M[a + b * ldm] = src[b + (int64_t)a * ls] * wv[a];
  }
  for (int b = tid; b < n; b += ID_T) sm.perm[b] = b;
  __syncthreads();
  id_core<ID_T>(sm.M, sm.nrm, sm.perm, sm.v, sm.c, nd, in, g, parent_mode, R, n, src, ls, P, ldp,
                samp, rank, skel, saturated);
}

// ---- the whole Fig. 5 sweep in one persistent launch --------------------------
// Work items (node, side) in order of decreasing level, over every instance of
// the forest; each workgroup takes the next item from a device counter until
// none is left.  A leaf item is ready at once; a parent item waits until both
// children of its side are done (their samp_t, skeletons and ranks are
// published with a release at agent scope and read after an acquire), builds
// Utmp = diag(samp_left, samp_right) Tr_t in LDS (k_utmp) and runs the ID on
// it (parent mode of k_cpqr_id).  Items are taken in an order in which every
// item's children were taken before it, by workgroups that are running, so
// every wait ends; a wait longer than the spin limit (never expected) marks
// the item done without doing it and sets *err, so that no workgroup waits
// forever.
constexpr int IDS_T = 1024;
constexpr int IDS_SPIN_LIMIT = 1 << 20;

// LDS of the sweep: a leaf item's candidate matrix ((R + 1) x 256), or a
// parent item's ((R + 1) x 2R) followed by samp_left | samp_right (R x R
// each), Tr_t and Utmp_t (2R x R each)
constexpr int IDS_RAW_LEAF = (HM_MAX_SAMPLES + 1) * (IDS_T / 4);
constexpr int IDS_RAW_PARENT =
    (HM_MAX_SAMPLES + 1) * 2 * HM_MAX_SAMPLES + 6 * HM_MAX_SAMPLES * HM_MAX_SAMPLES;
constexpr int IDS_RAW = IDS_RAW_LEAF > IDS_RAW_PARENT ? IDS_RAW_LEAF : IDS_RAW_PARENT;

// Polls with relaxed coherent loads (an acquire per poll would invalidate
// the L2 of the XCD each time, slowing every other workgroup there); the
// acquire follows once the flag is seen.
__device__ __forceinline__ bool id_wait(int32_t* flag) {
  for (int it = 0; it < IDS_SPIN_LIMIT; ++it) {
    if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return true;
    __builtin_amdgcn_s_sleep(2);
  }
  return false;
}

__global__ __launch_bounds__(IDS_T) void k_id_sweep(const Node* nodes, const Instance* inst,
                                                   const IdItem* items, int nitems,
                                                   IdSide side0, IdSide side1, int R,
                                                   int64_t ldb, int32_t* done, int32_t* next,
                                                   int32_t* err, int32_t* saturated) {
  __shared__ double raw[IDS_RAW];
  __shared__ double snrm[IDS_T / 4];
  __shared__ int sperm[IDS_T / 4];
  __shared__ double sv[HM_MAX_SAMPLES];
  __shared__ double sc[4];
  __shared__ int s_item, s_ok;
  const int tid = threadIdx.x;
  const int ldm = R + 1;
  const int RR = R * R;
  double* sM = raw;
  double* sA = raw + (R + 1) * 2 * R;   // parent items only
  double* sT = sA + 2 * RR;
  double* sU = sT + 2 * RR;
  // Control flow in this loop stays uniform across the workgroup (scalar
  // conditions only, outside id_core's own uniform loops): a branch on the
  // thread index around the loop's barriers would be structured by the
  // compiler so that thread 0's steps (taking an item, publishing one) run
  // only once the other lanes have left the loop, while those lanes loop on
  // at its barriers with a stale item.  The steps that need one thread are
  // done by all lanes of wave 0, under a branch on the wave index read into a
  // scalar register.
  const int wave_u = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  for (;;) {
    if (wave_u == 0) {
      // lane 0 adds 1, the others 0: lane 0's result is the counter's old value
      const int v = atomicAdd(next, lane == 0 ? 1 : 0);
      s_item = __builtin_amdgcn_readfirstlane(v);
    }
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();   // every thread has the index before wave 0 takes the next
    if (it >= nitems) break;
    const IdItem itm = items[it];
    const IdSide sd = itm.side ? side1 : side0;
    const int g = itm.node;
    const Node nd = nodes[g];
    const Instance in = inst[nd.inst];
    const bool parent = nd.left >= 0;
    const double* wv = sd.w + (int64_t)g * R;
    if (!parent) {
      const int n = (int)(nd.hi - nd.lo);
      const double* src = sd.basis + nd.lo;
      for (int idx = tid; idx < n * R; idx += IDS_T) {
        const int b = idx % n, a = idx / n;
        sM[a + b * ldm] = src[b + (int64_t)a * ldb] * wv[a];
      }
      for (int b = tid; b < n; b += IDS_T) sperm[b] = b;
      __syncthreads();
      id_core<IDS_T>(sM, snrm, sperm, sv, sc, nd, in, g, 0, R, n, src, ldb, sd.P, ldb, sd.samp,
                     sd.rank, sd.skel, saturated);
    } else {
      const int n = 2 * R;
      if (wave_u == 0) {
        const bool a = id_wait(done + 2 * nd.left + itm.side);
        const bool b = id_wait(done + 2 * nd.right + itm.side);
        const int okw = __builtin_amdgcn_readfirstlane((a && b) ? 1 : 0);
        s_ok = okw;
        if (!okw) atomicOr(err, 1);
      }
      __syncthreads();
      const bool go = __builtin_amdgcn_readfirstlane(s_ok) != 0;
      // every thread acquires the children's results for itself
      (void)__hip_atomic_load(done + 2 * nd.left + itm.side, __ATOMIC_ACQUIRE,
                              __HIP_MEMORY_SCOPE_AGENT);
      (void)__hip_atomic_load(done + 2 * nd.right + itm.side, __ATOMIC_ACQUIRE,
                              __HIP_MEMORY_SCOPE_AGENT);
      if (go) {
        const double* sl = sd.samp + (int64_t)nd.left * RR;
        const double* sr = sd.samp + (int64_t)nd.right * RR;
        const double* tr = sd.told + (int64_t)g * 2 * RR;
        for (int e = tid; e < RR; e += IDS_T) {
          sA[e] = sl[e];
          sA[RR + e] = sr[e];
        }
        for (int e = tid; e < 2 * RR; e += IDS_T) sT[e] = tr[e];
        __syncthreads();
        // Utmp(side R + i, j) = sum_m samp_side(i, m) Tr(side R + m, j)
        for (int e = tid; e < 2 * RR; e += IDS_T) {
          const int row = e % (2 * R), j = e / (2 * R);
          const int side = row >= R ? 1 : 0, i = row - side * R;
          const double* sa = sA + side * RR;
          double acc = 0.0;
          for (int m = 0; m < R; ++m) acc = fma(sa[i + m * R], sT[side * R + m + j * 2 * R], acc);
          sU[row + j * 2 * R] = acc;
        }
        __syncthreads();
        for (int idx = tid; idx < n * R; idx += IDS_T) {
          const int b = idx % n, a = idx / n;
          sM[a + b * ldm] = sU[b + a * 2 * R] * wv[a];
        }
        for (int b = tid; b < n; b += IDS_T) sperm[b] = b;
        __syncthreads();
        id_core<IDS_T>(sM, snrm, sperm, sv, sc, nd, in, g, 1, R, n, sU, 2 * R, sd.Pt, 2 * R,
                       sd.samp, sd.rank, sd.skel, saturated);
      }
    }
    // publish: every thread's stores (released at agent scope), then the
    // item's flag (wave 0's lanes all store the same 1)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (wave_u == 0)
      __hip_atomic_store(done + 2 * g + itm.side, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

void launch_id_sweep(const Node* nodes, const Instance* inst, const IdItem* items, int nitems,
                     const IdSide& u, const IdSide& v, int R, int64_t ldb, int32_t* done,
                     int32_t* next, int32_t* err, int32_t* saturated, int workgroups,
                     hipStream_t s) {
  if (nitems <= 0) return;
  const int grid = std::max(1, std::min(workgroups, nitems));
  hipLaunchKernelGGL(k_id_sweep, dim3(grid), dim3(IDS_T), 0, s, nodes, inst, items, nitems, u, v,
                     R, ldb, done, next, err, saturated);
  KCHK();
}

void launch_cpqr_id(const Node* nodes, const Instance* inst, const int32_t* list, int nlist,
                    int parent_mode, int R, const double* Src, int64_t lds, const double* w,
                    double* P, int64_t ldp, double* samp, int32_t* rank, int32_t* skel,
                    int32_t* saturated, hipStream_t s) {
  if (nlist <= 0) return;
  if (parent_mode)
    hipLaunchKernelGGL(k_cpqr_id<ID_T_PARENT>, dim3(nlist), dim3(ID_T_PARENT), 0, s, nodes, inst,
                       list, parent_mode, R, Src, lds, w, P, ldp, samp, rank, skel, saturated);
  else
    hipLaunchKernelGGL(k_cpqr_id<ID_T_LEAF>, dim3(nlist), dim3(ID_T_LEAF), 0, s, nodes, inst, list,
                       parent_mode, R, Src, lds, w, P, ldp, samp, rank, skel, saturated);
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

// 64 x 64 output tiles on the FP64 matrix cores, stored through LDS
// (column-contiguous writes)
__global__ __launch_bounds__(256) void k_node_nn(const Node* nodes, const int32_t* list, int K,
                                                 int N, const double* A, int64_t lda,
                                                 const double* Bn, int64_t bstride, int64_t ldb,
                                                 double* out, int64_t ldo, int from_sibling) {
  static_assert(STM == MF_T && STN == MF_T, "node products in the MFMA tile shape");
  __shared__ double smem[mf_smem_elems<double>()];
  const int g = list[blockIdx.y];
  const int gb = from_sibling ? nodes[g].sib : g;
  const Node nd = nodes[g];
  const int64_t i0 = nd.lo + (int64_t)blockIdx.x * STM;
  if (i0 >= nd.hi) return;
  const int M = (int)min<int64_t>(STM, nd.hi - i0);
  const int j0 = blockIdx.z * STN;
  MfAcc<double> acc;
  acc.zero();
  mf_tile<double>(M, N - j0, K, A + i0, 1, lda, Bn + (int64_t)gb * bstride + j0 * ldb, 1, ldb, acc,
                  smem);
  mf_store_lds<double>(M, N - j0, out + i0 + (int64_t)j0 * ldo, ldo, acc, 1.0, 0.0, smem);
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
