// Frontal matrix of nested dissection (Sec. 5.4): the black box
//   A x = B33 x - B31 B11^-1 B13 x - B32 B22^-1 B23 x
// of the conduction grid of Fig. 13 (H rows and W columns of nodes, bars of
// given conductivity between neighbours, B the network's Laplacian, I3 the
// middle column, I1 / I2 the columns left / right of it).
//
// Each side is block tridiagonal in grid rows: with the right side mirrored
// (local column j is grid column W-1-j) the node next to the middle column is
// local column w-1 on both sides, w = (W-1)/2.  Row i has a w x w diagonal
// block D_i (tridiagonal: the horizontal bars, plus every bar of a node on
// the diagonal) and the coupling C_i = T(i, i+1) = -diag(vertical bars of
// row i), T(i+1, i) = C_i^T.
//
// The factorisation is block cyclic reduction (odd-even elimination of block
// rows, the nested-dissection order of a strip).  At level l the active rows
// are i = p 2^l, p = 0 .. n_l - 1; the odd p are eliminated,
//   Dinv_q = D_q^-1,  gam_q = Dinv_q C_{q-1}^T,  del_q = Dinv_q C_q,
// and the even p keep the reduced system
//   D_p <- D_p - C_{p-1}^T del_{p-1} - C_p gam_{p+1},   C_p <- -C_p del_{p+1},
// until one row is left, whose inverse is the root.  The sides are symmetric
// positive definite, so every reduced block is too and Gauss-Jordan needs no
// pivoting.  A solve reduces the right-hand side the same way,
//   b_p <- b_p - del_{p-1}^T b_{p-1} - gam_{p+1}^T b_{p+1},
// solves the root and substitutes back, x_q = Dinv_q b_q - gam_q x_{q-1} -
// del_q x_{q+1}, level by level.
//
// The products with A solve only for right-hand sides on the column next to
// the middle (B13 x) and read only that column of the solution, so levels 0
// and 1 are taken apart: the level-0 right-hand sides are never formed (each
// is g_i e_{w-1}, g_i = c_link(i) x_i), the level-1 steps use small operators
// built once with the factor (the level-2 right-hand side of a row is a
// combination of seven g's, and a level-1 back substitution only needs the
// three projections of its solution that level 0 reads), and level 0's back
// substitution computes only the column next to the middle, fused with B33 x
// and the sum that forms A x.
#include <algorithm>

#include "handle.h"

struct hm_frontal_s {
  int64_t H = 0;
  int W = 0, w = 0;
  int wp = 0;            // w rounded up to a multiple of 4
  int levels = 0;        // reduction levels: n_levels == 1
  hm::DevBuf fac;        // [side][row][Dinv | gam | del], w x w column-major each
  hm::DevBuf edge;       // [side][row][gam(w-1, :) | del(w-1, :) | Dinv(w-1, w-1), 0]
  hm::DevBuf ops;        // level-1 operators: [side][level-1 position][recw]
  int recw = 0;
  hm::DevBuf ops2;       // level-2 operators (levels >= 3): [side][level-2 position][recw2]
  int recw2 = 0;
  hm::DevBuf bars;       // [row][cL, cR, cv_mid]: the middle column's bars
};

namespace hm {

constexpr int FR_WMAX = 32;

// ---- assembly -------------------------------------------------------------------
// D_i and C_i of both sides (entry e = r + k w of row i of side s), and the
// bars of the middle column.
__global__ __launch_bounds__(256) void k_fr_assemble(const double* ch, const double* cv,
                                                     int64_t H, int W, int w, double* Dw,
                                                     double* Cw, double* bars) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t per = (int64_t)w * w;
  const int mid = w;
  if (e < H) {
    const int64_t i = e;
    bars[3 * i + 0] = ch[i * (W - 1) + mid - 1];
    bars[3 * i + 1] = ch[i * (W - 1) + mid];
    bars[3 * i + 2] = i + 1 < H ? cv[i * W + mid] : 0.0;
  }
  if (e >= 2 * H * per) return;
  const int side = (int)(e / (H * per));
  const int64_t i = (e / per) % H;
  const int r = (int)((e % per) % w), k = (int)((e % per) / w);
  const int col = side == 0 ? r : W - 1 - r;
  double d = 0.0, c = 0.0;
  if (r == k) {
    if (col >= 1) d += ch[i * (W - 1) + col - 1];
    if (col <= W - 2) d += ch[i * (W - 1) + col];
    if (i >= 1) d += cv[(i - 1) * W + col];
    if (i + 1 < H) {
      d += cv[i * W + col];
      c = -cv[i * W + col];
    }
  } else if (r == k + 1 || k == r + 1) {
    // the bar between local columns j and j+1: grid columns j, j+1 on the
    // left, W-2-j, W-1-j on the right
    const int j = min(r, k);
    d = -ch[i * (W - 1) + (side == 0 ? j : W - 2 - j)];
  }
  Dw[e] = d;
  Cw[e] = c;
}

// ---- factorisation ----------------------------------------------------------------
__device__ inline int64_t fr_blk(int side, int64_t H, int64_t i, int w) {
  return ((int64_t)side * H + i) * w * w;
}

// Factor blocks: row i of a side holds Dinv, gam, del as wp x wp blocks
// (column-major, ld wp, zero past w), so the solve reads them without bounds.
__device__ inline int64_t fr_fac(int side, int64_t H, int64_t i, int wp) {
  return ((int64_t)side * H + i) * 3 * wp * wp;
}

// Eliminated rows of level l (odd p; p = 0 at the root): Dinv, gam, del.
// Also the row's edge entries (see the solve), zero-padded to wp.
__global__ __launch_bounds__(256) void k_fr_elim(const double* Dw, const double* Cw, double* fac,
                                                 double* edge, int64_t H, int w, int wp,
                                                 int64_t s, int64_t n, int root, int32_t* bad) {
  constexpr int LD = FR_WMAX + 1;
  __shared__ double A[FR_WMAX * LD];
  __shared__ double Cm[FR_WMAX * LD];   // C_{q-1}
  __shared__ double Cp[FR_WMAX * LD];   // C_q
  __shared__ double mult[FR_WMAX];
  const int side = blockIdx.z;
  const int tid = threadIdx.x;
  const int64_t q = root ? 0 : 2 * (int64_t)blockIdx.x + 1;
  const int64_t i = q * s;
  const int per = w * w;
  const bool has_prev = q >= 1, has_next = q + 1 < n;
  const double* D = Dw + fr_blk(side, H, i, w);
  for (int e = tid; e < per; e += 256) {
    const int r = e % w, k = e / w;
    A[r + k * LD] = D[e];
    Cm[r + k * LD] = has_prev ? Cw[fr_blk(side, H, i - s, w) + e] : 0.0;
    Cp[r + k * LD] = has_next ? Cw[fr_blk(side, H, i, w) + e] : 0.0;
  }
  __syncthreads();
  bool fail = false;
  for (int kk = 0; kk < w; ++kk) {
    const double piv = A[kk + kk * LD];
    if (!(piv > 0.0) || !isfinite(piv)) fail = true;
    const double rp = 1.0 / piv;
    for (int r = tid; r < w; r += 256) mult[r] = r == kk ? 0.0 : A[r + kk * LD];
    __syncthreads();
    for (int j = tid; j < w; j += 256) A[kk + j * LD] = (j == kk ? 1.0 : A[kk + j * LD]) * rp;
    __syncthreads();
    for (int e = tid; e < per; e += 256) {
      const int r = e % w, j = e / w;
      if (r == kk) continue;
      const double a = j == kk ? 0.0 : A[r + j * LD];
      A[r + j * LD] = fma(-mult[r], A[kk + j * LD], a);
    }
    __syncthreads();
  }
  double* F = fac + fr_fac(side, H, i, wp);
  double* E = edge + (2 * wp + 2) * ((int64_t)side * H + i);
  const int pp = wp * wp;
  for (int e = tid; e < pp; e += 256) {
    const int r = e % wp, c = e / wp;
    if (r >= w || c >= w) {
      F[e] = F[pp + e] = F[2 * pp + e] = 0.0;
      continue;
    }
    double g = 0.0, d = 0.0;
    for (int k = 0; k < w; ++k) {
      const double a = A[r + k * LD];
      g = fma(a, Cm[c + k * LD], g);   // Dinv C_{q-1}^T
      d = fma(a, Cp[k + c * LD], d);   // Dinv C_q
    }
    F[e] = A[r + c * LD];
    F[pp + e] = g;
    F[2 * pp + e] = d;
    if (r == w - 1) {
      E[c] = g;
      E[wp + c] = d;
    }
  }
  for (int j = w + tid; j < wp; j += 256) {
    E[j] = 0.0;
    E[wp + j] = 0.0;
  }
  if (tid == 0) {
    E[2 * wp] = A[(w - 1) + (w - 1) * LD];
    E[2 * wp + 1] = 0.0;
  }
  if (fail && tid == 0) atomicOr(bad, 1);
}

// Kept rows of level l (even p): the reduced D_p and C_p.
__global__ __launch_bounds__(256) void k_fr_reduce(double* Dw, double* Cw, const double* fac,
                                                   int64_t H, int w, int wp, int64_t s,
                                                   int64_t n) {
  constexpr int LD = FR_WMAX + 1;
  __shared__ double Cm[FR_WMAX * LD];   // C_{p-1}
  __shared__ double Dm[FR_WMAX * LD];   // del_{p-1}
  __shared__ double Cs[FR_WMAX * LD];   // C_p
  __shared__ double Gp[FR_WMAX * LD];   // gam_{p+1}
  __shared__ double Dp[FR_WMAX * LD];   // del_{p+1}
  const int side = blockIdx.z;
  const int tid = threadIdx.x;
  const int64_t p = 2 * (int64_t)blockIdx.x;
  const int64_t i = p * s;
  const int per = w * w;
  const bool has_prev = p >= 1, has_next = p + 1 < n;
  for (int e = tid; e < per; e += 256) {
    const int r = e % w, k = e / w;
    Cm[r + k * LD] = has_prev ? Cw[fr_blk(side, H, i - s, w) + e] : 0.0;
    const int f = r + k * wp, pp = wp * wp;
    Dm[r + k * LD] = has_prev ? fac[fr_fac(side, H, i - s, wp) + 2 * pp + f] : 0.0;
    Cs[r + k * LD] = Cw[fr_blk(side, H, i, w) + e];
    Gp[r + k * LD] = has_next ? fac[fr_fac(side, H, i + s, wp) + pp + f] : 0.0;
    Dp[r + k * LD] = has_next ? fac[fr_fac(side, H, i + s, wp) + 2 * pp + f] : 0.0;
  }
  __syncthreads();
  double* D = Dw + fr_blk(side, H, i, w);
  double* C = Cw + fr_blk(side, H, i, w);
  for (int e = tid; e < per; e += 256) {
    const int r = e % w, c = e / w;
    double d = D[e], cn = 0.0;
    for (int k = 0; k < w; ++k) {
      d = fma(-Cm[k + r * LD], Dm[k + c * LD], d);   // - C_{p-1}^T del_{p-1}
      d = fma(-Cs[r + k * LD], Gp[k + c * LD], d);   // - C_p gam_{p+1}
      cn = fma(-Cs[r + k * LD], Dp[k + c * LD], cn); // - C_p del_{p+1}
    }
    D[e] = d;
    C[e] = cn;
  }
}

// Level-1 operators, built once after the factorisation.  The level-1
// right-hand sides are sparse combinations of x: b1_j = g_j e - g_{j-1} Ed_{j-1}
// - g_{j+1} Eg_{j+1} (g_j = c_link(j) x_j, e = e_{w-1}, Ed_j = del_j(w-1, :)^T,
// Eg_j = gam_j(w-1, :)^T of the rows eliminated at level 0), so both level-1
// steps collapse to small fixed operators per row:
//  * reduction at row i (level-1 position p = i / 2 even):
//      b2_i = sum_{d=0..6} g_{i+d-3} W_d,  W_3 = e,
//      W_2 = -Ed_{i-1} + del_{i-2}^T Eg_{i-1},  W_1 = -del_{i-2}^T e,
//      W_0 = del_{i-2}^T Ed_{i-3},  W_4 = -Eg_{i+1} + gam_{i+2}^T Ed_{i+1},
//      W_5 = -gam_{i+2}^T e,  W_6 = gam_{i+2}^T Eg_{i+3}  (absent rows: 0);
//  * back substitution at row i (p odd, or p = 0 when level 1 is the root):
//    the output needs only P_i = Q_i x_i (rows e^T, Ed_{i-1}^T, Eg_{i+1}^T),
//      P_i = sum_{d=0..2} S_d g_{i+d-1} - A x_{i-2} - B x_{i+2},
//      A = Q_i gam_i, B = Q_i del_i, S_d = Q_i Dinv_i c_d,
//      c = (-Ed_{i-1}, e, -Eg_{i+1}).
// Record of (side, p): W_0..W_6 (wp each), or A, B (3 x wp each, row-major)
// and S (3 x 3, S[q][d]).
__global__ __launch_bounds__(256) void k_fr_lvl1_ops(const double* fac, const double* edge,
                                                     double* ops, int64_t H, int w, int wp,
                                                     int recw) {
  constexpr int WM = FR_WMAX;
  __shared__ double M0[WM * WM], M1[WM * WM], M2[WM * WM];   // ld wp
  __shared__ double E[6][WM];
  __shared__ double Yd[3][WM];
  const int side = blockIdx.z, tid = threadIdx.x;
  const int64_t p = blockIdx.x, i = 2 * p;
  const int pp = wp * wp, EW = 2 * wp + 2;
  const int64_t n1 = (H + 1) / 2;
  auto ed = [&](int64_t j) -> const double* {
    return (j >= 0 && j < H) ? edge + EW * ((int64_t)side * H + j) + wp : nullptr;
  };
  auto eg = [&](int64_t j) -> const double* {
    return (j >= 0 && j < H) ? edge + EW * ((int64_t)side * H + j) : nullptr;
  };
  double* R = ops + ((int64_t)side * n1 + p) * recw;
  if (!(p & 1) && n1 > 1) {
    const bool prv = p >= 1, nxt = i + 2 < H;
    for (int e = tid; e < pp; e += 256) {
      M1[e] = prv ? fac[fr_fac(side, H, i - 2, wp) + 2 * pp + e] : 0.0;   // del_{i-2}
      M2[e] = nxt ? fac[fr_fac(side, H, i + 2, wp) + pp + e] : 0.0;       // gam_{i+2}
    }
    for (int e = tid; e < 6 * wp; e += 256) {
      const int slot = e / wp, k = e % wp;
      const double* src = slot == 0 ? ed(i - 3) : slot == 1 ? ed(i - 1) : slot == 2 ? eg(i - 1)
                        : slot == 3 ? ed(i + 1) : slot == 4 ? eg(i + 1) : eg(i + 3);
      E[slot][k] = src ? src[k] : 0.0;
    }
    __syncthreads();
    for (int r = tid; r < wp; r += 256) {
      double w0 = 0.0, w1 = 0.0, w2 = 0.0, w4 = 0.0, w5 = 0.0, w6 = 0.0;
      if (r < w) {
        for (int k = 0; k < w; ++k) {
          w0 = fma(M1[k + r * wp], E[0][k], w0);
          w2 = fma(M1[k + r * wp], E[2][k], w2);
          w4 = fma(M2[k + r * wp], E[3][k], w4);
          w6 = fma(M2[k + r * wp], E[5][k], w6);
        }
        w1 = -M1[(w - 1) + r * wp];
        w5 = -M2[(w - 1) + r * wp];
        w2 -= E[1][r];
        w4 -= E[4][r];
      }
      R[0 * wp + r] = w0;
      R[1 * wp + r] = w1;
      R[2 * wp + r] = w2;
      R[3 * wp + r] = r == w - 1 ? 1.0 : 0.0;
      R[4 * wp + r] = w4;
      R[5 * wp + r] = w5;
      R[6 * wp + r] = w6;
    }
    return;
  }
  // back substitution (or the root): Dinv_i, gam_i, del_i of row i
  for (int e = tid; e < pp; e += 256) {
    const int64_t b = fr_fac(side, H, i, wp);
    M0[e] = fac[b + e];
    M1[e] = fac[b + pp + e];
    M2[e] = fac[b + 2 * pp + e];
  }
  for (int e = tid; e < 2 * wp; e += 256) {
    const int slot = e / wp, k = e % wp;
    const double* src = slot == 0 ? ed(i - 1) : eg(i + 1);
    E[slot][k] = src ? src[k] : 0.0;
  }
  __syncthreads();
  // Yd_d = Dinv_i c_d
  for (int r = tid; r < w; r += 256) {
    double y0 = 0.0, y2 = 0.0;
    for (int k = 0; k < w; ++k) {
      y0 = fma(-M0[r + k * wp], E[0][k], y0);
      y2 = fma(-M0[r + k * wp], E[1][k], y2);
    }
    Yd[0][r] = y0;
    Yd[1][r] = M0[r + (w - 1) * wp];
    Yd[2][r] = y2;
  }
  __syncthreads();
  for (int k = tid; k < wp; k += 256) {
    double a1 = 0.0, a2 = 0.0, b1 = 0.0, b2 = 0.0;
    for (int r = 0; r < w; ++r) {
      a1 = fma(E[0][r], M1[r + k * wp], a1);
      a2 = fma(E[1][r], M1[r + k * wp], a2);
      b1 = fma(E[0][r], M2[r + k * wp], b1);
      b2 = fma(E[1][r], M2[r + k * wp], b2);
    }
    R[0 * wp + k] = M1[(w - 1) + k * wp];
    R[1 * wp + k] = a1;
    R[2 * wp + k] = a2;
    R[3 * wp + k] = M2[(w - 1) + k * wp];
    R[4 * wp + k] = b1;
    R[5 * wp + k] = b2;
  }
  if (tid < 9) {
    const int q = tid / 3, d = tid % 3;
    double sv = 0.0;
    if (q == 0) {
      sv = Yd[d][w - 1];
    } else {
      for (int r = 0; r < w; ++r) sv = fma(E[q - 1][r], Yd[d][r], sv);
    }
    R[6 * wp + tid] = sv;
  }
}

// Level-2 operators (when the reduction has three or more levels), from the
// level-1 ones: the level-2 right-hand side of a row j = 0 mod 4 is
// b2_j = sum_{d=0..6} g_{j+d-3} W_{j,d}, so
//  * reduction at row i (level-2 position q = i / 4 even):
//      b3_i = sum_{e=0..14} g_{i+e-7} V_e,  V_e = W_{i,e-4} - del_{i-4}^T W_{i-4,e}
//             - gam_{i+4}^T W_{i+4,e-8}  (terms whose index is out of 0..6 or
//             whose row is absent: 0);
//  * back substitution at row i (q odd): x_i = sum_d g_{i+d-3} DW_d - gam_i x_{i-4}
//    - del_i x_{i+4}, DW_d = Dinv_i W_{i,d}.
// Record of (side, q): V_0..V_14 or DW_0..DW_6 (wp each).
__global__ __launch_bounds__(256) void k_fr_lvl2_ops(const double* fac, const double* ops1,
                                                     int recw1, double* ops2, int64_t H, int w,
                                                     int wp, int recw2) {
  constexpr int WM = FR_WMAX;
  __shared__ double M1[WM * WM], M2[WM * WM];   // ld wp
  __shared__ double Wc[7 * WM], Wm[7 * WM], Wp[7 * WM];
  const int side = blockIdx.z, tid = threadIdx.x;
  const int64_t q = blockIdx.x, i = 4 * q;
  const int pp = wp * wp;
  const int64_t n1 = (H + 1) / 2, n2 = (n1 + 1) / 2;
  auto rec1 = [&](int64_t row) { return ops1 + ((int64_t)side * n1 + row / 2) * recw1; };
  double* R = ops2 + ((int64_t)side * n2 + q) * recw2;
  for (int e = tid; e < 7 * wp; e += 256) Wc[e] = rec1(i)[e];
  if (!(q & 1)) {
    const bool prv = q >= 1, nxt = i + 4 < H;
    for (int e = tid; e < pp; e += 256) {
      M1[e] = prv ? fac[fr_fac(side, H, i - 4, wp) + 2 * pp + e] : 0.0;   // del_{i-4}
      M2[e] = nxt ? fac[fr_fac(side, H, i + 4, wp) + pp + e] : 0.0;       // gam_{i+4}
    }
    for (int e = tid; e < 7 * wp; e += 256) {
      Wm[e] = prv ? rec1(i - 4)[e] : 0.0;
      Wp[e] = nxt ? rec1(i + 4)[e] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < 15 * wp; e += 256) {
      const int ee = e / wp, r = e % wp;
      double v = (ee >= 4 && ee <= 10) ? Wc[(ee - 4) * wp + r] : 0.0;
      if (r < w) {
        if (ee <= 6)
          for (int k = 0; k < w; ++k) v = fma(-M1[k + r * wp], Wm[ee * wp + k], v);
        if (ee >= 8)
          for (int k = 0; k < w; ++k) v = fma(-M2[k + r * wp], Wp[(ee - 8) * wp + k], v);
      }
      R[e] = v;
    }
    return;
  }
  for (int e = tid; e < pp; e += 256) M1[e] = fac[fr_fac(side, H, i, wp) + e];   // Dinv_i
  __syncthreads();
  for (int e = tid; e < 7 * wp; e += 256) {
    const int d = e / wp, r = e % wp;
    double v = 0.0;
    if (r < w)
      for (int k = 0; k < w; ++k) v = fma(M1[r + k * wp], Wc[d * wp + k], v);
    R[e] = v;
  }
}

// ---- solve ----------------------------------------------------------------------
// Right-hand sides Z[side][row][column][j]: WP entries per column (w rounded
// up to a multiple of 4, the entries past w zero), contiguous per row, so a
// column is whole 16-byte vectors.  The level-0 kernels read the last rows of
// gam and del and the last diagonal entry of Dinv from the edge array:
// edge[side][row] = [gam(w-1, :) | del(w-1, :) | Dinv(w-1, w-1), 0], each row
// zero-padded to WP.
__device__ inline int64_t fr_rhs(int side, int64_t H, int64_t i, int m, int wp) {
  return (((int64_t)side * H + i) * m) * wp;
}

template <int WP>
__device__ inline void fr_load(double (&v)[WP], const double* src) {
#pragma unroll
  for (int j = 0; j < WP; j += 2) {
    const double2 t = *reinterpret_cast<const double2*>(src + j);
    v[j] = t.x;
    v[j + 1] = t.y;
  }
}

template <int WP>
__device__ inline void fr_store(double* dst, const double (&v)[WP]) {
#pragma unroll
  for (int j = 0; j < WP; j += 2) *reinterpret_cast<double2*>(dst + j) = make_double2(v[j], v[j + 1]);
}

// Reduction from the level-1 (NV = 7) or level-2 (NV = 15) operators: the
// next level's right-hand side of row i = spacing x, sum_e g_{i+e-(NV-1)/2} V_e,
// one column per lane (x transposed: XT[j m + c] = x_j(c), contiguous over
// the lanes), V in LDS read as broadcasts, the result through LDS for
// contiguous stores; 64 columns per workgroup.  Records are indexed by the
// row's position at their level, i / (spacing / 2).
template <int WP, int NV>
__global__ __launch_bounds__(64) void k_fr_gfwd(const double* __restrict__ ops, int recw,
                                                int64_t nrec, int64_t spacing,
                                                double* __restrict__ Z, const double* XT,
                                                const double* bars, int64_t H, int m) {
  __shared__ __attribute__((aligned(16))) double sW[NV * WP];
  __shared__ __attribute__((aligned(16))) double sB[64 * WP];   // the result, for contiguous stores
  constexpr int HALF = (NV - 1) / 2;
  const int side = blockIdx.z, lane = threadIdx.x;
  const int64_t T = gridDim.x;
  int64_t x = blockIdx.x;
  if ((T & 7) == 0) x = (x & 7) * (T >> 3) + (x >> 3);
  const int64_t i = spacing * x;
  // records are indexed by position at their level: i / (spacing / 2)
  const double* R = ops + ((int64_t)side * nrec + i / (spacing / 2)) * recw;
  for (int e = lane; e < NV * WP; e += 64) sW[e] = R[e];
  const int c = blockIdx.y * 64 + lane;
  double gv[NV];
#pragma unroll
  for (int d = 0; d < NV; ++d) {
    const int64_t j = i + d - HALF;
    gv[d] = (c < m && j >= 0 && j < H) ? bars[3 * j + side] * XT[j * m + c] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < WP; r += 2) {
    double b0 = 0.0, b1 = 0.0;
#pragma unroll
    for (int d = 0; d < NV; ++d) {
      const double2 wv = *reinterpret_cast<const double2*>(sW + d * WP + r);
      b0 = fma(wv.x, gv[d], b0);
      b1 = fma(wv.y, gv[d], b1);
    }
    *reinterpret_cast<double2*>(sB + lane * WP + r) = make_double2(b0, b1);
  }
  __syncthreads();
  // the group's columns are contiguous in Z: 16-byte stores, consecutive over the lanes
  const int c0 = blockIdx.y * 64;
  const int nv = (min(64, m - c0) * WP) / 2;
  double2* dst = reinterpret_cast<double2*>(Z + fr_rhs(side, H, i, m, WP) + (int64_t)c0 * WP);
  for (int e = lane; e < nv; e += 64) dst[e] = reinterpret_cast<const double2*>(sB)[e];
}

// Level-1 back substitution from the level-1 operators: P_i = sum_d S_d
// g_{i+d-1} - A x_{i-2} - B x_{i+2} for row i = 2 p (p odd; p = 0 when level 1
// is the root), one column per lane.  A x_{i-2} and B x_{i+2} come ready from
// the kernels that produced those solutions (NP).
template <int WP>
__global__ __launch_bounds__(64) void k_fr_l1bwd(const double* __restrict__ ops, int recw,
                                                 const double* __restrict__ NP, double* P,
                                                 const double* XT, const double* bars, int64_t H,
                                                 int m, int root) {
  __shared__ double sS[9];
  const int side = blockIdx.z, lane = threadIdx.x;
  const int64_t T = gridDim.x;
  int64_t x = blockIdx.x;
  if ((T & 7) == 0) x = (x & 7) * (T >> 3) + (x >> 3);
  const int64_t p = root ? 0 : 2 * x + 1, i = 2 * p;
  const int64_t n1 = (H + 1) / 2, Hq = (H + 3) / 4;
  const double* R = ops + ((int64_t)side * n1 + p) * recw;
  if (lane < 9) sS[lane] = R[6 * WP + lane];
  const int c = blockIdx.y * 64 + lane;
  const bool act = c < m;
  const bool prv = !root, nxt = !root && i + 2 < H;
  double gv[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int64_t j = i + d - 1;
    gv[d] = (act && j >= 0 && j < H) ? bars[3 * j + side] * XT[j * m + c] : 0.0;
  }
  double nm[3] = {0.0, 0.0, 0.0}, npx[3] = {0.0, 0.0, 0.0};
  if (act && prv) {
    const double* src = NP + (((int64_t)side * Hq + (i - 2) / 4) * m + c) * 6;
#pragma unroll
    for (int q = 0; q < 3; ++q) nm[q] = src[q];
  }
  if (act && nxt) {
    const double* src = NP + (((int64_t)side * Hq + (i + 2) / 4) * m + c) * 6;
#pragma unroll
    for (int q = 0; q < 3; ++q) npx[q] = src[3 + q];
  }
  __syncthreads();
  if (!act) return;
  double pv[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double t = -nm[q] - npx[q];
#pragma unroll
    for (int d = 0; d < 3; ++d) t = fma(sS[3 * q + d], gv[d], t);
    pv[q] = t;
  }
  double* dst = P + (((int64_t)side * m + c) * ((H + 1) / 2) + i / 2) * 4;
  *reinterpret_cast<double2*>(dst) = make_double2(pv[0], pv[1]);
  *reinterpret_cast<double2*>(dst + 2) = make_double2(pv[2], 0.0);
}

// One level l >= 2 of the solve for one row and 64 columns (blockIdx.y: the
// group of columns, blockIdx.z: the side).  mode 0 reduction (even p):
// b_p -= del_{p-1}^T b_{p-1} + gam_{p+1}^T b_{p+1}; mode 1 back substitution
// (odd p): x_p = Dinv_p b_p - gam_p x_{p-1} - del_p x_{p+1}; mode 2 root:
// x_0 = Dinv_0 b_0; mode 3, the level-2 back substitution from the level-2
// operators: x_p = sum_d g_{i+d-3} DW_d - gam_p x_{p-1} - del_p x_{p+1}.  A back
// substitution or root writes x to Z and the
// 4-entry projection P_i = (x_i(w-1), Ed_{i-1}^T x_i, Eg_{i+1}^T x_i, 0) the
// output kernel reads.
//
// Two waves of 64 lanes; lane (g, q) = (lane / 16, lane % 16) of wave v
// holds output rows g RB .. g RB + RB - 1 (RB = WP / 4) of the two columns
// c0 + 32 v + q + 16 u (u = 0, 1).  The row's matrices are staged in LDS as
// L_t(r, k), row r contiguous (transposed from the factor where the product
// needs it), so every 16-byte LDS read feeds four FMAs: two entries, two
// columns.  A right-hand side's loads are all issued before its products.
// Rows are taken in an XCD-aware order: workgroups dispatched to one XCD
// (every 8th) handle a contiguous run of rows, so the neighbours two rows
// share meet in that XCD's L2.
struct FrStep {
  int64_t H, s, n;
  int w, m;
  int mode;
  const double* edge;
  double* P;
  // mode 3 (level-2 back substitution from the level-2 operators)
  const double* XT;
  const double* bars;
  const double* ops2;
  int recw2;
  // the level-1 operators: a back substitution or root also writes NP, the
  // six projections of its x that the level-1 back substitutions of its
  // neighbours i -+ 2 read (A_{i+2} x_i, B_{i-2} x_i), at NP[side][i / 4][c][6]
  const double* ops1;
  int recw1;
  double* NP;
  int write_x;     // 0: only P and NP (no finer dense level reads this x)
};

template <int WP>
__global__ __launch_bounds__(128) void k_fr_step(const double* __restrict__ fac,
                                                 double* __restrict__ Z, FrStep a) {
  constexpr int PP = WP * WP, RB = WP / 4, EW = 2 * WP + 2;
  __shared__ __attribute__((aligned(16))) double sL[3 * PP];   // L_t(r, k) at t PP + r WP + k
  __shared__ double sQ[6 * WP];   // A_{i+2} (3 rows), B_{i-2} (3 rows), wp each (0 if absent)
  __shared__ double sD[7 * WP];   // mode 3: DW_0..DW_6
  const int side = blockIdx.z;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int g = lane >> 4, q = lane & 15;
  const int64_t T = gridDim.x;
  int64_t x = blockIdx.x;
  if ((T & 7) == 0) x = (x & 7) * (T >> 3) + (x >> 3);
  const int64_t p = a.mode == 2 ? 0 : 2 * x + (a.mode == 0 ? 0 : 1);
  const int64_t i = p * a.s;
  const int w = a.w;
  const bool has_prev = a.mode != 2 && p >= 1, has_next = a.mode != 2 && p + 1 < a.n;
  // ---- matrices: reduction: -, del_{p-1}, gam_{p+1}, L_t(r, k) = M_t(k, r)
  // (a straight copy of the column-major blocks); back substitution / root:
  // Dinv_p, gam_p, del_p, L_t(r, k) = M_t(r, k) (transposed while staged)
  const double* src[3];
  if (a.mode == 0) {
    src[0] = nullptr;
    src[1] = has_prev ? fac + fr_fac(side, a.H, i - a.s, WP) + 2 * PP : nullptr;
    src[2] = has_next ? fac + fr_fac(side, a.H, i + a.s, WP) + PP : nullptr;
  } else {
    const double* base = fac + fr_fac(side, a.H, i, WP);
    src[0] = a.mode == 3 ? nullptr : base;
    src[1] = has_prev ? base + PP : nullptr;
    src[2] = has_next ? base + 2 * PP : nullptr;
  }
  if (a.mode == 3) {
    const int64_t n2 = (((a.H + 1) / 2) + 1) / 2;
    const double* R = a.ops2 + ((int64_t)side * n2 + i / 4) * a.recw2;
    for (int e = tid; e < 7 * WP; e += 128) sD[e] = R[e];
  }
  if (a.mode != 0 && a.NP) {
    const int64_t n1 = (a.H + 1) / 2;
    for (int e = tid; e < 6 * WP; e += 128) {
      const int h = e / (3 * WP), k = e % (3 * WP);
      const int64_t nb = h == 0 ? i + 2 : i - 2;   // A from row i + 2, B from row i - 2
      sQ[e] = (nb >= 0 && nb < a.H)
                  ? a.ops1[((int64_t)side * n1 + nb / 2) * a.recw1 + (h == 0 ? 0 : 3 * WP) + k]
                  : 0.0;
    }
  }
  constexpr int NM = (3 * PP / 2 + 127) / 128;
  double2 mv[NM];
#pragma unroll
  for (int it = 0; it < NM; ++it) {
    const int e = 2 * (tid + 128 * it), t = e / PP;
    mv[it] = (t < 3 && src[t]) ? *reinterpret_cast<const double2*>(src[t] + (e - t * PP))
                               : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int it = 0; it < NM; ++it) {
    const int e = 2 * (tid + 128 * it), t = e / PP;
    if (t >= 3) continue;
    const int rk = e - t * PP;
    if (a.mode == 0) {
      *reinterpret_cast<double2*>(sL + e) = mv[it];
    } else {
      const int r = rk % WP, k = rk / WP;   // storage (r, k), (r + 1, k)
      sL[t * PP + r * WP + k] = mv[it].x;
      sL[t * PP + (r + 1) * WP + k] = mv[it].y;
    }
  }
  __syncthreads();
  int col[2];
  bool cok[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    col[u] = blockIdx.y * 64 + wv * 32 + q + 16 * u;
    cok[u] = col[u] < a.m;
  }
  auto rhs = [&](int64_t row, int c) {
    return Z + fr_rhs(side, a.H, row, a.m, WP) + (int64_t)c * WP;
  };
  // acc(rr, u) += sign sum_k L_t(g RB + rr, k) v(k, u)
  double acc[RB][2];
  auto product = [&](int t, int64_t row, double sign) {
    constexpr int NC = WP / 4;
    const double* L = sL + t * PP + g * RB * WP;
    const double* sp0 = rhs(row, cok[0] ? col[0] : 0);
    const double* sp1 = rhs(row, cok[1] ? col[1] : 0);
    // every load of the right-hand side first (all in flight together) ...
    double v[NC][4][2];
#pragma unroll
    for (int kc = 0; kc < NC; ++kc)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double2 t0 = cok[0] ? *reinterpret_cast<const double2*>(sp0 + 4 * kc + 2 * h)
                                  : make_double2(0.0, 0.0);
        const double2 t1 = cok[1] ? *reinterpret_cast<const double2*>(sp1 + 4 * kc + 2 * h)
                                  : make_double2(0.0, 0.0);
        v[kc][2 * h][0] = t0.x;
        v[kc][2 * h + 1][0] = t0.y;
        v[kc][2 * h][1] = t1.x;
        v[kc][2 * h + 1][1] = t1.y;
      }
    // ... then the products chunk by chunk, the LDS reads of a chunk held
    // back to it (the compiler barrier keeps them from all being hoisted
    // into registers at once)
#pragma unroll
    for (int kc = 0; kc < NC; ++kc) {
      asm volatile("" ::: "memory");
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) {
        const double2 m01 = *reinterpret_cast<const double2*>(L + rr * WP + 4 * kc);
        const double2 m23 = *reinterpret_cast<const double2*>(L + rr * WP + 4 * kc + 2);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          double d = m01.x * v[kc][0][u];
          d = fma(m01.y, v[kc][1][u], d);
          d = fma(m23.x, v[kc][2][u], d);
          d = fma(m23.y, v[kc][3][u], d);
          acc[rr][u] = fma(sign, d, acc[rr][u]);
        }
      }
    }
    asm volatile("" ::: "memory");
  };
  if (a.mode == 0) {
    // acc = b_p on the lane's rows
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const double* sp = rhs(i, cok[u] ? col[u] : 0) + g * RB;
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) acc[rr][u] = cok[u] ? sp[rr] : 0.0;
    }
    if (has_prev) product(1, i - a.s, -1.0);
    if (has_next) product(2, i + a.s, -1.0);
  } else {
    if (a.mode == 3) {
      // acc = sum_d g_{i+d-3} DW_d on the lane's rows
      double gv[7][2];
#pragma unroll
      for (int d = 0; d < 7; ++d)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int64_t j = i + d - 3;
          gv[d][u] = (cok[u] && j >= 0 && j < a.H) ? a.bars[3 * j + side] * a.XT[j * a.m + col[u]]
                                                   : 0.0;
        }
#pragma unroll
      for (int rr = 0; rr < RB; ++rr)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          double t = 0.0;
#pragma unroll
          for (int d = 0; d < 7; ++d) t = fma(sD[d * WP + g * RB + rr], gv[d][u], t);
          acc[rr][u] = t;
        }
    } else {
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) acc[rr][0] = acc[rr][1] = 0.0;
      product(0, i, 1.0);
    }
    if (has_prev) product(1, i - a.s, -1.0);
    if (has_next) product(2, i + a.s, -1.0);
  }
  // results: x (or the reduced b) of the lane's rows to Z
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    if (!cok[u] || (a.mode != 0 && !a.write_x)) continue;
    double* dp = rhs(i, col[u]) + g * RB;
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) dp[rr] = acc[rr][u];
  }
  if (a.mode == 0) return;
  // P of row i and, with the level-1 operators, NP: partial sums over the
  // lane's rows, summed over the four row groups (lanes q, q + 16, q + 32,
  // q + 48 of the wave) with cross-lane exchanges
  const double* Ed = i >= 1 ? a.edge + EW * ((int64_t)side * a.H + i - 1) + WP : nullptr;
  const double* Eg = i + 1 < a.H ? a.edge + EW * ((int64_t)side * a.H + i + 1) : nullptr;
  const bool np = a.NP != nullptr;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    double pv[9];
#pragma unroll
    for (int h = 0; h < 9; ++h) pv[h] = 0.0;
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int r = g * RB + rr;
      const double xv = acc[rr][u];
      if (r == w - 1) pv[0] = xv;
      if (Ed) pv[1] = fma(Ed[r], xv, pv[1]);
      if (Eg) pv[2] = fma(Eg[r], xv, pv[2]);
      if (np)
#pragma unroll
        for (int h = 0; h < 6; ++h) pv[3 + h] = fma(sQ[h * WP + r], xv, pv[3 + h]);
    }
#pragma unroll
    for (int h = 0; h < 9; ++h) {
      pv[h] += __shfl_xor(pv[h], 16);
      pv[h] += __shfl_xor(pv[h], 32);
    }
    const int c = blockIdx.y * 64 + wv * 32 + q + 16 * u;
    if (g == 0 && c < a.m) {
      const int64_t Hh = (a.H + 1) / 2;
      double* dst = a.P + (((int64_t)side * a.m + c) * Hh + i / 2) * 4;
      *reinterpret_cast<double2*>(dst) = make_double2(pv[0], pv[1]);
      *reinterpret_cast<double2*>(dst + 2) = make_double2(pv[2], 0.0);
      if (np) {
        const int64_t Hq = (a.H + 3) / 4;
        double* dn = a.NP + ((((int64_t)side * Hq + i / 4) * a.m) + c) * 6;
        *reinterpret_cast<double2*>(dn) = make_double2(pv[3], pv[4]);
        *reinterpret_cast<double2*>(dn + 2) = make_double2(pv[5], pv[6]);
        *reinterpret_cast<double2*>(dn + 4) = make_double2(pv[7], pv[8]);
      }
    }
  }
}

// Level-0 back substitution of the column next to the middle, fused with the
// output: per grid row i and column c,
//   x_i(w-1) = Dinv_i(w-1, w-1) g_i - gam_i(w-1, :) x_{i-1} - del_i(w-1, :) x_{i+1}
// for rows eliminated at level 0 (odd i, or the only row; the two products
// come from P of the even neighbours), x_i(w-1) from P otherwise, and
//   (A x)_i = (B33 x)_i - cL_i x^L_i(w-1) - cR_i x^R_i(w-1).
template <int WP>
__global__ __launch_bounds__(256) void k_fr_out(const double* X, int64_t ldx, double* Y,
                                                int64_t ldy, int m, const double* edge,
                                                const double* bars, const double* P, int64_t H) {
  constexpr int EW = 2 * WP + 2;
  // one thread per row and column, rows fastest (contiguous x, y and P)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= H) return;
  const int64_t Hh = (H + 1) / 2;
  const double xi = X[i + (int64_t)c * ldx];
  const double cL = bars[3 * i], cR = bars[3 * i + 1];
  const double up = i >= 1 ? bars[3 * (i - 1) + 2] : 0.0, dn = bars[3 * i + 2];
  double y = (cL + cR + up + dn) * xi;
  if (i >= 1) y = fma(-up, X[i - 1 + (int64_t)c * ldx], y);
  if (i + 1 < H) y = fma(-dn, X[i + 1 + (int64_t)c * ldx], y);
  const bool elim0 = (i & 1) || H == 1;
  for (int side = 0; side < 2; ++side) {
    const double cl = side == 0 ? cL : cR;
    const double* Ps = P + ((int64_t)side * m + c) * Hh * 4;
    double xs;
    if (elim0) {
      xs = edge[EW * ((int64_t)side * H + i) + 2 * WP] * (cl * xi);
      if (i >= 1) xs -= Ps[((i - 1) / 2) * 4 + 2];
      if (i + 1 < H) xs -= Ps[((i + 1) / 2) * 4 + 1];
    } else {
      xs = Ps[(i / 2) * 4];
    }
    y = fma(-cl, xs, y);
  }
  Y[i + (int64_t)c * ldy] = y;
}

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// Columns per pass of the apply (bounds the right-hand-side workspace).
constexpr int FR_COLS = 128;

static size_t fr_z_bytes(const hm_frontal_s* f, int m) {
  return ((size_t)(2 * f->H * m * f->wp) * sizeof(double) + 255) / 256 * 256;
}

static size_t fr_p_bytes(const hm_frontal_s* f, int m) {
  return ((size_t)(2 * ((f->H + 1) / 2) * m * 4) * sizeof(double) + 255) / 256 * 256;
}

static size_t fr_xt_bytes(const hm_frontal_s* f, int m) {
  return ((size_t)(f->H * m) * sizeof(double) + 255) / 256 * 256;
}

static size_t fr_np_bytes(const hm_frontal_s* f, int m) {
  return (size_t)(2 * ((f->H + 3) / 4) * m * 6) * sizeof(double);
}

// XT[j m + c] = X(j, c): 64 x 64 tiles through LDS, both sides contiguous.
__global__ __launch_bounds__(256) void k_fr_transpose(const double* X, int64_t ldx, int64_t H,
                                                      int m, double* XT) {
  __shared__ double t[64][65];
  const int64_t j0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
  for (int cc = ty; cc < 64; cc += 4)
    if (c0 + cc < m && j0 + tx < H) t[cc][tx] = X[j0 + tx + (int64_t)(c0 + cc) * ldx];
  __syncthreads();
  for (int jj = ty; jj < 64; jj += 4)
    if (j0 + jj < H && c0 + tx < m) XT[(j0 + jj) * m + c0 + tx] = t[tx][jj];
}

template <int WP>
static void frontal_apply_wp(const hm_frontal_s* f, int64_t ncols, const double* X, int64_t ldx,
                             double* Y, int64_t ldy, void* work, hipStream_t s) {
  const int64_t H = f->H;
  const int w = f->w;
  const double* fac = f->fac.as<double>();
  const double* edge = f->edge.as<double>();
  const double* bars = f->bars.as<double>();
  for (int64_t c0 = 0; c0 < ncols; c0 += FR_COLS) {
    const int m = (int)std::min<int64_t>(FR_COLS, ncols - c0);
    double* Z = static_cast<double*>(work);
    double* P = reinterpret_cast<double*>(static_cast<char*>(work) + fr_z_bytes(f, m));
    double* XT =
        reinterpret_cast<double*>(static_cast<char*>(work) + fr_z_bytes(f, m) + fr_p_bytes(f, m));
    double* NPw = reinterpret_cast<double*>(static_cast<char*>(work) + fr_z_bytes(f, m) +
                                            fr_p_bytes(f, m) + fr_xt_bytes(f, m));
    const double* Xc = X + c0 * ldx;
    double* Yc = Y + c0 * ldy;
    if (f->levels >= 1) {
      hipLaunchKernelGGL(k_fr_transpose, dim3((unsigned)((H + 63) / 64), (m + 63) / 64),
                         dim3(256), 0, s, Xc, ldx, H, m, XT);
      KCHK();
      const unsigned groups = (unsigned)((m + 63) / 64);
      const double* ops = f->ops.as<double>();
      auto step = [&](int mode, int64_t stride, int64_t n, int64_t rows, int write_x = 1) {
        if (rows <= 0) return;
        FrStep a{H,   stride, n,    w,         m,       mode,   edge,   P,
                 XT,  bars,   f->ops2.as<double>(), f->recw2, f->ops.as<double>(), f->recw,
                 f->levels >= 2 ? NPw : nullptr, write_x};
        hipLaunchKernelGGL(k_fr_step<WP>, dim3((unsigned)rows, groups, 2), dim3(128), 0, s, fac,
                           Z, a);
        KCHK();
      };
      // n_l: active rows of level l
      const int L = f->levels;
      std::vector<int64_t> nl(L + 1);
      nl[0] = H;
      for (int l = 1; l <= L; ++l) nl[l] = (nl[l - 1] + 1) / 2;
      const int64_t n1 = nl[1];
      if (L == 1) {
        hipLaunchKernelGGL(k_fr_l1bwd<WP>, dim3(1, groups, 2), dim3(64), 0, s, ops, f->recw, NPw,
                           P, XT, bars, H, m, 1);
        KCHK();
      } else if (L == 2) {
        hipLaunchKernelGGL((k_fr_gfwd<WP, 7>), dim3((unsigned)((n1 + 1) / 2), groups, 2), dim3(64),
                           0, s, ops, f->recw, n1, (int64_t)4, Z, XT, bars, H, m);
        KCHK();
        step(2, (int64_t)1 << L, 1, 1);
        hipLaunchKernelGGL(k_fr_l1bwd<WP>, dim3((unsigned)(n1 / 2), groups, 2), dim3(64), 0, s,
                           ops, f->recw, NPw, P, XT, bars, H, m, 0);
        KCHK();
      } else {
        // levels 1 and 2 through their operators, 3 .. L - 1 and the root dense
        const int64_t n2 = nl[2];
        hipLaunchKernelGGL((k_fr_gfwd<WP, 15>), dim3((unsigned)((n2 + 1) / 2), groups, 2),
                           dim3(64), 0, s, f->ops2.as<double>(), f->recw2, n2, (int64_t)8, Z, XT,
                           bars, H, m);
        KCHK();
        for (int l = 3; l < L; ++l) step(0, (int64_t)1 << l, nl[l], (nl[l] + 1) / 2);
        step(2, (int64_t)1 << L, 1, 1);
        for (int l = L - 1; l >= 3; --l) step(1, (int64_t)1 << l, nl[l], nl[l] / 2);
        step(3, (int64_t)4, n2, n2 / 2, 0);
        hipLaunchKernelGGL(k_fr_l1bwd<WP>, dim3((unsigned)(n1 / 2), groups, 2), dim3(64), 0, s,
                           ops, f->recw, NPw, P, XT, bars, H, m, 0);
        KCHK();
      }
    }
    hipLaunchKernelGGL(k_fr_out<WP>, dim3(nblk(H), m), dim3(256), 0, s, Xc, ldx, Yc, ldy, m,
                       edge, bars, P, H);
    KCHK();
  }
}

void frontal_apply(const hm_frontal_s* f, int64_t ncols, const double* X, int64_t ldx, double* Y,
                   int64_t ldy, void* work, hipStream_t s) {
  switch (f->wp) {
    case 4: frontal_apply_wp<4>(f, ncols, X, ldx, Y, ldy, work, s); break;
    case 8: frontal_apply_wp<8>(f, ncols, X, ldx, Y, ldy, work, s); break;
    case 12: frontal_apply_wp<12>(f, ncols, X, ldx, Y, ldy, work, s); break;
    case 16: frontal_apply_wp<16>(f, ncols, X, ldx, Y, ldy, work, s); break;
    case 20: frontal_apply_wp<20>(f, ncols, X, ldx, Y, ldy, work, s); break;
    case 24: frontal_apply_wp<24>(f, ncols, X, ldx, Y, ldy, work, s); break;
    case 28: frontal_apply_wp<28>(f, ncols, X, ldx, Y, ldy, work, s); break;
    case 32: frontal_apply_wp<32>(f, ncols, X, ldx, Y, ldy, work, s); break;
    default: HM_THROW(HM_ERR_ARG, "frontal: padded side width %d", f->wp);
  }
}

size_t frontal_work_bytes(const hm_frontal_s* f, int64_t ncols) {
  const int m = (int)std::min<int64_t>(FR_COLS, std::max<int64_t>(ncols, 1));
  return fr_z_bytes(f, m) + fr_p_bytes(f, m) + fr_xt_bytes(f, m) + fr_np_bytes(f, m);
}

int64_t frontal_n(const hm_frontal_s* f) { return f->H; }

}  // namespace hm

using namespace hm;

extern "C" {

int hm_frontal_create(int64_t height, int32_t width, const double* ch, const double* cv,
                      void* stream, hm_frontal** out) {
  try {
    set_error("%s", "");
    StreamScope scope(stream);
    if (!out) HM_THROW(HM_ERR_ARG, "frontal: out is NULL");
    *out = nullptr;
    if (height < 1 || width < 3 || width % 2 == 0)
      HM_THROW(HM_ERR_ARG, "frontal: height >= 1 and an odd width >= 3 (got %lld, %d)",
               (long long)height, width);
    if ((width - 1) / 2 > FR_WMAX)
      HM_THROW(HM_ERR_UNSUPPORTED, "frontal: width %d > %d", width, 2 * FR_WMAX + 1);
    if (height > ((int64_t)1 << 31)) HM_THROW(HM_ERR_UNSUPPORTED, "frontal: height > 2^31");
    if (!ch || (height > 1 && !cv)) HM_THROW(HM_ERR_ARG, "frontal: conductivities are NULL");
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<hm_frontal_s> F(new hm_frontal_s);
    const int64_t H = height;
    const int w = (width - 1) / 2;
    F->H = H;
    F->W = width;
    F->w = w;
    F->wp = (w + 3) / 4 * 4;
    int L = 0;
    for (int64_t n = H; n > 1; n = (n + 1) / 2) ++L;
    F->levels = L;
    const int64_t per = (int64_t)w * w;
    F->fac = DevBuf((size_t)(2 * H * 3 * F->wp * F->wp) * sizeof(double));
    F->bars = DevBuf((size_t)(3 * H) * sizeof(double));
    F->edge = DevBuf((size_t)(2 * H * (2 * F->wp + 2)) * sizeof(double));
    F->recw = 7 * F->wp + 12;
    F->ops = DevBuf((size_t)(2 * ((H + 1) / 2) * F->recw) * sizeof(double));
    const int64_t n2 = ((H + 1) / 2 + 1) / 2;
    F->recw2 = 15 * F->wp;
    if (L >= 3) F->ops2 = DevBuf((size_t)(2 * n2 * F->recw2) * sizeof(double));
    DevBuf Dw((size_t)(2 * H * per) * sizeof(double)), Cw((size_t)(2 * H * per) * sizeof(double));
    DevBuf bad(256);
    HIPCHK(hipMemsetAsync(bad.p, 0, 16, s));
    hipLaunchKernelGGL(k_fr_assemble, dim3(nblk(std::max<int64_t>(2 * H * per, H))), dim3(256), 0,
                       s, ch, cv, H, width, w, Dw.as<double>(), Cw.as<double>(),
                       F->bars.as<double>());
    KCHK();
    int64_t n = H;
    for (int l = 0; l < L; ++l) {
      const int64_t st = (int64_t)1 << l;
      hipLaunchKernelGGL(k_fr_elim, dim3((unsigned)(n / 2), 1, 2), dim3(256), 0, s,
                         Dw.as<double>(), Cw.as<double>(), F->fac.as<double>(),
                         F->edge.as<double>(), H, w, F->wp, st, n, 0, bad.as<int32_t>());
      KCHK();
      hipLaunchKernelGGL(k_fr_reduce, dim3((unsigned)((n + 1) / 2), 1, 2), dim3(256), 0, s,
                         Dw.as<double>(), Cw.as<double>(), F->fac.as<double>(), H, w, F->wp, st,
                         n);
      KCHK();
      n = (n + 1) / 2;
    }
    hipLaunchKernelGGL(k_fr_elim, dim3(1, 1, 2), dim3(256), 0, s, Dw.as<double>(),
                       Cw.as<double>(), F->fac.as<double>(), F->edge.as<double>(), H, w, F->wp,
                       (int64_t)1 << L, 1, 1, bad.as<int32_t>());
    KCHK();
    if (L >= 1) {
      hipLaunchKernelGGL(k_fr_lvl1_ops, dim3((unsigned)((H + 1) / 2), 1, 2), dim3(256), 0, s,
                         F->fac.as<double>(), F->edge.as<double>(), F->ops.as<double>(), H, w,
                         F->wp, F->recw);
      KCHK();
    }
    if (L >= 3) {
      hipLaunchKernelGGL(k_fr_lvl2_ops, dim3((unsigned)n2, 1, 2), dim3(256), 0, s,
                         F->fac.as<double>(), F->ops.as<double>(), F->recw, F->ops2.as<double>(),
                         H, w, F->wp, F->recw2);
      KCHK();
    }
    int hb[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(hb, bad.p, 16, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hb[0])
      HM_THROW(HM_ERR_SINGULAR, "frontal: a non-positive pivot (conductivities must be > 0)");
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

int hm_frontal_apply(const hm_frontal* f, int64_t ncols, const double* X, int64_t ldx, double* Y,
                     int64_t ldy, void* stream) {
  try {
    set_error("%s", "");
    StreamScope scope(stream);
    if (!f || ncols < 0 || (ncols > 0 && (!X || !Y)))
      HM_THROW(HM_ERR_ARG, "frontal apply: bad arguments");
    if (ldx < f->H || ldy < f->H) HM_THROW(HM_ERR_ARG, "frontal apply: ld < n");
    if (ncols == 0) return HM_OK;
    hipStream_t s = (hipStream_t)stream;
    DevBuf work(frontal_work_bytes(f, ncols));
    frontal_apply(f, ncols, X, ldx, Y, ldy, work.p, s);
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

void hm_frontal_free(hm_frontal* f) { delete f; }

}  // extern "C"
