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
// the middle (B13 x) and read only that column of the solution, so level 0 is
// taken apart: its reduction builds the level-1 right-hand side straight from
// x (a rank-one update per row) and its back substitution computes only that
// column, fused with B33 x and the sum that forms A x.
#include <algorithm>

#include "handle.h"

struct hm_frontal_s {
  int64_t H = 0;
  int W = 0, w = 0;
  int levels = 0;        // reduction levels: n_levels == 1
  hm::DevBuf fac;        // [side][row][Dinv | gam | del], w x w column-major each
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

// Eliminated rows of level l (odd p; p = 0 at the root): Dinv, gam, del.
__global__ __launch_bounds__(256) void k_fr_elim(const double* Dw, const double* Cw, double* fac,
                                                 int64_t H, int w, int64_t s, int64_t n, int root,
                                                 int32_t* bad) {
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
  double* F = fac + 3 * fr_blk(side, H, i, w);
  for (int e = tid; e < per; e += 256) {
    const int r = e % w, c = e / w;
    double g = 0.0, d = 0.0;
    for (int k = 0; k < w; ++k) {
      const double a = A[r + k * LD];
      g = fma(a, Cm[c + k * LD], g);   // Dinv C_{q-1}^T
      d = fma(a, Cp[k + c * LD], d);   // Dinv C_q
    }
    F[e] = A[r + c * LD];
    F[per + e] = g;
    F[2 * per + e] = d;
  }
  if (fail && tid == 0) atomicOr(bad, 1);
}

// Kept rows of level l (even p): the reduced D_p and C_p.
__global__ __launch_bounds__(256) void k_fr_reduce(double* Dw, double* Cw, const double* fac,
                                                   int64_t H, int w, int64_t s, int64_t n) {
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
    Dm[r + k * LD] = has_prev ? fac[3 * fr_blk(side, H, i - s, w) + 2 * per + e] : 0.0;
    Cs[r + k * LD] = Cw[fr_blk(side, H, i, w) + e];
    Gp[r + k * LD] = has_next ? fac[3 * fr_blk(side, H, i + s, w) + per + e] : 0.0;
    Dp[r + k * LD] = has_next ? fac[3 * fr_blk(side, H, i + s, w) + 2 * per + e] : 0.0;
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

// ---- solve ----------------------------------------------------------------------
// Right-hand sides Z[side][row][column][j] (w per column, contiguous per row).
__device__ inline int64_t fr_rhs(int side, int64_t H, int64_t i, int m, int w) {
  return (((int64_t)side * H + i) * m) * w;
}

// Level-0 reduction: the level-1 right-hand side of every even row p from the
// sparse level-0 one (b_i = g_i e_{w-1}, g_i = c_link(i) x_i):
//   b_p = g_p e_{w-1} - g_{p-1} del_{p-1}^T e_{w-1} - g_{p+1} gam_{p+1}^T e_{w-1}.
__global__ __launch_bounds__(256) void k_fr_fwd0(const double* X, int64_t ldx, int m,
                                                 const double* fac, const double* bars,
                                                 double* Z, int64_t H, int w) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t neven = (H + 1) / 2;
  const int64_t per_row = (int64_t)m * w;
  if (e >= 2 * neven * per_row) return;
  const int side = (int)(e / (neven * per_row));
  const int64_t p = 2 * ((e / per_row) % neven);
  const int c = (int)((e % per_row) / w), j = (int)(e % w);
  const int per = w * w;
  auto g = [&](int64_t i) { return bars[3 * i + side] * X[i + (int64_t)c * ldx]; };
  double b = j == w - 1 ? g(p) : 0.0;
  if (p >= 1) b = fma(-fac[3 * fr_blk(side, H, p - 1, w) + 2 * per + (w - 1) + j * w], g(p - 1), b);
  if (p + 1 < H) b = fma(-fac[3 * fr_blk(side, H, p + 1, w) + per + (w - 1) + j * w], g(p + 1), b);
  Z[fr_rhs(side, H, p, m, w) + (int64_t)c * w + j] = b;
}

// One level l >= 1 of the solve on a column chunk of one row (blockIdx.x: the
// row's index among the rows the step writes, blockIdx.y: the chunk,
// blockIdx.z: the side).  mode 0 reduction (even p): b_p -= del_{p-1}^T
// b_{p-1} + gam_{p+1}^T b_{p+1}; mode 1 back substitution (odd p):
// x_p = Dinv_p b_p - gam_p x_{p-1} - del_p x_{p+1}; mode 2 root: x_0 = Dinv_0 b_0.
// Thread (rg, cg) holds rows 4rg..4rg+3 and columns 2cg, 2cg+1 of the chunk;
// operands staged in LDS (matrices transposed for the reduction so that both
// modes read M(r, k) at k LDM + r), the result written back through LDS so
// the stores are contiguous.
struct FrStep {
  int64_t H, s, n;
  int w, m, cw;        // cw: chunk width (columns per workgroup, even)
  int mode;
};

__global__ __launch_bounds__(256) void k_fr_step(const double* fac, double* Z, FrStep a) {
  extern __shared__ double lds[];
  const int w = a.w, RG = (w + 3) / 4, LDM = 4 * RG, LDV = a.cw + 2;
  double* sM = lds;                    // 3 matrices, LDM x w each (k LDM + r)
  double* sV = lds + 3 * LDM * w;      // 3 chunks, w x LDV each (k LDV + c)
  const int side = blockIdx.z;
  const int tid = threadIdx.x;
  const int64_t p = a.mode == 2 ? 0 : 2 * (int64_t)blockIdx.x + (a.mode == 1 ? 1 : 0);
  const int64_t i = p * a.s;
  const int c0 = blockIdx.y * a.cw;
  const int cw = min(a.cw, a.m - c0);
  const int per = w * w;
  const bool has_prev = a.mode != 2 && p >= 1, has_next = a.mode != 2 && p + 1 < a.n;
  // operands: t = 0 the row itself, 1 its previous, 2 its next active row
  const int64_t rows[3] = {i, i - a.s, i + a.s};
  const bool live[3] = {true, has_prev, has_next};
  const double* Fs = fac + 3 * fr_blk(side, a.H, 0, w);
  // matrices: reduction: -, del_{p-1}^T, gam_{p+1}^T; back substitution:
  // Dinv_p, gam_p, del_p (all of row p)
  for (int e = tid; e < 3 * per; e += 256) {
    const int t = e / per, rk = e % per, r = rk % w, k = rk / w;
    double v = 0.0;
    if (a.mode == 0) {
      if (t == 1 && has_prev) v = Fs[3 * (i - a.s) * per + 2 * per + k + r * w];
      if (t == 2 && has_next) v = Fs[3 * (i + a.s) * per + per + k + r * w];
    } else if (t == 0 || (t == 1 && has_prev) || (t == 2 && has_next)) {
      v = Fs[3 * i * per + t * per + rk];
    }
    sM[t * LDM * w + k * LDM + r] = v;
  }
  for (int t = 0; t < 3; ++t) {
    if (!live[t]) continue;
    const double* src = Z + fr_rhs(side, a.H, rows[t], a.m, w) + (int64_t)c0 * w;
    for (int e = tid; e < cw * w; e += 256) {
      const int c = e / w, k = e % w;
      sV[t * w * LDV + k * LDV + c] = src[e];
    }
  }
  __syncthreads();
  const int rg = tid % RG, cg = tid / RG;
  const bool act = cg * 2 < cw;
  double acc[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  if (act) {
    for (int t = 0; t < 3; ++t) {
      if (!live[t]) continue;
      const double sign = t == 0 ? 1.0 : -1.0;
      const double* M = sM + t * LDM * w + 4 * rg;
      const double* V = sV + t * w * LDV + 2 * cg;
      if (t == 0 && a.mode == 0) {
        for (int u = 0; u < 4; ++u)
          if (4 * rg + u < w) {
            acc[u][0] = V[(4 * rg + u) * LDV];
            acc[u][1] = V[(4 * rg + u) * LDV + 1];
          }
        continue;
      }
      for (int k = 0; k < w; ++k) {
        const double2 v = *reinterpret_cast<const double2*>(V + k * LDV);
        const double2 m01 = *reinterpret_cast<const double2*>(M + k * LDM);
        const double2 m23 = *reinterpret_cast<const double2*>(M + k * LDM + 2);
        const double mm[4] = {sign * m01.x, sign * m01.y, sign * m23.x, sign * m23.y};
        for (int u = 0; u < 4; ++u) {
          acc[u][0] = fma(mm[u], v.x, acc[u][0]);
          acc[u][1] = fma(mm[u], v.y, acc[u][1]);
        }
      }
    }
  }
  __syncthreads();
  // result through the first chunk's LDS, then contiguous stores
  if (act)
    for (int u = 0; u < 4; ++u)
      if (4 * rg + u < w) {
        sV[(4 * rg + u) * LDV + 2 * cg] = acc[u][0];
        sV[(4 * rg + u) * LDV + 2 * cg + 1] = acc[u][1];
      }
  __syncthreads();
  double* dst = Z + fr_rhs(side, a.H, i, a.m, w) + (int64_t)c0 * w;
  for (int e = tid; e < cw * w; e += 256) {
    const int c = e / w, k = e % w;
    dst[e] = sV[k * LDV + c];
  }
}

// Level-0 back substitution of the column next to the middle, fused with the
// output: per grid row i and column c,
//   x_i(w-1) = Dinv_i(w-1, w-1) g_i - gam_i(w-1, :) x_{i-1} - del_i(w-1, :) x_{i+1}
// for rows eliminated at level 0 (odd i, or the only row), x_i(w-1) from the
// solve otherwise, and
//   (A x)_i = (B33 x)_i - cL_i x^L_i(w-1) - cR_i x^R_i(w-1).
__global__ __launch_bounds__(256) void k_fr_out(const double* X, int64_t ldx, double* Y,
                                                int64_t ldy, int m, const double* fac,
                                                const double* bars, const double* Z, int64_t H,
                                                int w) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= H * m) return;
  const int64_t i = e / m;
  const int c = (int)(e % m);
  const int per = w * w;
  const double xi = X[i + (int64_t)c * ldx];
  const double cL = bars[3 * i], cR = bars[3 * i + 1];
  const double up = i >= 1 ? bars[3 * (i - 1) + 2] : 0.0, dn = bars[3 * i + 2];
  double y = (cL + cR + up + dn) * xi;
  if (i >= 1) y = fma(-up, X[i - 1 + (int64_t)c * ldx], y);
  if (i + 1 < H) y = fma(-dn, X[i + 1 + (int64_t)c * ldx], y);
  const bool elim0 = (i & 1) || H == 1;
  for (int side = 0; side < 2; ++side) {
    const double cl = side == 0 ? cL : cR;
    double xs;
    if (elim0) {
      const double* F = fac + 3 * fr_blk(side, H, i, w);
      xs = F[(w - 1) + (w - 1) * w] * (cl * xi);
      if (i >= 1) {
        const double* zp = Z + fr_rhs(side, H, i - 1, m, w) + (int64_t)c * w;
        for (int j = 0; j < w; ++j) xs = fma(-F[per + (w - 1) + j * w], zp[j], xs);
      }
      if (i + 1 < H) {
        const double* zn = Z + fr_rhs(side, H, i + 1, m, w) + (int64_t)c * w;
        for (int j = 0; j < w; ++j) xs = fma(-F[2 * per + (w - 1) + j * w], zn[j], xs);
      }
    } else {
      xs = Z[fr_rhs(side, H, i, m, w) + (int64_t)c * w + (w - 1)];
    }
    y = fma(-cl, xs, y);
  }
  Y[i + (int64_t)c * ldy] = y;
}

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

static size_t fr_step_lds(int w, int cw) {
  const int RG = (w + 3) / 4;
  return (size_t)(3 * 4 * RG * w + 3 * w * (cw + 2)) * sizeof(double);
}

// Chunk width of k_fr_step: two columns per thread over 256 / RG threads,
// fewer if the operands would pass 64 KB of LDS.
static int fr_chunk(int w) {
  int cw = 2 * (256 / ((w + 3) / 4));
  while (cw > 2 && fr_step_lds(w, cw) > 65536) cw -= 2;
  return cw;
}

// Columns per pass of the apply (bounds the right-hand-side workspace).
constexpr int FR_COLS = 128;

void frontal_apply(const hm_frontal_s* f, int64_t ncols, const double* X, int64_t ldx, double* Y,
                   int64_t ldy, void* work, hipStream_t s) {
  const int64_t H = f->H;
  const int w = f->w;
  const double* fac = f->fac.as<double>();
  const double* bars = f->bars.as<double>();
  double* Z = static_cast<double*>(work);
  const int cwmax = fr_chunk(w);
  const size_t lds = fr_step_lds(w, cwmax);
  for (int64_t c0 = 0; c0 < ncols; c0 += FR_COLS) {
    const int m = (int)std::min<int64_t>(FR_COLS, ncols - c0);
    const double* Xc = X + c0 * ldx;
    double* Yc = Y + c0 * ldy;
    if (f->levels >= 1) {
      const int64_t neven = (H + 1) / 2;
      hipLaunchKernelGGL(k_fr_fwd0, dim3(nblk(2 * neven * m * w)), dim3(256), 0, s, Xc, ldx, m,
                         fac, bars, Z, H, w);
      KCHK();
      const int cw = std::min(cwmax, m + (m & 1));
      const unsigned chunks = (unsigned)((m + cw - 1) / cw);
      auto step = [&](int mode, int64_t stride, int64_t n, int64_t rows) {
        if (rows <= 0) return;
        FrStep a{H, stride, n, w, m, cw, mode};
        hipLaunchKernelGGL(k_fr_step, dim3((unsigned)rows, chunks, 2), dim3(256), lds, s, fac, Z,
                           a);
        KCHK();
      };
      // n_l: active rows of level l
      std::vector<int64_t> nl(f->levels + 1);
      nl[0] = H;
      for (int l = 1; l <= f->levels; ++l) nl[l] = (nl[l - 1] + 1) / 2;
      for (int l = 1; l < f->levels; ++l) step(0, (int64_t)1 << l, nl[l], (nl[l] + 1) / 2);
      step(2, (int64_t)1 << f->levels, 1, 1);
      for (int l = f->levels - 1; l >= 1; --l) step(1, (int64_t)1 << l, nl[l], nl[l] / 2);
    }
    hipLaunchKernelGGL(k_fr_out, dim3(nblk(H * m)), dim3(256), 0, s, Xc, ldx, Yc, ldy, m, fac,
                       bars, Z, H, w);
    KCHK();
  }
}

size_t frontal_work_bytes(const hm_frontal_s* f, int64_t ncols) {
  const int64_t m = std::min<int64_t>(FR_COLS, std::max<int64_t>(ncols, 1));
  return (size_t)(2 * f->H * m * f->w) * sizeof(double);
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
    int L = 0;
    for (int64_t n = H; n > 1; n = (n + 1) / 2) ++L;
    F->levels = L;
    const int64_t per = (int64_t)w * w;
    F->fac = DevBuf((size_t)(2 * H * 3 * per) * sizeof(double));
    F->bars = DevBuf((size_t)(3 * H) * sizeof(double));
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
                         Dw.as<double>(), Cw.as<double>(), F->fac.as<double>(), H, w, st, n, 0,
                         bad.as<int32_t>());
      KCHK();
      hipLaunchKernelGGL(k_fr_reduce, dim3((unsigned)((n + 1) / 2), 1, 2), dim3(256), 0, s,
                         Dw.as<double>(), Cw.as<double>(), F->fac.as<double>(), H, w, st, n);
      KCHK();
      n = (n + 1) / 2;
    }
    hipLaunchKernelGGL(k_fr_elim, dim3(1, 1, 2), dim3(256), 0, s, Dw.as<double>(),
                       Cw.as<double>(), F->fac.as<double>(), H, w, (int64_t)1 << L, 1, 1,
                       bad.as<int32_t>());
    KCHK();
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
