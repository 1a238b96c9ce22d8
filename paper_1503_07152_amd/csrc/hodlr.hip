// Host orchestration of the randomized HODLR compression (Fig. 2, SVD
// variant of eq. SVDtogetV / SVDtogetB) and the HODLR apply.
#include <algorithm>
#include <chrono>

#include "handle.h"

namespace hm {

// y = beta y + alpha A^(m) x  (levels 1..m of the HODLR form), or its adjoint
static void hodlr_truncated(const hm_hodlr_s* h, int m, bool adjoint, int c, const double* X,
                            int64_t ldx, double* Y, int64_t ldy, double alpha, double beta,
                            Workspace& ws, hipStream_t s) {
  const int64_t N = h->f.n_total;
  bool first = true;
  for (int l = 1; l <= m; ++l) {
    const ApplyLists& al = h->lvl[l];
    ws.ensure(apply_work_bytes<double>(h->f, al, h->R, c), s);
    hodlr_level_apply<double>(h->d_nodes.as<Node>(), al, h->U[l - 1].as<double>(),
                              h->V[l - 1].as<double>(), N, h->R, h->S.as<double>(), adjoint, c, X,
                              ldx, Y, ldy, alpha, first ? beta : 1.0, ws.base(),
                              h->f.nodes.size(), s);
    first = false;
  }
  if (first && beta != 1.0) {
    // nothing applied: Y = beta Y
    if (beta == 0.0) launch_fill(Y, N, c, ldy, 0.0, s);
    else HM_THROW(HM_ERR_ARG, "hodlr_truncated: unsupported beta");
  }
}

hm_hodlr_s* hodlr_compress_forest(Forest f, OpRunner& op, hipStream_t s, int* status) {
  auto t0 = std::chrono::steady_clock::now();
  forest_finish(f);
  if (f.inst.size() != 1) HM_THROW(HM_ERR_ARG, "HODLR compression takes one instance");
  std::unique_ptr<hm_hodlr_s> h(new hm_hodlr_s());
  const Instance in = f.inst[0];
  const int R = in.r;
  const int64_t N = f.n_total;
  const int nn = (int)f.nodes.size();
  const int L = in.L;
  const int nmax = f.nmax;
  h->R = R;
  h->f = f;
  h->d_nodes = upload(f.nodes, s);
  h->d_inst = upload(f.inst, s);
  const Node* dn = h->d_nodes.as<Node>();
  const Instance* di = h->d_inst.as<Instance>();
  Keeper kp;
  Workspace ws_svd, ws_apply;
  const int W = std::max(2 * R, nmax);
  DevBuf Om((size_t)N * W * 8), Y((size_t)N * W * 8), M((size_t)N * R * 8), Uq((size_t)N * R * 8);
  DevBuf Xr((size_t)nn * 2 * R * R * 8), flag(16), rk(nn * 4 + 16);
  h->S = DevBuf((size_t)nn * R * 8);
  HIPCHK(hipMemsetAsync(h->S.p, 0, h->S.bytes, s));
  HIPCHK(hipMemsetAsync(Xr.p, 0, Xr.bytes, s));
  HIPCHK(hipMemsetAsync(flag.p, 0, 16, s));
  HIPCHK(hipMemsetAsync(rk.p, 0, rk.bytes, s));
  h->lvl.resize(L + 1);
  for (int l = 1; l <= L; ++l) {
    std::vector<int> mv{l};
    build_apply_lists(f, mv, h->lvl[l], s);
  }
  double* om = Om.as<double>();
  double* y = Y.as<double>();
  for (int l = 0; l < L; ++l) {
    const std::vector<int32_t>& kids = f.level[l + 1];
    int64_t maxr = 0;
    for (int g : kids) maxr = std::max<int64_t>(maxr, f.nodes[g].hi - f.nodes[g].lo);
    const int32_t* dk = kp.put(kids, s);
    const int nk = (int)kids.size();
    // Y = A [Omega_2 | Omega_1] - A^(l) [Omega_2 | Omega_1]
    launch_gauss_masked(dn, di, dk, nk, maxr, l, R, om, N, s);
    op.apply(false, N, 2 * R, om, N, y, N);
    launch_nonfinite_check(y, N, 2 * R, N, flag.as<int>(), s);
    hodlr_truncated(h.get(), l, false, 2 * R, om, N, y, N, -1.0, 1.0, ws_apply, s);
    // U = qr(Y block)
    launch_build_node_block(dn, di, dk, nk, maxr, R, y, N, nullptr, N, nullptr, M.as<double>(), N,
                            s, 1);
    std::vector<SvdJob> jobs;
    for (int g : kids) {
      const Node& nd = f.nodes[g];
      jobs.push_back({g, (int)(nd.hi - nd.lo), R, R, nd.lo, f.inst[nd.inst].k,
                      sample_rank_eta(op.op.kind == HM_OP_KERNEL ? op.op.sample_dtype : HM_F64)});
    }
    launch_fill(Uq.as<double>(), N, R, N, 0.0, s);
    node_svd(jobs, M.as<double>(), N, Uq.as<double>(), N, nullptr, nullptr, R, true, ws_svd, kp, s);
    // Z = A^* [Psi_2 | Psi_1] - (A^(l))^* [...]
    launch_mask_basis(dn, di, dk, nk, maxr, R, Uq.as<double>(), N, om, N, s);
    op.apply(true, N, 2 * R, om, N, y, N);
    launch_nonfinite_check(y, N, 2 * R, N, flag.as<int>(), s);
    hodlr_truncated(h.get(), l, true, 2 * R, om, N, y, N, -1.0, 1.0, ws_apply, s);
    // [V_a, B_ba, U^_b] = svd(Z_1(I_a, :), eps); U_b <- U_b U^_b
    launch_build_node_block(dn, di, dk, nk, maxr, R, y, N, nullptr, N, nullptr, M.as<double>(), N,
                            s, 1);
    h->U.emplace_back((size_t)N * R * 8);
    h->V.emplace_back((size_t)N * R * 8);
    double* Ul = h->U.back().as<double>();
    double* Vl = h->V.back().as<double>();
    launch_fill(Vl, N, R, N, 0.0, s);
    node_svd(jobs, M.as<double>(), N, Vl, N, h->S.as<double>(), Xr.as<double>(), R, false, ws_svd,
             kp, s);
    launch_truncate(dn, di, dk, nk, maxr, R, Vl, N, h->S.as<double>(), Xr.as<double>(),
                    rk.as<int32_t>(), flag.as<int32_t>() + 1, s);
    launch_node_nn(dn, dk, nk, maxr, R, R, Uq.as<double>(), N, Xr.as<double>(), 2 * R * R, 2 * R,
                   Ul, N, s, 1);
  }
  // diagonal blocks
  h->D = DevBuf((size_t)N * nmax * 8);
  {
    const int32_t* dl = kp.put(f.leaves, s);
    int64_t maxl = 0;
    for (int g : f.leaves) maxl = std::max<int64_t>(maxl, f.nodes[g].hi - f.nodes[g].lo);
    launch_block_eye(dn, dl, (int)f.leaves.size(), maxl, nmax, om, N, s);
    op.apply(false, N, nmax, om, N, h->D.as<double>(), N);
    launch_nonfinite_check(h->D.as<double>(), N, nmax, N, flag.as<int>(), s);
    hodlr_truncated(h.get(), L, false, nmax, om, N, h->D.as<double>(), N, -1.0, 1.0, ws_apply, s);
    launch_zero_dpad(dn, dl, (int)f.leaves.size(), maxl, nmax, h->D.as<double>(), N, s);
  }
  std::vector<int> full{L};
  build_apply_lists(f, full, h->full, s);
  int hflag[4] = {0, 0, 0, 0};
  h->rank.assign(nn, 0);
  read_d2h({{hflag, flag.p, 16}, {h->rank.data(), rk.p, (size_t)nn * 4}}, s);
  if (hflag[0]) HM_THROW(HM_ERR_NONFINITE, "operator samples contain NaN or Inf");
  hm_info& inf = h->info;
  inf.n = N;
  inf.leaf_size = in.leaf;
  inf.levels = L;
  inf.rank_pad = R;
  inf.is_id = 0;
  inf.dtype = HM_F64;
  int mx = 0, mn = 1 << 30;
  int64_t st = 0;
  for (int g = 0; g < nn; ++g) {
    const Node& nd = f.nodes[g];
    if (nd.left < 0) st += (nd.hi - nd.lo) * (nd.hi - nd.lo);
    if (nd.parent < 0) continue;
    const int k = h->rank[g];
    mx = std::max(mx, k);
    mn = std::min(mn, k);
    // V_v (n_v x k) and U_sib (n_sib x k) of the block A(I_sib, I_v), and its k diagonal entries
    const Node& sb = f.nodes[nd.sib];
    st += (int64_t)k * ((nd.hi - nd.lo) + (sb.hi - sb.lo)) + k;
  }
  inf.max_rank = mx;
  inf.min_rank = mn == (1 << 30) ? 0 : mn;
  inf.storage_reals = st;
  inf.sample_columns = op.columns;
  inf.operator_calls = op.calls;
  inf.saturated = hflag[1];
  inf.adapt_rounds = 1;
  inf.err_estimate = -1.0;
  inf.t_operator_ms = op.elapsed_ms();
  inf.t_compress_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *status = hflag[1] > 0 ? HM_WARN_RANK_SATURATED : HM_OK;
  return h.release();
}

void hodlr_apply_full(const hm_hodlr_s* h, bool adjoint, int c, const double* X, int64_t ldx,
                      double* Y, int64_t ldy, hipStream_t s) {
  Workspace ws;
  const int64_t N = h->f.n_total;
  // D x (or D^* x) through the HBS leaf kernel with no basis term
  HbsView<double> hv;
  hv.Ulong = nullptr; hv.Vlong = nullptr; hv.ldl = N; hv.R = 0;
  hv.D = h->D.as<double>(); hv.ldd = N;
  ws.ensure(apply_work_bytes<double>(h->f, h->full, 1, c) + 4096, s);
  // The full-apply lists have the leaves as frontier; with R = 0 only D acts.
  apply_forest<double>(h->d_nodes.as<Node>(), h->full, hv, adjoint, c, X, ldx, Y, ldy, 1.0, 0.0,
                       ws.base(), h->f.nodes.size(), s);
  hodlr_truncated(h, h->f.inst[0].L, adjoint, c, X, ldx, Y, ldy, 1.0, 1.0, ws, s);
  HIPCHK(hipStreamSynchronize(s));
}

}  // namespace hm
