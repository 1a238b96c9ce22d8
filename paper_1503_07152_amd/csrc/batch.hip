// Many independent HBS compressions in one level-synchronous pass: the
// instances form one forest over a concatenated row space, so each level's
// test matrices, operator samples, subtraction, node factorisations and ID
// steps of all instances run in the same batched launches.  HBS operators of
// the instances are merged into one block-diagonal forest operator; the
// result is split back into one handle per instance.
#include <algorithm>
#include <numeric>

#include "handle.h"

namespace hm {

// Copy of row arrays (U, V, D) or per-node blocks (transfers 2R x R, sibling
// matrices R x R) between handles of different padded rank; FP64 source,
// FP64 or FP32 destination.
struct CopyDesc {
  const double* src;
  void* dst;
  int64_t src_ld, dst_ld;  // row arrays: leading dimensions
  int64_t count;           // row arrays: rows; block arrays: blocks
  int32_t cols;            // row arrays: columns copied
  int32_t Rs, Rd;          // block arrays: source / destination padded rank
  int32_t kind;            // 0 rows, 1 transfer blocks, 2 square blocks
  int32_t dst_f32;         // destination stored in FP32
};

__device__ __forceinline__ void copy_store(const CopyDesc& d, int64_t i, double v) {
  if (d.dst_f32) static_cast<float*>(d.dst)[i] = (float)v;
  else static_cast<double*>(d.dst)[i] = v;
}

__global__ void k_copy(const CopyDesc* descs) {
  const CopyDesc d = descs[blockIdx.y];
  if (d.kind == 0) {
    const int64_t total = d.count * d.cols;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
      const int64_t i = e % d.count, j = e / d.count;
      copy_store(d, i + j * d.dst_ld, d.src[i + j * d.src_ld]);
    }
    return;
  }
  const int Rm = min(d.Rs, d.Rd);
  const int rows = d.kind == 1 ? 2 * Rm : Rm;
  const int64_t per = (int64_t)rows * Rm;
  const int64_t total = d.count * per;
  const int64_t sblk = d.kind == 1 ? 2ll * d.Rs * d.Rs : (int64_t)d.Rs * d.Rs;
  const int64_t dblk = d.kind == 1 ? 2ll * d.Rd * d.Rd : (int64_t)d.Rd * d.Rd;
  const int sld = d.kind == 1 ? 2 * d.Rs : d.Rs;
  const int dld = d.kind == 1 ? 2 * d.Rd : d.Rd;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / per;
    const int r = (int)(e % per) % rows, c = (int)((e % per) / rows);
    const int rs = (d.kind == 1 && r >= Rm) ? d.Rs + (r - Rm) : r;
    const int rd = (d.kind == 1 && r >= Rm) ? d.Rd + (r - Rm) : r;
    copy_store(d, b * dblk + rd + (int64_t)c * dld, d.src[b * sblk + rs + (int64_t)c * sld]);
  }
}

static void run_copies(const std::vector<CopyDesc>& v, Keeper& kp, hipStream_t s) {
  if (v.empty()) return;
  const CopyDesc* d = kp.put(v, s);
  hipLaunchKernelGGL(k_copy, dim3(256, (unsigned)v.size()), dim3(256), 0, s, d);
  KCHK();
}

static void finish_lists(hm_hbs_s* h, hipStream_t s) {
  const Forest& f = h->f;
  std::vector<int> mvec(f.inst.size());
  for (size_t i = 0; i < f.inst.size(); ++i) mvec[i] = f.inst[i].L;
  build_apply_lists(f, mvec, h->full, s);
  h->grad_leaves = upload(f.leaves, s);
  std::vector<int32_t> all(f.nodes.size());
  std::iota(all.begin(), all.end(), 0);
  h->grad_nodes = upload(all, s);
}

// Block-diagonal forest operator from single-tree FP64 handles.
hm_hbs_s* merge_hbs(const std::vector<const hm_hbs_s*>& hs, hipStream_t s) {
  std::unique_ptr<hm_hbs_s> h(new hm_hbs_s());
  int R = 0;
  for (auto* x : hs) R = std::max(R, x->R);
  for (auto* x : hs) {
    const Instance& in = x->f.inst[0];
    forest_add_tree(h->f, in.n, in.leaf, x->R, x->R, 0, 0.0, 0);
  }
  forest_finish(h->f);
  const Forest& f = h->f;
  const int64_t N = f.n_total;
  const int nn = (int)f.nodes.size();
  h->R = R;
  h->dtype = HM_F64;
  h->d_nodes = upload(f.nodes, s);
  h->d_inst = upload(f.inst, s);
  h->U = DevBuf((size_t)N * R * 8);
  h->V = DevBuf((size_t)N * R * 8);
  h->Ut = DevBuf((size_t)nn * 2 * R * R * 8);
  h->Vt = DevBuf((size_t)nn * 2 * R * R * 8);
  h->B = DevBuf((size_t)nn * R * R * 8);
  h->D = DevBuf((size_t)N * f.nmax * 8);
  for (DevBuf* b : {&h->U, &h->V, &h->Ut, &h->Vt, &h->B, &h->D})
    HIPCHK(hipMemsetAsync(b->p, 0, b->bytes, s));
  std::vector<CopyDesc> cd;
  for (size_t i = 0; i < hs.size(); ++i) {
    const hm_hbs_s* x = hs[i];
    const Instance& in = f.inst[i];
    const int64_t n = in.n;
    const int64_t nni = (int64_t)x->f.nodes.size();
    const int64_t r0 = in.row0;
    const int64_t g0 = in.root;
    cd.push_back({x->U.as<double>(), h->U.as<double>() + r0, n, N, n, x->R, 0, 0, 0, 0});
    cd.push_back({x->V.as<double>(), h->V.as<double>() + r0, n, N, n, x->R, 0, 0, 0, 0});
    cd.push_back({x->D.as<double>(), h->D.as<double>() + r0, n, N, n, x->f.nmax, 0, 0, 0, 0});
    cd.push_back({x->Ut.as<double>(), h->Ut.as<double>() + g0 * 2 * R * R, 0, 0, nni, 0, x->R, R,
                  1, 0});
    cd.push_back({x->Vt.as<double>(), h->Vt.as<double>() + g0 * 2 * R * R, 0, 0, nni, 0, x->R, R,
                  1, 0});
    cd.push_back({x->B.as<double>(), h->B.as<double>() + g0 * R * R, 0, 0, nni, 0, x->R, R, 2, 0});
  }
  Keeper kp;
  run_copies(cd, kp, s);
  finish_lists(h.get(), s);
  HIPCHK(hipStreamSynchronize(s));
  h->rank_u.assign(nn, R);
  h->rank_v.assign(nn, R);
  return h.release();
}

// One handle per instance of a forest handle, each at padded rank r_i.
std::vector<hm_hbs_s*> split_hbs(const hm_hbs_s* src, hipStream_t s, int dtype) {
  const Forest& F = src->f;
  const int R = src->R;
  const size_t es = dtype == HM_F32 ? 4 : 8;
  const int32_t f32 = dtype == HM_F32 ? 1 : 0;
  std::vector<std::unique_ptr<hm_hbs_s>> out;
  std::vector<CopyDesc> cd;
  for (size_t i = 0; i < F.inst.size(); ++i) {
    const Instance& in = F.inst[i];
    std::unique_ptr<hm_hbs_s> h(new hm_hbs_s());
    forest_add_tree(h->f, in.n, in.leaf, in.r, in.k, in.p, in.tol, in.seed);
    forest_finish(h->f);
    const Forest& f = h->f;
    const int64_t n = in.n;
    const int nn = (int)f.nodes.size();
    const int Ri = in.r;
    h->R = Ri;
    h->dtype = dtype;
    h->is_id = src->is_id;
    h->d_nodes = upload(f.nodes, s);
    h->d_inst = upload(f.inst, s);
    h->U = DevBuf((size_t)n * Ri * es);
    h->V = DevBuf((size_t)n * Ri * es);
    h->Ut = DevBuf((size_t)nn * 2 * Ri * Ri * es);
    h->Vt = DevBuf((size_t)nn * 2 * Ri * Ri * es);
    h->B = DevBuf((size_t)nn * Ri * Ri * es);
    h->D = DevBuf((size_t)n * f.nmax * es);
    for (DevBuf* b : {&h->Ut, &h->Vt, &h->B}) HIPCHK(hipMemsetAsync(b->p, 0, b->bytes, s));
    const int64_t r0 = in.row0, g0 = in.root;
    cd.push_back({src->U.as<double>() + r0, h->U.p, F.n_total, n, n, Ri, 0, 0, 0, f32});
    cd.push_back({src->V.as<double>() + r0, h->V.p, F.n_total, n, n, Ri, 0, 0, 0, f32});
    cd.push_back({src->D.as<double>() + r0, h->D.p, F.n_total, n, n, f.nmax, 0, 0, 0, f32});
    cd.push_back({src->Ut.as<double>() + g0 * 2 * R * R, h->Ut.p, 0, 0, nn, 0, R, Ri, 1, f32});
    cd.push_back({src->Vt.as<double>() + g0 * 2 * R * R, h->Vt.p, 0, 0, nn, 0, R, Ri, 1, f32});
    cd.push_back({src->B.as<double>() + g0 * R * R, h->B.p, 0, 0, nn, 0, R, Ri, 2, f32});
    h->rank_u.assign(src->rank_u.begin() + g0, src->rank_u.begin() + g0 + nn);
    h->rank_v.assign(src->rank_v.begin() + g0, src->rank_v.begin() + g0 + nn);
    h->skel_in.assign((size_t)nn * Ri, -1);
    h->skel_out.assign((size_t)nn * Ri, -1);
    for (int g = 0; g < nn; ++g)
      for (int j = 0; j < Ri; ++j) {
        h->skel_in[(size_t)g * Ri + j] = src->skel_in[(size_t)(g0 + g) * R + j];
        h->skel_out[(size_t)g * Ri + j] = src->skel_out[(size_t)(g0 + g) * R + j];
      }
    finish_lists(h.get(), s);
    out.push_back(std::move(h));
  }
  Keeper kp;
  run_copies(cd, kp, s);
  HIPCHK(hipStreamSynchronize(s));
  std::vector<hm_hbs_s*> res;
  for (auto& h : out) {
    finish_handle_info(h.get());
    h->info.t_compress_ms = src->info.t_compress_ms;
    h->info.t_operator_ms = src->info.t_operator_ms;
    h->info.operator_calls = src->info.operator_calls;
    h->info.saturated = src->info.saturated;
    h->info.jacobi_sweeps = src->info.jacobi_sweeps;
    const Instance& in = h->f.inst[0];
    h->info.sample_columns = (int64_t)4 * in.r * in.L + in.nmax;
    res.push_back(h.release());
  }
  return res;
}

// Copy of a handle with its generators in another storage type (FP64 <->
// FP32); structure, ranks, skeletons and statistics are kept.
hm_hbs_s* convert_hbs(const hm_hbs_s* src, int dtype, hipStream_t s, bool sync) {
  std::unique_ptr<hm_hbs_s> h(new hm_hbs_s());
  h->f = src->f;
  h->R = src->R;
  h->dtype = dtype;
  h->is_id = src->is_id;
  h->d_nodes = upload(h->f.nodes, s);
  h->d_inst = upload(h->f.inst, s);
  const size_t es = dtype == HM_F32 ? 4 : 8;
  const size_t ses = src->dtype == HM_F32 ? 4 : 8;
  for (auto pr : {std::make_pair(&src->U, &h->U), std::make_pair(&src->V, &h->V),
                  std::make_pair(&src->Ut, &h->Ut), std::make_pair(&src->Vt, &h->Vt),
                  std::make_pair(&src->B, &h->B), std::make_pair(&src->D, &h->D)}) {
    const int64_t cnt = (int64_t)(pr.first->bytes / ses);
    *pr.second = DevBuf(std::max<size_t>((size_t)cnt * es, 256));
    launch_convert(pr.first->p, src->dtype, cnt, pr.second->p, dtype, cnt, cnt, 1, s);
  }
  h->rank_u = src->rank_u;
  h->rank_v = src->rank_v;
  h->skel_in = src->skel_in;
  h->skel_out = src->skel_out;
  finish_lists(h.get(), s);
  if (sync) HIPCHK(hipStreamSynchronize(s));
  h->info = src->info;
  h->info.dtype = dtype;
  return h.release();
}

}  // namespace hm
