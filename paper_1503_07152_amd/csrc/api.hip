// extern "C" entry points of libhbspeel (declared in include/hbspeel.h):
// argument validation, exception-to-status translation, handle management.
#include <chrono>
#include <cmath>
#include <cstring>

#include "grad.h"
#include "handle.h"

using namespace hm;

namespace {

template <class F>
int guarded(F&& f) {
  try {
    set_error("%s", "");
    return f();
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

void check_options(const hm_options* o) {
  if (!o) HM_THROW(HM_ERR_ARG, "options is NULL");
  if (o->n < 1) HM_THROW(HM_ERR_ARG, "n = %lld < 1", (long long)o->n);
  if (o->leaf_size < 1) HM_THROW(HM_ERR_ARG, "leaf_size = %lld < 1", (long long)o->leaf_size);
  if (o->rank < 1) HM_THROW(HM_ERR_ARG, "rank = %d < 1", o->rank);
  if (o->oversample < 0) HM_THROW(HM_ERR_ARG, "oversample = %d < 0", o->oversample);
  if (!(o->tol >= 0.0 && o->tol < 1.0)) HM_THROW(HM_ERR_ARG, "tol = %g outside [0, 1)", o->tol);
  if (o->rank + o->oversample > HM_MAX_SAMPLES)
    HM_THROW(HM_ERR_UNSUPPORTED, "rank + oversample = %d > %d", o->rank + o->oversample,
             HM_MAX_SAMPLES);
  if (o->n > ((int64_t)1 << 31)) HM_THROW(HM_ERR_UNSUPPORTED, "n > 2^31");
  if (o->store_dtype != HM_F64 && o->store_dtype != HM_F32)
    HM_THROW(HM_ERR_ARG, "store_dtype = %d (HM_F64 or HM_F32)", o->store_dtype);
  if (o->n > o->leaf_size && o->leaf_size > 256)
    HM_THROW(HM_ERR_UNSUPPORTED, "leaf_size %lld > 256", (long long)o->leaf_size);
}

void check_operator(const hm_operator* op, int64_t n, bool builtin_only) {
  if (!op) HM_THROW(HM_ERR_ARG, "operator is NULL");
  switch (op->kind) {
    case HM_OP_CALLBACK:
      if (builtin_only) HM_THROW(HM_ERR_ARG, "callback operators are not allowed here");
      if (!op->fn) HM_THROW(HM_ERR_ARG, "callback operator without function");
      if (op->sample_dtype != HM_F64 && op->sample_dtype != HM_F32 && op->sample_dtype != HM_BF16)
        HM_THROW(HM_ERR_ARG, "bad sample dtype %d", op->sample_dtype);
      break;
    case HM_OP_KERNEL:
      if (!op->points) HM_THROW(HM_ERR_ARG, "kernel operator without points");
      if (op->kernel_id != HM_KERNEL_LOG && op->kernel_id != HM_KERNEL_NEAR)
        HM_THROW(HM_ERR_ARG, "unknown kernel id %d", op->kernel_id);
      if (op->sample_dtype != HM_F64 && op->sample_dtype != HM_F32 && op->sample_dtype != HM_BF16)
        HM_THROW(HM_ERR_ARG, "bad sample dtype %d", op->sample_dtype);
      break;
    case HM_OP_DENSE:
      if (!op->dense || op->ld < n) HM_THROW(HM_ERR_ARG, "dense operator: null or ld < n");
      break;
    case HM_OP_HBS:
      if (!op->hbs || op->hbs->f.n_total != n || op->hbs->dtype != HM_F64)
        HM_THROW(HM_ERR_ARG, "HBS operator: null, size mismatch or not FP64");
      break;
    case HM_OP_HBS_PRODUCT:
      if (builtin_only) HM_THROW(HM_ERR_ARG, "HBS product operators are not allowed here");
      for (const hm_hbs* x : {op->hbs, op->hbs2})
        if (!x || x->f.n_total != n || x->dtype != HM_F64 || x->f.inst.size() != 1)
          HM_THROW(HM_ERR_ARG, "HBS product operator: null, size mismatch or not FP64");
      break;
    case HM_OP_FRONTAL:
      if (builtin_only) HM_THROW(HM_ERR_ARG, "frontal operators are not allowed here");
      if (!op->frontal || frontal_n(op->frontal) != n)
        HM_THROW(HM_ERR_ARG, "frontal operator: null or height != n");
      break;
    default:
      HM_THROW(HM_ERR_ARG, "unknown operator kind %d", op->kind);
  }
}

Forest single_forest(const hm_options* o) {
  Forest f;
  forest_add_tree(f, o->n, o->leaf_size, o->rank + o->oversample,
                  o->tol > 0.0 ? o->rank : o->rank, o->oversample, o->tol, o->seed);
  return f;
}

size_t dsize(int dtype) { return dtype == HM_F32 ? 4 : 8; }

}  // namespace

template <class T>
static void backward_impl(const hm_hbs* h, int c, const T* x, int64_t ldx, const T* gy,
                          int64_t ldgy, T* gx, int64_t ldgx, T* gU, T* gV, T* gUt, T* gVt, T* gB,
                          T* gD, hipStream_t s) {
  const Forest& f = h->f;
  const int64_t N = f.n_total;
  const int R = h->R;
  const int nn = (int)f.nodes.size();
  const size_t wb = apply_work_bytes<T>(f, h->full, R, c);
  StreamBuf sb1(wb, s), sb2(wb, s);
  void *w1 = sb1.p, *w2 = sb2.p;
  const HbsView<T> hv = h->view<T>();
  // forward expansions (outgoing qh, incoming uh) of x, and the adjoint apply
  // of gy: gx with its expansions g(uh) (upward) and g(qh) (downward); the
  // two sets of tree sweeps share their launches
  apply_forest_pair<T>(h->d_nodes.as<Node>(), h->full, hv, c, x, ldx, w1, gy, ldgy, gx, ldgx, w2,
                       nn, s);
  const size_t es = sizeof(T);
  // gUt, gVt, gB: every block is written by the node-gradient kernel
  int64_t maxl = 0, minl = INT64_MAX;
  for (int g : f.leaves) {
    maxl = std::max<int64_t>(maxl, f.nodes[g].hi - f.nodes[g].lo);
    minl = std::min<int64_t>(minl, f.nodes[g].hi - f.nodes[g].lo);
  }
  if (gD && minl < f.nmax) HIPCHK(hipMemsetAsync(gD, 0, (size_t)N * f.nmax * es, s));
  if (f.inst[0].L == 0) {
    if (gU) HIPCHK(hipMemsetAsync(gU, 0, (size_t)N * R * es, s));
    if (gV) HIPCHK(hipMemsetAsync(gV, 0, (size_t)N * R * es, s));
  }
  const T* QH = static_cast<const T*>(w1);
  const T* UH = QH + (size_t)R * c * nn;
  const T* GU = static_cast<const T*>(w2);
  const T* GQ = GU + (size_t)R * c * nn;
  launch_grad<T>(h->d_nodes.as<Node>(), h->grad_leaves.as<int32_t>(), (int)f.leaves.size(), maxl,
                 f.nmax, h->grad_nodes.as<int32_t>(), nn, R, c, x, ldx, gy, ldgy, QH, UH, GU, GQ,
                 gU, gV, gUt, gVt, gB, gD, N, N, s);
}

extern "C" {

const char* hm_last_error(void) { return get_error(); }
const char* hm_version(void) { return "hbspeel 0.1 (gfx950)"; }

int hm_set_allocator(hm_alloc_fn alloc, hm_free_fn free, void* ctx) {
  return guarded([&] {
    if ((alloc == nullptr) != (free == nullptr))
      HM_THROW(HM_ERR_ARG, "set_allocator: alloc and free must both be set or both be NULL");
    AllocHook hk;
    hk.alloc = alloc;
    hk.free = free;
    hk.ctx = alloc ? ctx : nullptr;
    set_alloc_hook(hk);
    return HM_OK;
  });
}

int hm_release_cached_memory(void) {
  return guarded([&] {
    release_cached_memory();
    return HM_OK;
  });
}

int hm_gauss(uint64_t seed, int32_t level, int32_t phase, int64_t row0, int64_t nrows,
             int32_t ncols, double* out, int64_t ld, void* stream) {
  return guarded([&] {
    StreamScope scope(stream);
    if (!out || nrows < 0 || ncols < 0 || ld < nrows || row0 < 0)
      HM_THROW(HM_ERR_ARG, "hm_gauss: bad arguments");
    launch_gauss_raw(seed, level, phase, row0, nrows, ncols, out, ld, (hipStream_t)stream);
    return HM_OK;
  });
}

int hm_operator_apply(const hm_operator* op, int64_t n, int32_t adjoint, int64_t ncols,
                      const double* X, int64_t ldx, double* Y, int64_t ldy, void* stream) {
  return guarded([&] {
    StreamScope scope(stream);
    if (n < 1 || ncols < 0 || !X || !Y || ldx < n || ldy < n)
      HM_THROW(HM_ERR_ARG, "operator_apply: bad arguments");
    check_operator(op, n, false);
    if (ncols == 0) return HM_OK;
    OpRunner run;
    run.op = *op;
    run.hbs = op->kind == HM_OP_HBS ? op->hbs : nullptr;
    run.s = (hipStream_t)stream;
    // built-in samplers take up to sampler_max_cols columns per pass over A
    // (the runner splits wider blocks); other operators get 128 at a time
    const int64_t chunk =
        op->kind == HM_OP_KERNEL ? sampler_max_cols(op->sample_dtype == HM_BF16 ? 2 : 0) : 128;
    for (int64_t c0 = 0; c0 < ncols; c0 += chunk) {
      const int c = (int)std::min<int64_t>(chunk, ncols - c0);
      run.apply(adjoint != 0, n, c, X + c0 * ldx, ldx, Y + c0 * ldy, ldy);
    }
    return HM_OK;
  });
}

int hbs_compress(const hm_options* opts, const hm_operator* op, void* stream, hm_hbs** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    StreamScope scope(stream);
    if (!out) HM_THROW(HM_ERR_ARG, "out is NULL");
    check_options(opts);
    check_operator(op, opts->n, false);
    OpRunner run;
    run.op = *op;
    run.hbs = op->kind == HM_OP_HBS ? op->hbs : nullptr;
    run.s = (hipStream_t)stream;
    std::vector<OpRunner*> ops{&run};
    int status = HM_OK;
    std::unique_ptr<hm_hbs_s> h(hbs_compress_forest(single_forest(opts), ops, opts->flags,
                                                    (hipStream_t)stream, &status));
    if (opts->store_dtype == HM_F32) {
      // factors computed in FP64, stored in FP32
      const double t = h->info.t_compress_ms;
      h.reset(convert_hbs(h.get(), HM_F32, (hipStream_t)stream));
      h->info.t_compress_ms = t;
    }
    *out = h.release();
    return status;
  });
}

// Posterior error estimate E of Sec. 5 for the handle h of the operator run:
// max over 10 probe columns w (phase 1 of the Gaussian stream keyed by seed)
// of |A w - A_H w| / |A w|.
static double estimate_E(const hm_hbs_s* h, OpRunner& run, uint64_t seed, hipStream_t s) {
  const int64_t n = h->f.n_total;
  const int c = 10;
  DevBuf W((size_t)n * c * 8), Ya((size_t)n * c * 8), Yh((size_t)n * c * 8), nr(2 * c * 8);
  launch_gauss_raw(seed, 0, 1, 0, n, c, W.as<double>(), n, s);
  run.apply(false, n, c, W.as<double>(), n, Ya.as<double>(), n);
  StreamBuf w(apply_work_bytes<double>(h->f, h->full, h->R, c), s);
  apply_forest<double>(h->d_nodes.as<Node>(), h->full, h->view<double>(), false, c, W.as<double>(),
                       n, Yh.as<double>(), n, 1.0, 0.0, w.p, h->f.nodes.size(), s);
  launch_col_err2(Ya.as<double>(), n, Yh.as<double>(), n, n, c, nr.as<double>(), s);
  double hn[2 * c];
  HIPCHK(hipMemcpyAsync(hn, nr.p, sizeof(hn), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double E = 0.0;
  for (int j = 0; j < c; ++j) {
    const double e = hn[2 * j + 1] > 0.0 ? std::sqrt(hn[2 * j] / hn[2 * j + 1]) : 0.0;
    E = std::isnan(e) ? e : std::max(E, e);
    if (std::isnan(E)) break;
  }
  return E;
}

int hbs_compress_adaptive(const hm_options* opts, const hm_operator* op, double e_target,
                          void* stream, hm_hbs** out) {
  if (out) *out = nullptr;
  return guarded([&]() -> int {
    StreamScope scope(stream);
    if (!out) HM_THROW(HM_ERR_ARG, "out is NULL");
    check_options(opts);
    check_operator(op, opts->n, false);
    if (!(opts->tol > 0.0)) HM_THROW(HM_ERR_ARG, "adaptive: tolerance mode (tol > 0) required");
    if (!(e_target > 0.0)) HM_THROW(HM_ERR_ARG, "adaptive: e_target must be positive");
    if (opts->flags & HM_FLAG_ORTHONORMAL)
      HM_THROW(HM_ERR_ARG, "adaptive: ranks are revealed by the HBS-ID sweep");
    hipStream_t s = (hipStream_t)stream;
    hm_options o = *opts;
    std::unique_ptr<hm_hbs_s> h;
    int status = HM_OK, rounds = 0, calls = 0;
    int64_t cols = 0;
    double t_ms = 0.0, op_ms = 0.0, E = 0.0;
    for (;;) {
      OpRunner run;
      run.op = *op;
      run.hbs = op->kind == HM_OP_HBS ? op->hbs : nullptr;
      run.s = s;
      std::vector<OpRunner*> ops{&run};
      h.reset(hbs_compress_forest(single_forest(&o), ops, o.flags, s, &status));
      ++rounds;
      calls += h->info.operator_calls;
      cols += h->info.sample_columns;
      t_ms += h->info.t_compress_ms;
      op_ms += h->info.t_operator_ms;
      E = estimate_E(h.get(), run, o.seed, s);
      const bool ok = status != HM_WARN_RANK_SATURATED && E <= e_target;
      if (ok || o.rank + o.oversample >= HM_MAX_SAMPLES) {
        if (!ok) status = HM_WARN_RANK_SATURATED;
        break;
      }
      o.rank = std::min(2 * o.rank, HM_MAX_SAMPLES - o.oversample);
    }
    h->info.adapt_rounds = rounds;
    h->info.err_estimate = E;
    h->info.operator_calls = calls;
    h->info.sample_columns = cols;
    h->info.t_compress_ms = t_ms;
    h->info.t_operator_ms = op_ms;
    if (o.store_dtype == HM_F32) {
      const hm_info keep = h->info;
      h.reset(convert_hbs(h.get(), HM_F32, s));
      h->info = keep;
      h->info.dtype = HM_F32;
    }
    *out = h.release();
    return status;
  });
}

int hm_autotune(const hm_options* opts, const hm_operator* op, int32_t reps, void* stream,
                hm_tune* out) {
  return guarded([&]() -> int {
    StreamScope scope(stream);
    if (!out || reps < 0) HM_THROW(HM_ERR_ARG, "autotune: bad arguments");
    check_options(opts);
    check_operator(op, opts->n, false);
    hipStream_t s = (hipStream_t)stream;
    Forest f = single_forest(opts);
    forest_finish(f);
    const int R = opts->rank + opts->oversample;
    const bool bf16 = op->kind == HM_OP_KERNEL && op->sample_dtype == HM_BF16;
    const TuneKey key = tune_key(f, bf16, R);
    if (reps == 0) {   // back to the built-in defaults for this shape
      tune_store(key, TuneParams{});
      *out = hm_tune{0, -1, 0, 0, 0.0, 0.0};
      return HM_OK;
    }
    std::vector<TuneParams> cand{TuneParams{}};    // the built-in defaults first
    if (bf16 && f.max_levels > 1) {
      const int cmax = sampler_max_cols(2);
      const int gmax = std::max(1, std::min(f.max_levels, cmax / (2 * R)));
      const int rmax = std::max(0, (cmax - 2 * R) / (2 * R));
      for (int g = 1; g <= gmax; ++g)
        for (int rd = 0; rd <= rmax; ++rd)
          for (int ks : {1, 2, 3, 4, 8}) cand.push_back(TuneParams{g, rd, ks});
    }
    auto run_once = [&](const TuneParams& tp) {
      tune_store(key, tp);
      OpRunner run;
      run.op = *op;
      run.hbs = op->kind == HM_OP_HBS ? op->hbs : nullptr;
      run.s = s;
      std::vector<OpRunner*> ops{&run};
      int status = HM_OK;
      HIPCHK(hipStreamSynchronize(s));
      const auto t0 = std::chrono::steady_clock::now();
      std::unique_ptr<hm_hbs_s> h(hbs_compress_forest(single_forest(opts), ops,
                                                      opts->flags | HM_FLAG_INTERNAL_NO_FALLBACK,
                                                      s, &status));
      return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
          .count();
    };
    (void)run_once(cand[0]);    // first launches, buffer growth
    double best = 0.0, t_def = 0.0;
    size_t bi = 0;
    for (size_t c = 0; c < cand.size(); ++c) {
      double t = 1e300;
      for (int q = 0; q < reps; ++q) t = std::min(t, run_once(cand[c]));
      if (c == 0) t_def = t;
      if (c == 0 || t < best) {
        best = t;
        bi = c;
      }
    }
    tune_store(key, cand[bi]);
    out->gfirst = cand[bi].gfirst;
    out->ride = cand[bi].ride;
    out->ksplit = cand[bi].ksplit;
    out->candidates = (int32_t)cand.size();
    out->t_default_ms = t_def;
    out->t_best_ms = best;
    return HM_OK;
  });
}

int hbs_compress_batched(int32_t count, const hm_options* opts, const hm_operator* ops,
                         void* stream, hm_hbs** outs) {
  if (outs && count > 0)
    for (int i = 0; i < count; ++i) outs[i] = nullptr;
  return guarded([&]() -> int {
    StreamScope scope(stream);
    if (count < 1 || !opts || !ops || !outs) HM_THROW(HM_ERR_ARG, "batched: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    Forest f;
    bool all_hbs = true;
    for (int i = 0; i < count; ++i) {
      check_options(&opts[i]);
      check_operator(&ops[i], opts[i].n, true);
      if (opts[i].flags != opts[0].flags) HM_THROW(HM_ERR_ARG, "batched: flags differ");
      if (opts[i].store_dtype != opts[0].store_dtype)
        HM_THROW(HM_ERR_ARG, "batched: store_dtype differs");
      all_hbs &= ops[i].kind == HM_OP_HBS;
      forest_add_tree(f, opts[i].n, opts[i].leaf_size, opts[i].rank + opts[i].oversample,
                      opts[i].rank, opts[i].oversample, opts[i].tol, opts[i].seed);
    }
    std::unique_ptr<hm_hbs_s> merged;
    std::vector<std::unique_ptr<OpRunner>> runners;
    std::vector<OpRunner*> rp;
    if (all_hbs) {
      std::vector<const hm_hbs_s*> hs;
      for (int i = 0; i < count; ++i) hs.push_back(ops[i].hbs);
      merged.reset(merge_hbs(hs, s));
      runners.emplace_back(new OpRunner());
      runners[0]->op = ops[0];
      runners[0]->hbs = merged.get();
      runners[0]->s = s;
    } else {
      for (int i = 0; i < count; ++i) {
        runners.emplace_back(new OpRunner());
        runners.back()->op = ops[i];
        runners.back()->hbs = ops[i].kind == HM_OP_HBS ? ops[i].hbs : nullptr;
        runners.back()->s = s;
      }
    }
    for (auto& r : runners) rp.push_back(r.get());
    int status = HM_OK;
    std::unique_ptr<hm_hbs_s> res(hbs_compress_forest(f, rp, opts[0].flags, s, &status));
    // factors computed in FP64; each instance's handle stored in store_dtype
    std::vector<hm_hbs_s*> parts = split_hbs(res.get(), s, opts[0].store_dtype);
    for (int i = 0; i < count; ++i) outs[i] = parts[i];
    return status;
  });
}

int hodlr_compress(const hm_options* opts, const hm_operator* op, void* stream, hm_hodlr** out) {
  if (out) *out = nullptr;
  return guarded([&]() -> int {
    StreamScope scope(stream);
    if (!out) HM_THROW(HM_ERR_ARG, "out is NULL");
    check_options(opts);
    check_operator(op, opts->n, false);
    if (opts->store_dtype != HM_F64) HM_THROW(HM_ERR_ARG, "HODLR handles are stored in FP64");
    OpRunner run;
    run.op = *op;
    run.hbs = op->kind == HM_OP_HBS ? op->hbs : nullptr;
    run.s = (hipStream_t)stream;
    int status = HM_OK;
    *out = hodlr_compress_forest(single_forest(opts), run, (hipStream_t)stream, &status);
    return status;
  });
}

static int apply_impl(const hm_hbs* h, bool adjoint, int64_t nrhs, const void* x, int64_t ldx,
                      void* y, int64_t ldy, void* stream) {
  return guarded([&] {
    StreamScope scope(stream);
    if (!h || !x || !y || nrhs < 0) HM_THROW(HM_ERR_ARG, "apply: bad arguments");
    const int64_t n = h->f.n_total;
    if (ldx < n || ldy < n) HM_THROW(HM_ERR_ARG, "apply: ld < n");
    if (nrhs == 0) return HM_OK;
    hipStream_t s = (hipStream_t)stream;
    const int cmax = 128;
    for (int64_t c0 = 0; c0 < nrhs; c0 += cmax) {
      const int c = (int)std::min<int64_t>(cmax, nrhs - c0);
      if (h->dtype == HM_F64) {
        StreamBuf w(apply_work_bytes<double>(h->f, h->full, h->R, c), s);
        apply_forest<double>(h->d_nodes.as<Node>(), h->full, h->view<double>(), adjoint, c,
                             static_cast<const double*>(x) + c0 * ldx, ldx,
                             static_cast<double*>(y) + c0 * ldy, ldy, 1.0, 0.0, w.p,
                             h->f.nodes.size(), s);
      } else {
        StreamBuf w(apply_work_bytes<float>(h->f, h->full, h->R, c), s);
        apply_forest<float>(h->d_nodes.as<Node>(), h->full, h->view<float>(), adjoint, c,
                            static_cast<const float*>(x) + c0 * ldx, ldx,
                            static_cast<float*>(y) + c0 * ldy, ldy, 1.0f, 0.0f, w.p,
                            h->f.nodes.size(), s);
      }
    }
    return HM_OK;
  });
}

int hss_apply(const hm_hbs* h, int64_t nrhs, const void* x, int64_t ldx, void* y, int64_t ldy,
              void* stream) {
  return apply_impl(h, false, nrhs, x, ldx, y, ldy, stream);
}

int hss_apply_adjoint(const hm_hbs* h, int64_t nrhs, const void* x, int64_t ldx, void* y,
                      int64_t ldy, void* stream) {
  return apply_impl(h, true, nrhs, x, ldx, y, ldy, stream);
}

int hm_hbs_from_generators(int64_t n, int64_t leaf_size, int32_t k, int32_t dtype, const void* U,
                           const void* V, const void* Ut, const void* Vt, const void* B,
                           const void* D, void* stream, hm_hbs** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    StreamScope scope(stream);
    if (!out || n < 1 || leaf_size < 1 || k < 1 || !U || !V || !Ut || !Vt || !B || !D)
      HM_THROW(HM_ERR_ARG, "from_generators: bad arguments");
    if (dtype != HM_F64 && dtype != HM_F32) HM_THROW(HM_ERR_ARG, "dtype must be F64 or F32");
    if (k > HM_MAX_SAMPLES)
      HM_THROW(HM_ERR_UNSUPPORTED, "rank %d > %d", k, HM_MAX_SAMPLES);
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<hm_hbs_s> h(new hm_hbs_s());
    forest_add_tree(h->f, n, leaf_size, k, k, 0, 0.0, 0);
    forest_finish(h->f);
    const Forest& f = h->f;
    for (int g : f.leaves)
      if (f.inst[0].L > 0 && f.nodes[g].hi - f.nodes[g].lo < k)
        HM_THROW(HM_ERR_ARG, "every leaf must hold at least k indices");
    h->R = k;
    h->dtype = dtype;
    h->is_id = 0;
    const size_t es = dsize(dtype);
    const int nn = (int)f.nodes.size();
    const int nmax = f.nmax;
    h->d_nodes = upload(f.nodes, s);
    h->d_inst = upload(f.inst, s);
    h->U = DevBuf((size_t)n * k * es);
    h->V = DevBuf((size_t)n * k * es);
    h->Ut = DevBuf((size_t)nn * 2 * k * k * es);
    h->Vt = DevBuf((size_t)nn * 2 * k * k * es);
    h->B = DevBuf((size_t)nn * k * k * es);
    h->D = DevBuf((size_t)n * nmax * es);
    auto cp = [&](DevBuf& d, const void* src, size_t off_elems, size_t elems) {
      HIPCHK(hipMemcpyAsync(d.p, static_cast<const char*>(src) + off_elems * es, elems * es,
                            hipMemcpyDeviceToDevice, s));
    };
    cp(h->U, U, 0, (size_t)n * k);
    cp(h->V, V, 0, (size_t)n * k);
    // flat layout is heap-indexed (block t), handles are node-indexed (g = t - 1)
    cp(h->Ut, Ut, (size_t)2 * k * k, (size_t)nn * 2 * k * k);
    cp(h->Vt, Vt, (size_t)2 * k * k, (size_t)nn * 2 * k * k);
    cp(h->B, B, (size_t)k * k, (size_t)nn * k * k);
    cp(h->D, D, 0, (size_t)n * nmax);
    std::vector<int> mvec{f.inst[0].L};
    build_apply_lists(f, mvec, h->full, s);
    h->grad_leaves = upload(f.leaves, s);
    {
      std::vector<int32_t> all(f.nodes.size());
      for (size_t g = 0; g < all.size(); ++g) all[g] = (int32_t)g;
      h->grad_nodes = upload(all, s);
    }
    h->rank_u.assign(nn, 0);
    h->rank_v.assign(nn, 0);
    for (int g = 1; g < nn; ++g) h->rank_u[g] = h->rank_v[g] = k;
    h->skel_in.assign((size_t)nn * k, -1);
    h->skel_out.assign((size_t)nn * k, -1);
    HIPCHK(hipStreamSynchronize(s));
    finish_handle_info(h.get());
    *out = h.release();
    return HM_OK;
  });
}

int hm_hbs_convert(const hm_hbs* h, int32_t dtype, void* stream, hm_hbs** out) {
  if (out) *out = nullptr;
  return guarded([&]() -> int {
    StreamScope scope(stream);
    if (!h || !out) HM_THROW(HM_ERR_ARG, "convert: bad arguments");
    if (dtype != HM_F64 && dtype != HM_F32) HM_THROW(HM_ERR_ARG, "convert: dtype must be F64 or F32");
    *out = convert_hbs(h, dtype, (hipStream_t)stream);
    return HM_OK;
  });
}

int hm_hbs_info(const hm_hbs* h, hm_info* o) {
  return guarded([&] {
    if (!h || !o) HM_THROW(HM_ERR_ARG, "info: bad arguments");
    *o = h->info;
    return HM_OK;
  });
}

int hm_hbs_generators(const hm_hbs* h, hm_views* o) {
  return guarded([&] {
    if (!h || !o) HM_THROW(HM_ERR_ARG, "generators: bad arguments");
    if (h->f.inst.size() != 1) HM_THROW(HM_ERR_ARG, "generators: single-tree handles only");
    hm_views v{};
    v.dtype = h->dtype;
    v.rank_pad = h->R;
    v.levels = h->f.inst[0].L;
    v.nmax = h->f.nmax;
    v.n = h->f.n_total;
    v.nodes = (int64_t)h->f.nodes.size();
    v.U = h->U.p;
    v.V = h->V.p;
    v.Ut = h->Ut.p;
    v.Vt = h->Vt.p;
    v.B = h->B.p;
    v.D = h->D.p;
    *o = v;
    return HM_OK;
  });
}

int hm_hbs_export(const hm_hbs* h, void* U, void* V, void* Ut, void* Vt, void* B, void* D,
                  int32_t* ranks_u, int32_t* ranks_v, int32_t* skel_in, int32_t* skel_out,
                  void* stream) {
  return guarded([&] {
    StreamScope scope(stream);
    if (!h) HM_THROW(HM_ERR_ARG, "export: NULL handle");
    hipStream_t s = (hipStream_t)stream;
    const Forest& f = h->f;
    const int64_t n = f.n_total;
    const int R = h->R;
    const int nn = (int)f.nodes.size();
    const size_t es = dsize(h->dtype);
    auto cp = [&](void* dst, const DevBuf& src, size_t dst_off_elems, size_t elems) {
      if (!dst) return;
      HIPCHK(hipMemcpyAsync(static_cast<char*>(dst) + dst_off_elems * es, src.p, elems * es,
                            hipMemcpyDeviceToDevice, s));
    };
    if (Ut) HIPCHK(hipMemsetAsync(Ut, 0, (size_t)2 * R * R * es, s));
    if (Vt) HIPCHK(hipMemsetAsync(Vt, 0, (size_t)2 * R * R * es, s));
    if (B) HIPCHK(hipMemsetAsync(B, 0, (size_t)R * R * es, s));
    cp(U, h->U, 0, (size_t)n * R);
    cp(V, h->V, 0, (size_t)n * R);
    cp(Ut, h->Ut, (size_t)2 * R * R, (size_t)nn * 2 * R * R);
    cp(Vt, h->Vt, (size_t)2 * R * R, (size_t)nn * 2 * R * R);
    cp(B, h->B, (size_t)R * R, (size_t)nn * R * R);
    cp(D, h->D, 0, (size_t)n * f.nmax);
    // host arrays are heap-indexed (entry t = node t - 1); entry 0 unused
    if (ranks_u) { ranks_u[0] = 0; std::memcpy(ranks_u + 1, h->rank_u.data(), nn * 4); }
    if (ranks_v) { ranks_v[0] = 0; std::memcpy(ranks_v + 1, h->rank_v.data(), nn * 4); }
    if (skel_in) {
      std::fill(skel_in, skel_in + R, -1);
      std::memcpy(skel_in + R, h->skel_in.data(), (size_t)nn * R * 4);
    }
    if (skel_out) {
      std::fill(skel_out, skel_out + R, -1);
      std::memcpy(skel_out + R, h->skel_out.data(), (size_t)nn * R * 4);
    }
    return HM_OK;
  });
}

void hm_hbs_free(hm_hbs* h) { delete h; }

int hss_apply_backward(const hm_hbs* h, int64_t nrhs, const void* x, int64_t ldx, const void* gy,
                       int64_t ldgy, void* gx, int64_t ldgx, void* gU, void* gV, void* gUt,
                       void* gVt, void* gB, void* gD, void* stream) {
  return guarded([&] {
    StreamScope scope(stream);
    if (!h || !x || !gy || !gx || nrhs < 1) HM_THROW(HM_ERR_ARG, "backward: bad arguments");
    const int64_t n = h->f.n_total;
    if (ldx < n || ldgy < n || ldgx < n) HM_THROW(HM_ERR_ARG, "backward: ld < n");
    if (nrhs > 128) HM_THROW(HM_ERR_UNSUPPORTED, "backward: nrhs %lld > 128", (long long)nrhs);
    if (h->f.inst.size() != 1) HM_THROW(HM_ERR_ARG, "backward: single-tree handles only");
    hipStream_t s = (hipStream_t)stream;
    const int c = (int)nrhs;
    if (h->dtype == HM_F64)
      backward_impl<double>(h, c, (const double*)x, ldx, (const double*)gy, ldgy, (double*)gx,
                            ldgx, (double*)gU, (double*)gV, (double*)gUt, (double*)gVt,
                            (double*)gB, (double*)gD, s);
    else
      backward_impl<float>(h, c, (const float*)x, ldx, (const float*)gy, ldgy, (float*)gx, ldgx,
                           (float*)gU, (float*)gV, (float*)gUt, (float*)gVt, (float*)gB,
                           (float*)gD, s);
    return HM_OK;
  });
}

int hodlr_apply(const hm_hodlr* h, int32_t adjoint, int64_t nrhs, const double* x, int64_t ldx,
                double* y, int64_t ldy, void* stream) {
  return guarded([&] {
    StreamScope scope(stream);
    if (!h || !x || !y || nrhs < 0) HM_THROW(HM_ERR_ARG, "hodlr_apply: bad arguments");
    const int64_t n = h->f.n_total;
    if (ldx < n || ldy < n) HM_THROW(HM_ERR_ARG, "hodlr_apply: ld < n");
    for (int64_t c0 = 0; c0 < nrhs; c0 += 128) {
      const int c = (int)std::min<int64_t>(128, nrhs - c0);
      hodlr_apply_full(h, adjoint != 0, c, x + c0 * ldx, ldx, y + c0 * ldy, ldy,
                       (hipStream_t)stream);
    }
    return HM_OK;
  });
}

int hm_hodlr_info(const hm_hodlr* h, hm_info* o) {
  return guarded([&] {
    if (!h || !o) HM_THROW(HM_ERR_ARG, "info: bad arguments");
    *o = h->info;
    return HM_OK;
  });
}

int hm_hodlr_export(const hm_hodlr* h, double* U, double* V, double* s, double* D, int32_t* ranks,
                    void* stream) {
  return guarded([&] {
    StreamScope scope(stream);
    if (!h) HM_THROW(HM_ERR_ARG, "export: NULL handle");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = h->f.n_total;
    const int R = h->R;
    const int nn = (int)h->f.nodes.size();
    for (size_t l = 0; l < h->U.size(); ++l) {
      if (U) HIPCHK(hipMemcpyAsync(U + l * n * R, h->U[l].p, (size_t)n * R * 8, hipMemcpyDeviceToDevice, st));
      if (V) HIPCHK(hipMemcpyAsync(V + l * n * R, h->V[l].p, (size_t)n * R * 8, hipMemcpyDeviceToDevice, st));
    }
    if (s) {
      HIPCHK(hipMemsetAsync(s, 0, (size_t)R * 8, st));
      HIPCHK(hipMemcpyAsync(s + R, h->S.p, (size_t)nn * R * 8, hipMemcpyDeviceToDevice, st));
    }
    if (D) HIPCHK(hipMemcpyAsync(D, h->D.p, (size_t)n * h->f.nmax * 8, hipMemcpyDeviceToDevice, st));
    if (ranks) { ranks[0] = 0; std::memcpy(ranks + 1, h->rank.data(), nn * 4); }
    return HM_OK;
  });
}

void hm_hodlr_free(hm_hodlr* h) { delete h; }

}  // extern "C"

