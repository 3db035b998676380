// smash_api.hip -- the C ABI (include/smash.h): argument checks, handle
// lifetime, error translation, info and export.  No exception crosses it.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "common.cuh"

using namespace smash;

static thread_local std::string g_last_error;

static int fail(int code, const std::string &msg) {
  g_last_error = msg;
  (void)hipGetLastError();  // a failed HIP call stays this thread's last error otherwise
  return code;
}

extern "C" const char *smash_last_error(void) { return g_last_error.c_str(); }

extern "C" int smash_default_options(smash_options *opt) {
  if (!opt) return fail(SMASH_E_INVALID_ARG, "options pointer is NULL");
  std::memset(opt, 0, sizeof(*opt));
  opt->struct_size = sizeof(smash_options);
  opt->tau = 0.0;  // 0: dimension default
  opt->eps_svd = -1.0;
  opt->srrqr_f = 2.0;
  opt->diag_value = 0.0;
  opt->eval_prec = SMASH_F64;
  opt->apply_prec = SMASH_F64;
  opt->has_root_box = 0;
  opt->root_side = 0.0;
  opt->max_depth = 0;
  opt->batched = 1;
  opt->timing = 0;
  opt->mv_split_nodes = 1024;
  opt->graphs = 1;
  opt->mv_xcd_run = 16;
  opt->coupling_mode = SMASH_COUPLING_AUTO;
  return SMASH_OK;
}

namespace smash {
void resolve_timers(Handle &h) {
  for (auto &e : h.tev) {
    float ms = 0.0f;
    if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
      h.phase_ms[e.phase] += ms;
      h.phase_calls[e.phase] += 1;
    }
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  h.tev.clear();
}
}  // namespace smash

static void free_handle(Handle *h) {
  if (!h) return;
  resolve_timers(*h);
  drop_graphs(*h);
  if (h->prod_done) {
    (void)hipEventSynchronize(h->prod_done);
    (void)hipEventDestroy(h->prod_done);
  }
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  (void)hipStreamSynchronize(h->stream);
  if (h->side) (void)hipStreamSynchronize(h->side);  // a failed build may leave work there
  for (auto &a : h->spent) a.release();
  if (h->ws_mem.stream != h->stream) (void)hipStreamSynchronize(h->ws_mem.stream);
  h->ws_mem.release();
  h->mem.release();
  delete h;
}

static void keep_pool_cached(int dev) {
  static bool done[64] = {false};
  if (dev < 0 || dev >= 64 || done[dev]) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  done[dev] = true;
}

static int build_impl(const double *x, int64_t nx, const double *y, int64_t ny, bool same,
                      int32_t dim, int32_t kid, int32_t leaf, int32_t p, int32_t adm, double tol,
                      const smash_options *opt_in, void *stream, smash_handle *out) {
  if (!out) return fail(SMASH_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  smash_options opt;
  smash_default_options(&opt);
  if (opt_in) {
    if (opt_in->struct_size != sizeof(smash_options))
      return fail(SMASH_E_INVALID_ARG, "smash_options.struct_size mismatch");
    opt = *opt_in;
  }
  if (!x || !y) return fail(SMASH_E_INVALID_ARG, "point pointer is NULL");
  if (dim < 1 || dim > 3) return fail(SMASH_E_INVALID_ARG, "dim must be 1, 2 or 3");
  if (nx < 1 || ny < 1 || nx > INT32_MAX / 2 || ny > INT32_MAX / 2)
    return fail(SMASH_E_INVALID_ARG, "point count out of range");
  if (kid < 0 || kid > 4) return fail(SMASH_E_INVALID_ARG, "unknown kernel id");
  if (kid == SMASH_KERNEL_CAUCHY && dim != 1)
    return fail(SMASH_E_UNSUPPORTED, "the 1/(x-y) kernel needs dim == 1");
  if (kid == SMASH_KERNEL_DOUBLE_LAYER) {
    if (dim != 2 || !same)
      return fail(SMASH_E_UNSUPPORTED, "the double-layer kernel needs dim == 2 and X = Y");
    if (!opt.point_data)
      return fail(SMASH_E_INVALID_ARG, "the double-layer kernel needs options.point_data");
    if (opt.coupling_mode == SMASH_COUPLING_EVALUATED)
      return fail(SMASH_E_UNSUPPORTED, "the double-layer kernel stores its coupling blocks");
  } else if (opt.point_data) {
    return fail(SMASH_E_INVALID_ARG, "options.point_data is for the double-layer kernel only");
  }
  if (opt.basis != SMASH_BASIS_CHEBYSHEV && opt.basis != SMASH_BASIS_TAYLOR)
    return fail(SMASH_E_INVALID_ARG, "unknown options.basis");
  if (opt.basis == SMASH_BASIS_TAYLOR && (dim != 1 || kid == SMASH_KERNEL_DOUBLE_LAYER))
    return fail(SMASH_E_UNSUPPORTED, "the Taylor basis needs dim == 1 (and not the double layer)");
  if (leaf < 1) return fail(SMASH_E_INVALID_ARG, "leaf_size must be >= 1");
  if (p < 1 || p > 64) return fail(SMASH_E_INVALID_ARG, "interp_order must be in [1, 64]");
  if (adm != SMASH_ADM_WEAK && adm != SMASH_ADM_STRONG)
    return fail(SMASH_E_INVALID_ARG, "unknown admissibility");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(SMASH_E_INVALID_ARG, "tol must be >= 0");
  double tau = opt.tau > 0.0 ? opt.tau : (dim == 1 ? 0.6 : 0.7);
  if (!(tau > 0.0 && tau < 1.0)) return fail(SMASH_E_INVALID_ARG, "tau must lie in (0, 1)");
  if (!(opt.srrqr_f > 1.0)) return fail(SMASH_E_INVALID_ARG, "srrqr_f must exceed 1");
  if (opt.apply_prec != SMASH_F64 && opt.apply_prec != SMASH_F32 && opt.apply_prec != SMASH_BF16)
    return fail(SMASH_E_INVALID_ARG, "apply_prec must be SMASH_F64, SMASH_F32 or SMASH_BF16");
  if (opt.eval_prec != SMASH_F64 && opt.eval_prec != SMASH_F32)
    return fail(SMASH_E_INVALID_ARG, "eval_prec must be SMASH_F64 or SMASH_F32");
  if (opt.has_root_box && !(opt.root_side >= 0.0 && std::isfinite(opt.root_side)))
    return fail(SMASH_E_INVALID_ARG, "root_side must be finite and >= 0");
  if (opt.mv_split_nodes < 0) return fail(SMASH_E_INVALID_ARG, "mv_split_nodes must be >= 0");
  if (opt.mv_xcd_run < 1 || opt.mv_xcd_run > 4096)
    return fail(SMASH_E_INVALID_ARG, "mv_xcd_run must lie in [1, 4096]");
  if (opt.coupling_mode != SMASH_COUPLING_AUTO && opt.coupling_mode != SMASH_COUPLING_STORED &&
      opt.coupling_mode != SMASH_COUPLING_EVALUATED)
    return fail(SMASH_E_INVALID_ARG, "coupling_mode must be SMASH_COUPLING_AUTO, _STORED or _EVALUATED");
  if (opt.coupling_chunk < 0) return fail(SMASH_E_INVALID_ARG, "coupling_chunk must be >= 0");
  if ((opt.alloc == nullptr) != (opt.free == nullptr))
    return fail(SMASH_E_INVALID_ARG, "set both allocator hooks or neither");

  Handle *h = nullptr;
  auto t0 = std::chrono::steady_clock::now();
  try {
    h = new Handle();
    h->hooks.alloc = opt.alloc;
    h->hooks.free = opt.free;
    h->hooks.ctx = opt.alloc_ctx;
    HooksScope hs(&h->hooks);
    AcctScope as(&h->acct);
    h->stream = (hipStream_t)stream;
    h->mem.stream = h->stream;
    h->ws_mem.stream = h->stream;
    SMASH_HIP(hipGetDevice(&h->device));
    keep_pool_cached(h->device);
    h->d = dim;
    h->kid = kid;
    h->adm = adm;
    h->leaf = leaf;
    h->p = p;
    h->tol = tol;
    h->tau = tau;
    h->eps_svd = opt.eps_svd >= 0.0 ? opt.eps_svd : tol;
    h->f = opt.srrqr_f;
    h->diag = kid == SMASH_KERNEL_EXP_R ? 1.0 : opt.diag_value;
    h->eval_prec = opt.eval_prec;
    h->apply_prec = opt.apply_prec;
    h->batched = opt.batched ? 1 : 0;
    h->timing = opt.timing != 0;
    h->mv_split_nodes = opt.mv_split_nodes;
    h->use_graphs = opt.graphs ? 1 : 0;
    h->mv_xcd_run = opt.mv_xcd_run;
    h->coupling_mode = opt.coupling_mode;
    h->coupling_chunk = opt.coupling_chunk;
    h->nx = nx;
    h->ny = ny;
    h->same_xy = same;
    h->reuse = same && kid != SMASH_KERNEL_CAUCHY && kid != SMASH_KERNEL_DOUBLE_LAYER;
    h->pdata_in = opt.point_data;
    // g of the Taylor basis (2.5): (2 pi r)^(1/(2r)) / e with r = p terms
    if (opt.basis == SMASH_BASIS_TAYLOR)
      h->taylor_g = std::pow(2.0 * M_PI * p, 1.0 / (2.0 * p)) / std::exp(1.0);
    h->bpl = adm == SMASH_ADM_WEAK ? 1 : dim;
    h->max_split = 63 / h->bpl;
    if (opt.max_depth > 0 && opt.max_depth - 1 < h->max_split) h->max_split = opt.max_depth - 1;
    h->has_root = opt.has_root_box != 0;
    if (h->has_root)
      for (int t = 0; t < dim; t++) {
        h->root_lo[t] = opt.root_lo[t];
        h->root_hi[t] = opt.root_lo[t] + opt.root_side;
      }
    {
      PhaseTimer pt(*h, SMASH_PHASE_TREE, h->stream);
      build_tree(*h, x, same ? x : y);
    }
    {
      PhaseTimer pt(*h, SMASH_PHASE_PAIRS, h->stream);
      build_pairs(*h);
    }
    // near-field blocks on the second stream from here on (they overlap the
    // first levels' compression; started any later, they compete with it)
    near_offsets(*h);
    near_launch(*h, read_one(h->stream, h->nboff + h->nLm));
    build_generators(*h);
    build_blocks(*h);  // ends with the stream synchronised
    for (auto &a : h->spent) a.release();
    h->spent.clear();
    h->build_peak = h->acct.peak.load();
    // (the leaf count came with the generators' last host read)
    h->build_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    SMASH_HIP(hipEventCreateWithFlags(&h->prod_done, hipEventDisableTiming));
    *out = (smash_handle)h;
    return SMASH_OK;
  } catch (const Error &e) {
    free_handle(h);
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc &) {
    free_handle(h);
    return fail(SMASH_E_OOM, "host allocation failed");
  } catch (...) {
    free_handle(h);
    return fail(SMASH_E_DEVICE, "unexpected failure");
  }
}

extern "C" int smash_build(const double *points, int64_t n, int32_t dim, int32_t kernel_id,
                           int32_t leaf_size, int32_t interp_order, int32_t admissibility,
                           double tol, const smash_options *opt, void *stream, smash_handle *out) {
  return build_impl(points, n, points, n, true, dim, kernel_id, leaf_size, interp_order,
                    admissibility, tol, opt, stream, out);
}

extern "C" int smash_build_xy(const double *x, int64_t nx, const double *y, int64_t ny,
                              int32_t dim, int32_t kernel_id, int32_t leaf_size,
                              int32_t interp_order, int32_t admissibility, double tol,
                              const smash_options *opt, void *stream, smash_handle *out) {
  return build_impl(x, nx, y, ny, false, dim, kernel_id, leaf_size, interp_order, admissibility,
                    tol, opt, stream, out);
}

extern "C" int smash_matvec(smash_handle hv, const void *X, int64_t ldx, int32_t nrhs,
                            int32_t dtype, void *Y, int64_t ldy, void *stream) {
  Handle *h = (Handle *)hv;
  if (!h) return fail(SMASH_E_INVALID_ARG, "handle is NULL");
  if (!X || !Y) return fail(SMASH_E_INVALID_ARG, "X or Y is NULL");
  if (nrhs < 1) return fail(SMASH_E_INVALID_ARG, "nrhs must be >= 1");
  if (ldx < nrhs || ldy < nrhs) return fail(SMASH_E_INVALID_ARG, "leading dimension < nrhs");
  if (dtype != (h->apply_prec == SMASH_F64 ? SMASH_F64 : SMASH_F32))
    return fail(SMASH_E_INVALID_ARG, "dtype differs from the handle's vector precision");
  try {
    HooksScope hs(&h->hooks);
    run_matvec(*h, X, ldx, nrhs, Y, ldy, (hipStream_t)stream);
    return SMASH_OK;
  } catch (const Error &e) {
    return fail(e.code, e.msg);
  } catch (...) {
    return fail(SMASH_E_DEVICE, "unexpected failure");
  }
}

extern "C" int smash_matvec_cauchy_like(smash_handle hv, const void *X, int64_t ldx,
                                        int32_t nrhs, int32_t dtype, const double *w,
                                        const double *v, int32_t p, void *Y, int64_t ldy,
                                        void *stream) {
  Handle *h = (Handle *)hv;
  if (!h) return fail(SMASH_E_INVALID_ARG, "handle is NULL");
  if (!X || !Y || !w || !v) return fail(SMASH_E_INVALID_ARG, "X, Y, w or v is NULL");
  if (nrhs < 1) return fail(SMASH_E_INVALID_ARG, "nrhs must be >= 1");
  if (p < 1 || p > SMASH_CAUCHY_LIKE_MAX_P)
    return fail(SMASH_E_INVALID_ARG, "generator count p out of range");
  if ((int64_t)p * nrhs > INT32_MAX / 2) return fail(SMASH_E_INVALID_ARG, "p * nrhs too large");
  if (ldx < nrhs || ldy < nrhs) return fail(SMASH_E_INVALID_ARG, "leading dimension < nrhs");
  if (dtype != (h->apply_prec == SMASH_F64 ? SMASH_F64 : SMASH_F32))
    return fail(SMASH_E_INVALID_ARG, "dtype differs from the handle's vector precision");
  try {
    HooksScope hs(&h->hooks);
    run_cauchy_like(*h, X, ldx, nrhs, w, v, p, Y, ldy, (hipStream_t)stream);
    return SMASH_OK;
  } catch (const Error &e) {
    return fail(e.code, e.msg);
  } catch (...) {
    return fail(SMASH_E_DEVICE, "unexpected failure");
  }
}

extern "C" int smash_matvec_noalloc(smash_handle hv, const void *X, int64_t ldx, int32_t nrhs,
                                    int32_t dtype, void *Y, int64_t ldy, void *stream) {
  Handle *h = (Handle *)hv;
  if (!h) return fail(SMASH_E_INVALID_ARG, "handle is NULL");
  if (!X || !Y) return fail(SMASH_E_INVALID_ARG, "X or Y is NULL");
  if (nrhs < 1) return fail(SMASH_E_INVALID_ARG, "nrhs must be >= 1");
  if (ldx < nrhs || ldy < nrhs) return fail(SMASH_E_INVALID_ARG, "leading dimension < nrhs");
  if (dtype != (h->apply_prec == SMASH_F64 ? SMASH_F64 : SMASH_F32))
    return fail(SMASH_E_INVALID_ARG, "dtype differs from the handle's vector precision");
  try {
    run_matvec_noalloc(*h, X, ldx, nrhs, Y, ldy, (hipStream_t)stream);
    return SMASH_OK;
  } catch (const Error &e) {
    return fail(e.code, e.msg);
  } catch (...) {
    return fail(SMASH_E_DEVICE, "unexpected failure");
  }
}

extern "C" int smash_matvec_batched(int32_t count, const smash_handle *hs,
                                    const void *const *Xs, const int64_t *ldx,
                                    const int32_t *nrhs, void *const *Ys, const int64_t *ldy,
                                    int32_t dtype, void *stream) {
  if (count < 0) return fail(SMASH_E_INVALID_ARG, "count must be >= 0");
  if (count == 0) return SMASH_OK;
  if (!hs || !Xs || !ldx || !nrhs || !Ys || !ldy)
    return fail(SMASH_E_INVALID_ARG, "an argument array is NULL");
  for (int32_t c = 0; c < count; c++) {
    const Handle *h = (const Handle *)hs[c];
    const std::string at = " (entry " + std::to_string(c) + ")";
    if (!h) return fail(SMASH_E_INVALID_ARG, "handle is NULL" + at);
    if (!Xs[c] || !Ys[c]) return fail(SMASH_E_INVALID_ARG, "X or Y is NULL" + at);
    if (nrhs[c] < 1) return fail(SMASH_E_INVALID_ARG, "nrhs must be >= 1" + at);
    if (ldx[c] < nrhs[c] || ldy[c] < nrhs[c])
      return fail(SMASH_E_INVALID_ARG, "leading dimension < nrhs" + at);
    if (dtype != (h->apply_prec == SMASH_F64 ? SMASH_F64 : SMASH_F32))
      return fail(SMASH_E_INVALID_ARG, "dtype differs from the handle's vector precision" + at);
  }
  try {
    for (int32_t c = 0; c < count; c++) {
      HooksScope scope(&((Handle *)hs[c])->hooks);
      run_matvec(*(Handle *)hs[c], Xs[c], ldx[c], nrhs[c], Ys[c], ldy[c], (hipStream_t)stream);
    }
    return SMASH_OK;
  } catch (const Error &e) {
    return fail(e.code, e.msg);
  } catch (...) {
    return fail(SMASH_E_DEVICE, "unexpected failure");
  }
}

extern "C" int smash_set_product_shape(smash_handle hv, int32_t mv_split_nodes,
                                       int32_t mv_xcd_run) {
  Handle *h = (Handle *)hv;
  if (!h) return fail(SMASH_E_INVALID_ARG, "handle is NULL");
  if (mv_split_nodes < 0) return fail(SMASH_E_INVALID_ARG, "mv_split_nodes must be >= 0");
  if (mv_xcd_run < 1 || mv_xcd_run > 4096)
    return fail(SMASH_E_INVALID_ARG, "mv_xcd_run must lie in [1, 4096]");
  try {
    drop_graphs(*h);
    h->mv_split_nodes = mv_split_nodes;
    h->mv_xcd_run = mv_xcd_run;
    return SMASH_OK;
  } catch (...) {
    return fail(SMASH_E_DEVICE, "unexpected failure");
  }
}

template <class T>
static std::vector<T> to_host(const T *p, int64_t n) {
  std::vector<T> v((size_t)(n > 0 ? n : 0));
  if (n > 0) SMASH_HIP(hipMemcpy(v.data(), p, sizeof(T) * n, hipMemcpyDeviceToHost));
  return v;
}

extern "C" int smash_info(smash_handle hv, smash_info_t *info) {
  Handle *h = (Handle *)hv;
  if (!h || !info) return fail(SMASH_E_INVALID_ARG, "NULL argument");
  try {
    std::memset(info, 0, sizeof(*info));
    info->nx = h->nx;
    info->ny = h->ny;
    info->dim = h->d;
    info->nlevels = h->nlevels;
    info->nnodes = h->nnodes;
    info->nleaves = h->nleaves;
    info->n_admissible = h->nL;
    info->n_inadmissible = h->nLm;
    info->coupling_entries = h->b_entries;
    info->near_entries = h->n_entries;
    info->apply_prec = h->apply_prec;
    info->eval_prec = h->eval_prec;
    info->symmetric_reuse = h->reuse ? 1 : 0;
    info->build_ms = h->build_ms;
    info->total_swaps = h->total_swaps;
    info->coupling_evaluated = h->coupling_eval ? 1 : 0;
    const bool chunked = h->coupling_eval && !h->coupling_fused;
    info->coupling_chunks = chunked ? (int32_t)h->cchunk_node.size() - 1 : 0;
    info->coupling_ws_entries = chunked ? h->bws_entries : 0;
    info->device_bytes = h->mem.bytes + h->ws_mem.bytes;
    info->build_peak_bytes = h->build_peak;
    info->graph_captures = h->graph_captures;
    info->graph_replays = h->graph_replays;
    resolve_timers(*h);
    for (int q = 0; q < 16; q++) {
      info->phase_ms[q] = h->phase_ms[q];
      info->phase_calls[q] = h->phase_calls[q];
    }
    int64_t sum_mk[2] = {0, 0}, sum_m[2] = {0, 0};
    auto side_stats = [&](Side &S, int64_t &sumk, int32_t &maxk, int64_t &gent, int q) {
      auto m = to_host(S.m, h->nnodes), k = to_host(S.k, h->nnodes);
      sumk = 0;
      maxk = 0;
      gent = 0;
      for (int i = 1; i < h->nnodes; i++) {
        sumk += k[i];
        maxk = k[i] > maxk ? k[i] : maxk;
        gent += (int64_t)(m[i] - k[i]) * k[i];
        sum_mk[q] += (int64_t)m[i] * k[i];
        sum_m[q] += m[i];
      }
    };
    side_stats(h->row, info->sum_rank_row, info->max_rank_row, info->g_entries_row, 0);
    side_stats(*h->col, info->sum_rank_col, info->max_rank_col, info->g_entries_col, 1);
    const int sides = h->reuse ? 1 : 2;
    info->bytes_dense = 8 * h->nx * h->ny;
    info->bytes_hss0 = 8 * (sum_mk[0] + (sides > 1 ? sum_mk[1] : 0) + h->b_entries + h->n_entries);
    info->bytes_smash = 8 * (info->g_entries_row + (sides > 1 ? info->g_entries_col : 0) +
                             h->n_entries) +
                        4 * (sum_m[0] + (sides > 1 ? sum_m[1] : 0) + 2 * (h->nL + h->nLm));
    int64_t idx = 2 * h->nx + 2 * h->ny + 2 * (h->nL + h->nLm) + h->row.nslots;
    for (int l = 2; l <= h->nlevels; l++) idx += h->row.lv[l].sel_n;
    if (!h->reuse) {
      idx += h->col->nslots;
      for (int l = 2; l <= h->nlevels; l++) idx += h->col->lv[l].sel_n;
    }
    info->index_entries = idx;
    return SMASH_OK;
  } catch (const Error &e) {
    return fail(e.code, e.msg);
  }
}

extern "C" int smash_export(smash_handle hv, int32_t what, void *buf, int64_t *count) {
  Handle *h = (Handle *)hv;
  if (!h || !count) return fail(SMASH_E_INVALID_ARG, "NULL argument");
  try {
    SMASH_HIP(hipStreamSynchronize(h->stream));
    const int nn = h->nnodes;
    std::vector<int32_t> iv;
    std::vector<double> dv;
    std::vector<float> fv;
    int kind = 0;  // 0 int32, 1 double, 2 apply type
    auto side_of = [&](int w) -> Side & {
      return (w == SMASH_EX_ROW_SEL || w == SMASH_EX_ROW_G || w == SMASH_EX_ROW_GRID) ? h->row
                                                                                     : *h->col;
    };
    switch (what) {
      case SMASH_EX_SIZES:
        iv = {(int)h->nx, (int)h->ny, nn, h->nlevels, (int)h->nL, (int)h->nLm, h->d, h->adm};
        break;
      case SMASH_EX_LEVELS:
        iv.assign(h->level_beg.begin(), h->level_beg.end());
        break;
      case SMASH_EX_PERM_X:
        iv = to_host(h->perm_x, h->nx);
        break;
      case SMASH_EX_PERM_Y:
        iv = to_host(h->perm_y, h->ny);
        break;
      case SMASH_EX_NODES: {
        auto a = to_host(h->level, nn), b = to_host(h->parent, nn), c = to_host(h->first_child, nn),
             d = to_host(h->nchild, nn), e = to_host(h->xb, nn), f = to_host(h->xe, nn),
             g = to_host(h->yb, nn), q = to_host(h->ye, nn);
        iv.resize((size_t)nn * 8);
        for (int i = 0; i < nn; i++) {
          int *o = &iv[(size_t)i * 8];
          o[0] = a[i];
          o[1] = b[i];
          o[2] = d[i] ? c[i] : -1;
          o[3] = d[i];
          o[4] = e[i];
          o[5] = f[i];
          o[6] = g[i];
          o[7] = q[i];
        }
        break;
      }
      case SMASH_EX_BOXES: {
        kind = 1;
        auto lo = to_host(h->lo, 3 * (int64_t)nn), hi = to_host(h->hi, 3 * (int64_t)nn);
        dv.resize((size_t)nn * 6);
        for (int i = 0; i < nn; i++)
          for (int t = 0; t < 3; t++) {
            dv[(size_t)i * 6 + t] = lo[3 * i + t];
            dv[(size_t)i * 6 + 3 + t] = hi[3 * i + t];
          }
        break;
      }
      case SMASH_EX_L:
      case SMASH_EX_LM: {
        bool l = what == SMASH_EX_L;
        int64_t n = l ? h->nL : h->nLm;
        auto a = to_host(l ? h->Li : h->Lmi, n), b = to_host(l ? h->Lj : h->Lmj, n);
        iv.resize((size_t)n * 2);
        for (int64_t e = 0; e < n; e++) {
          iv[2 * e] = a[e];
          iv[2 * e + 1] = b[e];
        }
        break;
      }
      case SMASH_EX_NEAR_PTR:
        if (h->Nrow) iv = to_host(h->Nrow, nn + 1);
        break;
      case SMASH_EX_NEAR_IDX:
        if (h->Nrow) iv = to_host(h->Ncol, h->nN);
        break;
      case SMASH_EX_RANKS: {
        Side &R = h->row, &C = *h->col;
        auto a = to_host(R.m, nn), b = to_host(R.k, nn), c = to_host(C.m, nn),
             d = to_host(C.k, nn), e = to_host(R.ks, nn), f = to_host(C.ks, nn);
        iv.resize((size_t)nn * 6);
        for (int i = 0; i < nn; i++) {
          int *o = &iv[(size_t)i * 6];
          bool root = i == 0;
          o[0] = root ? 0 : a[i];
          o[1] = root ? 0 : b[i];
          o[2] = root ? 0 : c[i];
          o[3] = root ? 0 : d[i];
          o[4] = root ? 0 : e[i];
          o[5] = root ? 0 : f[i];
        }
        break;
      }
      case SMASH_EX_ROW_SEL:
      case SMASH_EX_COL_SEL:
      case SMASH_EX_ROW_GRID:
      case SMASH_EX_COL_GRID:
      case SMASH_EX_ROW_G:
      case SMASH_EX_COL_G: {
        Side &S = side_of(what);
        auto m = to_host(S.m, nn), k = to_host(S.k, nn);
        auto gb = to_host(S.gbeg, nn), so = to_host(S.selo, nn), go = to_host(S.go, nn);
        bool grid = what == SMASH_EX_ROW_GRID || what == SMASH_EX_COL_GRID;
        bool gmat = what == SMASH_EX_ROW_G || what == SMASH_EX_COL_G;
        std::vector<int> slots;
        if (grid) slots = to_host(S.slot_id, S.nslots);
        if (gmat) kind = 1;
        for (int l = 2; l <= h->nlevels; l++) {
          LevelSide &L = S.lv[l];
          std::vector<int> sel;
          std::vector<double> G;
          if (!grid && !gmat) sel = to_host(L.sel, L.sel_n);
          if (gmat) G = to_host(L.G, L.g_n);
          for (int i = h->level_beg[l - 1]; i < h->level_beg[l]; i++) {
            if (grid)
              for (int a = 0; a < m[i]; a++) iv.push_back(slots[gb[i] + a]);
            else if (gmat)
              for (int64_t a = 0; a < (int64_t)(m[i] - k[i]) * k[i]; a++)
                dv.push_back(G[go[i] + a]);
            else
              for (int a = 0; a < m[i]; a++) iv.push_back(sel[so[i] + a]);
          }
        }
        break;
      }
      case SMASH_EX_COUPLING:
      case SMASH_EX_NEAR: {
        kind = 2;
        if (h->apply_prec == SMASH_BF16)
          return fail(SMASH_E_UNSUPPORTED, "blocks of a BF16-apply handle are not exported");
        int64_t n = what == SMASH_EX_COUPLING ? h->b_entries : h->n_entries;
        const void *src = what == SMASH_EX_COUPLING ? h->B : h->Bn;
        void *tmpb = nullptr;
        if (what == SMASH_EX_COUPLING && h->coupling_eval && n > 0) {
          // evaluated blocks: evaluate all of them once, for the copy
          const size_t es = h->apply_prec == SMASH_F64 ? sizeof(double) : sizeof(float);
          SMASH_HIP(hipMalloc(&tmpb, es * (size_t)n));
          try {
            eval_coupling_range(*h, 0, h->nL, tmpb, h->stream);
            SMASH_HIP(hipStreamSynchronize(h->stream));
          } catch (...) {
            (void)hipFree(tmpb);
            throw;
          }
          src = tmpb;
        }
        try {
          if (h->apply_prec == SMASH_F64)
            dv = to_host((const double *)src, n);
          else
            fv = to_host((const float *)src, n);
        } catch (...) {
          if (tmpb) (void)hipFree(tmpb);
          throw;
        }
        if (tmpb) SMASH_HIP(hipFree(tmpb));
        break;
      }
      default:
        return fail(SMASH_E_INVALID_ARG, "unknown export code");
    }
    int64_t n;
    size_t es;
    const void *src;
    if (kind == 0) {
      n = (int64_t)iv.size();
      es = sizeof(int32_t);
      src = iv.data();
    } else if (kind == 1 || (kind == 2 && h->apply_prec == SMASH_F64)) {
      n = (int64_t)dv.size();
      es = sizeof(double);
      src = dv.data();
    } else {
      n = (int64_t)fv.size();
      es = sizeof(float);
      src = fv.data();
    }
    if (!buf) {
      *count = n;
      return SMASH_OK;
    }
    if (*count < n) return fail(SMASH_E_INVALID_ARG, "export buffer too small");
    if (n > 0) std::memcpy(buf, src, es * (size_t)n);
    *count = n;
    return SMASH_OK;
  } catch (const Error &e) {
    return fail(e.code, e.msg);
  } catch (...) {
    return fail(SMASH_E_DEVICE, "unexpected failure");
  }
}

extern "C" int smash_estimate_footprint(int64_t n, int32_t dim, int32_t kid, int32_t leaf,
                                        int32_t p, int32_t adm, double tol, int32_t apply_prec,
                                        int64_t *bytes) {
  return smash_estimate_footprint_mode(n, dim, kid, leaf, p, adm, tol, apply_prec,
                                       SMASH_COUPLING_STORED, bytes);
}

extern "C" int smash_estimate_footprint_mode(int64_t n, int32_t dim, int32_t kid, int32_t leaf,
                                             int32_t p, int32_t adm, double tol,
                                             int32_t apply_prec, int32_t coupling_mode,
                                             int64_t *bytes) {
  if (!bytes) return fail(SMASH_E_INVALID_ARG, "bytes is NULL");
  if (coupling_mode != SMASH_COUPLING_AUTO && coupling_mode != SMASH_COUPLING_STORED &&
      coupling_mode != SMASH_COUPLING_EVALUATED)
    return fail(SMASH_E_INVALID_ARG, "unknown coupling_mode");
  if (n < 1 || dim < 1 || dim > 3 || leaf < 1 || p < 1 || p > 64 ||
      (adm != SMASH_ADM_WEAK && adm != SMASH_ADM_STRONG) || !(tol >= 0.0) ||
      kid < 0 || kid > 3 ||
      (apply_prec != SMASH_F64 && apply_prec != SMASH_F32 && apply_prec != SMASH_BF16))
    return fail(SMASH_E_INVALID_ARG, "parameter out of range");
  const double es = apply_prec == SMASH_F64 ? 8.0 : apply_prec == SMASH_F32 ? 4.0 : 2.0;
  const double vs = apply_prec == SMASH_F64 ? 8.0 : 4.0;  // vector element
  const double dn = (double)n;
  // leaves hold about leaf / 2^dim points or more on average (1.25 slack);
  // all levels together add 1 / (2^dim - 1) of that many inner nodes
  const double twod = (double)(1 << dim);
  const double leaves = std::max(1.0, dn * twod / (1.25 * (double)leaf));
  const double nodes = leaves * twod / (twod - 1.0);
  double pd = 1.0;
  for (int t = 0; t < dim; t++) pd *= p;
  const double c = adm == SMASH_ADM_STRONG ? pd : pd + leaf;  // HSS adds near vectors
  const double r = std::min(c, 0.75 * (double)leaf);
  double far = 1.0, near = 1.0;
  if (adm == SMASH_ADM_STRONG) {
    double s3 = 1.0, s6 = 1.0;
    for (int t = 0; t < dim; t++) {
      s3 *= 3.0;
      s6 *= 6.0;
    }
    far = s6 - s3;
    near = s3;
  }
  const double sides = (kid == SMASH_KERNEL_CAUCHY) ? 2.0 : 1.0;  // column side kept
  double b = 0.0;
  b += dn * (dim * 8.0 * 2.0 + 64.0);                  // points, permutations, tree
  b += nodes * (far + near) * 16.0;                    // pair lists and offsets
  b += sides * nodes * r * r * (8.0 * 2.0 + es * 2.0);  // G master, transpose, copies
  const double cb = nodes * far * r * r * es;          // coupling blocks
  // evaluated inside each product: a chunk workspace of at most 256 MiB
  // plus one node's blocks instead
  b += coupling_mode == SMASH_COUPLING_EVALUATED
           ? std::min(cb, 268435456.0 + far * r * r * es)
           : cb;
  b += leaves * near * (double)leaf * (double)leaf * es;  // near blocks
  b += 2.0 * (dn + sides * nodes * r) * 64.0 * vs;     // product workspace
  *bytes = (int64_t)std::min(b, 9.0e18);
  (void)tol;
  return SMASH_OK;
}

extern "C" int smash_trim(int32_t device) {
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return fail(SMASH_E_DEVICE, "hipGetDevice failed");
  const int dev = device < 0 ? cur : device;
  try {
    if (dev != cur) SMASH_HIP(hipSetDevice(dev));
    SMASH_HIP(hipDeviceSynchronize());
    trim_chunk_cache(dev);
    hipMemPool_t pool;
    SMASH_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
    SMASH_HIP(hipMemPoolTrimTo(pool, 0));
    if (dev != cur) SMASH_HIP(hipSetDevice(cur));
  } catch (const Error &e) {
    (void)hipSetDevice(cur);
    return fail(e.code, e.msg);
  }
  return SMASH_OK;
}

extern "C" int smash_destroy(smash_handle hv) {
  Handle *h = (Handle *)hv;
  if (!h) return SMASH_OK;
  free_handle(h);
  return SMASH_OK;
}
