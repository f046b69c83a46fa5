// C-ABI entry points of the coefficient surrogate: training, inference with
// the table fallback, the training data and the held-out check.
#include "pcmcc_runtime.hpp"

extern "C" {

namespace {

struct MlpDev {
  float *params = nullptr, *x = nullptr, *t = nullptr, *mask = nullptr, *partial = nullptr, *ploss = nullptr;
  float *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr, *hist = nullptr;
  ~MlpDev() {
    for (float* q : {params, x, t, mask, partial, ploss, m, v, grad, loss, hist}) dfree(q);
  }
};

int mlp_upload(pcmcc_ctx* c, MlpDev& d, const float* params, int64_t n, const float* x, const float* t,
               const float* mask, int nb, float* inv_cnt) {
  if (!params || !x || !t || !mask || n < 1) return fail(c, PCMCC_EINVAL, "invalid surrogate data");
  double cnt = 0;
  for (int64_t i = 0; i < n * PCMCC_MLP_OUT; ++i) {
    if (!(mask[i] == 0.0f || mask[i] == 1.0f)) return fail(c, PCMCC_EINVAL, "mask entries must be 0 or 1");
    if (mask[i] != 0.0f && !std::isfinite(t[i])) return fail(c, PCMCC_EINVAL, "non-finite unmasked target");
    cnt += mask[i];
  }
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return fail(c, PCMCC_EINVAL, "non-finite input");
  if (cnt <= 0) return fail(c, PCMCC_EINVAL, "no unmasked targets");
  *inv_cnt = (float)(1.0 / cnt);
  HIP_TRY(c, dalloc(&d.params, kMlpParams));
  HIP_TRY(c, dalloc(&d.x, n));
  HIP_TRY(c, dalloc(&d.t, n * PCMCC_MLP_OUT));
  HIP_TRY(c, dalloc(&d.mask, n * PCMCC_MLP_OUT));
  HIP_TRY(c, dalloc(&d.partial, (size_t)nb * kMlpParams));
  HIP_TRY(c, dalloc(&d.ploss, nb));
  HIP_TRY(c, hipMemcpyAsync(d.params, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(d.x, x, sizeof(float) * n, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(d.t, t, sizeof(float) * n * PCMCC_MLP_OUT, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(d.mask, mask, sizeof(float) * n * PCMCC_MLP_OUT, hipMemcpyHostToDevice, c->stream));
  return PCMCC_OK;
}

}  // namespace

int pcmcc_mlp_grad(pcmcc_ctx* c, const float* params, int64_t n, const float* x, const float* t, const float* mask,
                   float* grad_out, double* loss_out) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (!grad_out || !loss_out) return fail(c, PCMCC_EINVAL, "null output");
  HIP_TRY(c, hipSetDevice(c->device));
  const int nb = (int)std::min<int64_t>((n + 63) / 64, 1024);
  MlpDev d;
  float inv_cnt = 0;
  int rc = mlp_upload(c, d, params, n, x, t, mask, std::max(nb, 1), &inv_cnt);
  if (rc) return rc;
  HIP_TRY(c, dalloc(&d.grad, kMlpParams));
  HIP_TRY(c, dalloc(&d.loss, 1));
  MlpArgs A{};
  A.params = d.params;
  A.x = d.x;
  A.t = d.t;
  A.mask = d.mask;
  A.n = n;
  A.inv_cnt = inv_cnt;
  A.partial = d.partial;
  A.ploss = d.ploss;
  HIP_TRY(c, launch_mlp_grad(A, nb, c->stream));
  HIP_TRY(c, launch_mlp_reduce(d.partial, d.ploss, nb, d.grad, d.loss, c->stream));
  float lsum = 0;
  HIP_TRY(c, hipMemcpyAsync(grad_out, d.grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(&lsum, d.loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *loss_out = (double)lsum * inv_cnt;
  return PCMCC_OK;
}

int pcmcc_mlp_train(pcmcc_ctx* c, const float* params_in, int64_t n, const float* x, const float* t,
                    const float* mask, const pcmcc_mlp_train_opts* o, float* params_out, float* loss_hist,
                    pcmcc_stats* stats) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!o || !params_out) return fail(c, PCMCC_EINVAL, "null argument");
  if (o->epochs < 1 || !(o->lr0 > 0) || !(o->lr_min >= 0) || !(o->beta1 >= 0 && o->beta1 < 1) ||
      !(o->beta2 >= 0 && o->beta2 < 1) || !(o->eps > 0))
    return fail(c, PCMCC_EINVAL, "invalid training options");
  HIP_TRY(c, hipSetDevice(c->device));
  int per_cu = 0;
  HIP_TRY(c, occupancy_mlp_train(&per_cu));
  if (per_cu < 1) return fail(c, PCMCC_EHIP, "training kernel does not fit on a compute unit");
  const int nb = (int)std::min<int64_t>(std::min<int64_t>((n + 63) / 64, (int64_t)per_cu * c->num_cu), 1024);
  MlpDev d;
  float inv_cnt = 0;
  int rc = mlp_upload(c, d, params_in, n, x, t, mask, std::max(nb, 1), &inv_cnt);
  if (rc) return rc;
  HIP_TRY(c, dalloc(&d.m, kMlpParams));
  HIP_TRY(c, dalloc(&d.v, kMlpParams));
  HIP_TRY(c, hipMemsetAsync(d.m, 0, sizeof(float) * kMlpParams, c->stream));
  HIP_TRY(c, hipMemsetAsync(d.v, 0, sizeof(float) * kMlpParams, c->stream));
  if (loss_hist) HIP_TRY(c, dalloc(&d.hist, o->epochs));
  MlpArgs A{};
  A.params = d.params;
  A.x = d.x;
  A.t = d.t;
  A.mask = d.mask;
  A.n = n;
  A.inv_cnt = inv_cnt;
  A.partial = d.partial;
  A.ploss = d.ploss;
  A.m = d.m;
  A.v = d.v;
  A.loss_hist = d.hist;
  A.epochs = o->epochs;
  A.lr0 = o->lr0;
  A.lr_min = o->lr_min;
  A.beta1 = (float)o->beta1;
  A.beta2 = (float)o->beta2;
  A.eps = (float)o->eps;
  HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
  HIP_TRY(c, launch_mlp_train(A, nb, c->stream));
  HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
  HIP_TRY(c, hipMemcpyAsync(params_out, d.params, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, c->stream));
  if (loss_hist)
    HIP_TRY(c, hipMemcpyAsync(loss_hist, d.hist, sizeof(float) * o->epochs, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (stats) {
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    stats->step_kernel_ms = ms;
    stats->steps_done = o->epochs;
    stats->launch_block = 256;
    stats->launch_grid = nb;
  }
  return PCMCC_OK;
}

int pcmcc_mlp_infer(pcmcc_ctx* c, const float* params, const pcmcc_mlp_infer_opts* o, int64_t n, const float* EN_dev,
                    float* out_dev, pcmcc_stats* stats) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!params || !o || n < 0 || (n > 0 && (!EN_dev || !out_dev))) return fail(c, PCMCC_EINVAL, "invalid arguments");
  if (!(o->sd_x > 0)) return fail(c, PCMCC_EINVAL, "sd_x must be positive");
  if (o->n_cells < 0 || (o->n_cells > 0 && (!o->fallback || !(o->cell_hi > o->cell_lo) || o->n_nodes < 2 ||
                                             !o->table || !(o->table_hi > o->table_lo))))
    return fail(c, PCMCC_EINVAL, "invalid fallback description");
  if (n == 0) return PCMCC_OK;
  HIP_TRY(c, hipSetDevice(c->device));
  float* dparams = nullptr;
  uint8_t* dmask = nullptr;
  float* dtable = nullptr;
  auto cleanup = [&]() {
    dfree(dparams);
    dfree(dmask);
    dfree(dtable);
  };
  InferArgs A{};
  hipError_t e = dalloc(&dparams, kMlpParams);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dparams, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && o->n_cells > 0) {
    e = dalloc(&dmask, o->n_cells);
    if (e == hipSuccess) e = hipMemcpyAsync(dmask, o->fallback, o->n_cells, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = dalloc(&dtable, (size_t)o->n_nodes * PCMCC_MLP_OUT);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dtable, o->table, sizeof(float) * o->n_nodes * PCMCC_MLP_OUT, hipMemcpyHostToDevice,
                         c->stream);
  }
  if (e != hipSuccess) {
    cleanup();
    return fail(c, PCMCC_EHIP, "surrogate upload: %s", hipGetErrorString(e));
  }
  A.params = dparams;
  A.EN = EN_dev;
  A.out = out_dev;
  A.n = n;
  A.mu_x = (float)o->mu_x;
  A.inv_sd_x = (float)(1.0 / o->sd_x);
  for (int k = 0; k < PCMCC_MLP_OUT; ++k) {
    A.mu_y[k] = (float)o->mu_y[k];
    A.sd_y[k] = (float)o->sd_y[k];
  }
  A.n_cells = o->n_cells;
  if (o->n_cells > 0) {
    A.cell_lo = (float)o->cell_lo;
    A.inv_cell_w = (float)(o->n_cells / (o->cell_hi - o->cell_lo));
    A.fb_mask = dmask;
    A.n_nodes = o->n_nodes;
    A.tab_lo = (float)o->table_lo;
    A.inv_tab_w = (float)((o->n_nodes - 1) / (o->table_hi - o->table_lo));
    A.table = dtable;
  }
  const int grid = (int)std::min<int64_t>((n + 127) / 128, (int64_t)8 * c->num_cu);
  e = hipEventRecord(c->ev[0], c->stream);
  if (e == hipSuccess) e = launch_mlp_infer(A, grid, c->stream);
  if (e == hipSuccess) e = hipEventRecord(c->ev[1], c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
  cleanup();
  if (e != hipSuccess) return fail(c, PCMCC_EHIP, "surrogate inference: %s", hipGetErrorString(e));
  if (stats) {
    stats->step_kernel_ms = ms;
    stats->launch_block = 256;
    stats->launch_grid = grid;
  }
  return PCMCC_OK;
}

int pcmcc_mlp_dataset(int n, const double* EN_Td, const pcmcc_swarm_result* res, double gas_N, double max_rel_err,
                      int compute_norm, pcmcc_mlp_infer_opts* norm, float* x_out, float* t_out, float* mask_out,
                      float* ln_out, float* sig_out, double ln_floor) {
  if (n < 1 || !EN_Td || !res || !norm || !x_out || !t_out || !mask_out || !(gas_N > 0) || !(max_rel_err > 0))
    return fail(nullptr, PCMCC_EINVAL, "invalid surrogate dataset arguments");
  std::vector<double> lx(n), ly((size_t)n * PCMCC_MLP_OUT), sg((size_t)n * PCMCC_MLP_OUT);
  std::vector<char> ok((size_t)n * PCMCC_MLP_OUT);
  for (int i = 0; i < n; ++i) {
    if (!(EN_Td[i] > 0)) return fail(nullptr, PCMCC_EINVAL, "E/N must be positive");
    lx[i] = std::log(EN_Td[i]);
    const double* v = res[i].value;
    const double* e = res[i].error;
    const double val[PCMCC_MLP_OUT] = {v[PCMCC_Q_MU] * gas_N, v[PCMCC_Q_DL_FLUX] * gas_N, v[PCMCC_Q_ALPHA] / gas_N,
                                       v[PCMCC_Q_ETA] / gas_N, v[PCMCC_Q_MEAN_EPS], v[PCMCC_Q_BULK_FLUX_RATIO]};
    const double rel[PCMCC_MLP_OUT] = {e[PCMCC_Q_MU] / std::fabs(v[PCMCC_Q_MU]),
                                       e[PCMCC_Q_DL_FLUX] / std::fabs(v[PCMCC_Q_DL_FLUX]),
                                       e[PCMCC_Q_ALPHA] / std::fabs(v[PCMCC_Q_ALPHA]),
                                       e[PCMCC_Q_ETA] / std::fabs(v[PCMCC_Q_ETA]),
                                       e[PCMCC_Q_MEAN_EPS] / std::fabs(v[PCMCC_Q_MEAN_EPS]),
                                       e[PCMCC_Q_BULK_FLUX_RATIO] / std::fabs(v[PCMCC_Q_BULK_FLUX_RATIO])};
    for (int k = 0; k < PCMCC_MLP_OUT; ++k) {
      const bool good = val[k] > 0 && std::isfinite(val[k]) && rel[k] <= max_rel_err;
      ok[(size_t)i * PCMCC_MLP_OUT + k] = good;
      ly[(size_t)i * PCMCC_MLP_OUT + k] = good ? std::log(val[k]) : ln_floor;
      sg[(size_t)i * PCMCC_MLP_OUT + k] = good ? rel[k] : NAN;
    }
  }
  if (compute_norm) {
    double m = 0, q = 0;
    for (int i = 0; i < n; ++i) m += lx[i];
    m /= n;
    for (int i = 0; i < n; ++i) q += (lx[i] - m) * (lx[i] - m);
    norm->mu_x = m;
    norm->sd_x = n > 1 ? std::sqrt(q / (n - 1)) : 1.0;
    if (!(norm->sd_x > 0)) norm->sd_x = 1.0;
    for (int k = 0; k < PCMCC_MLP_OUT; ++k) {
      double mk = 0, qk = 0;
      int c = 0;
      for (int i = 0; i < n; ++i)
        if (ok[(size_t)i * PCMCC_MLP_OUT + k]) {
          mk += ly[(size_t)i * PCMCC_MLP_OUT + k];
          ++c;
        }
      mk = c ? mk / c : 0.0;
      for (int i = 0; i < n; ++i)
        if (ok[(size_t)i * PCMCC_MLP_OUT + k]) {
          const double d = ly[(size_t)i * PCMCC_MLP_OUT + k] - mk;
          qk += d * d;
        }
      norm->mu_y[k] = mk;
      norm->sd_y[k] = c > 1 ? std::sqrt(qk / (c - 1)) : 1.0;
      if (!(norm->sd_y[k] > 0)) norm->sd_y[k] = 1.0;
    }
  } else if (!(norm->sd_x > 0)) {
    return fail(nullptr, PCMCC_EINVAL, "norm.sd_x must be positive");
  }
  for (int i = 0; i < n; ++i) {
    x_out[i] = (float)((lx[i] - norm->mu_x) / norm->sd_x);
    for (int k = 0; k < PCMCC_MLP_OUT; ++k) {
      const size_t j = (size_t)i * PCMCC_MLP_OUT + k;
      mask_out[j] = ok[j] ? 1.0f : 0.0f;
      t_out[j] = ok[j] ? (float)((ly[j] - norm->mu_y[k]) / norm->sd_y[k]) : 0.0f;
      if (ln_out) ln_out[j] = (float)ly[j];
      if (sig_out) sig_out[j] = (float)sg[j];
    }
  }
  return PCMCC_OK;
}

int pcmcc_mlp_fallback(pcmcc_ctx* c, const float* params, const pcmcc_mlp_infer_opts* norm, int n_held,
                       const double* EN_held, const float* ln_held, const float* mask_held, const float* sig_held,
                       double tol_ln, double z_sig, int n_cells, double cell_lo, double cell_hi,
                       uint8_t* fallback_out, float* err_out) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (!params || !norm || n_held < 1 || !EN_held || !ln_held || !mask_held || !(tol_ln > 0) || !std::isfinite(z_sig) ||
      n_cells < 1 || !(cell_hi > cell_lo) || !fallback_out)
    return fail(c, PCMCC_EINVAL, "invalid fallback arguments");
  HIP_TRY(c, hipSetDevice(c->device));
  std::vector<float> en(n_held), y((size_t)PCMCC_MLP_OUT * n_held);
  for (int i = 0; i < n_held; ++i) en[i] = (float)EN_held[i];
  float *den = nullptr, *dout = nullptr;
  HIP_TRY(c, dalloc(&den, n_held));
  hipError_t e = dalloc(&dout, (size_t)PCMCC_MLP_OUT * n_held);
  if (e == hipSuccess) e = hipMemcpyAsync(den, en.data(), sizeof(float) * n_held, hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) {
    dfree(den);
    dfree(dout);
    return fail(c, PCMCC_EHIP, "fallback upload: %s", hipGetErrorString(e));
  }
  pcmcc_mlp_infer_opts o = *norm;
  o.n_cells = 0;
  int rc = pcmcc_mlp_infer(c, params, &o, n_held, den, dout, nullptr);
  if (rc == PCMCC_OK) {
    e = hipMemcpy(y.data(), dout, sizeof(float) * y.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = fail(c, PCMCC_EHIP, "fallback copy: %s", hipGetErrorString(e));
  }
  dfree(den);
  dfree(dout);
  if (rc) return rc;
  // A cell without a held-out point falls back in every output; otherwise
  // output k falls back if it is unresolved or misses at any of the cell's
  // held-out points.
  const uint8_t all = (uint8_t)((1u << PCMCC_MLP_OUT) - 1u);
  std::vector<char> seen(n_cells, 0);
  for (int k = 0; k < n_cells; ++k) fallback_out[k] = all;
  const double w = (cell_hi - cell_lo) / n_cells;
  for (int i = 0; i < n_held; ++i) {
    const int cell = std::min(std::max((int)std::floor((std::log(EN_held[i]) - cell_lo) / w), 0), n_cells - 1);
    if (!seen[cell]) {
      seen[cell] = 1;
      fallback_out[cell] = 0;
    }
    for (int k = 0; k < PCMCC_MLP_OUT; ++k) {
      const size_t j = (size_t)i * PCMCC_MLP_OUT + k;
      float err = NAN;
      if (mask_held[j] == 0.0f) {
        fallback_out[cell] |= (uint8_t)(1u << k);
      } else {
        err = std::fabs(y[(size_t)k * n_held + i] - ln_held[j]);
        const double sig = sig_held ? (double)sig_held[j] : 0.0;
        if (!(err <= tol_ln + z_sig * (std::isfinite(sig) ? sig : 0.0))) fallback_out[cell] |= (uint8_t)(1u << k);
      }
      if (err_out) err_out[j] = err;
    }
  }
  return PCMCC_OK;
}

}  // extern "C"
