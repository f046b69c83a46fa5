// C-ABI entry points of the PIC-MCC electron library (include/pcmcc.h):
// the context, species and tables, the step loop with the deposit
// (Sec. 2.1), super-particle weights (Sec. 2.1.2), the deposit alone and the
// self-tests of the generator and the tables.  The context owns the device
// tables, the scratch buffers of the step loop (ping-pong particle buffer,
// newborn queues, hole lists, counters) and the per-cell field bounds.
#include "pcmcc_runtime.hpp"

extern "C" {

const char* pcmcc_version(void) { return "pcmcc 0.1 (gfx950)"; }

const char* pcmcc_last_error(pcmcc_ctx* ctx) { return ctx ? ctx->err.c_str() : g_last_error.c_str(); }

int pcmcc_create(pcmcc_ctx** out, int device, void* hip_stream) {
  if (!out) return fail(nullptr, PCMCC_EINVAL, "out is null");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0)
    return fail(nullptr, PCMCC_EHIP, "no HIP device: %s", e != hipSuccess ? hipGetErrorString(e) : "count 0");
  if (device < 0 || device >= ndev) return fail(nullptr, PCMCC_EINVAL, "device %d out of range", device);
  e = hipSetDevice(device);
  if (e != hipSuccess) return fail(nullptr, PCMCC_EHIP, "hipSetDevice: %s", hipGetErrorString(e));
  pcmcc_ctx* c = new pcmcc_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) {
    delete c;
    return fail(nullptr, PCMCC_EHIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  }
  c->num_cu = prop.multiProcessorCount;
  noalloc_setup(device);
  for (auto& ev : c->ev) {
    if (hipEventCreate(&ev) != hipSuccess) {
      pcmcc_destroy(c);
      return fail(nullptr, PCMCC_EHIP, "hipEventCreate failed");
    }
  }
  if (dalloc(&c->ctl, 1) != hipSuccess || dalloc(&c->emax_bits, 1) != hipSuccess ||
      dalloc(&c->dep_err, 1) != hipSuccess ||
      hipHostMalloc((void**)&c->host_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->host_n, sizeof(int64_t), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->host_err, sizeof(unsigned), hipHostMallocDefault) != hipSuccess) {
    pcmcc_destroy(c);
    return fail(nullptr, PCMCC_ENOMEM, "context allocation failed");
  }
  *out = c;
  return PCMCC_OK;
}

int pcmcc_destroy(pcmcc_ctx* c) {
  if (!c) return PCMCC_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  free_scratch(c);
  free_swarm(c);
  dfree(c->dC);
  dfree(c->dP);
  dfree(c->dNu);
  dfree(c->partial);
  dfree(c->ctl);
  dfree(c->fbound);
  dfree(c->fpack);
  dfree(c->dep.tile_count);
  dfree(c->dep.tile_start);
  dfree(c->dep.dump);
  dfree(c->dep.sorted);
  dfree(c->wt.cls);
  dfree(c->wt.idx0);
  dfree(c->wt.idx1);
  dfree(c->wt.key0);
  dfree(c->wt.key1);
  dfree(c->wt.key2);
  dfree(c->wt.pos);
  dfree(c->wt.cnt);
  dfree(c->wt.counters);
  dfree(c->wt.temp);
  dfree(c->wt_rho);
  dfree(c->dev_n);
  dfree(c->mg_store);
  dfree(c->mg_rhs);
  dfree(c->mg_part);
  dfree(c->phi_prev);
  dfree(c->ph_cnt);
  dfree(c->ph_off);
  if (c->ph_temp) (void)hipFree(c->ph_temp);
  dfree(c->sc_E);
  dfree(c->sc_ne);
  dfree(c->ev_store);
  dfree(c->sc_red);
  dfree(c->sel);
  dfree(c->sel_hist);
  dfree(c->fl_store);
  dfree(c->fl_tab);
  if (c->sc_host) (void)hipHostFree(c->sc_host);
  dfree(c->emax_bits);
  dfree(c->dep_err);
  if (c->host_ctl) (void)hipHostFree(c->host_ctl);
  if (c->host_n) (void)hipHostFree(c->host_n);
  if (c->host_err) (void)hipHostFree(c->host_err);
  for (auto& ev : c->ev)
    if (ev) (void)hipEventDestroy(ev);
  delete c;
  return PCMCC_OK;
}

int pcmcc_init_species(pcmcc_ctx* c, double mass_kg, double charge_C, double gas_N_m3, double target_mass_kg) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (!(mass_kg > 0) || !std::isfinite(mass_kg) || !(charge_C != 0) || !std::isfinite(charge_C) ||
      !(gas_N_m3 >= 0) || !std::isfinite(gas_N_m3) || !(target_mass_kg > 0) || !std::isfinite(target_mass_kg))
    return fail(c, PCMCC_EINVAL, "invalid species parameters");
  c->mass = mass_kg;
  c->charge = charge_C;
  c->gas_N = gas_N_m3;
  c->target_mass = target_mass_kg;
  c->species_ok = true;
  c->tables_ok = false;
  return PCMCC_OK;
}

int pcmcc_init_tables(pcmcc_ctx* c, int n_e, double eps_min_eV, double eps_max_eV, int n_proc, const int* kind,
                      const double* threshold_eV, const double* sigma_m2, int flags) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (!c->species_ok) return fail(c, PCMCC_ESTATE, "species not initialised");
  c->tables_ok = false;
  if (!kind || !threshold_eV || !sigma_m2) return fail(c, PCMCC_EINVAL, "null table array");
  if (n_e < 2 || n_e > 4096 || n_proc < 1 || n_proc > kMaxProc)
    return fail(c, PCMCC_ETABLE, "table size out of range (n_e=%d, n_proc=%d)", n_e, n_proc);
  if ((size_t)(n_proc + 1) * n_e > kMaxTableFloats)
    return fail(c, PCMCC_ETABLE, "(n_proc + 1) * n_e exceeds %zu", kMaxTableFloats);
  if (!(eps_min_eV > 0) || !(eps_max_eV > eps_min_eV) || !std::isfinite(eps_max_eV))
    return fail(c, PCMCC_ETABLE, "bad energy range");
  if (flags & ~(PCMCC_EFFECTIVE_TO_ELASTIC | PCMCC_RATES)) return fail(c, PCMCC_EINVAL, "unknown flags");
  for (int k = 0; k < n_proc; ++k) {
    if (kind[k] < PCMCC_ELASTIC || kind[k] > PCMCC_ATTACHMENT) return fail(c, PCMCC_ETABLE, "bad kind %d", kind[k]);
    if (!(threshold_eV[k] >= 0) || !std::isfinite(threshold_eV[k])) return fail(c, PCMCC_ETABLE, "bad threshold");
  }
  for (size_t i = 0; i < (size_t)n_proc * n_e; ++i)
    if (!(sigma_m2[i] >= 0) || !std::isfinite(sigma_m2[i]))
      return fail(c, PCMCC_ETABLE, "negative or non-finite table value at %zu", i);
  HIP_TRY(c, hipSetDevice(c->device));
  dfree(c->dC);
  dfree(c->dP);
  dfree(c->dNu);
  c->dC = c->dP = c->dNu = nullptr;
  HIP_TRY(c, dalloc(&c->dC, (size_t)n_proc * n_e));
  HIP_TRY(c, dalloc(&c->dNu, (size_t)n_proc * n_e));
  HIP_TRY(c, dalloc(&c->dP, (size_t)n_e));
  double *dsig = nullptr, *dtot = nullptr;
  HIP_TRY(c, dalloc(&dsig, (size_t)n_proc * n_e));
  HIP_TRY(c, dalloc(&dtot, (size_t)n_e));
  TableBuild B{};
  B.n = n_e;
  B.nproc = n_proc;
  B.lnmin = std::log(eps_min_eV);
  B.dlog = (std::log(eps_max_eV) - B.lnmin) / (n_e - 1);
  B.ev = kEV;
  B.mass = c->mass;
  B.gas_N = c->gas_N;
  B.rates = (flags & PCMCC_RATES) ? 1 : 0;
  B.effective = (flags & PCMCC_EFFECTIVE_TO_ELASTIC) ? 1 : 0;
  for (int k = 0; k < n_proc; ++k) B.kind[k] = kind[k];
  B.sigma = dsig;
  B.total = dtot;
  hipError_t e = hipMemcpyAsync(dsig, sigma_m2, sizeof(double) * n_proc * n_e, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_build_tables(B, c->dC, c->dP, c->dNu, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dfree(dsig);
  dfree(dtot);
  if (e != hipSuccess) return fail(c, PCMCC_EHIP, "table build: %s", hipGetErrorString(e));
  c->n_e = n_e;
  c->n_proc = n_proc;
  c->eps_min = eps_min_eV;
  c->eps_max = eps_max_eV;
  for (int k = 0; k < kMaxProc; ++k) {
    c->kind[k] = k < n_proc ? kind[k] : PCMCC_ELASTIC;
    c->thr[k] = k < n_proc ? (float)threshold_eV[k] : 0.0f;
  }
  c->tables_ok = true;
  return PCMCC_OK;
}

int pcmcc_push_collide_deposit(pcmcc_ctx* c, const pcmcc_particles* p, const pcmcc_grid* field, double dt,
                               int n_steps, uint64_t seed, uint64_t step0, int64_t* rho, pcmcc_stats* stats) {
  return push_impl(c, p, field, dt, n_steps, seed, step0, rho, stats, nullptr);
}

int pcmcc_set_schedule(pcmcc_ctx* c, const pcmcc_schedule* s) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  const pcmcc_schedule v = s ? *s : pcmcc_schedule{};
  const int rc = check_schedule(c, v);
  if (rc) return rc;
  c->sched = v;
  return PCMCC_OK;
}

int pcmcc_get_schedule(pcmcc_ctx* c, pcmcc_schedule* out) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!out) return fail(c, PCMCC_EINVAL, "out is null");
  HIP_TRY(c, hipSetDevice(c->device));
  StepLaunch L;
  rc = resolve_launch(c, c->sched, pic_lds_bytes_s, occupancy_pic_steps, table_view(c), 0, &L);
  if (rc) return rc;
  *out = pcmcc_schedule{L.block, L.bpc, L.refill, L.chunk};
  return PCMCC_OK;
}

int pcmcc_autotune_steps(pcmcc_ctx* c, const pcmcc_particles* p, const pcmcc_grid* field, double dt, int n_steps,
                         uint64_t seed, uint64_t step0, const char* tune_cache, pcmcc_schedule* chosen,
                         float* tuned_ms, float* default_ms) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (tuned_ms) *tuned_ms = 0;
  if (default_ms) *default_ms = 0;
  if (!p || !p->x || !p->y || !p->z || !p->vx || !p->vy || !p->vz || !p->w || !p->id || !p->n_dev)
    return fail(c, PCMCC_EINVAL, "null particle array");
  if (!valid_grid(field)) return fail(c, PCMCC_EINVAL, "invalid field grid");
  if (n_steps < 1) return fail(c, PCMCC_EINVAL, "n_steps must be >= 1");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(c->host_n, p->n_dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int64_t n0 = *c->host_n;
  if (n0 < 0 || n0 > p->capacity) return fail(c, PCMCC_EINVAL, "particle count %lld outside [0, capacity]", (long long)n0);
  char keybuf[200];
  std::snprintf(keybuf, sizeof(keybuf), "gfx950:k_pic_steps:n2^%d:g%dx%dx%d:ne%d:np%d",
                n0 > 0 ? (int)std::lround(std::log2((double)n0)) : 0, field->nx, field->ny, field->nz, c->n_e,
                c->n_proc);
  const std::string key(keybuf);
  const uint64_t nh = (uint64_t)std::max<int64_t>(n0, 1);  // the population the schedules are resolved for
  load_tune_cache(c, tune_cache);
  if (c->tuned.count(key)) {
    const auto& t = c->tuned[key];
    const pcmcc_schedule s{t[0], t[1], t[2], t[3]};
    StepLaunch L;
    if (check_schedule(c, s) == PCMCC_OK &&
        resolve_launch(c, s, pic_lds_bytes_s, occupancy_pic_steps, table_view(c), 0, &L, nh) == PCMCC_OK) {
      c->sched = s;
      if (chosen) *chosen = pcmcc_schedule{L.block, L.bpc, L.refill, L.chunk};
      return PCMCC_OK;
    }
    c->err.clear();  // a stored schedule that no longer fits: tune again
  }
  // One copy of the input (7 float arrays, the ids, the count), restored
  // before every candidate and at the end; weight control is off meanwhile.
  const size_t nn = (size_t)std::max<int64_t>(n0, 1);
  char* bk = nullptr;
  HIP_TRY(c, hipMalloc((void**)&bk, nn * 36 + 8));
  float* const arr[7] = {p->x, p->y, p->z, p->vx, p->vy, p->vz, p->w};
  auto copy_all = [&](bool save) -> hipError_t {
    hipError_t e = hipSuccess;
    for (int k = 0; k < 7 && e == hipSuccess; ++k) {
      char* b = bk + (size_t)k * nn * 4;
      e = save ? hipMemcpyAsync(b, arr[k], (size_t)n0 * 4, hipMemcpyDeviceToDevice, c->stream)
               : hipMemcpyAsync(arr[k], b, (size_t)n0 * 4, hipMemcpyDeviceToDevice, c->stream);
    }
    char* bid = bk + 28 * nn;
    char* bn = bk + 36 * nn;
    if (e == hipSuccess)
      e = save ? hipMemcpyAsync(bid, p->id, (size_t)n0 * 8, hipMemcpyDeviceToDevice, c->stream)
               : hipMemcpyAsync(p->id, bid, (size_t)n0 * 8, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
      e = save ? hipMemcpyAsync(bn, p->n_dev, 8, hipMemcpyDeviceToDevice, c->stream)
               : hipMemcpyAsync(p->n_dev, bn, 8, hipMemcpyDeviceToDevice, c->stream);
    return e;
  };
  const pcmcc_schedule user = c->sched;
  const double wc_ppc = c->wc_n_ppc;
  const int64_t wc_ref = c->wc_n_ref;
  c->wc_n_ppc = 0;
  float best = 1e30f, t_default = 0;
  pcmcc_schedule best_s{};
  auto time_one = [&](const pcmcc_schedule& s, float* t_out) -> int {
    StepLaunch L;
    int r = resolve_launch(c, s, pic_lds_bytes_s, occupancy_pic_steps, table_view(c), 0, &L, nh);
    if (r) return r;
    c->sched = s;
    HIP_TRY(c, copy_all(false));
    pcmcc_stats st;
    r = push_impl(c, p, field, dt, n_steps, seed, step0, nullptr, &st, nullptr);
    if (r) return r;
    const float t = (float)st.step_kernel_ms;
    if (t_out) *t_out = t;
    if (t < best) {
      best = t;
      best_s = pcmcc_schedule{L.block, L.bpc, L.refill, L.chunk};
    }
    return (int)PCMCC_OK;
  };
  auto search = [&]() -> int {
    HIP_TRY(c, copy_all(true));
    int r = time_one(pcmcc_schedule{}, &t_default);
    if (r) return r;
    for (int b : {64, 128, 256, 512}) {
      StepLaunch fit;
      if (resolve_launch(c, pcmcc_schedule{b, 0, 0, 0}, pic_lds_bytes_s, occupancy_pic_steps, table_view(c), 0,
                         &fit)) {
        c->err.clear();
        continue;  // does not fit at this block size
      }
      for (int k = 1; k <= fit.bpc; k = (k * 2 > fit.bpc && k < fit.bpc) ? fit.bpc : k * 2) {
        r = time_one(pcmcc_schedule{b, k, 0, 0}, nullptr);
        if (r) return r;
      }
    }
    const pcmcc_schedule shape = best_s;
    for (int rf : kRefillChoices)
      for (int ch : {128, 256, 512, 1024}) {
        r = time_one(pcmcc_schedule{shape.block, shape.blocks_per_cu, rf, ch}, nullptr);
        if (r) return r;
      }
    return (int)PCMCC_OK;
  };
  rc = search();
  const hipError_t e = copy_all(false);  // the input state again, also after an error
  const hipError_t e2 = hipStreamSynchronize(c->stream);
  (void)hipFree(bk);
  c->wc_n_ppc = wc_ppc;
  c->wc_n_ref = wc_ref;
  if (rc) {
    c->sched = user;
    return rc;
  }
  HIP_TRY(c, e);
  HIP_TRY(c, e2);
  c->sched = best_s;
  c->tuned[key] = {best_s.block, best_s.blocks_per_cu, best_s.refill_min, best_s.chunk};
  save_tune_cache(c, tune_cache);
  if (chosen) *chosen = best_s;
  if (tuned_ms) *tuned_ms = best;
  if (default_ms) *default_ms = t_default;
  return PCMCC_OK;
}

int pcmcc_set_weight_control(pcmcc_ctx* c, double n_ppc, double growth) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (!(n_ppc >= 0) || !std::isfinite(n_ppc) || !(growth >= 1) || !std::isfinite(growth))
    return fail(c, PCMCC_EINVAL, "n_ppc must be >= 0 and growth >= 1");
  c->wc_n_ppc = n_ppc;
  c->wc_growth = growth;
  c->wc_n_ref = 0;
  return PCMCC_OK;
}

int pcmcc_update_weights(pcmcc_ctx* c, const pcmcc_particles* p, const pcmcc_grid* grid, double n_ppc,
                         uint64_t seed, uint64_t update_index, int64_t* merged_pairs, int64_t* splits) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (!p || !p->x || !p->y || !p->z || !p->vx || !p->vy || !p->vz || !p->w || !p->id || !p->n_dev)
    return fail(c, PCMCC_EINVAL, "null particle array");
  if (p->capacity < 1 || (uint64_t)p->capacity > 0xFFFFFFFFull)
    return fail(c, PCMCC_EINVAL, "capacity must be in [1, 2^32)");
  if (!valid_grid(grid)) return fail(c, PCMCC_EINVAL, "invalid grid");
  if (!(n_ppc > 0) || !std::isfinite(n_ppc)) return fail(c, PCMCC_EINVAL, "n_ppc must be positive");
  if (update_index > 0xFFFFFFFFull) return fail(c, PCMCC_EINVAL, "update index exceeds 32 bits");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(c->host_n, p->n_dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int64_t n = *c->host_n;
  if (n < 0 || n > p->capacity) return fail(c, PCMCC_EINVAL, "particle count %lld outside [0, capacity]", (long long)n);
  int rc = ensure_scratch(c, (uint64_t)p->capacity);
  if (rc) return rc;
  const Soa user{p->x, p->y, p->z, p->vx, p->vy, p->vz, p->w, p->id};
  uint64_t n_new = 0, pairs = 0, spl = 0;
  rc = weight_update(c, user, c->scratch, (uint64_t)n, grid, n_ppc, seed, update_index, (uint64_t)p->capacity,
                     &n_new, &pairs, &spl);
  if (rc) return rc;
  if (n > 0) {
    float* const dst[7] = {p->x, p->y, p->z, p->vx, p->vy, p->vz, p->w};
    float* const src[7] = {c->scratch.x, c->scratch.y, c->scratch.z, c->scratch.vx, c->scratch.vy, c->scratch.vz,
                           c->scratch.w};
    for (int k = 0; k < 7; ++k)
      HIP_TRY(c, hipMemcpyAsync(dst[k], src[k], n_new * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(p->id, c->scratch.id, n_new * sizeof(uint64_t), hipMemcpyDeviceToDevice, c->stream));
    *c->host_n = (int64_t)n_new;
    HIP_TRY(c, hipMemcpyAsync(p->n_dev, c->host_n, sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (merged_pairs) *merged_pairs = (int64_t)pairs;
  if (splits) *splits = (int64_t)spl;
  return PCMCC_OK;
}

int pcmcc_deposit(pcmcc_ctx* c, const float* x, const float* y, const float* z, const float* w,
                  const int64_t* n_dev, const pcmcc_grid* grid, int64_t* rho) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (!x || !y || !z || !w || !n_dev || !rho) return fail(c, PCMCC_EINVAL, "null array");
  if (!grid || grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || !(grid->dx > 0))
    return fail(c, PCMCC_EINVAL, "invalid grid");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(c->host_n, n_dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int64_t n = *c->host_n;
  if (n < 0) return fail(c, PCMCC_EINVAL, "negative particle count");
  const int rc = run_deposit(c, x, y, z, w, n_dev, (uint64_t)n, grid, rho);
  if (rc) return rc;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PCMCC_OK;
}

int pcmcc_philox4x32_10(pcmcc_ctx* c, int64_t n, const uint32_t* ctr, uint64_t seed, uint32_t* out) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (n < 0 || (n > 0 && (!ctr || !out))) return fail(c, PCMCC_EINVAL, "invalid arguments");
  if (n == 0) return PCMCC_OK;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, launch_philox(ctr, Key{(uint32_t)seed, (uint32_t)(seed >> 32)}, out, n, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PCMCC_OK;
}

int pcmcc_tables_lookup(pcmcc_ctx* c, int64_t n, const float* eps, float* cum_out, const float* s_ub,
                        float* maj_out) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (n < 0 || (n > 0 && (!eps || !cum_out))) return fail(c, PCMCC_EINVAL, "invalid arguments");
  if (maj_out && !s_ub) return fail(c, PCMCC_EINVAL, "majorant needs s_ub");
  if (n == 0) return PCMCC_OK;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, launch_lookup(table_view(c), species_view(c), eps, cum_out, s_ub, maj_out, n, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PCMCC_OK;
}

}  // extern "C"
