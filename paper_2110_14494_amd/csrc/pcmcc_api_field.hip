// C-ABI entry points of the self-consistent step (Sec. 2.5, Sec. 2.3,
// Sec. 2.1.4) and the discrete photoionization (Sec. 2.4).
#include "pcmcc_runtime.hpp"

extern "C" {

int pcmcc_solve_potential(pcmcc_ctx* c, const pcmcc_grid* grid, const int64_t* n_pos, const int64_t* n_e,
                          const int64_t* n_neg, double* phi, double tol, int max_cycles, int* cycles_out,
                          double* rel_residual_out) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (!valid_grid(grid) || !n_pos || !n_e || !n_neg || !phi) return fail(c, PCMCC_EINVAL, "invalid arguments");
  if (!(tol > 0) || max_cycles < 1) return fail(c, PCMCC_EINVAL, "tol must be > 0 and max_cycles >= 1");
  HIP_TRY(c, hipSetDevice(c->device));
  int rc = ensure_sc(c, grid);
  if (rc) return rc;
  int cyc = 0;
  double rel = 0;
  rc = solve_potential(c, grid, n_pos, n_e, n_neg, phi, tol, max_cycles, &cyc, &rel);
  if (rc) return rc;
  if (cycles_out) *cycles_out = cyc;
  if (rel_residual_out) *rel_residual_out = rel;
  return PCMCC_OK;
}

int pcmcc_photoionize(pcmcc_ctx* c, const pcmcc_grid* grid, const float* ev_x, const float* ev_y, const float* ev_z,
                      const float* ev_w, int64_t n_ev, const pcmcc_photo_opts* opts, uint64_t seed, uint64_t step,
                      const pcmcc_particles* p, int64_t* n_pos, int64_t* photons_out, int64_t* absorbed_out) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (!valid_grid(grid) || n_ev < 0 || (n_ev > 0 && (!ev_x || !ev_y || !ev_z || !ev_w)))
    return fail(c, PCMCC_EINVAL, "invalid grid or events");
  if (!valid_photo(opts)) return fail(c, PCMCC_EINVAL, "invalid photoionization options (eta >= 0, 0 < k1 < k2)");
  if (!p || !p->x || !p->y || !p->z || !p->vx || !p->vy || !p->vz || !p->w || !p->id || !p->n_dev ||
      p->capacity < 0)
    return fail(c, PCMCC_EINVAL, "invalid particle set");
  HIP_TRY(c, hipSetDevice(c->device));
  int64_t ph = 0, ab = 0;
  double ms = 0;
  const int rc = photoionize(c, grid, ev_x, ev_y, ev_z, ev_w, (uint64_t)n_ev, opts, seed, step, p, n_pos, &ph, &ab,
                             &ms);
  if (photons_out) *photons_out = ph;
  if (absorbed_out) *absorbed_out = ab;
  return rc;
}

int pcmcc_field_from_potential(pcmcc_ctx* c, const pcmcc_grid* applied, const double* phi, float* E_out) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (!valid_grid(applied) || !phi || !E_out) return fail(c, PCMCC_EINVAL, "invalid arguments");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, launch_sc_field((const float4*)applied->E, phi, applied->nx, applied->ny, applied->nz, applied->dx,
                             (float4*)E_out, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PCMCC_OK;
}

int pcmcc_speed_quantile(pcmcc_ctx* c, const float* vx, const float* vy, const float* vz, const int64_t* n_dev,
                         double* v90_out) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (!vx || !vy || !vz || !n_dev || !v90_out) return fail(c, PCMCC_EINVAL, "null argument");
  HIP_TRY(c, hipSetDevice(c->device));
  int rc = ensure_red(c);
  if (rc) return rc;
  HIP_TRY(c, hipMemcpyAsync(c->host_n, n_dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int64_t n = *c->host_n;
  if (n < 0) return fail(c, PCMCC_EINVAL, "negative count");
  *v90_out = 0;
  if (n == 0) return PCMCC_OK;
  HIP_TRY(c, launch_speed_select(vx, vy, vz, n_dev, (uint64_t)n, c->sel, c->sel_hist, c->stream));
  SelState st;
  HIP_TRY(c, hipMemcpyAsync(&st, c->sel, sizeof(st), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  float key;
  std::memcpy(&key, &st.prefix, sizeof(key));
  *v90_out = std::sqrt((double)key);
  return PCMCC_OK;
}

int pcmcc_streamer_steps(pcmcc_ctx* c, const pcmcc_particles* p, const pcmcc_grid* applied, int64_t* n_pos,
                         int64_t* n_neg, double* phi, float* E_out, const pcmcc_sc_opts* o, int n_steps, uint64_t seed,
                         uint64_t step0, double* dt_inout, double* dt_hist, pcmcc_stats* stats) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!p || !p->x || !p->n_dev || !valid_grid(applied) || !n_pos || !n_neg || !phi || !o || !dt_inout)
    return fail(c, PCMCC_EINVAL, "null argument");
  if (!(*dt_inout > 0) || !std::isfinite(*dt_inout) || n_steps < 0) return fail(c, PCMCC_EINVAL, "invalid dt or steps");
  if (o->adaptive && (!(o->dt_max > 0) || !(o->cfl > 0) || !(o->growth_max > 1) || o->mu_n < 1 || !o->mu_N ||
                      (o->mu_n > 1 && !(o->mu_EN_hi > o->mu_EN_lo && o->mu_EN_lo > 0))))
    return fail(c, PCMCC_EINVAL, "invalid time-step options");
  if (!(o->mg_tol > 0) || o->mg_max_cycles < 1) return fail(c, PCMCC_EINVAL, "invalid multigrid options");
  if (o->photo && !valid_photo(o->photo))
    return fail(c, PCMCC_EINVAL, "invalid photoionization options (eta >= 0, 0 < k1 < k2)");
  HIP_TRY(c, hipSetDevice(c->device));
  rc = ensure_sc(c, applied);
  if (rc) return rc;
  const size_t ncell = (size_t)applied->nx * applied->ny * applied->nz;
  // event lists: up to `capacity` ionizations and attachments per step
  const uint64_t cap = (uint64_t)p->capacity;
  if (c->ev_cap < cap) {
    dfree(c->ev_store);
    c->ev_store = nullptr;
    c->ev_cap = 0;
    HIP_TRY(c, dalloc(&c->ev_store, 8 * (size_t)cap));
    c->ev_cap = cap;
  }
  EventSink ev;
  float* e = c->ev_store;
  const size_t ec = (size_t)c->ev_cap;
  ev.ix = e; ev.iy = e + ec; ev.iz = e + 2 * ec; ev.iw = e + 3 * ec;
  ev.ax = e + 4 * ec; ev.ay = e + 5 * ec; ev.az = e + 6 * ec; ev.aw = e + 7 * ec;
  ev.n = c->sc_red + 5;
  ev.cap = c->ev_cap;
  ev.overflow = &c->ctl->overflow;
  pcmcc_grid cur = *applied;
  cur.E = (const float*)c->sc_E;
  const double gas_N = c->gas_N;
  double field_ms = 0, dep_ms = 0;
  int64_t mg_cycles = 0;
  // densities, potential and field of the present state
  int n_sol = 0;         // solutions so far (start-value extrapolation)
  double dt_last = 0;    // the step between the last two solutions
  auto refresh = [&](double dt_taken) -> int {
    HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
    int r0 = solve_start(c, phi, ncell, n_sol, dt_last > 0 ? dt_taken / dt_last : 0.0);
    if (r0) return r0;
    HIP_TRY(c, hipMemsetAsync(c->sc_ne, 0, ncell * sizeof(int64_t), c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->host_n, p->n_dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int r = run_deposit(c, p->x, p->y, p->z, p->w, p->n_dev, (uint64_t)*c->host_n, applied, c->sc_ne);
    if (r) return r;
    int cyc = 0;
    double rel = 0;
    r = solve_potential(c, applied, n_pos, c->sc_ne, n_neg, phi, o->mg_tol, o->mg_max_cycles, &cyc, &rel);
    if (r) return r;
    mg_cycles += cyc;
    if (n_sol >= 1) dt_last = dt_taken;
    ++n_sol;
    HIP_TRY(c, launch_sc_field((const float4*)applied->E, phi, applied->nx, applied->ny, applied->nz, applied->dx,
                               c->sc_E, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev[3], c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
    field_ms += ms;
    return PCMCC_OK;
  };
  auto weight_total = [&](double* out) -> int {
    HIP_TRY(c, hipMemsetAsync(c->sc_red + 4, 0, sizeof(unsigned long long), c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->host_n, p->n_dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, launch_weight_sum(p->w, p->n_dev, (uint64_t)*c->host_n, (double*)(c->sc_red + 4), c->stream));
    int r = read_red(c, 4, 1);
    if (r) return r;
    std::memcpy(out, &c->sc_host[4], sizeof(double));
    return PCMCC_OK;
  };
  rc = refresh(0.0);
  if (rc) return rc;
  double n_old = 0;
  if (o->adaptive) {
    rc = weight_total(&n_old);
    if (rc) return rc;
  }
  double dt = *dt_inout;
  pcmcc_stats tot{};
  int s = 0;
  for (; s < n_steps; ++s) {
    HIP_TRY(c, hipMemsetAsync(ev.n, 0, 2 * sizeof(unsigned long long), c->stream));
    pcmcc_stats st{};
    rc = push_impl(c, p, &cur, dt, 1, seed, step0 + (uint64_t)s, nullptr, &st, &ev);
    if (rc) break;
    tot.n = st.n;
    tot.steps_done += st.steps_done;
    tot.particle_steps += st.particle_steps;
    tot.trials += st.trials;
    tot.null_collisions += st.null_collisions;
    for (int k = 0; k < 4; ++k) tot.real_collisions[k] += st.real_collisions[k];
    tot.lost += st.lost;
    tot.out_of_table += st.out_of_table;
    tot.errors += st.errors;
    tot.majorant_violations += st.majorant_violations;
    tot.step_kernel_ms += st.step_kernel_ms;
    tot.launch_block = st.launch_block;
    tot.launch_grid = st.launch_grid;
    tot.launch_refill = st.launch_refill;
    tot.launch_chunk = st.launch_chunk;
    tot.weight_updates += st.weight_updates;
    tot.merged_pairs += st.merged_pairs;
    tot.splits += st.splits;
    tot.weight_ms += st.weight_ms;
    // ions of the step's events
    rc = read_red(c, 5, 2);
    if (rc) break;
    const uint64_t n_ion = c->sc_host[5], n_att = c->sc_host[6];
    HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
    if (n_ion) {
      rc = run_deposit(c, ev.ix, ev.iy, ev.iz, ev.iw, (const int64_t*)ev.n, n_ion, applied, n_pos);
      if (rc) break;
    }
    if (n_att) {
      rc = run_deposit(c, ev.ax, ev.ay, ev.az, ev.aw, (const int64_t*)(ev.n + 1), n_att, applied, n_neg);
      if (rc) break;
    }
    HIP_TRY(c, hipEventRecord(c->ev[3], c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
    dep_ms += ms;
    if (o->photo && n_ion) {
      int64_t ph = 0, ab = 0;
      double pms = 0;
      rc = photoionize(c, applied, ev.ix, ev.iy, ev.iz, ev.iw, n_ion, o->photo, seed, step0 + (uint64_t)s, p, n_pos,
                       &ph, &ab, &pms);
      tot.photons += ph;
      tot.photoelectrons += ab;
      tot.photo_ms += pms;
      if (rc) break;
    }
    rc = refresh(dt);
    if (rc) break;
    if (dt_hist) dt_hist[s] = dt;
    if (o->adaptive) {
      double v90 = 0;
      rc = pcmcc_speed_quantile(c, p->vx, p->vy, p->vz, p->n_dev, &v90);
      if (rc) break;
      // the densest cell and the field there
      c->sc_host[2] = 0x8000000000000000ull;
      c->sc_host[3] = ~0ull;
      HIP_TRY(c, hipMemcpyAsync(c->sc_red + 2, c->sc_host + 2, 2 * sizeof(unsigned long long), hipMemcpyHostToDevice,
                                c->stream));
      HIP_TRY(c, launch_densest(c->sc_ne, ncell, (long long*)(c->sc_red + 2), c->sc_red + 3, c->stream));
      rc = read_red(c, 2, 2);
      if (rc) break;
      const long long ne_units = (long long)c->sc_host[2];
      const uint64_t cell = c->sc_host[3];
      double ne_max = 0, e_at = 0;
      if (ne_units > 0 && cell < ncell) {
        float4 Ec;
        HIP_TRY(c, hipMemcpyAsync(&Ec, c->sc_E + cell, sizeof(Ec), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        ne_max = (double)ne_units * 0x1p-32 / (applied->dx * applied->dx * applied->dx);
        const double ex = Ec.x, ey = Ec.y, ez = Ec.z;
        e_at = std::sqrt(ex * ex + ey * ey + ez * ez);
      }
      const double mu_e = ne_max > 0 ? mobility(o, e_at / gas_N * 1e21, gas_N) : 0.0;
      double n_new = 0;
      rc = weight_total(&n_new);
      if (rc) break;
      double nd = o->dt_max;
      if (v90 > 0) nd = std::min(nd, o->cfl * applied->dx / v90);
      if (ne_max > 0 && mu_e > 0) nd = std::min(nd, kEps0 / (kQe * ne_max * mu_e));
      if (n_old > 0 && n_new > n_old) nd = std::min(nd, dt * std::log(o->growth_max) / std::log(n_new / n_old));
      dt = nd;
      n_old = n_new;
    }
  }
  *dt_inout = dt;
  if (E_out) {
    HIP_TRY(c, hipMemcpyAsync(E_out, c->sc_E, ncell * sizeof(float4), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  if (stats) {
    *stats = tot;
    stats->deposit_kernel_ms = dep_ms;
    stats->field_ms = field_ms;
    stats->mg_cycles = mg_cycles;
  }
  return rc;
}

}  // extern "C"
