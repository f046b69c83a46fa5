// C-ABI entry point of the fluid step (Sec. 2.2).
#include "pcmcc_runtime.hpp"

extern "C" {

int pcmcc_fluid_steps(pcmcc_ctx* c, const pcmcc_grid* applied, double* n_e, double* n_pos, double* n_neg,
                      double* phi, const pcmcc_fluid_table* tab, double dt_max, double mg_tol, int mg_max_cycles,
                      int n_steps, double* dt_hist, float* E_out, pcmcc_stats* stats) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!c->species_ok) return fail(c, PCMCC_ESTATE, "species not initialised (the gas density is needed)");
  if (!(c->gas_N > 0)) return fail(c, PCMCC_EINVAL, "the fluid step needs a gas density > 0");
  if (!valid_grid(applied) || !n_e || !n_pos || !n_neg || !phi || !tab) return fail(c, PCMCC_EINVAL, "null argument");
  if (tab->n < 2 || !(tab->EN_lo > 0) || !(tab->EN_hi > tab->EN_lo) || !tab->muN || !tab->DN || !tab->alphaN ||
      !tab->etaN)
    return fail(c, PCMCC_EINVAL, "invalid transport table");
  if (!(dt_max > 0) || !(mg_tol > 0) || mg_max_cycles < 1 || n_steps < 0)
    return fail(c, PCMCC_EINVAL, "invalid dt_max, multigrid options or step count");
  HIP_TRY(c, hipSetDevice(c->device));
  int rc = ensure_sc(c, applied);
  if (rc) return rc;
  const size_t ncell = (size_t)applied->nx * applied->ny * applied->nz;
  if (c->fl_cells < ncell) {
    dfree(c->fl_store);
    c->fl_store = nullptr;
    c->fl_cells = 0;
    HIP_TRY(c, dalloc(&c->fl_store, 6 * ncell));
    c->fl_cells = ncell;
  }
  if (c->fl_tab_n < tab->n) {
    dfree(c->fl_tab);
    c->fl_tab = nullptr;
    c->fl_tab_n = 0;
    HIP_TRY(c, dalloc(&c->fl_tab, 4 * (size_t)tab->n));
    c->fl_tab_n = tab->n;
  }
  const double* src[4] = {tab->muN, tab->DN, tab->alphaN, tab->etaN};
  for (int q = 0; q < 4; ++q)
    HIP_TRY(c, hipMemcpyAsync(c->fl_tab + (size_t)q * tab->n, src[q], tab->n * sizeof(double), hipMemcpyHostToDevice,
                              c->stream));
  FluidArgs A{};
  A.nx = applied->nx;
  A.ny = applied->ny;
  A.nz = applied->nz;
  A.dx = applied->dx;
  A.E = c->sc_E;
  A.ne = n_e;
  A.np = n_pos;
  A.nn = n_neg;
  double* q = c->fl_store;
  A.se = q;
  A.sp = q + ncell;
  A.sn = q + 2 * ncell;
  A.k1e = q + 3 * ncell;
  A.k1p = q + 4 * ncell;
  A.k1n = q + 5 * ncell;
  A.T.n = tab->n;
  A.T.ln_lo = std::log(tab->EN_lo);
  A.T.ln_span = std::log(tab->EN_hi) - A.T.ln_lo;
  A.T.muN = c->fl_tab;
  A.T.DN = c->fl_tab + tab->n;
  A.T.aN = c->fl_tab + 2 * (size_t)tab->n;
  A.T.eN = c->fl_tab + 3 * (size_t)tab->n;
  A.T.gas_N = c->gas_N;
  A.T.pos_scale = (double)(tab->n - 1) / A.T.ln_span;
  A.T.inv_gas_N = 1.0 / c->gas_N;
  A.T.ln_td = std::log(1e21 / c->gas_N);
  double field_ms = 0, stage_ms = 0;
  int64_t cycles = 0;
  auto field = [&](const double* ne, const double* np, const double* nn) -> int {
    HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
    HIP_TRY(c, hipMemsetAsync(c->sc_red, 0, 2 * sizeof(unsigned long long), c->stream));
    HIP_TRY(c, launch_fluid_rhs(np, ne, nn, ncell, c->mg.rhs, c->sc_red, c->stream));
    int cyc = 0;
    double rel = 0;
    int r = mg_iterate(c, applied, phi, mg_tol, mg_max_cycles, &cyc, &rel);
    if (r) return r;
    cycles += cyc;
    HIP_TRY(c, launch_sc_field((const float4*)applied->E, phi, applied->nx, applied->ny, applied->nz, applied->dx,
                               c->sc_E, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev[3], c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
    field_ms += ms;
    return PCMCC_OK;
  };
  rc = field(n_e, n_pos, n_neg);
  if (rc) return rc;
  int n_sol = 1;       // solutions of the states at whole steps (start-value extrapolation)
  double dt_last = 0;  // the step between the last two of them
  int s = 0;
  for (; s < n_steps; ++s) {
    HIP_TRY(c, hipMemsetAsync(c->sc_red + 2, 0, 2 * sizeof(unsigned long long), c->stream));
    HIP_TRY(c, launch_fluid_dt(n_e, c->sc_E, ncell, A.T, applied->dx, c->sc_red + 2, c->stream));
    rc = read_red(c, 2, 2);
    if (rc) break;
    double cm, dm;
    std::memcpy(&cm, &c->sc_host[2], sizeof(double));
    std::memcpy(&dm, &c->sc_host[3], sizeof(double));
    const double dt_cfl = cm > 0 ? 0.5 / cm : HUGE_VAL, dt_drt = dm > 0 ? 1.0 / dm : HUGE_VAL;
    const double dt = std::min(dt_max, 0.9 * std::min(dt_cfl, dt_drt));
    A.dt = dt;
    HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
    HIP_TRY(c, launch_fluid_stage(A, 1, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    stage_ms += ms;
    rc = solve_start(c, phi, ncell, n_sol, dt_last > 0 ? dt / dt_last : 0.0);  // from the last two steps' fields
    if (rc) break;
    rc = field(A.se, A.sp, A.sn);
    if (rc) break;
    HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
    HIP_TRY(c, launch_fluid_stage(A, 2, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    stage_ms += ms;
    rc = field(n_e, n_pos, n_neg);
    if (rc) break;
    if (n_sol >= 1) dt_last = dt;
    ++n_sol;
    if (dt_hist) dt_hist[s] = dt;
  }
  if (E_out) {
    HIP_TRY(c, hipMemcpyAsync(E_out, c->sc_E, ncell * sizeof(float4), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  if (stats) {
    stats->steps_done = s;
    stats->step_kernel_ms = stage_ms;
    stats->field_ms = field_ms;
    stats->mg_cycles = cycles;
  }
  return rc;
}

}  // extern "C"
