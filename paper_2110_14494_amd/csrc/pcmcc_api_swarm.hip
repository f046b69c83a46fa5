// C-ABI entry point of the batched uniform-field swarms (Sec. 2.2.2 flux and
// bulk coefficients): scratch, launch-shape tuning and the estimators.
#include "pcmcc_runtime.hpp"

extern "C" {

namespace {

// One run of the swarm step loop with a given launch schedule (inputs
// already on the device); the kernel time in ms goes to *ms.
int swarm_run(pcmcc_ctx* c, SwarmArgs& A, int S, const std::vector<uint64_t>& n0h, const StepLaunch& L, float* ms) {
  A.chunk = (uint32_t)L.chunk;
  auto& w = c->sw;
  HIP_TRY(c, hipMemsetAsync(w.n_nxt, 0, sizeof(unsigned long long) * S, c->stream));
  HIP_TRY(c, hipMemsetAsync(w.cum_ion, 0, sizeof(unsigned long long) * S, c->stream));
  HIP_TRY(c, hipMemsetAsync(w.cum_att, 0, sizeof(unsigned long long) * S, c->stream));
  HIP_TRY(c, hipMemsetAsync(w.pc_k, 0, sizeof(int) * S, c->stream));
  HIP_TRY(c, hipMemsetAsync(w.L, 0, sizeof(long long) * S, c->stream));
  HIP_TRY(c, hipMemsetAsync(w.mom, 0, sizeof(unsigned long long) * S * A.n_samples * kNMom * 2, c->stream));
  HIP_TRY(c, hipMemsetAsync(w.cnt, 0, sizeof(long long) * S * A.n_samples * 4, c->stream));
  HIP_TRY(c, hipMemsetAsync(w.ctl, 0, sizeof(SwarmCtl), c->stream));
  HIP_TRY(c, hipMemcpyAsync(w.n_cur, n0h.data(), sizeof(uint64_t) * S, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_swarm_init(w.buf[0], w.base, w.n0, S, c->stream));
  HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
  HIP_TRY(c, launch_swarm_steps(A, L.grid, L.block, L.refill, c->stream));
  HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
  HIP_TRY(c, hipEventSynchronize(c->ev[1]));
  HIP_TRY(c, hipEventElapsedTime(ms, c->ev[0], c->ev[1]));
  return PCMCC_OK;
}

}  // namespace

int pcmcc_swarm_batch(pcmcc_ctx* c, int n_swarms, const double* EN_Td, const int32_t* n0, double dt, int n_steps,
                      uint64_t seed, const pcmcc_swarm_opts* opts, pcmcc_swarm_result* out, double* moments_out,
                      int64_t* counters_out, pcmcc_stats* stats) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!EN_Td || !n0 || !opts || !out) return fail(c, PCMCC_EINVAL, "null argument");
  const int S = n_swarms;
  if (S < 1 || S > 4096) return fail(c, PCMCC_EINVAL, "n_swarms must be in [1, 4096]");
  if (!(dt > 0) || !std::isfinite(dt) || n_steps < 1) return fail(c, PCMCC_EINVAL, "invalid dt or n_steps");
  if (opts->sample_every < 1 || opts->n_batches < 2 || opts->cap_factor < 4 || !std::isfinite(opts->window_start_s))
    return fail(c, PCMCC_EINVAL, "invalid swarm options");
  const int J = n_steps / opts->sample_every;
  if (J < 2 * opts->n_batches) return fail(c, PCMCC_EINVAL, "fewer samples than 2 * n_batches");
  std::vector<uint64_t> base(S), caps(S), n0h(S);
  std::vector<double> az(S);
  uint64_t slots = 0;
  for (int s = 0; s < S; ++s) {
    if (n0[s] < 1) return fail(c, PCMCC_EINVAL, "n0[%d] < 1", s);
    if (!(EN_Td[s] >= 0) || !std::isfinite(EN_Td[s])) return fail(c, PCMCC_EINVAL, "bad EN_Td[%d]", s);
    base[s] = slots;
    caps[s] = (uint64_t)opts->cap_factor * (uint64_t)n0[s];
    n0h[s] = (uint64_t)n0[s];
    slots += caps[s];
    az[s] = (c->charge / c->mass) * EN_Td[s] * 1e-21 * c->gas_N;
  }
  if (slots > 0xFFFFFFFFull) return fail(c, PCMCC_EINVAL, "total swarm slots exceed 2^32");
  HIP_TRY(c, hipSetDevice(c->device));
  const TableView T = table_view(c);
  // Launch schedule: explicit fields, else the tuned (cached) ones for this
  // workload, else the defaults.
  char keybuf[160];
  std::snprintf(keybuf, sizeof(keybuf), "gfx950:k_swarm_steps:S%d:N%llu:cap%d:se%d:ne%d:np%d", S,
                (unsigned long long)(slots / opts->cap_factor), opts->cap_factor, opts->sample_every, c->n_e,
                c->n_proc);
  const std::string key(keybuf);
  load_tune_cache(c, opts->tune_cache);
  pcmcc_schedule want{opts->block, opts->blocks_per_cu, opts->refill_min, opts->chunk};
  rc = check_schedule(c, want);
  if (rc) return rc;
  if (!opts->autotune && c->tuned.count(key)) {
    const auto& t = c->tuned[key];
    if (!want.block) {
      want.block = t[0];
      if (!want.blocks_per_cu) want.blocks_per_cu = t[1];
    }
    if (!want.refill_min) want.refill_min = t[2];
    if (!want.chunk) want.chunk = t[3];
    if (check_schedule(c, want)) want = pcmcc_schedule{opts->block, opts->blocks_per_cu, opts->refill_min, opts->chunk};
  }
  auto resolve = [&](const pcmcc_schedule& s, StepLaunch* L) {
    return resolve_launch(c, s, swarm_lds_bytes_s, occupancy_swarm_steps, T, S, L);
  };
  const int max_grid = 32 * c->num_cu;
  rc = ensure_swarm(c, S, slots, J, max_grid);
  if (rc) return rc;
  auto& w = c->sw;
  HIP_TRY(c, hipMemcpyAsync(w.base, base.data(), sizeof(uint64_t) * S, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(w.cap_s, caps.data(), sizeof(uint64_t) * S, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(w.n0, n0, sizeof(int32_t) * S, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(w.az, az.data(), sizeof(double) * S, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(w.EN, EN_Td, sizeof(double) * S, hipMemcpyHostToDevice, c->stream));
  SwarmArgs A{};
  A.buf[0] = w.buf[0];
  A.buf[1] = w.buf[1];
  A.pend[0] = w.pend[0];
  A.pend[1] = w.pend[1];
  A.pend_cap = w.pend_cap;
  A.n_swarms = S;
  A.base = w.base;
  A.cap_s = w.cap_s;
  A.n0 = w.n0;
  A.az = w.az;
  A.ctl = w.ctl;
  A.n_cur = w.n_cur;
  A.n_nxt = w.n_nxt;
  A.pc_k = w.pc_k;
  A.L = w.L;
  A.cum_ion = w.cum_ion;
  A.cum_att = w.cum_att;
  A.mom = w.mom;
  A.cnt_out = w.cnt;
  A.partial = w.partial;
  A.partial_ps = w.partial_ps;
  A.T = T;
  A.S = species_view(c);
  A.key = Key{(uint32_t)seed, (uint32_t)(seed >> 32)};
  A.dt = (float)dt;
  A.sample_every = opts->sample_every;
  A.n_samples = J;
  A.pop_control = opts->population_control ? 1 : 0;
  float ms = 0;
  if (opts->autotune) {
    // Time the candidates on the first min(n_steps, 200) steps: block x
    // blocks per CU at the default refill and chunk, then refill x chunk at
    // the fastest shape.
    SwarmArgs probe = A;
    probe.n_steps = std::min(n_steps, 200);
    float best = 1e30f;
    pcmcc_schedule best_s{};
    auto time_one = [&](const pcmcc_schedule& s) {
      StepLaunch L;
      int r = resolve(s, &L);
      if (r) return r;
      float t = 0;
      r = swarm_run(c, probe, S, n0h, L, &t);
      if (r) return r;
      if (t < best) {
        best = t;
        best_s = pcmcc_schedule{L.block, L.bpc, L.refill, L.chunk};
      }
      return (int)PCMCC_OK;
    };
    for (int b : {64, 128, 256, 512}) {
      StepLaunch fit;
      if (resolve(pcmcc_schedule{b, 0, 0, 0}, &fit)) {
        c->err.clear();
        continue;  // does not fit at this block size
      }
      const int kmax = std::min(fit.bpc, 32);
      for (int k = 1; k <= kmax; k = (k * 2 > kmax && k < kmax) ? kmax : k * 2) {
        rc = time_one(pcmcc_schedule{b, k, 0, 0});
        if (rc) return rc;
      }
    }
    const pcmcc_schedule shape = best_s;
    for (int r : kRefillChoices)
      for (int ch : {128, 256, 512, 1024}) {
        rc = time_one(pcmcc_schedule{shape.block, shape.blocks_per_cu, r, ch});
        if (rc) return rc;
      }
    want = best_s;
    c->tuned[key] = {want.block, want.blocks_per_cu, want.refill_min, want.chunk};
    save_tune_cache(c, opts->tune_cache);
  }
  StepLaunch L;
  rc = resolve(want, &L);
  if (rc == PCMCC_EINVAL && want.blocks_per_cu && !opts->blocks_per_cu) {  // a cached shape that no longer fits
    want.blocks_per_cu = 0;
    rc = resolve(want, &L);
  }
  if (rc) return rc;
  const int block = L.block, grid = L.grid;
  A.n_steps = n_steps;
  rc = swarm_run(c, A, S, n0h, L, &ms);
  if (rc) return rc;
  SwarmCtl hc;
  HIP_TRY(c, hipMemcpy(&hc, w.ctl, sizeof(SwarmCtl), hipMemcpyDeviceToHost));
  if (hc.status == PCMCC_OK) {
    HIP_TRY(c, launch_swarm_estimate(w.mom, w.cnt, S, J, opts->sample_every * dt, opts->window_start_s,
                                     opts->n_batches, w.EN, c->gas_N, w.values, w.errors, w.work, c->stream));
    std::vector<double> vals((size_t)S * kNQ), errs((size_t)S * kNQ);
    HIP_TRY(c, hipMemcpyAsync(vals.data(), w.values, sizeof(double) * S * kNQ, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(errs.data(), w.errors, sizeof(double) * S * kNQ, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int s = 0; s < S; ++s)
      for (int k = 0; k < kNQ; ++k) {
        out[s].value[k] = vals[(size_t)s * kNQ + k];
        out[s].error[k] = errs[(size_t)s * kNQ + k];
      }
  }
  if (moments_out || counters_out) {
    std::vector<unsigned long long> m((size_t)S * J * kNMom * 2);
    std::vector<long long> cn((size_t)S * J * 4);
    HIP_TRY(c, hipMemcpy(m.data(), w.mom, sizeof(unsigned long long) * m.size(), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(cn.data(), w.cnt, sizeof(long long) * cn.size(), hipMemcpyDeviceToHost));
    if (moments_out)
      for (size_t i = 0; i < (size_t)S * J * kNMom; ++i) {
        const double v = (double)(long long)m[2 * i + 1] * 18446744073709551616.0 + (double)m[2 * i];
        moments_out[i] = std::ldexp(v, -kMomExpHost[i % kNMom]);
      }
    if (counters_out)
      for (size_t i = 0; i < cn.size(); ++i) counters_out[i] = (int64_t)cn[i];
  }
  if (stats) {
    stats->steps_done = hc.steps_done;
    stats->particle_steps = hc.particle_steps;
    stats->trials = hc.tot[C_TRIALS];
    stats->null_collisions = hc.tot[C_NULL];
    for (int k = 0; k < 4; ++k) stats->real_collisions[k] = hc.tot[C_EL + k];
    stats->out_of_table = hc.tot[C_OOT];
    stats->errors = hc.tot[C_ERR];
    stats->majorant_violations = hc.tot[C_MAJ];
    stats->step_kernel_ms = ms;
    stats->launch_block = block;
    stats->launch_grid = grid;
    stats->launch_refill = L.refill;
    stats->launch_chunk = L.chunk;
  }
  if (hc.status == PCMCC_ECAPACITY)
    return fail(c, hc.status, "a swarm outgrew its %d x n0 slots after %lld steps", opts->cap_factor,
                (long long)hc.steps_done);
  if (hc.status != PCMCC_OK) return fail(c, hc.status, "swarm step loop stopped (status %d)", hc.status);
  return PCMCC_OK;
}

}  // extern "C"
