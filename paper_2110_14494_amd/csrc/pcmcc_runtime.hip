// Host runtime helpers of the PIC-MCC electron library (declared in
// pcmcc_runtime.hpp): error text, device buffers of the context, argument
// checks, field preparation, the charge deposit and the weight update.
#include "pcmcc_runtime.hpp"

namespace pcmcc_rt {

std::string g_last_error;

int fail(pcmcc_ctx* ctx, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx)
    ctx->err = buf;
  else
    g_last_error = buf;
  return code;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

void free_scratch(pcmcc_ctx* c) {
  float** fs[] = {&c->scratch.x, &c->scratch.y, &c->scratch.z, &c->scratch.vx, &c->scratch.vy, &c->scratch.vz,
                  &c->scratch.w};
  for (float** f : fs) {
    dfree(*f);
    *f = nullptr;
  }
  dfree(c->scratch.id);
  c->scratch.id = nullptr;
  for (auto& q : c->pend) {
    float** qs[] = {&q.x, &q.y, &q.z, &q.vx, &q.vy, &q.vz, &q.w, &q.tb};
    for (float** f : qs) {
      dfree(*f);
      *f = nullptr;
    }
    dfree(q.id);
    q.id = nullptr;
  }
  dfree(c->holes);
  dfree(c->flags);
  dfree(c->donor);
  c->holes = c->flags = c->donor = nullptr;
  c->cap = c->pend_cap = 0;
}

// Scratch for `cap` particles: the second particle buffer, two newborn
// queues of cap/2 each (at least 4096), and the hole lists.
int ensure_scratch(pcmcc_ctx* c, uint64_t cap) {
  if (c->cap >= cap && c->scratch.x) return PCMCC_OK;
  free_scratch(c);
  const uint64_t pc = std::max<uint64_t>(cap / 2, 4096);
  float** fs[] = {&c->scratch.x, &c->scratch.y, &c->scratch.z, &c->scratch.vx, &c->scratch.vy, &c->scratch.vz,
                  &c->scratch.w};
  for (float** f : fs) HIP_TRY(c, dalloc(f, cap));
  HIP_TRY(c, dalloc(&c->scratch.id, cap));
  for (auto& q : c->pend) {
    float** qs[] = {&q.x, &q.y, &q.z, &q.vx, &q.vy, &q.vz, &q.w, &q.tb};
    for (float** f : qs) HIP_TRY(c, dalloc(f, pc));
    HIP_TRY(c, dalloc(&q.id, pc));
  }
  HIP_TRY(c, dalloc(&c->holes, cap));
  HIP_TRY(c, dalloc(&c->flags, cap));
  HIP_TRY(c, dalloc(&c->donor, cap));
  c->cap = cap;
  c->pend_cap = pc;
  return PCMCC_OK;
}

void free_soa(Soa& b) {
  float** fs[] = {&b.x, &b.y, &b.z, &b.vx, &b.vy, &b.vz, &b.w};
  for (float** f : fs) {
    dfree(*f);
    *f = nullptr;
  }
  dfree(b.id);
  b.id = nullptr;
}

void free_pend(PendSoa& q) {
  float** qs[] = {&q.x, &q.y, &q.z, &q.vx, &q.vy, &q.vz, &q.w, &q.tb};
  for (float** f : qs) {
    dfree(*f);
    *f = nullptr;
  }
  dfree(q.id);
  dfree(q.sw);
  q.id = nullptr;
  q.sw = nullptr;
}

void free_swarm(pcmcc_ctx* c) {
  auto& w = c->sw;
  for (auto& b : w.buf) free_soa(b);
  for (auto& q : w.pend) free_pend(q);
  void* ps[] = {w.base, w.cap_s, w.n0, w.az, w.EN, w.n_cur, w.n_nxt, w.cum_ion, w.cum_att, w.pc_k, w.L,
                w.mom, w.cnt, w.partial, w.partial_ps, w.ctl, w.values, w.errors, w.work};
  for (void* q : ps) dfree(q);
  w = pcmcc_ctx::Swarm{};
}

int alloc_soa(pcmcc_ctx* c, Soa& b, uint64_t n) {
  float** fs[] = {&b.x, &b.y, &b.z, &b.vx, &b.vy, &b.vz, &b.w};
  for (float** f : fs) HIP_TRY(c, dalloc(f, n));
  HIP_TRY(c, dalloc(&b.id, n));
  return PCMCC_OK;
}

int alloc_pend(pcmcc_ctx* c, PendSoa& q, uint64_t n, bool with_sw) {
  float** qs[] = {&q.x, &q.y, &q.z, &q.vx, &q.vy, &q.vz, &q.w, &q.tb};
  for (float** f : qs) HIP_TRY(c, dalloc(f, n));
  HIP_TRY(c, dalloc(&q.id, n));
  if (with_sw) HIP_TRY(c, dalloc(&q.sw, n));
  return PCMCC_OK;
}

// Swarm scratch for S swarms, `slots` particle slots, J samples, `grid` blocks.
int ensure_swarm(pcmcc_ctx* c, int S, uint64_t slots, int J, int grid) {
  auto& w = c->sw;
  if (w.S >= S && w.slots >= slots && w.J >= J && w.grid >= grid && w.ctl) return PCMCC_OK;
  free_swarm(c);
  int rc;
  for (auto& b : w.buf)
    if ((rc = alloc_soa(c, b, slots))) return rc;
  const uint64_t pc = std::max<uint64_t>(slots / 4, 1 << 16);
  for (auto& q : w.pend)
    if ((rc = alloc_pend(c, q, pc, true))) return rc;
  HIP_TRY(c, dalloc(&w.base, S));
  HIP_TRY(c, dalloc(&w.cap_s, S));
  HIP_TRY(c, dalloc(&w.n0, S));
  HIP_TRY(c, dalloc(&w.az, S));
  HIP_TRY(c, dalloc(&w.EN, S));
  HIP_TRY(c, dalloc(&w.n_cur, S));
  HIP_TRY(c, dalloc(&w.n_nxt, S));
  HIP_TRY(c, dalloc(&w.cum_ion, S));
  HIP_TRY(c, dalloc(&w.cum_att, S));
  HIP_TRY(c, dalloc(&w.pc_k, S));
  HIP_TRY(c, dalloc(&w.L, S));
  HIP_TRY(c, dalloc(&w.mom, (size_t)S * J * kNMom * 2));
  HIP_TRY(c, dalloc(&w.cnt, (size_t)S * J * 4));
  HIP_TRY(c, dalloc(&w.partial, (size_t)grid * NCNT));
  HIP_TRY(c, dalloc(&w.partial_ps, (size_t)grid));
  HIP_TRY(c, dalloc(&w.ctl, 1));
  HIP_TRY(c, dalloc(&w.values, (size_t)S * kNQ));
  HIP_TRY(c, dalloc(&w.errors, (size_t)S * kNQ));
  HIP_TRY(c, dalloc(&w.work, (size_t)S * 11 * J));
  w.S = S;
  w.slots = slots;
  w.J = J;
  w.grid = grid;
  w.pend_cap = pc;
  return PCMCC_OK;
}

int check_schedule(pcmcc_ctx* c, const pcmcc_schedule& s) {
  if (s.block != 0 && s.block != 64 && s.block != 128 && s.block != 256 && s.block != 512)
    return fail(c, PCMCC_EINVAL, "block must be 0, 64, 128, 256 or 512");
  if (s.blocks_per_cu < 0 || s.blocks_per_cu > 32) return fail(c, PCMCC_EINVAL, "blocks_per_cu must be in [0, 32]");
  if (s.refill_min != 0 && s.refill_min != 16 && s.refill_min != 24 && s.refill_min != 32)
    return fail(c, PCMCC_EINVAL, "refill_min must be 0, 16, 24 or 32");
  if (s.chunk != 0 && (s.chunk < (int)kChunkMin || s.chunk > (int)kChunkMax || (s.chunk & (s.chunk - 1))))
    return fail(c, PCMCC_EINVAL, "chunk must be 0 or a power of two in [64, 4096]");
  return PCMCC_OK;
}

int resolve_launch(pcmcc_ctx* c, const pcmcc_schedule& s, size_t (*lds)(const TableView&, int, int),
                   hipError_t (*occ)(int, int, int, size_t, int*), const TableView& T, int S, StepLaunch* out,
                   uint64_t n_hint) {
  const int rc = check_schedule(c, s);
  if (rc) return rc;
  const bool small = n_hint > 0 && n_hint < kSmallPopulation && !s.block;
  const int refill = s.refill_min ? s.refill_min : 24;
  const int chunk = s.chunk ? s.chunk : (small ? 64 : 512);
  int block = 0, per_cu = 0;
  for (int b : {512, 256, 128, 64}) {
    if ((s.block && b != s.block) || (small && b != 64)) continue;
    int k = 0;
    HIP_TRY(c, occ(b, refill, table_row(T.nproc), lds(T, S, b), &k));
    if (k >= 1 && k * b > per_cu * block) {  // most resident waves; ties keep the larger block
      block = b;
      per_cu = k;
    }
  }
  if (!block) return fail(c, PCMCC_EHIP, "the step kernel does not fit on a compute unit (block %d)", s.block);
  if (s.blocks_per_cu > per_cu)
    return fail(c, PCMCC_EINVAL, "blocks_per_cu %d exceeds the %d blocks of %d that fit", s.blocks_per_cu, per_cu,
                block);
  const int bpc = s.blocks_per_cu ? s.blocks_per_cu : (small ? 1 : per_cu);
  *out = StepLaunch{block, bpc, refill, chunk, bpc * c->num_cu};
  return PCMCC_OK;
}

// Tuning cache: a flat JSON object {"key": [block, blocks_per_cu, refill,
// chunk], ...} (entries of two numbers leave refill and chunk at 0).
void load_tune_cache(pcmcc_ctx* c, const char* path) {
  if (!path) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t p = 0;
  while ((p = t.find('"', p)) != std::string::npos) {
    const size_t q = t.find('"', p + 1);
    if (q == std::string::npos) break;
    const std::string key = t.substr(p + 1, q - p - 1);
    int b = 0, k = 0, r = 0, ch = 0;
    const size_t lb = t.find('[', q);
    if (lb == std::string::npos) break;
    const int got = std::sscanf(t.c_str() + lb, "[%d , %d , %d , %d]", &b, &k, &r, &ch);
    if (got >= 2 && b > 0 && k > 0) c->tuned[key] = {b, k, got == 4 ? r : 0, got == 4 ? ch : 0};
    p = t.find(']', lb);
    if (p == std::string::npos) break;
  }
}

void save_tune_cache(pcmcc_ctx* c, const char* path) {
  if (!path) return;
  std::ofstream f(path);
  if (!f) return;
  f << "{\n";
  size_t i = 0;
  for (const auto& kv : c->tuned) {
    const auto& v = kv.second;
    f << "  \"" << kv.first << "\": [" << v[0] << ", " << v[1] << ", " << v[2] << ", " << v[3] << "]";
    f << (++i < c->tuned.size() ? ",\n" : "\n");
  }
  f << "}\n";
}

bool valid_grid(const pcmcc_grid* g) {
  return g && g->E && g->nx >= 1 && g->ny >= 1 && g->nz >= 1 && g->dx > 0 && std::isfinite(g->dx) &&
         std::isfinite(g->x0) && std::isfinite(g->y0) && std::isfinite(g->z0) &&
         (double)g->nx * g->ny * g->nz < 4.0e9;
}

TableView table_view(const pcmcc_ctx* c) {
  TableView T{};
  T.C = c->dC;
  T.P = c->dP;
  T.nu = c->dNu;
  T.n = c->n_e;
  T.nproc = c->n_proc;
  const double lnmin = std::log(c->eps_min);
  const double dlog = (std::log(c->eps_max) - lnmin) / (c->n_e - 1);
  T.u_scale = (float)(std::log(2.0) / dlog);
  T.u_offset = (float)(-lnmin / dlog);
  T.eps_top = (float)c->eps_max;
  for (int k = 0; k < kMaxProc; ++k) {
    T.thr[k] = c->thr[k];
    T.kind[k] = c->kind[k];
  }
  return T;
}

SpeciesView species_view(const pcmcc_ctx* c) {
  SpeciesView S{};
  S.qm = c->charge / c->mass;
  S.k_eps = (float)(0.5 * c->mass / kEV);
  S.inv_k = (float)(2.0 * kEV / c->mass);
  S.recoil = (float)(2.0 * c->mass / c->target_mass);
  S.k_eps_d = 0.5 * c->mass / kEV;
  S.inv_k_d = 2.0 * kEV / c->mass;
  return S;
}

int check_ready(pcmcc_ctx* c) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (!c->species_ok) return fail(c, PCMCC_ESTATE, "species not initialised");
  if (!c->tables_ok) return fail(c, PCMCC_ESTATE, "tables not initialised");
  return PCMCC_OK;
}

// Field bounds of the majorant (per cell and global) and the corner-packed
// field for `g`.
int prepare_field(pcmcc_ctx* c, const pcmcc_grid* g) {
  const size_t ncell = (size_t)g->nx * g->ny * g->nz;
  const size_t nrec = ((size_t)g->nx + 2) * ((size_t)g->ny + 2) * ((size_t)g->nz + 2);
  if (nrec >= ((size_t)1 << 31)) return fail(c, PCMCC_EINVAL, "grid too large: (nx+2)(ny+2)(nz+2) must be below 2^31");
  if (c->fbound_cells < ncell) {
    dfree(c->fbound);
    c->fbound = nullptr;
    c->fbound_cells = 0;
    HIP_TRY(c, dalloc(&c->fbound, ncell));
    c->fbound_cells = ncell;
  }
  if (c->fpack_recs < nrec) {
    dfree(c->fpack);
    c->fpack = nullptr;
    c->fpack_recs = 0;
    if (dalloc(&c->fpack, nrec * (kRecFloats / 4)) != hipSuccess) {
      (void)hipGetLastError();
      c->fpack = nullptr;
      return fail(c, PCMCC_ENOMEM, "cannot allocate the packed field (%zu bytes)", nrec * kRecFloats * sizeof(float));
    }
    c->fpack_recs = nrec;
  }
  HIP_TRY(c, hipMemsetAsync(c->emax_bits, 0, sizeof(unsigned), c->stream));
  HIP_TRY(c, launch_field_bounds((const float4*)g->E, g->nx, g->ny, g->nz, c->fbound, c->emax_bits, c->stream));
  HIP_TRY(c, launch_pack_field((const float4*)g->E, c->fbound, g->nx, g->ny, g->nz, c->fpack, c->stream));
  return PCMCC_OK;
}

// Charge deposit of n particles (n_dev holds the same count on the device):
// direct kernel for small n, binned schedule from kDepositBinnedMin on.
// Reads the deposit's range flag back (synchronises the stream).
int deposit_range_check(pcmcc_ctx* c) {
  HIP_TRY(c, hipMemcpyAsync(c->host_err, c->dep_err, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (*c->host_err)
    return fail(c, PCMCC_ERANGE, "charge outside the deposit's fixed-point range (a weight outside [0, 2^31) or "
                "more than 2^31 electrons in one cell)");
  return PCMCC_OK;
}

// Deposit of n particles into rho on the context stream; with check, waits
// and reports a range error (else the caller calls deposit_range_check).
// A step call of this many particles and steps or more starts from the
// population sorted by tile (a shorter call does not earn the sort back).
constexpr uint64_t kSortStartMin = 1u << 20;
constexpr int kSortStartSteps = 8;

// Binned-deposit buffers for d (the sorted copy only with `sorted`).
static int ensure_dep_work(pcmcc_ctx* c, const DepositNeeds& d, bool sorted) {
  auto grow = [&](auto** ptr, uint64_t& have, uint64_t need) -> int {
    if (have >= need) return PCMCC_OK;
    dfree(*ptr);
    *ptr = nullptr;
    have = 0;
    if (dalloc(ptr, need) != hipSuccess) {
      (void)hipGetLastError();
      *ptr = nullptr;
      return fail(c, PCMCC_ENOMEM, "cannot allocate deposit buffers");
    }
    have = need;
    return PCMCC_OK;
  };
  // tile_count and tile_start share one capacity (n_tiles + 1 entries each)
  int rc = PCMCC_OK;
  if (c->dep_tiles < d.n_tiles + 1) {
    uint64_t have = 0;
    rc = grow(&c->dep.tile_count, have, d.n_tiles + 1);
    have = 0;
    if (!rc) rc = grow(&c->dep.tile_start, have, d.n_tiles + 1);
    c->dep_tiles = rc ? 0 : d.n_tiles + 1;
    if (rc) return rc;
  }
  rc = grow(&c->dep.dump, c->dep_dump, d.dump_entries);
  if (!rc && sorted) rc = grow(&c->dep.sorted, c->dep_sorted, d.sorted);
  return rc;
}

int run_deposit(pcmcc_ctx* c, const float* x, const float* y, const float* z, const float* w, const int64_t* n_dev,
                uint64_t n, const pcmcc_grid* grid, int64_t* rho, bool check) {
  const DepositGeom g{grid->nx, grid->ny, grid->nz, grid->x0, grid->y0, grid->z0, 1.0 / grid->dx, c->dep_err};
  const DepositNeeds d = deposit_needs(g, n);
  HIP_TRY(c, hipMemsetAsync(c->dep_err, 0, sizeof(unsigned), c->stream));
  if (!d.binned) {
    HIP_TRY(c, launch_deposit(x, y, z, w, n_dev, g, rho, c->stream));
    return check ? deposit_range_check(c) : PCMCC_OK;
  }
  if (n >= 0xFFFFFFFFull) return fail(c, PCMCC_EINVAL, "deposit of 2^32 or more particles");
  const int rc = ensure_dep_work(c, d, true);
  if (rc) return rc;
  HIP_TRY(c, launch_deposit_binned(x, y, z, w, n, g, rho, c->dep, c->stream));
  return check ? deposit_range_check(c) : PCMCC_OK;
}

// Buffers of the weight update for n particles on `ncell` cells.
int ensure_weights(pcmcc_ctx* c, uint64_t n, size_t ncell) {
  if (c->wt_n < n) {
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
    c->wt = WeightWork{};
    c->wt_n = 0;
    // room for growth: the count rises between updates of a run
    n = n + n / 2;
    size_t tb = 0;
    HIP_TRY(c, weight_temp_bytes(n, &tb));
    if (dalloc(&c->wt.cls, n) != hipSuccess || dalloc(&c->wt.idx0, n) != hipSuccess ||
        dalloc(&c->wt.idx1, n) != hipSuccess || dalloc(&c->wt.key0, n) != hipSuccess ||
        dalloc(&c->wt.key1, n) != hipSuccess || dalloc(&c->wt.key2, n) != hipSuccess ||
        dalloc(&c->wt.pos, n) != hipSuccess ||
        dalloc(&c->wt.cnt, n) != hipSuccess || dalloc(&c->wt.counters, 4) != hipSuccess ||
        hipMalloc(&c->wt.temp, std::max<size_t>(tb, 16)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, PCMCC_ENOMEM, "cannot allocate weight-update buffers for %llu particles", (unsigned long long)n);
    }
    c->wt.temp_bytes = std::max<size_t>(tb, 16);
    c->wt_n = n;
  }
  if (c->wt_cells < ncell) {
    dfree(c->wt_rho);
    c->wt_rho = nullptr;
    c->wt_cells = 0;
    if (dalloc(&c->wt_rho, ncell) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, PCMCC_ENOMEM, "cannot allocate the weight-update density grid");
    }
    c->wt_cells = ncell;
  }
  if (!c->dev_n) HIP_TRY(c, dalloc(&c->dev_n, 1));
  return PCMCC_OK;
}

// Weight update of the n particles of `cur` into `out` (at most capacity):
// density of `cur` on the grid, then the update.  *n_new = the new count
// (nothing is written to `out` when it exceeds the capacity: ECAPACITY).
int weight_update(pcmcc_ctx* c, const Soa& cur, const Soa& out, uint64_t n, const pcmcc_grid* g, double n_ppc,
                  uint64_t seed, uint64_t update_index, uint64_t capacity, uint64_t* n_new, uint64_t* pairs,
                  uint64_t* splits) {
  *n_new = n;
  *pairs = *splits = 0;
  if (n == 0) return PCMCC_OK;
  const size_t ncell = (size_t)g->nx * g->ny * g->nz;
  int rc = ensure_weights(c, n, ncell);
  if (rc) return rc;
  HIP_TRY(c, hipMemsetAsync(c->wt_rho, 0, ncell * sizeof(int64_t), c->stream));
  const int64_t nn = (int64_t)n;
  HIP_TRY(c, hipMemcpyAsync(c->dev_n, &nn, sizeof(nn), hipMemcpyHostToDevice, c->stream));
  rc = run_deposit(c, cur.x, cur.y, cur.z, cur.w, c->dev_n, n, g, c->wt_rho);
  if (rc) return rc;
  WeightGeom wg{g->nx, g->ny, g->nz, g->x0, g->y0, g->z0, 1.0 / g->dx, n_ppc, 1, capacity};
  while (wg.cell_bits < 31 && ((uint64_t)1 << wg.cell_bits) < ncell) ++wg.cell_bits;
  HIP_TRY(c, launch_weight_update(cur, out, n, wg, c->wt_rho, Key{(uint32_t)seed, (uint32_t)(seed >> 32)},
                                  (uint32_t)update_index, c->wt, n_new, pairs, splits, c->stream));
  if (*n_new > capacity)
    return fail(c, PCMCC_ECAPACITY, "weight update needs %llu slots, capacity %llu", (unsigned long long)*n_new,
                (unsigned long long)capacity);
  return PCMCC_OK;
}

// The step loop; with ev, the ionization and attachment events of the
// committed steps are appended to its lists.
int push_impl(pcmcc_ctx* c, const pcmcc_particles* p, const pcmcc_grid* field, double dt, int n_steps,
              uint64_t seed, uint64_t step0, int64_t* rho, pcmcc_stats* stats, const EventSink* ev) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!p || !p->x || !p->y || !p->z || !p->vx || !p->vy || !p->vz || !p->w || !p->id || !p->n_dev)
    return fail(c, PCMCC_EINVAL, "null particle array");
  if (p->capacity < 1 || (uint64_t)p->capacity > 0xFFFFFFFFull)
    return fail(c, PCMCC_EINVAL, "capacity must be in [1, 2^32)");
  if (!valid_grid(field)) return fail(c, PCMCC_EINVAL, "invalid field grid");
  if (!(dt > 0) || !std::isfinite(dt) || n_steps < 0) return fail(c, PCMCC_EINVAL, "invalid dt or n_steps");
  if (step0 + (uint64_t)n_steps > 0xFFFFFFFFull) return fail(c, PCMCC_EINVAL, "step counter exceeds 32 bits");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(c->host_n, p->n_dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int64_t n0 = *c->host_n;
  if (n0 < 0 || n0 > p->capacity) return fail(c, PCMCC_EINVAL, "particle count %lld outside [0, capacity]", (long long)n0);
  rc = ensure_scratch(c, (uint64_t)p->capacity);
  if (rc) return rc;
  rc = prepare_field(c, field);
  if (rc) return rc;

  const TableView T = table_view(c);
  StepLaunch sl;
  rc = resolve_launch(c, c->sched, pic_lds_bytes_s, occupancy_pic_steps, T, 0, &sl, (uint64_t)std::max<int64_t>(n0, 1));
  if (rc) return rc;
  const int block = sl.block, grid = sl.grid;
  if (c->partial_blocks < grid) {
    dfree(c->partial);
    c->partial = nullptr;
    HIP_TRY(c, dalloc(&c->partial, (size_t)grid * NCNT));
    c->partial_blocks = grid;
  }
  std::memset(c->host_ctl, 0, sizeof(Ctl));
  c->host_ctl->n_cur = (unsigned long long)n0;
  // The steps alternate between the caller's arrays and the scratch buffer.
  // A large population over several steps starts sorted by 8^3-cell tile, so that the electrons
  // a wave takes from the work counter gather from a few field records that
  // stay in cache (the sort goes into the scratch buffer and, for an even
  // step count, is copied back).  For an odd step count the steps start from
  // the scratch buffer so that the last step lands in the caller's arrays:
  // copying the start population is cheaper than copying back the grown one
  // (any other outcome is copied back at the end as usual).
  const Soa user{p->x, p->y, p->z, p->vx, p->vy, p->vz, p->w, p->id};
  const bool sort_start = n0 >= (int64_t)kSortStartMin && n_steps >= kSortStartSteps;
  auto copy_soa = [&](const Soa& from, const Soa& to) -> hipError_t {
    float* const f[7] = {from.x, from.y, from.z, from.vx, from.vy, from.vz, from.w};
    float* const t[7] = {to.x, to.y, to.z, to.vx, to.vy, to.vz, to.w};
    hipError_t e = hipSuccess;
    for (int k = 0; k < 7 && e == hipSuccess; ++k)
      e = hipMemcpyAsync(t[k], f[k], (size_t)n0 * sizeof(float), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(to.id, from.id, (size_t)n0 * sizeof(uint64_t), hipMemcpyDeviceToDevice, c->stream);
    return e;
  };
  if (sort_start) {
    const DepositGeom g{field->nx, field->ny, field->nz, field->x0, field->y0, field->z0, 1.0 / field->dx,
                        c->dep_err};
    rc = ensure_dep_work(c, deposit_needs(g, (uint64_t)n0), false);
    if (rc) return rc;
    HIP_TRY(c, launch_sort_tiles(user, (uint64_t)n0, g, c->dep, c->scratch, c->stream));
    if (n_steps & 1)
      c->host_ctl->cur_sel = 1;
    else
      HIP_TRY(c, copy_soa(c->scratch, user));
  } else if ((n_steps & 1) && n0 > 0) {
    HIP_TRY(c, copy_soa(user, c->scratch));
    c->host_ctl->cur_sel = 1;
  }
  HIP_TRY(c, hipMemcpyAsync(c->ctl, c->host_ctl, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));

  PicArgs A{};
  A.buf[0] = Soa{p->x, p->y, p->z, p->vx, p->vy, p->vz, p->w, p->id};
  A.buf[1] = c->scratch;
  A.pend[0] = c->pend[0];
  A.pend[1] = c->pend[1];
  A.holes = c->holes;
  A.flags = c->flags;
  A.donor = c->donor;
  A.partial = c->partial;
  A.cap = (uint64_t)p->capacity;
  A.pend_cap = c->pend_cap;
  A.ctl = c->ctl;
  A.emax_bits = c->emax_bits;
  A.T = T;
  A.S = species_view(c);
  GridView& G = A.G;
  G.P = c->fpack;
  G.nx = field->nx;
  G.ny = field->ny;
  G.nz = field->nz;
  G.px = field->nx + 2;
  G.py = field->ny + 2;
  G.o[0] = field->x0;
  G.o[1] = field->y0;
  G.o[2] = field->z0;
  G.nd[0] = (double)field->nx;
  G.nd[1] = (double)field->ny;
  G.nd[2] = (double)field->nz;
  G.dx = (float)field->dx;
  G.inv_dx = 1.0 / field->dx;
  G.lo[0] = field->x0;
  G.lo[1] = field->y0;
  G.lo[2] = field->z0;
  G.hi[0] = field->x0 + field->nx * field->dx;
  G.hi[1] = field->y0 + field->ny * field->dx;
  G.hi[2] = field->z0 + field->nz * field->dx;
  G.qm_abs = (float)std::fabs(A.S.qm);
  G.qm = A.S.qm;
  A.key = Key{(uint32_t)seed, (uint32_t)(seed >> 32)};
  A.dt = (float)dt;
  A.chunk = (uint32_t)sl.chunk;
  if (ev) A.ev = *ev;
  // Step loop launches.  With weight control the kernel stops after the step
  // that takes the count above floor(growth * n_ref); the weights are then
  // updated (into the other particle buffer) and the loop resumes.
  const bool wctl = c->wc_n_ppc > 0;
  if (wctl && c->wc_n_ref <= 0) c->wc_n_ref = n0;
  uint64_t w_updates = 0, w_pairs = 0, w_splits = 0;
  double step_ms = 0, weight_ms = 0;
  int done = 0;
  rc = PCMCC_OK;
  while (done < n_steps) {
    A.step0 = (uint32_t)(step0 + (uint64_t)done);
    A.n_steps = n_steps - done;
    A.n_limit = wctl ? (uint64_t)std::floor(c->wc_growth * (double)c->wc_n_ref) : 0;
    HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
    HIP_TRY(c, launch_pic_steps(A, grid, block, sl.refill, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->host_ctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    step_ms += ms;
    Ctl& h = *c->host_ctl;
    done = (int)h.steps_done;
    if (h.status != kStatusWeightsDue) {
      rc = h.status;
      break;
    }
    const Soa cur = A.buf[h.cur_sel], other = A.buf[h.cur_sel ^ 1];
    uint64_t n_new = 0, pairs = 0, splits = 0;
    HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
    const int urc = weight_update(c, cur, other, h.n_cur, field, c->wc_n_ppc, seed, step0 + (uint64_t)done - 1,
                                  (uint64_t)p->capacity, &n_new, &pairs, &splits);
    HIP_TRY(c, hipEventRecord(c->ev[3], c->stream));
    h.status = PCMCC_OK;
    h.stop = 0;
    if (urc == PCMCC_OK) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
      weight_ms += ms;
      ++w_updates;
      w_pairs += pairs;
      w_splits += splits;
      c->wc_n_ref = (int64_t)n_new;
      h.cur_sel ^= 1;
      h.n_cur = n_new;
    }
    HIP_TRY(c, hipMemcpyAsync(c->ctl, c->host_ctl, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
    if (urc != PCMCC_OK) {
      rc = urc;
      break;
    }
  }
  HIP_TRY(c, launch_finalize(A.buf[0], A.buf[1], c->ctl, p->n_dev, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->host_ctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const Ctl& h = *c->host_ctl;
  if (rc == PCMCC_OK) rc = h.status;
  int drc = PCMCC_OK;
  if (rc == PCMCC_OK && rho) {
    HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
    drc = run_deposit(c, p->x, p->y, p->z, p->w, p->n_dev, h.n_cur, field, rho, false);
    if (drc) return drc;
    HIP_TRY(c, hipEventRecord(c->ev[3], c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
    if (stats) stats->deposit_kernel_ms = ms;
    drc = deposit_range_check(c);
  }
  if (stats) {
    stats->step_kernel_ms = step_ms;
    stats->launch_block = block;
    stats->launch_grid = grid;
    stats->launch_refill = sl.refill;
    stats->launch_chunk = sl.chunk;
    stats->n = (int64_t)h.n_cur;
    stats->steps_done = h.steps_done;
    stats->particle_steps = h.particle_steps;
    stats->trials = h.tot[C_TRIALS];
    stats->null_collisions = h.tot[C_NULL];
    for (int k = 0; k < 4; ++k) stats->real_collisions[k] = h.tot[C_EL + k];
    stats->lost = h.tot[C_LOST];
    stats->out_of_table = h.tot[C_OOT];
    stats->errors = h.tot[C_ERR];
    stats->majorant_violations = h.tot[C_MAJ];
    stats->weight_updates = (int64_t)w_updates;
    stats->merged_pairs = (int64_t)w_pairs;
    stats->splits = (int64_t)w_splits;
    stats->weight_ms = weight_ms;
  }
  if (rc == PCMCC_ECAPACITY)
    return fail(c, rc, "particle capacity %lld exceeded after %lld committed steps", (long long)p->capacity,
                (long long)h.steps_done);
  if (rc == PCMCC_ELIMIT) return fail(c, rc, "newborn generation limit reached after %lld steps", (long long)h.steps_done);
  return rc != PCMCC_OK ? rc : drc;
}

// The small reduction buffers.
int ensure_red(pcmcc_ctx* c) {
  if (!c->sc_red) {
    HIP_TRY(c, dalloc(&c->sc_red, 8));
    HIP_TRY(c, dalloc(&c->sel, 1));
    HIP_TRY(c, dalloc(&c->sel_hist, 1u << 12));
    HIP_TRY(c, hipHostMalloc((void**)&c->sc_host, 8 * sizeof(unsigned long long), hipHostMallocDefault));
  }
  return PCMCC_OK;
}

// Multigrid levels, field and density grids for g.
int ensure_sc(pcmcc_ctx* c, const pcmcc_grid* g) {
  const size_t ncell = (size_t)g->nx * g->ny * g->nz;
  int r = ensure_red(c);
  if (r) return r;
  if (c->mg_dims0.nx != g->nx || c->mg_dims0.ny != g->ny || c->mg_dims0.nz != g->nz) {
    MgDims d[kMgMaxLevels];
    const int L = mg_levels(g->nx, g->ny, g->nz, d);
    const MgDims dl = d[L - 1];
    if ((size_t)dl.nx * dl.ny * dl.nz > (size_t)kMgCoarseMax)
      return fail(c, PCMCC_EINVAL, "grid %dx%dx%d coarsens only to %dx%dx%d (> %d cells): use dimensions with more "
                  "factors of two", g->nx, g->ny, g->nz, dl.nx, dl.ny, dl.nz, kMgCoarseMax);
    size_t need = 0;  // u and f of every level
    for (int l = 0; l < L; ++l) need += 2 * (size_t)d[l].nx * d[l].ny * d[l].nz;
    if (c->mg_store_n < need) {
      dfree(c->mg_store);
      c->mg_store = nullptr;
      c->mg_store_n = 0;
      HIP_TRY(c, dalloc(&c->mg_store, need));
      c->mg_store_n = need;
    }
    if (c->mg_rhs_n < ncell) {
      dfree(c->mg_rhs);
      c->mg_rhs = nullptr;
      c->mg_rhs_n = 0;
      HIP_TRY(c, dalloc(&c->mg_rhs, ncell));
      c->mg_rhs_n = ncell;
    }
    const size_t nparts = defect_blocks(g->nx, g->ny, g->nz);
    if (c->mg_part_n < nparts) {
      dfree(c->mg_part);
      c->mg_part = nullptr;
      c->mg_part_n = 0;
      HIP_TRY(c, dalloc(&c->mg_part, nparts));
      c->mg_part_n = nparts;
    }
    c->mg = MgWork{};
    c->mg.levels = L;
    c->mg.rhs = c->mg_rhs;
    c->mg.part = c->mg_part;
    float* q = c->mg_store;
    for (int l = 0; l < L; ++l) {
      c->mg.dims[l] = d[l];
      const size_t n = (size_t)d[l].nx * d[l].ny * d[l].nz;
      c->mg.u[l] = q;
      c->mg.f[l] = q + n;
      q += 2 * n;
    }
    c->mg_dims0 = MgDims{g->nx, g->ny, g->nz};
  }
  c->mg.dx = g->dx;
  if (c->sc_cells < ncell) {
    dfree(c->sc_E);
    dfree(c->sc_ne);
    c->sc_E = nullptr;
    c->sc_ne = nullptr;
    c->sc_cells = 0;
    HIP_TRY(c, dalloc(&c->sc_E, ncell));
    HIP_TRY(c, dalloc(&c->sc_ne, ncell));
    c->sc_cells = ncell;
  }
  return PCMCC_OK;
}

int read_red(pcmcc_ctx* c, int first, int count) {
  HIP_TRY(c, hipMemcpyAsync(c->sc_host + first, c->sc_red + first, count * sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PCMCC_OK;
}


// phi (device, level-0 u) for the densities; cycles and relative residual out.
int solve_potential(pcmcc_ctx* c, const pcmcc_grid* g, const int64_t* np, const int64_t* ne, const int64_t* nn,
                    double* phi, double tol, int max_cycles, int* cycles, double* rel) {
  const size_t ncell = (size_t)g->nx * g->ny * g->nz;
  HIP_TRY(c, hipMemsetAsync(c->sc_red, 0, 2 * sizeof(unsigned long long), c->stream));
  const double scale = -(kQe * 0x1p-32 / (g->dx * g->dx * g->dx)) / kEps0;
  HIP_TRY(c, launch_sc_rhs(np, ne, nn, ncell, scale, c->mg.rhs, c->sc_red, c->stream));
  return mg_iterate(c, g, phi, tol, max_cycles, cycles, rel);
}

// Defect correction on phi for the right-hand side in mg.rhs (its largest
// magnitude in sc_red[0], set by the kernel that wrote it): the double
// defect, checked against tol, then one single-precision V-cycle for the
// correction, until the relative defect is at most tol or max_cycles cycles.
int mg_iterate(pcmcc_ctx* c, const pcmcc_grid* g, double* phi, double tol, int max_cycles, int* cycles,
               double* rel) {
  const size_t ncell = (size_t)g->nx * g->ny * g->nz;
  c->mg.phi = phi;
  int rc = read_red(c, 0, 1);
  if (rc) return rc;
  double fmax;
  std::memcpy(&fmax, &c->sc_host[0], sizeof(double));
  *cycles = 0;
  *rel = 0;
  if (fmax == 0) {  // no space charge: phi = 0
    HIP_TRY(c, hipMemsetAsync(phi, 0, ncell * sizeof(double), c->stream));
    return PCMCC_OK;
  }
  for (int it = 0;; ++it) {
    HIP_TRY(c, hipMemsetAsync(c->sc_red + 1, 0, sizeof(unsigned long long), c->stream));
    HIP_TRY(c, launch_defect(c->mg, c->sc_red + 1, c->stream));
    rc = read_red(c, 1, 1);
    if (rc) return rc;
    double rmax;
    std::memcpy(&rmax, &c->sc_host[1], sizeof(double));
    *cycles = it;
    *rel = rmax / fmax;
    if (*rel <= tol || it >= max_cycles) break;
    HIP_TRY(c, hipMemsetAsync(c->mg.u[0], 0, ncell * sizeof(float), c->stream));
    HIP_TRY(c, mg_vcycle(c->mg, 0, c->stream));
    HIP_TRY(c, launch_correct(c->mg, c->stream));
  }
  return PCMCC_OK;
}

double mobility(const pcmcc_sc_opts* o, double EN_Td, double gas_N) {
  if (o->mu_n == 1) return o->mu_N[0] / gas_N;
  const double lo = std::log(o->mu_EN_lo), hi = std::log(o->mu_EN_hi);
  double u = (std::log(std::max(EN_Td, 1e-300)) - lo) / (hi - lo) * (o->mu_n - 1);
  u = std::min(std::max(u, 0.0), o->mu_n - 1.0);
  const int i = std::min((int)std::floor(u), o->mu_n - 2);
  const double f = u - i;
  return ((1.0 - f) * o->mu_N[i] + f * o->mu_N[i + 1]) / gas_N;
}

// Photoionization from n_ev events (device arrays): counts the photons,
// checks the capacity, appends the photoelectrons at p's count and deposits
// their charge into n_pos (nullable).
int photoionize(pcmcc_ctx* c, const pcmcc_grid* g, const float* ex, const float* ey, const float* ez, const float* ew,
                uint64_t n_ev, const pcmcc_photo_opts* o, uint64_t seed, uint64_t step, const pcmcc_particles* p,
                int64_t* n_pos, int64_t* photons, int64_t* absorbed, double* ms) {
  *photons = 0;
  *absorbed = 0;
  *ms = 0;
  if (n_ev == 0) return PCMCC_OK;
  int rc = ensure_red(c);
  if (rc) return rc;
  PhotoArgs A{};
  A.ex = ex;
  A.ey = ey;
  A.ez = ez;
  A.ew = ew;
  A.n = n_ev;
  A.eta = o->eta;
  A.w_ph = o->w_photon;
  A.k1 = o->k1;
  A.k2 = o->k2;
  A.ln_k = std::log(o->k2 / o->k1);
  A.s_lo = std::log(1e-6 / o->k2);
  A.s_hi = std::log(60.0 / o->k1);
  A.key = Key{(uint32_t)seed ^ 0x50484F54u, (uint32_t)(seed >> 32) ^ (uint32_t)step};
  A.lo[0] = g->x0;
  A.lo[1] = g->y0;
  A.lo[2] = g->z0;
  A.hi[0] = g->x0 + g->nx * g->dx;
  A.hi[1] = g->y0 + g->ny * g->dx;
  A.hi[2] = g->z0 + g->nz * g->dx;
  A.x = p->x;
  A.y = p->y;
  A.z = p->z;
  A.vx = p->vx;
  A.vy = p->vy;
  A.vz = p->vz;
  A.w = p->w;
  A.id = p->id;
  A.n_dev = (unsigned long long*)p->n_dev;
  if (c->ph_n < n_ev) {
    dfree(c->ph_cnt);
    dfree(c->ph_off);
    c->ph_cnt = nullptr;
    c->ph_off = nullptr;
    c->ph_n = 0;
    HIP_TRY(c, dalloc(&c->ph_cnt, n_ev));
    HIP_TRY(c, dalloc(&c->ph_off, n_ev));
    c->ph_n = n_ev;
  }
  size_t tb = 0;
  HIP_TRY(c, photo_scan_bytes(n_ev, &tb));
  if (c->ph_temp_bytes < tb) {
    if (c->ph_temp) (void)hipFree(c->ph_temp);
    c->ph_temp = nullptr;
    c->ph_temp_bytes = 0;
    HIP_TRY(c, hipMalloc(&c->ph_temp, std::max<size_t>(tb, 16)));
    c->ph_temp_bytes = std::max<size_t>(tb, 16);
  }
  HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
  HIP_TRY(c, launch_photo_count(A, c->ph_cnt, c->ph_temp, c->ph_temp_bytes, c->ph_off, c->stream));
  uint64_t last_off = 0;  // offset and count of the last event: their sum is the total
  uint32_t last_cnt = 0;
  HIP_TRY(c, hipMemcpyAsync(&last_off, c->ph_off + (n_ev - 1), sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(&last_cnt, c->ph_cnt + (n_ev - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->host_n, p->n_dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const uint64_t total = last_off + last_cnt;
  const int64_t n_cur = *c->host_n;
  if (n_cur < 0 || n_cur > p->capacity) return fail(c, PCMCC_EINVAL, "particle count outside [0, capacity]");
  if (total > (uint64_t)(p->capacity - n_cur))
    return fail(c, PCMCC_ECAPACITY, "photoionization: %llu photons for %lld free slots", (unsigned long long)total,
                (long long)(p->capacity - n_cur));
  *photons = (int64_t)total;
  if (total == 0) return PCMCC_OK;
  A.offs = c->ph_off;
  A.total = total;
  HIP_TRY(c, launch_photo_emit(A, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->host_n, p->n_dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int64_t n_new = *c->host_n;
  *absorbed = n_new - n_cur;
  if (n_pos && *absorbed > 0) {
    c->sc_host[7] = (unsigned long long)*absorbed;
    HIP_TRY(c, hipMemcpyAsync(c->sc_red + 7, c->sc_host + 7, sizeof(unsigned long long), hipMemcpyHostToDevice,
                              c->stream));
    rc = run_deposit(c, p->x + n_cur, p->y + n_cur, p->z + n_cur, p->w + n_cur, (const int64_t*)(c->sc_red + 7),
                     (uint64_t)*absorbed, g, n_pos);
    if (rc) return rc;
  }
  HIP_TRY(c, hipEventRecord(c->ev[3], c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  float t = 0;
  HIP_TRY(c, hipEventElapsedTime(&t, c->ev[2], c->ev[3]));
  *ms = t;
  return PCMCC_OK;
}

bool valid_photo(const pcmcc_photo_opts* o) {
  return o && std::isfinite(o->eta) && o->eta >= 0 && std::isfinite(o->k1) && std::isfinite(o->k2) && o->k1 > 0 &&
         o->k2 > o->k1 && std::isfinite(o->w_photon);
}

// Start value of a sequence of solves in time: with two earlier solutions
// (n_sol >= 2) phi becomes phi + r (phi - prev), r = dt_next / dt_last, and
// prev the old phi; after the first solution prev is set to it.  The
// converged potential is the same to the solve's tolerance; the extrapolated
// start saves cycles.
int solve_start(pcmcc_ctx* c, double* phi, size_t ncell, int n_sol, double r) {
  if (n_sol < 1) return PCMCC_OK;
  if (c->phi_prev_n < ncell) {
    dfree(c->phi_prev);
    c->phi_prev = nullptr;
    c->phi_prev_n = 0;
    HIP_TRY(c, dalloc(&c->phi_prev, ncell));
    c->phi_prev_n = ncell;
  }
  if (n_sol == 1 || !(r > 0) || !std::isfinite(r)) {
    HIP_TRY(c, hipMemcpyAsync(c->phi_prev, phi, ncell * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return PCMCC_OK;
  }
  HIP_TRY(c, launch_extrapolate(phi, c->phi_prev, r, ncell, c->stream));
  return PCMCC_OK;
}

}  // namespace pcmcc_rt
