// C ABI and host runtime of the PIC-MCC electron library (see include/pcmcc.h).
//
// The runtime owns the device tables, the scratch buffers of the step loop
// (ping-pong particle buffer, newborn queues, hole lists, counters) and the
// per-cell field bounds; it validates arguments, sizes and launches the
// kernels on the context's stream and copies back the counters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "pcmcc.h"
#include "pcmcc_field.hpp"
#include "pcmcc_internal.hpp"
#include "pcmcc_photo.hpp"

using namespace pcmcc;

namespace {

constexpr double kEV = 1.602176634e-19;  // J per eV
constexpr size_t kMaxTableFloats = 16384;  // (n_proc + 1) n_e staged in LDS

std::string g_last_error;

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
};

}  // namespace

struct pcmcc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int num_cu = 0;
  // species
  bool species_ok = false;
  double mass = 0, charge = 0, gas_N = 0, target_mass = 0;
  // tables
  bool tables_ok = false;
  int n_e = 0, n_proc = 0;
  double eps_min = 0, eps_max = 0;
  int kind[kMaxProc] = {0};
  float thr[kMaxProc] = {0};
  float *dC = nullptr, *dP = nullptr, *dNu = nullptr;
  // scratch of the step loop
  uint64_t cap = 0, pend_cap = 0;
  Soa scratch{};
  PendSoa pend[2]{};
  uint32_t *holes = nullptr, *flags = nullptr, *donor = nullptr;
  unsigned long long* partial = nullptr;
  int partial_blocks = 0;
  Ctl* ctl = nullptr;
  Ctl* host_ctl = nullptr;  // pinned
  float2* fbound = nullptr;
  size_t fbound_cells = 0;
  float4* fpack = nullptr;  // corner-packed field records
  size_t fpack_recs = 0;
  DepositWork dep{};        // binned deposit buffers
  uint64_t dep_tiles = 0, dep_dump = 0, dep_sorted = 0;
  unsigned* emax_bits = nullptr;
  int64_t* host_n = nullptr;  // pinned
  unsigned* dep_err = nullptr;    // deposit range flag (device)
  unsigned* host_err = nullptr;   // pinned copy of it
  // super-particle weights: control settings, update buffers
  double wc_n_ppc = 0, wc_growth = 1.25;
  int64_t wc_n_ref = 0;
  WeightWork wt{};
  uint64_t wt_n = 0;
  int64_t* wt_rho = nullptr;
  size_t wt_cells = 0;
  int64_t* dev_n = nullptr;  // a device count for the deposit of the update
  // self-consistent field: multigrid levels (u[0] is the correction of the potential),
  // the field the electrons see, the electron density, event lists, and the
  // small reduction results
  MgWork mg{};
  float* mg_store = nullptr;  // single-precision correction levels
  size_t mg_store_n = 0;
  double* mg_rhs = nullptr;
  size_t mg_rhs_n = 0;
  double* mg_part = nullptr;  // per-block maxima of the defect pass
  size_t mg_part_n = 0;
  double* phi_prev = nullptr;  // the potential of the solve before the last (start-value extrapolation)
  size_t phi_prev_n = 0;
  uint32_t* ph_cnt = nullptr;  // photoionization: photon counts per event
  uint64_t* ph_off = nullptr;  // and their exclusive scan
  uint64_t ph_n = 0;
  void* ph_temp = nullptr;
  size_t ph_temp_bytes = 0;
  MgDims mg_dims0{0, 0, 0};
  float4* sc_E = nullptr;
  int64_t* sc_ne = nullptr;
  size_t sc_cells = 0;
  float* ev_store = nullptr;  // 8 lists of ev_cap floats
  uint64_t ev_cap = 0;
  unsigned long long* sc_red = nullptr;  // [0] max |f| bits [1] max |r| bits [2] ne max [3] first cell [4] sum w [5..6] events [7] photons
  unsigned long long* sc_host = nullptr;  // pinned copy
  SelState* sel = nullptr;
  unsigned* sel_hist = nullptr;
  // fluid step: predicted densities and first-stage derivatives (6 grids), table
  double* fl_store = nullptr;
  size_t fl_cells = 0;
  double* fl_tab = nullptr;
  int fl_tab_n = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // swarm batch scratch
  struct Swarm {
    uint64_t slots = 0, pend_cap = 0;
    int S = 0, J = 0, grid = 0;
    Soa buf[2]{};
    PendSoa pend[2]{};
    uint64_t *base = nullptr, *cap_s = nullptr;
    int32_t* n0 = nullptr;
    double *az = nullptr, *EN = nullptr;
    unsigned long long *n_cur = nullptr, *n_nxt = nullptr, *cum_ion = nullptr, *cum_att = nullptr;
    int* pc_k = nullptr;
    long long* L = nullptr;
    unsigned long long* mom = nullptr;
    long long* cnt = nullptr;
    unsigned long long *partial = nullptr, *partial_ps = nullptr;
    SwarmCtl* ctl = nullptr;
    double *values = nullptr, *errors = nullptr, *work = nullptr;
  } sw;
  std::map<std::string, std::pair<int, int>> tuned;  // shape key -> (block, blocks per CU)
};

namespace {

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

#define HIP_TRY(ctx, call)                                                                         \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return fail((ctx), e_ == hipErrorOutOfMemory ? PCMCC_ENOMEM : PCMCC_EHIP, "%s: %s (%s:%d)", #call, \
                  hipGetErrorString(e_), __FILE__, __LINE__);                                      \
  } while (0)

template <class T>
hipError_t dalloc(T** p, size_t n) {
  return hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T));
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

// Tuning cache: a flat JSON object {"key": [block, blocks_per_cu], ...}.
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
    int b = 0, k = 0;
    const size_t lb = t.find('[', q);
    if (lb == std::string::npos) break;
    if (std::sscanf(t.c_str() + lb, "[%d , %d]", &b, &k) == 2 && b > 0 && k > 0) c->tuned[key] = {b, k};
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
    f << "  \"" << kv.first << "\": [" << kv.second.first << ", " << kv.second.second << "]";
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
int run_deposit(pcmcc_ctx* c, const float* x, const float* y, const float* z, const float* w, const int64_t* n_dev,
                uint64_t n, const pcmcc_grid* grid, int64_t* rho, bool check = true) {
  const DepositGeom g{grid->nx, grid->ny, grid->nz, grid->x0, grid->y0, grid->z0, 1.0 / grid->dx, c->dep_err};
  const DepositNeeds d = deposit_needs(g, n);
  HIP_TRY(c, hipMemsetAsync(c->dep_err, 0, sizeof(unsigned), c->stream));
  if (!d.binned) {
    HIP_TRY(c, launch_deposit(x, y, z, w, n_dev, g, rho, c->stream));
    return check ? deposit_range_check(c) : PCMCC_OK;
  }
  if (n >= 0xFFFFFFFFull) return fail(c, PCMCC_EINVAL, "deposit of 2^32 or more particles");
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
  if (!rc) rc = grow(&c->dep.sorted, c->dep_sorted, d.sorted);
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

}  // namespace

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

// The step loop; with ev, the ionization and attachment events of the
// committed steps are appended to its lists.
static int push_impl(pcmcc_ctx* c, const pcmcc_particles* p, const pcmcc_grid* field, double dt, int n_steps,
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

  const int block = 256;
  const TableView T = table_view(c);
  const size_t lds = pic_lds_bytes(T, block);
  int per_cu = 0;
  HIP_TRY(c, occupancy_pic_steps(block, lds, &per_cu));
  if (per_cu < 1) return fail(c, PCMCC_EHIP, "step kernel does not fit on a compute unit");
  const int grid = per_cu * c->num_cu;
  if (c->partial_blocks < grid) {
    dfree(c->partial);
    c->partial = nullptr;
    HIP_TRY(c, dalloc(&c->partial, (size_t)grid * NCNT));
    c->partial_blocks = grid;
  }
  std::memset(c->host_ctl, 0, sizeof(Ctl));
  c->host_ctl->n_cur = (unsigned long long)n0;
  // The steps alternate between the caller's arrays and the scratch buffer.
  // For an odd step count, start from a copy in the scratch buffer so that
  // the last step lands in the caller's arrays: copying the start population
  // is cheaper than copying back the grown one (any other outcome is copied
  // back at the end as usual).
  if ((n_steps & 1) && n0 > 0) {
    float* const from[7] = {p->x, p->y, p->z, p->vx, p->vy, p->vz, p->w};
    float* const to[7] = {c->scratch.x, c->scratch.y, c->scratch.z, c->scratch.vx, c->scratch.vy, c->scratch.vz,
                          c->scratch.w};
    for (int k = 0; k < 7; ++k)
      HIP_TRY(c, hipMemcpyAsync(to[k], from[k], (size_t)n0 * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->scratch.id, p->id, (size_t)n0 * sizeof(uint64_t), hipMemcpyDeviceToDevice,
                              c->stream));
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
    HIP_TRY(c, launch_pic_steps(A, grid, block, c->stream));
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

int pcmcc_push_collide_deposit(pcmcc_ctx* c, const pcmcc_particles* p, const pcmcc_grid* field, double dt,
                               int n_steps, uint64_t seed, uint64_t step0, int64_t* rho, pcmcc_stats* stats) {
  return push_impl(c, p, field, dt, n_steps, seed, step0, rho, stats, nullptr);
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

namespace {

// One run of the swarm step loop with a given launch shape (inputs already
// on the device); the kernel time in ms goes to *ms.
int swarm_run(pcmcc_ctx* c, SwarmArgs& A, int S, const std::vector<uint64_t>& n0h, int block, int grid,
              float* ms) {
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
  HIP_TRY(c, launch_swarm_steps(A, grid, block, c->stream));
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
  // Launch shape: explicit, tuned (cached), or the default block of 256.
  const int blocks[4] = {64, 128, 256, 512};
  char keybuf[160];
  std::snprintf(keybuf, sizeof(keybuf), "gfx950:k_swarm_steps:S%d:N%llu:cap%d:se%d:ne%d:np%d", S,
                (unsigned long long)(slots / opts->cap_factor), opts->cap_factor, opts->sample_every, c->n_e,
                c->n_proc);
  const std::string key(keybuf);
  load_tune_cache(c, opts->tune_cache);
  int block = opts->block, bpc = opts->blocks_per_cu;
  auto occ = [&](int b) {
    int k = 0;
    if (occupancy_swarm_steps(b, swarm_lds_bytes(T, S, b), &k) != hipSuccess) return 0;
    return k;
  };
  if (block == 0 && !opts->autotune && c->tuned.count(key)) {
    block = c->tuned[key].first;
    bpc = c->tuned[key].second;
  }
  if (block == 0) block = 256;
  if (block != 64 && block != 128 && block != 256 && block != 512)
    return fail(c, PCMCC_EINVAL, "block must be 64, 128, 256 or 512");
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
    // Time each candidate shape on the first min(n_steps, 200) steps.
    SwarmArgs probe = A;
    probe.n_steps = std::min(n_steps, 200);
    float best = 1e30f;
    int best_b = 256, best_k = 1;
    for (int b : blocks) {
      const int kmax = std::min(occ(b), 32);
      for (int k = 1; k <= kmax; k *= 2) {
        float t = 0;
        rc = swarm_run(c, probe, S, n0h, b, k * c->num_cu, &t);
        if (rc) return rc;
        if (t < best) {
          best = t;
          best_b = b;
          best_k = k;
        }
      }
    }
    block = best_b;
    bpc = best_k;
    c->tuned[key] = {block, bpc};
    save_tune_cache(c, opts->tune_cache);
  }
  const int kmax = std::min(occ(block), 32);
  if (kmax < 1) return fail(c, PCMCC_EHIP, "swarm kernel does not fit on a compute unit");
  if (bpc <= 0 || bpc > kmax) bpc = kmax;
  const int grid = bpc * c->num_cu;
  A.n_steps = n_steps;
  rc = swarm_run(c, A, S, n0h, block, grid, &ms);
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
  }
  if (hc.status == PCMCC_ECAPACITY)
    return fail(c, hc.status, "a swarm outgrew its %d x n0 slots after %lld steps", opts->cap_factor,
                (long long)hc.steps_done);
  if (hc.status != PCMCC_OK) return fail(c, hc.status, "swarm step loop stopped (status %d)", hc.status);
  return PCMCC_OK;
}


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
  if (!params || !norm || n_held < 1 || !EN_held || !ln_held || !mask_held || !(tol_ln > 0) || !(z_sig >= 0) ||
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
  for (int k = 0; k < n_cells; ++k) fallback_out[k] = 0;
  const double w = (cell_hi - cell_lo) / n_cells;
  for (int i = 0; i < n_held; ++i) {
    const int cell = std::min(std::max((int)std::floor((std::log(EN_held[i]) - cell_lo) / w), 0), n_cells - 1);
    for (int k = 0; k < PCMCC_MLP_OUT; ++k) {
      const size_t j = (size_t)i * PCMCC_MLP_OUT + k;
      float err = NAN;
      if (mask_held[j] == 0.0f) {
        fallback_out[cell] = 1;
      } else {
        err = std::fabs(y[(size_t)k * n_held + i] - ln_held[j]);
        const double sig = sig_held ? (double)sig_held[j] : 0.0;
        if (!(err <= tol_ln + z_sig * (std::isfinite(sig) ? sig : 0.0))) fallback_out[cell] = 1;
      }
      if (err_out) err_out[j] = err;
    }
  }
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


// ---------------------------------------------------------------------------
// Self-consistent step (Sec. 2.5, Sec. 2.3, Sec. 2.1.4).

namespace {

constexpr double kEps0 = 8.8541878128e-12;
constexpr double kQe = 1.602176634e-19;

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

int mg_iterate(pcmcc_ctx* c, const pcmcc_grid* g, double* phi, double tol, int max_cycles, int* cycles,
               double* rel);

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

}  // namespace

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


// ---------------------------------------------------------------------------
// Fluid step (Sec. 2.2).

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
