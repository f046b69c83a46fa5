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
#include <string>
#include <vector>

#include "pcmcc.h"
#include "pcmcc_internal.hpp"

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
  unsigned* emax_bits = nullptr;
  int64_t* host_n = nullptr;  // pinned
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
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

// Field bounds of the majorant (per cell and global) for `g`.
int field_bounds(pcmcc_ctx* c, const pcmcc_grid* g) {
  const size_t ncell = (size_t)g->nx * g->ny * g->nz;
  if (c->fbound_cells < ncell) {
    dfree(c->fbound);
    c->fbound = nullptr;
    HIP_TRY(c, dalloc(&c->fbound, ncell));
    c->fbound_cells = ncell;
  }
  HIP_TRY(c, hipMemsetAsync(c->emax_bits, 0, sizeof(unsigned), c->stream));
  HIP_TRY(c, launch_field_bounds((const float4*)g->E, g->nx, g->ny, g->nz, c->fbound, c->emax_bits, c->stream));
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
      hipHostMalloc((void**)&c->host_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->host_n, sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
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
  dfree(c->dC);
  dfree(c->dP);
  dfree(c->dNu);
  dfree(c->partial);
  dfree(c->ctl);
  dfree(c->fbound);
  dfree(c->emax_bits);
  if (c->host_ctl) (void)hipHostFree(c->host_ctl);
  if (c->host_n) (void)hipHostFree(c->host_n);
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
  rc = field_bounds(c, field);
  if (rc) return rc;

  const int block = 256;
  const TableView T = table_view(c);
  const size_t lds = table_lds_bytes(T);
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
  G.E = (const float4*)field->E;
  G.bound = c->fbound;
  G.nx = field->nx;
  G.ny = field->ny;
  G.nz = field->nz;
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
  A.key = Key{(uint32_t)seed, (uint32_t)(seed >> 32)};
  A.step0 = (uint32_t)step0;
  A.n_steps = n_steps;
  A.dt = (float)dt;
  HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
  if (n_steps > 0) HIP_TRY(c, launch_pic_steps(A, grid, block, c->stream));
  HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
  HIP_TRY(c, launch_finalize(A.buf[0], A.buf[1], c->ctl, p->n_dev, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->host_ctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const Ctl& h = *c->host_ctl;
  rc = h.status;
  if (rc == PCMCC_OK && rho) {
    DepositGeom g{field->nx, field->ny, field->nz, field->x0, field->y0, field->z0, 1.0 / field->dx};
    HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
    HIP_TRY(c, launch_deposit(p->x, p->y, p->z, p->w, p->n_dev, g, rho, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev[3], c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
    if (stats) stats->deposit_kernel_ms = ms;
  }
  if (stats) {
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    stats->step_kernel_ms = ms;
    stats->n = (int64_t)h.n_cur;
    stats->steps_done = h.steps_done;
    stats->particle_steps = h.particle_steps;
    stats->trials = h.tot[C_TRIALS];
    stats->null_collisions = h.tot[C_NULL];
    for (int k = 0; k < 4; ++k) stats->real_collisions[k] = h.tot[C_EL + k];
    stats->lost = h.tot[C_LOST];
    stats->out_of_table = h.tot[C_OOT];
    stats->errors = h.tot[C_ERR];
  }
  if (rc == PCMCC_ECAPACITY)
    return fail(c, rc, "particle capacity %lld exceeded after %lld committed steps", (long long)p->capacity,
                (long long)h.steps_done);
  if (rc == PCMCC_ELIMIT) return fail(c, rc, "newborn generation limit reached after %lld steps", (long long)h.steps_done);
  return rc;
}

int pcmcc_deposit(pcmcc_ctx* c, const float* x, const float* y, const float* z, const float* w,
                  const int64_t* n_dev, const pcmcc_grid* grid, int64_t* rho) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (!x || !y || !z || !w || !n_dev || !rho) return fail(c, PCMCC_EINVAL, "null array");
  if (!grid || grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || !(grid->dx > 0))
    return fail(c, PCMCC_EINVAL, "invalid grid");
  HIP_TRY(c, hipSetDevice(c->device));
  DepositGeom g{grid->nx, grid->ny, grid->nz, grid->x0, grid->y0, grid->z0, 1.0 / grid->dx};
  HIP_TRY(c, launch_deposit(x, y, z, w, n_dev, g, rho, c->stream));
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
