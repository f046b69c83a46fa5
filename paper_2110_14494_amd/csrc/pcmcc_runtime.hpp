// Host runtime of the PIC-MCC electron library shared by the C-ABI entry
// points (include/pcmcc.h): the context, which owns the device tables and
// every scratch buffer, and the helpers that validate arguments, size the
// scratch and launch the kernels on the context's stream.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
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
  // launch schedules: the step kernel's (zero fields: defaults), and the
  // tuned ones by workload key: (block, blocks per CU, refill, chunk)
  pcmcc_schedule sched{};
  std::map<std::string, std::array<int, 4>> tuned;
};

namespace pcmcc_rt {

constexpr double kEV = 1.602176634e-19;  // J per eV
constexpr size_t kMaxTableFloats = 16384;  // (n_proc + 1) n_e staged in LDS
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kQe = 1.602176634e-19;

extern std::string g_last_error;  // text of the last failure without a context

// Records the error text on the context (or globally) and returns code.
int fail(pcmcc_ctx* ctx, int code, const char* fmt, ...);

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

void dfree(void* p);

void free_scratch(pcmcc_ctx* c);
int ensure_scratch(pcmcc_ctx* c, uint64_t cap);
void free_soa(Soa& b);
void free_pend(PendSoa& q);
void free_swarm(pcmcc_ctx* c);
int alloc_soa(pcmcc_ctx* c, Soa& b, uint64_t n);
int alloc_pend(pcmcc_ctx* c, PendSoa& q, uint64_t n, bool with_sw);
int ensure_swarm(pcmcc_ctx* c, int S, uint64_t slots, int J, int grid);
// A schedule resolved against the kernel's resources: every field set.
struct StepLaunch {
  int block, bpc, refill, chunk, grid;
};
int check_schedule(pcmcc_ctx* c, const pcmcc_schedule& s);
inline size_t pic_lds_bytes_s(const TableView& T, int, int block) { return pic_lds_bytes(T, block); }
inline size_t swarm_lds_bytes_s(const TableView& T, int S, int block) { return swarm_lds_bytes(T, S, block); }
// lds(block): dynamic LDS bytes of the kernel at that block size; occ(block,
// refill, lds, &per_cu) its occupancy query.
// n_hint (0: none) is the start population of a step call: below
// kSmallPopulation electrons the unset fields default to one 64-thread block
// per CU and chunks of 64, since grid barriers over fewer, smaller blocks
// cost less and a small population fills few waves anyway.
constexpr uint64_t kSmallPopulation = 1u << 17;
int resolve_launch(pcmcc_ctx* c, const pcmcc_schedule& s, size_t (*lds)(const TableView&, int, int),
                   hipError_t (*occ)(int, int, int, size_t, int*), const TableView& T, int S, StepLaunch* out,
                   uint64_t n_hint = 0);
void load_tune_cache(pcmcc_ctx* c, const char* path);
void save_tune_cache(pcmcc_ctx* c, const char* path);
bool valid_grid(const pcmcc_grid* g);
TableView table_view(const pcmcc_ctx* c);
SpeciesView species_view(const pcmcc_ctx* c);
int check_ready(pcmcc_ctx* c);
int prepare_field(pcmcc_ctx* c, const pcmcc_grid* g);
int deposit_range_check(pcmcc_ctx* c);
int run_deposit(pcmcc_ctx* c, const float* x, const float* y, const float* z, const float* w, const int64_t* n_dev,
                uint64_t n, const pcmcc_grid* grid, int64_t* rho, bool check = true);
int ensure_weights(pcmcc_ctx* c, uint64_t n, size_t ncell);
int weight_update(pcmcc_ctx* c, const Soa& cur, const Soa& out, uint64_t n, const pcmcc_grid* g, double n_ppc,
                  uint64_t seed, uint64_t update_index, uint64_t capacity, uint64_t* n_new, uint64_t* pairs,
                  uint64_t* splits);
// The step loop; with ev, the ionization and attachment events of the
// committed steps are appended to its lists.
int push_impl(pcmcc_ctx* c, const pcmcc_particles* p, const pcmcc_grid* field, double dt, int n_steps,
              uint64_t seed, uint64_t step0, int64_t* rho, pcmcc_stats* stats, const EventSink* ev);
int ensure_red(pcmcc_ctx* c);
int ensure_sc(pcmcc_ctx* c, const pcmcc_grid* g);
int read_red(pcmcc_ctx* c, int first, int count);
// Defect correction of phi for the right-hand side in mg.rhs; cycles and
// relative residual out.
int mg_iterate(pcmcc_ctx* c, const pcmcc_grid* g, double* phi, double tol, int max_cycles, int* cycles,
               double* rel);
// phi (device, level-0 u) for the densities; cycles and relative residual out.
int solve_potential(pcmcc_ctx* c, const pcmcc_grid* g, const int64_t* np, const int64_t* ne, const int64_t* nn,
                    double* phi, double tol, int max_cycles, int* cycles, double* rel);
double mobility(const pcmcc_sc_opts* o, double EN_Td, double gas_N);
int photoionize(pcmcc_ctx* c, const pcmcc_grid* g, const float* ex, const float* ey, const float* ez, const float* ew,
                uint64_t n_ev, const pcmcc_photo_opts* o, uint64_t seed, uint64_t step, const pcmcc_particles* p,
                int64_t* n_pos, int64_t* photons, int64_t* absorbed, double* ms);
bool valid_photo(const pcmcc_photo_opts* o);
int solve_start(pcmcc_ctx* c, double* phi, size_t ncell, int n_sol, double r);
// Looks up this device's allocation-free deposit scratch (once per device;
// the device must be current).
void noalloc_setup(int device);

}  // namespace pcmcc_rt

using namespace pcmcc_rt;
