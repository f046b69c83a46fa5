// Internal types shared by the kernels and the host runtime of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pcmcc.h"
#include "pcmcc_device.hpp"

namespace pcmcc {

struct PState {
  float x, y, z, vx, vy, vz, w;
  uint64_t id;
  double xd, yd, zd;  // end position before rounding (domain test)
};

// Particle arrays (structure of arrays).
struct Soa {
  float *x, *y, *z, *vx, *vy, *vz, *w;
  uint64_t* id;
};

// Newborn queue: particle arrays plus the birth time within the step.
struct PendSoa {
  float *x, *y, *z, *vx, *vy, *vz, *w, *tb;
  uint64_t* id;
  uint32_t* sw;  // swarm index (swarm queues only, else null)
};

// Per-step event counters.
// C_MAJ: candidate collisions at an energy whose total rate exceeds the
// majorant the flight segment was drawn with (the null-collision method
// needs nu_hat >= nu_tot; any count means the bound is wrong).
enum CntIdx { C_TRIALS, C_NULL, C_EL, C_EXC, C_ION, C_ATT, C_LOST, C_OOT, C_ERR, C_MAJ, NCNT };

enum Overflow : unsigned { OVF_CAPACITY = 1u, OVF_LIMIT = 2u };

// Event lists of the self-consistent step (ix == nullptr: not recorded):
// where each ionization left a positive ion (the newborn's position) and each
// attachment a negative ion (the electron's position), with the weight.
struct EventSink {
  float *ix = nullptr, *iy = nullptr, *iz = nullptr, *iw = nullptr;
  float *ax = nullptr, *ay = nullptr, *az = nullptr, *aw = nullptr;
  unsigned long long* n = nullptr;  // [2]: ionizations, attachments
  uint64_t cap = 0;                 // entries per list
  unsigned* overflow = nullptr;
};

// Internal status of the step loop: stopped after a step because the count
// exceeds the weight-control limit (not an error; the host updates the
// weights and resumes).
constexpr int kStatusWeightsDue = 1;

// Device control block of a step loop.
struct Ctl {
  unsigned long long n_cur;   // live particles in the current buffer
  unsigned long long holes;   // removed particles of this step (slots in the next buffer)
  unsigned long long child;   // newborn survivors placed so far
  unsigned long long donors;  // tail donors found (hole filling)
  unsigned long long fill;    // holes filled from the tail
  unsigned long long pend[kMaxGenerations + 1];  // newborns queued per generation
  unsigned long long take[kMaxGenerations + 1];  // work counters: current buffer, then each generation
  unsigned overflow;          // Overflow bits of the running step
  int cur_sel;                // 0: the caller's arrays are current, 1: the scratch buffer
  int stop;
  int status;
  long long steps_done;
  unsigned long long particle_steps;
  unsigned long long tot[NCNT];
};

// Schedule choices of the mover (chosen per workload by the launch-shape
// tuner): refill thresholds the step kernels are built for, and the range
// of the work-counter chunk.
constexpr int kRefillChoices[3] = {16, 24, 32};
constexpr uint32_t kChunkMin = 64, kChunkMax = 4096;

struct PicArgs {
  Soa buf[2];
  PendSoa pend[2];
  uint32_t* holes;
  uint32_t* flags;
  uint32_t* donor;
  unsigned long long* partial;  // [grid][NCNT]
  uint64_t cap, pend_cap;
  Ctl* ctl;
  const unsigned* emax_bits;  // max |E| over the cells, as float bits
  TableView T;
  SpeciesView S;
  GridView G;
  Key key;
  uint32_t step0;
  int n_steps;
  float dt;
  uint64_t n_limit;  // stop after a step that leaves more particles (0: no limit)
  uint32_t chunk;    // electrons per work-counter grab (power of two, 64..4096)
  EventSink ev;
};

struct DepositGeom {
  int nx, ny, nz;
  double x0, y0, z0, inv_dx;
  unsigned* range_err;  // set to 1 on a weight outside [0, 2^31) or an int64 cell overflow
};

// Binned deposit: used from this many particles on (below, the direct
// kernel), and the device buffers it needs.
constexpr uint64_t kDepositBinnedMin = 1u << 18;
struct DepositNeeds {
  bool binned;
  uint64_t n_tiles, dump_entries, sorted;
};
struct DepositWork {
  uint32_t* tile_count;  // [n_tiles]
  uint32_t* tile_start;  // [n_tiles + 1]
  uint2* dump;           // [dump_entries]
  float4* sorted;        // [n]
};

struct TableBuild {
  int n, nproc;
  double lnmin, dlog, ev, mass, gas_N;
  int rates, effective;
  int kind[kMaxProc];
  const double* sigma;  // device [nproc][n]
  double* total;        // device scratch [n]
};

// Super-particle weight update: geometry and parameters, and device buffers.
struct WeightGeom {
  int nx, ny, nz;
  double x0, y0, z0, inv_dx;
  double n_ppc;
  int cell_bits;      // bits of the largest cell index
  uint64_t capacity;  // slots of the output buffer
};
struct WeightWork {
  uint8_t* cls;                 // [n] class per particle
  uint32_t *idx0, *idx1;        // [n] candidate indices (sort ping-pong)
  uint64_t *key0, *key1;        // [n] sort keys
  uint64_t* key2;               // [n] candidates' (cell, energy) keys by slot
  uint32_t *pos, *cnt;          // [n] output counts and positions
  unsigned long long* counters;  // [4] candidates, merged pairs
  void* temp;
  size_t temp_bytes;
};
hipError_t weight_temp_bytes(uint64_t n, size_t* bytes);
hipError_t launch_weight_update(const Soa& cur, const Soa& out, uint64_t n, const WeightGeom& g, const int64_t* rho,
                                Key key, uint32_t update_index, const WeightWork& W, uint64_t* n_out,
                                uint64_t* pairs_out, uint64_t* splits_out, hipStream_t stream);

// Swarm moments per sample and the coefficients derived from them.
constexpr int kNMom = 14;
// Fixed-point exponents of the moment sums: each particle adds
// round(value * 2^e) with |value * 2^e| < 2^54, summed in 128 bits.
constexpr int kMomExpHost[kNMom] = {0, 53, 53, 53, 53, 53, 25, 25, 25, 24, 24, 36, 0, 0};
enum Quantity {
  Q_W_FLUX, Q_W_BULK, Q_DL_FLUX, Q_DL_BULK, Q_DT_FLUX, Q_DT_BULK, Q_NU_ION,
  Q_NU_ATT, Q_NU_EFF, Q_MEAN_EPS, Q_MU, Q_ALPHA, Q_ETA, Q_RATIO, kNQ
};

// Device control block of the swarm step loop.
struct SwarmCtl {
  unsigned long long pend[kMaxGenerations + 1];
  unsigned long long take[kMaxGenerations + 1];  // work counters: current buffers, then each generation
  unsigned overflow;
  int cur_sel;
  int stop;
  int status;
  long long steps_done;
  unsigned long long particle_steps;
  unsigned long long tot[NCNT];
};

struct SwarmArgs {
  Soa buf[2];
  PendSoa pend[2];
  uint64_t pend_cap;
  int n_swarms;
  const uint64_t* base;         // [S] first slot of swarm s
  const uint64_t* cap_s;        // [S] slots of swarm s
  const int32_t* n0;            // [S]
  const double* az;             // [S] acceleration along z
  SwarmCtl* ctl;
  unsigned long long* n_cur;    // [S]
  unsigned long long* n_nxt;    // [S]
  int* pc_k;                    // [S] population control for the next load
  long long* L;                 // [S] log2 of the weight scale
  unsigned long long* cum_ion;  // [S]
  unsigned long long* cum_att;  // [S]
  unsigned long long* mom;      // [S][J][kNMom][2] 128-bit sums (lo, hi)
  long long* cnt_out;           // [S][J][4]: count, L, ionizations, attachments
  unsigned long long* partial;  // [grid][NCNT]
  unsigned long long* partial_ps;  // [grid]
  TableView T;
  SpeciesView S;
  Key key;
  int n_steps;
  float dt;
  int sample_every;
  int n_samples;
  int pop_control;
  uint32_t chunk;  // electrons per work-counter grab (power of two, 64..4096)
  EventSink ev;    // no event lists (the newborn queues' event view)
};

// Coefficient surrogate (1 -> 64 -> 64 -> 6 perceptron).
constexpr int kMlpParams = 4678;

struct MlpArgs {
  float* params;        // [kMlpParams], updated in place by training
  const float* x;       // [n] standardised inputs
  const float* t;       // [n][6] standardised targets
  const float* mask;    // [n][6] 1 = use the entry
  int64_t n;
  float inv_cnt;        // 1 / number of used entries
  float* partial;       // [grid][kMlpParams]
  float* ploss;         // [grid]
  float* m;             // Adam first moments
  float* v;             // Adam second moments
  float* loss_hist;     // [epochs] or null
  int epochs;
  double lr0, lr_min;
  float beta1, beta2, eps;
};

struct InferArgs {
  const float* params;  // [kMlpParams] (device)
  const float* EN;      // [n] reduced fields in Td
  float* out;           // [6][n] ln coefficients
  int64_t n;
  float mu_x, inv_sd_x;
  float mu_y[6], sd_y[6];
  int n_cells;          // fallback cells in ln(E/N), 0 = none
  float cell_lo, inv_cell_w;
  const uint8_t* fb_mask;
  int n_nodes;          // fallback table nodes, uniform in ln(E/N)
  float tab_lo, inv_tab_w;
  const float* table;   // [n_nodes][6] ln coefficients
};

size_t mlp_lds_bytes();
hipError_t launch_mlp_grad(const MlpArgs& a, int grid, hipStream_t stream);
hipError_t launch_mlp_reduce(const float* partial, const float* ploss, int nb, float* grad, float* loss,
                             hipStream_t stream);
hipError_t occupancy_mlp_train(int* blocks_per_cu);
hipError_t launch_mlp_train(const MlpArgs& a, int grid, hipStream_t stream);
hipError_t launch_mlp_infer(const InferArgs& a, int grid, hipStream_t stream);

size_t table_lds_bytes(const TableView& T);
size_t pic_lds_bytes(const TableView& T, int block);  // step kernel: tables and per-wave staging lists
size_t swarm_lds_bytes(const TableView& T, int S, int block);
// Blocks of kernel k (block threads, lds dynamic LDS bytes) that are
// resident on a compute unit together: the occupancy query, bounded by the
// LDS of a compute unit (160 KiB) over the block's static plus dynamic LDS
// rounded up to 1280 bytes.  The bound matters for cooperative launches,
// whose grid-wide barriers need every block resident: the query's own
// rounding can admit one block more than fit when a block's LDS comes
// within a granule of a 1/k share of the compute unit.
hipError_t coresident_blocks(const void* k, int block, size_t lds, int* blocks_per_cu);
// refill: one of kRefillChoices (free lanes that trigger a refill batch)
// row: floats per table node (table_row(nproc)), which selects the kernel build
hipError_t occupancy_swarm_steps(int block, int refill, int row, size_t lds, int* blocks_per_cu);
hipError_t launch_swarm_steps(const SwarmArgs& args, int grid, int block, int refill, hipStream_t stream);
hipError_t launch_swarm_init(const Soa& buf, const uint64_t* base, const int32_t* n0, int S, hipStream_t stream);
hipError_t launch_swarm_estimate(const unsigned long long* mom, const long long* cnt, int S, int J, double dt_sample,
                                 double t_window, int n_batches, const double* EN, double gas_N, double* values,
                                 double* errors, double* work, hipStream_t stream);
hipError_t launch_pic_steps(const PicArgs& args, int grid, int block, int refill, hipStream_t stream);
hipError_t occupancy_pic_steps(int block, int refill, int row, size_t lds, int* blocks_per_cu);
hipError_t launch_finalize(const Soa& user, const Soa& scratch, Ctl* ctl, int64_t* n_dev, hipStream_t stream);
DepositNeeds deposit_needs(const DepositGeom& g, uint64_t n);
hipError_t launch_deposit_binned(const float* x, const float* y, const float* z, const float* w, uint64_t n,
                                 const DepositGeom& g, int64_t* rho, const DepositWork& W, hipStream_t stream);
hipError_t launch_deposit(const float* x, const float* y, const float* z, const float* w, const int64_t* n_dev,
                          const DepositGeom& g, int64_t* rho, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t stream);
// Sorts n particles of src into dst by deposit tile (8^3 cells, clamped to
// the grid); needs W's tile counts, starts and dump as the binned deposit.
hipError_t launch_sort_tiles(const Soa& src, uint64_t n, const DepositGeom& g, const DepositWork& W, const Soa& dst,
                             hipStream_t stream);
hipError_t launch_field_bounds(const float4* E, int nx, int ny, int nz, float2* out, unsigned* emax_bits,
                               hipStream_t stream);
hipError_t launch_pack_field(const float4* E, const float2* bound, int nx, int ny, int nz, float4* P,
                             hipStream_t stream);
hipError_t launch_build_tables(const TableBuild& B, float* C, float* P, float* nu, hipStream_t stream);
hipError_t launch_philox(const uint32_t* ctr, Key key, uint32_t* out, int64_t n, hipStream_t stream);
hipError_t launch_lookup(const TableView& T, const SpeciesView& S, const float* eps, float* cum, const float* s_ub,
                         float* maj, int64_t n, hipStream_t stream);

}  // namespace pcmcc
