// Device-side declarations of the self-consistent field (multigrid, field
// from the potential, time-step ingredients) and of the fluid step.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pcmcc {

// Row-stencil launches: a one-dimensional grid of xb * ny * nz blocks, xb
// blocks of kRowThreads threads along each row of n_x threads.  Consecutive
// workgroups go to the eight XCDs in turn (block b to XCD b % 8); the remap
// gives each XCD one contiguous run of rows, so the neighbouring rows and
// planes a stencil reads were mostly fetched into that XCD's L2 by its own
// blocks.
constexpr int kRowThreads = 128;
struct RowPos {
  int x0, j, k;  // first thread's x, the row's y and z
};
// Logical index of this block: XCD b % 8 takes the b / 8-th block of its run.
__device__ __forceinline__ unsigned xcd_block() {
  const unsigned G = gridDim.x, b = blockIdx.x;
  const unsigned q = G >> 3, r = G & 7u, x = b & 7u;
  return x * q + (x < r ? x : r) + (b >> 3);
}
// Position of logical row block L (xb = ceil(n_x / kRowThreads) per row).
__device__ __forceinline__ RowPos row_at(unsigned L, int n_x, int ny) {
  const unsigned xb = (unsigned)((n_x + kRowThreads - 1) / kRowThreads);
  const unsigned row = L / xb;
  return RowPos{(int)(L - row * xb) * kRowThreads, (int)(row % (unsigned)ny), (int)(row / (unsigned)ny)};
}
__device__ __forceinline__ RowPos row_pos(int n_x, int ny) { return row_at(xcd_block(), n_x, ny); }
inline dim3 row_grid(int n_x, int ny, int nz) {
  return dim3((unsigned)((size_t)((n_x + kRowThreads - 1) / kRowThreads) * (size_t)ny * (size_t)nz));
}
// The defect pass: kDefectRows consecutive row blocks per block.
constexpr unsigned kDefectRows = 8;
inline unsigned defect_blocks(int nx, int ny, int nz) { return (row_grid(nx, ny, nz).x + kDefectRows - 1) / kDefectRows; }

// Self-consistent field: multigrid levels and the time-step selection state.
constexpr int kMgMaxLevels = 16;
constexpr int kMgCoarseMax = 4096;  // cells of the coarsest level (solved in LDS)
struct MgDims {
  int nx, ny, nz;
};
struct MgWork {
  int levels;
  MgDims dims[kMgMaxLevels];
  float* u[kMgMaxLevels];  // correction cycle: u[0] the correction of the potential
  float* f[kMgMaxLevels];  // f[0]: the defect of the potential
  double* rhs;             // right-hand side of the potential
  double* phi;             // the potential
  double dx;               // finest spacing
  double* part;            // per-block maxima of the defect pass (defect_blocks of the finest level)
};
struct SelState {
  uint32_t prefix;
  uint32_t pad;
  uint64_t rank;  // wanted rank (1-based) within the prefix
};
int mg_levels(int nx, int ny, int nz, MgDims* dims);
hipError_t launch_sc_rhs(const int64_t* np, const int64_t* ne, const int64_t* nn, size_t n, double scale, double* f,
                         unsigned long long* fmax, hipStream_t s);
hipError_t mg_vcycle(const MgWork& W, int l, hipStream_t s);
hipError_t launch_defect(const MgWork& W, unsigned long long* rmax, hipStream_t s);
hipError_t launch_correct(const MgWork& W, hipStream_t s);
hipError_t launch_extrapolate(double* phi, double* prev, double r, size_t n, hipStream_t s);
hipError_t launch_sc_field(const float4* Ea, const double* phi, int nx, int ny, int nz, double dx, float4* E,
                           hipStream_t s);
hipError_t launch_speed_select(const float* vx, const float* vy, const float* vz, const int64_t* n_dev, uint64_t n,
                               SelState* st, unsigned* hist, hipStream_t s);
hipError_t launch_densest(const int64_t* ne, size_t n, long long* mx, unsigned long long* first, hipStream_t s);
hipError_t launch_weight_sum(const float* w, const int64_t* n_dev, uint64_t n, double* out, hipStream_t s);

// Fluid step: local-field tables on the device and the stage arguments.
constexpr double kFlQe = 1.602176634e-19;
constexpr double kFlEps0 = 8.8541878128e-12;
struct FluidTab {
  int n;
  double ln_lo, ln_span;  // ln of the first E/N node (Td), ln(last / first)
  const double *muN, *DN, *aN, *eN;
  double gas_N;
  // precomputed so that the kernels multiply instead of dividing
  double pos_scale;  // (n - 1) / ln_span: table position per unit of ln(E/N)
  double inv_gas_N;  // 1 / N
  double ln_td;      // ln(1e21 / N): ln(E/N in Td) = ln|E| + ln_td
};
struct FluidArgs {
  int nx, ny, nz;
  double dx, dt;
  const float4* E;
  double *ne, *np, *nn;     // densities (m^-3), updated in place by stage 2
  double *se, *sp, *sn;     // predicted densities
  double *k1e, *k1p, *k1n;  // first-stage derivatives
  FluidTab T;
};
hipError_t launch_fluid_stage(const FluidArgs& A, int stage, hipStream_t s);
hipError_t launch_fluid_rhs(const double* np, const double* ne, const double* nn, size_t n, double* f,
                            unsigned long long* fmax_bits, hipStream_t s);
hipError_t launch_fluid_dt(const double* ne, const float4* E, size_t n, const FluidTab& T, double dx,
                           unsigned long long* out, hipStream_t s);

}  // namespace pcmcc
