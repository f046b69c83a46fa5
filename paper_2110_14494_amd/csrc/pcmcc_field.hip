// Self-consistent field of the particle step (arXiv:2110.14494: Sec. 2.5
// Poisson's equation and E = -grad phi, Sec. 2.3 boundary conditions,
// Sec. 2.1.4 time step).
//
// * Space charge rho = e (n_+ - n_e - n_-) from the three int64 fixed-point
//   density grids (2^-32 electrons per unit), lap phi = -rho / eps0.
// * phi = 0 on the two z faces (Dirichlet), zero normal derivative on the x
//   and y faces (homogeneous Neumann): 7-point stencil on cell centres with
//   ghost cells (Dirichlet ghost = -phi of the boundary cell, Neumann ghost =
//   phi).  The caller's field is the applied field; the field the electrons
//   see is E_applied - grad phi (central differences, same ghosts).
// * Geometric multigrid as defect correction: the defect of the potential is
//   computed in double precision, the correction solved by one V(2,2) cycle in
//   single precision (red-black Gauss-Seidel smoothing, restriction by the
//   mean of the 8 children, trilinear prolongation with the error's ghost
//   rules, every dimension halved while all are even and above 2, the levels
//   of at most 4096 cells run by one block in LDS) and added to the potential; the
//   iteration converges to the double-precision solution of the discrete
//   system while the cycles move half the bytes.  All passes are
//   HBM-streaming stencils.
// * Time-step ingredients: the 90 % speed quantile by a three-pass radix
//   selection on |v|^2 keys (exact), the densest cell (largest fixed-point
//   density, first in x-fastest order), and the sum of the weights.
#include <hip/hip_runtime.h>

#include <climits>

#include "pcmcc_field.hpp"
#include "pcmcc_internal.hpp"

namespace pcmcc {

namespace {

__device__ __forceinline__ size_t idx3(int i, int j, int k, int nx, int ny) {
  return ((size_t)k * ny + j) * nx + i;
}

// Non-negative doubles compare like their bit patterns.
__device__ __forceinline__ void atomic_max_pos(unsigned long long* a, double v) {
  atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ double wave_max(double v) {
  for (int d = 32; d > 0; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
  return v;
}

// Largest non-negative value of the block into *a (one atomic per block).
__device__ __forceinline__ void block_max_to(unsigned long long* a, double v) {
  __shared__ double s_w[16];
  v = wave_max(v);
  const int wid = threadIdx.x / 64, nw = (blockDim.x + 63) / 64;
  if ((threadIdx.x & 63) == 0) s_w[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < nw; ++w) m = fmax(m, s_w[w]);
    if (m > 0.0) atomic_max_pos(a, m);
  }
}

// Sum of the neighbours present and the diagonal of the stencil at (i,j,k):
// a missing x/y neighbour is a Neumann ghost (diagonal 6 -> one less), a
// missing z neighbour a Dirichlet ghost (one more).  The six loads are issued
// together (a missing neighbour reads the cell itself and is then replaced by
// zero) and summed in the order -x, +x, -y, +y, -z, +z.
template <class T>
__device__ __forceinline__ T nb_sum(const T* u, int i, int j, int k, int nx, int ny, int nz, T& diag) {
  const size_t c = idx3(i, j, k, nx, ny);
  const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
  const bool xm = i > 0, xp = i < nx - 1, ym = j > 0, yp = j < ny - 1, zm = k > 0, zp = k < nz - 1;
  const T a = u[xm ? c - 1 : c], b = u[xp ? c + 1 : c];
  const T e = u[ym ? c - sy : c], f = u[yp ? c + sy : c];
  const T g = u[zm ? c - sz : c], h = u[zp ? c + sz : c];
  T s = 0;
  s += xm ? a : T(0);
  s += xp ? b : T(0);
  s += ym ? e : T(0);
  s += yp ? f : T(0);
  s += zm ? g : T(0);
  s += zp ? h : T(0);
  diag = (T)(6 - (int)!xm - (int)!xp - (int)!ym - (int)!yp + (int)!zm + (int)!zp);
  return s;
}

// Storage of a level's u and f: natural (x fastest), or split by colour
// (the finest launched level): the red cells ((i + j + k) even) fill the
// first half and the black cells the second, each in natural order at index
// c / 2 (c the natural index; nx even, so every pair 2m, 2m + 1 of a row
// holds one cell of each colour).  A half sweep then streams the other
// colour and its own right-hand side: half the bytes of the natural layout.
template <bool kSplit>
struct Lay {
  size_t half;
  __device__ __forceinline__ size_t at(size_t c, int parity) const {
    return kSplit ? (parity ? half : 0) + (c >> 1) : c;
  }
};

// nb_sum in layout L (the neighbours have the opposite parity).
template <bool kSplit, class T>
__device__ __forceinline__ T nb_sum_l(const T* u, Lay<kSplit> L, int i, int j, int k, int nx, int ny, int nz,
                                      T& diag) {
  const size_t c = idx3(i, j, k, nx, ny);
  const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
  const int q = 1 - ((i + j + k) & 1);
  const bool xm = i > 0, xp = i < nx - 1, ym = j > 0, yp = j < ny - 1, zm = k > 0, zp = k < nz - 1;
  const T a = u[L.at(xm ? c - 1 : c, q)], b = u[L.at(xp ? c + 1 : c, q)];
  const T e = u[L.at(ym ? c - sy : c, q)], f = u[L.at(yp ? c + sy : c, q)];
  const T g = u[L.at(zm ? c - sz : c, q)], h = u[L.at(zp ? c + sz : c, q)];
  T s = 0;
  s += xm ? a : T(0);
  s += xp ? b : T(0);
  s += ym ? e : T(0);
  s += yp ? f : T(0);
  s += zm ? g : T(0);
  s += zp ? h : T(0);
  diag = (T)(6 - (int)!xm - (int)!xp - (int)!ym - (int)!yp + (int)!zm + (int)!zp);
  return s;
}

}  // namespace

// Right-hand side of the finest level and its largest magnitude.
__global__ void k_sc_rhs(const int64_t* __restrict__ np, const int64_t* __restrict__ ne,
                         const int64_t* __restrict__ nn, size_t n, double scale, double* __restrict__ f,
                         unsigned long long* fmax_bits) {
#pragma clang fp contract(off)
  double m = 0.0;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) {
    const double v = (((double)np[c] - (double)ne[c]) - (double)nn[c]) * scale;
    f[c] = v;
    m = fmax(m, fabs(v));
  }
  block_max_to(fmax_bits, m);
}

// The level kernels are row stencils (row_pos: XCD-local runs of rows).

// One red-black Gauss-Seidel half sweep: cells with (i + j + k) % 2 == color.
template <bool kSplit>
__global__ __launch_bounds__(kRowThreads) void k_mg_smooth(float* __restrict__ u, const float* __restrict__ f,
                                                           int nx, int ny, int nz, float h2, int color) {
#pragma clang fp contract(off)
  const Lay<kSplit> L{(size_t)nx * ny * nz / 2};
  const RowPos P = row_pos((nx + 1) / 2, ny);
  const int j = P.j, k = P.k;
  const int i = 2 * (P.x0 + (int)threadIdx.x) + ((j + k + color) & 1);
  if (i >= nx) return;
  float d;
  const float s = nb_sum_l(u, L, i, j, k, nx, ny, nz, d);
  const size_t c = L.at(idx3(i, j, k, nx, ny), color);
  u[c] = (s - h2 * f[c]) / d;
}

// Residual r = f - L u of the 8 children of every coarse cell, averaged into
// the coarse right-hand side.  The restriction follows the pre-smoothing,
// whose last half sweep relaxed the black cells ((i + j + k) odd): their
// residual is zero up to rounding, so only the four red children are summed
// (child offsets 000, 110, 101, 011).
template <bool kSplit>
__global__ __launch_bounds__(kRowThreads) void k_mg_restrict(const float* __restrict__ u,
                                                             const float* __restrict__ f, int nx, int ny, int nz,
                                                             float inv_h2, float* __restrict__ fc) {
#pragma clang fp contract(off)
  const Lay<kSplit> L{(size_t)nx * ny * nz / 2};
  const int cx = nx / 2, cy = ny / 2;
  const RowPos P = row_pos(cx, cy);
  const int I = P.x0 + (int)threadIdx.x, J = P.j, K = P.k;
  if (I < cx) {
    float acc = 0.0f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (((q ^ (q >> 1) ^ (q >> 2)) & 1) != 0) continue;
      const int i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = 2 * K + (q >> 2);
      float d;
      const float s = nb_sum_l(u, L, i, j, k, nx, ny, nz, d);
      const size_t c = L.at(idx3(i, j, k, nx, ny), 0);  // red
      acc += f[c] - (s - d * u[c]) * inv_h2;
    }
    fc[idx3(I, J, K, cx, cy)] = 0.125f * acc;
  }
}

// Coarse value with the error's ghost rule outside the grid.
__device__ __forceinline__ float coarse_at(const float* U, int I, int J, int K, int cx, int cy, int cz) {
  float sgn = 1.0f;
  I = min(max(I, 0), cx - 1);
  J = min(max(J, 0), cy - 1);
  if (K < 0) {
    K = 0;
    sgn = -1.0f;
  } else if (K >= cz) {
    K = cz - 1;
    sgn = -1.0f;
  }
  return sgn * U[idx3(I, J, K, cx, cy)];
}

// u_fine += trilinear interpolation of the coarse correction.  A thread
// takes four consecutive fine cells of a row, 4t .. 4t + 3: they read the
// coarse columns 2t - 1 .. 2t + 2 of the same four coarse rows, sixteen loads
// instead of eight per cell.
template <bool kSplit>
__global__ __launch_bounds__(kRowThreads) void k_mg_prolong(float* __restrict__ u, const float* __restrict__ U,
                                                            int nx, int ny, int nz) {
#pragma clang fp contract(off)
  const Lay<kSplit> L{(size_t)nx * ny * nz / 2};
  const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
  const RowPos P = row_pos((nx + 3) / 4, ny);
  const int t = P.x0 + (int)threadIdx.x, j = P.j, k = P.k;
  if (4 * t >= nx) return;
  const int J = j >> 1, K = k >> 1;
  const int J2 = J + ((j & 1) ? 1 : -1), K2 = K + ((k & 1) ? 1 : -1);
  float a[4][4];  // [coarse column 2t - 1 + x][(J, K), (J2, K), (J, K2), (J2, K2)]
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int I = 2 * t - 1 + x;
    a[x][0] = coarse_at(U, I, J, K, cx, cy, cz);
    a[x][1] = coarse_at(U, I, J2, K, cx, cy, cz);
    a[x][2] = coarse_at(U, I, J, K2, cx, cy, cz);
    a[x][3] = coarse_at(U, I, J2, K2, cx, cy, cz);
  }
  const size_t c0 = idx3(4 * t, j, k, nx, ny);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (4 * t + e >= nx) break;
    const int xi = (e >> 1) + 1, xi2 = (e & 1) ? xi + 1 : xi - 1;  // columns of I and I2
    const float v = 27.0f * a[xi][0] + 9.0f * (a[xi2][0] + a[xi][1] + a[xi][2]) +
                    3.0f * (a[xi2][1] + a[xi2][2] + a[xi][3]) + a[xi2][3];
    u[L.at(c0 + e, (4 * t + e + j + k) & 1)] += v * (1.0f / 64.0f);
  }
}

// The levels of a V(2,2) cycle from the first one of at most kMgCoarseMax
// cells down to the coarsest, run by one block with every level in LDS (the
// same arithmetic as the level kernels; one launch instead of about eleven
// per level).  The coarsest level takes `coarse_iters` red-black sweeps.
constexpr int kMgTailCells = 4696;  // >= kMgCoarseMax * (1 + 1/8 + 1/64 + ...)
struct MgTailArgs {
  float* u;        // the first tail level's correction (global; starts at zero)
  const float* f;  // its right-hand side (global)
  int first, levels, coarse_iters;
  MgDims d[kMgMaxLevels];
  float h2[kMgMaxLevels];
  float inv_h2[kMgMaxLevels];
};

__device__ void tail_smooth(float* u, const float* f, MgDims d, float h2, int color) {
#pragma clang fp contract(off)
  const int n = d.nx * d.ny * d.nz;
  if ((d.nx & 1) == 0) {  // threads visit the cells of the colour only
    const int hx = d.nx >> 1;
    for (int q = threadIdx.x; q < (n >> 1); q += blockDim.x) {
      const int row = q / hx, j = row % d.ny, k = row / d.ny;
      const int i = 2 * (q - row * hx) + ((j + k + color) & 1);
      const int c = (k * d.ny + j) * d.nx + i;
      float dg;
      const float s = nb_sum(u, i, j, k, d.nx, d.ny, d.nz, dg);
      u[c] = (s - h2 * f[c]) / dg;
    }
  } else {
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
      const int i = c % d.nx, j = (c / d.nx) % d.ny, k = c / (d.nx * d.ny);
      if (((i + j + k) & 1) != color) continue;
      float dg;
      const float s = nb_sum(u, i, j, k, d.nx, d.ny, d.nz, dg);
      u[c] = (s - h2 * f[c]) / dg;
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(512) void k_mg_tail(MgTailArgs A) {
#pragma clang fp contract(off)
  __shared__ float s_u[kMgTailCells];
  __shared__ float s_f[kMgTailCells];
  __shared__ int off[kMgMaxLevels];  // level offsets in s_u / s_f
  if (threadIdx.x == 0) {
    int o = 0;
    for (int l = A.first; l < A.levels; ++l) {
      off[l] = o;
      o += A.d[l].nx * A.d[l].ny * A.d[l].nz;
    }
  }
  const MgDims d0 = A.d[A.first];
  const int n0 = d0.nx * d0.ny * d0.nz;
  for (int c = threadIdx.x; c < n0; c += blockDim.x) {
    s_u[c] = 0.0f;
    s_f[c] = A.f[c];
  }
  __syncthreads();
  for (int l = A.first; l < A.levels - 1; ++l) {  // down: pre-smoothing, restriction
    const MgDims d = A.d[l], dc = A.d[l + 1];
    float *u = s_u + off[l], *uc = s_u + off[l + 1], *fc = s_f + off[l + 1];
    const float* f = s_f + off[l];
    for (int it = 0; it < 2; ++it)
      for (int color = 0; color < 2; ++color) tail_smooth(u, f, d, A.h2[l], color);
    const int nc = dc.nx * dc.ny * dc.nz;
    for (int C = threadIdx.x; C < nc; C += blockDim.x) {
      const int I = C % dc.nx, J = (C / dc.nx) % dc.ny, K = C / (dc.nx * dc.ny);
      float acc = 0.0f;
      for (int q = 0; q < 8; ++q) {  // red children only, as in k_mg_restrict
        if (((q ^ (q >> 1) ^ (q >> 2)) & 1) != 0) continue;
        const int i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = 2 * K + (q >> 2);
        float dg;
        const float s = nb_sum(u, i, j, k, d.nx, d.ny, d.nz, dg);
        const size_t c = idx3(i, j, k, d.nx, d.ny);
        acc += f[c] - (s - dg * u[c]) * A.inv_h2[l];
      }
      fc[C] = 0.125f * acc;
      uc[C] = 0.0f;
    }
    __syncthreads();
  }
  {
    const int l = A.levels - 1;
    for (int it = 0; it < A.coarse_iters; ++it)
      for (int color = 0; color < 2; ++color) tail_smooth(s_u + off[l], s_f + off[l], A.d[l], A.h2[l], color);
  }
  for (int l = A.levels - 2; l >= A.first; --l) {  // up: prolongation, post-smoothing
    const MgDims d = A.d[l], dc = A.d[l + 1];
    float* u = s_u + off[l];
    const float* U = s_u + off[l + 1];
    const int n = d.nx * d.ny * d.nz;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
      const int i = c % d.nx, j = (c / d.nx) % d.ny, k = c / (d.nx * d.ny);
      const int I = i >> 1, J = j >> 1, K = k >> 1;
      const int I2 = I + ((i & 1) ? 1 : -1), J2 = J + ((j & 1) ? 1 : -1), K2 = K + ((k & 1) ? 1 : -1);
      const float v = 27.0f * coarse_at(U, I, J, K, dc.nx, dc.ny, dc.nz) +
                      9.0f * (coarse_at(U, I2, J, K, dc.nx, dc.ny, dc.nz) + coarse_at(U, I, J2, K, dc.nx, dc.ny, dc.nz) +
                              coarse_at(U, I, J, K2, dc.nx, dc.ny, dc.nz)) +
                      3.0f * (coarse_at(U, I2, J2, K, dc.nx, dc.ny, dc.nz) +
                              coarse_at(U, I2, J, K2, dc.nx, dc.ny, dc.nz) +
                              coarse_at(U, I, J2, K2, dc.nx, dc.ny, dc.nz)) +
                      coarse_at(U, I2, J2, K2, dc.nx, dc.ny, dc.nz);
      u[c] += v * (1.0f / 64.0f);
    }
    __syncthreads();
    for (int it = 0; it < 2; ++it)
      for (int color = 0; color < 2; ++color) tail_smooth(u, s_f + off[l], d, A.h2[l], color);
  }
  for (int c = threadIdx.x; c < n0; c += blockDim.x) A.u[c] = s_u[c];
}

// Defect of the potential, r = rhs - L phi in double precision: stored in
// single precision as the right-hand side of the correction cycle; a block
// takes kDefectRows consecutive row blocks and its largest magnitude goes to
// part[block] (k_max_parts reduces them:
// one same-address atomic per block would serialise in the memory-side
// atomic unit).
template <bool kSplit>
__global__ __launch_bounds__(kRowThreads) void k_mg_defect(const double* __restrict__ phi,
                                                           const double* __restrict__ rhs, int nx, int ny, int nz,
                                                           double inv_h2, float* __restrict__ r,
                                                           double* __restrict__ part) {
#pragma clang fp contract(off)
  const Lay<kSplit> lay{(size_t)nx * ny * nz / 2};
  __shared__ double s_w[kRowThreads / 64];
  const unsigned nrb = (unsigned)((nx + kRowThreads - 1) / kRowThreads) * (unsigned)ny * (unsigned)nz;
  const unsigned L0 = xcd_block() * kDefectRows;
  double m = 0.0;
  for (unsigned L = L0; L < L0 + kDefectRows && L < nrb; ++L) {
    const RowPos P = row_at(L, nx, ny);
    const int i = P.x0 + (int)threadIdx.x, j = P.j, k = P.k;
    if (i < nx) {
      const size_t c = idx3(i, j, k, nx, ny);
      double d;
      const double s = nb_sum(phi, i, j, k, nx, ny, nz, d);
      const double v = rhs[c] - (s - d * phi[c]) * inv_h2;
      r[lay.at(c, (i + j + k) & 1)] = (float)v;
      m = fmax(m, fabs(v));
    }
  }
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kRowThreads / 64; ++w) m = fmax(m, s_w[w]);
    part[blockIdx.x] = m;
  }
}

// Largest of n non-negative partial maxima, stored as its bit pattern.
__global__ __launch_bounds__(1024) void k_max_parts(const double* __restrict__ part, unsigned n,
                                                    unsigned long long* out) {
  __shared__ double s_w[16];
  double m = 0.0;
  for (unsigned q = threadIdx.x; q < n; q += blockDim.x) m = fmax(m, part[q]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)blockDim.x / 64; ++w) m = fmax(m, s_w[w]);
    *out = (unsigned long long)__double_as_longlong(m);
  }
}

// phi += the correction (a row kernel: the split layout needs the parity).
template <bool kSplit>
__global__ __launch_bounds__(kRowThreads) void k_mg_correct(double* __restrict__ phi, const float* __restrict__ e,
                                                            int nx, int ny, int nz) {
  const Lay<kSplit> L{(size_t)nx * ny * nz / 2};
  const RowPos P = row_pos(nx, ny);
  const int i = P.x0 + (int)threadIdx.x;
  if (i < nx) {
    const size_t c = idx3(i, P.j, P.k, nx, ny);
    phi[c] += (double)e[L.at(c, (i + P.j + P.k) & 1)];
  }
}



// Start value of the next solve from the last two solutions: phi <- phi +
// r (phi - prev) (linear in time, r the ratio of the coming to the last time
// step), prev <- the old phi.
__global__ void k_extrapolate(double* __restrict__ phi, double* __restrict__ prev, double r, size_t n) {
#pragma clang fp contract(off)
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) {
    const double t = phi[c];
    phi[c] = t + r * (t - prev[c]);
    prev[c] = t;
  }
}

// E = E_applied - grad phi at the centres (central differences with ghosts).
__global__ __launch_bounds__(kRowThreads) void k_sc_field(const float4* __restrict__ Ea, const double* __restrict__ phi,
                                                  int nx, int ny, int nz, double two_dx, float4* __restrict__ E) {
#pragma clang fp contract(off)
  const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
  const RowPos P = row_pos(nx, ny);
  const int i = P.x0 + (int)threadIdx.x, j = P.j, k = P.k;
  if (i < nx) {
    const size_t c = idx3(i, j, k, nx, ny);
    const double p = phi[c];
    const double xm = i > 0 ? phi[c - 1] : p, xp = i < nx - 1 ? phi[c + 1] : p;
    const double ym = j > 0 ? phi[c - sy] : p, yp = j < ny - 1 ? phi[c + sy] : p;
    const double zm = k > 0 ? phi[c - sz] : -p, zp = k < nz - 1 ? phi[c + sz] : -p;
    const float4 a = Ea[c];
    E[c] = make_float4((float)((double)a.x - (xp - xm) / two_dx), (float)((double)a.y - (yp - ym) / two_dx),
                       (float)((double)a.z - (zp - zm) / two_dx), 0.0f);
  }
}

// ---------------------------------------------------------------------------
// Time-step ingredients.

__device__ __forceinline__ uint32_t speed_key(float vx, float vy, float vz) {
#pragma clang fp contract(off)
  const double a = (double)vx, b = (double)vy, c = (double)vz;
  return __float_as_uint((float)((a * a + b * b) + c * c));
}

// Radix-selection pass: histogram of the key bits [shift, shift + bits) of
// the particles whose higher bits equal the state's prefix.
__global__ __launch_bounds__(256) void k_sel_hist(const float* __restrict__ vx, const float* __restrict__ vy,
                                                  const float* __restrict__ vz, const int64_t* n_dev,
                                                  const SelState* st, int shift, int bits,
                                                  unsigned* __restrict__ hist) {
  __shared__ unsigned h[1 << 12];
  const int nb = 1 << bits;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const uint64_t n = (uint64_t)*n_dev;
  const int hi = shift + bits;
  const uint32_t want = st->prefix;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t key = speed_key(vx[p], vy[p], vz[p]);
    if (hi >= 32 || (key >> hi) == (want >> hi)) atomicAdd(&h[(key >> shift) & (uint32_t)(nb - 1)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// Picks the bin holding the wanted rank (one wave: each lane sums a
// contiguous chunk of bins, a prefix over the lanes finds the chunk, its lane
// the bin); the first pass sets the rank ceil(9 n / 10) from the count.  The
// histogram is cleared for the next pass.
__global__ __launch_bounds__(64) void k_sel_pick(const int64_t* n_dev, unsigned* __restrict__ hist, SelState* st,
                                                 int shift, int bits, int first) {
  const int lane = threadIdx.x;
  const int nb = 1 << bits, per = nb / 64;
  uint64_t rank = first ? ((uint64_t)*n_dev ? (9 * (uint64_t)*n_dev + 9) / 10 : 0) : st->rank;
  uint64_t mine = 0;
  for (int b = lane * per; b < (lane + 1) * per; ++b) mine += hist[b];
  uint64_t incl = mine;
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = __shfl_up(incl, d, 64);
    if (lane >= d) incl += o;
  }
  const uint64_t excl = incl - mine;
  const bool here = rank > 0 && excl < rank && rank <= incl;
  if (here) {
    uint64_t acc = excl;
    for (int b = lane * per; b < (lane + 1) * per; ++b) {
      const uint64_t h = hist[b];
      if (acc + h >= rank) {
        st->prefix = (first ? 0u : st->prefix) | ((uint32_t)b << shift);
        st->rank = rank - acc;
        break;
      }
      acc += h;
    }
  }
  if (lane == 0 && first && rank == 0) {
    st->prefix = 0;
    st->rank = 0;
  }
  __syncthreads();
  for (int b = lane; b < nb; b += 64) hist[b] = 0;
}

// Largest fixed-point electron density, then the first cell holding it.
__global__ void k_ne_max(const int64_t* __restrict__ ne, size_t n, long long* out) {
  __shared__ long long s_w[16];
  long long m = LLONG_MIN;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x)
    m = max(m, (long long)ne[c]);
  for (int d = 32; d > 0; d >>= 1) m = max(m, (long long)__shfl_xor(m, d, 64));
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x + 63) / 64; ++w) m = max(m, s_w[w]);
    atomicMax(out, max(m, s_w[0]));
  }
}

__global__ void k_ne_first(const int64_t* __restrict__ ne, size_t n, const long long* mx,
                           unsigned long long* first) {
  const long long m = *mx;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x)
    if ((long long)ne[c] == m) atomicMin(first, (unsigned long long)c);
}

__global__ void k_weight_sum(const float* __restrict__ w, const int64_t* n_dev, double* out) {
  const uint64_t n = (uint64_t)*n_dev;
  double s = 0.0;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (uint64_t)gridDim.x * blockDim.x)
    s += (double)w[p];
  for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
  if ((threadIdx.x & 63) == 0 && s != 0.0) atomicAdd(out, s);
}

// ---------------------------------------------------------------------------
// Host launchers.


static unsigned grid_for(size_t n, unsigned cap = 16384) {
  const size_t b = (n + 255) / 256;
  return (unsigned)(b < cap ? (b > 0 ? b : 1) : cap);
}

int mg_levels(int nx, int ny, int nz, MgDims* dims) {
  int L = 0;
  dims[L++] = MgDims{nx, ny, nz};
  while (L < kMgMaxLevels && nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0 && nx > 2 && ny > 2 && nz > 2) {
    nx /= 2;
    ny /= 2;
    nz /= 2;
    dims[L++] = MgDims{nx, ny, nz};
  }
  return L;
}

hipError_t launch_sc_rhs(const int64_t* np, const int64_t* ne, const int64_t* nn, size_t n, double scale, double* f,
                         unsigned long long* fmax, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_rhs, dim3(grid_for(n, 2048)), dim3(256), 0, s, np, ne, nn, n, scale, f, fmax);
  return hipGetLastError();
}

// The finest level is stored split by colour when it is swept by launches
// (above kMgCoarseMax cells; then every dimension is even).
static bool split_finest(const MgWork& W) {
  const MgDims d = W.dims[0];
  return (size_t)d.nx * d.ny * d.nz > (size_t)kMgCoarseMax && d.nx % 2 == 0 && W.levels > 1;
}

// One V(2,2) cycle of the correction from level l down.  u[l], f[l]: the
// level's single-precision arrays (level 0 in the layout of split_finest).
hipError_t mg_vcycle(const MgWork& W, int l, hipStream_t s) {
  const MgDims d = W.dims[l];
  const double h = W.dx * (double)(1 << l);
  const float h2 = (float)(h * h);
  if ((size_t)d.nx * d.ny * d.nz <= (size_t)kMgCoarseMax) {
    MgTailArgs A{};
    A.u = W.u[l];
    A.f = W.f[l];
    A.first = l;
    A.levels = W.levels;
    size_t cells = 0;
    for (int q = l; q < W.levels; ++q) {
      cells += (size_t)W.dims[q].nx * W.dims[q].ny * W.dims[q].nz;
      const double hq = W.dx * (double)(1 << q);
      A.d[q] = W.dims[q];
      A.h2[q] = (float)(hq * hq);
      A.inv_h2[q] = 1.0f / A.h2[q];
    }
    const MgDims dl = W.dims[W.levels - 1];
    const int m = dl.nx > dl.ny ? (dl.nx > dl.nz ? dl.nx : dl.nz) : (dl.ny > dl.nz ? dl.ny : dl.nz);
    int iters = 4 * m * m;  // enough red-black sweeps for a grid of m cells a side
    A.coarse_iters = iters < 16 ? 16 : (iters > 4096 ? 4096 : iters);
    if (cells > (size_t)kMgTailCells) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mg_tail, dim3(1), dim3(512), 0, s, A);
    return hipGetLastError();
  }
  const dim3 gs = row_grid((d.nx + 1) / 2, d.ny, d.nz);
  const bool split = l == 0 && split_finest(W);
  auto smooth = [&](int color) {
    if (split)
      hipLaunchKernelGGL(k_mg_smooth<true>, gs, dim3(kRowThreads), 0, s, W.u[l], W.f[l], d.nx, d.ny, d.nz, h2, color);
    else
      hipLaunchKernelGGL(k_mg_smooth<false>, gs, dim3(kRowThreads), 0, s, W.u[l], W.f[l], d.nx, d.ny, d.nz, h2, color);
  };
  for (int it = 0; it < 2; ++it)
    for (int color = 0; color < 2; ++color) smooth(color);
  const MgDims dc = W.dims[l + 1];
  const size_t nc = (size_t)dc.nx * dc.ny * dc.nz;
  if (split)
    hipLaunchKernelGGL(k_mg_restrict<true>, row_grid(dc.nx, dc.ny, dc.nz), dim3(kRowThreads), 0, s, W.u[l], W.f[l],
                       d.nx, d.ny, d.nz, 1.0f / h2, W.f[l + 1]);
  else
    hipLaunchKernelGGL(k_mg_restrict<false>, row_grid(dc.nx, dc.ny, dc.nz), dim3(kRowThreads), 0, s, W.u[l], W.f[l],
                       d.nx, d.ny, d.nz, 1.0f / h2, W.f[l + 1]);
  hipError_t e = hipSuccess;
  if (nc > (size_t)kMgCoarseMax) e = hipMemsetAsync(W.u[l + 1], 0, nc * sizeof(float), s);  // the tail zeroes its own
  if (e != hipSuccess) return e;
  e = mg_vcycle(W, l + 1, s);
  if (e != hipSuccess) return e;
  const dim3 gp = row_grid((d.nx + 3) / 4, d.ny, d.nz);
  if (split)
    hipLaunchKernelGGL(k_mg_prolong<true>, gp, dim3(kRowThreads), 0, s, W.u[l], W.u[l + 1], d.nx, d.ny, d.nz);
  else
    hipLaunchKernelGGL(k_mg_prolong<false>, gp, dim3(kRowThreads), 0, s, W.u[l], W.u[l + 1], d.nx, d.ny, d.nz);
  for (int it = 0; it < 2; ++it)
    for (int color = 0; color < 2; ++color) smooth(color);
  return hipGetLastError();
}

hipError_t launch_defect(const MgWork& W, unsigned long long* rmax, hipStream_t s) {
  const MgDims d = W.dims[0];
  const unsigned nb = defect_blocks(d.nx, d.ny, d.nz);
  const double ih2 = 1.0 / (W.dx * W.dx);
  if (split_finest(W))
    hipLaunchKernelGGL(k_mg_defect<true>, dim3(nb), dim3(kRowThreads), 0, s, W.phi, W.rhs, d.nx, d.ny, d.nz, ih2,
                       W.f[0], W.part);
  else
    hipLaunchKernelGGL(k_mg_defect<false>, dim3(nb), dim3(kRowThreads), 0, s, W.phi, W.rhs, d.nx, d.ny, d.nz, ih2,
                       W.f[0], W.part);
  hipLaunchKernelGGL(k_max_parts, dim3(1), dim3(1024), 0, s, W.part, nb, rmax);
  return hipGetLastError();
}

hipError_t launch_correct(const MgWork& W, hipStream_t s) {
  const MgDims d = W.dims[0];
  if (split_finest(W))
    hipLaunchKernelGGL(k_mg_correct<true>, row_grid(d.nx, d.ny, d.nz), dim3(kRowThreads), 0, s, W.phi, W.u[0], d.nx,
                       d.ny, d.nz);
  else
    hipLaunchKernelGGL(k_mg_correct<false>, row_grid(d.nx, d.ny, d.nz), dim3(kRowThreads), 0, s, W.phi, W.u[0], d.nx,
                       d.ny, d.nz);
  return hipGetLastError();
}

hipError_t launch_extrapolate(double* phi, double* prev, double r, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_extrapolate, dim3(grid_for(n, 4096)), dim3(256), 0, s, phi, prev, r, n);
  return hipGetLastError();
}

hipError_t launch_sc_field(const float4* Ea, const double* phi, int nx, int ny, int nz, double dx, float4* E,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_sc_field, row_grid(nx, ny, nz), dim3(kRowThreads), 0, s, Ea, phi, nx, ny, nz, 2.0 * dx, E);
  return hipGetLastError();
}

hipError_t launch_speed_select(const float* vx, const float* vy, const float* vz, const int64_t* n_dev, uint64_t n,
                               SelState* st, unsigned* hist, hipStream_t s) {
  const unsigned g = grid_for(n, 1024);
  const int shifts[3] = {20, 8, 0}, bits[3] = {12, 12, 8};
  for (int pass = 0; pass < 3; ++pass) {
    if (pass == 0) {  // the first pick sets the rank; the histogram needs the prefix 0
      hipError_t e = hipMemsetAsync(st, 0, sizeof(SelState), s);
      if (e == hipSuccess) e = hipMemsetAsync(hist, 0, (1u << 12) * sizeof(unsigned), s);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_sel_hist, dim3(g), dim3(256), 0, s, vx, vy, vz, n_dev, st, shifts[pass], bits[pass], hist);
    hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(64), 0, s, n_dev, hist, st, shifts[pass], bits[pass],
                       pass == 0 ? 1 : 0);
  }
  return hipGetLastError();
}

hipError_t launch_densest(const int64_t* ne, size_t n, long long* mx, unsigned long long* first, hipStream_t s) {
  hipLaunchKernelGGL(k_ne_max, dim3(grid_for(n, 2048)), dim3(256), 0, s, ne, n, mx);
  hipLaunchKernelGGL(k_ne_first, dim3(grid_for(n)), dim3(256), 0, s, ne, n, mx, first);
  return hipGetLastError();
}

hipError_t launch_weight_sum(const float* w, const int64_t* n_dev, uint64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_weight_sum, dim3(grid_for(n, 2048)), dim3(256), 0, s, w, n_dev, out);
  return hipGetLastError();
}

}  // namespace pcmcc
