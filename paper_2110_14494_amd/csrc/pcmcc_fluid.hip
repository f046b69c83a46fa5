// Drift-diffusion-reaction fluid step with the local field approximation
// (arXiv:2110.14494 Sec. 2.2): electrons with Koren-limited advective fluxes
// and central diffusive fluxes, ionization / attachment sources, immobile
// ions, Heun's method with the space-charge field recomputed for the
// predicted densities, and the fluid time-step limits.
//
// * Electrons drift with v = -mu E; flux = v n_face - D (n_R - n_L) / dx;
//   dn_e/dt = -div(flux) + (alpha - eta) mu |E| n_e; positive ions gain
//   alpha mu |E| n_e, negative ions eta mu |E| n_e.
// * Face field = mean of the two cells' field vectors; mu and D from its
//   magnitude; the upwind face density adds half the Koren-limited slope
//   (slope form, psi(r) = max(0, min(2r, (1 + 2r) / 3, 2))).
// * Densities have homogeneous Neumann boundaries as mirror ghost cells
//   (n_-1 = n_0, n_-2 = n_1); a ghost cell's field is the boundary cell's.
// * Transport data: tables of mu N, D N, alpha / N, eta / N on log-spaced E/N
//   nodes, linear in ln(E/N), held constant outside.
// One thread per cell computes its six face fluxes (each face twice: no
// flux array, one pass over the densities and fields per stage); rows are
// handed out in XCD-local runs (row_pos).
#include <hip/hip_runtime.h>

#include "pcmcc_field.hpp"
#include "pcmcc_internal.hpp"

namespace pcmcc {

namespace {

__device__ __forceinline__ int mirror(int i, int m) {
  i = i < 0 ? -i - 1 : (i >= m ? 2 * m - i - 1 : i);
  return min(max(i, 0), m - 1);
}

// Table position of a field of squared magnitude E2: u = (ln(E/N in Td) -
// ln_lo) (n - 1) / ln_span with ln(E/N) = ln(E2) / 2 + ln(1e21 / N), clamped.
// (Reciprocals and logarithms of the constants are precomputed: the kernel
// multiplies where the definition divides, a difference of an ulp or so.)
struct TabPos {
  int i;
  double f;
};
__device__ __forceinline__ TabPos tab_pos(const FluidTab& T, double E2) {
#pragma clang fp contract(off)
  double u = (0.5 * log(fmax(E2, 1e-300)) + T.ln_td - T.ln_lo) * T.pos_scale;
  u = fmin(fmax(u, 0.0), (double)(T.n - 1));
  const int i = min((int)floor(u), T.n - 2);
  return TabPos{i, u - (double)i};
}
__device__ __forceinline__ double tab_at(const TabPos& p, const double* v) {
#pragma clang fp contract(off)
  return (1.0 - p.f) * v[p.i] + p.f * v[p.i + 1];
}

// Koren-limited slope from the upwind slope a and the downwind slope b.
__device__ __forceinline__ double koren(double a, double b) {
#pragma clang fp contract(off)
  if (!(a * b > 0.0)) return 0.0;
  const double aa = fabs(a), ab = fabs(b);
  const double m = fmin(fmin(2.0 * ab, (aa + 2.0 * ab) * (1.0 / 3.0)), 2.0 * aa);
  return a > 0.0 ? m : -m;
}

__device__ __forceinline__ double3 e3(float4 e) { return make_double3((double)e.x, (double)e.y, (double)e.z); }

}  // namespace

// One Heun stage on cell (i, j, k).  Stage 1: k1 = F(n0); out = n0 + dt k1.
// Stage 2: n0 += dt/2 (k1 + F(n_s)) in place (n_s: the predicted densities).
__global__ __launch_bounds__(kRowThreads) void k_fl_stage(FluidArgs A, int stage) {
#pragma clang fp contract(off)
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const RowPos P = row_pos(nx, ny);
  const int i = P.x0 + (int)threadIdx.x, j = P.j, k = P.k;
  if (i >= nx) return;
  const double* __restrict__ n = stage == 1 ? A.ne : A.se;
  const size_t c = ((size_t)k * ny + j) * nx + i;
  const double3 Ec = e3(A.E[c]);
  const double inv_dx = 1.0 / A.dx;
  double div = 0.0;
  const int dims[3] = {nx, ny, nz};
  const int pos[3] = {i, j, k};
  const size_t stride[3] = {1, (size_t)nx, (size_t)nx * ny};
  for (int ax = 0; ax < 3; ++ax) {
    const int m = dims[ax], p = pos[ax];
    const size_t base = c - (size_t)p * stride[ax];
    double nv[5];  // cells p-2 .. p+2 along the axis (mirror ghosts)
#pragma unroll
    for (int q = 0; q < 5; ++q) nv[q] = n[base + (size_t)mirror(p - 2 + q, m) * stride[ax]];
    const double3 Em = p > 0 ? e3(A.E[c - stride[ax]]) : Ec;
    const double3 Ep = p < m - 1 ? e3(A.E[c + stride[ax]]) : Ec;
    double fl[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {  // face between cells (p-1+side) and (p+side)
      const double3 EL = side ? Ec : Em, ER = side ? Ep : Ec;
      const double3 Ef = make_double3(0.5 * (EL.x + ER.x), 0.5 * (EL.y + ER.y), 0.5 * (EL.z + ER.z));
      const TabPos tp = tab_pos(A.T, (Ef.x * Ef.x + Ef.y * Ef.y) + Ef.z * Ef.z);
      const double mu = tab_at(tp, A.T.muN) * A.T.inv_gas_N;
      const double D = tab_at(tp, A.T.DN) * A.T.inv_gas_N;
      const double En = ax == 0 ? Ef.x : (ax == 1 ? Ef.y : Ef.z);
      const double v = -mu * En;
      const double nLL = nv[side], nL = nv[side + 1], nR = nv[side + 2], nRR = nv[side + 3];
      const double up = v >= 0.0 ? nL + 0.5 * koren(nL - nLL, nR - nL) : nR + 0.5 * koren(nR - nRR, nL - nR);
      fl[side] = v * up - D * (nR - nL) * inv_dx;
    }
    div += (fl[1] - fl[0]) * inv_dx;
  }
  const double E2 = (Ec.x * Ec.x + Ec.y * Ec.y) + Ec.z * Ec.z;
  const double Emag = sqrt(E2);
  const TabPos tp = tab_pos(A.T, E2);
  const double mu = tab_at(tp, A.T.muN) * A.T.inv_gas_N;
  const double alpha = tab_at(tp, A.T.aN) * A.T.gas_N;
  const double eta = tab_at(tp, A.T.eN) * A.T.gas_N;
  const double rate = mu * Emag * n[c];
  const double ke = -div + (alpha - eta) * rate, kp = alpha * rate, kn = eta * rate;
  if (stage == 1) {
    A.k1e[c] = ke;
    A.k1p[c] = kp;
    A.k1n[c] = kn;
    A.se[c] = A.ne[c] + A.dt * ke;
    A.sp[c] = A.np[c] + A.dt * kp;
    A.sn[c] = A.nn[c] + A.dt * kn;
  } else {
    const double h = 0.5 * A.dt;
    A.ne[c] = A.ne[c] + h * (A.k1e[c] + ke);
    A.np[c] = A.np[c] + h * (A.k1p[c] + kp);
    A.nn[c] = A.nn[c] + h * (A.k1n[c] + kn);
  }
}

// Poisson right-hand side from the double densities: -e ((n+ - n_e) - n-) / eps0.
__global__ void k_fl_rhs(const double* __restrict__ np, const double* __restrict__ ne,
                         const double* __restrict__ nn, size_t n, double* __restrict__ f,
                         unsigned long long* fmax_bits) {
#pragma clang fp contract(off)
  __shared__ double s_w[4];
  double m = 0.0;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) {
    const double q = ((np[c] - ne[c]) - nn[c]) * kFlQe;
    const double v = -q / kFlEps0;
    f[c] = v;
    m = fmax(m, fabs(v));
  }
  for (int d = 32; d > 0; d >>= 1) m = fmax(m, __shfl_xor(m, d, 64));
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)blockDim.x / 64; ++w) m = fmax(m, s_w[w]);
    if (m > 0.0) atomicMax(fmax_bits, (unsigned long long)__double_as_longlong(m));
  }
}

// Time-step inputs: max of 2 N_dim D / dx^2 + sum |v_i| / dx and of e n mu / eps0.
__global__ __launch_bounds__(256) void k_fl_dt(const double* __restrict__ ne, const float4* __restrict__ E,
                                               size_t n, FluidTab T, double dx, unsigned long long* out) {
#pragma clang fp contract(off)
  __shared__ double s_c[4], s_d[4];
  double mc = 0.0, md = 0.0;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) {
    const double3 e = e3(E[c]);
    const TabPos tp = tab_pos(T, (e.x * e.x + e.y * e.y) + e.z * e.z);
    const double mu = tab_at(tp, T.muN) * T.inv_gas_N;
    const double D = tab_at(tp, T.DN) * T.inv_gas_N;
    const double cfl = 2.0 * 3.0 * D / (dx * dx) + (mu * ((fabs(e.x) + fabs(e.y)) + fabs(e.z))) / dx;
    const double drt = kFlQe * ne[c] * mu / kFlEps0;
    mc = fmax(mc, cfl);
    md = fmax(md, drt);
  }
  for (int d = 32; d > 0; d >>= 1) {
    mc = fmax(mc, __shfl_xor(mc, d, 64));
    md = fmax(md, __shfl_xor(md, d, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    s_c[threadIdx.x / 64] = mc;
    s_d[threadIdx.x / 64] = md;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)blockDim.x / 64; ++w) {
      mc = fmax(mc, s_c[w]);
      md = fmax(md, s_d[w]);
    }
    if (mc > 0.0) atomicMax(&out[0], (unsigned long long)__double_as_longlong(mc));
    if (md > 0.0) atomicMax(&out[1], (unsigned long long)__double_as_longlong(md));
  }
}

static unsigned fl_blocks(size_t n) {
  const size_t b = (n + 255) / 256;
  return (unsigned)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

hipError_t launch_fluid_stage(const FluidArgs& A, int stage, hipStream_t s) {
  hipLaunchKernelGGL(k_fl_stage, row_grid(A.nx, A.ny, A.nz), dim3(kRowThreads), 0, s, A, stage);
  return hipGetLastError();
}

hipError_t launch_fluid_rhs(const double* np, const double* ne, const double* nn, size_t n, double* f,
                            unsigned long long* fmax_bits, hipStream_t s) {
  hipLaunchKernelGGL(k_fl_rhs, dim3(fl_blocks(n)), dim3(256), 0, s, np, ne, nn, n, f, fmax_bits);
  return hipGetLastError();
}

hipError_t launch_fluid_dt(const double* ne, const float4* E, size_t n, const FluidTab& T, double dx,
                           unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_fl_dt, dim3(fl_blocks(n)), dim3(256), 0, s, ne, E, n, T, dx, out);
  return hipGetLastError();
}

}  // namespace pcmcc
