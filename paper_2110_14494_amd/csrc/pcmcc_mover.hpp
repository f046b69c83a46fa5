// Device code shared by the PIC step and the swarm kernels: the field policy
// of the grid, staged rate tables, isotropic scattering, newborn queues,
// wave-aggregated slot reservation and particle record access.
//
// Method: arXiv:2110.14494 Sec. 2.1.1 (velocity Verlet, eq. (1)-(2), and the
// null-collision method) and Sec. 2.1.5 (rates from cross sections).
#pragma once

#include <hip/hip_runtime.h>

#include "pcmcc_device.hpp"
#include "pcmcc_internal.hpp"

namespace pcmcc {

// ---------------------------------------------------------------------------
// small device helpers

template <class T>
__device__ __forceinline__ T ld_acq(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t rank_in(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Reserves one slot per calling lane in a counter with a single atomic for
// the wave: every active lane that calls it gets base + its rank.
__device__ __forceinline__ uint64_t wave_reserve(unsigned long long* counter) {
  const uint64_t mask = __ballot(1);
  const int leader = __ffsll((unsigned long long)mask) - 1;
  uint64_t base = 0;
  if ((int)lane_id() == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)base, leader);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(base >> 32), leader);
  return (((uint64_t)hi << 32) | lo) + rank_in(mask);
}

struct Cnt {
  uint32_t v[NCNT];
};

__device__ __forceinline__ void load_p(const Soa& s, uint64_t i, PState& p) {
  p.x = s.x[i];
  p.y = s.y[i];
  p.z = s.z[i];
  p.vx = s.vx[i];
  p.vy = s.vy[i];
  p.vz = s.vz[i];
  p.w = s.w[i];
  p.id = s.id[i];
}

__device__ __forceinline__ void store_p(const Soa& s, uint64_t i, const PState& p) {
  s.x[i] = p.x;
  s.y[i] = p.y;
  s.z[i] = p.z;
  s.vx[i] = p.vx;
  s.vy[i] = p.vy;
  s.vz[i] = p.vz;
  s.w[i] = p.w;
  s.id[i] = p.id;
}

__device__ __forceinline__ void load_pend(const PendSoa& s, uint64_t i, PState& p, float& tb) {
  p.x = s.x[i];
  p.y = s.y[i];
  p.z = s.z[i];
  p.vx = s.vx[i];
  p.vy = s.vy[i];
  p.vz = s.vz[i];
  p.w = s.w[i];
  p.id = s.id[i];
  tb = s.tb[i];
}

// A structure in the launch's kernel-argument memory, read where it is used
// (scalar loads through a pointer made opaque there) instead of being held in
// scalar registers for the whole mover loop: the mover's loop-invariant
// pointer sets exceed the scalar registers of a wave, and spilled ones come
// back one v_readlane (a vector instruction) each.
template <class T>
struct KArg {
  const __attribute__((address_space(4))) T* p;
  __device__ __forceinline__ T get() const {
#if defined(__HIP_DEVICE_COMPILE__)
    const __attribute__((address_space(4))) T* q = p;
    asm volatile("" : "+s"(q));
    return *q;
#else
    return T{};  // host pass: never called
#endif
  }
};

// Queue of newborns of one generation (arrays and event lists in
// kernel-argument memory).
struct BirthSink {
  KArg<PendSoa> qk;
  unsigned long long* count;
  uint64_t cap;
  unsigned* overflow;
  uint32_t tag;  // swarm index of the items being advanced (swarm queues only)
  KArg<EventSink> evk;
  __device__ __forceinline__ void push(const PState& c, float tb) const {
    const uint64_t slot = wave_reserve(count);
    if (slot < cap) {
      const PendSoa q = qk.get();
      if (q.sw) q.sw[slot] = tag;
      q.x[slot] = c.x;
      q.y[slot] = c.y;
      q.z[slot] = c.z;
      q.vx[slot] = c.vx;
      q.vy[slot] = c.vy;
      q.vz[slot] = c.vz;
      q.w[slot] = c.w;
      q.id[slot] = c.id;
      q.tb[slot] = tb;
    } else {
      atomicOr(overflow, OVF_CAPACITY);
    }
  }
};

// Field of the PIC step: the grid.
struct GridField {
  GridView G;
  double qm;
  // Interface of the segment-pipelined mover (one group: the tag is 0): the
  // run's key, a gather that also returns its record, and the bound from
  // that record.
  Key k;
  // The same view in kernel-argument memory.  The gather reads its
  // constants from there through a pointer made opaque at each use, so they
  // come back with a few scalar loads per segment instead of living in
  // scalar registers for the whole mover loop (where they would spill into
  // vector lanes and return one v_readlane each).
  const __attribute__((address_space(4))) GridView* gk;
  using Where = const float4*;
  // The key passes through an empty asm statement at every use, so that the
  // Philox round keys are derived there with scalar adds instead of being
  // hoisted out of the mover loop as twenty more uniform values (which spill
  // into vector lanes and come back one v_readlane each).
  __device__ __forceinline__ Key key(uint32_t) const {
    uint32_t k0 = k.k0, k1 = k.k1;
    asm volatile("" : "+s"(k0), "+s"(k1));
    return Key{k0, k1};
  }
  __device__ __forceinline__ double3 accel(double x, double y, double z, uint32_t, Where& w) const {
    const __attribute__((address_space(4))) GridView* g = gk;
    asm volatile("" : "+s"(g));
    GridView v;
    v.P = g->P;
    v.nx = g->nx;
    v.ny = g->ny;
    v.nz = g->nz;
    v.px = g->px;
    v.py = g->py;
    v.o[0] = g->o[0];
    v.o[1] = g->o[1];
    v.o[2] = g->o[2];
    v.nd[0] = g->nd[0];
    v.nd[1] = g->nd[1];
    v.nd[2] = g->nd[2];
    v.inv_dx = g->inv_dx;
    return gather(v, g->qm, x, y, z, &w);
  }
  __device__ __forceinline__ void bound_at(Where w, uint32_t, float speed, float t_rem, float& a_abs,
                                           float& da) const {
    accel_bound_at(G, w, speed, t_rem, a_abs, da);
  }
};

// Tables as the kernels read them (staged in LDS).  C is node-major: row i
// holds the cumulative rates of all processes at node i, padded with zeros
// to `row` entries, so one node is one or two 16-byte reads.
struct Tab {
  const float* C;
  const float* P;
  const float* thr;
  const int* kind;
  int n, nproc, row;
  float u_scale, u_offset, eps_max;
};

// The scalars a flight segment needs from the tables and the species, kept
// at a fixed LDS address and read at each use through an offset made opaque
// there: held in scalar registers for the whole mover loop they would spill
// into vector lanes and come back one v_readlane each, while one LDS read
// brings four of them.
struct TabConst {
  float u_scale, u_offset, u_top, fl_top;  // table position; clamps n - 1 and n - 2
  float k_eps;                             // eps[eV] = k_eps |v|^2
  float recoil;                            // 2 m / M
  int row;                                 // floats per node of C
  int p_off;                               // P at C + p_off
  double k_eps_d, inv_k_d;                 // k_eps and 1 / k_eps in double precision
  double eps_max;                          // last node energy
};
static __shared__ TabConst g_tab_const;

__device__ __forceinline__ TabConst tab_const() {
  uint32_t off = 0;
  asm volatile("" : "+v"(off));
  return *reinterpret_cast<const TabConst*>(reinterpret_cast<const char*>(&g_tab_const) + off);
}

// Cumulative rates at table position (i, f), linear between nodes i and
// i + 1 (entries at and beyond nproc are zero).
__device__ __forceinline__ void cum_rates(const Tab& T, int i, float f, float c[kMaxProc], int row) {
  const float4* a = reinterpret_cast<const float4*>(T.C + (size_t)i * row);
  const float4* b = reinterpret_cast<const float4*>(T.C + (size_t)(i + 1) * row);
  auto put = [&](int o, float4 lo, float4 hi) {
    c[o] = fmaf(f, hi.x - lo.x, lo.x);
    c[o + 1] = fmaf(f, hi.y - lo.y, lo.y);
    c[o + 2] = fmaf(f, hi.z - lo.z, lo.z);
    c[o + 3] = fmaf(f, hi.w - lo.w, lo.w);
  };
  put(0, a[0], b[0]);
  if (row == 8) {
    put(4, a[1], b[1]);
  } else {
#pragma unroll
    for (int k = 4; k < kMaxProc; ++k) c[k] = 0.0f;
  }
}
__device__ __forceinline__ void cum_rates(const Tab& T, int i, float f, float c[kMaxProc]) {
  cum_rates(T, i, f, c, T.row);
}

// The cumulative rates of a table of ROW (4 or 8) floats per node, the
// row fixed at compile time.
template <int ROW>
__device__ __forceinline__ void cum_rates_row(const Tab& T, int i, float f, float c[ROW]) {
  const float4* a = reinterpret_cast<const float4*>(T.C + (size_t)i * ROW);
  const float4* b = reinterpret_cast<const float4*>(T.C + (size_t)(i + 1) * ROW);
#pragma unroll
  for (int h = 0; h < ROW / 4; ++h) {
    const float4 lo = a[h], hi = b[h];
    c[4 * h] = fmaf(f, hi.x - lo.x, lo.x);
    c[4 * h + 1] = fmaf(f, hi.y - lo.y, lo.y);
    c[4 * h + 2] = fmaf(f, hi.z - lo.z, lo.z);
    c[4 * h + 3] = fmaf(f, hi.w - lo.w, lo.w);
  }
}

// First process whose cumulative rate exceeds y, or -1 (a null collision),
// over a row of ROW entries (entries past the last process are zero).
template <int ROW>
__device__ __forceinline__ int pick_process_row(const float c[ROW], float y) {
  int k = -1;
#pragma unroll
  for (int kk = ROW - 1; kk >= 0; --kk)
    if (y < c[kk]) k = kk;
  return k;
}

// First process whose cumulative rate exceeds y, or -1 (a null collision).
__device__ __forceinline__ int pick_process(const float c[kMaxProc], float y) {
  int k = -1;
#pragma unroll
  for (int kk = kMaxProc - 1; kk >= 0; --kk)
    if (y < c[kk]) k = kk;
  return k;
}

// x clamped to [lo, hi] (lo <= hi, x not NaN) in one v_med3_f32; fminf and
// fmaxf would first quiet every operand read from memory.
__device__ __forceinline__ float clamp_med3(float x, float lo, float hi) {
  return __builtin_amdgcn_fmed3f(x, lo, hi);
}

__device__ __forceinline__ float majorant_t(const Tab& T, const TabConst& c, float s_ub) {
  const float s = s_ub * kGuard;
  const float eps = c.k_eps * s * s;
  float u = fmaf(__log2f(eps), c.u_scale, c.u_offset);
  u = clamp_med3(u, 0.0f, c.u_top);
  const float fl = clamp_med3(floorf(u), 0.0f, c.fl_top);
  const int i = (int)fl;
  return lerp_at(T.C + c.p_off, i, u - fl);
}
__device__ __forceinline__ float majorant_t(const Tab& T, const SpeciesView&, float s_ub) {
  return majorant_t(T, tab_const(), s_ub);
}

// Square root of x >= 0 (0 for x <= 0) from the hardware reciprocal square
// root refined by one Newton step: the hardware value is within 5.2e-8
// relative and the step squares that, to within 4.3e-15 (measured over 2^22
// values log-uniform in [2^-60, 2^60]); the mover takes new speeds, cos(chi)
// and polar sines from it, and its results leave a step in single precision.
__device__ __forceinline__ double sqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-0.5 * x * r, r, 1.5);
  return x > 0.0 ? x * r : 0.0;
}

// 1/sqrt(x) for x > 0, as above.
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  return r * fma(-0.5 * x * r, r, 1.5);
}

// Isotropic unit vector from two uniforms: cos(theta) = 1 - 2 U1 and
// sin(theta) = 2 sqrt(U1 (1 - U1)) (no cancellation near the poles; U1 and
// 1 - U1 are exact), azimuth 2 pi U2.  The azimuth's sine and cosine are the
// hardware ones, which take the angle in turns (v_sin_f32, v_cos_f32: within
// 1.3e-7 of sin(2 pi U2), cos(2 pi U2) over all 2^23 uniforms), so s2 =
// cos^2 + sin^2 is within 3e-7 of 1 and 1/sqrt(s2) = 3/2 - s2/2 to about
// 4e-14: |n| = 1 to that accuracy.
__device__ __forceinline__ void iso_dir(uint32_t r1, uint32_t r2, double& nx, double& ny, double& nz) {
  const double u = (double)unif(r1);
  const double cth = fma(-2.0, u, 1.0);
  const double sth_half = sqrt_nr(u * (1.0 - u));  // u (1 - u) > 2^-25: never zero or subnormal
  const float t = unif(r2);
  const float sp = __builtin_amdgcn_sinf(t), cp = __builtin_amdgcn_cosf(t);
  const double s2 = fma((double)sp, (double)sp, (double)cp * cp);
  // sin(theta) (3/2 - s2/2) = sth_half (3 - s2), the factor 2 moved exactly
  const double inv = sth_half * fma(-1.0, s2, 3.0);
  nx = inv * cp;
  ny = inv * sp;
  nz = cth;
}

// Inside the grid, judged on the double-precision end position.
__device__ __forceinline__ bool inside(const GridView& G, const PState& p) {
  return p.xd >= G.lo[0] && p.xd < G.hi[0] && p.yd >= G.lo[1] && p.yd < G.hi[1] && p.zd >= G.lo[2] &&
         p.zd < G.hi[2];
}

// Stages the tables in LDS; returns the view the kernels read.
__device__ inline Tab stage_tables(const TableView& TV, const SpeciesView& S, float* smem) {
  const int row = table_row(TV.nproc);
  const int nC = row * TV.n;
  for (int e = threadIdx.x; e < nC; e += blockDim.x) {
    const int i = e / row, k = e % row;
    smem[e] = k < TV.nproc ? TV.C[(size_t)k * TV.n + i] : 0.0f;
  }
  for (int i = threadIdx.x; i < TV.n; i += blockDim.x) smem[nC + i] = TV.P[i];
  float* thr = smem + nC + TV.n;
  int* kind = (int*)(thr + kMaxProc);
  if (threadIdx.x < (unsigned)kMaxProc) {
    thr[threadIdx.x] = TV.thr[threadIdx.x];
    kind[threadIdx.x] = TV.kind[threadIdx.x];
  }
  if (threadIdx.x == 0) {
    TabConst c;
    c.u_scale = TV.u_scale;
    c.u_offset = TV.u_offset;
    c.u_top = (float)(TV.n - 1);
    c.fl_top = (float)(TV.n - 2);
    c.k_eps = S.k_eps;
    c.recoil = S.recoil;
    c.row = row;
    c.p_off = nC;
    c.k_eps_d = S.k_eps_d;
    c.inv_k_d = S.inv_k_d;
    c.eps_max = (double)TV.eps_top;
    g_tab_const = c;
  }
  __syncthreads();
  Tab T;
  T.C = smem;
  T.P = smem + nC;
  T.thr = thr;
  T.kind = kind;
  T.n = TV.n;
  T.nproc = TV.nproc;
  T.row = row;
  T.u_scale = TV.u_scale;
  T.u_offset = TV.u_offset;
  T.eps_max = TV.eps_top;
  return T;
}

// Sums per-thread counters over the block into partial[blockIdx.x][*].
__device__ inline void block_counters(const Cnt& c, unsigned long long* partial) {
  __shared__ unsigned long long red[NCNT];
  if (threadIdx.x < NCNT) red[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NCNT; ++k) {
    uint32_t v = c.v[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane_id() == 0) atomicAdd(&red[k], (unsigned long long)v);
  }
  __syncthreads();
  if (threadIdx.x < NCNT) partial[(size_t)blockIdx.x * NCNT + threadIdx.x] = red[threadIdx.x];
}


}  // namespace pcmcc
