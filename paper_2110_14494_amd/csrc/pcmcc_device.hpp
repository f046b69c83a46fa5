// Device-side building blocks of the PIC-MCC electron update for gfx950:
// Philox4x32-10, single-precision collision tables, the collision-frequency
// majorant, trilinear field interpolation and the velocity-Verlet step.
//
// Method: arXiv:2110.14494 Sec. 2.1.1 (velocity Verlet, eq. (1)-(2), and the
// null-collision method), Sec. 2.1.3 (trilinear interpolation on the
// cell-centred grid), Sec. 2.1.5 (rates from cross sections).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcmcc {

constexpr int kMaxProc = 8;
constexpr int kMaxSegments = 1 << 20;  // per particle and step; beyond it the particle is dropped
constexpr int kMaxGenerations = 64;    // newborn generations within one step
constexpr float kKappa = 4.0f;         // flight horizon in expected candidate collisions
constexpr float kGuard = 1.0f + 0x1p-16f;

enum Kind { ELASTIC = 0, EXCITATION = 1, IONIZATION = 2, ATTACHMENT = 3 };
enum Tag : uint32_t { TAG_MAIN = 0, TAG_BIRTH = 1, TAG_AUX = 2 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The key is the run
// seed, so the ten round keys are wave-uniform and live in scalar registers.
struct Key {
  uint32_t k0, k1;
};

__device__ __forceinline__ uint4 philox(uint4 c, Key key) {
  uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32 -> 64-bit product per multiplier (v_mad_u64_u32); each
    // three-way xor is one v_bitop3_b32 (truth table 0x96), which the
    // compiler does not form from two xors by itself
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96), (uint32_t)p1,
                   __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96), (uint32_t)p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ uint4 draw(Key key, uint64_t id, uint32_t step, uint32_t j, uint32_t tag) {
  return philox(make_uint4((uint32_t)id, (uint32_t)(id >> 32), step, (j << 2) | tag), key);
}

// An electron's draws within a step share the counter's first three words
// (id, step), so three of the twenty products of each draw are the same for
// all of them: the first round's product of the id's low word, the second
// round's product of its first word and the third round's product of its
// third word (the first round's product of the step is wave-uniform).  They
// are formed once when the electron starts its step; draw_pre then gives
// exactly philox(id, step, w) from them.
struct PhiloxPre {
  uint32_t a;  // high word of the first round's product of the id's low word
  uint32_t b;  // low word of the second round's first product
  uint32_t c, d;  // high and low words of the third round's second product
};

__device__ __forceinline__ PhiloxPre philox_pre(Key key, uint64_t id, uint32_t step) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * (uint32_t)id;
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * step;
  const uint32_t x = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), (uint32_t)(id >> 32), key.k0, 0x96);
  const uint64_t q0 = (uint64_t)0xD2511F53u * x;  // round 2, first product
  const uint32_t z = __builtin_amdgcn_bitop3_b32((uint32_t)(q0 >> 32), (uint32_t)p0, key.k1 + 0xBB67AE85u, 0x96);
  const uint64_t r1 = (uint64_t)0xCD9E8D57u * z;  // round 3, second product
  return PhiloxPre{(uint32_t)(p0 >> 32), (uint32_t)q0, (uint32_t)(r1 >> 32), (uint32_t)r1};
}

// philox((id, id >> 32, step, w), key) for the electron whose PhiloxPre is pre.
__device__ __forceinline__ uint4 draw_pre(Key key, const PhiloxPre& pre, uint32_t step, uint32_t w) {
  uint32_t k0 = key.k0, k1 = key.k1;
  const uint32_t y1 = (uint32_t)((uint64_t)0xCD9E8D57u * step);  // round 1's second word (uniform)
  const uint32_t z1 = __builtin_amdgcn_bitop3_b32(pre.a, w, k1, 0x96);
  k0 += 0x9E3779B9u;
  k1 += 0xBB67AE85u;
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * z1;  // round 2, second product
  const uint32_t x2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), y1, k0, 0x96);
  const uint32_t y2 = (uint32_t)p1;
  k0 += 0x9E3779B9u;
  k1 += 0xBB67AE85u;
  const uint64_t p0 = (uint64_t)0xD2511F53u * x2;  // round 3, first product
  uint4 c = make_uint4(__builtin_amdgcn_bitop3_b32(pre.c, y2, k0, 0x96), pre.d,
                       __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), pre.b, k1, 0x96), (uint32_t)p0);
  k0 += 0x9E3779B9u;
  k1 += 0xBB67AE85u;
#pragma unroll
  for (int r = 3; r < 10; ++r) {
    const uint64_t q0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t q1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(q1 >> 32), c.y, k0, 0x96), (uint32_t)q1,
                   __builtin_amdgcn_bitop3_b32((uint32_t)(q0 >> 32), c.w, k1, 0x96), (uint32_t)q0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Uniform in (0,1) from the top 23 bits: ((r >> 9) + 1/2) 2^-23, exact in FP32
// (one multiply-add: k 2^-23 + 2^-24 = (2k + 1) 2^-24 has at most 24
// significant bits, so the fused result is the exact value).
__device__ __forceinline__ float unif(uint32_t r) { return fmaf((float)(r >> 9), 0x1p-23f, 0x1p-24f); }

// ---------------------------------------------------------------------------
// Collision tables: cumulative rates C[k][i] in process order and the prefix
// maximum P[i] of the total, at energies linear in ln(eps).  The table
// position is u = log2(eps) * u_scale + u_offset.
struct TableView {
  const float* C;   // [nproc][n]
  const float* P;   // [n]
  const float* nu;  // [nproc][n]
  int n, nproc;
  float u_scale, u_offset;
  float eps_top;  // last node energy
  float thr[kMaxProc];
  int kind[kMaxProc];
};

// Processes per node of the staged cumulative table (padded with zero
// entries, which no draw selects): 4 or 8.
__host__ __device__ inline int table_row(int nproc) { return nproc <= 4 ? 4 : 8; }

// Floats of LDS the staged tables take: C (node-major rows) and P,
// thresholds and kinds.
__host__ __device__ inline size_t table_lds_floats(const TableView& T) {
  return (size_t)(table_row(T.nproc) + 1) * T.n + 2 * kMaxProc;
}

// Physical constants of the species and gas, single precision.
struct SpeciesView {
  double qm;       // q/m
  float k_eps;     // eps[eV] = k_eps |v|^2
  float inv_k;     // 1 / k_eps
  float recoil;    // 2 m / M
  double k_eps_d;  // the same two in double precision
  double inv_k_d;
};

__device__ __forceinline__ void locate(const TableView& T, float eps, int& i, float& f) {
  float u = fmaf(__log2f(eps), T.u_scale, T.u_offset);  // eps = 0 gives -inf
  u = fminf(fmaxf(u, 0.0f), (float)(T.n - 1));
  const float fl = fminf(floorf(u), (float)(T.n - 2));
  i = (int)fl;
  f = u - fl;
}

__device__ __forceinline__ float lerp_at(const float* row, int i, float f) {
  const float a = row[i], b = row[i + 1];
  return fmaf(f, b - a, a);
}

// Majorant of the total rate for speeds below s_ub (prefix maximum
// interpolated at the energy of s_ub, inflated as a rounding guard).
__device__ __forceinline__ float majorant(const TableView& T, const SpeciesView& S, const float* P, float s_ub) {
  const float s = s_ub * kGuard;
  int i;
  float f;
  locate(T, S.k_eps * s * s, i, f);
  return lerp_at(P, i, f);
}

// Largest speed reachable within h from v under acceleration a0 now, when
// |a| <= a_abs and |a - a0| <= da along the way.
__device__ __forceinline__ float speed_bound(float3 v, float3 a0, float speed, float a_abs, float da, float h) {
  const float wx = fmaf(a0.x, h, v.x), wy = fmaf(a0.y, h, v.y), wz = fmaf(a0.z, h, v.z);
  const float s_dir = fmaf(da, h, fmaxf(speed, __builtin_amdgcn_sqrtf(fmaf(wz, wz, fmaf(wy, wy, wx * wx)))));
  return fminf(fmaf(a_abs, h, speed), s_dir);
}

// ---------------------------------------------------------------------------
// Field on the cell-centred grid, corner-packed.  The trilinear interpolation
// at a point reads the fields at the 8 cell centres around it: lower centre
// index (i, j, k) = floor((x - x0)/dx - 1/2) per axis, in [-1, n] after
// clamping the coordinate to [-1, n], and the upper one i + 1, both clamped
// to the grid.  The packed field holds, for every lower index (n + 2 per
// axis), one 128-byte record: floats 3c .. 3c+2 = E at corner
// c = 4 dz + 2 dy + dx for dx = 0, and the single-precision difference
// E(c) - E(c - 1) along x for dx = 1 (so that each x interpolation is one
// multiply-add; the gather's result is the same as from the plain corner
// values), floats 24 and 25 = the local bound of the cell
// clamp(i, j, k) (max |E| and field-range norm over its 4x4x4 centres).  A
// gather therefore reads a single cache line.
constexpr int kRecFloats = 32;

struct GridView {
  const float4* P;  // packed records, kRecFloats / 4 float4 each
  int nx, ny, nz;
  int px, py;       // records per row and per plane stride: nx + 2, ny + 2
  double o[3];      // origin
  double nd[3];     // nx, ny, nz as doubles (the coordinate clamp)
  double inv_dx;
  float dx;
  double lo[3], hi[3];  // domain
  float a_glob;         // |q/m| max |E|
  float qm_abs;
  double qm;  // q/m of the species (the gather's factor)
};

// Cell-centre coordinate u = (x - x0)/dx - 1/2 of one axis, clamped to
// [-1, n], split into the lower centre index and the fraction.
__device__ __forceinline__ void cell_coord(double x, double o, double inv_dx, double n, int& i, float& f) {
  double u = fma(x - o, inv_dx, -0.5);
  u = fmin(fmax(u, -1.0), n);
  const double fl = floor(u);
  i = (int)fl;
  f = (float)(u - fl);
}

// Record of lower centre index (i, j, k), each in [-1, n].
__device__ __forceinline__ const float4* grid_record(const GridView& G, int i, int j, int k) {
  const uint32_t r = ((uint32_t)(k + 1) * (uint32_t)G.py + (uint32_t)(j + 1)) * (uint32_t)G.px + (uint32_t)(i + 1);
  return G.P + (size_t)r * (kRecFloats / 4);
}

// Trilinear interpolation with clamped indices (constant outside the
// outermost centres), returned as acceleration (q/m) E with q/m applied in
// double precision.
// `rec_out` receives the record read (its bound words serve accel_bound_at).
__device__ __forceinline__ double3 gather(const GridView& G, double qm, double x, double y, double z,
                                          const float4** rec_out = nullptr) {
  int i, j, k;
  float gx, gy, gz;
  cell_coord(x, G.o[0], G.inv_dx, G.nd[0], i, gx);
  cell_coord(y, G.o[1], G.inv_dx, G.nd[1], j, gy);
  cell_coord(z, G.o[2], G.inv_dx, G.nd[2], k, gz);
  const float4* rec = grid_record(G, i, j, k);
  if (rec_out) *rec_out = rec;
  const float4 q0 = rec[0], q1 = rec[1], q2 = rec[2], q3 = rec[3], q4 = rec[4], q5 = rec[5];
  // corners (dz, dy, dx): 000 = q0.xyz, 001 = q0.w q1.xy, 010 = q1.zw q2.x,
  // 011 = q2.yzw, 100 = q3.xyz, 101 = q3.w q4.xy, 110 = q4.zw q5.x, 111 = q5.yzw;
  // the dx = 1 corners hold the x-differences
  auto lx = [&](float ax, float ay, float az, float dx_, float dy_, float dz_) {
    return make_float3(fmaf(gx, dx_, ax), fmaf(gx, dy_, ay), fmaf(gx, dz_, az));
  };
  auto l3 = [](float t, float3 a, float3 b) {
    return make_float3(fmaf(t, b.x - a.x, a.x), fmaf(t, b.y - a.y, a.y), fmaf(t, b.z - a.z, a.z));
  };
  const float3 e00 = lx(q0.x, q0.y, q0.z, q0.w, q1.x, q1.y);
  const float3 e01 = lx(q1.z, q1.w, q2.x, q2.y, q2.z, q2.w);
  const float3 e10 = lx(q3.x, q3.y, q3.z, q3.w, q4.x, q4.y);
  const float3 e11 = lx(q4.z, q4.w, q5.x, q5.y, q5.z, q5.w);
  const float3 e0 = l3(gy, e00, e01), e1 = l3(gy, e10, e11);
  const float3 e = l3(gz, e0, e1);
  return make_double3(qm * e.x, qm * e.y, qm * e.z);
}

// Acceleration bounds for the rest of a step of length t_rem, from the record
// of the particle's position: local ones if the particle cannot leave its
// cell neighbourhood (displacement below one cell with a 2^-10 margin), else
// the global bound.
__device__ __forceinline__ void accel_bound_at(const GridView& G, const float4* rec, float speed, float t_rem,
                                               float& a_abs, float& da) {
  const float D = fmaf(0.5f * G.a_glob * t_rem, t_rem, speed * t_rem);
  if (!(D < G.dx * (1.0f - 0x1p-10f))) {
    a_abs = G.a_glob;
    da = 2.0f * G.a_glob;
    return;
  }
  const float4 m = rec[6];
  a_abs = G.qm_abs * m.x;
  da = G.qm_abs * m.y;
}

}  // namespace pcmcc
