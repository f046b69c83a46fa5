// Charge deposit (arXiv:2110.14494 Sec. 2.1.3): trilinear weighting of each
// particle's charge to the 8 nearest cell centres.
//
// Fixed-point rule (both paths): weights in double precision without
// contraction, each corner rounded to 2^-32 fixed point and the last corner
// taking the remainder, so the integer sum is independent of order and
// exactly conserves round(w 2^32) per particle.
//
// Range: a particle's charge must fit one corner (0 <= w < 2^31) and every
// cell sum must stay within int64 (2^31 electrons).  Every addition, in LDS
// and in global memory, checks its own signed overflow from the value the
// atomic returns; as the corner charges are non-negative (the remainder
// corner can be a few units below zero) a cell whose sum leaves the range
// overflows in one of them.  Either case raises range_err and drops nothing
// else: the caller reports the error and rho is then unspecified.
//
// Two schedules of the same sums:
//  * direct: one thread per particle, 8 global int64 atomics;
//  * binned (large inputs): the grid is cut into tiles of 8^3 cells, the
//    particles are counted per tile (per-block LDS hash of tiles, one global
//    atomic per block and tile), scattered into tile order, and then summed
//    per tile in an LDS int64 buffer of 9^3 cells (the tile plus its upper
//    neighbour layer) that is flushed once per block and tile.  Global
//    atomics drop from 8 per particle to about 8 per thousand particles in
//    dense regions: device-wide int64 atomics are executed at the memory
//    side and were the limit of the direct schedule.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pcmcc_internal.hpp"

namespace pcmcc {

constexpr int kTile = 8;                                // cells per tile edge
constexpr int kTileBuf = kTile + 1;                     // with the upper neighbour layer
constexpr int kTileCells = kTileBuf * kTileBuf * kTileBuf;
constexpr int kBinRange = 4096;                         // particles per block, count and scatter
constexpr int kBinHash = 4096;                          // hash entries per block (>= distinct tiles)
constexpr int kAccRange = 32768;                        // sorted particles per block, accumulation
constexpr uint32_t kEmpty = 0xFFFFFFFFu;

// Lower and upper centre index of one axis, clamped to the grid, and the
// weights (1 - f, f).
__device__ __forceinline__ void dep_axis(double p, double o, double inv_dx, int n, int ic[2], double W[2]) {
#pragma clang fp contract(off)
  double u = (p - o) * inv_dx - 0.5;
  u = fmin(fmax(u, -1.0), (double)n);
  const double fl = floor(u);
  const double f = u - fl;
  const int i = (int)fl;
  ic[0] = min(max(i, 0), n - 1);
  ic[1] = min(max(i + 1, 0), n - 1);
  W[0] = 1.0 - f;
  W[1] = f;
}

// Cells (lower/upper per axis) and fixed-point charges of the 8 corners in
// (dz, dy, dx) order.  A weight outside [0, 2^31) raises range_err and
// deposits nothing.
__device__ __forceinline__ void corner_charges(const DepositGeom& g, float x, float y, float z, float w, int ic[3][2],
                                               long long q[8]) {
#pragma clang fp contract(off)
  double W[3][2];
  dep_axis((double)x, g.x0, g.inv_dx, g.nx, ic[0], W[0]);
  dep_axis((double)y, g.y0, g.inv_dx, g.ny, ic[1], W[1]);
  dep_axis((double)z, g.z0, g.inv_dx, g.nz, ic[2], W[2]);
  double wd = (double)w;
  if (!(wd >= 0.0 && wd < 2147483648.0)) {
    atomicOr(g.range_err, 1u);
    wd = 0.0;
  }
  const long long qw = __double2ll_rn(wd * 4294967296.0);
  long long given = 0;
#pragma unroll
  for (int c = 0; c < 7; ++c) {
    const int dz = c >> 2, dy = (c >> 1) & 1, dx = c & 1;
    const double frac = (W[0][dx] * W[1][dy]) * W[2][dz];
    q[c] = __double2ll_rn((wd * frac) * 4294967296.0);
    given += q[c];
  }
  q[7] = qw - given;
}

__device__ __forceinline__ size_t cell_index(const DepositGeom& g, int i, int j, int k) {
  return ((size_t)k * g.ny + j) * g.nx + i;
}

// rho[i] += v (int64, global or LDS), raising *err on signed overflow.
__device__ __forceinline__ void add_checked(unsigned long long* a, long long v, unsigned* err) {
  const long long old = (long long)atomicAdd(a, (unsigned long long)v);
  const long long res = (long long)((unsigned long long)old + (unsigned long long)v);
  if (((old ^ res) & (v ^ res)) < 0) atomicOr(err, 1u);
}

__global__ void k_deposit(const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
                          const float* __restrict__ w, const int64_t* n_dev, DepositGeom g,
                          unsigned long long* rho) {
  const uint64_t n = (uint64_t)*n_dev;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (uint64_t)gridDim.x * blockDim.x) {
    int ic[3][2];
    long long q[8];
    corner_charges(g, x[p], y[p], z[p], w[p], ic, q);
#pragma unroll
    for (int c = 0; c < 8; ++c)
      add_checked(&rho[cell_index(g, ic[0][c & 1], ic[1][(c >> 1) & 1], ic[2][c >> 2])], q[c], g.range_err);
  }
}

// ---------------------------------------------------------------------------
// Binned schedule.

struct TileGeom {
  DepositGeom g;
  int tx, ty, tz;  // tiles per axis
};

// Tile of a particle: the one holding its lower (clamped) centre indices.
__device__ __forceinline__ uint32_t tile_of(const TileGeom& T, float x, float y, float z) {
  int ic[2];
  double W[2];
  dep_axis((double)x, T.g.x0, T.g.inv_dx, T.g.nx, ic, W);
  const int i = ic[0] / kTile;
  dep_axis((double)y, T.g.y0, T.g.inv_dx, T.g.ny, ic, W);
  const int j = ic[0] / kTile;
  dep_axis((double)z, T.g.z0, T.g.inv_dx, T.g.nz, ic, W);
  const int k = ic[0] / kTile;
  return ((uint32_t)k * T.ty + j) * T.tx + i;
}

__device__ __forceinline__ uint32_t tile_hash(uint32_t t) { return (t * 2654435761u) >> 20; }  // 12 bits

// Slot of tile t in the block's table, inserting it if new.  The table has
// at least as many entries as the block has particles, so it never fills.
__device__ __forceinline__ int hash_insert(uint32_t* keys, uint32_t t) {
  uint32_t h = tile_hash(t);
  for (;;) {
    const uint32_t old = atomicCAS(&keys[h], kEmpty, t);
    if (old == kEmpty || old == t) return (int)h;
    h = (h + 1) & (kBinHash - 1);
  }
}

// Slot of tile t, which the counting pass inserted (bounded probe; -1 only
// if it is absent, which the identical tile computation of both passes rules
// out).
__device__ __forceinline__ int hash_find(const uint32_t* keys, uint32_t t) {
  uint32_t h = tile_hash(t);
  for (int probe = 0; probe < kBinHash; ++probe) {
    if (keys[h] == t) return (int)h;
    h = (h + 1) & (kBinHash - 1);
  }
  return -1;
}

// Pass 1: particles per tile.  Block b covers particles
// [b kBinRange, (b+1) kBinRange) and records, per tile, its offset within the
// tile (the value of the tile's counter when it added its count).
__global__ __launch_bounds__(256) void k_dep_count(const float* __restrict__ x, const float* __restrict__ y,
                                                    const float* __restrict__ z, uint64_t n, TileGeom T,
                                                    uint32_t* __restrict__ tile_count, uint2* __restrict__ dump) {
  __shared__ uint32_t keys[kBinHash];
  __shared__ uint32_t cnt[kBinHash];
  for (int e = threadIdx.x; e < kBinHash; e += blockDim.x) {
    keys[e] = kEmpty;
    cnt[e] = 0;
  }
  __syncthreads();
  const uint64_t p0 = (uint64_t)blockIdx.x * kBinRange;
  const uint64_t p1 = p0 + kBinRange < n ? p0 + kBinRange : n;
  for (uint64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    const int e = hash_insert(keys, tile_of(T, x[p], y[p], z[p]));
    atomicAdd(&cnt[e], 1u);
  }
  __syncthreads();
  uint2* d = dump + (size_t)blockIdx.x * kBinHash;
  for (int e = threadIdx.x; e < kBinHash; e += blockDim.x) {
    const uint32_t t = keys[e];
    d[e] = t == kEmpty ? make_uint2(kEmpty, 0u) : make_uint2(t, atomicAdd(&tile_count[t], cnt[e]));
  }
}

// Exclusive prefix sum of the tile counts (one block): start[t], and
// start[n_tiles] = total.
__global__ __launch_bounds__(1024) void k_dep_scan(const uint32_t* __restrict__ count, uint32_t n_tiles,
                                                    uint32_t* __restrict__ start) {
  __shared__ uint32_t part[1024];
  const uint32_t per = (n_tiles + blockDim.x - 1) / blockDim.x;
  const uint32_t a = threadIdx.x * per, b = min(a + per, n_tiles);
  uint32_t s = 0;
  for (uint32_t t = a; t < b; ++t) s += count[t];
  part[threadIdx.x] = s;
  __syncthreads();
  for (uint32_t off = 1; off < blockDim.x; off <<= 1) {
    const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - s;
  for (uint32_t t = a; t < b; ++t) {
    start[t] = run;
    run += count[t];
  }
  if (threadIdx.x == blockDim.x - 1) start[n_tiles] = part[threadIdx.x];
}

// Pass 2: scatter (x, y, z, w) into tile order.
__global__ __launch_bounds__(256) void k_dep_scatter(const float* __restrict__ x, const float* __restrict__ y,
                                                      const float* __restrict__ z, const float* __restrict__ w,
                                                      uint64_t n, TileGeom T, const uint32_t* __restrict__ start,
                                                      const uint2* __restrict__ dump, float4* __restrict__ sorted) {
  __shared__ uint32_t keys[kBinHash];
  __shared__ uint32_t next[kBinHash];
  const uint2* d = dump + (size_t)blockIdx.x * kBinHash;
  for (int e = threadIdx.x; e < kBinHash; e += blockDim.x) {
    const uint2 v = d[e];
    keys[e] = v.x;
    next[e] = v.x == kEmpty ? 0u : start[v.x] + v.y;
  }
  __syncthreads();
  const uint64_t p0 = (uint64_t)blockIdx.x * kBinRange;
  const uint64_t p1 = p0 + kBinRange < n ? p0 + kBinRange : n;
  for (uint64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    const float px = x[p], py = y[p], pz = z[p];
    const int e = hash_find(keys, tile_of(T, px, py, pz));
    if (e >= 0) sorted[atomicAdd(&next[e], 1u)] = make_float4(px, py, pz, w[p]);
  }
}

// Particle sort by tile (the step loop's start order): the count and scan
// passes above, then every array of a particle moved to its tile's range.
// Within a tile the order follows the atomics and is not fixed.
__global__ __launch_bounds__(256) void k_sort_scatter(Soa src, uint64_t n, TileGeom T,
                                                       const uint32_t* __restrict__ start,
                                                       const uint2* __restrict__ dump, Soa dst) {
  __shared__ uint32_t keys[kBinHash];
  __shared__ uint32_t next[kBinHash];
  const uint2* d = dump + (size_t)blockIdx.x * kBinHash;
  for (int e = threadIdx.x; e < kBinHash; e += blockDim.x) {
    const uint2 v = d[e];
    keys[e] = v.x;
    next[e] = v.x == kEmpty ? 0u : start[v.x] + v.y;
  }
  __syncthreads();
  const uint64_t p0 = (uint64_t)blockIdx.x * kBinRange;
  const uint64_t p1 = p0 + kBinRange < n ? p0 + kBinRange : n;
  for (uint64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    const float px = src.x[p], py = src.y[p], pz = src.z[p];
    const int e = hash_find(keys, tile_of(T, px, py, pz));
    if (e < 0) continue;  // never: both passes compute the same tile
    const uint32_t q = atomicAdd(&next[e], 1u);
    dst.x[q] = px;
    dst.y[q] = py;
    dst.z[q] = pz;
    dst.vx[q] = src.vx[p];
    dst.vy[q] = src.vy[p];
    dst.vz[q] = src.vz[p];
    dst.w[q] = src.w[p];
    dst.id[q] = src.id[p];
  }
}

// One tile run [cur, e) of sorted particles into the LDS buffer of the tile
// at (oi, oj, ok).  The plain pass adds without overflow checks (it cannot
// overflow while the run carries fewer than 2^31 electrons, which the caller
// checks with the returned weight sum) and sends a corner outside the buffer
// to rho directly; the checked pass repeats only the LDS part.
template <bool kChecked>
__device__ __forceinline__ double accum_run(const float4* __restrict__ sorted, uint64_t cur, uint64_t e,
                                            const TileGeom& T, int oi, int oj, int ok, unsigned long long* acc,
                                            unsigned long long* rho) {
  double wsum = 0.0;
  for (uint64_t p = cur + threadIdx.x; p < e; p += blockDim.x) {
    const float4 v = sorted[p];
    int ic[3][2];
    long long q[8];
    corner_charges(T.g, v.x, v.y, v.z, v.w, ic, q);
    if (v.w >= 0.0f) wsum += (double)v.w;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int ci = ic[0][c & 1], cj = ic[1][(c >> 1) & 1], ck = ic[2][c >> 2];
      const int li = ci - oi, lj = cj - oj, lk = ck - ok;
      if ((unsigned)li < (unsigned)kTileBuf && (unsigned)lj < (unsigned)kTileBuf && (unsigned)lk < (unsigned)kTileBuf) {
        unsigned long long* a = &acc[(lk * kTileBuf + lj) * kTileBuf + li];
        if (kChecked)
          add_checked(a, q[c], T.g.range_err);
        else
          atomicAdd(a, (unsigned long long)q[c]);
      } else if (!kChecked) {  // a particle outside its tile's buffer: never expected, kept exact
        add_checked(&rho[cell_index(T.g, ci, cj, ck)], q[c], T.g.range_err);
      }
    }
  }
  return wsum;
}

// A tile run carrying this many electrons or more is summed again with
// overflow checks (2^31 electrons is the int64 limit of one cell).
constexpr double kAccGuard = 1073741824.0;

// Pass 3: per-tile sums.  Block b covers sorted particles
// [b kAccRange, (b+1) kAccRange), one tile at a time.
__global__ __launch_bounds__(256) void k_dep_accum(const float4* __restrict__ sorted, uint64_t n, TileGeom T,
                                                    const uint32_t* __restrict__ start, unsigned long long* rho) {
  __shared__ unsigned long long acc[kTileCells];
  __shared__ uint32_t s_tile;
  __shared__ uint64_t s_end;
  __shared__ double s_wsum;
  for (int c = threadIdx.x; c < kTileCells; c += blockDim.x) acc[c] = 0;
  uint64_t cur = (uint64_t)blockIdx.x * kAccRange;
  const uint64_t end = cur + kAccRange < n ? cur + kAccRange : n;
  while (cur < end) {
    if (threadIdx.x == 0) {
      const float4 q = sorted[cur];
      const uint32_t t = tile_of(T, q.x, q.y, q.z);
      s_tile = t;
      // the run of tile t ends at start[t + 1] (at least one particle on)
      uint64_t te = start[t + 1];
      te = te > cur ? te : cur + 1;
      s_end = te < end ? te : end;
      s_wsum = 0.0;
    }
    __syncthreads();
    const uint32_t t = s_tile;
    const uint64_t e = s_end;
    const int oi = (int)(t % T.tx) * kTile;
    const int oj = (int)((t / T.tx) % T.ty) * kTile;
    const int ok = (int)(t / ((uint32_t)T.tx * T.ty)) * kTile;
    const double ws = accum_run<false>(sorted, cur, e, T, oi, oj, ok, acc, rho);
    if (ws > 0.0) atomicAdd(&s_wsum, ws);
    __syncthreads();
    if (s_wsum >= kAccGuard) {  // block-uniform
      for (int c = threadIdx.x; c < kTileCells; c += blockDim.x) acc[c] = 0;
      __syncthreads();
      accum_run<true>(sorted, cur, e, T, oi, oj, ok, acc, rho);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < kTileCells; c += blockDim.x) {
      const unsigned long long v = acc[c];
      if (v != 0) {
        const int ci = oi + c % kTileBuf, cj = oj + (c / kTileBuf) % kTileBuf, ck = ok + c / (kTileBuf * kTileBuf);
        if (ci < T.g.nx && cj < T.g.ny && ck < T.g.nz)
          add_checked(&rho[cell_index(T.g, ci, cj, ck)], (long long)v, T.g.range_err);
        acc[c] = 0;
      }
    }
    __syncthreads();
    cur = e;
  }
}

// ---------------------------------------------------------------------------

// Sets n words to v (a kernel rather than a memset node, so that the deposit
// may be recorded into a graph).
__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, v);
  return hipGetLastError();
}

hipError_t launch_deposit(const float* x, const float* y, const float* z, const float* w, const int64_t* n_dev,
                          const DepositGeom& g, int64_t* rho, hipStream_t stream) {
  hipLaunchKernelGGL(k_deposit, dim3(4096), dim3(256), 0, stream, x, y, z, w, n_dev, g,
                     (unsigned long long*)rho);
  return hipGetLastError();
}

DepositNeeds deposit_needs(const DepositGeom& g, uint64_t n) {
  DepositNeeds d;
  d.binned = n >= kDepositBinnedMin;
  const uint64_t tx = ((uint64_t)g.nx + kTile - 1) / kTile, ty = ((uint64_t)g.ny + kTile - 1) / kTile,
                 tz = ((uint64_t)g.nz + kTile - 1) / kTile;
  d.n_tiles = tx * ty * tz;
  d.dump_entries = ((n + kBinRange - 1) / kBinRange) * kBinHash;
  d.sorted = n;
  return d;
}

hipError_t launch_sort_tiles(const Soa& src, uint64_t n, const DepositGeom& g, const DepositWork& W, const Soa& dst,
                             hipStream_t stream) {
  if (n == 0) return hipSuccess;
  TileGeom T;
  T.g = g;
  T.tx = (g.nx + kTile - 1) / kTile;
  T.ty = (g.ny + kTile - 1) / kTile;
  T.tz = (g.nz + kTile - 1) / kTile;
  const uint32_t n_tiles = (uint32_t)T.tx * T.ty * T.tz;
  hipError_t e = launch_fill_u32(W.tile_count, n_tiles, 0u, stream);
  if (e != hipSuccess) return e;
  const uint64_t nb = (n + kBinRange - 1) / kBinRange;
  hipLaunchKernelGGL(k_dep_count, dim3((unsigned)nb), dim3(256), 0, stream, src.x, src.y, src.z, n, T, W.tile_count,
                     W.dump);
  hipLaunchKernelGGL(k_dep_scan, dim3(1), dim3(1024), 0, stream, W.tile_count, n_tiles, W.tile_start);
  hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)nb), dim3(256), 0, stream, src, n, T, W.tile_start, W.dump, dst);
  return hipGetLastError();
}

hipError_t launch_deposit_binned(const float* x, const float* y, const float* z, const float* w, uint64_t n,
                                 const DepositGeom& g, int64_t* rho, const DepositWork& W, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  TileGeom T;
  T.g = g;
  T.tx = (g.nx + kTile - 1) / kTile;
  T.ty = (g.ny + kTile - 1) / kTile;
  T.tz = (g.nz + kTile - 1) / kTile;
  const uint32_t n_tiles = (uint32_t)T.tx * T.ty * T.tz;
  hipError_t e = launch_fill_u32(W.tile_count, n_tiles, 0u, stream);
  if (e != hipSuccess) return e;
  const uint64_t nb = (n + kBinRange - 1) / kBinRange;
  hipLaunchKernelGGL(k_dep_count, dim3((unsigned)nb), dim3(256), 0, stream, x, y, z, n, T, W.tile_count, W.dump);
  hipLaunchKernelGGL(k_dep_scan, dim3(1), dim3(1024), 0, stream, W.tile_count, n_tiles, W.tile_start);
  hipLaunchKernelGGL(k_dep_scatter, dim3((unsigned)nb), dim3(256), 0, stream, x, y, z, w, n, T, W.tile_start, W.dump,
                     W.sorted);
  const uint64_t na = (n + kAccRange - 1) / kAccRange;
  hipLaunchKernelGGL(k_dep_accum, dim3((unsigned)na), dim3(256), 0, stream, W.sorted, n, T, W.tile_start,
                     (unsigned long long*)rho);
  return hipGetLastError();
}

}  // namespace pcmcc
