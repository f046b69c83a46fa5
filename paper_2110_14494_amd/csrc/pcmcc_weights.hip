// Super-particle weight update (arXiv:2110.14494 Sec. 2.1.2).
//
// Desired weight of cell c: omega_c = n_e dV / N_ppc with n_e dV the
// electrons the CIC mapping puts on the cell (Sec. 2.1.3), at least 1.
// Particles with w < (2/3) omega_c are merge candidates, those with
// w > (3/2) omega_c are split.  Candidates of a cell are ordered by energy
// (|v|^2 rounded to single precision), ties by id, and consecutive ones are
// paired; the merged particle keeps the position, velocity and id of one of
// the pair, the first with probability w_a / (w_a + w_b) (weight-update draw
// of the smaller id, purpose 3, counter (id, update index, 0)), and carries
// w_a + w_b.  A split halves the weight and adds a copy whose id is the
// (second, third) words of the particle's weight-update draw.
//
// Schedule: classify (blocks of 2048 particles read in order; candidates
// appended with one atomic per block, each with its id and its (cell,
// energy) key), two stable radix sorts of the candidates (by id, then by
// cell and energy; rocPRIM), run starts of the cells by a max-scan, pairing
// (one thread per candidate position), and an exclusive scan of the output
// counts (0 removed, 1 kept, 2 split) that places every particle and copy in
// the other particle buffer.  All the decisions are integer or taken in the
// same precision as the definition above, so the result is the same set of
// particles for any schedule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>  // rocPRIM's headers use memset without including it
#include <rocprim/rocprim.hpp>

#include "pcmcc_device.hpp"
#include "pcmcc_internal.hpp"
#include "pcmcc_mover.hpp"

namespace pcmcc {

enum WeightClass : uint8_t { WC_KEEP = 0, WC_MERGE = 1, WC_SPLIT = 2, WC_REMOVED = 3 };
constexpr uint32_t TAG_WEIGHT = 3;

// Cell containing a particle: floor((x - x0)/dx) per axis, clamped.
__device__ __forceinline__ int wt_axis(float x, double o, double inv_dx, int n) {
#pragma clang fp contract(off)
  const int i = (int)floor(((double)x - o) * inv_dx);
  return min(max(i, 0), n - 1);
}

__device__ __forceinline__ uint64_t wt_cell(const WeightGeom& g, float x, float y, float z) {
  return ((uint64_t)wt_axis(z, g.z0, g.inv_dx, g.nz) * g.ny + wt_axis(y, g.y0, g.inv_dx, g.ny)) * g.nx +
         wt_axis(x, g.x0, g.inv_dx, g.nx);
}

// Energy ordering key: |v|^2 in double from the single-precision components,
// summed as (vx^2 + vy^2) + vz^2, rounded to single precision.
__device__ __forceinline__ uint32_t wt_energy_bits(float vx, float vy, float vz) {
#pragma clang fp contract(off)
  const double a = (double)vx, b = (double)vy, c = (double)vz;
  return __float_as_uint((float)((a * a + b * b) + c * c));
}

constexpr int kWtBlock = 256;
constexpr int kWtPer = 8;                       // particles per thread and tile
constexpr int kWtTile = kWtBlock * kWtPer;

// Classification of tile [base, base + kWtTile): particle base + j kWtBlock
// + threadIdx.x for j < kWtPer (coalesced).  The merge candidates of a tile
// take consecutive slots reserved with one atomic; slot k holds the
// particle's index, id and (cell << 32 | energy bits) key.
__global__ __launch_bounds__(kWtBlock) void k_wt_classify(Soa cur, uint64_t n, WeightGeom g,
                                                           const int64_t* __restrict__ rho, uint8_t* __restrict__ cls,
                                                           uint32_t* __restrict__ cand_idx,
                                                           uint64_t* __restrict__ cand_id,
                                                           uint64_t* __restrict__ cand_key,
                                                           unsigned long long* n_cand) {
#pragma clang fp contract(off)
  __shared__ uint32_t s_wave[kWtBlock / 64];
  __shared__ unsigned long long s_base;
  const uint32_t wave = threadIdx.x / 64;
  for (uint64_t base = (uint64_t)blockIdx.x * kWtTile; base < n; base += (uint64_t)gridDim.x * kWtTile) {
    uint32_t merge = 0;  // bit j: item j is a merge candidate
    uint64_t cell[kWtPer];
#pragma unroll
    for (int j = 0; j < kWtPer; ++j) {
      const uint64_t i = base + (uint64_t)j * kWtBlock + threadIdx.x;
      cell[j] = 0;
      if (i < n) {
        cell[j] = wt_cell(g, cur.x[i], cur.y[i], cur.z[i]);
        const double omega = fmax(ldexp((double)rho[cell[j]], -32) / g.n_ppc, 1.0);
        const double w = (double)cur.w[i];
        uint8_t c = WC_KEEP;
        if (w < (2.0 / 3.0) * omega) {
          c = WC_MERGE;
          merge |= 1u << j;
        } else if (w > 1.5 * omega) {
          c = WC_SPLIT;
        }
        cls[i] = c;
      }
    }
    // block-wide exclusive prefix of the candidate counts
    const uint32_t mine = (uint32_t)__popc(merge);
    uint32_t incl = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t o = __shfl_up(incl, d, 64);
      if ((int)lane_id() >= d) incl += o;
    }
    if (lane_id() == 63) s_wave[wave] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWtBlock / 64; ++w) {
      const uint32_t t = s_wave[w];
      before += (uint32_t)w < wave ? t : 0u;
      total += t;
    }
    if (threadIdx.x == 0) s_base = total ? atomicAdd(n_cand, (unsigned long long)total) : 0ull;
    __syncthreads();
    uint64_t k = s_base + before + (incl - mine);
#pragma unroll
    for (int j = 0; j < kWtPer; ++j) {
      if (merge & (1u << j)) {
        const uint64_t i = base + (uint64_t)j * kWtBlock + threadIdx.x;
        cand_idx[k] = (uint32_t)i;
        cand_id[k] = cur.id[i];
        cand_key[k] = (cell[j] << 32) | wt_energy_bits(cur.vx[i], cur.vy[i], cur.vz[i]);
        ++k;
      }
    }
    __syncthreads();  // s_wave and s_base are reused by the next tile
  }
}

// After the sort by id (values: candidate slots), the slots' particle
// indices and (cell, energy) keys in that order.
__global__ void k_wt_key2(const uint32_t* __restrict__ slot, uint64_t m, const uint32_t* __restrict__ cand_idx,
                          const uint64_t* __restrict__ cand_key, uint32_t* __restrict__ idx,
                          uint64_t* __restrict__ key2) {
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t sk = slot[k];
    idx[k] = cand_idx[sk];
    key2[k] = cand_key[sk];
  }
}

__global__ void k_wt_iota(uint32_t* __restrict__ a, uint64_t m) {
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (uint64_t)gridDim.x * blockDim.x)
    a[k] = (uint32_t)k;
}

__global__ void k_wt_heads(const uint64_t* __restrict__ key2, uint64_t m, uint32_t* __restrict__ head) {
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (uint64_t)gridDim.x * blockDim.x)
    head[k] = (k == 0 || (key2[k] >> 32) != (key2[k - 1] >> 32)) ? (uint32_t)k : 0u;
}

__global__ void k_wt_pair(const uint64_t* __restrict__ key2, const uint32_t* __restrict__ idx,
                          const uint32_t* __restrict__ run_start, uint64_t m, Soa cur, uint8_t* __restrict__ cls,
                          Key key, uint32_t update_index, unsigned long long* n_pairs) {
  unsigned long long pairs = 0;  // the wave's pairs, counted by lane 0
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < m; base += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = base + threadIdx.x;
    bool paired = false;
    if (k < m && ((k - run_start[k]) & 1) == 0 && k + 1 < m && (key2[k + 1] >> 32) == (key2[k] >> 32)) {
      const uint32_t a = idx[k], b = idx[k + 1];
      const float wa = cur.w[a], wb = cur.w[b];
      const uint64_t ia = cur.id[a], ib = cur.id[b];
      const uint4 d = draw(key, ia < ib ? ia : ib, update_index, 0, TAG_WEIGHT);
      const double pa = (double)wa / ((double)wa + (double)wb);
      const float wsum = wa + wb;
      if ((double)unif(d.x) < pa) {
        cur.w[a] = wsum;
        cls[b] = WC_REMOVED;
      } else {
        cur.w[b] = wsum;
        cls[a] = WC_REMOVED;
      }
      paired = true;
    }
    pairs += (unsigned long long)__popcll(__ballot(paired));
  }
  if (lane_id() == 0 && pairs) atomicAdd(n_pairs, pairs);
}

__global__ void k_wt_counts(const uint8_t* __restrict__ cls, uint64_t n, uint32_t* __restrict__ cnt) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint8_t c = cls[i];
    cnt[i] = c == WC_REMOVED ? 0u : (c == WC_SPLIT ? 2u : 1u);
  }
}

__global__ void k_wt_emit(Soa cur, Soa out, uint64_t n, const uint8_t* __restrict__ cls,
                          const uint32_t* __restrict__ pos, Key key, uint32_t update_index) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint8_t c = cls[i];
    if (c == WC_REMOVED) continue;
    PState p;
    load_p(cur, i, p);
    const uint64_t o = pos[i];
    if (c == WC_SPLIT) {
      p.w = 0.5f * p.w;
      const uint4 d = draw(key, p.id, update_index, 0, TAG_WEIGHT);
      PState q = p;
      q.id = (uint64_t)d.y | ((uint64_t)d.z << 32);
      store_p(out, o + 1, q);
    }
    store_p(out, o, p);
  }
}

// ---------------------------------------------------------------------------

static unsigned blocks_for(uint64_t n) {
  const uint64_t b = (n + 255) / 256;
  return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

hipError_t weight_temp_bytes(uint64_t n, size_t* bytes) {
  size_t a = 0, b = 0, c = 0;
  hipError_t e = rocprim::radix_sort_pairs(nullptr, a, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                           (const uint32_t*)nullptr, (uint32_t*)nullptr, (size_t)n, 0, 64);
  if (e != hipSuccess) return e;
  e = rocprim::inclusive_scan(nullptr, b, (const uint32_t*)nullptr, (uint32_t*)nullptr, (size_t)n,
                              rocprim::maximum<uint32_t>());
  if (e != hipSuccess) return e;
  e = rocprim::exclusive_scan(nullptr, c, (const uint32_t*)nullptr, (uint32_t*)nullptr, 0u, (size_t)n,
                              rocprim::plus<uint32_t>());
  if (e != hipSuccess) return e;
  *bytes = std::max(a, std::max(b, c));
  return hipSuccess;
}

hipError_t launch_weight_update(const Soa& cur, const Soa& out, uint64_t n, const WeightGeom& g, const int64_t* rho,
                                Key key, uint32_t update_index, const WeightWork& W, uint64_t* n_out,
                                uint64_t* pairs_out, uint64_t* splits_out, hipStream_t stream) {
  hipError_t e = hipMemsetAsync(W.counters, 0, 4 * sizeof(unsigned long long), stream);
  if (e != hipSuccess) return e;
  const uint64_t tiles = (n + kWtTile - 1) / kWtTile;
  hipLaunchKernelGGL(k_wt_classify, dim3((unsigned)(tiles < 8192 ? tiles : 8192)), dim3(kWtBlock), 0, stream, cur, n,
                     g, rho, W.cls, W.idx0, W.key0, W.key2, W.counters);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  unsigned long long m = 0;
  if ((e = hipMemcpyAsync(&m, W.counters, sizeof(m), hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
  size_t tb = W.temp_bytes;
  if (m > 1) {
    // candidates by id (values: slots), then (stable) by cell and energy
    hipLaunchKernelGGL(k_wt_iota, dim3(blocks_for(m)), dim3(256), 0, stream, W.pos, (uint64_t)m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = rocprim::radix_sort_pairs(W.temp, tb, W.key0, W.key1, W.pos, W.cnt, (size_t)m, 0, 64, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wt_key2, dim3(blocks_for(m)), dim3(256), 0, stream, W.cnt, (uint64_t)m, W.idx0, W.key2,
                       W.idx1, W.key0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    tb = W.temp_bytes;
    e = rocprim::radix_sort_pairs(W.temp, tb, W.key0, W.key1, W.idx1, W.idx0, (size_t)m, 0, 32 + g.cell_bits,
                                  stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wt_heads, dim3(blocks_for(m)), dim3(256), 0, stream, W.key1, (uint64_t)m, W.pos);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    tb = W.temp_bytes;
    e = rocprim::inclusive_scan(W.temp, tb, W.pos, W.idx1, (size_t)m, rocprim::maximum<uint32_t>(), stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wt_pair, dim3(blocks_for(m)), dim3(256), 0, stream, W.key1, W.idx0, W.idx1, (uint64_t)m,
                       cur, W.cls, key, update_index, W.counters + 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_wt_counts, dim3(blocks_for(n)), dim3(256), 0, stream, W.cls, n, W.cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  tb = W.temp_bytes;
  e = rocprim::exclusive_scan(W.temp, tb, W.cnt, W.pos, 0u, (size_t)n, rocprim::plus<uint32_t>(), stream);
  if (e != hipSuccess) return e;
  uint32_t tail[2] = {0, 0};
  unsigned long long pairs = 0;
  if ((e = hipMemcpyAsync(&tail[0], W.pos + (n - 1), 4, hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(&tail[1], W.cnt + (n - 1), 4, hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(&pairs, W.counters + 1, sizeof(pairs), hipMemcpyDeviceToHost, stream)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
  const uint64_t total = (uint64_t)tail[0] + tail[1];
  *n_out = total;
  *pairs_out = pairs;
  *splits_out = total - (n - pairs);  // n - pairs kept or split, each split adds one
  if (total > g.capacity) return hipSuccess;  // the caller reports the capacity; nothing written
  hipLaunchKernelGGL(k_wt_emit, dim3(blocks_for(n)), dim3(256), 0, stream, cur, out, n, W.cls, W.pos, key,
                     update_index);
  return hipGetLastError();
}

}  // namespace pcmcc
