// HIP kernels of the PIC-MCC electron update (gfx950, wave64).
//
// Method: arXiv:2110.14494 Sec. 2.1.  Per time step every electron is
// advanced with velocity Verlet (Sec. 2.1.1 eq. (1)-(2)) through flight
// segments that end in real or null collisions (null-collision method,
// Sec. 2.1.1) against tabulated rates (Sec. 2.1.5); ionization appends a
// newborn electron that is advanced from its birth time in the same step,
// attachment removes the electron; the charge is then mapped to the grid by
// trilinear weighting (Sec. 2.1.3).
//
// Layout: particles are structure-of-arrays single precision (x, y, z, vx,
// vy, vz, w) plus a 64-bit id.  Waves take electrons in chunks (512
// consecutive slots by default, shrinking towards the end of a phase) from a
// grid-wide counter and keep every lane busy with
// the segment-pipelined mover (pcmcc_flight.hpp).  The survivors of a chunk
// stay within that chunk's slot range of the next buffer (ping-pong, so a
// step that would overflow the capacity leaves the previous state intact),
// written to its front in the order they finish; the rest of the range is
// holes that the step's newborns fill first, and any holes left over are
// filled from the tail.  Only newborns and holes take global atomics, one
// per wave and batch.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "pcmcc_device.hpp"
#include "pcmcc_internal.hpp"
#include "pcmcc_flight.hpp"
#include "pcmcc_mover.hpp"

namespace cg = cooperative_groups;

namespace pcmcc {

// ---------------------------------------------------------------------------
// Electron sources and destinations of the two phases of a step.

// Phase 1 source: the current buffer, every electron from t = 0.
struct SoaSource {
  KArg<Soa> sk;
  __device__ __forceinline__ uint32_t hint(uint64_t) const { return 0u; }
  __device__ __forceinline__ void load(uint64_t i, Flight& f, uint32_t) const {
    PState p;
    load_p(sk.get(), i, p);
    flight_start(f, p, 0.0, (uint32_t)i);
  }
};

// Phase 2 source: a newborn queue, each electron from its birth time.
struct PendSource {
  KArg<PendSoa> sk;
  __device__ __forceinline__ uint32_t hint(uint64_t) const { return 0u; }
  __device__ __forceinline__ void load(uint64_t i, Flight& f, uint32_t) const {
    PState p;
    float tb;
    load_pend(sk.get(), i, p, tb);
    flight_start(f, p, (double)tb, (uint32_t)i);
  }
};

// Phase 1 destination: a survivor keeps its slot in the next buffer; a
// removed electron leaves a hole there (hole slots are staged per wave).
// A negative ion where an electron was attached (self-consistent step only).
__device__ __forceinline__ void record_attachment(const EventSink& ev, const Flight& f) {
  const uint64_t es = wave_reserve(&ev.n[1]);
  if (es < ev.cap) {
    ev.ax[es] = (float)f.x;
    ev.ay[es] = (float)f.y;
    ev.az[es] = (float)f.z;
    ev.aw[es] = f.w;
  } else {
    atomicOr(ev.overflow, OVF_CAPACITY);
  }
}

// Phase 1 destination: the survivors of a chunk of slots the wave took are
// written to the front of that chunk's range in the next buffer, in the
// order they finish; once every electron of the chunk has finished, the rest
// of its range is a run of holes (staged per wave).  The chunks a wave has
// open are kept in its ring in LDS; an electron's tag is its chunk's ring
// entry.  Writing each chunk's survivors consecutively keeps a few partly
// written lines per chunk open in the cache instead of one per survivor.
struct ChunkRing {
  static constexpr uint32_t kR = 64;  // more than the 64 lanes can keep open, plus the chunk being loaded
  uint64_t base[kR];
  uint32_t size[kR], cursor[kR], remaining[kR];
  uint32_t head;
  uint32_t pad;
  __device__ __forceinline__ void reset() {
    remaining[lane_id()] = 0u;
    if (lane_id() == 0) head = 0u;
  }
};

struct KeepInPlace {
  KArg<GridView> G;
  KArg<Soa> nxt;
  uint32_t* holes;
  unsigned long long* n_holes;
  KArg<EventSink> ev;
  ChunkRing* R;  // the wave's ring (LDS)
  __device__ __forceinline__ bool can_open() const {
    const uint32_t h = __builtin_amdgcn_readfirstlane(R->head);
    return __builtin_amdgcn_readfirstlane(R->remaining[h]) == 0u;
  }
  __device__ __forceinline__ uint32_t open_chunk(uint64_t first, uint32_t size) const {
    const uint32_t h = __builtin_amdgcn_readfirstlane(R->head);
    if (lane_id() == 0) {
      R->base[h] = first;
      R->size[h] = size;
      R->cursor[h] = 0u;
      R->remaining[h] = size;
      R->head = (h + 1u) % ChunkRing::kR;
    }
    return h;
  }
  __device__ __forceinline__ void tag(Flight& f, uint32_t t) const { f.src = t; }
  // Stages the hole slots [first, first + k) of the next buffer.
  __device__ __forceinline__ uint32_t push_holes(WaveStage* L, uint32_t n_staged, uint32_t first, uint32_t k) const {
    uint32_t off = 0;
    while (off < k) {
      if (n_staged == kStage) {
        flush(L, n_staged);
        n_staged = 0;
      }
      const uint32_t take = k - off < kStage - n_staged ? k - off : kStage - n_staged;
      if (lane_id() < take) reinterpret_cast<uint32_t*>(L->s[0])[n_staged + lane_id()] = first + off + lane_id();
      n_staged += take;
      off += take;
    }
    return n_staged;
  }
  __device__ __forceinline__ uint32_t done_all(const Flight& f, bool parked, Cnt& cnt, WaveStage* L,
                                               uint32_t n_staged) const {
    PState p;
    bool alive = false;
    if (parked) {
      if (f.seg == EV_ATTACHED) {
        const EventSink e = ev.get();
        if (e.ax) record_attachment(e, f);
      }
      p = flight_record(f);
      alive = f.seg == EV_DONE;
      if (alive && !inside(G.get(), p)) {
        alive = false;
        cnt.v[C_LOST]++;
      }
    }
    // One round per chunk among the finishing electrons: the survivors take
    // the chunk's next slots, and a chunk whose electrons have all finished
    // hands the rest of its range to the hole list.
    const uint32_t lane = lane_id();
    uint64_t pending = __ballot(parked);
    uint32_t slot = 0;
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const uint32_t r = __builtin_amdgcn_readlane(f.src, leader);
      const uint64_t m_all = __ballot(parked && f.src == r);
      const uint64_t m_alive = __ballot(parked && alive && f.src == r);
      const uint32_t base = __builtin_amdgcn_readfirstlane((uint32_t)R->base[r]);
      const uint32_t cur = __builtin_amdgcn_readfirstlane(R->cursor[r]);
      const uint32_t rem = __builtin_amdgcn_readfirstlane(R->remaining[r]);
      const uint32_t size = __builtin_amdgcn_readfirstlane(R->size[r]);
      if ((m_alive >> lane) & 1) slot = base + cur + rank_in(m_alive);
      const uint32_t cur2 = cur + (uint32_t)__popcll(m_alive);
      const uint32_t rem2 = rem - (uint32_t)__popcll(m_all);
      if (lane == 0) {
        R->cursor[r] = cur2;
        R->remaining[r] = rem2;
      }
      if (rem2 == 0u && cur2 < size) n_staged = push_holes(L, n_staged, base + cur2, size - cur2);
      pending &= ~m_all;
    }
    if (alive) store_p(nxt.get(), slot, p);
    return n_staged;
  }
  __device__ __forceinline__ void flush(WaveStage* L, uint32_t n) const {
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(n_holes, (unsigned long long)n);
    const uint64_t b = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(base >> 32)) << 32) |
                       __builtin_amdgcn_readfirstlane((uint32_t)base);
    const uint32_t l = lane_id();
    if (l < n) holes[b + l] = reinterpret_cast<const uint32_t*>(L->s[0])[l];
  }
};

// Phase 2 destination: a surviving newborn fills the next hole, or appends
// after the current count once the holes are used up (placements are staged
// per wave).
struct PlaceNewborn {
  KArg<GridView> G;
  KArg<Soa> nxt;
  const uint32_t* holes;
  uint64_t n_holes, n_cur, cap;
  unsigned long long* child;
  unsigned* overflow;
  KArg<EventSink> ev;
  __device__ __forceinline__ void place(uint64_t slot, const PState& p) const {
    const uint64_t dst = slot < n_holes ? (uint64_t)holes[slot] : n_cur + (slot - n_holes);
    if (dst < cap)
      store_p(nxt.get(), dst, p);
    else
      atomicOr(overflow, OVF_CAPACITY);
  }
  __device__ __forceinline__ bool can_open() const { return true; }
  __device__ __forceinline__ uint32_t open_chunk(uint64_t, uint32_t) const { return 0u; }
  __device__ __forceinline__ void tag(Flight&, uint32_t) const {}
  __device__ __forceinline__ uint32_t done_all(const Flight& f, bool parked, Cnt& cnt, WaveStage* L,
                                               uint32_t n_staged) const {
    bool staged = false;
    if (parked) {
      if (f.seg == EV_ATTACHED) {
        const EventSink e = ev.get();
        if (e.ax) record_attachment(e, f);
      }
      const PState p = flight_record(f);
      bool alive = f.seg == EV_DONE;
      if (alive && !inside(G.get(), p)) {
        alive = false;
        cnt.v[C_LOST]++;
      }
      if (alive) {
        const uint32_t s = n_staged + rank_in(__ballot(1));
        if (s < kStage) {
          L->s[0][s] = p.x;
          L->s[1][s] = p.y;
          L->s[2][s] = p.z;
          L->s[3][s] = p.vx;
          L->s[4][s] = p.vy;
          L->s[5][s] = p.vz;
          L->s[6][s] = p.w;
          L->sid[s] = p.id;
          staged = true;
        } else {
          place(wave_reserve(child), p);
        }
      }
    }
    return n_staged + (uint32_t)__popcll(__ballot(staged));
  }
  __device__ __forceinline__ void flush(WaveStage* L, uint32_t n) const {
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(child, (unsigned long long)n);
    const uint64_t b = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(base >> 32)) << 32) |
                       __builtin_amdgcn_readfirstlane((uint32_t)base);
    const uint32_t l = lane_id();
    if (l < n) {
      PState p;
      p.x = L->s[0][l];
      p.y = L->s[1][l];
      p.z = L->s[2][l];
      p.vx = L->s[3][l];
      p.vy = L->s[4][l];
      p.vz = L->s[5][l];
      p.w = L->s[6][l];
      p.id = L->sid[l];
      place(b + l, p);
    }
  }
};

// ---------------------------------------------------------------------------
// The step loop.  One cooperative launch runs all n_steps steps; grid-wide
// barriers separate the phases of a step, and every loop bound that decides
// a barrier is read after a barrier, so all blocks take the same path.
// Four waves per SIMD (at most 128 registers a lane): the mover waits on
// one gather per segment, and a fourth wave hides that latency better than
// the registers the compiler would otherwise keep.
template <int REFILL, int ROW>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_pic_steps(PicArgs A) {
  extern __shared__ float smem[];
  cg::grid_group grid = cg::this_grid();
  const Tab T = stage_tables(A.T, A.S, smem);
  WaveStage* L = reinterpret_cast<WaveStage*>(smem + pic_stage_offset_floats(A.T)) + (threadIdx.x >> 6);
  ChunkRing* ring = reinterpret_cast<ChunkRing*>(reinterpret_cast<WaveStage*>(smem + pic_stage_offset_floats(A.T)) +
                                                 (blockDim.x >> 6)) +
                    (threadIdx.x >> 6);
  GridView G = A.G;
  G.a_glob = G.qm_abs * __uint_as_float(*A.emax_bits);
  const auto* ka = (const __attribute__((address_space(4))) PicArgs*)__builtin_amdgcn_kernarg_segment_ptr();
  const GridField F{G, A.S.qm, A.key, &ka->G};
  const unsigned lane = lane_id();
  Ctl* ctl = A.ctl;

  for (int s = 0; s < A.n_steps; ++s) {
    if (ld_acq(&ctl->stop)) break;
    const int sel = __builtin_amdgcn_readfirstlane(ld_acq(&ctl->cur_sel));  // grid-uniform
    const Soa nxt = A.buf[sel ^ 1];
    const KArg<Soa> cur_k{&ka->buf[sel]}, nxt_k{&ka->buf[sel ^ 1]};
    const KArg<GridView> grid_k{&ka->G};
    const KArg<EventSink> ev_k{&ka->ev};
    const KArg<uint32_t> chunk_k{&ka->chunk};
    const uint64_t n_cur = ld_acq(&ctl->n_cur);
    const uint32_t step = A.step0 + (uint32_t)s;
    Cnt cnt;
#pragma unroll
    for (int k = 0; k < NCNT; ++k) cnt.v[k] = 0;

    // Phase 1: every particle of the current buffer, from t = 0.
    {
      const BirthSink sink{{&ka->pend[0]}, &ctl->pend[0], A.pend_cap, &ctl->overflow, 0u, ev_k};
      const SoaSource src{cur_k};
      const KeepInPlace fin{grid_k, nxt_k, A.holes, &ctl->holes, ev_k, ring};
      ring->reset();
      fly_all<REFILL, ROW, true>(n_cur, &ctl->take[0], chunk_k, A.dt, F, T, A.S, step, cnt, sink, nullptr, L, src, fin);
    }
    grid.sync();

    // Phase 2: newborns, one generation at a time.  Survivors fill the holes
    // first, then append after the current count.
    const uint64_t h = ld_acq(&ctl->holes);
    for (int g = 0;; ++g) {
      const uint64_t np_raw = ld_acq(&ctl->pend[g]);
      if (np_raw == 0) break;
      if (g >= kMaxGenerations) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&ctl->overflow, OVF_LIMIT);
        break;
      }
      const uint64_t np = np_raw < A.pend_cap ? np_raw : A.pend_cap;
      const BirthSink sink{{&ka->pend[(g + 1) & 1]}, &ctl->pend[g + 1], A.pend_cap, &ctl->overflow, 0u, ev_k};
      const PendSource src{{&ka->pend[g & 1]}};
      const PlaceNewborn fin{grid_k, nxt_k, A.holes, h, n_cur, A.cap, &ctl->child, &ctl->overflow, ev_k};
      fly_all<REFILL, ROW, true>(np, &ctl->take[g + 1], chunk_k, A.dt, F, T, A.S, step, cnt, sink, nullptr, L, src, fin);
      grid.sync();
    }

    // Phase 3: holes not filled by newborns are filled from the tail.
    const uint64_t nc = ld_acq(&ctl->child);
    if (nc < h) {
      const uint64_t r = h - nc;
      const uint64_t n_new = n_cur - r;
      const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
      const uint64_t nthr = (uint64_t)gridDim.x * blockDim.x;
      for (uint64_t k = tid; k < r; k += nthr) A.flags[k] = 0;
      grid.sync();
      for (uint64_t k = tid; k < r; k += nthr) {
        const uint64_t d = A.holes[nc + k];
        if (d >= n_new) A.flags[d - n_new] = 1;
      }
      grid.sync();
      for (uint64_t k = tid; k < r; k += nthr)
        if (!A.flags[k]) A.donor[atomicAdd(&ctl->donors, 1ull)] = (uint32_t)(n_new + k);
      grid.sync();
      const uint64_t nd = ld_acq(&ctl->donors);
      for (uint64_t k = tid; k < r; k += nthr) {
        const uint64_t d = A.holes[nc + k];
        if (d < n_new) {
          const uint64_t m = atomicAdd(&ctl->fill, 1ull);
          const uint64_t src = m < nd ? A.donor[m] : A.cap;
          if (src < A.cap) {
            PState p;
            load_p(nxt, src, p);
            store_p(nxt, d, p);
          } else {
            atomicOr(&ctl->overflow, OVF_LIMIT);  // inconsistent hole count: never expected
          }
        }
      }
    }
    block_counters(cnt, A.partial);
    grid.sync();

    // Commit (block 0): accept the step, or stop and keep the previous state.
    if (blockIdx.x == 0) {
      __shared__ unsigned long long sums[NCNT];
      if (threadIdx.x < NCNT) sums[threadIdx.x] = 0;
      __syncthreads();
      for (int k = 0; k < NCNT; ++k) {
        unsigned long long acc = 0;
        for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x) acc += A.partial[(size_t)b * NCNT + k];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) atomicAdd(&sums[k], acc);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        const unsigned of = ld_acq(&ctl->overflow);
        if (of) {
          ctl->stop = 1;
          ctl->status = (of & OVF_LIMIT) ? PCMCC_ELIMIT : PCMCC_ECAPACITY;
        } else {
          ctl->particle_steps += n_cur;
          ctl->n_cur = n_cur + nc - h;
          ctl->cur_sel = sel ^ 1;
          ctl->steps_done += 1;
          for (int k = 0; k < NCNT; ++k) ctl->tot[k] += sums[k];
          if (A.n_limit && ctl->n_cur > A.n_limit) {  // weights are due: back to the host
            ctl->stop = 1;
            ctl->status = kStatusWeightsDue;
          }
        }
        ctl->holes = 0;
        ctl->child = 0;
        ctl->donors = 0;
        ctl->fill = 0;
        ctl->overflow = 0;
        for (int g = 0; g <= kMaxGenerations; ++g) {
          ctl->pend[g] = 0;
          ctl->take[g] = 0;
        }
      }
    }
    grid.sync();
  }
}

// Copies the final state back to the caller's arrays if it ended in the
// scratch buffer, and publishes the count.
__global__ void k_finalize(Soa user, Soa scratch, Ctl* ctl, int64_t* n_dev) {
  const uint64_t n = ctl->n_cur;
  if (ctl->cur_sel == 1) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
      PState p;
      load_p(scratch, i, p);
      store_p(user, i, p);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_dev = (int64_t)n;
}

// ---------------------------------------------------------------------------
// Field bounds per cell: largest |E| over the 4x4x4 centres (i-1..i+2 per
// axis, clamped) and the norm of the per-component ranges there; plus the
// global maximum of |E| (as ordered bits of a non-negative float).
// The box maximum and minimum are separable: a block owns kFbTX x kFbTY
// output columns and marches through a range of planes; per input plane it
// stages the tile with its halo (|E| computed once per cell, next plane's
// loads in flight meanwhile), reduces 4-wide along x into LDS, then 4-wide
// along y per output column, and keeps the last four planes' results in
// registers for the z window.  The sums of squares are written as explicit
// fused multiply-adds (z, then x over y), the rounding these bounds have
// always had.
constexpr int kFbTX = 64, kFbTY = 4, kFbThreads = kFbTX * kFbTY;
constexpr int kFbIX = kFbTX + 3, kFbIY = kFbTY + 3, kFbIn = kFbIX * kFbIY;  // input tile: halo -1 .. +2
constexpr int kFbLoads = (kFbIn + kFbThreads - 1) / kFbThreads;
constexpr int kFbXR = kFbIY * kFbTX;  // x-reduced entries per plane

struct Box7 {
  float m, lo0, lo1, lo2, hi0, hi1, hi2;
};
__device__ __forceinline__ Box7 box_empty() { return Box7{0.0f, INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY}; }
__device__ __forceinline__ void box_add(Box7& b, const Box7& o) {
  b.m = fmaxf(b.m, o.m);
  b.lo0 = fminf(b.lo0, o.lo0);
  b.lo1 = fminf(b.lo1, o.lo1);
  b.lo2 = fminf(b.lo2, o.lo2);
  b.hi0 = fmaxf(b.hi0, o.hi0);
  b.hi1 = fmaxf(b.hi1, o.hi1);
  b.hi2 = fmaxf(b.hi2, o.hi2);
}

__global__ __launch_bounds__(kFbThreads) void k_field_bounds(const float4* __restrict__ E, int nx, int ny, int nz,
                                                             float2* __restrict__ out, unsigned* __restrict__ emax_bits) {
  __shared__ float4 s_e[kFbIn];  // (Ex, Ey, Ez, |E|), |E| < 0 outside the grid
  __shared__ float s_x[7][kFbXR];
  __shared__ float s_w[kFbThreads / 64];
  const int gx0 = (int)blockIdx.x * kFbTX - 1, gy0 = (int)blockIdx.y * kFbTY - 1;
  const int per = (nz + (int)gridDim.z - 1) / (int)gridDim.z;
  const int k0 = (int)blockIdx.z * per, k1 = min(nz, k0 + per);
  const int tid = threadIdx.x, tx = tid % kFbTX, ty = tid / kFbTX;
  float local_max = 0.0f;
  if (k0 < k1) {  // block-uniform
    float4 pre[kFbLoads];
    auto load = [&](int kk) {
#pragma unroll
      for (int q = 0; q < kFbLoads; ++q) {
        const int e = tid + q * kFbThreads;
        const int gx = gx0 + e % kFbIX, gy = gy0 + e / kFbIX;
        pre[q] = make_float4(0.0f, 0.0f, 0.0f, -1.0f);
        if (e < kFbIn && kk >= 0 && kk < nz && gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
          const float4 v = E[((size_t)kk * ny + gy) * nx + gx];
          pre[q] = make_float4(v.x, v.y, v.z, sqrtf(fmaf(v.z, v.z, fmaf(v.x, v.x, v.y * v.y))));
        }
      }
    };
    Box7 r0 = box_empty(), r1 = box_empty(), r2 = box_empty(), r3 = box_empty();  // planes kk-3 .. kk
    load(k0 - 1);
    for (int kk = k0 - 1; kk <= k1 + 1; ++kk) {
      __syncthreads();  // the previous plane's readers are done
#pragma unroll
      for (int q = 0; q < kFbLoads; ++q)
        if (tid + q * kFbThreads < kFbIn) s_e[tid + q * kFbThreads] = pre[q];
      if (kk + 1 <= k1 + 1) load(kk + 1);
      __syncthreads();
      for (int e = tid; e < kFbXR; e += kFbThreads) {  // 4-wide x windows of the tile's 7 rows
        const int row = e / kFbTX, col = e % kFbTX;
        Box7 b = box_empty();
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const float4 v = s_e[row * kFbIX + col + d];
          if (v.w >= 0.0f) box_add(b, Box7{v.w, v.x, v.y, v.z, v.x, v.y, v.z});
        }
        s_x[0][e] = b.m;
        s_x[1][e] = b.lo0;
        s_x[2][e] = b.lo1;
        s_x[3][e] = b.lo2;
        s_x[4][e] = b.hi0;
        s_x[5][e] = b.hi1;
        s_x[6][e] = b.hi2;
      }
      __syncthreads();
      Box7 nv = box_empty();  // 4-wide y window of this thread's column
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int e = (ty + d) * kFbTX + tx;
        box_add(nv, Box7{s_x[0][e], s_x[1][e], s_x[2][e], s_x[3][e], s_x[4][e], s_x[5][e], s_x[6][e]});
      }
      r0 = r1;
      r1 = r2;
      r2 = r3;
      r3 = nv;
      const int k = kk - 2, i = gx0 + 1 + tx, j = gy0 + 1 + ty;
      if (k >= k0 && i < nx && j < ny) {
        Box7 b = r0;
        box_add(b, r1);
        box_add(b, r2);
        box_add(b, r3);
        const float d0 = b.hi0 - b.lo0, d1 = b.hi1 - b.lo1, d2 = b.hi2 - b.lo2;
        out[((size_t)k * ny + j) * nx + i] = make_float2(b.m, sqrtf(fmaf(d2, d2, fmaf(d0, d0, d1 * d1))));
        local_max = fmaxf(local_max, b.m);  // every cell lies in its own box
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) local_max = fmaxf(local_max, __shfl_xor(local_max, off));
  if ((tid & 63) == 0) s_w[tid / 64] = local_max;
  __syncthreads();
  if (tid == 0) {
    float m = 0.0f;
    for (int w = 0; w < kFbThreads / 64; ++w) m = fmaxf(m, s_w[w]);
    if (m > 0.0f) atomicMax(emax_bits, __float_as_uint(m));
  }
}

// Corner-packed field (layout in pcmcc_device.hpp): one thread per record,
// the record of lower centre index (i, j, k) in [-1, n]^3 holding the fields
// of the 8 centres around it (indices clamped to the grid) and the bound of
// the cell clamp(i, j, k).  A block takes 128 consecutive records of the flat
// record order, forms them in registers, stages them in LDS and writes them
// out as consecutive float4s: each store instruction then covers 1 KiB of
// consecutive records instead of one 16-byte piece of 64 different records.
constexpr int kPackThreads = 128;
constexpr int kPackStride = kRecFloats / 4 + 1;  // float4 per record in LDS (one of padding spreads the banks)
__global__ __launch_bounds__(kPackThreads) void k_pack_field(const float4* __restrict__ E,
                                                             const float2* __restrict__ bound, int nx, int ny,
                                                             int nz, float4* __restrict__ P) {
  __shared__ float4 st[kPackThreads * kPackStride];
  const uint32_t px = (uint32_t)nx + 2, py = (uint32_t)ny + 2;
  const uint32_t nrec = px * py * ((uint32_t)nz + 2);  // below 2^31 (checked by the caller)
  const uint32_t r0 = blockIdx.x * kPackThreads;
  const uint32_t r = r0 + threadIdx.x;
  if (r < nrec) {
    const uint32_t row = r / px, ri = r - row * px;
    const uint32_t rk = row / py, rj = row - rk * py;
    const int i = (int)ri - 1, j = (int)rj - 1, k = (int)rk - 1;
    const int ci[2] = {min(max(i, 0), nx - 1), min(max(i + 1, 0), nx - 1)};
    const int cj[2] = {min(max(j, 0), ny - 1), min(max(j + 1, 0), ny - 1)};
    const int ck[2] = {min(max(k, 0), nz - 1), min(max(k + 1, 0), nz - 1)};
    float v[kRecFloats];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const float4 e = E[((size_t)ck[c >> 2] * ny + cj[(c >> 1) & 1]) * nx + ci[c & 1]];
      v[3 * c] = e.x;
      v[3 * c + 1] = e.y;
      v[3 * c + 2] = e.z;
    }
    // the dx = 1 corners as differences along x (rounded as the gather
    // would round them)
#pragma unroll
    for (int c = 1; c < 8; c += 2)
#pragma unroll
      for (int q = 0; q < 3; ++q) v[3 * c + q] = v[3 * c + q] - v[3 * (c - 1) + q];
    const float2 b = bound[((size_t)ck[0] * ny + cj[0]) * nx + ci[0]];
    v[24] = b.x;
    v[25] = b.y;
#pragma unroll
    for (int q = 26; q < kRecFloats; ++q) v[q] = 0.0f;
#pragma unroll
    for (int q = 0; q < kRecFloats / 4; ++q)
      st[threadIdx.x * kPackStride + q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  }
  __syncthreads();
  const uint32_t nb = min((uint32_t)kPackThreads, nrec - r0);  // records of this block
  float4* out = P + (size_t)r0 * (kRecFloats / 4);
  for (uint32_t f = threadIdx.x; f < nb * (kRecFloats / 4); f += kPackThreads)
    out[f] = st[(f / (kRecFloats / 4)) * kPackStride + f % (kRecFloats / 4)];
}

// ---------------------------------------------------------------------------
// Collision tables in double precision, stored as single precision: rates
// nu_k = N sigma_k v at each node (Sec. 2.1.5), cumulative sums in process
// order, prefix maximum of the total.
__global__ void k_build_tables(TableBuild B, float* __restrict__ C, float* __restrict__ P,
                               float* __restrict__ nu_out) {
  const int n = B.n, np = B.nproc;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double eps = exp(B.lnmin + i * B.dlog);
    const double v = sqrt(2.0 * B.ev * eps / B.mass);
    double inel = 0.0;
    for (int k = 0; k < np; ++k)
      if (B.kind[k] != ELASTIC) inel += B.sigma[(size_t)k * n + i];
    double acc = 0.0;
    for (int k = 0; k < np; ++k) {
      double s = B.sigma[(size_t)k * n + i];
      if (B.effective && B.kind[k] == ELASTIC) s = fmax(0.0, s - inel);
      const double rate = B.rates ? s : B.gas_N * s * v;
      acc += rate;
      nu_out[(size_t)k * n + i] = (float)rate;
      C[(size_t)k * n + i] = (float)acc;
      B.total[i] = acc;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double run = 0.0;
    for (int i = 0; i < n; ++i) {
      run = fmax(run, B.total[i]);
      P[i] = (float)run;
    }
  }
}

// Self-test entry: raw Philox4x32-10 words.
__global__ void k_philox(const uint4* __restrict__ ctr, Key key, uint4* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = philox(ctr[i], key);
}

// Table lookups exactly as the step kernel does them (LDS-staged tables).
__global__ void k_lookup(TableView TV, SpeciesView S, const float* __restrict__ eps, float* __restrict__ cum,
                         const float* __restrict__ s_ub, float* __restrict__ maj, int64_t n) {
  extern __shared__ float smem[];
  const Tab T = stage_tables(TV, S, smem);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
    const float e = eps[q];
    float u = fmaf(__log2f(e), T.u_scale, T.u_offset);
    u = fminf(fmaxf(u, 0.0f), (float)(T.n - 1));
    const float fl = fminf(floorf(u), (float)(T.n - 2));
    const int i = (int)fl;
    const float f = u - fl;
    float c[kMaxProc];
    cum_rates(T, i, f, c);
    for (int k = 0; k < T.nproc; ++k) cum[q * T.nproc + k] = c[k];
    if (maj) maj[q] = majorant_t(T, S, s_ub[q]);
  }
}

// ---------------------------------------------------------------------------
// launch wrappers

size_t table_lds_bytes(const TableView& T) { return table_lds_floats(T) * sizeof(float); }

size_t pic_lds_bytes(const TableView& T, int block) {
  return pic_stage_offset_floats(T) * sizeof(float) + (size_t)(block / 64) * (sizeof(WaveStage) + sizeof(ChunkRing));
}

template <int ROW>
static const void* pic_steps_kernel_row(int refill) {
  switch (refill) {
    case 16: return (const void*)k_pic_steps<16, ROW>;
    case 24: return (const void*)k_pic_steps<24, ROW>;
    case 32: return (const void*)k_pic_steps<32, ROW>;
    default: return nullptr;
  }
}

static const void* pic_steps_kernel(int refill, int row) {
  return row == 4 ? pic_steps_kernel_row<4>(refill) : row == 8 ? pic_steps_kernel_row<8>(refill) : nullptr;
}

hipError_t launch_pic_steps(const PicArgs& args, int grid, int block, int refill, hipStream_t stream) {
  const void* k = pic_steps_kernel(refill, table_row(args.T.nproc));
  if (!k) return hipErrorInvalidValue;
  void* kargs[] = {(void*)&args};
  return hipLaunchCooperativeKernel(k, dim3(grid), dim3(block), kargs, (unsigned)pic_lds_bytes(args.T, block),
                                    stream);
}

hipError_t coresident_blocks(const void* k, int block, size_t lds, int* blocks_per_cu) {
  constexpr size_t kLdsPerCu = 160 * 1024, kLdsGranule = 1280;
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, block, lds);
  if (e != hipSuccess) return e;
  hipFuncAttributes a;
  e = hipFuncGetAttributes(&a, k);
  if (e != hipSuccess) return e;
  const size_t per = (a.sharedSizeBytes + lds + kLdsGranule - 1) / kLdsGranule * kLdsGranule;
  const int by_lds = per ? (int)(kLdsPerCu / per) : occ;
  *blocks_per_cu = occ < by_lds ? occ : by_lds;
  return hipSuccess;
}

hipError_t occupancy_pic_steps(int block, int refill, int row, size_t lds, int* blocks_per_cu) {
  const void* k = pic_steps_kernel(refill, row);
  if (!k) return hipErrorInvalidValue;
  return coresident_blocks(k, block, lds, blocks_per_cu);
}

hipError_t launch_finalize(const Soa& user, const Soa& scratch, Ctl* ctl, int64_t* n_dev, hipStream_t stream) {
  hipLaunchKernelGGL(k_finalize, dim3(2048), dim3(256), 0, stream, user, scratch, ctl, n_dev);
  return hipGetLastError();
}

hipError_t launch_field_bounds(const float4* E, int nx, int ny, int nz, float2* out, unsigned* emax_bits,
                               hipStream_t stream) {
  const unsigned tx = (unsigned)((nx + kFbTX - 1) / kFbTX), ty = (unsigned)((ny + kFbTY - 1) / kFbTY);
  unsigned chunks = (2048 + tx * ty - 1) / (tx * ty);  // plane ranges: about 2048 blocks, at least 16 planes each
  if (chunks > (unsigned)(nz / 16)) chunks = (unsigned)(nz / 16);
  if (chunks < 1) chunks = 1;
  hipLaunchKernelGGL(k_field_bounds, dim3(tx, ty, chunks), dim3(kFbThreads), 0, stream, E, nx, ny, nz, out,
                     emax_bits);
  return hipGetLastError();
}

hipError_t launch_pack_field(const float4* E, const float2* bound, int nx, int ny, int nz, float4* P,
                             hipStream_t stream) {
  const uint64_t nrec = ((uint64_t)nx + 2) * ((uint64_t)ny + 2) * ((uint64_t)nz + 2);
  if (nrec >= ((uint64_t)1 << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pack_field, dim3((unsigned)((nrec + kPackThreads - 1) / kPackThreads)), dim3(kPackThreads), 0,
                     stream, E, bound, nx, ny, nz, P);
  return hipGetLastError();
}

hipError_t launch_build_tables(const TableBuild& B, float* C, float* P, float* nu, hipStream_t stream) {
  hipLaunchKernelGGL(k_build_tables, dim3(1), dim3(1024), 0, stream, B, C, P, nu);
  return hipGetLastError();
}

hipError_t launch_philox(const uint32_t* ctr, Key key, uint32_t* out, int64_t n, hipStream_t stream) {
  const int blocks = (int)std::min<int64_t>((n + 255) / 256 + 1, 4096);
  hipLaunchKernelGGL(k_philox, dim3(blocks), dim3(256), 0, stream, (const uint4*)ctr, key, (uint4*)out, n);
  return hipGetLastError();
}

hipError_t launch_lookup(const TableView& T, const SpeciesView& S, const float* eps, float* cum, const float* s_ub,
                         float* maj, int64_t n, hipStream_t stream) {
  const int blocks = (int)std::min<int64_t>((n + 255) / 256 + 1, 4096);
  hipLaunchKernelGGL(k_lookup, dim3(blocks), dim3(256), table_lds_bytes(T), stream, T, S, eps, cum, s_ub, maj, n);
  return hipGetLastError();
}

}  // namespace pcmcc
